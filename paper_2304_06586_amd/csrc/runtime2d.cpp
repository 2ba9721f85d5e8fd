// Host runtime of the 2D (TE / TM) path: validation, the stability
// pre-flight, workspace carving, the launch sequence of a pass and the
// C-ABI entry points declared in gfdtd2d.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "gfdtd.h"
#include "gfdtd2d.h"
#include "gfdtd2d_internal.h"
#include "gfdtd_internal.h"
#include "runtime.h"

namespace gfdtd {

namespace {

using cplx = std::complex<double>;

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

gfdtd_status validate2d(const gfdtd2d_problem *p, int64_t steps)
{
    if (!p)
        return fail(GFDTD_E_INVALID, "problem is NULL");
    if (p->struct_size < sizeof(gfdtd2d_problem))
        return fail(GFDTD_E_INVALID, "problem struct_size %u < %zu", p->struct_size,
                    sizeof(gfdtd2d_problem));
    if (p->pol != GFDTD2D_TE && p->pol != GFDTD2D_TM)
        return fail(GFDTD_E_INVALID, "unknown polarization %d", p->pol);
    if (p->precision != GFDTD_F32 && p->precision != GFDTD_F64)
        return fail(GFDTD_E_INVALID, "unknown precision %d", p->precision);
    if (p->abc != GFDTD_ABC_MUR1 && p->abc != GFDTD_ABC_PEC &&
        p->abc != GFDTD_ABC_PERIODIC)
        return fail(GFDTD_E_INVALID, "unknown end condition %d", p->abc);
    if (p->flags & ~(uint32_t)(GFDTD_FLAG_RECORD_TRACE | GFDTD_FLAG_ALLOW_UNSTABLE))
        return fail(GFDTD_E_UNSUPPORTED, "flags 0x%x: only RECORD_TRACE and "
                    "ALLOW_UNSTABLE apply to 2D runs", p->flags);
    if (p->nx < 1 || p->nx > (int64_t(1) << 20))
        return fail(GFDTD_E_INVALID, "nx = %lld outside 1..2^20", (long long)p->nx);
    if (p->nz < 8 || p->nz > (int64_t(1) << 24))
        return fail(GFDTD_E_INVALID, "nz = %lld outside 8..2^24", (long long)p->nz);
    if (p->nx * p->nz > (int64_t(1) << 31))
        return fail(GFDTD_E_INVALID, "nx * nz above 2^31");
    if (steps < 0)
        return fail(GFDTD_E_INVALID, "steps = %lld < 0", (long long)steps);
    if (!finite_pos(p->courant))
        return fail(GFDTD_E_INVALID, "Courant number must be finite and > 0");
    if (!std::isfinite(p->beta) || std::fabs(p->beta) >= 1.0)
        return fail(GFDTD_E_INVALID, "|beta| must be < 1");
    if (std::fabs(p->beta * p->courant) > 0.9)
        return fail(GFDTD_E_INVALID, "|beta| S must be <= 0.9");
    if (!p->eps_rest || !p->mu_rest)
        return fail(GFDTD_E_INVALID, "eps_rest / mu_rest missing");
    for (int64_t i = 0; i < p->nz; ++i)
        if (!finite_pos(p->eps_rest[i]) || !finite_pos(p->mu_rest[i]))
            return fail(GFDTD_E_INVALID, "eps_rest/mu_rest[%lld] not finite > 0",
                        (long long)i);
    const bool ring = p->abc == GFDTD_ABC_PERIODIC;
    if (ring ? (p->src_row < 0 || p->src_row > p->nz - 1)
             : (p->src_row < 1 || p->src_row > p->nz - 2))
        return fail(GFDTD_E_INVALID, "src_row %lld outside %s", (long long)p->src_row,
                    ring ? "0..nz-1" : "1..nz-2");
    if (p->src_profile)
        for (int64_t i = 0; i < p->nx; ++i)
            if (!std::isfinite(p->src_profile[i]))
                return fail(GFDTD_E_INVALID, "src_profile[%lld] not finite", (long long)i);
    if (!std::isfinite(p->src_amp) || !std::isfinite(p->src_omega) ||
        !std::isfinite(p->src_t0) || !std::isfinite(p->src_phase) ||
        !std::isfinite(p->src_t_off))
        return fail(GFDTD_E_INVALID, "source parameters must be finite");
    if (p->src_amp != 0.0 && !finite_pos(p->src_tau))
        return fail(GFDTD_E_INVALID, "src_tau must be > 0");
    if (p->nprobe < 0 || p->nprobe > GFDTD_MAX_PROBES)
        return fail(GFDTD_E_INVALID, "nprobe %d outside 0..%d", p->nprobe, GFDTD_MAX_PROBES);
    if (p->nprobe > 0 && (!p->probe_x || !p->probe_z))
        return fail(GFDTD_E_INVALID, "probe_x / probe_z missing");
    for (int q = 0; q < p->nprobe; ++q)
        if (p->probe_x[q] < 0 || p->probe_x[q] >= p->nx || p->probe_z[q] < 0 ||
            p->probe_z[q] >= p->nz)
            return fail(GFDTD_E_INVALID, "probe %d at (%lld, %lld) outside the grid", q,
                        (long long)p->probe_x[q], (long long)p->probe_z[q]);
    if (p->nfreq < 0 || (p->nfreq > 0 && !p->omegas))
        return fail(GFDTD_E_INVALID, "bad nfreq / omegas");
    for (int f = 0; f < p->nfreq; ++f)
        if (!std::isfinite(p->omegas[f]))
            return fail(GFDTD_E_INVALID, "omegas[%d] not finite", f);
    const int64_t cells = p->nx * p->nz;
    for (const double *a : {p->init_d, p->init_b, p->init_c})
        if (a)
            for (int64_t i = 0; i < cells; ++i)
                if (!std::isfinite(a[i]))
                    return fail(GFDTD_E_INVALID, "initial field value %lld not finite",
                                (long long)i);
    return GFDTD_OK;
}

// One step of the scheme applied to the plane wave exp(i (kx i + kz k)) of
// every unknown (index phases) in a uniform medium: u = (D, B, C) -> G u.
// Z = e^{i kz}, X = e^{i kx}; the Table 1 stencils of column a (v >= 0) or
// b (v < 0) give the B average aB, the D average aD and the upwind
// difference up.
struct Symbol {
    bool te;
    double S, beta, ce, ch;
    cplx Z, X, aB, aD, up;

    void apply(const cplx in[3], cplx out[3]) const
    {
        const double bS = beta * S;
        const cplx D = in[0], B = in[1], C = in[2];
        const cplx keep = 1.0 - bS * up;
        if (te) {
            const cplx Es = ce * D + beta * aB * B;
            const cplx Bn = keep * B + S * (Z - 1.0) * Es;
            const cplx Cn = keep * C - S * (X - 1.0) * Es;
            const cplx Hs = ch * Bn + beta * aD * D;
            const cplx Hc = ch * Cn;
            out[0] = keep * D + S * (1.0 - 1.0 / Z) * Hs - S * (1.0 - 1.0 / X) * Hc;
            out[1] = Bn;
            out[2] = Cn;
        } else {
            const cplx Es = ce * D - beta * aB * B;
            const cplx Ec = ce * C;
            const cplx Bn = keep * B - S * (Z - 1.0) * Es + S * (X - 1.0) * Ec;
            const cplx Hs = ch * Bn - beta * aD * D;
            out[0] = keep * D - S * (1.0 - 1.0 / Z) * Hs;
            out[1] = Bn;
            out[2] = keep * C + S * (1.0 - 1.0 / X) * Hs;
        }
    }
};

// Largest eigenvalue modulus of G.  One eigenvalue is known in closed form:
// the discrete divergence of B (TE) or D (TM) is a left eigenvector with
// eigenvalue 1 - beta S up, because the curls are divergence-free.  The
// characteristic cubic is deflated by it and the quadratic solved.
double mode_growth(const Symbol &sy)
{
    cplx G[3][3];
    for (int c = 0; c < 3; ++c) {
        cplx e[3] = {0.0, 0.0, 0.0}, o[3];
        e[c] = 1.0;
        sy.apply(e, o);
        for (int r = 0; r < 3; ++r)
            G[r][c] = o[r];
    }
    const cplx tr = G[0][0] + G[1][1] + G[2][2];
    const cplx m2 = G[0][0] * G[1][1] - G[0][1] * G[1][0] + G[0][0] * G[2][2] -
                    G[0][2] * G[2][0] + G[1][1] * G[2][2] - G[1][2] * G[2][1];
    const cplx l3 = 1.0 - sy.beta * sy.S * sy.up;
    // l^3 - tr l^2 + m2 l - det = (l - l3)(l^2 + p l + q)
    const cplx p = l3 - tr;
    const cplx q = m2 + l3 * p;
    const cplx disc = std::sqrt(p * p - 4.0 * q);
    const cplx a = -p + (std::real(std::conj(-p) * disc) >= 0.0 ? disc : -disc);
    cplx l1, l2;
    if (std::abs(a) > 0.0) {
        l1 = 0.5 * a;
        l2 = 2.0 * q / a;
    } else {
        l1 = l2 = 0.0;
    }
    return std::max({std::abs(l1), std::abs(l2), std::abs(l3)});
}

double spectral_radius2d(bool te, double eps, double mu, double S, double beta)
{
    const bool cola = beta >= 0.0;
    double g = 0.0;
    const int NX = 64, NZ = 128;
    for (int jx = 0; jx <= NX; ++jx) {
        const double kx = M_PI * jx / NX;
        for (int jz = 1; jz <= NZ; ++jz) {
            const double kz = -M_PI + 2.0 * M_PI * jz / NZ;
            Symbol sy;
            sy.te = te;
            sy.S = S;
            sy.beta = beta;
            sy.ce = 1.0 / eps;
            sy.ch = 1.0 / mu;
            sy.Z = std::polar(1.0, kz);
            sy.X = std::polar(1.0, kx);
            sy.aD = 0.5 * (sy.Z + 1.0);
            sy.aB = cola ? 0.5 * (1.0 / sy.Z + 1.0 / (sy.Z * sy.Z)) : 0.5 * (sy.Z + 1.0);
            sy.up = cola ? 1.0 - 1.0 / sy.Z : sy.Z - 1.0;
            g = std::max(g, mode_growth(sy));
        }
    }
    return g;
}

gfdtd_status preflight2d(const gfdtd2d_problem *p, int64_t steps, double *growth)
{
    std::vector<std::pair<double, double>> media;
    for (int64_t i = 0; i < p->nz; ++i)
        media.emplace_back(p->eps_rest[i], p->mu_rest[i]);
    std::sort(media.begin(), media.end(),
              [](const std::pair<double, double> &a, const std::pair<double, double> &b) {
                  const double na = a.first * a.second, nb = b.first * b.second;
                  return na != nb ? na < nb : a < b;
              });
    media.erase(std::unique(media.begin(), media.end()), media.end());
    std::vector<std::pair<double, double>> pick;
    if (media.size() <= 32) {
        pick = media;
    } else {
        for (int q = 0; q < 32; ++q)
            pick.push_back(media[(size_t)((media.size() - 1) * (double)q / 31.0)]);
    }
    double g = 0.0;
    for (const auto &m : pick)
        g = std::max(g, spectral_radius2d(p->pol == GFDTD2D_TE, m.first, m.second,
                                          p->courant, p->beta));
    if (growth)
        *growth = g;
    // the worst mode may grow by GFDTD2D_MAX_RUN_GROWTH over the run
    const double run_log = (double)steps * std::log(std::max(g, 1.0));
    if (run_log > std::log(GFDTD2D_MAX_RUN_GROWTH) + 1e-12 &&
        !(p->flags & GFDTD_FLAG_ALLOW_UNSTABLE))
        return fail(GFDTD_E_UNSTABLE,
                    "pre-flight: 2D amplification factor %.12g per step grows the worst "
                    "mode by %.3g over %lld steps (limit %g; beta %.4g, S %.4g)",
                    g, std::exp(std::min(run_log, 700.0)), (long long)steps,
                    GFDTD2D_MAX_RUN_GROWTH, p->beta, p->courant);
    return GFDTD_OK;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int64_t column_stride(int64_t nz) { return (int64_t)round_up((size_t)nz, 64); }

int64_t source_samples2d(const gfdtd2d_problem *p, int64_t steps)
{
    if (p->src_amp == 0.0 || steps <= 0)
        return 0;
    double est = std::floor(p->src_t_off / p->courant);
    int64_t n = est < 0 ? 0 : (int64_t)std::min<double>(est, (double)steps);
    while (n < steps && (double)(n + 1) * p->courant <= p->src_t_off)
        ++n;
    while (n > 0 && !((double)n * p->courant <= p->src_t_off))
        --n;
    return n;
}

struct Layout2D {
    size_t desc = 0, dft_desc = 0, eps = 0, mu = 0, prof = 0, src = 0, px = 0, pz = 0;
    size_t omegas = 0, trace = 0, dft = 0, field[6] = {0, 0, 0, 0, 0, 0};
    size_t init[3] = {0, 0, 0};
    size_t total = 0;
};

Layout2D carve2d(const gfdtd2d_problem *p, int64_t steps)
{
    Carver cv;
    Layout2D L;
    const size_t w = p->precision == GFDTD_F32 ? 4 : 8;
    const size_t nz = (size_t)p->nz, nx = (size_t)p->nx;
    L.desc = cv.take(sizeof(Run2D));
    L.dft_desc = cv.take(sizeof(DftDesc));
    L.eps = cv.take(nz * 8);
    L.mu = cv.take(nz * 8);
    L.prof = cv.take(nx * 8);
    L.src = cv.take((size_t)std::max<int64_t>(source_samples2d(p, steps), 1) * 8);
    L.px = cv.take((size_t)std::max(p->nprobe, 1) * 8);
    L.pz = cv.take((size_t)std::max(p->nprobe, 1) * 8);
    L.omegas = cv.take((size_t)std::max(p->nfreq, 1) * 8);
    L.trace = cv.take((size_t)std::max<int64_t>((int64_t)p->nprobe * steps, 1) * 8);
    L.dft = cv.take((size_t)std::max(p->nprobe * p->nfreq, 1) * 16);
    const size_t fbytes = nx * (size_t)column_stride(p->nz) * w;
    for (int f = 0; f < 6; ++f)
        L.field[f] = cv.take(fbytes);
    const double *init[3] = {p->init_d, p->init_b, p->init_c};
    for (int f = 0; f < 3; ++f)
        L.init[f] = init[f] ? cv.take(nx * nz * 8) : 0;
    L.total = cv.off;
    return L;
}

}  // namespace

}  // namespace gfdtd

using namespace gfdtd;

struct gfdtd2d_run {
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    gfdtd2d_problem p{};
    int64_t steps = 0;
    Layout2D L;
    Run2D host{};
    Launch2D launch;             // T steps a launch
    Launch2D single;             // one step a launch (a pass's last steps)
    int64_t launches = 0;
    int final_par = 0;           // the half of each pair the pass ended in
    std::vector<double> eps, mu, prof, omegas, init[3];
    std::vector<int64_t> px, pz;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    bool ran = false;
    double step_ms = 0.0, pass_ms = 0.0;

    ~gfdtd2d_run()
    {
        if (stream || ws)
            (void)hipStreamSynchronize(stream);
        for (hipEvent_t &e : ev)
            if (e)
                (void)hipEventDestroy(e);
    }
};

namespace {

gfdtd_status prepare2d(const gfdtd2d_problem *p, int64_t steps, const gfdtd2d_exec *ex,
                       void *ws, size_t ws_bytes, hipStream_t stream, gfdtd2d_run **out)
{
    gfdtd_status st = validate2d(p, steps);
    if (st != GFDTD_OK)
        return st;
    if ((st = preflight2d(p, steps, nullptr)) != GFDTD_OK)
        return st;
    if (ex && ex->struct_size < sizeof(gfdtd2d_exec))
        return fail(GFDTD_E_INVALID, "exec struct_size %u < %zu", ex->struct_size,
                    sizeof(gfdtd2d_exec));
    int C = ex ? ex->cells_per_lane : 0;
    const int xch = ex ? ex->columns_per_wave : 0;
    int T = ex ? ex->block_steps : 0;
    if (C != 0) {
        const bool ok = p->precision == GFDTD_F32 ? (C == 2 || C == 4 || C == 8)
                                                  : (C == 2 || C == 4);
        if (!ok)
            return fail(GFDTD_E_INVALID, "cells_per_lane %d not available for this "
                        "precision (FP32: 2, 4, 8; FP64: 2, 4)", C);
    }
    if (xch < 0 || xch > 4096)
        return fail(GFDTD_E_INVALID, "columns_per_wave %d outside 0..4096", xch);
    if (T < 0 || T > 4)
        return fail(GFDTD_E_INVALID, "block_steps %d outside 0..4", T);
    const int narrow = p->precision == GFDTD_F32 ? 4 : 2;     // widest multi-step lane
    const bool ring = p->abc == GFDTD_ABC_PERIODIC;
    if (T > 1 && ((C != 0 && C > narrow) || ring))
        return fail(GFDTD_E_INVALID, "block_steps %d needs at most %d cells per lane "
                    "and non-periodic ends", T, narrow);
    if (T == 0)   // several steps a launch where the tiling allows it (measured
                  // best: four, FP32 and FP64, at 2 cells per lane)
        T = (ring || (C != 0 && C > narrow)) ? 1 : 4;
    Layout2D L = carve2d(p, steps);
    if (!ws || ws_bytes < L.total)
        return fail(GFDTD_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, L.total);

    auto *r = new gfdtd2d_run();
    r->stream = stream;
    r->ws = static_cast<char *>(ws);
    r->p = *p;
    r->steps = steps;
    r->L = L;
    const int64_t nx = p->nx, nz = p->nz;
    r->eps.assign(p->eps_rest, p->eps_rest + nz);
    r->mu.assign(p->mu_rest, p->mu_rest + nz);
    r->prof = p->src_profile ? std::vector<double>(p->src_profile, p->src_profile + nx)
                             : std::vector<double>((size_t)nx, 1.0);
    r->omegas.assign(p->omegas, p->omegas + std::max(p->nfreq, 0));
    r->px.assign(p->probe_x, p->probe_x + std::max(p->nprobe, 0));
    r->pz.assign(p->probe_z, p->probe_z + std::max(p->nprobe, 0));
    const double *init[3] = {p->init_d, p->init_b, p->init_c};
    for (int f = 0; f < 3; ++f)
        if (init[f])
            r->init[f].assign(init[f], init[f] + nx * nz);
    r->p.eps_rest = r->eps.data();
    r->p.mu_rest = r->mu.data();
    r->p.src_profile = r->prof.data();
    r->p.omegas = r->omegas.data();
    r->p.probe_x = r->px.data();
    r->p.probe_z = r->pz.data();
    r->p.init_d = r->p.init_b = r->p.init_c = nullptr;

    Run2D &h = r->host;
    char *base = r->ws;
    h.nx = nx;
    h.nz = nz;
    h.ld = column_stride(nz);
    h.nh = ring ? nz : nz - 1;
    h.nc = p->pol == GFDTD2D_TE ? nz : h.nh;
    h.src_row = p->src_row;
    h.nsrc = source_samples2d(p, steps);
    h.steps = steps;
    h.S = p->courant;
    h.beta = p->beta;
    h.amp = p->src_amp;
    h.omega = p->src_omega;
    h.t0 = p->src_t0;
    h.tau = p->src_tau;
    h.phase = p->src_phase;
    h.pol = p->pol;
    h.abc = p->abc;
    h.nprobe = p->nprobe;
    h.precision = p->precision;
    h.eps = reinterpret_cast<const double *>(base + L.eps);
    h.mu = reinterpret_cast<const double *>(base + L.mu);
    h.prof = reinterpret_cast<const double *>(base + L.prof);
    h.src = reinterpret_cast<double *>(base + L.src);
    h.px = reinterpret_cast<const int64_t *>(base + L.px);
    h.pz = reinterpret_cast<const int64_t *>(base + L.pz);
    h.trace = reinterpret_cast<double *>(base + L.trace);
    for (int f = 0; f < 6; ++f)
        h.f[f] = base + L.field[f];
    for (int f = 0; f < 3; ++f)
        h.init[f] = init[f] ? reinterpret_cast<const double *>(base + L.init[f]) : nullptr;
    r->launch = plan_launch2d(nx, nz, p->precision, C, xch, T);
    r->single = plan_launch2d(nx, nz, p->precision, r->launch.C, r->launch.xch, 1);

    DftDesc dd{};
    dd.steps = steps;
    dd.S = p->courant;
    dd.nprobe = p->nprobe;
    dd.nfreq = p->nfreq;
    dd.trace = h.trace;
    dd.omegas = reinterpret_cast<const double *>(base + L.omegas);
    dd.out = reinterpret_cast<double *>(base + L.dft);

    hipError_t e = hipSuccess;
    auto up = [&](size_t off, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes > 0)
            e = hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, stream);
    };
    up(L.desc, &r->host, sizeof(Run2D));
    up(L.dft_desc, &dd, sizeof(DftDesc));
    up(L.eps, r->eps.data(), (size_t)nz * 8);
    up(L.mu, r->mu.data(), (size_t)nz * 8);
    up(L.prof, r->prof.data(), (size_t)nx * 8);
    up(L.px, r->px.data(), r->px.size() * 8);
    up(L.pz, r->pz.data(), r->pz.size() * 8);
    up(L.omegas, r->omegas.data(), r->omegas.size() * 8);
    for (int f = 0; f < 3; ++f)
        if (init[f])
            up(L.init[f], r->init[f].data(), r->init[f].size() * 8);
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
        e = hipEventCreate(&r->ev[k]);
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);   // host copies may go after this
    if (e != hipSuccess) {
        delete r;
        return hip_fail(e, "2D prepare");
    }
    *out = r;
    return GFDTD_OK;
}

gfdtd_status run_pass2d(gfdtd2d_run *r)
{
    hipError_t e;
    const Run2D *dev = reinterpret_cast<const Run2D *>(r->ws + r->L.desc);
    if ((e = hipEventRecord(r->ev[0], r->stream)))
        return hip_fail(e, "event");
    if ((e = launch_prep2d(dev, r->host, r->stream)))
        return hip_fail(e, "2D prep launch");
    if ((e = hipEventRecord(r->ev[1], r->stream)))
        return hip_fail(e, "event");
    int par = 0;
    int64_t launches = 0;
    for (int64_t n = 1; n <= r->steps;) {
        const Launch2D &L = (r->steps - n + 1 >= r->launch.T) ? r->launch : r->single;
        if ((e = launch_step2d(r->host, L, n, par, r->stream)))
            return hip_fail(e, "2D step launch");
        n += L.T;
        par ^= 1;
        ++launches;
    }
    r->launches = launches;
    r->final_par = par;
    if ((e = hipEventRecord(r->ev[2], r->stream)))
        return hip_fail(e, "event");
    if (r->p.nprobe * r->p.nfreq > 0 && r->steps > 0) {
        const DftDesc *dd = reinterpret_cast<const DftDesc *>(r->ws + r->L.dft_desc);
        if ((e = launch_dft(dd, 1, r->p.nprobe * r->p.nfreq, r->stream)))
            return hip_fail(e, "2D DFT launch");
    }
    r->ran = true;
    return GFDTD_OK;
}

gfdtd_status collect2d(gfdtd2d_run *r, gfdtd2d_result *out)
{
    if (!out || out->struct_size < sizeof(gfdtd2d_result))
        return fail(GFDTD_E_INVALID, "result struct missing or too small");
    if (!r->ran)
        return fail(GFDTD_E_INVALID, "no pass has run");
    hipError_t e;
    if ((e = hipStreamSynchronize(r->stream)))
        return hip_fail(e, "2D collect");
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r->ev[1], r->ev[2]) == hipSuccess)
        r->step_ms = ms;
    if (hipEventElapsedTime(&ms, r->ev[0], r->ev[2]) == hipSuccess)
        r->pass_ms = ms;
    const gfdtd2d_problem &p = r->p;
    const int np = p.nprobe, nf = p.nfreq;
    const int64_t steps = r->steps;
    std::vector<double> dft((size_t)np * nf * 2);
    if (np * nf > 0 && (e = hipMemcpy(dft.data(), r->ws + r->L.dft, dft.size() * 8,
                                      hipMemcpyDeviceToHost)))
        return hip_fail(e, "copy DFT");
    const bool want_trace = out->trace && (p.flags & GFDTD_FLAG_RECORD_TRACE);
    std::vector<double> trace;
    if (np > 0 && steps > 0 && (want_trace || nf == 0)) {
        trace.resize((size_t)np * steps);
        if ((e = hipMemcpy(trace.data(), r->ws + r->L.trace, trace.size() * 8,
                           hipMemcpyDeviceToHost)))
            return hip_fail(e, "copy trace");
    }
    bool finite = true;
    for (double v : dft)
        finite = finite && std::isfinite(v);
    for (double v : trace)
        finite = finite && std::isfinite(v);
    out->run_status = finite ? GFDTD_OK : GFDTD_E_BLOWUP;
    out->steps_done = steps;
    if (out->dft_re && out->dft_im)
        for (int i = 0; i < np * nf; ++i) {
            out->dft_re[i] = dft[2 * i];
            out->dft_im[i] = dft[2 * i + 1];
        }
    if (want_trace && !trace.empty())
        std::memcpy(out->trace, trace.data(), trace.size() * 8);
    // final fields: the half of each pair the last launch wrote
    const int fin = r->final_par;
    const size_t w = p.precision == GFDTD_F32 ? 4 : 8;
    const int64_t nx = p.nx, nz = p.nz, ld = r->host.ld;
    const int64_t nlat[3] = {nz, r->host.nh, r->host.nc};
    double *dst[3] = {out->final_d, out->final_b, out->final_c};
    std::vector<char> buf;
    for (int f = 0; f < 3; ++f) {
        if (!dst[f])
            continue;
        buf.resize((size_t)nx * ld * w);
        if ((e = hipMemcpy(buf.data(), r->ws + r->L.field[2 * f + fin], buf.size(),
                           hipMemcpyDeviceToHost)))
            return hip_fail(e, "copy fields");
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t k = 0; k < nz; ++k) {
                const int64_t s = i * ld + k;
                double v = 0.0;
                if (k < nlat[f])
                    v = w == 4 ? (double)reinterpret_cast<const float *>(buf.data())[s]
                               : reinterpret_cast<const double *>(buf.data())[s];
                dst[f][i * nz + k] = v;
            }
    }
    return GFDTD_OK;
}

}  // namespace

extern "C" {

gfdtd_status gfdtd2d_check(const gfdtd2d_problem *p, int64_t steps, double *max_growth)
{
    clear_error();
    gfdtd_status st = validate2d(p, steps);
    if (st != GFDTD_OK)
        return st;
    return preflight2d(p, steps, max_growth);
}

gfdtd_status gfdtd2d_workspace_bytes(const gfdtd2d_problem *p, int64_t steps, size_t *bytes)
{
    clear_error();
    gfdtd_status st = validate2d(p, steps);
    if (st != GFDTD_OK)
        return st;
    if (!bytes)
        return fail(GFDTD_E_INVALID, "bytes is NULL");
    *bytes = carve2d(p, steps).total;
    return GFDTD_OK;
}

gfdtd_status gfdtd2d_prepare(const gfdtd2d_problem *p, int64_t steps,
                             const gfdtd2d_exec *exec, void *ws, size_t ws_bytes,
                             void *stream, gfdtd2d_run **out)
{
    clear_error();
    if (!out)
        return fail(GFDTD_E_INVALID, "out is NULL");
    *out = nullptr;
    return prepare2d(p, steps, exec, ws, ws_bytes, static_cast<hipStream_t>(stream), out);
}

gfdtd_status gfdtd2d_run_pass(gfdtd2d_run *r)
{
    clear_error();
    if (!r)
        return fail(GFDTD_E_INVALID, "run is NULL");
    return run_pass2d(r);
}

gfdtd_status gfdtd2d_collect(gfdtd2d_run *r, gfdtd2d_result *out)
{
    clear_error();
    if (!r)
        return fail(GFDTD_E_INVALID, "run is NULL");
    return collect2d(r, out);
}

gfdtd_status gfdtd2d_get_stats(const gfdtd2d_run *r, gfdtd2d_stats *s)
{
    clear_error();
    if (!r || !s || s->struct_size < sizeof(gfdtd2d_stats))
        return fail(GFDTD_E_INVALID, "run or stats missing or too small");
    s->cells_per_lane = r->launch.C;
    s->columns_per_wave = r->launch.xch;
    s->waves = (int32_t)r->launch.waves;
    s->launches = r->launches;
    s->block_steps = r->launch.T;
    s->cell_updates = (double)r->p.nx * (double)r->p.nz * (double)r->steps;
    s->step_ms = r->step_ms;
    s->pass_ms = r->pass_ms;
    return GFDTD_OK;
}

void gfdtd2d_destroy(gfdtd2d_run *r) { delete r; }

gfdtd_status gfdtd2d_solve(const gfdtd2d_problem *p, int64_t steps, void *ws,
                           size_t ws_bytes, void *stream, gfdtd2d_result *out)
{
    clear_error();
    gfdtd2d_run *r = nullptr;
    gfdtd_status st =
        prepare2d(p, steps, nullptr, ws, ws_bytes, static_cast<hipStream_t>(stream), &r);
    if (st != GFDTD_OK)
        return st;
    st = run_pass2d(r);
    if (st == GFDTD_OK)
        st = collect2d(r, out);
    delete r;
    return st;
}

}  // extern "C"
