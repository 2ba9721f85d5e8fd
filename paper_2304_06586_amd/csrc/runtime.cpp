// Host runtime of the generalized-FDTD library: argument validation, the
// stability pre-flight, workspace carving, batch plans (run tables, tile
// tables, launch sequences, optional hipGraph capture) and the C-ABI
// entry points.  The continuous-batching server lives in server.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "gfdtd.h"
#include "gfdtd_internal.h"
#include "runtime.h"

namespace gfdtd {

// ------------------------------------------------------------------ errors

static thread_local std::string g_error;

gfdtd_status fail(gfdtd_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

gfdtd_status hip_fail(hipError_t e, const char *what)
{
    return fail(GFDTD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_error.clear(); }
const char *last_error() { return g_error.c_str(); }

// -------------------------------------------------------------- validation

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

gfdtd_status validate(const gfdtd_problem *p, int64_t steps)
{
    if (!p)
        return fail(GFDTD_E_INVALID, "problem is NULL");
    if (p->struct_size < sizeof(gfdtd_problem))
        return fail(GFDTD_E_INVALID, "problem struct_size %u < %zu",
                    p->struct_size, sizeof(gfdtd_problem));
    if (p->kind != GFDTD_MODULATION && p->kind != GFDTD_MATTER)
        return fail(GFDTD_E_INVALID, "unknown kind %d", p->kind);
    if (p->precision != GFDTD_F32 && p->precision != GFDTD_F64)
        return fail(GFDTD_E_INVALID, "unknown precision %d", p->precision);
    if (p->abc != GFDTD_ABC_MUR1 && p->abc != GFDTD_ABC_PEC &&
        p->abc != GFDTD_ABC_PERIODIC)
        return fail(GFDTD_E_INVALID, "unknown end condition %d", p->abc);
    if (p->nz < 8)
        return fail(GFDTD_E_INVALID, "nz = %lld < 8", (long long)p->nz);
    if (p->nz > (int64_t(1) << 31) - (int64_t(1) << 20))
        return fail(GFDTD_E_INVALID, "nz = %lld too large (limit 2^31 - 2^20)",
                    (long long)p->nz);
    if (steps < 0)
        return fail(GFDTD_E_INVALID, "steps = %lld < 0", (long long)steps);
    if (!finite_pos(p->courant))
        return fail(GFDTD_E_INVALID, "Courant number must be finite and > 0");
    if (!std::isfinite(p->beta) || std::fabs(p->beta) >= 1.0)
        return fail(GFDTD_E_INVALID, "|beta| must be < 1");
    // the profile then moves at most one cell per step at each node type
    // (every stable problem has |beta| S <= 1/2)
    if (std::fabs(p->beta * p->courant) > 0.9)
        return fail(GFDTD_E_INVALID, "|beta| S must be <= 0.9");
    if (!p->eps_rest || !p->mu_rest)
        return fail(GFDTD_E_INVALID, "eps_rest / mu_rest missing");
    for (int64_t i = 0; i < p->nz; ++i)
        if (!finite_pos(p->eps_rest[i]) || !finite_pos(p->mu_rest[i]))
            return fail(GFDTD_E_INVALID, "eps_rest/mu_rest[%lld] not finite > 0",
                        (long long)i);
    const bool ring = p->abc == GFDTD_ABC_PERIODIC;
    if (ring ? (p->src_cell < 0 || p->src_cell > p->nz - 1)
             : (p->src_cell < 1 || p->src_cell > p->nz - 2))
        return fail(GFDTD_E_INVALID, "src_cell %lld outside %s",
                    (long long)p->src_cell, ring ? "0..nz-1" : "1..nz-2");
    if (!std::isfinite(p->src_amp) || !std::isfinite(p->src_omega) ||
        !std::isfinite(p->src_t0) || !std::isfinite(p->src_phase) ||
        !std::isfinite(p->src_t_off))
        return fail(GFDTD_E_INVALID, "source parameters must be finite");
    if (p->src_amp != 0.0 && !finite_pos(p->src_tau))
        return fail(GFDTD_E_INVALID, "src_tau must be > 0");
    if (p->nprobe < 0 || p->nprobe > GFDTD_MAX_PROBES)
        return fail(GFDTD_E_INVALID, "nprobe %d outside 0..%d", p->nprobe,
                    GFDTD_MAX_PROBES);
    if (p->nprobe > 0 && !p->probe_cells)
        return fail(GFDTD_E_INVALID, "probe_cells missing");
    for (int q = 0; q < p->nprobe; ++q)
        if (p->probe_cells[q] < 0 || p->probe_cells[q] >= p->nz)
            return fail(GFDTD_E_INVALID, "probe %d at %lld outside the grid", q,
                        (long long)p->probe_cells[q]);
    if (p->nfreq < 0 || (p->nfreq > 0 && !p->omegas))
        return fail(GFDTD_E_INVALID, "bad nfreq / omegas");
    for (int f = 0; f < p->nfreq; ++f)
        if (!std::isfinite(p->omegas[f]))
            return fail(GFDTD_E_INVALID, "omegas[%d] not finite", f);
    if (p->flags & GFDTD_FLAG_TIME_WINDOW) {
        if (p->kind != GFDTD_MODULATION)
            return fail(GFDTD_E_UNSUPPORTED,
                        "a time window applies to a moving modulation only");
        if (std::isnan(p->t_on) || std::isnan(p->t_off))
            return fail(GFDTD_E_INVALID, "t_on / t_off must not be NaN");
        if (!finite_pos(p->eps_bg) || !finite_pos(p->mu_bg))
            return fail(GFDTD_E_INVALID, "eps_bg / mu_bg must be finite and > 0");
    }
    for (int64_t i = 0; i < p->nz; ++i)
        if ((p->init_d && !std::isfinite(p->init_d[i])) ||
            (p->init_b && !std::isfinite(p->init_b[i])))
            return fail(GFDTD_E_INVALID, "init_d/init_b[%lld] not finite",
                        (long long)i);
    return GFDTD_OK;
}

// ------------------------------------------------------ stability pre-flight

// Largest |eigenvalue| over theta of the one-step amplification matrix of
// the scheme in a uniform medium with eps' mu' = n2 (Section 5, App. A).
// A plane wave D_k = D exp(i theta k), B_{k+1/2} = B exp(i theta (k+1/2))
// is pushed through (10c), (10a), (10d), (10b) with the Table 1 terms.
// The theta-dependent phase factors are computed once per scan.
namespace {
using cd = std::complex<double>;
struct ThetaFactors {
    cd curl, bbar, dlt, dbar;
};

std::vector<ThetaFactors> theta_factors(bool colA, int ntheta)
{
    std::vector<ThetaFactors> f(ntheta);
    for (int t = 1; t <= ntheta; ++t) {
        const double th = M_PI * t / ntheta;
        const cd h = std::polar(1.0, 0.5 * th);          // e^{i th/2}
        const cd e1 = h * h;                             // e^{i th}
        ThetaFactors &x = f[t - 1];
        x.curl = h - 1.0 / h;
        x.bbar = colA ? 0.5 * (1.0 / h + 1.0 / (h * e1)) : 0.5 * (h * e1 + h);
        x.dlt = colA ? 1.0 - 1.0 / e1 : e1 - 1.0;
        x.dbar = 0.5 * (h + 1.0 / h);
    }
    return f;
}

double spectral_radius(double n2, double S, double beta, int kind,
                       const std::vector<ThetaFactors> &tf)
{
    double aE, aH, bE, bH;
    if (kind == GFDTD_MATTER) {
        const double g = (1.0 - beta * beta) / (n2 - beta * beta);
        aE = g;          // the eigenvalues depend on aE aH = g^2 n2 only
        aH = g * n2;
        bE = bH = g * beta;
    } else {
        aE = 1.0 / n2;
        aH = 1.0;
        bE = bH = beta;
    }
    double best = 0.0;
    for (const ThetaFactors &x : tf) {
        cd G[2][2];
        for (int col = 0; col < 2; ++col) {
            const cd D = col == 0 ? 1.0 : 0.0;
            const cd B = col == 1 ? 1.0 : 0.0;
            const cd Es = aE * D - bE * x.bbar * B;
            const cd Bn = B - S * x.curl * Es - beta * S * x.dlt * B;
            const cd Hs = aH * Bn - bH * x.dbar * D;
            const cd Dn = D - S * x.curl * Hs - beta * S * x.dlt * D;
            G[0][col] = Dn;
            G[1][col] = Bn;
        }
        const cd tr = G[0][0] + G[1][1];
        const cd det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
        const cd disc = std::sqrt(tr * tr - 4.0 * det);
        best = std::max(best, std::max(std::abs(0.5 * (tr + disc)),
                                       std::abs(0.5 * (tr - disc))));
    }
    return best;
}
}  // namespace

// The one-step matrix depends on the medium only through eps' mu' (for a
// modulation through 1/(eps mu) and for matter through g), so distinct
// products are scanned: all of them when few, else the two extremes and
// 30 quantiles between them.
gfdtd_status preflight(const gfdtd_problem *p, double *growth)
{
    // The distinct products, collected in one pass while there are at most
    // 32 of them (piecewise-constant profiles: no sort of the whole grid),
    // else sorted and deduplicated.
    std::vector<double> n2;
    bool few = true;
    auto add = [&](double v) {
        if (few && std::find(n2.begin(), n2.end(), v) == n2.end()) {
            n2.push_back(v);
            few = n2.size() <= 32;
        }
    };
    for (int64_t i = 0; i < p->nz && few; ++i)
        add(p->eps_rest[i] * p->mu_rest[i]);
    if (p->flags & GFDTD_FLAG_TIME_WINDOW)
        add(p->eps_bg * p->mu_bg);
    if (!few) {
        n2.resize(p->nz);
        for (int64_t i = 0; i < p->nz; ++i)
            n2[i] = p->eps_rest[i] * p->mu_rest[i];
        if (p->flags & GFDTD_FLAG_TIME_WINDOW)
            n2.push_back(p->eps_bg * p->mu_bg);
    }
    std::sort(n2.begin(), n2.end());
    n2.erase(std::unique(n2.begin(), n2.end()), n2.end());
    std::vector<double> pick;
    if (n2.size() <= 32) {
        pick = n2;
    } else {
        for (int q = 0; q < 32; ++q)
            pick.push_back(n2[(size_t)((n2.size() - 1) * (double)q / 31.0)]);
    }
    const std::vector<ThetaFactors> tf = theta_factors(p->beta >= 0.0, 512);
    double g = 0.0;
    for (double v : pick)
        g = std::max(g, spectral_radius(v, p->courant, p->beta, p->kind, tf));
    if (growth)
        *growth = g;
    if (g > 1.0 + 1e-9 && !(p->flags & GFDTD_FLAG_ALLOW_UNSTABLE))
        return fail(GFDTD_E_UNSTABLE,
                    "pre-flight: amplification factor %.12g > 1 (beta %.4g, "
                    "S %.4g, largest eps'mu' %.4g)",
                    g, p->beta, p->courant, n2.back());
    return GFDTD_OK;
}

// ------------------------------------------------------------------ layout

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t Carver::take(size_t bytes)
{
    off = round_up(off, 256);
    const size_t r = off;
    off += round_up(bytes, 256);
    return r;
}

int64_t source_samples(const gfdtd_problem *p, int64_t steps)
{
    if (p->src_amp == 0.0 || steps <= 0)
        return 0;
    // largest n <= steps with n S <= t_off, with the same FP test as the
    // per-step rule
    double est = std::floor(p->src_t_off / p->courant);
    int64_t n = est < 0 ? 0 : (int64_t)std::min<double>(est, (double)steps);
    while (n < steps && (double)(n + 1) * p->courant <= p->src_t_off)
        ++n;
    while (n > 0 && !((double)n * p->courant <= p->src_t_off))
        --n;
    return n;
}

int64_t field_cells(int64_t nz) { return (int64_t)round_up((size_t)(nz + 2 * kPad), 64); }

void carve_run(Carver &cv, const gfdtd_problem *p, int64_t steps, RunLayout &L)
{
    const size_t w = p->precision == GFDTD_F32 ? 4 : 8;
    const size_t nz = (size_t)p->nz;
    L.eps = cv.take(nz * 8);
    L.mu = cv.take(nz * 8);
    L.cE = cv.take(nz * w);
    L.cH = cv.take(nz * w);
    L.gB = p->kind == GFDTD_MATTER ? cv.take(nz * w) : 0;
    L.murL = cv.take(nz * 8);
    L.murR = cv.take(nz * 8);
    L.nsrc = source_samples(p, steps);
    L.src = cv.take((size_t)std::max<int64_t>(L.nsrc, 1) * 8);
    L.probes = cv.take((size_t)std::max(p->nprobe, 1) * 8);
    L.omegas = cv.take((size_t)std::max(p->nfreq, 1) * 8);
    L.trace = cv.take((size_t)std::max<int64_t>((int64_t)p->nprobe * steps, 1) * 8);
    L.dft = cv.take((size_t)std::max(p->nprobe * p->nfreq, 1) * 16);
    const size_t fb = (size_t)field_cells(p->nz) * w;
    for (int f = 0; f < 4; ++f)
        L.field[f] = cv.take(fb);
    L.has_init_d = p->init_d != nullptr;
    L.has_init_b = p->init_b != nullptr;
    L.init_d = L.has_init_d ? cv.take(nz * 8) : 0;
    L.init_b = L.has_init_b ? cv.take(nz * 8) : 0;
}

RunHost make_run_host(const gfdtd_problem &p, int64_t steps)
{
    RunHost r;
    r.p = p;
    r.steps = steps;
    r.eps.assign(p.eps_rest, p.eps_rest + p.nz);
    r.mu.assign(p.mu_rest, p.mu_rest + p.nz);
    r.probes.assign(p.probe_cells, p.probe_cells + p.nprobe);
    r.omegas.assign(p.omegas, p.omegas + p.nfreq);
    if (p.init_d)
        r.init_d.assign(p.init_d, p.init_d + p.nz);
    if (p.init_b)
        r.init_b.assign(p.init_b, p.init_b + p.nz);
    r.p.eps_rest = r.eps.data();
    r.p.mu_rest = r.mu.data();
    r.p.probe_cells = r.probes.data();
    r.p.omegas = r.omegas.data();
    r.p.init_d = p.init_d ? r.init_d.data() : nullptr;
    r.p.init_b = p.init_b ? r.init_b.data() : nullptr;
    return r;
}

hipError_t upload_run_inputs(char *base, const RunHost &r, hipStream_t stream)
{
    const size_t nz = (size_t)r.p.nz;
    hipError_t e;
    if ((e = hipMemcpyAsync(base + r.L.eps, r.eps.data(), nz * 8, hipMemcpyHostToDevice, stream)) ||
        (e = hipMemcpyAsync(base + r.L.mu, r.mu.data(), nz * 8, hipMemcpyHostToDevice, stream)))
        return e;
    if (r.p.nprobe &&
        (e = hipMemcpyAsync(base + r.L.probes, r.probes.data(), r.probes.size() * 8,
                            hipMemcpyHostToDevice, stream)))
        return e;
    if (r.p.nfreq &&
        (e = hipMemcpyAsync(base + r.L.omegas, r.omegas.data(), r.omegas.size() * 8,
                            hipMemcpyHostToDevice, stream)))
        return e;
    if (r.L.has_init_d &&
        (e = hipMemcpyAsync(base + r.L.init_d, r.init_d.data(), nz * 8,
                            hipMemcpyHostToDevice, stream)))
        return e;
    if (r.L.has_init_b &&
        (e = hipMemcpyAsync(base + r.L.init_b, r.init_b.data(), nz * 8,
                            hipMemcpyHostToDevice, stream)))
        return e;
    return hipSuccess;
}

size_t table_bytes(int nruns, int64_t max_tiles)
{
    Carver cv;
    cv.take((size_t)nruns * sizeof(RunDesc));
    cv.take((size_t)std::max<int64_t>(max_tiles, 1) * sizeof(TileRef));
    cv.take((size_t)nruns * sizeof(PrepDesc));
    cv.take((size_t)nruns * sizeof(DftDesc));
    return cv.off;
}

// Upper bound of wave tiles of one run for any tiling (C >= 4, at least
// one owned lane).
int64_t max_tiles_of(int64_t nz) { return nz / 4 + 1; }

// Runs of one (precision, kind, ends) group in launch order, longest first
// (stable), split into the parts whose launches go to separate streams.  A
// launch ends with a drain in which its last waves leave most of the GPU
// idle, and the next launch of the same runs cannot start before it ends.
// A large group is therefore split into two halves (alternate runs, so both
// keep long runs to the end), each with its own tables, whose launches are
// issued to two streams: one half's waves fill the other's drain.  Measured
// on 4096 crystal runs: FP32 3.42e12 -> 3.71e12 cell-updates/s, FP64
// 2.14e12 -> 2.22e12; four parts were slower than two.  Smaller batches
// gain more (their launches are shorter, so the drain is a larger share):
// 128 runs of 2.7 M cells in all, 9600 steps, FP32 1.71e12 -> 2.37e12, and
// 16 runs of 0.31 M cells 5.2e11 -> 5.4e11.  Groups under kPartCells cells
// stay whole.
constexpr int kParts = 2;
static_assert(kParts == 2, "parts above 0 share the one second stream");
constexpr int64_t kPartCells = (int64_t)1 << 18;

template <typename StepsOf>
std::vector<std::vector<int>> stream_parts(std::vector<int> members, int64_t cells,
                                           bool allow, StepsOf steps_of)
{
    std::stable_sort(members.begin(), members.end(),
                     [&](int a, int b) { return steps_of(a) > steps_of(b); });
    const int n = (allow && members.size() >= 2 && cells >= kPartCells) ? kParts : 1;
    std::vector<std::vector<int>> parts(n);
    for (size_t m = 0; m < members.size(); ++m)
        parts[m % n].push_back(members[m]);
    return parts;
}

// --------------------------------------------------------------- tiling

// Tiling defaults from measurements on MI355X, crystal runs split over two
// streams (cell-updates/s, every run live unless stated):
// - from 8 M cells, 16 cells per lane and 48 steps per launch (FP32
//   3.43-3.63e12 from 11 M cells up; on the full 4096-run pass FP64 ran 2 %
//   faster at 16 than at 12 cells per lane, 2.32e12 against 2.28e12);
// - from 4 M to 8 M cells, 8 and 48 (5.3 M cells: FP32 2.77e12 against
//   2.26e12 at 16 cells per lane, FP64 2.22e12 against 1.86e12);
// - below 4 M cells, 4 and 24: more, narrower tiles keep more SIMDs busy.
void choose_tiling(int precision, const gfdtd_exec *ex, int64_t max_steps,
                   int64_t total_cells, bool ring, int &C, int &T, int &G, int &K)
{
    const int variant = ex ? ex->variant : GFDTD_VARIANT_AUTO;
    (void)precision;
    const bool small = total_cells < (int64_t)4 << 20;
    const bool mid = !small && total_cells < (int64_t)8 << 20;
    C = (ex && ex->cells_per_lane) ? ex->cells_per_lane : (small ? 4 : mid ? 8 : 16);
    if (variant == GFDTD_VARIANT_STEP)
        T = 1;
    else if (ex && ex->block_steps > 0)
        T = ex->block_steps;
    else
        T = small ? 24 : 48;
    if (max_steps > 0 && T > max_steps)
        T = (int)std::max<int64_t>(1, max_steps);
    G = (ex && ex->tile_waves > 0) ? ex->tile_waves : 1;
    if (ring || variant == GFDTD_VARIANT_STEP)
        G = 1;                           // rings and single steps: one-wave tiles
    K = (ex && ex->exchange_steps > 0) ? ex->exchange_steps : 8;
}

// Halo lanes of a T-step block.  Cells next to a wave edge lose their
// outside neighbour (the lane shift brings in zero), and the error spreads
// by the reach of one step: for column a (beta >= 0) D by 2 cells a step
// upwind (left) plus 1 in the first step, B by 2, and 1 cell downwind; for
// column b the mirror: 1 cell left, 2 right.  A probe's E at the owned
// cell k also reads B at k-1, k-2 (column a) or k+1 (column b) after the
// last step, and the end condition at node nz-1 (which may be the first
// owned cell) reads D and B at nz-2.  The owned lanes must stay clear of
// all of it: 2T + 2 cells upwind for column a and T downwind; T + 1 cells
// left and 2T + 1 right for column b.
bool halo_lanes(double beta, int C, int T, int &hl, int &hr)
{
    auto lanes = [C](int cells) { return (cells + C - 1) / C; };
    if (beta >= 0.0) {
        hl = lanes(2 * T + 2);
        hr = lanes(T);
    } else {
        hl = lanes(T + 1);
        hr = lanes(2 * T + 1);
    }
    return hl + hr < kWave;
}

bool tile_geometry(double beta, int C, int T, int G, int K, TileGeom &g)
{
    g = TileGeom{};
    if (!halo_lanes(beta, C, T, g.hl, g.hr))
        return false;
    if (G <= 1) {
        g.own = (int64_t)(kWave - g.hl - g.hr) * C;
        return true;
    }
    if (G > kMaxTileWaves || K < 1)
        return false;
    // overlaps: the reach of K steps on each side, as the halos of a block
    int xl, xr;
    halo_lanes(beta, C, K, xl, xr);
    const int ov = xl + xr;
    // the lanes a wave hands over must stay valid between refreshes: clear
    // of the outer halos and of the wave's own far overlap
    if (xl * C > kXSlot || xr * C > kXSlot || g.hl + ov > kWave || g.hr + ov > kWave ||
        ov + std::max(xl, xr) > kWave)
        return false;
    g.G = G;
    g.xl = xl;
    g.xr = xr;
    g.xk = K;
    g.own = ((int64_t)kWave * G - (int64_t)(G - 1) * ov - g.hl - g.hr) * C;
    return true;
}

// A tile that holds a whole grid with open ends needs no field halo for
// its block depth: nothing outside the grid reaches a node inside, since
// the end condition rewrites D at nodes 0 and nz-1 and the ghost fill
// resets B beyond the ends from inside values every step.  The coefficient
// windows are not reset: each move of the profile shifts them one cell and
// brings an undefined cell in at the upwind wave edge, so that side holds
// the block's moves, at most ceil(|beta S| T) + 1, plus the two ghost cells
// the stencil and the probe averages read; the other side one lane.
bool whole_grid_geometry(const gfdtd_problem &p, int C, int T, int G, int K, TileGeom &g)
{
    g = TileGeom{};
    const int64_t moves = (int64_t)std::ceil(std::fabs(p.beta * p.courant) * T) + 1;
    const int up = (int)((moves + 2 + C - 1) / C);
    g.hl = p.beta >= 0.0 ? up : 1;
    g.hr = p.beta >= 0.0 ? 1 : up;
    int ov = 0;
    if (G > 1) {
        if (G > kMaxTileWaves || K < 1)
            return false;
        int xl, xr;
        halo_lanes(p.beta, C, K, xl, xr);
        ov = xl + xr;
        if (xl * C > kXSlot || xr * C > kXSlot || g.hl + ov > kWave || g.hr + ov > kWave ||
            ov + std::max(xl, xr) > kWave)
            return false;
        g.G = G;
        g.xl = xl;
        g.xr = xr;
        g.xk = K;
    } else if (g.hl + g.hr >= kWave) {
        return false;
    }
    g.own = ((int64_t)kWave * G - (int64_t)(G - 1) * ov - g.hl - g.hr) * C;
    return g.own >= p.nz;
}

bool run_geometry(const gfdtd_problem &p, int C, int T, int G, int K, TileGeom &g)
{
    if (p.abc != GFDTD_ABC_PERIODIC && whole_grid_geometry(p, C, T, G, K, g))
        return true;
    return tile_geometry(p.beta, C, T, G, K, g);
}

// ------------------------------------------------------------------- batch

gfdtd_status Batch::prepare(const gfdtd_problem *probs, const int64_t *steps_in,
                            int32_t count, const gfdtd_exec *ex, void *ws_,
                            size_t ws_bytes_, hipStream_t stream_)
{
    stream = stream_;
    ws = static_cast<char *>(ws_);
    ws_bytes = ws_bytes_;
    if (count < 0 || (count > 0 && (!probs || !steps_in)))
        return fail(GFDTD_E_INVALID, "bad batch arguments");
    if (ex && ex->struct_size < sizeof(gfdtd_exec))
        return fail(GFDTD_E_INVALID, "exec struct_size too small");
    if (ex && ex->cells_per_lane && ex->cells_per_lane != 4 &&
        ex->cells_per_lane != 8 && ex->cells_per_lane != 12 && ex->cells_per_lane != 16)
        return fail(GFDTD_E_INVALID, "cells_per_lane must be 4, 8, 12 or 16");
    if (ex && (ex->block_steps < 0 || ex->block_steps > 256))
        return fail(GFDTD_E_INVALID, "block_steps outside 0..256");
    if (ex && (ex->tile_waves < 0 || ex->tile_waves > kMaxTileWaves))
        return fail(GFDTD_E_INVALID, "tile_waves outside 0..%d", kMaxTileWaves);
    if (ex && (ex->exchange_steps < 0 || ex->exchange_steps > 16))
        return fail(GFDTD_E_INVALID, "exchange_steps outside 0..16");
    runs.resize(count);
    for (int i = 0; i < count; ++i) {
        gfdtd_status st = validate(&probs[i], steps_in[i]);
        if (st != GFDTD_OK)
            return fail(st, "run %d: %s", i, last_error());
        st = preflight(&probs[i], nullptr);
        if (st != GFDTD_OK)
            return fail(st, "run %d: %s", i, last_error());
        runs[i] = make_run_host(probs[i], steps_in[i]);
    }
    use_graph = ex ? ex->use_graph : -1;
    // groups by (precision, kind, ring)
    Carver cv;
    for (auto &r : runs)
        carve_run(cv, &r.p, r.steps, r.L);
    for (int g = 0; g < kGroups; ++g) {
        Group G;
        G.precision = group_precision(g);
        G.kind = group_kind(g);
        G.ring = group_ring(g);
        int64_t max_steps = 0, cells = 0;
        for (int i = 0; i < count; ++i)
            if (group_of(runs[i].p.precision, runs[i].p.kind, runs[i].p.abc) == g) {
                G.has_window = G.has_window || (runs[i].p.flags & GFDTD_FLAG_TIME_WINDOW);
                G.members.push_back(i);
                max_steps = std::max(max_steps, runs[i].steps);
                cells += runs[i].p.nz;
            }
        if (G.members.empty())
            continue;
        choose_tiling(G.precision, ex, max_steps, cells, G.ring, G.C, G.T, G.Gw, G.K);
        for (int i : G.members)
            runs[i].T = G.T;
        // the allocation-free entry point has no second stream, and a
        // captured pass puts every launch on one stream, where two halves
        // would only double the launches
        auto parts = stream_parts(G.members, cells, !no_alloc && use_graph != 1,
                                  [&](int i) { return runs[i].steps; });
        for (size_t q = 0; q < parts.size(); ++q) {
            Group H = G;
            H.members = parts[q];
            H.part = (int)q;
            int64_t maxt = 0;
            for (int i : H.members)
                maxt += max_tiles_of(runs[i].p.nz);
            H.table_off = cv.take(table_bytes((int)H.members.size(), maxt));
            groups.push_back(H);
        }
    }
    if (cv.off > ws_bytes)
        return fail(GFDTD_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, cv.off);
    if (count > 0 && !ws)
        return fail(GFDTD_E_INVALID, "workspace pointer is NULL");

    hipError_t e;
    // uploads
    for (auto &r : runs)
        if ((e = upload_run_inputs(ws, r, stream)))
            return hip_fail(e, "upload run inputs");
    // per-group descriptor tables
    for (auto &G : groups) {
        const int nr = (int)G.members.size();
        // longest runs first, so the live runs of any block are a prefix
        std::stable_sort(G.members.begin(), G.members.end(), [&](int a, int b) {
            return runs[a].steps > runs[b].steps;
        });
        G.host_pd.assign(nr, PrepDesc{});
        G.host_dd.assign(nr, DftDesc{});
        G.max_cells = 0;
        G.max_init = 0;
        G.max_field = 0;
        G.max_pf = 0;
        for (int m = 0; m < nr; ++m) {
            RunHost &r = runs[G.members[m]];
            RunDesc rd;
            TileGeom g0;
            g0.own = kWave - 2;
            fill_desc(r, G, g0, 0, rd, G.host_pd[m], G.host_dd[m]);
            G.max_cells = std::max<int64_t>(G.max_cells, std::max(r.p.nz, r.L.nsrc));
            if (r.L.has_init_d || r.L.has_init_b)
                G.max_init = std::max<int64_t>(G.max_init, r.p.nz);
            G.max_field = std::max<int64_t>(G.max_field, field_cells(r.p.nz));
            G.max_pf = std::max(G.max_pf, r.p.nprobe * r.p.nfreq);
        }
        Carver tc;
        tc.off = G.table_off;
        int64_t maxt = 0;
        for (int i : G.members)
            maxt += max_tiles_of(runs[i].p.nz);
        G.runs_off = tc.take((size_t)nr * sizeof(RunDesc));
        G.tiles_off = tc.take((size_t)std::max<int64_t>(maxt, 1) * sizeof(TileRef));
        G.prep_off = tc.take((size_t)nr * sizeof(PrepDesc));
        G.dft_off = tc.take((size_t)nr * sizeof(DftDesc));
        gfdtd_status st = build_tiles(G);
        if (st != GFDTD_OK)
            return st;
        if ((e = hipMemcpyAsync(ws + G.prep_off, G.host_pd.data(), nr * sizeof(PrepDesc),
                                hipMemcpyHostToDevice, stream)) ||
            (e = hipMemcpyAsync(ws + G.dft_off, G.host_dd.data(), nr * sizeof(DftDesc),
                                hipMemcpyHostToDevice, stream)))
            return hip_fail(e, "upload run tables");
        if ((e = launch_prep(reinterpret_cast<const PrepDesc *>(ws + G.prep_off), nr,
                             (int)std::min<int64_t>(G.max_cells, 1 << 30), stream)))
            return hip_fail(e, "launch set-up kernel");
    }
    if ((e = hipStreamSynchronize(stream)))
        return hip_fail(e, "prepare");
    for (auto &r : runs)
        cell_updates += (double)r.p.nz * (double)r.steps;
    count_launches();
    if (no_alloc)
        return GFDTD_OK;
    if ((e = hipEventCreate(&ev[0])) || (e = hipEventCreate(&ev[1])) ||
        (e = hipEventCreate(&ev[2])) || (e = hipEventCreate(&ev[3])))
        return hip_fail(e, "create events");
    bool two = false;
    for (auto &G : groups)
        two = two || G.part > 0;
    if (two && ((e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking)) ||
                (e = hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming)) ||
                (e = hipEventCreateWithFlags(&join_ev, hipEventDisableTiming))))
        return hip_fail(e, "create second stream");
    if (use_graph == 1 || (use_graph < 0 && auto_graph()))
        return build_graphs();
    return GFDTD_OK;
}

void Batch::count_launches()
{
    launches = 0;
    tiles_total = 0;
    for (auto &G : groups)
        for (int64_t b = 0; b < G.nblocks; ++b) {
            launches += G.has_window ? 2 : 1;
            tiles_total += live_tiles(G, b);
        }
}

// Run and tile tables of a group for its current (C, T); uploads them on
// the batch stream.
gfdtd_status Batch::build_tiles(Group &G)
{
    const int nr = (int)G.members.size();
    G.host_rd.assign(nr, RunDesc{});
    G.host_tiles.clear();
    G.blocks_of.assign(nr, 0);
    G.tiles_prefix.assign(nr + 1, 0);
    for (int m = 0; m < nr; ++m) {
        RunHost &r = runs[G.members[m]];
        r.T = G.T;
        TileGeom g;
        if (!run_geometry(r.p, G.C, G.T, G.Gw, G.K, g))
            return fail(GFDTD_E_INVALID,
                        "block of %d steps too deep for %d cells per lane "
                        "(%d-wave tiles, refresh every %d steps)",
                        G.T, G.C, G.Gw, G.K);
        const int64_t own = g.own;
        const int64_t nt = (r.p.nz + own - 1) / own;
        PrepDesc pd;
        DftDesc dd;
        fill_desc(r, G, g, 0, G.host_rd[m], pd, dd);
        for (int64_t t = 0; t < nt; ++t)
            G.host_tiles.push_back(make_tile_ref(r, G.host_rd[m], m, G.C, G.Gw, t));
        G.tiles_prefix[m + 1] = G.tiles_prefix[m] + nt;
        G.blocks_of[m] = (r.steps + G.T - 1) / G.T;
    }
    G.nblocks = nr ? G.blocks_of[0] : 0;
    hipError_t e;
    if ((e = hipMemcpyAsync(ws + G.runs_off, G.host_rd.data(), nr * sizeof(RunDesc),
                            hipMemcpyHostToDevice, stream)) ||
        (!G.host_tiles.empty() &&
         (e = hipMemcpyAsync(ws + G.tiles_off, G.host_tiles.data(),
                             G.host_tiles.size() * sizeof(TileRef), hipMemcpyHostToDevice,
                             stream))))
        return hip_fail(e, "upload run tables");
    return GFDTD_OK;
}

// ------------------------------------------------------------- autotuner

namespace {
struct TuneKey {
    int group, neg, runs_log2, cells_log2, steps_log2;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(group, neg, runs_log2, cells_log2, steps_log2) <
               std::tie(o.group, o.neg, o.runs_log2, o.cells_log2, o.steps_log2);
    }
};
struct TuneChoice {
    int C, T, G;
};
std::map<TuneKey, TuneChoice> g_tune_cache;
std::mutex g_tune_mutex;

int ilog2(double x) { return x < 1.0 ? 0 : (int)std::floor(std::log2(x)); }
}  // namespace

// Time `trial` blocks of each candidate (cells per lane C, steps per launch
// T) on the prepared runs and keep the fastest per cell-update; the result
// of a pass does not depend on the choice.  Choices are cached in memory by
// the group's precision, kind, sign mix and the size scales of its runs.
gfdtd_status Batch::autotune(int trial, gfdtd_exec *chosen)
{
    hipError_t e;
    gfdtd_status st;
    if (trial < 1)
        trial = 4;
    // trial timing events, destroyed on every return path
    struct Events {
        hipEvent_t t0 = nullptr, t1 = nullptr;
        ~Events()
        {
            if (t0)
                (void)hipEventDestroy(t0);
            if (t1)
                (void)hipEventDestroy(t1);
        }
    } evs;
    if ((e = hipEventCreate(&evs.t0)) || (e = hipEventCreate(&evs.t1)))
        return hip_fail(e, "create events");
    hipEvent_t t0 = evs.t0, t1 = evs.t1;
    // The parts of one (precision, kind, ends) group are consecutive in
    // `groups` and take one choice, timed with their launches on their own
    // streams as a pass issues them (with two streams, larger tiles win:
    // the other stream fills each launch's drain).
    for (size_t f0 = 0; f0 < groups.size();) {
        size_t f1 = f0 + 1;
        while (f1 < groups.size() && groups[f1].part > 0)
            ++f1;
        std::vector<Group *> fam;
        for (size_t g = f0; g < f1; ++g)
            fam.push_back(&groups[g]);
        f0 = f1;
        const Group &G = *fam[0];
        const bool split = side != nullptr && fam.size() > 1;
        double cells = 0.0, steps = 0.0;
        int neg = 0;
        size_t nmem = 0;
        for (Group *H : fam) {
            for (int i : H->members) {
                cells += (double)runs[i].p.nz;
                steps = std::max(steps, (double)runs[i].steps);
                neg |= runs[i].p.beta < 0.0 ? 2 : 1;
            }
            nmem += H->members.size();
        }
        const TuneKey key{G.precision * 4 + G.kind * 2 + (G.ring ? 1 : 0), neg,
                          ilog2((double)nmem), ilog2(cells), ilog2(steps)};
        auto apply = [&](int C, int T, int Gw) {
            for (Group *H : fam) {
                H->C = C;
                H->T = T;
                H->Gw = Gw;
                gfdtd_status s2 = build_tiles(*H);
                if (s2 != GFDTD_OK)
                    return s2;
            }
            return GFDTD_OK;
        };
        {
            std::lock_guard<std::mutex> lk(g_tune_mutex);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                if ((st = apply(it->second.C, it->second.T, it->second.G)) != GFDTD_OK)
                    return st;
                continue;
            }
        }
        auto fork = [&]() {
            if (!split)
                return hipSuccess;
            hipError_t x = hipEventRecord(fork_ev, stream);
            return x ? x : hipStreamWaitEvent(side, fork_ev, 0);
        };
        auto join = [&]() {
            if (!split)
                return hipSuccess;
            hipError_t x = hipEventRecord(join_ev, side);
            return x ? x : hipStreamWaitEvent(stream, join_ev, 0);
        };
        // blocks [from, to) of every part, in the order a pass issues them
        auto blocks = [&](int64_t from, int64_t to) {
            for (int64_t b = from; b < to; ++b)
                for (Group *H : fam) {
                    if (b >= H->nblocks)
                        continue;
                    hipStream_t hs = (split && H->part > 0) ? side : stream;
                    for (int w = 0; w < (H->has_window ? 2 : 1); ++w) {
                        hipError_t le = launch_tiles(
                            H->precision, H->kind, H->ring, w == 1, H->C, H->Gw,
                            reinterpret_cast<const RunDesc *>(ws + H->runs_off),
                            reinterpret_cast<const TileRef *>(ws + H->tiles_off), b, H->T,
                            live_tiles(*H, b), hs);
                        if (le)
                            return le;
                    }
                }
            return hipSuccess;
        };
        const int defC = G.C, defT = G.T, defG = G.Gw;
        int bestC = G.C, bestT = G.T, bestG = G.Gw;
        double best = 1e300, def_time = 1e300;
        const int Cs[] = {4, 8, 12, 16};
        const int Ts[] = {8, 16, 24, 32, 48, 64};
        const int nG = G.ring ? 1 : 2;
        const int Gs[] = {1, kMaxTileWaves};
        for (int gi = 0; gi < nG; ++gi)
        for (int C : Cs)
            for (int T : Ts) {
                const int Gw = Gs[gi];
                if ((double)T > steps && T != 8)
                    continue;
                bool ok = true;
                TileGeom tg;
                for (Group *H : fam)
                    for (int i : H->members)
                        ok = ok && run_geometry(runs[i].p, C, T, Gw, H->K, tg);
                if (!ok)
                    continue;
                if ((st = apply(C, T, Gw)) != GFDTD_OK)
                    return st;
                int64_t nblocks = 0;
                for (Group *H : fam)
                    nblocks = std::max(nblocks, H->nblocks);
                // every candidate is timed over about the same number of
                // steps (trial blocks of 48 steps), and a small group (a lone
                // run: launch-bound, short launches) over at least 1536, so
                // deeper blocks are not favoured by covering more steps or
                // by fewer, noisier launches; block 0 is not timed
                const int64_t span = (int64_t)trial * 48 * (cells < 4.0e6 ? 8 : 1);
                const int64_t nb = std::min<int64_t>(
                    std::max<int64_t>(2, (span + T - 1) / T) + 1, nblocks);
                if (nb < 1)
                    continue;
                // a lone run is timed from the middle of its run: its early
                // blocks (the source still on) are not typical of it; a
                // batch from its start, where every run is live
                const int64_t b0 = nmem == 1 ? std::max<int64_t>(0, (nblocks - nb) / 2) : 0;
                double upd = 0.0;
                for (Group *H : fam)
                    for (int64_t b = b0 + 1; b < b0 + nb; ++b)
                        for (size_t m = 0; m < H->members.size() && H->blocks_of[m] > b; ++m) {
                            const RunHost &r = runs[H->members[m]];
                            upd += (double)r.p.nz *
                                   (double)std::min<int64_t>(T, r.steps - b * (int64_t)T);
                        }
                for (Group *H : fam)
                    if ((e = launch_zero(reinterpret_cast<const PrepDesc *>(ws + H->prep_off),
                                         (int)H->members.size(), H->max_field, H->precision,
                                         stream)))
                        return hip_fail(e, "autotune trial");
                if ((e = fork()) || (e = blocks(b0, b0 + 1)) || (e = join()) ||
                    (e = hipEventRecord(t0, stream)) || (e = fork()) ||
                    (e = blocks(b0 + 1, b0 + nb)) || (e = join()))
                    return hip_fail(e, "autotune trial");
                float ms = 0.f;
                if ((e = hipEventRecord(t1, stream)) || (e = hipEventSynchronize(t1)) ||
                    (e = hipEventElapsedTime(&ms, t0, t1)))
                    return hip_fail(e, "autotune timing");
                const double per = upd > 0.0 ? ms / upd : (double)ms;
                if (C == defC && T == defT && Gw == defG)
                    def_time = per;
                if (per < best) {
                    best = per;
                    bestC = C;
                    bestT = T;
                    bestG = Gw;
                }
            }
        // keep the default unless a candidate is clearly faster (trial
        // timings carry a few per cent of noise)
        if (def_time < 1e300 && best > def_time / 1.03) {
            bestC = defC;
            bestT = defT;
            bestG = defG;
        }
        if ((st = apply(bestC, bestT, bestG)) != GFDTD_OK)
            return st;
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        g_tune_cache[key] = {bestC, bestT, bestG};
    }
    if ((e = hipStreamSynchronize(stream)))
        return hip_fail(e, "autotune");
    count_launches();
    if (graph_on) {
        for (int k = 0; k < 3; ++k) {
            if (execs[k])
                (void)hipGraphExecDestroy(execs[k]);
            if (graphs[k])
                (void)hipGraphDestroy(graphs[k]);
            execs[k] = nullptr;
            graphs[k] = nullptr;
        }
        graph_on = false;
        if ((st = build_graphs()) != GFDTD_OK)
            return st;
    }
    if (chosen && chosen->struct_size >= sizeof(gfdtd_exec) && !groups.empty()) {
        chosen->variant = GFDTD_VARIANT_TILED;
        chosen->cells_per_lane = groups[0].C;
        chosen->block_steps = groups[0].T;
        chosen->tile_waves = groups[0].Gw;
        chosen->exchange_steps = groups[0].K;
        chosen->use_graph = graph_on ? 1 : 0;
    }
    return GFDTD_OK;
}

void Batch::fill_desc(RunHost &r, const Group &G, const TileGeom &g, int64_t start_block,
                      RunDesc &rd, PrepDesc &pd, DftDesc &dd)
{
    fill_run_desc(ws, r, G.precision, g, start_block, rd, pd, dd);
}

TileRef make_tile_ref(const RunHost &r, const RunDesc &rd, int m, int C, int G, int64_t t)
{
    TileRef ref{m, (int32_t)t, 0, 0};
    // wave w's owned cells [lo, hi): k_tiles' x0, own_l and own_r
    const int ov = G > 1 ? rd.xl + rd.xr : 0;
    for (int w = 0; w < G; ++w) {
        const int64_t x0 = t * rd.own_cells - (int64_t)rd.hl * C + (int64_t)w * (kWave - ov) * C;
        const int own_l = w == 0 ? rd.hl : rd.xl;
        const int own_r = w == G - 1 ? kWave - rd.hr : kWave - rd.xr;
        const int64_t lo = x0 + (int64_t)own_l * C, hi = x0 + (int64_t)own_r * C;
        for (int64_t kp : r.probes)
            if (kp >= lo && kp < hi) {
                ref.probe_waves |= 1 << w;
                break;
            }
    }
    return ref;
}

void fill_run_desc(char *base, const RunHost &r, int precision, const TileGeom &g,
                   int64_t start_block, RunDesc &rd, PrepDesc &pd, DftDesc &dd)
{
    const size_t w = precision == GFDTD_F32 ? 4 : 8;
    const gfdtd_problem &p = r.p;
    std::memset(&rd, 0, sizeof rd);
    rd.nz = p.nz;
    rd.steps = r.steps;
    rd.start_block = start_block;
    rd.nsrc = r.L.nsrc;
    rd.src_cell = p.src_cell;
    rd.own_cells = g.own;
    rd.S = p.courant;
    rd.beta = p.beta;
    rd.bS = p.beta * p.courant;
    rd.hb = 0.5 * p.beta * p.courant;
    rd.neg = p.beta < 0.0;
    rd.hl = g.hl;
    rd.hr = g.hr;
    rd.xl = g.xl;
    rd.xr = g.xr;
    rd.xk = g.xk;
    rd.nprobe = p.nprobe;
    rd.abc = p.abc;
    rd.windowed = (p.flags & GFDTD_FLAG_TIME_WINDOW) ? 1 : 0;
    if (rd.windowed) {
        rd.t_on = p.t_on;
        rd.t_off = p.t_off;
        rd.cEb = p.courant / p.eps_bg;
        rd.cHb = p.courant / p.mu_bg;
        // background Mur coefficient (S u - 1)/(S u + 1), u = 1/n
        const double u = 1.0 / std::sqrt(p.eps_bg * p.mu_bg);
        rd.murB = (p.courant * u - 1.0) / (p.courant * u + 1.0);
    }
    for (int f = 0; f < 2; ++f) {
        rd.D[f] = base + r.L.field[f] + kPad * w;
        rd.B[f] = base + r.L.field[2 + f] + kPad * w;
    }
    rd.cE = base + r.L.cE;
    rd.cH = base + r.L.cH;
    rd.gB = p.kind == GFDTD_MATTER ? base + r.L.gB : nullptr;
    rd.murL = reinterpret_cast<const double *>(base + r.L.murL);
    rd.murR = reinterpret_cast<const double *>(base + r.L.murR);
    rd.src = reinterpret_cast<const double *>(base + r.L.src);
    rd.probes = reinterpret_cast<const int64_t *>(base + r.L.probes);
    rd.trace = reinterpret_cast<double *>(base + r.L.trace);

    std::memset(&pd, 0, sizeof pd);
    pd.nz = p.nz;
    pd.nsrc = r.L.nsrc;
    pd.S = p.courant;
    pd.beta = p.beta;
    pd.amp = p.src_amp;
    pd.omega = p.src_omega;
    pd.t0 = p.src_t0;
    pd.tau = p.src_tau;
    pd.phase = p.src_phase;
    pd.kind = p.kind;
    pd.precision = p.precision;
    pd.abc = p.abc;
    pd.eps = reinterpret_cast<const double *>(base + r.L.eps);
    pd.mu = reinterpret_cast<const double *>(base + r.L.mu);
    pd.cE = base + r.L.cE;
    pd.cH = base + r.L.cH;
    pd.gB = p.kind == GFDTD_MATTER ? base + r.L.gB : nullptr;
    pd.murL = reinterpret_cast<double *>(base + r.L.murL);
    pd.murR = reinterpret_cast<double *>(base + r.L.murR);
    pd.src = reinterpret_cast<double *>(base + r.L.src);
    pd.fields[0] = rd.D[0];
    pd.fields[1] = rd.D[1];
    pd.fields[2] = rd.B[0];
    pd.fields[3] = rd.B[1];
    pd.field_cells = field_cells(p.nz);
    pd.init_d = r.L.has_init_d ? reinterpret_cast<const double *>(base + r.L.init_d) : nullptr;
    pd.init_b = r.L.has_init_b ? reinterpret_cast<const double *>(base + r.L.init_b) : nullptr;

    std::memset(&dd, 0, sizeof dd);
    dd.steps = r.steps;
    dd.S = p.courant;
    dd.nprobe = p.nprobe;
    dd.nfreq = p.nfreq;
    dd.trace = rd.trace;
    dd.omegas = reinterpret_cast<const double *>(base + r.L.omegas);
    dd.out = reinterpret_cast<double *>(base + r.L.dft);
}

int Batch::live_tiles(const Group &G, int64_t b) const
{
    // members are sorted by step count, so the live ones form a prefix
    int lo = 0, hi = (int)G.members.size();
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (G.blocks_of[mid] > b)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (int)G.tiles_prefix[lo];
}

bool Batch::auto_graph() const
{
    // plain launches cost a few microseconds each; a graph pays off when
    // launches are many and each is short.  Not for a batch split over two
    // streams: a captured pass would run both halves on one stream
    for (auto &G : groups)
        if (G.part > 0)
            return false;
    double updates_per_launch = launches ? cell_updates / (double)launches : 0.0;
    return launches >= 64 && updates_per_launch < 2e7;
}

gfdtd_status Batch::enqueue_zero(hipStream_t s)
{
    for (auto &G : groups) {
        const PrepDesc *pd = reinterpret_cast<const PrepDesc *>(ws + G.prep_off);
        hipError_t e = launch_zero(pd, (int)G.members.size(), G.max_field, G.precision, s);
        if (!e && G.max_init > 0)
            e = launch_init(pd, (int)G.members.size(), G.max_init, G.precision, s);
        if (e)
            return hip_fail(e, "launch zero fill");
    }
    return GFDTD_OK;
}

// Stepping launches of every group, block by block.  With `fork` (and a
// second stream), groups of part 1 launch on the second stream, which
// starts after the work already on `s` and is joined back to `s` at the end;
// otherwise everything goes to `s` in the same order.
gfdtd_status Batch::enqueue_steps(hipStream_t s, bool fork)
{
    hipError_t e;
    fork = fork && side;
    if (fork && ((e = hipEventRecord(fork_ev, s)) || (e = hipStreamWaitEvent(side, fork_ev, 0))))
        return hip_fail(e, "fork second stream");
    int64_t nb = 0;
    for (auto &G : groups)
        nb = std::max(nb, G.nblocks);
    gfdtd_status st = GFDTD_OK;
    for (int64_t b = 0; b < nb && st == GFDTD_OK; ++b)
        for (auto &G : groups) {
            if (b >= G.nblocks)
                continue;
            hipStream_t gs = (fork && G.part > 0) ? side : s;
            for (int w = 0; w < (G.has_window ? 2 : 1); ++w) {
                e = launch_tiles(G.precision, G.kind, G.ring, w == 1, G.C, G.Gw,
                                 reinterpret_cast<const RunDesc *>(ws + G.runs_off),
                                 reinterpret_cast<const TileRef *>(ws + G.tiles_off), b, G.T,
                                 live_tiles(G, b), gs);
                if (e) {
                    st = hip_fail(e, "launch step kernel");
                    break;
                }
            }
            if (st != GFDTD_OK)
                break;
        }
    // join even after a failed launch, so `s` orders everything issued
    if (fork && ((e = hipEventRecord(join_ev, side)) || (e = hipStreamWaitEvent(s, join_ev, 0))) &&
        st == GFDTD_OK)
        return hip_fail(e, "join second stream");
    return st;
}

gfdtd_status Batch::enqueue_dft(hipStream_t s)
{
    for (auto &G : groups) {
        hipError_t e = launch_dft(reinterpret_cast<const DftDesc *>(ws + G.dft_off),
                                  (int)G.members.size(), G.max_pf, s);
        if (e)
            return hip_fail(e, "launch DFT kernel");
    }
    return GFDTD_OK;
}

gfdtd_status Batch::build_graphs()
{
    hipError_t e;
    if (!cap_stream && (e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking)))
        return hip_fail(e, "create capture stream");
    for (int k = 0; k < 3; ++k) {
        if ((e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed)))
            return hip_fail(e, "begin capture");
        gfdtd_status st = k == 0 ? enqueue_zero(cap_stream)
                          : k == 1 ? enqueue_steps(cap_stream, false)
                                   : enqueue_dft(cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap_stream, &g);
        if (st != GFDTD_OK)
            return st;
        if (e2)
            return hip_fail(e2, "end capture");
        graphs[k] = g;
        if ((e = hipGraphInstantiate(&execs[k], g, nullptr, nullptr, 0)))
            return hip_fail(e, "instantiate graph");
    }
    graph_on = true;
    return GFDTD_OK;
}

gfdtd_status Batch::run()
{
    hipError_t e;
    if (ev[0] && (e = hipEventRecord(ev[0], stream)))
        return hip_fail(e, "record event");
    gfdtd_status st;
    if (graph_on) {
        if ((e = hipGraphLaunch(execs[0], stream)))
            return hip_fail(e, "launch zero graph");
    } else if ((st = enqueue_zero(stream)) != GFDTD_OK) {
        return st;
    }
    if (ev[1])
        (void)hipEventRecord(ev[1], stream);
    if (graph_on) {
        if ((e = hipGraphLaunch(execs[1], stream)))
            return hip_fail(e, "launch step graph");
    } else if ((st = enqueue_steps(stream, true)) != GFDTD_OK) {
        return st;
    }
    if (ev[2])
        (void)hipEventRecord(ev[2], stream);
    if (graph_on) {
        if ((e = hipGraphLaunch(execs[2], stream)))
            return hip_fail(e, "launch DFT graph");
    } else if ((st = enqueue_dft(stream)) != GFDTD_OK) {
        return st;
    }
    if (ev[3] && (e = hipEventRecord(ev[3], stream)))
        return hip_fail(e, "record event");
    ran = true;
    return GFDTD_OK;
}

void initial_fields(const RunHost &r, double *d, double *b)
{
    const int64_t nz = r.p.nz;
    const bool f32 = r.p.precision == GFDTD_F32;
    const bool ring = r.p.abc == GFDTD_ABC_PERIODIC;
    auto fill = [&](const std::vector<double> &src, double *dst, int64_t n) {
        for (int64_t i = 0; i < nz; ++i) {
            const double v = (i < n && !src.empty()) ? src[i] : 0.0;
            dst[i] = f32 ? (double)(float)v : v;
        }
    };
    if (d)
        fill(r.init_d, d, nz);
    if (b)
        fill(r.init_b, b, ring ? nz : nz - 1);
}

gfdtd_status copy_results(const char *ws, const RunHost &r, const gfdtd_result *out_in,
                          hipStream_t stream, gfdtd_result *out)
{
    (void)out_in;
    hipError_t e;
    const gfdtd_problem &p = r.p;
    const int np = p.nprobe, nf = p.nfreq;
    std::vector<double> dft((size_t)np * nf * 2);
    if (np * nf > 0 &&
        (e = hipMemcpyAsync(dft.data(), ws + r.L.dft, dft.size() * 8,
                            hipMemcpyDeviceToHost, stream)))
        return hip_fail(e, "copy DFT");
    std::vector<double> trace;
    const bool want_trace = out->trace && (p.flags & GFDTD_FLAG_RECORD_TRACE);
    // The blow-up check reads the DFT: a non-finite trace value makes its
    // sums non-finite.  Without frequencies it reads the trace instead.
    if (np > 0 && r.steps > 0 && (want_trace || nf == 0)) {
        trace.resize((size_t)np * r.steps);
        if ((e = hipMemcpyAsync(trace.data(), ws + r.L.trace, trace.size() * 8,
                                hipMemcpyDeviceToHost, stream)))
            return hip_fail(e, "copy trace");
    }
    const size_t w = p.precision == GFDTD_F32 ? 4 : 8;
    std::vector<char> fd, fb;
    const int fin = (int)(((r.steps + r.T - 1) / r.T) & 1);   // buffer of the last write
    if (out->final_d || out->final_b) {
        fd.resize((size_t)p.nz * w);
        fb.resize((size_t)p.nz * w);
        const char *d = ws + r.L.field[fin] + kPad * w;
        const char *b = ws + r.L.field[2 + fin] + kPad * w;
        if ((e = hipMemcpyAsync(fd.data(), d, fd.size(), hipMemcpyDeviceToHost, stream)) ||
            (e = hipMemcpyAsync(fb.data(), b, fb.size(), hipMemcpyDeviceToHost, stream)))
            return hip_fail(e, "copy fields");
    }
    if ((e = hipStreamSynchronize(stream)))
        return hip_fail(e, "collect");
    bool finite = true;
    for (double v : dft)
        finite = finite && std::isfinite(v);
    for (double v : trace)
        finite = finite && std::isfinite(v);
    out->run_status = finite ? GFDTD_OK : GFDTD_E_BLOWUP;
    out->steps_done = r.steps;
    if (out->dft_re && out->dft_im)
        for (int i = 0; i < np * nf; ++i) {
            out->dft_re[i] = dft[2 * i];
            out->dft_im[i] = dft[2 * i + 1];
        }
    if (want_trace && !trace.empty())
        std::memcpy(out->trace, trace.data(), trace.size() * 8);
    auto conv = [&](const std::vector<char> &src, double *dst, int64_t n) {
        for (int64_t i = 0; i < n; ++i)
            dst[i] = w == 4 ? (double)reinterpret_cast<const float *>(src.data())[i]
                            : reinterpret_cast<const double *>(src.data())[i];
    };
    if (r.steps == 0) {
        initial_fields(r, out->final_d, out->final_b);
    } else {
        if (out->final_d)
            conv(fd, out->final_d, p.nz);
        if (out->final_b) {
            const bool ring = p.abc == GFDTD_ABC_PERIODIC;
            conv(fb, out->final_b, ring ? p.nz : p.nz - 1);
            if (!ring)
                out->final_b[p.nz - 1] = 0.0;
        }
    }
    return GFDTD_OK;
}

gfdtd_status Batch::collect(gfdtd_result *outs)
{
    if (!ran)
        return fail(GFDTD_E_INVALID, "collect before run");
    if (!outs && !runs.empty())
        return fail(GFDTD_E_INVALID, "outs is NULL");
    hipError_t e;
    if ((e = hipStreamSynchronize(stream)))
        return hip_fail(e, "synchronize");
    for (size_t i = 0; i < runs.size(); ++i) {
        if (outs[i].struct_size < sizeof(gfdtd_result))
            return fail(GFDTD_E_INVALID, "result %zu struct_size too small", i);
        gfdtd_status st = copy_results(ws, runs[i], nullptr, stream, &outs[i]);
        if (st != GFDTD_OK)
            return st;
    }
    return GFDTD_OK;
}

void Batch::stats(gfdtd_stats *s) const
{
    s->cells_per_lane = groups.empty() ? 0 : groups[0].C;
    s->block_steps = groups.empty() ? 0 : groups[0].T;
    s->tile_waves = groups.empty() ? 0 : groups[0].Gw;
    s->exchange_steps = groups.empty() ? 0 : groups[0].K;
    s->graph = graph_on ? 1 : 0;
    // a captured pass keeps every launch on one stream
    s->streams = (side && !graph_on) ? 2 : 1;
    s->reserved = 0;
    s->launches = launches;
    s->tiles = tiles_total;
    s->cell_updates = cell_updates;
    s->step_ms = 0.0;
    s->pass_ms = 0.0;
    if (ran && ev[3] && hipEventSynchronize(ev[3]) == hipSuccess) {
        float a = 0.f, b = 0.f;
        (void)hipEventElapsedTime(&a, ev[1], ev[2]);
        (void)hipEventElapsedTime(&b, ev[0], ev[3]);
        s->step_ms = a;
        s->pass_ms = b;
    }
}

Batch::~Batch()
{
    // kernels or uploads of this batch may still be running on its stream
    // (a destroy without collect, or an error path): the caller frees the
    // workspace, and this object the upload sources, right after
    if (side)
        (void)hipStreamSynchronize(side);
    if (stream)
        (void)hipStreamSynchronize(stream);
    for (int k = 0; k < 3; ++k) {
        if (execs[k])
            (void)hipGraphExecDestroy(execs[k]);
        if (graphs[k])
            (void)hipGraphDestroy(graphs[k]);
    }
    if (cap_stream)
        (void)hipStreamDestroy(cap_stream);
    if (side)
        (void)hipStreamDestroy(side);
    if (fork_ev)
        (void)hipEventDestroy(fork_ev);
    if (join_ev)
        (void)hipEventDestroy(join_ev);
    for (auto &x : ev)
        if (x)
            (void)hipEventDestroy(x);
}

}  // namespace gfdtd

// ======================================================================
// C-ABI
// ======================================================================
using namespace gfdtd;

extern "C" {

const char *gfdtd_status_str(gfdtd_status s)
{
    switch (s) {
    case GFDTD_OK: return "ok";
    case GFDTD_E_INVALID: return "invalid argument";
    case GFDTD_E_UNSTABLE: return "unstable (pre-flight)";
    case GFDTD_E_NOMEM: return "workspace or pool too small";
    case GFDTD_E_DEVICE: return "device error";
    case GFDTD_E_NOT_READY: return "not ready";
    case GFDTD_E_BLOWUP: return "non-finite probe values";
    case GFDTD_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *gfdtd_last_error(void) { return last_error(); }

gfdtd_status gfdtd_check(const gfdtd_problem *p, double *max_growth)
{
    clear_error();
    gfdtd_status st = validate(p, 0);
    if (st != GFDTD_OK)
        return st;
    return preflight(p, max_growth);
}

gfdtd_status gfdtd_result_sizes(const gfdtd_problem *p, int64_t steps,
                                size_t *trace_len, size_t *dft_len)
{
    clear_error();
    gfdtd_status st = validate(p, steps);
    if (st != GFDTD_OK)
        return st;
    if (trace_len)
        *trace_len = (size_t)p->nprobe * (size_t)steps;
    if (dft_len)
        *dft_len = (size_t)p->nprobe * (size_t)p->nfreq;
    return GFDTD_OK;
}

gfdtd_status gfdtd_batch_workspace_bytes(const gfdtd_problem *probs,
                                         const int64_t *steps, int32_t count,
                                         size_t *bytes)
{
    clear_error();
    if (!bytes || count < 0 || (count > 0 && (!probs || !steps)))
        return fail(GFDTD_E_INVALID, "bad arguments");
    Carver cv;
    std::vector<int> members[kGroups];
    int64_t cells[kGroups] = {};
    for (int i = 0; i < count; ++i) {
        gfdtd_status st = validate(&probs[i], steps[i]);
        if (st != GFDTD_OK)
            return fail(st, "run %d: %s", i, last_error());
        RunLayout L;
        carve_run(cv, &probs[i], steps[i], L);
        const int g = group_of(probs[i].precision, probs[i].kind, probs[i].abc);
        members[g].push_back(i);
        cells[g] += probs[i].nz;
    }
    // the tables of every stream part (a batch that keeps a group whole
    // needs no more than this)
    for (int g = 0; g < kGroups; ++g)
        for (auto &part : stream_parts(members[g], cells[g], true,
                                       [&](int i) { return steps[i]; })) {
            if (part.empty())
                continue;
            int64_t maxt = 0;
            for (int i : part)
                maxt += max_tiles_of(probs[i].nz);
            cv.take(table_bytes((int)part.size(), maxt));
        }
    *bytes = cv.off;
    return GFDTD_OK;
}

gfdtd_status gfdtd_workspace_bytes(const gfdtd_problem *p, int64_t steps, size_t *bytes)
{
    return gfdtd_batch_workspace_bytes(p, &steps, 1, bytes);
}

gfdtd_status gfdtd_batch_prepare(const gfdtd_problem *probs, const int64_t *steps,
                                 int32_t count, const gfdtd_exec *exec, void *ws,
                                 size_t ws_bytes, void *stream, gfdtd_batch **out)
{
    clear_error();
    if (!out)
        return fail(GFDTD_E_INVALID, "out is NULL");
    *out = nullptr;
    std::unique_ptr<Batch> b(new Batch);
    gfdtd_status st = b->prepare(probs, steps, count, exec, ws, ws_bytes,
                                 static_cast<hipStream_t>(stream));
    if (st != GFDTD_OK)
        return st;
    *out = reinterpret_cast<gfdtd_batch *>(b.release());
    return GFDTD_OK;
}

gfdtd_status gfdtd_batch_run(gfdtd_batch *b)
{
    clear_error();
    if (!b)
        return fail(GFDTD_E_INVALID, "batch is NULL");
    return reinterpret_cast<Batch *>(b)->run();
}

gfdtd_status gfdtd_batch_collect(gfdtd_batch *b, gfdtd_result *outs)
{
    clear_error();
    if (!b)
        return fail(GFDTD_E_INVALID, "batch is NULL");
    return reinterpret_cast<Batch *>(b)->collect(outs);
}

gfdtd_status gfdtd_batch_stats(const gfdtd_batch *b, gfdtd_stats *s)
{
    clear_error();
    if (!b || !s || s->struct_size < sizeof(gfdtd_stats))
        return fail(GFDTD_E_INVALID, "bad arguments");
    reinterpret_cast<const Batch *>(b)->stats(s);
    return GFDTD_OK;
}

gfdtd_status gfdtd_batch_autotune(gfdtd_batch *b, int32_t trial_blocks,
                                  gfdtd_exec *chosen)
{
    clear_error();
    if (!b)
        return fail(GFDTD_E_INVALID, "batch is NULL");
    return reinterpret_cast<Batch *>(b)->autotune(trial_blocks, chosen);
}

void gfdtd_batch_destroy(gfdtd_batch *b) { delete reinterpret_cast<Batch *>(b); }

gfdtd_status gfdtd_solve_batch(const gfdtd_problem *probs, const int64_t *steps,
                               int32_t count, void *ws, size_t ws_bytes, void *stream,
                               gfdtd_result *outs)
{
    gfdtd_batch *b = nullptr;
    gfdtd_status st = gfdtd_batch_prepare(probs, steps, count, nullptr, ws, ws_bytes,
                                          stream, &b);
    if (st == GFDTD_OK)
        st = gfdtd_batch_run(b);
    if (st == GFDTD_OK)
        st = gfdtd_batch_collect(b, outs);
    gfdtd_batch_destroy(b);
    return st;
}

gfdtd_status gfdtd_solve(const gfdtd_problem *p, int64_t steps, void *ws,
                         size_t ws_bytes, void *stream, gfdtd_result *out)
{
    return gfdtd_solve_batch(p, &steps, 1, ws, ws_bytes, stream, out);
}

}  // extern "C"
