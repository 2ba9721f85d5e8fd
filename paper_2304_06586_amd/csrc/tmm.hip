// Batched transfer-matrix evaluation of moving multilayers (App. B.3): one
// thread per (stack, frequency), FP64 complex 2x2 chains.  The kernel reads
// the rest parameters of every layer and does all of the method's
// arithmetic; the host only validates, packs the layer tables and copies.
//
// State vector: the star amplitudes (A, B) of the forward and backward
// waves in a layer.  Across the interface m|m+1, continuity of E* = A + B
// and H* = (A - B)/eta gives
//     (A, B)_{m+1} = [[a, b], [b, a]] (A, B)_m,
//     a = (1 + r)/2, b = (1 - r)/2, r = eta_{m+1} / eta_m;
// through layer m of lab width w the forward wave gains the phase
// n_m w+_m w and the backward one -n_m w-_m w, with the Doppler frequencies
// w+-_m = omega (1 - n_0 beta) / (1 -+ n_m beta).  From the total matrix M
// the star reflection and transmission are -M10/M11 and det M / M11, with
// det M carried as the product of the factors' determinants (r per
// interface, the two phases per layer): forming it from the entries of M
// cancels catastrophically where M grows (a long crystal's stopband).  The
// lab-frame E-field ratios follow by the factors (1 - n_0 beta)/(1 + n_0
// beta) and (1 - n_0 beta)/(1 - n_{N-1} beta).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gfdtd.h"
#include "gfdtd_internal.h"
#include "runtime.h"

namespace gfdtd {

struct TmmDesc {
    int64_t layer0;        // first layer's index in the layer tables
    int32_t nlayers;
    int32_t pad0;
    double beta;
};

struct cplx {
    double re, im;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

__device__ __forceinline__ cplx cdiv(cplx a, cplx b)
{
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

__global__ __launch_bounds__(256) void k_tmm(const TmmDesc *__restrict__ stacks,
                                             const double *__restrict__ eps,
                                             const double *__restrict__ mu,
                                             const double *__restrict__ width,
                                             const double *__restrict__ omegas,
                                             int nstacks, int nomega,
                                             double *__restrict__ out_t,
                                             double *__restrict__ out_g)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nstacks * nomega)
        return;
    const int s = (int)(idx / nomega);
    const int f = (int)(idx % nomega);
    const TmmDesc d = stacks[s];
    const double beta = d.beta;
    const double omega = omegas[f];
    const double *e = eps + d.layer0;
    const double *u = mu + d.layer0;
    const double *w = width + d.layer0;     // width of layer m at w[m]

    const double n0 = sqrt(e[0] * u[0]);
    const double inv = omega * (1.0 - n0 * beta);
    cplx m00 = {1.0, 0.0}, m01 = {0.0, 0.0}, m10 = {0.0, 0.0}, m11 = {1.0, 0.0};
    cplx det = {1.0, 0.0};
    double eta = sqrt(u[0] / e[0]);
    double nm = n0;
    for (int m = 0; m < d.nlayers - 1; ++m) {
        if (m >= 1) {                         // propagate through layer m
            const double wp = inv / (1.0 - nm * beta);
            const double wm = inv / (1.0 + nm * beta);
            double sp, cp, sm, cm;
            sincos(nm * wp * w[m], &sp, &cp);
            sincos(-nm * wm * w[m], &sm, &cm);
            const cplx pp = {cp, sp}, pm = {cm, sm};
            m00 = cmul(pp, m00);
            m01 = cmul(pp, m01);
            m10 = cmul(pm, m10);
            m11 = cmul(pm, m11);
            det = cmul(det, cmul(pp, pm));
        }
        // interface m | m+1
        const double eta1 = sqrt(u[m + 1] / e[m + 1]);
        const double r = eta1 / eta;
        const double a = 0.5 * (1.0 + r), b = 0.5 * (1.0 - r);
        const cplx n00 = {a * m00.re + b * m10.re, a * m00.im + b * m10.im};
        const cplx n01 = {a * m01.re + b * m11.re, a * m01.im + b * m11.im};
        const cplx n10 = {b * m00.re + a * m10.re, b * m00.im + a * m10.im};
        const cplx n11 = {b * m01.re + a * m11.re, b * m01.im + a * m11.im};
        m00 = n00;
        m01 = n01;
        m10 = n10;
        m11 = n11;
        det = {det.re * r, det.im * r};
        eta = eta1;
        nm = sqrt(e[m + 1] * u[m + 1]);
    }
    const cplx ts = cdiv(det, m11);
    const cplx rs = cdiv({-m10.re, -m10.im}, m11);
    const double fg = (1.0 - n0 * beta) / (1.0 + n0 * beta);
    const double ft = (1.0 - n0 * beta) / (1.0 - nm * beta);
    out_t[2 * idx] = ts.re * ft;
    out_t[2 * idx + 1] = ts.im * ft;
    out_g[2 * idx] = rs.re * fg;
    out_g[2 * idx + 1] = rs.im * fg;
}

// ------------------------------------------------------------- host side

static gfdtd_status validate_stack(const gfdtd_tmm_stack *st, int i)
{
    auto pos = [](double x) { return std::isfinite(x) && x > 0.0; };
    if (st->struct_size < sizeof(gfdtd_tmm_stack))
        return fail(GFDTD_E_INVALID, "stack %d: struct_size too small", i);
    if (st->nlayers < 2)
        return fail(GFDTD_E_INVALID, "stack %d: nlayers %d < 2", i, st->nlayers);
    if (!std::isfinite(st->beta) || std::fabs(st->beta) >= 1.0)
        return fail(GFDTD_E_INVALID, "stack %d: |beta| must be < 1", i);
    if (!st->eps || (st->nlayers > 2 && !st->widths))
        return fail(GFDTD_E_INVALID, "stack %d: eps / widths missing", i);
    for (int m = 0; m < st->nlayers; ++m) {
        const double mu = st->mu ? st->mu[m] : 1.0;
        if (!pos(st->eps[m]) || !pos(mu))
            return fail(GFDTD_E_INVALID, "stack %d layer %d: eps, mu must be > 0", i, m);
        if (std::fabs(st->beta) * std::sqrt(st->eps[m] * mu) >= 1.0)
            return fail(GFDTD_E_INVALID,
                        "stack %d layer %d: |beta| n >= 1 (no transfer matrix)", i, m);
    }
    for (int m = 0; m + 2 < st->nlayers; ++m)
        if (!std::isfinite(st->widths[m]) || st->widths[m] < 0.0)
            return fail(GFDTD_E_INVALID, "stack %d: width %d must be finite and >= 0", i, m);
    return GFDTD_OK;
}

namespace {
// Byte offsets of the tables in the workspace, and its total size.
struct TmmLayout {
    size_t desc = 0, eps = 0, mu = 0, width = 0, omegas = 0, t = 0, g = 0;
    size_t bytes = 0;
    int64_t layers = 0;
};

gfdtd_status tmm_layout(const gfdtd_tmm_stack *stacks, int32_t nstacks,
                        int32_t nomega, TmmLayout &L)
{
    if (nstacks < 0 || nomega < 0 || (nstacks > 0 && !stacks))
        return fail(GFDTD_E_INVALID, "bad stack arguments");
    L.layers = 0;
    for (int i = 0; i < nstacks; ++i) {
        gfdtd_status st = validate_stack(&stacks[i], i);
        if (st != GFDTD_OK)
            return st;
        L.layers += stacks[i].nlayers;
    }
    Carver cv;
    L.desc = cv.take((size_t)std::max(nstacks, 1) * sizeof(TmmDesc));
    const size_t lb = (size_t)std::max<int64_t>(L.layers, 1) * 8;
    L.eps = cv.take(lb);
    L.mu = cv.take(lb);
    L.width = cv.take(lb);
    L.omegas = cv.take((size_t)std::max(nomega, 1) * 8);
    const size_t rb = (size_t)std::max<int64_t>((int64_t)nstacks * nomega, 1) * 16;
    L.t = cv.take(rb);
    L.g = cv.take(rb);
    L.bytes = cv.off;
    return GFDTD_OK;
}
}  // namespace

}  // namespace gfdtd

using namespace gfdtd;

namespace {
// device time of the calling thread's last k_tmm launch (HIP events on its
// stream), for gfdtd_tmm_kernel_ms
thread_local double g_tmm_kernel_ms = -1.0;
}  // namespace

extern "C" {

gfdtd_status gfdtd_tmm_workspace_bytes(const gfdtd_tmm_stack *stacks, int32_t nstacks,
                                       int32_t nomega, size_t *bytes)
{
    clear_error();
    if (!bytes)
        return fail(GFDTD_E_INVALID, "bytes is NULL");
    TmmLayout L;
    gfdtd_status st = tmm_layout(stacks, nstacks, nomega, L);
    if (st != GFDTD_OK)
        return st;
    *bytes = L.bytes;
    return GFDTD_OK;
}

gfdtd_status gfdtd_tmm(const gfdtd_tmm_stack *stacks, int32_t nstacks,
                       const double *omegas, int32_t nomega, void *ws_,
                       size_t ws_bytes, void *stream_, double *t, double *gamma)
{
    clear_error();
    TmmLayout L;
    gfdtd_status st = tmm_layout(stacks, nstacks, nomega, L);
    if (st != GFDTD_OK)
        return st;
    if (nomega > 0 && !omegas)
        return fail(GFDTD_E_INVALID, "omegas is NULL");
    for (int f = 0; f < nomega; ++f)
        if (!std::isfinite(omegas[f]))
            return fail(GFDTD_E_INVALID, "omegas[%d] not finite", f);
    const int64_t nres = (int64_t)nstacks * nomega;
    if (nres > 0 && (!t || !gamma))
        return fail(GFDTD_E_INVALID, "t / gamma is NULL");
    if (nres > ((int64_t)1 << 31) - 256)
        return fail(GFDTD_E_INVALID, "too many (stack, omega) pairs in one call");
    const size_t need = L.bytes;
    if (ws_bytes < need)
        return fail(GFDTD_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    if (nres == 0)
        return GFDTD_OK;
    char *ws = static_cast<char *>(ws_);
    if (!ws)
        return fail(GFDTD_E_INVALID, "workspace pointer is NULL");
    hipStream_t stream = static_cast<hipStream_t>(stream_);

    // pack the layer tables (widths at the index of their layer; the outer
    // layers' slots are unused)
    std::vector<TmmDesc> desc(nstacks);
    std::vector<double> eps(L.layers), mu(L.layers), width(L.layers, 0.0);
    int64_t o = 0;
    for (int i = 0; i < nstacks; ++i) {
        const gfdtd_tmm_stack &s = stacks[i];
        desc[i].layer0 = o;
        desc[i].nlayers = s.nlayers;
        desc[i].pad0 = 0;
        desc[i].beta = s.beta;
        for (int m = 0; m < s.nlayers; ++m) {
            eps[o + m] = s.eps[m];
            mu[o + m] = s.mu ? s.mu[m] : 1.0;
            if (m >= 1 && m + 1 < s.nlayers)
                width[o + m] = s.widths[m - 1];
        }
        o += s.nlayers;
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(ws + L.desc, desc.data(), desc.size() * sizeof(TmmDesc),
                            hipMemcpyHostToDevice, stream)) ||
        (e = hipMemcpyAsync(ws + L.eps, eps.data(), eps.size() * 8, hipMemcpyHostToDevice,
                            stream)) ||
        (e = hipMemcpyAsync(ws + L.mu, mu.data(), mu.size() * 8, hipMemcpyHostToDevice,
                            stream)) ||
        (e = hipMemcpyAsync(ws + L.width, width.data(), width.size() * 8,
                            hipMemcpyHostToDevice, stream)) ||
        (e = hipMemcpyAsync(ws + L.omegas, omegas, (size_t)nomega * 8,
                            hipMemcpyHostToDevice, stream)))
        return hip_fail(e, "upload stacks");
    const unsigned blocks = (unsigned)((nres + 255) / 256);
    // events bracketing the kernel alone; destroyed on every return path
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events()
        {
            if (a)
                (void)hipEventDestroy(a);
            if (b)
                (void)hipEventDestroy(b);
        }
    } ev;
    g_tmm_kernel_ms = -1.0;
    if ((e = hipEventCreate(&ev.a)) || (e = hipEventCreate(&ev.b)) ||
        (e = hipEventRecord(ev.a, stream)))
        return hip_fail(e, "transfer-matrix timing events");
    hipLaunchKernelGGL(k_tmm, dim3(blocks), dim3(256), 0, stream,
                       reinterpret_cast<const TmmDesc *>(ws + L.desc),
                       reinterpret_cast<const double *>(ws + L.eps),
                       reinterpret_cast<const double *>(ws + L.mu),
                       reinterpret_cast<const double *>(ws + L.width),
                       reinterpret_cast<const double *>(ws + L.omegas), nstacks, nomega,
                       reinterpret_cast<double *>(ws + L.t),
                       reinterpret_cast<double *>(ws + L.g));
    if ((e = hipGetLastError()) || (e = hipEventRecord(ev.b, stream)))
        return hip_fail(e, "launch transfer-matrix kernel");
    if ((e = hipMemcpyAsync(t, ws + L.t, (size_t)nres * 16, hipMemcpyDeviceToHost, stream)) ||
        (e = hipMemcpyAsync(gamma, ws + L.g, (size_t)nres * 16, hipMemcpyDeviceToHost,
                            stream)) ||
        (e = hipStreamSynchronize(stream)))
        return hip_fail(e, "transfer-matrix results");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess)
        g_tmm_kernel_ms = ms;
    return GFDTD_OK;
}

gfdtd_status gfdtd_tmm_kernel_ms(double *ms)
{
    clear_error();
    if (!ms)
        return fail(GFDTD_E_INVALID, "ms is NULL");
    if (g_tmm_kernel_ms < 0.0)
        return fail(GFDTD_E_INVALID, "no transfer-matrix kernel has run on this thread");
    *ms = g_tmm_kernel_ms;
    return GFDTD_OK;
}

}  // extern "C"
