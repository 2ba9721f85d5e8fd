// HIP kernels of the 2D (TE / TM) path, gfx950.
//
// The 2D step is bound by HBM traffic: a cell-update reads and writes its
// three unknowns (D, B, C) once, 6 words, while its arithmetic is about 30
// flops.  One launch advances the whole grid by one step of the scheme
// (the 1D step of eq. (10a)-(10d) with Table 1 along z, Yee curls along x):
//   E*  from D^{n-1/2}, B^{n-1}                      (10c)
//   B^n, TE B_z^n from the curl of E* and the upwind dB/dz      (10a)
//   H*  from B^n, D^{n-1/2}                          (10d)
//   D^{n+1/2}, TM D_z^{n+1/2} from the curl of H* and dD/dz     (10b)
//   then the source row, the z ends and the probes.
//
// Work decomposition.  A 64-lane wave owns a z-strip of 64 * C rows, C
// consecutive rows per lane (z-neighbours are in the same lane or one lane
// over, reached with one DPP move), and marches along x over a chunk of
// columns.  Along the march every column's D, B, C are loaded once and its
// new values stored once; the quantities a column shares with the next
// (E*, H* and the cross-field terms of the previous column) stay in
// registers, and the loads of the next column are issued before the current
// column is computed.  The material coefficients depend on z only, so a
// lane loads them once per launch.  A step's z-reach is 3 rows upwind and
// 2 downwind; strips overlap by 4 rows on each side and store only their
// inner rows.  A chunk starts one column early (a warm-up column that is
// computed but not stored).  Blocks of 4 waves are numbered so that each
// XCD takes a contiguous range of strips.
//
// Temporal blocking: a launch may advance the grid by T steps (T = 2..4
// off a z-ring).  The march then runs T stages, stage t one column behind
// stage t - 1 and taking its input fields from registers, so a cell-update
// moves 6/T words through HBM plus the warm-up columns; strips overlap by
// 3T rows a side (rounded up to a multiple of 4), and between stages the
// rows off the grid take the fields' edge values again, as the step reads
// them.
//
// Arithmetic: each update is the oracle's sum of terms, with division by
// eps, mu replaced by a multiply with the reciprocal and each term's
// product folded into a fused multiply-add written out as one.
// Floating-point contraction is off in this file, so every cell-update is
// the same sequence of roundings wherever the cell sits in a strip, chunk
// or stage: results do not depend on the launch geometry (bit for bit), and
// FP64 runs agree with the oracle to rounding.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "gfdtd.h"
#include "gfdtd2d.h"
#include "gfdtd2d_internal.h"

#pragma clang fp contract(off)

namespace gfdtd {

namespace {

__device__ __forceinline__ int dpp_left(int v)      // lane i <- lane i-1
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true);
}

__device__ __forceinline__ int dpp_right(int v)     // lane i <- lane i+1
{
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true);
}

__device__ __forceinline__ float lane_left(float v)
{
    return __int_as_float(dpp_left(__float_as_int(v)));
}

__device__ __forceinline__ float lane_right(float v)
{
    return __int_as_float(dpp_right(__float_as_int(v)));
}

__device__ __forceinline__ double lane_left(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = dpp_left((int)(u & 0xffffffffLL));
    const int hi = dpp_left((int)(u >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_right(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = dpp_right((int)(u & 0xffffffffLL));
    const int hi = dpp_right((int)(u >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Fused multiply-add, written out: contraction is off in this file, so
// every fused operation is one of these and the same in every copy of a
// stage, whatever the tiling.
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Row shifts of a lane's C consecutive rows: the value at row r-1, r-2, r+1.
template <typename R, int C>
__device__ __forceinline__ void prev1(const R (&a)[C], R (&o)[C])
{
    o[0] = lane_left(a[C - 1]);
#pragma unroll
    for (int q = 1; q < C; ++q)
        o[q] = a[q - 1];
}

template <typename R, int C>
__device__ __forceinline__ void prev2(const R (&a)[C], R (&o)[C])
{
    o[0] = lane_left(a[C - 2]);
    o[1] = lane_left(a[C - 1]);
#pragma unroll
    for (int q = 2; q < C; ++q)
        o[q] = a[q - 2];
}

template <typename R, int C>
__device__ __forceinline__ void next1(const R (&a)[C], R (&o)[C])
{
#pragma unroll
    for (int q = 0; q < C - 1; ++q)
        o[q] = a[q + 1];
    o[C - 1] = lane_right(a[0]);
}

// The vector type of one lane's C rows: 16 bytes (float4, double2), or 8
// for two FP32 rows (float2).
template <typename R, int C> struct RowVec;
template <int C> struct RowVec<float, C> {
    using T = typename std::conditional<C % 4 == 0, float4, float2>::type;
};
template <int C> struct RowVec<double, C> { using T = double2; };

__device__ __forceinline__ int clampi(int i, int lo, int hi)
{
    return i < lo ? lo : (i > hi ? hi : i);
}

__device__ __forceinline__ int wrapi(int i, int n)
{
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// Rows r0..r0+C-1 of a column whose lattice has n nodes: vector loads
// when they all lie on the lattice, else per row with the edge value off
// the grid (wrapped on a z-ring).
template <typename R, int C, bool INSIDE = false>
__device__ __forceinline__ void load_rows(const R *__restrict__ col, int r0, int n, int nz,
                                          bool ring, R (&a)[C])
{
    if (INSIDE || (r0 >= 0 && r0 + C <= n)) {
        using V = typename RowVec<R, C>::T;
        constexpr int U = sizeof(V) / sizeof(R);
        const V *p = reinterpret_cast<const V *>(col + r0);
#pragma unroll
        for (int u = 0; u < C / U; ++u) {
            const V v = p[u];
            __builtin_memcpy(&a[u * U], &v, sizeof(V));
        }
    } else {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int r = r0 + q;
            a[q] = col[ring ? wrapi(r, nz) : clampi(r, 0, n - 1)];
        }
    }
}

// Store the rows of r0..r0+C-1 that lie in [lo, hi).
template <typename R, int C>
__device__ __forceinline__ void store_rows(R *__restrict__ col, int r0, int lo, int hi,
                                           const R (&a)[C])
{
    if (r0 >= lo && r0 + C <= hi) {
        using V = typename RowVec<R, C>::T;
        constexpr int U = sizeof(V) / sizeof(R);
        V *p = reinterpret_cast<V *>(col + r0);
#pragma unroll
        for (int u = 0; u < C / U; ++u) {
            V v;
            __builtin_memcpy(&v, &a[u * U], sizeof(V));
            p[u] = v;
        }
    } else {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int r = r0 + q;
            if (r >= lo && r < hi)
                col[r] = a[q];
        }
    }
}

// Rest cell under lattice position x when the profile has moved m cells.
__device__ __forceinline__ int rest_cell(int x, int m, int hi, int nz, bool ring)
{
    return ring ? wrapi(x - m, nz) : clampi(x - m, 0, hi);
}

// Whole-cell shift m = rint(beta S tau) as the index arithmetic needs it:
// on a z-ring reduced modulo nz (indices wrap); otherwise clamped to
// +-4 nz, which changes no index of a grid node (those clamp to the grid).
__device__ __forceinline__ int shift_at(double bS, double tau, int nz, bool ring)
{
    const int64_t m = (int64_t)rint(bS * tau);
    if (ring) {
        const int64_t r = m % nz;
        return (int)(r < 0 ? r + nz : r);
    }
    const int64_t lim = 4 * (int64_t)nz;
    return (int)(m > lim ? lim : (m < -lim ? -lim : m));
}

__device__ __forceinline__ float readlane_r(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double readlane_r(double v, int l)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Halo rows of a strip for T steps a launch: a step reaches 3 rows upwind
// and 2 downwind, so 3T on each side, rounded up to a multiple of 4 (which
// keeps every lane's rows 16-byte aligned).
constexpr int halo_rows(int T) { return (3 * T + 3) / 4 * 4; }

// The step kernel.  T steps a launch (T = 1 on a z-ring): the march along
// x runs T stages, stage t performing step n0 + t one column behind stage
// t - 1, whose new fields it takes from registers; only the last stage
// stores.  Stage t at column j needs stage t - 1's fields up to column
// j + 1, and every stage needs two columns before its first valid one
// (its carried E*/H* terms), so the march starts T + 1 columns before the
// chunk and runs T - 1 columns past it.
//
// EDGE: the wave holds an end of the z lattices, rows off them, the source
// row or a probe; every other wave runs a march compiled without that code
// (no source, end or probe updates, no edge values, vector loads only).
template <typename R, int C, bool TE, bool COLA, int T, bool EDGE>
__device__ __forceinline__ void step2d_wave(const Run2D &rd, int64_t n0, int par, int xch,
                                            int nstrips, int w)
{
    const int lane = threadIdx.x & 63;
    constexpr int H = halo_rows(T);
    constexpr int STRIDE = 64 * C - 2 * H;
    const int s = w % nstrips;
    const int chunk = w / nstrips;
    const int nx = (int)rd.nx, nz = (int)rd.nz, nh = (int)rd.nh, nc = (int)rd.nc;
    const int64_t ld = rd.ld;
    const bool ring = rd.abc == GFDTD_ABC_PERIODIC;
    const int vlo = s * STRIDE;
    const int vhi = vlo + STRIDE < nz ? vlo + STRIDE : nz;
    const int z0 = vlo - H;                  // first row the wave holds
    const int r0 = z0 + lane * C;
    const int i0 = chunk * xch;
    const int i1 = i0 + xch < nx ? i0 + xch : nx;

    const double Sd = rd.S, betad = rd.beta, bSd = betad * Sd;
    // S, -S, -beta S and +-beta/2 (the sign of the star fields' velocity
    // part: TE +, TM -)
    const R S = (R)Sd, nS = (R)(-Sd), nbS = (R)(-bSd);
    const R hb = (R)(TE ? 0.5 * betad : -0.5 * betad);

    // the rows a wave holds that need the source, the ends or the grid-edge
    // values (halo rows included: later stages read them)
    const int src_row = (int)rd.src_row;
    const bool src_here = EDGE && src_row >= z0 && src_row < z0 + 64 * C;
    const bool lo_edge = EDGE && !ring && z0 < 0;
    const bool hi_edge_d = EDGE && !ring && z0 + 64 * C > nz - 1;

    // per-stage constants: material coefficients (z only), source sample,
    // end coefficients, the shift for the probes' eps
    R ce[T][C], chB[T][C], cc[T][C];
    double gs[T];
    R cLs[T], cRs[T];
    int mEs[T];
#pragma unroll
    for (int st = 0; st < T; ++st) {
        const int64_t n = n0 + st;
        const int mEp = shift_at(bSd, (double)n - 0.5, nz, ring);   // E* of step n-1
        const int mH = shift_at(bSd, (double)n, nz, ring);
        const int mE = shift_at(bSd, (double)n + 0.5, nz, ring);
        mEs[st] = mE;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int r = r0 + q;
            ce[st][q] = (R)(1.0 / rd.eps[rest_cell(r, mEp, nz - 1, nz, ring)]);
            chB[st][q] = (R)(1.0 / rd.mu[rest_cell(r, mH, ring ? nz - 1 : nz - 2, nz, ring)]);
            if (TE)   // B_z at (i+1/2, k): mu cell k
                cc[st][q] = (R)(1.0 / rd.mu[rest_cell(r, mH, nz - 1, nz, ring)]);
            else      // D_z at (i, j+1/2): eps cell j+1
                cc[st][q] = (R)(1.0 / rd.eps[rest_cell(r + 1, mEp, nz - 1, nz, ring)]);
        }
        gs[st] = (src_here && n <= rd.nsrc) ? rd.src[n - 1] : 0.0;
        cLs[st] = cRs[st] = (R)0;
        if (rd.abc == GFDTD_ABC_MUR1 && (lo_edge || hi_edge_d)) {
            const double nL = sqrt(rd.eps[clampi(-mE, 0, nz - 1)] * rd.mu[clampi(-mE, 0, nz - 2)]);
            const double nR = sqrt(rd.eps[clampi(nz - 1 - mE, 0, nz - 1)] *
                                   rd.mu[clampi(nz - 2 - mE, 0, nz - 2)]);
            const double uL = 1.0 / nL, uR = 1.0 / nR;
            cLs[st] = (R)((Sd * uL - 1.0) / (Sd * uL + 1.0));
            cRs[st] = (R)((Sd * uR - 1.0) / (Sd * uR + 1.0));
        }
    }

    const R *Din = static_cast<const R *>(par ? rd.f[1] : rd.f[0]);
    const R *Bin = static_cast<const R *>(par ? rd.f[3] : rd.f[2]);
    const R *Cin = static_cast<const R *>(par ? rd.f[5] : rd.f[4]);
    R *Dout = static_cast<R *>(par ? rd.f[0] : rd.f[1]);
    R *Bout = static_cast<R *>(par ? rd.f[2] : rd.f[3]);
    R *Cout = static_cast<R *>(par ? rd.f[4] : rd.f[5]);
    // column i (i0 - T - 1 <= i <= i1 + T - 1) wrapped onto 0..nx-1: one
    // conditional add or subtract once nx exceeds the march's overhang
    auto wrapc = [&](int i) {
        if (nx <= 2 * T + 2) {
            const int r = i % nx;
            return r < 0 ? r + nx : r;
        }
        return i < 0 ? i + nx : (i >= nx ? i - nx : i);
    };
    auto colp = [&](const R *base, int i) { return base + (int64_t)wrapc(i) * ld; };

    uint64_t own = 0;                        // probes this wave records
    for (int q = 0; EDGE && q < rd.nprobe; ++q) {
        const int64_t x = rd.px[q], z = rd.pz[q];
        if (z >= vlo && z < vhi && x >= i0 && x < i1)
            own |= 1ull << q;
    }

    // E* = D/eps +- beta * (Table 1 B average), TE +, TM -
    auto star_e = [&](const R (&cE)[C], const R (&D)[C], const R (&B)[C], R (&E)[C]) {
        R a1[C], a2[C];
        if (COLA) {
            prev1<R, C>(B, a1);
            prev2<R, C>(B, a2);
        } else {
            next1<R, C>(B, a1);
#pragma unroll
            for (int q = 0; q < C; ++q)
                a2[q] = B[q];
        }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            // D/eps +- beta (B1 + B2)/2, hb = +-beta/2
            E[q] = fmad(hb, a1[q] + a2[q], D[q] * cE[q]);
        }
    };
    // Table 1 upwind z-difference: F - F(r-1) (v >= 0) or F(r+1) - F (v < 0)
    auto dz_up = [&](const R (&F)[C], R (&d)[C]) {
        R t[C];
        if (COLA) {
            prev1<R, C>(F, t);
#pragma unroll
            for (int q = 0; q < C; ++q)
                d[q] = F[q] - t[q];
        } else {
            next1<R, C>(F, t);
#pragma unroll
            for (int q = 0; q < C; ++q)
                d[q] = t[q] - F[q];
        }
    };
    // source, z ends and probes on the new D of column j at stage st
    auto finish_d = [&](int st, int j, const R (&Dold)[C], R (&Dn)[C]) {
        const int64_t n = n0 + st;
        if (src_here && n <= rd.nsrc) {
            const double add = rd.prof[wrapc(j)] * gs[st];
#pragma unroll
            for (int q = 0; q < C; ++q)
                if (r0 + q == src_row)
                    Dn[q] = (R)((double)Dn[q] + add);
        }
        if (rd.abc == GFDTD_ABC_MUR1) {
            if (lo_edge) {           // D'(0) = D(1) + cL (D'(1) - D(0))
                R dn1[C], do1[C];
                next1<R, C>(Dn, dn1);
                next1<R, C>(Dold, do1);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    if (r0 + q == 0)
                        Dn[q] = do1[q] + cLs[st] * (dn1[q] - Dold[q]);
            }
            if (hi_edge_d) {         // D'(nz-1) = D(nz-2) + cR (D'(nz-2) - D(nz-1))
                R dm1[C], om1[C];
                prev1<R, C>(Dn, dm1);
                prev1<R, C>(Dold, om1);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    if (r0 + q == nz - 1)
                        Dn[q] = om1[q] + cRs[st] * (dm1[q] - Dold[q]);
            }
        } else if (rd.abc == GFDTD_ABC_PEC && (lo_edge || hi_edge_d)) {
#pragma unroll
            for (int q = 0; q < C; ++q)
                if (r0 + q == 0 || r0 + q == nz - 1)
                    Dn[q] = (R)0;
        }
        if (own && j >= i0 && j < i1) {
            for (uint64_t m = own; m; m &= m - 1) {
                const int q = __builtin_ctzll(m);
                if (rd.px[q] != j)
                    continue;
                const int z = (int)rd.pz[q];
                const int off = z - z0;
                const int lp = off / C, qq = off % C;
                R v = Dn[0];
#pragma unroll
                for (int t = 1; t < C; ++t)
                    if (t == qq)
                        v = Dn[t];
                if (lane == lp)
                    rd.trace[(int64_t)q * rd.steps + (n - 1)] =
                        (double)v / rd.eps[rest_cell(z, mEs[st], nz - 1, nz, ring)];
            }
        }
    };
    // Off-lattice rows of a stage's new field (rows < 0 or >= nlat) take the
    // edge values of that field, as the step reads them (grid ends only).
    auto edge_values = [&](R (&a)[C], int nlat) {
        if (lo_edge) {
            constexpr int L0 = H / C, Q0 = H % C;     // row 0 of strip 0
            const R e = readlane_r(a[Q0], L0);
#pragma unroll
            for (int q = 0; q < C; ++q)
                if (r0 + q < 0)
                    a[q] = e;
        }
        if (EDGE && !ring && z0 + 64 * C > nlat) {
            const int off = nlat - 1 - z0;
            const int lr = off / C, qr = off % C;
            R v = a[0];
#pragma unroll
            for (int t = 1; t < C; ++t)
                if (t == qr)
                    v = a[t];
            const R e = readlane_r(v, lr);
#pragma unroll
            for (int q = 0; q < C; ++q)
                if (r0 + q >= nlat)
                    a[q] = e;
        }
    };

    // carried state per stage (zero until the stage's warm-up columns set it)
    R k1[T][C], k2[T][C], k3[T][C], k4[T][C];   // TE: D, B, E*, H*_z; TM: C, E*_z, H*_y
    R dl[T][C], dl2[T][C];                       // TE: delayed C; TM: delayed D, B
#pragma unroll
    for (int st = 0; st < T; ++st)
#pragma unroll
        for (int q = 0; q < C; ++q)
            k1[st][q] = k2[st][q] = k3[st][q] = k4[st][q] = dl[st][q] = dl2[st][q] = (R)0;

    const int kbeg = i0 - T - 1, kend = i1 + T - 2;   // stage 0's columns
    // loads of stage 0's first column: TE D, B at k + 1 and C at k; TM D, B
    // at k and C at k + 1
    R Ld[C], Lb[C], Lc[C];
    load_rows<R, C, !EDGE>(colp(Din, TE ? kbeg + 1 : kbeg), r0, nz, nz, ring, Ld);
    load_rows<R, C, !EDGE>(colp(Bin, TE ? kbeg + 1 : kbeg), r0, nh, nz, ring, Lb);
    load_rows<R, C, !EDGE>(colp(Cin, TE ? kbeg : kbeg + 1), r0, nc, nz, ring, Lc);
    R dd[C], t1[C], t2[C];
    for (int k = kbeg; k <= kend; ++k) {
        R inD[C], inB[C], inC[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
            inD[q] = Ld[q];
            inB[q] = Lb[q];
            inC[q] = Lc[q];
        }
        if (k < kend) {            // next column's loads, in flight meanwhile
            const int kn = k + 1;
            load_rows<R, C, !EDGE>(colp(Din, TE ? kn + 1 : kn), r0, nz, nz, ring, Ld);
            load_rows<R, C, !EDGE>(colp(Bin, TE ? kn + 1 : kn), r0, nh, nz, ring, Lb);
            load_rows<R, C, !EDGE>(colp(Cin, TE ? kn : kn + 1), r0, nc, nz, ring, Lc);
        }
        R nxt[T][C], nxt2[T][C];   // delayed inputs for the next column
#pragma unroll
        for (int st = 0; st < T; ++st) {
            const int j = k - st;                      // this stage's column
            R oD[C], oB[C], oC[C];
            if (TE) {
                // inputs: D, B at column j + 1; C at column j
                R Cj[C];
#pragma unroll
                for (int q = 0; q < C; ++q)
                    Cj[q] = st == 0 ? inC[q] : dl[st][q];
                R En[C], Hs[C], Hc[C];
                star_e(ce[st], inD, inB, En);
                // (10a): B_x^n and B_z^n
                next1<R, C>(k3[st], t1);
                dz_up(k2[st], dd);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    oB[q] = fmad(nbS, dd[q], fmad(S, t1[q] - k3[st][q], k2[st][q]));
                dz_up(Cj, dd);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    oC[q] = fmad(nbS, dd[q], fmad(nS, En[q] - k3[st][q], Cj[q]));
                // (10d): H*_x = B_x/mu + beta Dbar, H*_z = B_z/mu
                next1<R, C>(k1[st], t1);
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    Hs[q] = fmad(hb, t1[q] + k1[st][q], oB[q] * chB[st][q]);
                    Hc[q] = oC[q] * cc[st][q];
                }
                // (10b): D_y^{n+1/2}
                prev1<R, C>(Hs, t2);
                dz_up(k1[st], dd);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    oD[q] = fmad(nbS, dd[q], fmad(nS, Hc[q] - k4[st][q],
                                                  fmad(S, Hs[q] - t2[q], k1[st][q])));
                finish_d(st, j, k1[st], oD);
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    k4[st][q] = Hc[q];
                    k3[st][q] = En[q];
                    k1[st][q] = inD[q];
                    k2[st][q] = inB[q];
                }
            } else {
                // inputs: D, B at column j; C at column j + 1
                R Dj[C], Bj[C];
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    Dj[q] = st == 0 ? inD[q] : dl[st][q];
                    Bj[q] = st == 0 ? inB[q] : dl2[st][q];
                }
                R Es[C], Ecn[C], Hs[C];
                star_e(ce[st], Dj, Bj, Es);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    Ecn[q] = inC[q] * cc[st][q];
                // (10a): B_y^n
                next1<R, C>(Es, t1);
                dz_up(Bj, dd);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    oB[q] = fmad(nbS, dd[q], fmad(S, Ecn[q] - k2[st][q],
                                                  fmad(nS, t1[q] - Es[q], Bj[q])));
                // (10d): H*_y = B_y/mu - beta Dbar
                next1<R, C>(Dj, t1);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    Hs[q] = fmad(hb, t1[q] + Dj[q], oB[q] * chB[st][q]);
                // (10b): D_x^{n+1/2} and D_z^{n+1/2}
                prev1<R, C>(Hs, t2);
                dz_up(Dj, dd);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    oD[q] = fmad(nbS, dd[q], fmad(nS, Hs[q] - t2[q], Dj[q]));
                dz_up(k1[st], dd);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    oC[q] = fmad(nbS, dd[q], fmad(S, Hs[q] - k3[st][q], k1[st][q]));
                finish_d(st, j, Dj, oD);
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    k3[st][q] = Hs[q];
                    k2[st][q] = Ecn[q];
                    k1[st][q] = inC[q];
                }
            }
            if (st + 1 < T) {
                // the next stage's inputs: its new fields, with the grid's
                // edge values on off-lattice rows
                edge_values(oD, nz);
                edge_values(oB, nh);
                edge_values(oC, nc);
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    if (TE) {
                        inD[q] = oD[q];
                        inB[q] = oB[q];
                        nxt[st + 1][q] = oC[q];
                    } else {
                        inC[q] = oC[q];
                        nxt[st + 1][q] = oD[q];
                        nxt2[st + 1][q] = oB[q];
                    }
                }
            } else if (j >= i0 && j < i1) {
                const int64_t o = (int64_t)j * ld;
                store_rows<R, C>(Dout + o, r0, vlo, vhi, oD);
                store_rows<R, C>(Bout + o, r0, vlo, vhi < nh ? vhi : nh, oB);
                store_rows<R, C>(Cout + o, r0, vlo, vhi < nc ? vhi : nc, oC);
            }
        }
#pragma unroll
        for (int st = 1; st < T; ++st)
#pragma unroll
            for (int q = 0; q < C; ++q) {
                dl[st][q] = nxt[st][q];
                if (!TE)
                    dl2[st][q] = nxt2[st][q];
            }
    }
}

// Waves per SIMD the register allocation must allow: FP32 at 2 cells per
// lane and 3 steps a launch fits 4 without spilling (left to itself the
// compiler takes one register more); elsewhere its own choice (1: no
// constraint).
template <typename R, int C, int T>
constexpr int occupancy2d()
{
    return (sizeof(R) == 4 && C == 2 && T == 3) ? 4 : 1;
}

// One wave a workgroup: a wave's slot is free for the next as soon as it
// ends, not when the slowest of a group ends (measured 2-3 % faster than four
// waves a group on the 4096 x 4096 slab, both precisions and polarizations).
template <typename R, int C, bool TE, bool COLA, int T>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(occupancy2d<R, C, T>()))) void k_step2d(
    const Run2D rd, int64_t n0, int par, int xch, int nstrips, int waves, int blocks)
{
    // each XCD (blocks b = x mod 8) takes a contiguous range of wave ids
    const int b = blockIdx.x;
    const int w = (b & 7) * (blocks >> 3) + (b >> 3);
    if (w >= waves)
        return;
    // the wave's rows [z0, z0 + 64 C) and columns [i0, i1), as step2d_wave
    // takes them: it runs the full march if they hold the source row, a row
    // off any lattice (an end, or a wrap on a ring) or a probe
    constexpr int H = halo_rows(T);
    constexpr int STRIDE = 64 * C - 2 * H;
    const int s = w % nstrips;
    const int z0 = s * STRIDE - H;
    const int nlat = (int)(rd.nh < rd.nc ? rd.nh : rd.nc);   // nh <= nc <= nz
    bool edge = z0 < 0 || z0 + 64 * C > nlat ||
                (rd.src_row >= z0 && rd.src_row < z0 + 64 * C);
    if (!edge) {
        const int vlo = s * STRIDE;
        const int vhi = vlo + STRIDE < rd.nz ? vlo + STRIDE : (int)rd.nz;
        const int i0 = (w / nstrips) * xch;
        const int i1 = i0 + xch < rd.nx ? i0 + xch : (int)rd.nx;
        for (int q = 0; q < rd.nprobe && !edge; ++q)
            edge = rd.pz[q] >= vlo && rd.pz[q] < vhi && rd.px[q] >= i0 && rd.px[q] < i1;
    }
    if (edge)
        step2d_wave<R, C, TE, COLA, T, true>(rd, n0, par, xch, nstrips, w);
    else
        step2d_wave<R, C, TE, COLA, T, false>(rd, n0, par, xch, nstrips, w);
}

// Source samples g(n S) and the initial fields of both halves of every
// ping-pong pair (a plain fill kernel: no memset nodes).
__global__ __launch_bounds__(256) void k_prep2d(const Run2D *__restrict__ rdp)
{
    const Run2D &rd = *rdp;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = tid; k < rd.nsrc; k += nth) {
        const double t = (double)(k + 1) * rd.S;
        const double u = (t - rd.t0) / rd.tau;
        rd.src[k] = rd.amp * sin(rd.omega * (t - rd.t0) + rd.phase) * exp(-u * u);
    }
    const int64_t cells = rd.nx * rd.ld;
    const int64_t nlat[3] = {rd.nz, rd.nh, rd.nc};
    for (int64_t e = tid; e < 3 * cells; e += nth) {
        const int fld = (int)(e / cells);
        const int64_t c = e - (int64_t)fld * cells;
        const int64_t i = c / rd.ld, k = c - i * rd.ld;
        const double *src = rd.init[fld];
        const double v = (src && k < nlat[fld]) ? src[i * rd.nz + k] : 0.0;
        if (rd.precision == GFDTD_F32) {
            static_cast<float *>(rd.f[2 * fld])[c] = (float)v;
            static_cast<float *>(rd.f[2 * fld + 1])[c] = (float)v;
        } else {
            static_cast<double *>(rd.f[2 * fld])[c] = v;
            static_cast<double *>(rd.f[2 * fld + 1])[c] = v;
        }
    }
}

template <typename R, int C, int T>
hipError_t step_as(const Run2D &h, const Launch2D &L, int64_t n, int par, hipStream_t s)
{
    const dim3 grid((unsigned)L.blocks), block(64);
    const bool te = h.pol == GFDTD2D_TE, cola = h.beta >= 0.0;
    const int xch = L.xch, ns = (int)L.nstrips, waves = (int)L.waves, blocks = (int)L.blocks;
    if (te && cola)
        hipLaunchKernelGGL((k_step2d<R, C, true, true, T>), grid, block, 0, s, h, n, par, xch,
                           ns, waves, blocks);
    else if (te)
        hipLaunchKernelGGL((k_step2d<R, C, true, false, T>), grid, block, 0, s, h, n, par, xch,
                           ns, waves, blocks);
    else if (cola)
        hipLaunchKernelGGL((k_step2d<R, C, false, true, T>), grid, block, 0, s, h, n, par, xch,
                           ns, waves, blocks);
    else
        hipLaunchKernelGGL((k_step2d<R, C, false, false, T>), grid, block, 0, s, h, n, par,
                           xch, ns, waves, blocks);
    return hipGetLastError();
}

// Instantiated tilings: several steps a launch for the narrow lanes only
// (FP32 2 or 4 cells, FP64 2): wider lanes exceed the register file there.
template <typename R, int C>
hipError_t step_ct(const Run2D &h, const Launch2D &L, int64_t n, int par, hipStream_t s)
{
    constexpr bool narrow = C * sizeof(R) <= 16;
    switch (L.T) {
    case 1: return step_as<R, C, 1>(h, L, n, par, s);
    case 2: if constexpr (narrow) return step_as<R, C, 2>(h, L, n, par, s); else break;
    case 3: if constexpr (narrow) return step_as<R, C, 3>(h, L, n, par, s); else break;
    case 4: if constexpr (narrow) return step_as<R, C, 4>(h, L, n, par, s); else break;
    default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

int64_t strip_rows(int C, int T) { return 64 * (int64_t)C - 2 * halo_rows(T); }

Launch2D plan_launch2d(int64_t nx, int64_t nz, int precision, int C, int xch, int T)
{
    Launch2D L;
    if (C <= 0)
        C = 2;
    if (T <= 0)
        T = 1;
    L.C = C;
    L.T = T;
    L.nstrips = (nz + strip_rows(C, T) - 1) / strip_rows(C, T);
    if (xch <= 0) {
        // a march of T steps starts T + 1 columns early, so deeper blocks
        // want longer marches: at most 8, 16, 16 and 16 (FP32) or 20 (FP64)
        // columns for T = 1..4, fewer when the grid would give under 2048
        // waves.  Measured on the 4096 x 4096 grid at 2 cells per lane and
        // 4 steps a launch: FP32 3.6e11 updates/s with 16 columns against
        // 3.0e11 with 32 (TE; TM 3.3e11 against 3.1e11); FP64 TE flat from
        // 20 to 32, TM 2.41e11 with 20 against 2.33e11 with 24; one step a
        // launch with 8-16
        static const int cap_of[5] = {8, 8, 16, 16, 16};
        const int64_t x = nx * L.nstrips / 2048;
        int64_t cap = cap_of[T < 0 ? 0 : (T > 4 ? 4 : T)];
        if (T >= 4 && precision != GFDTD_F32)
            cap = 20;
        xch = (int)(x < 2 ? 2 : (x > cap ? cap : x));
    }
    if (xch > nx)
        xch = (int)nx;
    L.xch = xch;
    L.nchunks = (nx + xch - 1) / xch;
    L.waves = L.nstrips * L.nchunks;
    L.blocks = (L.waves + 7) / 8 * 8;   // one wave a workgroup
    return L;
}

hipError_t launch_prep2d(const Run2D *dev, const Run2D &h, hipStream_t s)
{
    const int64_t work = 3 * h.nx * h.ld;
    int64_t bx = (work + 255) / 256;
    bx = bx < 1 ? 1 : (bx > 4096 ? 4096 : bx);
    hipLaunchKernelGGL(k_prep2d, dim3((unsigned)bx), dim3(256), 0, s, dev);
    return hipGetLastError();
}

hipError_t launch_step2d(const Run2D &h, const Launch2D &L, int64_t n, int par,
                         hipStream_t s)
{
    if (h.precision == GFDTD_F32) {
        if (L.C == 2)
            return step_ct<float, 2>(h, L, n, par, s);
        if (L.C == 4)
            return step_ct<float, 4>(h, L, n, par, s);
        if (L.C == 8)
            return step_ct<float, 8>(h, L, n, par, s);
    } else {
        if (L.C == 2)
            return step_ct<double, 2>(h, L, n, par, s);
        if (L.C == 4)
            return step_ct<double, 4>(h, L, n, par, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gfdtd
