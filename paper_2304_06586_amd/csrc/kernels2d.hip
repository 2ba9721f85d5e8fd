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
// Arithmetic follows the oracle's order of operations per term (division
// by eps, mu replaced by a multiply with the reciprocal), with floating-point
// contraction off in this file: every cell-update is the same sequence of
// roundings wherever the cell sits in a strip or chunk, so results do not
// depend on the launch geometry, and FP64 runs agree with the oracle to
// rounding.

#include <hip/hip_runtime.h>

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

template <typename R> struct Vec16;
template <> struct Vec16<float> { using T = float4; };
template <> struct Vec16<double> { using T = double2; };

__device__ __forceinline__ int clampi(int i, int lo, int hi)
{
    return i < lo ? lo : (i > hi ? hi : i);
}

__device__ __forceinline__ int wrapi(int i, int n)
{
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// Rows r0..r0+C-1 of a column whose lattice has n nodes: one 16-byte load
// per 16 bytes when they all lie on the lattice, else per row with the
// edge value off the grid (wrapped on a z-ring).
template <typename R, int C>
__device__ __forceinline__ void load_rows(const R *__restrict__ col, int r0, int n, int nz,
                                          bool ring, R (&a)[C])
{
    if (r0 >= 0 && r0 + C <= n) {
        using V = typename Vec16<R>::T;
        constexpr int U = 16 / sizeof(R);
        const V *p = reinterpret_cast<const V *>(col + r0);
#pragma unroll
        for (int u = 0; u < C / U; ++u) {
            const V v = p[u];
            __builtin_memcpy(&a[u * U], &v, 16);
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
        using V = typename Vec16<R>::T;
        constexpr int U = 16 / sizeof(R);
        V *p = reinterpret_cast<V *>(col + r0);
#pragma unroll
        for (int u = 0; u < C / U; ++u) {
            V v;
            __builtin_memcpy(&v, &a[u * U], 16);
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

template <typename R, int C, bool TE, bool COLA>
__global__ __launch_bounds__(256) void k_step2d(const Run2D rd, int64_t n, int par, int xch,
                                                int nstrips, int waves, int blocks)
{
    const int lane = threadIdx.x & 63;
    // each XCD (blocks b = x mod 8) takes a contiguous range of wave ids
    const int b = blockIdx.x;
    const int lb = (b & 7) * (blocks >> 3) + (b >> 3);
    const int w = lb * 4 + (int)(threadIdx.x >> 6);
    if (w >= waves)
        return;
    constexpr int STRIDE = 64 * C - 2 * HALO2D;
    const int s = w % nstrips;
    const int chunk = w / nstrips;
    const int nx = (int)rd.nx, nz = (int)rd.nz, nh = (int)rd.nh, nc = (int)rd.nc;
    const int64_t ld = rd.ld;
    const bool ring = rd.abc == GFDTD_ABC_PERIODIC;
    const int vlo = s * STRIDE;
    const int vhi = vlo + STRIDE < nz ? vlo + STRIDE : nz;
    const int r0 = vlo - HALO2D + lane * C;
    const int i0 = chunk * xch;
    const int i1 = i0 + xch < nx ? i0 + xch : nx;

    const double Sd = rd.S, betad = rd.beta, bSd = betad * Sd;
    const R S = (R)Sd, beta = (R)betad, bS = (R)bSd, half = (R)0.5;
    const int mEp = shift_at(bSd, (double)n - 0.5, nz, ring);   // E* of step n-1
    const int mH = shift_at(bSd, (double)n, nz, ring);
    const int mE = shift_at(bSd, (double)n + 0.5, nz, ring);

    // per-row material coefficients (z only)
    R ce[C], chB[C], cc[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const int r = r0 + q;
        ce[q] = (R)(1.0 / rd.eps[rest_cell(r, mEp, nz - 1, nz, ring)]);
        chB[q] = (R)(1.0 / rd.mu[rest_cell(r, mH, ring ? nz - 1 : nz - 2, nz, ring)]);
        if (TE)   // B_z at (i+1/2, k): mu cell k
            cc[q] = (R)(1.0 / rd.mu[rest_cell(r, mH, nz - 1, nz, ring)]);
        else      // D_z at (i, j+1/2): eps cell j+1
            cc[q] = (R)(1.0 / rd.eps[rest_cell(r + 1, mEp, nz - 1, nz, ring)]);
    }

    const R *Din = static_cast<const R *>(par ? rd.f[1] : rd.f[0]);
    const R *Bin = static_cast<const R *>(par ? rd.f[3] : rd.f[2]);
    const R *Cin = static_cast<const R *>(par ? rd.f[5] : rd.f[4]);
    R *Dout = static_cast<R *>(par ? rd.f[0] : rd.f[1]);
    R *Bout = static_cast<R *>(par ? rd.f[2] : rd.f[3]);
    R *Cout = static_cast<R *>(par ? rd.f[4] : rd.f[5]);
    // column i (i0 - 1 <= i <= i1 + 1) wrapped onto 0..nx-1
    auto colp = [&](const R *base, int i) {
        const int iw = nx == 1 ? 0 : (i < 0 ? i + nx : (i >= nx ? i - nx : i));
        return base + (int64_t)iw * ld;
    };

    // step-wide scalars: source sample, end coefficients, probes of this wave
    const int src_row = (int)rd.src_row;
    const bool has_src = n <= rd.nsrc && src_row >= vlo && src_row < vhi;
    const double g = has_src ? rd.src[n - 1] : 0.0;
    const bool left_end = !ring && vlo == 0;
    const bool right_end = !ring && vhi == nz;
    R cL = 0, cR = 0;
    if (rd.abc == GFDTD_ABC_MUR1 && (left_end || right_end)) {
        const double nL = sqrt(rd.eps[clampi(-mE, 0, nz - 1)] * rd.mu[clampi(-mE, 0, nz - 2)]);
        const double nR = sqrt(rd.eps[clampi(nz - 1 - mE, 0, nz - 1)] *
                               rd.mu[clampi(nz - 2 - mE, 0, nz - 2)]);
        const double uL = 1.0 / nL, uR = 1.0 / nR;
        cL = (R)((Sd * uL - 1.0) / (Sd * uL + 1.0));
        cR = (R)((Sd * uR - 1.0) / (Sd * uR + 1.0));
    }
    uint64_t own = 0;
    for (int q = 0; q < rd.nprobe; ++q) {
        const int64_t x = rd.px[q], z = rd.pz[q];
        if (z >= vlo && z < vhi && x >= i0 && x < i1)
            own |= 1ull << q;
    }

    // E* = D/eps +- beta * (Table 1 B average), TE +, TM -
    auto star_e = [&](const R (&D)[C], const R (&B)[C], R (&E)[C]) {
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
            const R bb = half * (a1[q] + a2[q]);
            E[q] = TE ? D[q] * ce[q] + beta * bb : D[q] * ce[q] - beta * bb;
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
    // source, z ends and probes on the new D of column i, then store
    auto finish_d = [&](int i, const R (&Dold)[C], R (&Dn)[C]) {
        if (has_src) {
            const double add = rd.prof[i] * g;
#pragma unroll
            for (int q = 0; q < C; ++q)
                if (r0 + q == src_row)
                    Dn[q] = (R)((double)Dn[q] + add);
        }
        if (rd.abc == GFDTD_ABC_MUR1) {
            if (left_end) {          // D'(0) = D(1) + cL (D'(1) - D(0))
                R dn1[C], do1[C];
                next1<R, C>(Dn, dn1);
                next1<R, C>(Dold, do1);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    if (r0 + q == 0)
                        Dn[q] = do1[q] + cL * (dn1[q] - Dold[q]);
            }
            if (right_end) {         // D'(nz-1) = D(nz-2) + cR (D'(nz-2) - D(nz-1))
                R dm1[C], om1[C];
                prev1<R, C>(Dn, dm1);
                prev1<R, C>(Dold, om1);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    if (r0 + q == nz - 1)
                        Dn[q] = om1[q] + cR * (dm1[q] - Dold[q]);
            }
        } else if (rd.abc == GFDTD_ABC_PEC && (left_end || right_end)) {
#pragma unroll
            for (int q = 0; q < C; ++q)
                if (r0 + q == 0 || r0 + q == nz - 1)
                    Dn[q] = (R)0;
        }
        if (own) {
            for (uint64_t m = own; m; m &= m - 1) {
                const int q = __builtin_ctzll(m);
                if (rd.px[q] != i)
                    continue;
                const int z = (int)rd.pz[q];
                const int off = z - (vlo - HALO2D);
                const int lp = off / C, qq = off % C;
                R v = Dn[0];
#pragma unroll
                for (int t = 1; t < C; ++t)
                    if (t == qq)
                        v = Dn[t];
                if (lane == lp)
                    rd.trace[(int64_t)q * rd.steps + (n - 1)] =
                        (double)v / rd.eps[rest_cell(z, mE, nz - 1, nz, ring)];
            }
        }
    };

    R dd[C], t1[C], t2[C];
    if (TE) {
        // prologue and warm-up column i0-1: E*(i0-1), E*(i0), Hc(i0-1)
        R Dc[C], Bc[C], Ep[C], Hcp[C], Cc[C];
        load_rows<R, C>(colp(Din, i0 - 1), r0, nz, nz, ring, Dc);
        load_rows<R, C>(colp(Bin, i0 - 1), r0, nh, nz, ring, Bc);
        star_e(Dc, Bc, Ep);
        load_rows<R, C>(colp(Din, i0), r0, nz, nz, ring, Dc);
        load_rows<R, C>(colp(Bin, i0), r0, nh, nz, ring, Bc);
        load_rows<R, C>(colp(Cin, i0 - 1), r0, nc, nz, ring, Cc);
        {
            R En[C];
            star_e(Dc, Bc, En);
            dz_up(Cc, dd);
#pragma unroll
            for (int q = 0; q < C; ++q)
                Hcp[q] = (Cc[q] - S * (En[q] - Ep[q]) - bS * dd[q]) * cc[q];
#pragma unroll
            for (int q = 0; q < C; ++q)
                Ep[q] = En[q];
        }
        // loads of the first column
        R Dl[C], Bl[C], Cl[C];
        load_rows<R, C>(colp(Din, i0 + 1), r0, nz, nz, ring, Dl);
        load_rows<R, C>(colp(Bin, i0 + 1), r0, nh, nz, ring, Bl);
        load_rows<R, C>(colp(Cin, i0), r0, nc, nz, ring, Cl);
        for (int i = i0; i < i1; ++i) {
            R Dx[C], Bx[C];
#pragma unroll
            for (int q = 0; q < C; ++q) {
                Dx[q] = Dl[q];
                Bx[q] = Bl[q];
                Cc[q] = Cl[q];
            }
            if (i + 1 < i1) {        // next column's loads, in flight meanwhile
                load_rows<R, C>(colp(Din, i + 2), r0, nz, nz, ring, Dl);
                load_rows<R, C>(colp(Bin, i + 2), r0, nh, nz, ring, Bl);
                load_rows<R, C>(colp(Cin, i + 1), r0, nc, nz, ring, Cl);
            }
            R En[C], Bn[C], Cn[C], Hs[C], Hc[C], Dn[C];
            star_e(Dx, Bx, En);
            // (10a): B_x^n and B_z^n
            next1<R, C>(Ep, t1);
            dz_up(Bc, dd);
#pragma unroll
            for (int q = 0; q < C; ++q)
                Bn[q] = Bc[q] + S * (t1[q] - Ep[q]) - bS * dd[q];
            dz_up(Cc, dd);
#pragma unroll
            for (int q = 0; q < C; ++q)
                Cn[q] = Cc[q] - S * (En[q] - Ep[q]) - bS * dd[q];
            // (10d): H*_x = B_x/mu + beta Dbar, H*_z = B_z/mu
            next1<R, C>(Dc, t1);
#pragma unroll
            for (int q = 0; q < C; ++q) {
                Hs[q] = Bn[q] * chB[q] + beta * (half * (t1[q] + Dc[q]));
                Hc[q] = Cn[q] * cc[q];
            }
            // (10b): D_y^{n+1/2}
            prev1<R, C>(Hs, t2);
            dz_up(Dc, dd);
#pragma unroll
            for (int q = 0; q < C; ++q)
                Dn[q] = Dc[q] + S * (Hs[q] - t2[q]) - S * (Hc[q] - Hcp[q]) - bS * dd[q];
            finish_d(i, Dc, Dn);
            const int64_t o = (int64_t)i * ld;
            store_rows<R, C>(Dout + o, r0, vlo, vhi, Dn);
            store_rows<R, C>(Bout + o, r0, vlo, vhi < nh ? vhi : nh, Bn);
            store_rows<R, C>(Cout + o, r0, vlo, vhi < nc ? vhi : nc, Cn);
#pragma unroll
            for (int q = 0; q < C; ++q) {
                Hcp[q] = Hc[q];
                Ep[q] = En[q];
                Dc[q] = Dx[q];
                Bc[q] = Bx[q];
            }
        }
    } else {
        // prologue: E*_z(i0-1); warm-up column i0-1 gives H*_y(i0-1)
        R Cr[C], Ecp[C], Hsp[C];
        load_rows<R, C>(colp(Cin, i0 - 1), r0, nc, nz, ring, Cr);
#pragma unroll
        for (int q = 0; q < C; ++q)
            Ecp[q] = Cr[q] * cc[q];
        R Dl[C], Bl[C], Cl[C];
        load_rows<R, C>(colp(Din, i0 - 1), r0, nz, nz, ring, Dl);
        load_rows<R, C>(colp(Bin, i0 - 1), r0, nh, nz, ring, Bl);
        load_rows<R, C>(colp(Cin, i0), r0, nc, nz, ring, Cl);
        for (int i = i0 - 1; i < i1; ++i) {
            R Dc[C], Bc[C], Cx[C];
#pragma unroll
            for (int q = 0; q < C; ++q) {
                Dc[q] = Dl[q];
                Bc[q] = Bl[q];
                Cx[q] = Cl[q];
            }
            if (i + 1 < i1) {
                load_rows<R, C>(colp(Din, i + 1), r0, nz, nz, ring, Dl);
                load_rows<R, C>(colp(Bin, i + 1), r0, nh, nz, ring, Bl);
                load_rows<R, C>(colp(Cin, i + 2), r0, nc, nz, ring, Cl);
            }
            R Es[C], Ecn[C], Bn[C], Hs[C];
            star_e(Dc, Bc, Es);
#pragma unroll
            for (int q = 0; q < C; ++q)
                Ecn[q] = Cx[q] * cc[q];
            // (10a): B_y^n
            next1<R, C>(Es, t1);
            dz_up(Bc, dd);
#pragma unroll
            for (int q = 0; q < C; ++q)
                Bn[q] = Bc[q] - S * (t1[q] - Es[q]) + S * (Ecn[q] - Ecp[q]) - bS * dd[q];
            // (10d): H*_y = B_y/mu - beta Dbar
            next1<R, C>(Dc, t1);
#pragma unroll
            for (int q = 0; q < C; ++q)
                Hs[q] = Bn[q] * chB[q] - beta * (half * (t1[q] + Dc[q]));
            if (i >= i0) {
                // (10b): D_x^{n+1/2} and D_z^{n+1/2}
                R Dn[C], Cn[C];
                prev1<R, C>(Hs, t2);
                dz_up(Dc, dd);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    Dn[q] = Dc[q] - S * (Hs[q] - t2[q]) - bS * dd[q];
                dz_up(Cr, dd);
#pragma unroll
                for (int q = 0; q < C; ++q)
                    Cn[q] = Cr[q] + S * (Hs[q] - Hsp[q]) - bS * dd[q];
                finish_d(i, Dc, Dn);
                const int64_t o = (int64_t)i * ld;
                store_rows<R, C>(Dout + o, r0, vlo, vhi, Dn);
                store_rows<R, C>(Bout + o, r0, vlo, vhi < nh ? vhi : nh, Bn);
                store_rows<R, C>(Cout + o, r0, vlo, vhi < nc ? vhi : nc, Cn);
            }
#pragma unroll
            for (int q = 0; q < C; ++q) {
                Hsp[q] = Hs[q];
                Ecp[q] = Ecn[q];
                Cr[q] = Cx[q];
            }
        }
    }
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

template <typename R, int C>
hipError_t step_as(const Run2D &h, const Launch2D &L, int64_t n, int par, hipStream_t s)
{
    const dim3 grid((unsigned)L.blocks), block(256);
    const bool te = h.pol == GFDTD2D_TE, cola = h.beta >= 0.0;
    const int xch = L.xch, ns = (int)L.nstrips, waves = (int)L.waves, blocks = (int)L.blocks;
    if (te && cola)
        hipLaunchKernelGGL((k_step2d<R, C, true, true>), grid, block, 0, s, h, n, par, xch,
                           ns, waves, blocks);
    else if (te)
        hipLaunchKernelGGL((k_step2d<R, C, true, false>), grid, block, 0, s, h, n, par, xch,
                           ns, waves, blocks);
    else if (cola)
        hipLaunchKernelGGL((k_step2d<R, C, false, true>), grid, block, 0, s, h, n, par, xch,
                           ns, waves, blocks);
    else
        hipLaunchKernelGGL((k_step2d<R, C, false, false>), grid, block, 0, s, h, n, par, xch,
                           ns, waves, blocks);
    return hipGetLastError();
}

}  // namespace

int64_t strip_rows(int C) { return 64 * (int64_t)C - 2 * HALO2D; }

Launch2D plan_launch2d(int64_t nx, int64_t nz, int precision, int C, int xch)
{
    Launch2D L;
    if (C <= 0)
        C = precision == GFDTD_F32 ? 4 : 2;
    L.C = C;
    L.nstrips = (nz + strip_rows(C) - 1) / strip_rows(C);
    if (xch <= 0) {
        // 2..8 columns a wave, fewer when the grid gives under ~8 waves per
        // SIMD (1024 SIMDs): on the 4096 x 4096 grid 8 columns (8704 FP32,
        // 17920 FP64 waves) beat both shorter marches (more warm-up columns)
        // and longer ones (fewer waves in flight)
        const int64_t want = 8192;
        int64_t x = nx * L.nstrips / want;
        xch = (int)(x < 2 ? 2 : (x > 8 ? 8 : x));
    }
    if (xch > nx)
        xch = (int)nx;
    L.xch = xch;
    L.nchunks = (nx + xch - 1) / xch;
    L.waves = L.nstrips * L.nchunks;
    const int64_t b4 = (L.waves + 3) / 4;
    L.blocks = (b4 + 7) / 8 * 8;
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
        if (L.C == 4)
            return step_as<float, 4>(h, L, n, par, s);
        if (L.C == 8)
            return step_as<float, 8>(h, L, n, par, s);
    } else {
        if (L.C == 2)
            return step_as<double, 2>(h, L, n, par, s);
        if (L.C == 4)
            return step_as<double, 4>(h, L, n, par, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace gfdtd
