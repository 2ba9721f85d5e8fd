// HIP kernels of the generalized-FDTD library (gfx950 / CDNA4).
//
// The hot kernel, k_tiles, advances wave tiles of one or many runs by a
// temporal block of T time steps.  A tile is one 64-lane wavefront holding
// 64*C consecutive cells in registers (C cells per lane, D and B for each);
// neighbouring values move between lanes with wave shuffles, so a tile
// needs no LDS and no barriers.  Tiles overlap: a cell next to a tile edge
// lacks its outside neighbour, and the error spreads by the reach of a
// step of eq. (10) with the Table 1 terms, 2 cells upwind (plus 1 in the
// first step) and 1 downwind, so after T steps only the lanes away from
// the tile edges hold valid values; those "owned" lanes are written back,
// to the other half of a ping-pong pair.  HBM traffic per cell-update is
// therefore about 2 * 2 * sizeof(R) / T plus the halo overhead.  Optional
// multi-wave tiles put G waves side by side and refresh the cells they
// share through LDS every K steps (one barrier per refresh).
//
// Per step and cell (all in registers), with the star fields carried
// scaled by the Courant number S (E~ = S E*, H~ = S H*):
//   E~   = cE D - hb (B_a + B_b)          (10c) with the Table 1 B average
//   B'   = B - (E~_{+1} - E~) - bS dB     (10a) with the Table 1 dB/dz
//   H~   = cH B' - hb (D_{+1} + D)        (10d) with the Table 1 D average
//   D'   = D - (H~ - H~_{-1}) - bS dD     (10b) with the Table 1 dD/dz
// then the source, the end conditions and the probes.  cE, cH are S/eps',
// S/mu' and hb = S beta / 2 for a moving modulation; for moving matter
// cE = S g mu', cH = S g eps' and hb is the per-cell S g beta / 2.  The
// curl and velocity terms of (10a)/(10b) are telescoped into one
// difference of per-cell sums (P = E~ + bS B_up, X = H~ + bS D_sel), which
// keeps a uniform field exactly uniform.  For a moving modulation E~ and
// H~ are folded into P and X (one multiply and two fused multiply-adds
// each): 10 floating-point instructions per cell and step (12 for moving
// matter, whose hb varies per cell).
//
// The moving profile: at time tau*S the rest profile has moved by
// m = rint(beta S tau) whole cells (FP64 on every path), so each lane keeps
// its cells' coefficients in registers and shifts them by one cell, with
// one shuffle, whenever m changes.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "gfdtd.h"
#include "gfdtd_internal.h"

namespace gfdtd {

// ------------------------------------------------------------ wave helpers

// Whole-wavefront shifts by one lane with DPP (wave_shr:1 / wave_shl:1):
// one VALU move per 32-bit word, no LDS traffic.  The lane shifted in at
// the wave edge reads 0 (bound_ctrl), so no old value is needed.
__device__ __forceinline__ int dpp_from_left(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true);
}

__device__ __forceinline__ int dpp_from_right(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true);
}

__device__ __forceinline__ float from_left(float v)     // lane i <- lane i-1
{
    return __int_as_float(dpp_from_left(__float_as_int(v)));
}

__device__ __forceinline__ float from_right(float v)    // lane i <- lane i+1
{
    return __int_as_float(dpp_from_right(__float_as_int(v)));
}

__device__ __forceinline__ double from_left(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = dpp_from_left((int)(u & 0xffffffffLL));
    const int hi = dpp_from_left((int)(u >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double from_right(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = dpp_from_right((int)(u & 0xffffffffLL));
    const int hi = dpp_from_right((int)(u >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float fmad(float a, float b, float c)
{
    return __builtin_fmaf(a, b, c);
}

__device__ __forceinline__ double fmad(double a, double b, double c)
{
    return __builtin_fma(a, b, c);
}

// The same pointer in the global address space: loads and stores through
// it are global (not flat) instructions, which count on the vector memory
// counter only.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *glb(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// Lane l's value of v, for a wave-uniform l (v_readlane, no LDS).
__device__ __forceinline__ int readlane_i(int v, int l)
{
    return __builtin_amdgcn_readlane(v, l);
}

__device__ __forceinline__ float readlane_r(float v, int l)
{
    return __int_as_float(readlane_i(__float_as_int(v), l));
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const long long u = __double_as_longlong(v);
    const int lo = readlane_i((int)(u & 0xffffffffLL), l);
    const int hi = readlane_i((int)(u >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane_r(double v, int l) { return readlane_d(v, l); }

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l)
{
    const int lo = readlane_i((int)(v & 0xffffffffLL), l);
    const int hi = readlane_i((int)(v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int64_t profile_shift(double bS, double tau)
{
    return (int64_t)rint(bS * tau);
}

// Same value for |beta S tau| < 2^31 (always the case: |beta S| < 1 and
// fewer than 2^31 steps), with 32-bit conversions.
__device__ __forceinline__ int profile_shift32(double bS, double tau)
{
    return (int)rint(bS * tau);
}

__device__ __forceinline__ int64_t clampi(int64_t i, int64_t lo, int64_t hi)
{
    return i < lo ? lo : (i > hi ? hi : i);
}

// i mod n in [0, n), for any sign of i (ring indexing).
__device__ __forceinline__ int64_t wrapi(int64_t i, int64_t n)
{
    const int64_t r = i % n;
    return r < 0 ? r + n : r;
}

// Next index on a ring of n >= 2 cells.
__device__ __forceinline__ int64_t ring_next(int64_t i, int64_t n)
{
    return i + 1 == n ? 0 : i + 1;
}

template <typename R, int C>
__device__ __forceinline__ void load_cells(const R *__restrict__ p, R (&v)[C])
{
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int q = 0; q < C / 4; ++q) {
            const float4 t = reinterpret_cast<const float4 *>(p)[q];
            v[4 * q + 0] = t.x;
            v[4 * q + 1] = t.y;
            v[4 * q + 2] = t.z;
            v[4 * q + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < C / 2; ++q) {
            const double2 t = reinterpret_cast<const double2 *>(p)[q];
            v[2 * q + 0] = t.x;
            v[2 * q + 1] = t.y;
        }
    }
}

template <typename R, int C>
__device__ __forceinline__ void store_cells(R *__restrict__ p, const R (&v)[C])
{
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int q = 0; q < C / 4; ++q)
            reinterpret_cast<float4 *>(p)[q] =
                make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
        for (int q = 0; q < C / 2; ++q)
            reinterpret_cast<double2 *>(p)[q] = make_double2(v[2 * q], v[2 * q + 1]);
    }
}

// Move a lane-distributed coefficient window one cell in the direction
// the profile moves: towards higher cells for v >= 0 (NEG false), lower
// cells for v < 0.  The value entering at a tile edge is not meaningful;
// it only ever reaches lanes outside the valid region.
template <typename R, int C, bool NEG>
__device__ __forceinline__ void shift_window(R (&a)[C])
{
    if constexpr (!NEG) {
        const R in = from_left(a[C - 1]);
#pragma unroll
        for (int c = C - 1; c > 0; --c)
            a[c] = a[c - 1];
        a[0] = in;
    } else {
        const R in = from_right(a[0]);
#pragma unroll
        for (int c = 0; c < C - 1; ++c)
            a[c] = a[c + 1];
        a[C - 1] = in;
    }
}

// a[idx] for a register array and a wave-uniform runtime idx, written as
// a chain of selects with constant indices only (an indexed read would
// force the array out of registers; a flat select loop over the registers
// is turned back into one by the compiler).
template <typename R, int C, int I = C - 1>
__device__ __forceinline__ R pick(const R (&a)[C], int idx)
{
    if constexpr (I == 0)
        return a[0];
    else
        return idx == I ? a[I] : pick<R, C, I - 1>(a, idx);
}

// The same wave-uniform (s) or per-lane (v) integer, taken by the
// compiler as produced anew where this is called (an empty asm statement,
// no instruction).  Inside a step loop, masks derived from it are then
// recomputed each step instead of being hoisted and held across the loop,
// C of them per use: more than the scalar register file holds, and what
// spills is reloaded each step.
__device__ __forceinline__ int fresh_s(int v)
{
    asm volatile("" : "+s"(v));
    return v;
}

__device__ __forceinline__ int fresh_v(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// a[idx] for a wave-uniform idx in [0, C), as the multiply-add chain
// sum_c [idx == c] a[c] with weights 1 and 0: exact for finite values (the
// other terms add signed zeros), no branch and no lane mask.  (A select
// chain on idx is turned into a branch tree by the compiler.)
template <typename R, int C>
__device__ __forceinline__ R pick_w(const R (&a)[C], int idx)
{
    R r = (idx == 0 ? (R)1 : (R)0) * a[0];
#pragma unroll
    for (int c = 1; c < C; ++c)
        r = fmad(idx == c ? (R)1 : (R)0, a[c], r);
    return r;
}

// ------------------------------------------------------------- the tile

// Workgroup barrier of a multi-wave tile.  A wave takes part only while
// it has active lanes: where the compiler lays out a wave-uniform branch
// as lane-masked code, the side a wave does not take runs with an empty
// mask and must not count as a barrier.  On the side it takes, all 64
// lanes are active at every barrier.
__device__ __forceinline__ void tile_barrier()
{
    if (__builtin_amdgcn_read_exec() != 0ull)
        __syncthreads();
}

// EDGE: this wave runs the full step (an end, the source or a probe is in
// it, as full_step_wave decides); every other wave runs the interior step,
// compiled without any of that code.
template <typename R, int C, int KIND, bool NEG, bool RING, bool WIN, bool MW, bool EDGE>
__device__ __forceinline__ void tile_body(const RunDesc *__restrict__ rd,
                                          int tile, int w, int G_, int64_t block, int T,
                                          R *__restrict__ xbuf)
{
    const int G = MW ? G_ : 1;          // one-wave tiles carry no refresh code
    // The full step's single-cell updates (source, end nodes, probe reads)
    // at a wave-uniform register: for narrow lanes as selects over the
    // registers (no branches: a lone run is bound by the latency of a step),
    // for wide lanes as branches to the one register (throughput tilings,
    // where the full-step tiles share the SIMDs with the others and
    // O(C) selects per step cost more than the branches).
    constexpr bool kSelects = C <= 8;
    constexpr bool kMatter = (KIND == GFDTD_MATTER);
    const int lane = threadIdx.x & (kWave - 1);

    const int64_t nz = rd->nz;
    const int64_t steps = rd->steps;
    const int64_t lb = block - rd->start_block;
    const int64_t n0 = lb * T + 1;
    if (lb < 0 || n0 > steps)
        return;
    const int nsub = (int)((steps - n0 + 1) < T ? (steps - n0 + 1) : T);
    const bool last = (n0 + nsub - 1 == steps);
    const int par = (int)(lb & 1);

    const double bS64 = rd->bS;
    const double beta64 = rd->beta;
    const double invS64 = 1.0 / rd->S;
    // Star fields are carried scaled by S (E~ = S E*, H~ = S H*), with
    // S-scaled coefficients.
    const R bS = (R)bS64;
    const R hb = (R)rd->hb;             // S beta / 2
    const R k1 = (R)(bS64 - rd->hb);    // weights of the folded updates
    const R k2 = (R)(-rd->hb);
    const int hl = rd->hl;
    const int hr = rd->hr;
    const int abc = rd->abc;
    const int nprobe = rd->nprobe;
    const int64_t W = (int64_t)kWave * C;
    // A tile is G waves side by side (wave w of the tile here).  Adjacent
    // waves share ov = xl + xr lanes: every xk steps each refreshes its
    // outer xl (left) and xr (right) lanes from its neighbours, which hold
    // them inside their own valid region.  The tile's outer ends carry the
    // halos hl and hr of the whole T-step block.
    const int xl = G > 1 ? rd->xl : 0;
    const int xr = G > 1 ? rd->xr : 0;
    const int xk = rd->xk;
    const int ov = xl + xr;
    const int64_t x0 = (int64_t)tile * rd->own_cells - (int64_t)hl * C +
                       (int64_t)w * (kWave - ov) * C;
    const int64_t kb = x0 + (int64_t)lane * C;
    if (MW && G > 1 && !RING && x0 >= nz) {
        // entirely past the grid end: nothing to step, but the tile's
        // waves meet at every refresh; the left neighbour reads zeros
        const int nx = (nsub - 1) / xk;
        for (int e = 0; e < nx; ++e) {
            R *p = xbuf + ((e & 1) * kMaxTileWaves + w) * kXStride +
                   (NEG ? 2 * kXSlot : kXCoefFields * kXSlot);
            for (int i = lane; i < (NEG ? kXCoefFields : 2) * kXSlot; i += kWave)
                p[i] = (R)0;
            tile_barrier();
        }
        return;
    }
    const int own_l = w == 0 ? hl : xl;             // owned lanes [own_l, own_r)
    const int own_r = w == G - 1 ? kWave - hr : kWave - xr;

    const R *__restrict__ Dsrc = static_cast<const R *>(rd->D[par]);
    const R *__restrict__ Bsrc = static_cast<const R *>(rd->B[par]);
    const auto Dsg = glb(Dsrc);        // the same, in the global address space
    const auto Bsg = glb(Bsrc);
    R *__restrict__ Ddst = static_cast<R *>(rd->D[par ^ 1]);
    R *__restrict__ Bdst = static_cast<R *>(rd->B[par ^ 1]);
    const auto cEp = glb(static_cast<const R *>(rd->cE));
    const auto cHp = glb(static_cast<const R *>(rd->cH));
    const auto gBp = glb(static_cast<const R *>(rd->gB));

    // On a ring every index is taken modulo nz: a window that crosses an
    // end (or a ring shorter than the window) loads cell by cell.
    const int64_t kw = RING ? wrapi(kb, nz) : kb;
    R D[C], B[C];
    if (RING && (x0 < 0 || x0 + W > nz)) {
        int64_t i = kw;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            D[c] = Dsg[i];
            B[c] = Bsg[i];
            i = ring_next(i, nz);
        }
    } else {
        load_cells<R, C>(Dsrc + kb, D);
        load_cells<R, C>(Bsrc + kb, B);
    }

    // Coefficient windows.  A window holds the coefficients of this lane's
    // cells for a profile displaced by m cells (clamped to the grid, or
    // wrapped on a ring); with a finite-duration modulation it holds the
    // background coefficient while the profile is switched off.
    R ce[C], ch[C], ge[C], gh[C];
    // Window indices are clamped in 32 bits: nz < 2^31 - 2^20 is validated,
    // and kb - m is saturated to a range whose ends clamp to the same grid
    // cells, so base + c cannot overflow.
    const int nz32 = (int)nz;
    auto win_base = [&](int m) __attribute__((always_inline)) {
        const int64_t b = kb - m;
        constexpr int64_t lo = -(int64_t(1) << 30), hi = (int64_t(1) << 31) - 64;
        return (int)(b < lo ? lo : (b > hi ? hi : b));
    };
    auto load_e = [&](int m) __attribute__((always_inline)) {
        if constexpr (RING) {
            int64_t i = wrapi(kb - m, nz);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                ce[c] = cEp[i];
                if constexpr (kMatter)
                    ge[c] = gBp[i];
                i = ring_next(i, nz);
            }
        } else {
            const int base = win_base(m);
            if (x0 - m >= 0 && x0 - m + W <= nz) {
                // the whole wave's window lies on the grid: no clamps
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    ce[c] = cEp[base + c];
                    if constexpr (kMatter)
                        ge[c] = gBp[base + c];
                }
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int i = min(max(base + c, 0), nz32 - 1);
                    ce[c] = cEp[i];
                    if constexpr (kMatter)
                        ge[c] = gBp[i];
                }
            }
        }
    };
    auto load_h = [&](int m) __attribute__((always_inline)) {
        if constexpr (RING) {
            int64_t i = wrapi(kb - m, nz);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                ch[c] = cHp[i];
                if constexpr (kMatter)
                    gh[c] = gBp[i];
                i = ring_next(i, nz);
            }
        } else {
            const int base = win_base(m);
            if (x0 - m >= 0 && x0 - m + W <= nz - 1) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    ch[c] = cHp[base + c];
                    if constexpr (kMatter)
                        gh[c] = gBp[base + c];
                }
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int i = min(max(base + c, 0), nz32 - 2);
                    ch[c] = cHp[i];
                    if constexpr (kMatter)
                        gh[c] = gBp[i];
                }
            }
        }
    };
    // Finite-duration modulation (moving modulation only): whether the
    // profile exists at node time tau S, and the background windows.
    constexpr bool windowed = !kMatter && WIN;
    const double S64 = rd->S;
    auto active = [&](double tau) __attribute__((always_inline)) {
        const double t = tau * S64;
        return t >= rd->t_on && t < rd->t_off;
    };
    auto fill_e = [&]() __attribute__((always_inline)) {
        const R v = (R)rd->cEb;
#pragma unroll
        for (int c = 0; c < C; ++c)
            ce[c] = v;
    };
    auto fill_h = [&]() __attribute__((always_inline)) {
        const R v = (R)rd->cHb;
#pragma unroll
        for (int c = 0; c < C; ++c)
            ch[c] = v;
    };

    // coefficients for the first step of the block: E nodes at n0-1/2,
    // H nodes at n0 (times exact in FP64).
    const int mE = profile_shift32(bS64, (double)n0 - 0.5);
    const int mH = profile_shift32(bS64, (double)n0);
    if (windowed && !active((double)n0 - 0.5))
        fill_e();
    else
        load_e(mE);
    if (windowed && !active((double)n0))
        fill_h();
    else
        load_h(mH);
    (void)fill_e;
    (void)fill_h;

    // Full step: its reads (the probe table; the first chunk's source
    // samples and end coefficients, lane j for step j) are issued here,
    // with the field and coefficient loads, so their latencies overlap.
    int64_t kpl0 = -1;
    double src0 = 0.0, cL0 = 0.0, cR0 = 0.0;
    if constexpr (EDGE) {
        if (lane < nprobe)
            kpl0 = glb(rd->probes)[lane];
        const int64_t nl = n0 + lane;
        if (lane < nsub && nl <= rd->nsrc)
            src0 = glb(rd->src)[nl - 1];
        if (!RING && abc == GFDTD_ABC_MUR1 && lane < nsub) {
            const double te = (double)nl + 0.5;
            const int mEl = profile_shift32(bS64, te);
            const bool onl = !windowed || active(te);
            if (x0 < 0)
                cL0 = onl ? glb(rd->murL)[clampi(-mEl, 0, nz - 1)] : rd->murB;
            if (x0 + W > nz - 1)
                cR0 = onl ? glb(rd->murR)[clampi(nz - 1 - mEl, 0, nz - 1)] : rd->murB;
        }
    }

    // a ring has no ends
    const bool touchL = EDGE && !RING && x0 < 0;            // E node 0 (and ghosts)
    const bool touchR = EDGE && !RING && x0 + W > nz - 1;   // node nz-1 (and ghosts)

    // Off the grid B takes the edge value (zero-gradient extension).  A
    // cell on the grid reads only two ghost cells: B_{-1}, B_{-2} through
    // the column a terms (E nodes 0 and 1), B_{nz-1}, B_{nz} through the
    // column b terms (E node nz-1).  Every other off-grid value reaches
    // only the end nodes, which the end condition then overwrites, and
    // other off-grid cells.  Narrow lanes set just those two cells, on the
    // side the active column reads; wide lanes fill every off-grid cell.
    // Narrow lanes, from ln = this lane, l0 = the lane whose register 0 is
    // node 0 and dR = ln * C - (nz - 1 - x0) (node nz-1 is where dR + c ==
    // 0); an end the wave does not hold has l0 or dR that no cell matches
    // (end_index below).
    auto ghosts_n = [&](R (&Bv)[C], int ln, int l0, int dR) __attribute__((always_inline)) {
        if constexpr (!NEG) {
            // x0 is a multiple of C: the ghosts are registers C-1, C-2 of
            // lane l0 - 1
            const R b0 = from_right(Bv[0]);
            const bool at = ln == l0 - 1;
            Bv[C - 1] = at ? b0 : Bv[C - 1];
            Bv[C - 2] = at ? b0 : Bv[C - 2];
        } else {
            // cell nz-1 (dR + c == 0) takes its left neighbour, cell nz
            // (dR + c == 1) the one two to its left: both B_{nz-2}
            const R l1 = from_left(Bv[C - 1]), l2 = from_left(Bv[C - 2]);
            R nb[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const R p1 = c >= 1 ? Bv[c >= 1 ? c - 1 : 0] : l1;
                const R p2 = c >= 2 ? Bv[c >= 2 ? c - 2 : 0] : (c == 1 ? l1 : l2);
                nb[c] = (dR == -c) ? p1 : ((dR == 1 - c) ? p2 : Bv[c]);
            }
#pragma unroll
            for (int c = 0; c < C; ++c)
                Bv[c] = nb[c];
        }
    };
    constexpr int kNoCell = -(1 << 30);
    auto end_index = [&](int ln, int &l0, int &dR) __attribute__((always_inline)) {
        l0 = touchL ? (int)(-x0 / C) : kNoCell;
        dR = touchR ? ln * C - (int)(nz - 1 - x0) : kNoCell;
    };
    auto ghosts = [&](R (&Bv)[C]) __attribute__((always_inline)) {
        if constexpr (kSelects) {
            int l0, dR;
            end_index(lane, l0, dR);
            ghosts_n(Bv, lane, l0, dR);
            return;
        }
        if (touchL) {
            const int l0 = (int)(-x0 / C);
            const R b0 = readlane_r(Bv[0], l0);
#pragma unroll
            for (int c = 0; c < C; ++c)
                Bv[c] = (kb + c < 0) ? b0 : Bv[c];
        }
        if (touchR) {
            const int64_t r = nz - 2 - x0;
            const R bl = readlane_r(pick<R, C>(Bv, (int)(r % C)), (int)(r / C));
#pragma unroll
            for (int c = 0; c < C; ++c)
                Bv[c] = (kb + c >= nz - 1) ? bl : Bv[c];
        }
    };
    if (touchL || touchR)
        ghosts(B);

    // The source cell: lane ls, register cs.  On a ring every copy of the
    // source cell inside the window takes the source: bit c of smask for
    // register c of this lane.
    const int64_t ks = rd->src_cell;
    bool hasSrc = false;
    int ls = -1, cs = 0;
    unsigned smask = 0u;
    if (EDGE && rd->nsrc > 0) {
        if constexpr (RING) {
            int64_t i = kw;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (i == ks)
                    smask |= 1u << c;
                i = ring_next(i, nz);
            }
            hasSrc = __ballot(smask != 0u) != 0;
        } else if (ks >= x0 && ks < x0 + W) {
            hasSrc = true;
            ls = (int)((ks - x0) / C);
            cs = (int)((ks - x0) % C);
        }
    }
    const int64_t own_lo = x0 + (int64_t)own_l * C;
    const int64_t own_hi = x0 + (int64_t)own_r * C;

    R Es[C], sums[C];
    R D2[C], B2[C];   // second register set of the ping-pong step pair
    R Bup = (R)0;     // B of the cell just outside this lane, upwind side

    // E~ = S E* of every cell from the current (D, B) and the E
    // coefficients ((10c) with the Table 1 B average, scaled by S).
    auto compute_es = [&](const R (&Dc)[C], const R (&Bc)[C]) __attribute__((always_inline)) {
        if constexpr (!NEG) {
            const R Bm1 = from_left(Bc[C - 1]);
            const R Bm2 = from_left(Bc[C - 2]);
            Bup = Bm1;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const R b1 = (c >= 1) ? Bc[c >= 1 ? c - 1 : 0] : Bm1;
                const R b2 = (c >= 2) ? Bc[c >= 2 ? c - 2 : 0] : (c == 1 ? Bm1 : Bm2);
                sums[c] = b1 + b2;
            }
        } else {
            const R Bp1 = from_right(Bc[0]);
            Bup = Bp1;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const R b1 = (c + 1 < C) ? Bc[c + 1 < C ? c + 1 : 0] : Bp1;
                sums[c] = b1 + Bc[c];
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if constexpr (kMatter)
                Es[c] = fmad(Dc[c], ce[c], -(ge[c] * sums[c]));
            else
                Es[c] = fmad(Dc[c], ce[c], -(hb * sums[c]));
        }
    };

    // Physical E = E* + beta Bbar at the owned probes, for time n-1/2
    // (E* = E~ / S).  Lane q of the probe table describes probe q: plc =
    // lane * C + register of its cell in this tile, prow = its trace row
    // (the value for time n-1/2 goes to prow[n-2]); bit q of pmask says this
    // tile owns it.
    // E at time n-1/2 from E~ and the B average sm: E* + beta Bbar =
    // E~ / S + beta sm / 2.
    auto probe_value = [&](R e, R sm) __attribute__((always_inline)) {
        return fmad((double)e, invS64, beta64 * (0.5 * (double)sm));
    };
    // The general probe path (Es and sums of every cell computed first):
    // one probe after another from the table, the owning lane storing.
    auto record = [&](int64_t n, int plc, double *prow, uint64_t pm)
                      __attribute__((always_inline)) {
        for (uint64_t m = pm; m != 0ull; m &= m - 1ull) {
            const int q = (int)__builtin_ctzll(m);
            const int pc = readlane_i(plc, q);
            double *row = reinterpret_cast<double *>(
                readlane_i64(reinterpret_cast<int64_t>(prow), q));
            const R e = pick<R, C>(Es, pc % C);
            const R sm = pick<R, C>(sums, pc % C);
            if (lane == pc / C)
                glb(row)[n - 2] = probe_value(e, sm);
        }
    };
    // One probe at register reg of lane pl (both wave-uniform), from Es and
    // sums already formed: the two values picked in the vector unit, read
    // from lane pl, and the wave-uniform result stored by every lane to one
    // address (no branch, no change of the execution mask).
    auto record_one = [&](int64_t n, int pl, int reg, double *row) __attribute__((always_inline)) {
        const int rg = fresh_s(reg);
        const R e = readlane_r(pick_w<R, C>(Es, rg), pl);
        const R sm = readlane_r(pick_w<R, C>(sums, rg), pl);
        glb(row)[n - 2] = probe_value(e, sm);
    };

    // Shifts of the coefficient windows.  Over one step the profile moves
    // by 0 or dir = sign(beta) cells at each node type (|beta S| <= 0.9), so
    // a shift moves a window by exactly one cell.
    constexpr int dir = NEG ? -1 : 1;
    auto shift_e = [&]() __attribute__((always_inline)) {
        shift_window<R, C, NEG>(ce);
        if constexpr (kMatter)
            shift_window<R, C, NEG>(ge);
    };
    auto shift_h = [&]() __attribute__((always_inline)) {
        shift_window<R, C, NEG>(ch);
        if constexpr (kMatter)
            shift_window<R, C, NEG>(gh);
    };

    // What the full step needs besides the fields, per 64-step chunk (see
    // steps_loop).
    struct EdgeChunk {
        R src, cL, cR;          // lane j: step j's source sample, end coefficients
        int nsrc_q;             // steps q < nsrc_q of the chunk add the source
        int plc;                // lane q: probe q's cell in the wave (lane * C + reg)
        double *prow;           // lane q: probe q's trace row
        uint64_t pmask;         // bit q: this tile owns probe q
        uint64_t prest;         // owned probes left to the general path
        int np;                 // owned probes held as wave-uniform values (0..2)
        int pl0, pr0, pl1, pr1; // their lane and register
        double *row0, *row1;    // their trace rows
    };

    // One time step n (step q of its chunk) with fixed coefficient windows,
    // from (Di, Bi) to (Dn, Bn).  The full step also adds the source,
    // imposes the end conditions and records the probes from ec.
    auto one_step = [&](auto edge_tag, int64_t n, int q, const EdgeChunk &ec,
                        const R (&Di)[C], const R (&Bi)[C], R (&Dn)[C], R (&Bn)[C])
                        __attribute__((always_inline)) {
        constexpr bool kEdge = decltype(edge_tag)::value;
        // E at time n-1/2 of the owned probes (none at step 1, the run's
        // first E time being 3/2)
        auto probes_now = [&]() __attribute__((always_inline)) {
            if constexpr (kSelects) {
                // np >= 1 here (narrow lanes take the first two owned
                // probes as wave-uniform values)
                if constexpr (!kMatter)
                    compute_es(Di, Bi);
                record_one(n, ec.pl0, ec.pr0, ec.row0);
                if (ec.np >= 2) {
                    record_one(n, ec.pl1, ec.pr1, ec.row1);
                    if (ec.prest != 0ull)
                        record(n, ec.plc, ec.prow, ec.prest);
                }
            } else {
                if constexpr (!kMatter)
                    compute_es(Di, Bi);
                record(n, ec.plc, ec.prow, ec.pmask);
            }
        };

        // (10a) Faraday with the Table 1 dB/dz, in telescoped form:
        //   P_k = E~_k + bS B_up(k),  B' = B + (P_k - P_{k+1}),
        // B_up(k) = B_{k-1} (column a) or B_k (column b).  A uniform field
        // stays exactly uniform.  For a moving modulation E~ (10c) is
        // folded in: P_k = cE D_k + (bS - hb) B_1 - hb B_2 with
        // (B_1, B_2) = (B_{k-1}, B_{k-2}) in column a, (B_k, B_{k+1}) in
        // column b; E~ itself is formed only where a probe needs it.
        R P[C];
        if constexpr (!kMatter) {
            if (kEdge && ec.pmask != 0ull && n != 1)
                probes_now();
            if constexpr (!NEG) {
                const R Bm1 = from_left(Bi[C - 1]);
                const R Bm2 = from_left(Bi[C - 2]);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const R b1 = (c >= 1) ? Bi[c >= 1 ? c - 1 : 0] : Bm1;
                    const R b2 = (c >= 2) ? Bi[c >= 2 ? c - 2 : 0] : (c == 1 ? Bm1 : Bm2);
                    P[c] = fmad(Di[c], ce[c], fmad(k1, b1, k2 * b2));
                }
            } else {
                const R Bp1 = from_right(Bi[0]);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const R b2 = (c + 1 < C) ? Bi[c + 1 < C ? c + 1 : 0] : Bp1;
                    P[c] = fmad(Di[c], ce[c], fmad(k1, Bi[c], k2 * b2));
                }
            }
        } else {
            compute_es(Di, Bi);
            if (kEdge && ec.pmask != 0ull && n != 1)
                probes_now();
#pragma unroll
            for (int c = 0; c < C; ++c) {
                R bsel;
                if constexpr (!NEG)
                    bsel = (c >= 1) ? Bi[c >= 1 ? c - 1 : 0] : Bup;
                else
                    bsel = Bi[c];
                P[c] = fmad(bS, bsel, Es[c]);
            }
        }
        const R PR = from_right(P[0]);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const R pn = (c + 1 < C) ? P[c + 1 < C ? c + 1 : 0] : PR;
            Bn[c] = Bi[c] + (P[c] - pn);
        }
        // (10d) H~ = S H* with the Table 1 D average and (10b) Ampere with
        // the Table 1 dD/dz, telescoped:
        //   X_k = H~_k + bS D_sel(k),  D' = D + (X_{k-1} - X_k),
        // D_sel(k) = D_k (column a) or D_{k+1} (column b); for a moving
        // modulation X_k = cH B'_k + (bS - hb) D_1 - hb D_2 with
        // (D_1, D_2) = (D_k, D_{k+1}) in column a, (D_{k+1}, D_k) in column b.
        const R DR = from_right(Di[0]);
        R X[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const R dn = (c + 1 < C) ? Di[c + 1 < C ? c + 1 : 0] : DR;
            if constexpr (!kMatter) {
                if constexpr (!NEG)
                    X[c] = fmad(Bn[c], ch[c], fmad(k1, Di[c], k2 * dn));
                else
                    X[c] = fmad(Bn[c], ch[c], fmad(k1, dn, k2 * Di[c]));
            } else {
                const R hs = fmad(Bn[c], ch[c], -(gh[c] * (dn + Di[c])));
                X[c] = fmad(bS, NEG ? dn : Di[c], hs);
            }
        }
        const R XL = from_left(X[C - 1]);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const R xp = (c >= 1) ? X[c >= 1 ? c - 1 : 0] : XL;
            Dn[c] = Di[c] + (xp - X[c]);
        }
        // soft source
        if (kEdge && hasSrc && q < ec.nsrc_q) {
            const R g = readlane_r(ec.src, q);
            if constexpr (RING) {
                if (smask) {
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        if ((smask >> c) & 1u)
                            Dn[c] += g;
                }
            } else if constexpr (kSelects) {
                // the source cell is where d + c == 0
                const int d = fresh_v(lane) * C - (int)(ks - x0);
#pragma unroll
                for (int c = 0; c < C; ++c)
                    Dn[c] = (d == -c) ? Dn[c] + g : Dn[c];
            } else if (lane == ls) {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (c == cs)
                        Dn[c] += g;
            }
        }
        // end nodes, at time n+1/2, and the ghost cells; narrow lanes do
        // both ends in one block without branches
        if constexpr (kSelects && !RING) {
            if (kEdge && (touchL || touchR)) {
                const bool mur = abc == GFDTD_ABC_MUR1;
                const int ln = fresh_v(lane);
                int l0, dR;
                end_index(ln, l0, dR);
                const R cL = readlane_r(ec.cL, q);
                const R vL = mur ? fmad(cL, Dn[1] - Di[0], Di[1]) : (R)0;
                Dn[0] = (ln == l0) ? vL : Dn[0];
                // node nz-1 from its left neighbour's old and new values,
                // formed in every cell and kept in that one
                const R cR = readlane_r(ec.cR, q);
                const R dlo = from_left(Di[C - 1]);
                const R dln = from_left(Dn[C - 1]);
                R nd[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const R po = c >= 1 ? Di[c >= 1 ? c - 1 : 0] : dlo;
                    const R pn = c >= 1 ? Dn[c >= 1 ? c - 1 : 0] : dln;
                    const R v = mur ? fmad(cR, pn - Di[c], po) : (R)0;
                    nd[c] = (dR == -c) ? v : Dn[c];
                }
#pragma unroll
                for (int c = 0; c < C; ++c)
                    Dn[c] = nd[c];
                ghosts_n(Bn, ln, l0, dR);
            }
            return;
        }
        if (kEdge && touchL) {
            const int l0 = (int)(-x0 / C);
            const R cL = readlane_r(ec.cL, q);
            const R v = (abc == GFDTD_ABC_MUR1) ? fmad(cL, Dn[1] - Di[0], Di[1]) : (R)0;
            Dn[0] = (lane == l0) ? v : Dn[0];
        }
        if (kEdge && touchR) {
            const int64_t r = nz - 1 - x0;
            const int lr = (int)(r / C);
            const int cr = (int)(r % C);
            const R cR = readlane_r(ec.cR, q);
            const R dlo = from_left(Di[C - 1]);
            const R dln = from_left(Dn[C - 1]);
            const bool atR = lane == lr;
            if (atR) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if (c == cr) {
                        const R po = (c >= 1) ? Di[c >= 1 ? c - 1 : 0] : dlo;
                        const R pn = (c >= 1) ? Dn[c >= 1 ? c - 1 : 0] : dln;
                        Dn[c] = (abc == GFDTD_ABC_MUR1) ? fmad(cR, pn - Di[c], po) : (R)0;
                    }
                }
            }
        }
        if (kEdge && (touchL || touchR))
            ghosts(Bn);
    };

    // Overlap refresh of a multi-wave tile through LDS.  Per wave and
    // buffer: slot R = the lanes [64-ov, 64-xr) the right neighbour holds
    // as its left overlap, slot L = the lanes [xl, ov) the left neighbour
    // holds as its right overlap; D and B, and on the side where window
    // shifts bring in a cell from the neighbouring lane (the left for
    // column a, the right for column b) also the coefficient windows,
    // whose new edge cell is only valid inside the halo.  Two buffers
    // alternate, so one barrier per refresh suffices: a wave rewrites a
    // buffer only after the next barrier, which every wave reaches after
    // its reads of that buffer.
    int nxch = 0;
    constexpr int offL = NEG ? 2 * kXSlot : kXCoefFields * kXSlot;
    auto put = [&](R *p, auto coef_tag) __attribute__((always_inline)) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            p[c] = D[c];
            p[kXSlot + c] = B[c];
            if constexpr (decltype(coef_tag)::value) {
                p[2 * kXSlot + c] = ce[c];
                p[3 * kXSlot + c] = ch[c];
                if constexpr (kMatter) {
                    p[4 * kXSlot + c] = ge[c];
                    p[5 * kXSlot + c] = gh[c];
                }
            }
        }
    };
    auto get = [&](const R *p, auto coef_tag) __attribute__((always_inline)) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            D[c] = p[c];
            B[c] = p[kXSlot + c];
            if constexpr (decltype(coef_tag)::value) {
                ce[c] = p[2 * kXSlot + c];
                ch[c] = p[3 * kXSlot + c];
                if constexpr (kMatter) {
                    ge[c] = p[4 * kXSlot + c];
                    gh[c] = p[5 * kXSlot + c];
                }
            }
        }
    };
    using CoefR = std::integral_constant<bool, !NEG>;   // slot R carries windows
    using CoefL = std::integral_constant<bool, NEG>;    // slot L carries windows
    auto exchange = [&]() __attribute__((always_inline)) {
        // every address is lane * C plus a wave-uniform offset
        R *lp = xbuf + lane * C + ((nxch & 1) * kMaxTileWaves + w) * kXStride;
        if (w + 1 < G && lane >= kWave - ov && lane < kWave - xr)
            put(lp - (kWave - ov) * C, CoefR{});
        if (w > 0 && lane >= xl && lane < ov)
            put(lp + offL - xl * C, CoefL{});
        tile_barrier();
        if (w > 0 && lane < xl)
            get(lp - kXStride, CoefR{});
        if (w + 1 < G && lane >= kWave - xr)
            get(lp + kXStride + offL - (kWave - xr) * C, CoefL{});
        ++nxch;
    };

    // The step loop.  The shift schedule of 64 steps at a time is computed
    // in FP64 by the per-node rule m = rint(beta S tau), one step per lane,
    // and kept as wave-wide bit masks: bit j of hmask = the H window moves
    // before step j of the chunk, bit j of emask = the E window moves after
    // it.  The steps between two moves run with fixed windows.  The loop is
    // compiled twice: tiles holding an end, the source or a probe run the
    // full step; interior tiles (nearly all of them) run one without that
    // code.
    auto steps_loop = [&](auto edge_tag) __attribute__((always_inline)) {
        constexpr bool kEdge = decltype(edge_tag)::value;
        int mEc = mE;                       // E shift at the current n - 1/2
        int mHc = mH;                       // H shift at the current n
        int nextx = G > 1 ? xk : nsub;      // step count of the next refresh
        // Full step only: the probe table (lane q: probe q), the first two
        // owned probes as wave-uniform values, and per 64-step chunk lane j
        // holds step j's source sample and end coefficients, so the steps
        // read no memory.  Kept inside this loop: declared for the whole
        // tile they raise the register allocation of the interior loop too.
        EdgeChunk ec{};
        if constexpr (kEdge) {
            const int64_t kpl = kpl0;
            const bool own = lane < nprobe && kpl >= own_lo && kpl < own_hi;
            ec.pmask = __ballot(own);
            ec.plc = own ? (int)(kpl - x0) : 0;
            ec.prow = rd->trace + (lane < nprobe ? (int64_t)lane * steps : 0);
            uint64_t m = ec.pmask;
            if constexpr (kSelects) {
                if (m != 0ull) {
                    const int q = (int)__builtin_ctzll(m);
                    const int pc = readlane_i(ec.plc, q);
                    ec.pl0 = pc / C;
                    ec.pr0 = pc % C;
                    ec.row0 = reinterpret_cast<double *>(
                        readlane_i64(reinterpret_cast<int64_t>(ec.prow), q));
                    ec.np = 1;
                    m &= m - 1ull;
                }
                if (m != 0ull) {
                    const int q = (int)__builtin_ctzll(m);
                    const int pc = readlane_i(ec.plc, q);
                    ec.pl1 = pc / C;
                    ec.pr1 = pc % C;
                    ec.row1 = reinterpret_cast<double *>(
                        readlane_i64(reinterpret_cast<int64_t>(ec.prow), q));
                    ec.np = 2;
                    m &= m - 1ull;
                }
            }
            ec.prest = m;
        }
        for (int s0 = 0; s0 < nsub; s0 += kWave) {
            const int len = nsub - s0 < kWave ? nsub - s0 : kWave;
            const int sl = s0 + lane;
            const double tn = (double)(n0 + sl);
            const bool hbit = sl > 0 && sl < nsub &&
                              profile_shift32(bS64, tn) != profile_shift32(bS64, tn - 1.0);
            const bool ebit = sl < nsub &&
                              profile_shift32(bS64, tn + 0.5) != profile_shift32(bS64, tn - 0.5);
            const uint64_t hmask = __ballot(hbit);
            const uint64_t emask = __ballot(ebit);
            if constexpr (kEdge) {
                // this lane's step n = n0 + sl: its source sample and, at
                // the E time n+1/2, the end coefficients of the medium then
                // under the end nodes (the background one while a time
                // window has the profile off)
                const int64_t nl = n0 + sl;
                // chunk 0's were read at the start of the tile
                double srcv = s0 == 0 ? src0 : 0.0;
                double cLv = s0 == 0 ? cL0 : 0.0, cRv = s0 == 0 ? cR0 : 0.0;
                if (s0 > 0 && hasSrc && sl < nsub && nl <= rd->nsrc)
                    srcv = glb(rd->src)[nl - 1];
                if (s0 > 0 && (touchL || touchR) && abc == GFDTD_ABC_MUR1 && sl < nsub) {
                    const int mEl = profile_shift32(bS64, tn + 0.5);
                    const bool onl = !windowed || active(tn + 0.5);
                    if (touchL)
                        cLv = onl ? glb(rd->murL)[clampi(-mEl, 0, nz - 1)] : rd->murB;
                    if (touchR)
                        cRv = onl ? glb(rd->murR)[clampi(nz - 1 - mEl, 0, nz - 1)] : rd->murB;
                }
                ec.src = (R)srcv;
                ec.cL = (R)cLv;
                ec.cR = (R)cRv;
                // steps n0 + s0 + q <= nsrc take the source
                const int64_t ns = rd->nsrc - (n0 + s0) + 1;
                ec.nsrc_q = ns < 0 ? 0 : (ns > kWave ? kWave : (int)ns);
            }
            // finite-duration modulation: bit j of hsw / esw = the H / E
            // window switches (on or off) before / after step j; hact /
            // eact = the profile exists at the H time of step j / at the
            // E time after it
            uint64_t hsw = 0, esw = 0, hact = ~0ull, eact = ~0ull;
            if constexpr (windowed) {
                const bool aH = active(tn), aE = active(tn + 0.5);
                hact = __ballot(aH);
                eact = __ballot(aE);
                hsw = __ballot(sl > 0 && sl < nsub && aH != active(tn - 1.0));
                esw = __ballot(sl < nsub && aE != active(tn - 0.5));
            }
            // a move, switch or overlap refresh (every xk steps of a
            // multi-wave tile, not after the last) after step j
            const uint64_t bmask =
                emask | (hmask >> 1) | esw | (hsw >> 1) |
                (G > 1 ? __ballot(sl + 1 < nsub && (sl + 1) % xk == 0) : 0ull);
            auto update_h = [&](int q) __attribute__((always_inline)) {
                if ((hmask >> q) & 1ull) {
                    shift_h();
                    mHc += dir;
                }
                if constexpr (windowed) {
                    if ((hsw >> q) & 1ull) {
                        if ((hact >> q) & 1ull)
                            load_h(mHc);
                        else
                            fill_h();
                    }
                }
            };
            update_h(0);
            int j = 0;
            while (j < len) {
                const uint64_t rest = bmask >> j;
                const int stop = rest ? j + (int)__builtin_ctzll(rest) : len - 1;
                // two steps at a time, ping-ponging between register sets
                // (D, B) and (D2, B2), so no copies between steps
                int q = j;
                for (; q + 1 <= stop; q += 2) {
                    one_step(edge_tag, n0 + s0 + q, q, ec, D, B, D2, B2);
                    one_step(edge_tag, n0 + s0 + q + 1, q + 1, ec, D2, B2, D, B);
                }
                if (q <= stop) {
                    one_step(edge_tag, n0 + s0 + q, q, ec, D, B, D2, B2);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        D[c] = D2[c];
                        B[c] = B2[c];
                    }
                }
                if (MW && s0 + stop + 1 == nextx && nextx < nsub) {
                    exchange();
                    nextx += xk;
                }
                if ((emask >> stop) & 1ull) {
                    shift_e();
                    mEc += dir;
                }
                if constexpr (windowed) {
                    if ((esw >> stop) & 1ull) {
                        if ((eact >> stop) & 1ull)
                            load_e(mEc);
                        else
                            fill_e();
                    }
                }
                if (stop + 1 < len)
                    update_h(stop + 1);
                j = stop + 1;
            }
        }

        if (kEdge && last && ec.pmask != 0ull) {   // the run ends in this block: E at N+1/2
            compute_es(D, B);
            record(steps + 1, ec.plc, ec.prow, ec.pmask);
        }
    };
    steps_loop(std::integral_constant<bool, EDGE>{});

    if (lane >= own_l && lane < own_r) {
        store_cells<R, C>(Ddst + kb, D);
        store_cells<R, C>(Bdst + kb, B);
    }
}

// Occupancy target: waves per SIMD the register allocation must allow
// (512 registers per SIMD lane, at most 8 waves).  Stated because the
// compiler, left to itself, may give up a wave for one or two registers of
// the full-step loop (FP64 at 12 cells per lane took 169 registers, 2 waves,
// instead of 168, 3).  Some targets leave a few bytes of spill in the
// full-step (edge) code, kept where measured faster than one wave less:
// FP64 modulation at 12 cells per lane, 3 waves with 28 bytes a lane, ran
// the crystal batch at 2.30e12 against 2.22e12 with 2 waves and none.  FP32
// at 8 and FP64 at 4 cells per lane take 6 waves without spill (the FP64
// slab 1.32e11 against 1.29e11 with 7 waves and 28 bytes).
template <typename R, int C, int KIND, bool MW>
constexpr int occupancy_target()
{
    if constexpr (sizeof(R) == 4) {
        if constexpr (KIND == GFDTD_MODULATION)
            return C == 4 ? 8 : C == 8 ? 6 : C == 12 ? 5 : 4;
        return C == 4 ? 8 : C == 8 ? 5 : C == 12 ? 4 : 3;
    } else {
        if constexpr (KIND == GFDTD_MODULATION)
            return C == 4 ? (MW ? 5 : 6) : C == 8 ? 4 : C == 12 ? 3 : 2;
        return C == 4 ? 5 : C == 8 ? 3 : C == 12 ? 2 : 1;
    }
}

// Whether wave w of a tile runs the full step: it holds an end node (or an
// off-grid cell), the source cell (on a ring, any copy of it), or a probe
// it owns (owns_probe, from the tile reference).  The tile origin x0 is the
// one tile_body computes.
template <int C, bool RING, bool MW>
__device__ __forceinline__ bool full_step_wave(const RunDesc *__restrict__ rd, int tile,
                                               int w, int G_, bool owns_probe)
{
    if (owns_probe)
        return true;
    const int G = MW ? G_ : 1;
    const int ov = G > 1 ? rd->xl + rd->xr : 0;
    const int64_t W = (int64_t)kWave * C;
    const int64_t nz = rd->nz;
    const int64_t x0 = (int64_t)tile * rd->own_cells - (int64_t)rd->hl * C +
                       (int64_t)w * (kWave - ov) * C;
    if (!RING && (x0 < 0 || x0 + W > nz - 1))
        return true;
    if (rd->nsrc > 0) {
        const int64_t ks = rd->src_cell;
        if constexpr (RING)
            return wrapi(ks - x0, nz) < W;       // some cell x0 + j, j < W, is ks mod nz
        else
            return ks >= x0 && ks < x0 + W;
    }
    return false;
}

// MW = false: kWavesPerGroup independent one-wave tiles per workgroup (one).
// MW = true: one tile of G waves per workgroup (blockDim = 64 G).
template <typename R, int C, int KIND, bool RING, bool WIN, bool MW>
__global__ __launch_bounds__(kWave *(MW ? kMaxTileWaves : kWavesPerGroup))
__attribute__((amdgpu_waves_per_eu(occupancy_target<R, C, KIND, MW>()))) void k_tiles(
    const RunDesc *__restrict__ runs, const TileRef *__restrict__ tiles,
    int64_t block, int T, int ntiles, int G)
{
    __shared__ __align__(16) R xbuf[MW ? 2 * kMaxTileWaves * kXStride : 1];
    const int wv = (int)(threadIdx.x / kWave);
    const int t = __builtin_amdgcn_readfirstlane(
        MW ? (int)blockIdx.x : (int)(blockIdx.x * kWavesPerGroup) + wv);
    const int w = __builtin_amdgcn_readfirstlane(MW ? wv : 0);
    if (t >= ntiles)
        return;
    const TileRef ref = tiles[t];
    const RunDesc *rd = runs + ref.run;
    // Runs with a finite-duration modulation are stepped by the WIN
    // kernel, the others by the plain one (each skips the other's tiles),
    // so the plain kernel carries none of the window code.
    if ((KIND != GFDTD_MATTER && rd->windowed != 0) != WIN)
        return;
    // The choice of step loop is made here, before any work of the tile:
    // a value the full step alone needs, computed before a branch between
    // the two loops, would be held across the interior one too.
    const bool owns_probe = ((ref.probe_waves >> w) & 1) != 0;
    const bool edge = full_step_wave<C, RING, MW>(rd, ref.tile, w, G, owns_probe);
    if (rd->neg) {
        if (edge)
            tile_body<R, C, KIND, true, RING, WIN, MW, true>(rd, ref.tile, w, G, block, T, xbuf);
        else
            tile_body<R, C, KIND, true, RING, WIN, MW, false>(rd, ref.tile, w, G, block, T, xbuf);
    } else {
        if (edge)
            tile_body<R, C, KIND, false, RING, WIN, MW, true>(rd, ref.tile, w, G, block, T, xbuf);
        else
            tile_body<R, C, KIND, false, RING, WIN, MW, false>(rd, ref.tile, w, G, block, T, xbuf);
    }
}

template <typename R, int KIND, bool RING, bool WIN, bool MW>
static hipError_t launch_tiles_g(int C, int G, const RunDesc *runs,
                                 const TileRef *tiles, int64_t block, int T,
                                 int ntiles, hipStream_t stream)
{
    const dim3 grid(MW ? ntiles : (ntiles + kWavesPerGroup - 1) / kWavesPerGroup);
    const dim3 blk(kWave * (MW ? G : kWavesPerGroup));
    switch (C) {
    case 4:
        hipLaunchKernelGGL((k_tiles<R, 4, KIND, RING, WIN, MW>), grid, blk, 0, stream, runs,
                           tiles, block, T, ntiles, G);
        break;
    case 8:
        hipLaunchKernelGGL((k_tiles<R, 8, KIND, RING, WIN, MW>), grid, blk, 0, stream, runs,
                           tiles, block, T, ntiles, G);
        break;
    case 12:
        hipLaunchKernelGGL((k_tiles<R, 12, KIND, RING, WIN, MW>), grid, blk, 0, stream, runs,
                           tiles, block, T, ntiles, G);
        break;
    case 16:
        hipLaunchKernelGGL((k_tiles<R, 16, KIND, RING, WIN, MW>), grid, blk, 0, stream, runs,
                           tiles, block, T, ntiles, G);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Multi-wave tiles only off rings.
template <typename R, int KIND, bool RING, bool WIN>
static hipError_t launch_tiles_c(int C, int G, const RunDesc *runs,
                                 const TileRef *tiles, int64_t block, int T,
                                 int ntiles, hipStream_t stream)
{
    if (ntiles <= 0)
        return hipSuccess;
    if (G < 1 || G > kMaxTileWaves || (RING && G > 1))
        return hipErrorInvalidValue;
    if constexpr (!RING) {
        if (G > 1)
            return launch_tiles_g<R, KIND, RING, WIN, true>(C, G, runs, tiles, block, T,
                                                            ntiles, stream);
    }
    return launch_tiles_g<R, KIND, RING, WIN, false>(C, G, runs, tiles, block, T, ntiles,
                                                     stream);
}

template <typename R>
static hipError_t launch_tiles_r(int kind, bool ring, bool win, int C, int G,
                                 const RunDesc *runs, const TileRef *tiles,
                                 int64_t block, int T, int ntiles, hipStream_t stream)
{
    if (kind == GFDTD_MATTER) {        // moving matter has no time window
        if (win)
            return hipSuccess;
        return ring ? launch_tiles_c<R, GFDTD_MATTER, true, false>(C, G, runs, tiles, block, T, ntiles, stream)
                    : launch_tiles_c<R, GFDTD_MATTER, false, false>(C, G, runs, tiles, block, T, ntiles, stream);
    }
    if (win)
        return ring ? launch_tiles_c<R, GFDTD_MODULATION, true, true>(C, G, runs, tiles, block, T, ntiles, stream)
                    : launch_tiles_c<R, GFDTD_MODULATION, false, true>(C, G, runs, tiles, block, T, ntiles, stream);
    return ring ? launch_tiles_c<R, GFDTD_MODULATION, true, false>(C, G, runs, tiles, block, T, ntiles, stream)
                : launch_tiles_c<R, GFDTD_MODULATION, false, false>(C, G, runs, tiles, block, T, ntiles, stream);
}

hipError_t launch_tiles(int precision, int kind, bool ring, bool win, int C, int G,
                        const RunDesc *runs, const TileRef *tiles, int64_t block,
                        int T, int ntiles, hipStream_t stream)
{
    if (precision == GFDTD_F32)
        return launch_tiles_r<float>(kind, ring, win, C, G, runs, tiles, block, T, ntiles, stream);
    return launch_tiles_r<double>(kind, ring, win, C, G, runs, tiles, block, T, ntiles, stream);
}

// ------------------------------------------------------------- set-up

// Exit speed of a wave leaving through an end (dir = +1 right, -1 left):
// 1/n in a moving modulation, relativistic addition in moving matter.
__device__ __forceinline__ double exit_speed(int kind, double n, double beta,
                                             double dir)
{
    if (kind != GFDTD_MATTER)
        return 1.0 / n;
    const double b = dir * beta;
    return (1.0 / n + b) / (1.0 + b / n);
}

template <typename R>
__device__ __forceinline__ void prep_cell(const PrepDesc &d, int64_t i)
{
    const int64_t nz = d.nz;
    const double eps = d.eps[i];
    const double mu = d.mu[i];
    const double b = d.beta;
    // coefficients of the S-scaled star fields (E~ = S E*, H~ = S H*)
    if (d.kind == GFDTD_MATTER) {
        const double gS = (1.0 - b * b) / (eps * mu - b * b) * d.S;
        static_cast<R *>(d.cE)[i] = (R)(gS * mu);
        static_cast<R *>(d.cH)[i] = (R)(gS * eps);
        static_cast<R *>(d.gB)[i] = (R)(gS * b * 0.5);
    } else {
        static_cast<R *>(d.cE)[i] = (R)(d.S / eps);
        static_cast<R *>(d.cH)[i] = (R)(d.S / mu);
    }
    // Mur coefficients (S u - 1)/(S u + 1) for the medium an end node sees
    // when rest cell i sits under it: the left end pairs E cell i with H
    // cell i, the right end pairs E cell i with H cell i-1.
    const double nL = sqrt(eps * d.mu[i < nz - 2 ? i : nz - 2]);
    const double nR = sqrt(eps * d.mu[i > 0 ? i - 1 : 0]);
    const double uL = exit_speed(d.kind, nL, b, -1.0);
    const double uR = exit_speed(d.kind, nR, b, 1.0);
    d.murL[i] = (d.S * uL - 1.0) / (d.S * uL + 1.0);
    d.murR[i] = (d.S * uR - 1.0) / (d.S * uR + 1.0);
    if (i < d.nsrc) {      // modulated Gaussian (App. B.1) at t = (i+1) S
        const double t = (double)(i + 1) * d.S;
        const double u = (t - d.t0) / d.tau;
        d.src[i] = d.amp * sin(d.omega * (t - d.t0) + d.phase) * exp(-u * u);
    }
}

__global__ __launch_bounds__(256) void k_prep(const PrepDesc *__restrict__ descs)
{
    const PrepDesc &d = descs[blockIdx.y];
    const int64_t n = d.nz > d.nsrc ? d.nz : d.nsrc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < d.nz) {
            if (d.precision == GFDTD_F32)
                prep_cell<float>(d, i);
            else
                prep_cell<double>(d, i);
        } else if (i < d.nsrc) {
            const double t = (double)(i + 1) * d.S;
            const double u = (t - d.t0) / d.tau;
            d.src[i] = d.amp * sin(d.omega * (t - d.t0) + d.phase) * exp(-u * u);
        }
    }
}

hipError_t launch_prep(const PrepDesc *dev_descs, int count, int max_cells,
                       hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    int bx = (max_cells + 255) / 256;
    bx = bx < 1 ? 1 : (bx > 1024 ? 1024 : bx);
    hipLaunchKernelGGL(k_prep, dim3(bx, count), dim3(256), 0, stream, dev_descs);
    return hipGetLastError();
}

// Zero both halves of every field pair, padding included (a plain fill
// kernel: usable inside captured graphs).
__global__ __launch_bounds__(256) void k_zero(const PrepDesc *__restrict__ descs,
                                              int word)
{
    const PrepDesc &d = descs[blockIdx.y];
    const int64_t words16 = d.field_cells * word / 16;
    for (int f = 0; f < 4; ++f) {
        uint4 *p = reinterpret_cast<uint4 *>(static_cast<char *>(d.fields[f]) -
                                             kPad * word);
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
             i < words16; i += (int64_t)gridDim.x * blockDim.x)
            p[i] = make_uint4(0u, 0u, 0u, 0u);
    }
}

// Initial state D^{1/2}, B^0 from FP64 copies, rounded to the run
// precision, into the first half of each field pair (after k_zero).  Off a
// ring, B has nz-1 nodes and its last slot stays zero.
template <typename R>
__device__ __forceinline__ void init_cell(const PrepDesc &d, int64_t i)
{
    if (d.init_d)
        static_cast<R *>(d.fields[0])[i] = (R)d.init_d[i];
    if (d.init_b && (d.abc == GFDTD_ABC_PERIODIC || i < d.nz - 1))
        static_cast<R *>(d.fields[2])[i] = (R)d.init_b[i];
}

__global__ __launch_bounds__(256) void k_init(const PrepDesc *__restrict__ descs)
{
    const PrepDesc &d = descs[blockIdx.y];
    if (!d.init_d && !d.init_b)
        return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.nz;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (d.precision == GFDTD_F32)
            init_cell<float>(d, i);
        else
            init_cell<double>(d, i);
    }
}

hipError_t launch_init(const PrepDesc *dev_descs, int count, int64_t max_nz,
                       int precision, hipStream_t stream)
{
    (void)precision;
    if (count <= 0)
        return hipSuccess;
    int64_t bx = (max_nz + 255) / 256;
    bx = bx < 1 ? 1 : (bx > 512 ? 512 : bx);
    hipLaunchKernelGGL(k_init, dim3((unsigned)bx, count), dim3(256), 0, stream,
                       dev_descs);
    return hipGetLastError();
}

hipError_t launch_zero(const PrepDesc *dev_descs, int count,
                       int64_t max_field_cells, int precision,
                       hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    const int word = precision == GFDTD_F32 ? 4 : 8;
    int64_t bx = (max_field_cells * word / 16 + 255) / 256;
    bx = bx < 1 ? 1 : (bx > 512 ? 512 : bx);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)bx, count), dim3(256), 0, stream,
                       dev_descs, word);
    return hipGetLastError();
}

// ------------------------------------------------------------- probe DFT

// X(w) = sum_n E_n S exp(+i w t_n), t_n = (n + 1/2) S, in FP64; one block
// per (run, probe, frequency), a fixed-order reduction.
__global__ __launch_bounds__(256) void k_dft(const DftDesc *__restrict__ descs)
{
    const DftDesc &d = descs[blockIdx.y];
    const int pf = blockIdx.x;
    if (pf >= d.nprobe * d.nfreq)
        return;
    const int q = pf / d.nfreq;
    const int f = pf % d.nfreq;
    const double w = d.omegas[f];
    const double *tr = d.trace + (int64_t)q * d.steps;
    double re = 0.0, im = 0.0;
    for (int64_t i = threadIdx.x; i < d.steps; i += blockDim.x) {
        const double t = ((double)(i + 1) + 0.5) * d.S;
        double s, c;
        sincos(w * t, &s, &c);
        const double e = tr[i] * d.S;
        re += e * c;
        im += e * s;
    }
    __shared__ double sre[256];
    __shared__ double sim[256];
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sre[threadIdx.x] += sre[threadIdx.x + h];
            sim[threadIdx.x] += sim[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d.out[2 * pf] = sre[0];
        d.out[2 * pf + 1] = sim[0];
    }
}

hipError_t launch_dft(const DftDesc *dev_descs, int count, int max_pf,
                      hipStream_t stream)
{
    if (count <= 0 || max_pf <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_dft, dim3(max_pf, count), dim3(256), 0, stream, dev_descs);
    return hipGetLastError();
}

}  // namespace gfdtd
