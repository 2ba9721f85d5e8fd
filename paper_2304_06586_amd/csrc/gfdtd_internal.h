// Internal declarations shared by the HIP kernels and the host runtime of
// the generalized-FDTD library.  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gfdtd.h"

namespace gfdtd {

constexpr int kWave = 64;            // CDNA wavefront width
// Independent one-wave tiles go one per workgroup: a workgroup starts only
// when all its waves fit on a CU, so grouping independent tiles of unequal
// lifetimes leaves wave slots idle (4 per group measured 5-8 % slower).
constexpr int kWavesPerGroup = 1;
constexpr int kMaxTileWaves = 4;     // waves of one multi-wave tile (<= 4)
constexpr int kXSlot = 64;           // cells per overlap slot (>= xl C, xr C)
constexpr int kXCoefFields = 6;      // D, B and up to 4 coefficient windows
// LDS per wave and buffer: one slot of D, B, one of D, B and the windows
constexpr int kXStride = (2 + kXCoefFields) * kXSlot;
constexpr int64_t kPad = 2048;       // cells of padding before and after
                                     // every field array (>= 64 * C)

// One run as the stepping kernels see it.  Field arrays are offset so
// that index 0 is E node / H node 0 and indices [-kPad, nz + kPad) are
// addressable.  Coefficient arrays hold one entry per rest cell.
struct RunDesc {
    int64_t nz;
    int64_t steps;
    int64_t start_block;   // global block index at which step 1 runs
    int64_t nsrc;          // source samples for steps 1..nsrc
    int64_t src_cell;
    int64_t own_cells;     // cells each tile of this run stores (all waves)
    double S;              // Courant number
    double beta;
    double bS;             // beta * S (one rounding; also the shift rate)
    double hb;             // S beta / 2 (the star fields are S-scaled)
    int32_t neg;           // beta < 0: Table 1 column b
    int32_t hl;            // halo lanes left of the owned lanes
    int32_t hr;            // halo lanes right of the owned lanes
    int32_t nprobe;
    int32_t abc;           // GFDTD_ABC_* (GFDTD_ABC_PERIODIC: a ring)
    int32_t windowed;      // finite-duration modulation (t_on, t_off)
    int32_t xl, xr;        // multi-wave tiles: overlap lanes refreshed from
                           // the left / right neighbour wave
    int32_t xk;            // steps between refreshes (>= 1)
    int32_t pad0;
    void *D[2];            // ping-pong D (run precision)
    void *B[2];            // ping-pong B
    const void *cE;        // E-node coefficient: S/eps' or S g mu'
    const void *cH;        // H-node coefficient: S/mu'  or S g eps'
    const void *gB;        // moving matter: S g beta / 2 (else unused)
    const double *murL;    // left-end Mur coefficient per rest cell
    const double *murR;    // right-end Mur coefficient per rest cell
    const double *src;     // source samples, step n at [n-1]
    const int64_t *probes; // probe cells
    double *trace;         // nprobe * steps, probe q at row q
    // finite-duration modulation: the profile exists for t_on <= t < t_off
    double t_on, t_off;
    double cEb, cHb;       // background coefficients S/eps_bg, S/mu_bg
    double murB;           // background Mur coefficient (both ends)
};

struct TileRef {
    int32_t run;           // index into the RunDesc array of the launch
    int32_t tile;          // tile index within that run
    int32_t probe_waves;   // bit w: wave w of the tile owns a probe
    int32_t reserved;
};

// Per-run arguments of the set-up kernels.
struct PrepDesc {
    int64_t nz;
    int64_t nsrc;
    double S, beta;
    double amp, omega, t0, tau, phase;
    int32_t kind;
    int32_t precision;
    int32_t abc;
    int32_t pad0;
    const double *eps;     // rest profile (device copy)
    const double *mu;
    void *cE;
    void *cH;
    void *gB;
    double *murL;
    double *murR;
    double *src;
    void *fields[4];       // D0, D1, B0, B1 (offset by kPad)
    int64_t field_cells;   // nz + 2 kPad
    const double *init_d;  // initial D^{1/2} (device copy, nz) or null
    const double *init_b;  // initial B^0 (device copy, nz) or null
};

struct DftDesc {
    int64_t steps;
    double S;
    int32_t nprobe;
    int32_t nfreq;
    const double *trace;
    const double *omegas;
    double *out;           // nprobe * nfreq * 2 (re, im)
};

// Launchers (kernels.hip).  Each returns hipSuccess or the launch error.
hipError_t launch_prep(const PrepDesc *dev_descs, int count, int max_cells,
                       hipStream_t stream);
hipError_t launch_zero(const PrepDesc *dev_descs, int count,
                       int64_t max_field_cells, int precision,
                       hipStream_t stream);
hipError_t launch_init(const PrepDesc *dev_descs, int count, int64_t max_nz,
                       int precision, hipStream_t stream);
// Steps the first ntiles tiles by one block.  win selects the kernel for
// runs with a finite-duration modulation; each kernel skips the other's
// runs, so a group holding both is stepped by two launches.  G = waves per
// tile (1..kMaxTileWaves); every run of the launch is tiled with that G.
hipError_t launch_tiles(int precision, int kind, bool ring, bool win, int C, int G,
                        const RunDesc *runs, const TileRef *tiles, int64_t block,
                        int T, int ntiles, hipStream_t stream);

// Runs are stepped in groups that share one kernel instantiation: by
// precision, kind and ring (periodic ends) or not.
constexpr int kGroups = 8;
inline int group_of(int precision, int kind, int abc)
{
    return precision * 4 + kind * 2 + (abc == GFDTD_ABC_PERIODIC ? 1 : 0);
}
inline int group_precision(int g) { return g >> 2; }
inline int group_kind(int g) { return (g >> 1) & 1; }
inline bool group_ring(int g) { return (g & 1) != 0; }
hipError_t launch_dft(const DftDesc *dev_descs, int count, int max_pf,
                      hipStream_t stream);

}  // namespace gfdtd
