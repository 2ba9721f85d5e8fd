// Device-side descriptors and launchers of the 2D path (not part of the
// C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gfdtd2d.h"

namespace gfdtd {

// One 2D run as the kernels see it (lives in the workspace).
struct Run2D {
    int64_t nx, nz;
    int64_t ld;                 // column stride of the field arrays (elements)
    int64_t nh;                 // H-lattice nodes: nz - 1, nz on a z-ring
    int64_t nc;                 // C-field nodes: TE nz, TM nh
    int64_t src_row, nsrc, steps;
    double S, beta;
    double amp, omega, t0, tau, phase;   // source pulse (App. B.1)
    int32_t pol, abc, nprobe, precision;
    const double *eps, *mu;     // rest profile, nz each
    const double *prof;         // source profile, nx
    double *src;                // source samples g(n S), n = 1..nsrc
    const int64_t *px, *pz;     // probes
    double *trace;              // nprobe * steps
    void *f[6];                 // D0, D1, B0, B1, C0, C1: nx * ld each
    const double *init[3];      // initial D, B, C (nx * nz, FP64) or null
};

// Launch geometry of the stepping kernel: a wave holds 64 * C rows of a
// z-strip (halo rows on each side are recomputed, not stored) and advances
// `xch` consecutive columns by T steps (T in {1, 2, 4}).
struct Launch2D {
    int C = 4;
    int xch = 16;
    int T = 1;
    int64_t nstrips = 0, nchunks = 0, waves = 0, blocks = 0;
};

int64_t strip_rows(int C, int T);
Launch2D plan_launch2d(int64_t nx, int64_t nz, int precision, int C, int xch, int T);

hipError_t launch_prep2d(const Run2D *dev, const Run2D &host, hipStream_t s);
// One stepping launch; the descriptor travels by value as a kernel argument.
hipError_t launch_step2d(const Run2D &host, const Launch2D &L, int64_t n, int par,
                         hipStream_t s);

}  // namespace gfdtd
