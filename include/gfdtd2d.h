/*
 * gfdtd2d.h -- C-ABI of the 2D (TE / TM) generalized-FDTD path.
 *
 * The paper discretizes the 1D problem (Section 4, eq. (10a)-(10d) with the
 * dynamic terms of Table 1).  This path applies the same scheme in the
 * (x, z) plane for fields independent of y, motion v = beta z^ and a
 * moving modulation eps(z - vt), mu(z - vt) whose interfaces are normal to
 * v (the case of Section 3, eq. (3)).  It reads the mixed-field equations
 * (6) with the star fields of eq. (2), using div B = 0 and, away from the
 * source, div D = 0, as
 *   dB/dt = -curl E* - v dB/dz,   dD/dt = curl H* - v dD/dz,
 * component by component:
 *   TE (E_y, H_x, H_z):  E*_y = E_y + beta B_x,  H*_x = H_x + beta D_y,
 *                        H*_z = H_z;
 *   TM (H_y, E_x, E_z):  E*_x = E_x - beta B_y,  H*_y = H_y - beta D_x,
 *                        E*_z = E_z.
 * Every z-difference of a velocity term and every velocity average takes
 * the Table 1 stencil and time level of the 1D scheme (column a for
 * v >= 0, column b for v < 0) on that field's own lattice; the curls are
 * the Yee differences.  For x-uniform fields each column is exactly the 1D
 * scheme, TE as the pair (D_y, -B_x) and TM as (D_x, B_y).
 *
 * Units, status codes, workspace and stream conventions are those of
 * gfdtd.h: c = eps0 = mu0 = 1, square cells dx = dz = 1, time step
 * S = dt/dz; host inputs are only read during a call; the caller provides
 * a device workspace of at least the reported size and the library never
 * allocates device memory; work is ordered on the caller's stream.
 *
 * Grid: nx columns i = 0..nx-1, periodic in x.  Along z, E-lattice nodes
 * k = 0..nz-1 and H-lattice nodes j = 0..nz-2 at j + 1/2 (both ends are
 * E-lattice nodes); with periodic z ends, nz of each.  The three unknowns
 * of a polarization, named as the 1D pair (D, B) plus the cross field C:
 *   TE  D = D_y at (i, k)       B = B_x at (i, j+1/2)     C = B_z at (i+1/2, k)
 *   TM  D = D_x at (i+1/2, k)   B = B_y at (i+1/2, j+1/2)  C = D_z at (i, j+1/2)
 * Host field arrays are row-major (nx, nz): element [i * nz + k].
 */
#ifndef GFDTD2D_H
#define GFDTD2D_H

#include <stddef.h>
#include <stdint.h>

#include "gfdtd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GFDTD2D_TE 0
#define GFDTD2D_TM 1

/*
 * One 2D solve of a moving modulation.
 *  eps_rest, mu_rest  the stratified rest profile, one value per rest cell
 *    along z exactly as in gfdtd_problem (eps cell i covers [i-1/2, i+1/2),
 *    mu cell i covers [i, i+1)).  The profile moves rigidly by
 *    m = rint(beta S tau) whole cells at time tau S; a node at position z
 *    reads the rest cell that contains z - m (clamped to the grid, wrapped
 *    on a z-ring), at its own time: E-lattice fields at tau = n + 1/2,
 *    H-lattice fields at tau = n.  So TE's B_z at (i+1/2, k) reads mu cell
 *    k - m and TM's D_z at (i, j+1/2) reads eps cell j + 1 - m.
 *  Source: soft source on D (D_y for TE, D_x for TM) along the row
 *    src_row after the D update of step n: src_profile[i] * g(n S), g the
 *    modulated Gaussian of App. B.1 (as gfdtd_problem), for n S <= t_off.
 *    For TM a profile that varies along x also deposits charge (the
 *    source current is not divergence-free); the update keeps the
 *    advective form regardless.
 *  Ends along z: first-order Mur on D at k = 0 and k = nz-1 of every
 *    column with the normal-incidence coefficient of the 1D scheme for the
 *    medium under the end node, PEC (D = 0 there) or periodic.
 *  Probes: physical E of the sourced component (E_y for TE, E_x for TM)
 *    at (probe_x[q], probe_z[q]) at t = (n + 1/2) S, with the DFT of
 *    gfdtd_problem.
 *  Initial state: zero, or D^{1/2}, B^0 and C (TE: B_z^0, TM: D_z^{1/2})
 *    from init_d / init_b / init_c (nx * nz values each; on a grid with
 *    ends the last entry of every row of B, and of C for TM, is ignored).
 */
typedef struct gfdtd2d_problem {
    uint32_t struct_size;
    int32_t pol;                 /* GFDTD2D_TE / GFDTD2D_TM                */
    int32_t precision;           /* GFDTD_F32 / GFDTD_F64                  */
    int32_t abc;                 /* z ends: GFDTD_ABC_*                    */
    uint32_t flags;              /* GFDTD_FLAG_RECORD_TRACE,
                                    GFDTD_FLAG_ALLOW_UNSTABLE              */
    int32_t nprobe;              /* 0..GFDTD_MAX_PROBES                    */
    int32_t nfreq;               /* >= 0                                   */
    int32_t reserved0;
    int64_t nx;                  /* 1 <= nx <= 2^20                        */
    int64_t nz;                  /* 8 <= nz <= 2^24, nx * nz <= 2^31       */
    double courant;              /* S > 0                                  */
    double beta;                 /* |beta| < 1, |beta| S <= 0.9            */
    const double *eps_rest;      /* host, nz values > 0, finite            */
    const double *mu_rest;       /* host, nz values > 0, finite            */
    int64_t src_row;             /* 1..nz-2 (ring: 0..nz-1)                */
    const double *src_profile;   /* host, nx finite values, or NULL = 1    */
    double src_amp, src_omega, src_t0, src_tau, src_phase, src_t_off;
    const int64_t *probe_x;      /* host, nprobe values in 0..nx-1         */
    const int64_t *probe_z;      /* host, nprobe values in 0..nz-1         */
    const double *omegas;        /* host, nfreq finite values              */
    const double *init_d;        /* host, nx * nz finite values, or NULL   */
    const double *init_b;
    const double *init_c;
} gfdtd2d_problem;

/*
 * Results in caller-allocated host buffers (any pointer may be NULL):
 *  trace    nprobe * steps doubles (needs GFDTD_FLAG_RECORD_TRACE);
 *  dft_re/im nprobe * nfreq doubles;
 *  final_d, final_b, final_c  nx * nz doubles each, converted from the run
 *           precision; unused lattice slots are 0.
 */
typedef struct gfdtd2d_result {
    uint32_t struct_size;
    int32_t run_status;          /* GFDTD_OK or GFDTD_E_BLOWUP             */
    int64_t steps_done;
    double *trace;
    double *dft_re;
    double *dft_im;
    double *final_d;
    double *final_b;
    double *final_c;
} gfdtd2d_result;

/*
 * Validate and run the stability pre-flight.  For every distinct medium of
 * the rest profile (up to 32 of them, spread over the sorted eps' mu') the
 * one-step amplification matrix of a plane wave exp(i (kx x + kz z)) in
 * that uniform medium is evaluated on a 64 x 128 grid of kx in [0, pi],
 * kz in (-pi, pi]; *max_growth (may be NULL) receives its largest
 * eigenvalue modulus g.
 * The 2D reading is not strictly stable for a moving modulation: oblique
 * grid-scale modes (kx near pi) grow by g = 1 + O(|beta| S^4) per step
 * (e.g. 1.1e-4 at S = 0.25, |beta| = 0.5, vacuum), while the 1D scheme
 * (kx = 0) is.  A run of `steps` steps is therefore accepted when that
 * worst mode grows by at most GFDTD2D_MAX_RUN_GROWTH over the whole run,
 * g^steps <= 10 (rounding seeds it at the precision's unit roundoff).
 * GFDTD_E_INVALID for a malformed problem; GFDTD_E_UNSTABLE when g^steps
 * exceeds the bound and GFDTD_FLAG_ALLOW_UNSTABLE is not set.  Host only.
 */
#define GFDTD2D_MAX_RUN_GROWTH 10.0
gfdtd_status gfdtd2d_check(const gfdtd2d_problem *p, int64_t steps, double *max_growth);

/* Device workspace needed by one 2D solve of `steps` steps. */
gfdtd_status gfdtd2d_workspace_bytes(const gfdtd2d_problem *p, int64_t steps,
                                     size_t *bytes);

/*
 * Execution options (NULL = automatic).  cells_per_lane: z cells a lane
 * holds (FP32: 2, 4 or 8, FP64: 2 or 4; 0 = auto); columns_per_wave:
 * columns a wave steps in one launch (0 = auto); block_steps: steps a
 * launch advances the grid, 1 to 4 (0 = auto); more than 1 needs the
 * narrow lanes (FP32 at most 4 cells, FP64 2) and ends other than
 * periodic.  A run whose
 * step count is not a multiple finishes with one-step launches.  Results
 * do not depend on these options (bit for bit).
 */
typedef struct gfdtd2d_exec {
    uint32_t struct_size;
    int32_t cells_per_lane;
    int32_t columns_per_wave;
    int32_t block_steps;
} gfdtd2d_exec;

typedef struct gfdtd2d_run gfdtd2d_run;

/*
 * Validate, pre-flight (as gfdtd2d_check for `steps`), carve the workspace
 * and upload the problem's inputs on `stream` (waits for the uploads).
 */
gfdtd_status gfdtd2d_prepare(const gfdtd2d_problem *p, int64_t steps,
                             const gfdtd2d_exec *exec, void *ws,
                             size_t ws_bytes, void *stream, gfdtd2d_run **out);
/*
 * Enqueue one complete pass: set the initial fields, one stepping launch
 * per time step, then the probe DFT.  Returns without waiting.  Each pass
 * starts again from the initial state.
 */
gfdtd_status gfdtd2d_run_pass(gfdtd2d_run *r);
/* Wait for the stream and copy the results of the last pass. */
gfdtd_status gfdtd2d_collect(gfdtd2d_run *r, gfdtd2d_result *out);

typedef struct gfdtd2d_stats {
    uint32_t struct_size;
    int32_t cells_per_lane;
    int32_t columns_per_wave;
    int32_t waves;               /* waves per stepping launch              */
    int64_t launches;            /* stepping launches per pass             */
    double cell_updates;         /* nx * nz * steps                        */
    double step_ms;              /* device time of the last pass's stepping
                                    launches (HIP events on the stream)    */
    double pass_ms;              /* device time of the whole last pass     */
    int32_t block_steps;         /* steps per launch (the last launches of
                                    a pass may take one)                   */
    int32_t reserved0;
} gfdtd2d_stats;

gfdtd_status gfdtd2d_get_stats(const gfdtd2d_run *r, gfdtd2d_stats *s);
void gfdtd2d_destroy(gfdtd2d_run *r);

/* prepare + run_pass + collect + destroy; synchronous. */
gfdtd_status gfdtd2d_solve(const gfdtd2d_problem *p, int64_t steps, void *ws,
                           size_t ws_bytes, void *stream, gfdtd2d_result *out);

#ifdef __cplusplus
}
#endif

#endif /* GFDTD2D_H */
