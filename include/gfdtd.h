/*
 * gfdtd.h -- C-ABI of the MI355X generalized-FDTD library.
 *
 * The library time-steps the generalized FDTD scheme of Deck-Leger,
 * Bahrami, Li and Caloz (arXiv 2304.06586) for electromagnetic scattering
 * in 1D moving structures: the extended Yee cell of Section 3 (Fig. 2),
 * whose tangential unknowns are the auxiliary fields
 *     E* = E + v x B,   H* = H - v x D          (eq. (2)),
 * updated by the leapfrog equations (10a)-(10d) with the dynamic
 * (velocity) terms of Table 1.  Every step re-samples the moving material
 * profile eps(z - v t), mu(z - v t) (eq. (5)), so the moving-boundary
 * conditions (1a)-(1d) hold implicitly at every cell the moving structure
 * crosses.  Each step also injects a source, absorbs at the grid ends and
 * records probes.  All of that runs in HIP kernels on the GPU.
 *
 * Units: c = eps0 = mu0 = 1, cell size dz = 1, time step S = dt/dz
 * (Courant number, below eq. (10)), beta = v/c.
 *
 * Grid: nz E nodes k = 0..nz-1 (D_x, E*_x at times n+1/2) and nz-1 H nodes
 * j = 0..nz-2 at positions j+1/2 (B_y, H*_y at integer times n).  With
 * periodic ends (a ring) there are nz H nodes and node nz-1 neighbours
 * node 0.
 *
 * Conventions
 *  - Every function returns a gfdtd_status; nothing throws across the ABI.
 *    gfdtd_last_error() returns a message for the calling thread's last
 *    failure.
 *  - Host inputs are caller-owned and only read during the call.
 *  - Device memory is caller-owned: the caller allocates a workspace of
 *    at least the size the *_bytes queries report and passes its device
 *    pointer and size.  The library carves it and never calls hipMalloc.
 *    The workspace must stay allocated while a batch or server that uses
 *    it exists.
 *  - Streams are passed as void* (a hipStream_t); work is ordered on that
 *    stream.
 *  - Structs start with struct_size = sizeof(struct) for ABI evolution.
 *  - Different batches/servers are independent; one batch or server must
 *    not be used from two threads at once.
 */
#ifndef GFDTD_H
#define GFDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef enum gfdtd_status {
    GFDTD_OK = 0,
    GFDTD_E_INVALID = 1,     /* bad argument or problem description        */
    GFDTD_E_UNSTABLE = 2,    /* pre-flight: amplification factor above 1   */
    GFDTD_E_NOMEM = 3,       /* workspace / server pool too small          */
    GFDTD_E_DEVICE = 4,      /* a HIP call failed                          */
    GFDTD_E_NOT_READY = 5,   /* server: request still queued or running    */
    GFDTD_E_BLOWUP = 6,      /* a probe recorded NaN or Inf                */
    GFDTD_E_UNSUPPORTED = 7  /* option not implemented                     */
} gfdtd_status;

/* Message naming a status; static storage. */
const char *gfdtd_status_str(gfdtd_status s);
/* Message describing the calling thread's last failure ("" if none). */
const char *gfdtd_last_error(void);

/* ----------------------------------------------------------- the problem */
#define GFDTD_MODULATION 0   /* moving perturbation: eps(z-vt), mu(z-vt)
                                stay isotropic (Section 2)                  */
#define GFDTD_MATTER 1       /* moving matter: bianisotropic in the lab
                                frame (footnote to eq. (5)), here in the
                                solved form E* = g (mu' D - beta Bbar),
                                H* = g (eps' B - beta Dbar),
                                g = (1-beta^2)/(eps' mu' - beta^2)          */

#define GFDTD_F32 0          /* FP32 fields and stencil arithmetic; moving-
                                boundary shifts, coefficients before
                                rounding, source samples, probes and DFT in
                                FP64                                        */
#define GFDTD_F64 1          /* everything in FP64                          */

#define GFDTD_ABC_MUR1 0     /* first-order Mur on D at both end nodes      */
#define GFDTD_ABC_PEC 1      /* D = 0 at both end nodes                     */
#define GFDTD_ABC_PERIODIC 2 /* a ring: nz E and nz H nodes, node nz-1 next
                                to node 0; every index (fields, rest cells,
                                moving-profile samples) wraps modulo nz.
                                The uniform-medium case is the plane-wave
                                setting of the stability analysis (Section
                                5, App. A, Fig. 4)                         */

#define GFDTD_FLAG_RECORD_TRACE 1u   /* copy probe time traces on collect  */
#define GFDTD_FLAG_ALLOW_UNSTABLE 2u /* skip the pre-flight rejection      */
#define GFDTD_FLAG_KEEP_FIELDS 4u    /* server: keep the final fields until
                                        the request is polled              */
#define GFDTD_FLAG_TIME_WINDOW 8u    /* finite-duration modulation: see
                                        t_on, t_off, eps_bg, mu_bg         */

#define GFDTD_MAX_PROBES 64

/*
 * One scattering solve.
 *  eps_rest[i]  rest permittivity eps' of the cell centred on E node i
 *               (covering z in [i-1/2, i+1/2) at t = 0), i = 0..nz-1;
 *  mu_rest[i]   rest permeability mu' of the cell centred on H node i
 *               (covering [i, i+1)); entry nz-1 is read only by the
 *               moving-matter end treatment and by rings, and may
 *               otherwise be any positive value.
 *  The profile moves rigidly at beta (eq. (5): eps(z - v t)), in whole
 *  cells: at time tau*S it has moved by m = rint(beta*S*tau) cells and a
 *  node at lattice index x reads rest cell clamp(x - m) (on a ring
 *  (x - m) mod nz).  E nodes read at tau = n+1/2, H nodes at tau = n.
 *  For moving matter both eps' and mu' are read at the node's own
 *  lattice index.
 *  Initial state: all fields zero, or D^{1/2} = init_d and B^0 = init_b
 *  when given (E*^{1/2} then follows from them by (10c)).
 *  Finite-duration modulation (GFDTD_FLAG_TIME_WINDOW, moving modulation
 *  only): the moving profile exists only at node times t with
 *  t_on <= t < t_off (E nodes at t = (n+1/2) S, H nodes at t = n S); at
 *  other times every node sees the uniform background eps_bg, mu_bg.  D
 *  and B carry over across the switches (temporal interfaces), which with
 *  the moving boundaries form the corners of a space-time slab (the case
 *  the footnote to the transfer-matrix method of App. B.3 sets apart).
 *  Source: soft source added to D at src_cell after (10b) of step n,
 *    src_amp * sin(src_omega (t - src_t0) + src_phase)
 *            * exp(-((t - src_t0)/src_tau)^2),  t = n S,
 *  for t <= src_t_off (the modulated Gaussian of App. B.1).
 *  Probes: physical E = E* + beta Bbar (inverse of eq. (2), Bbar the
 *  Table 1 average of (10c)) at probe_cells, at t = (n+1/2) S, n = 1..steps;
 *  DFT X(w) = sum_n E_n S exp(+i w t_n) at the nfreq angular frequencies.
 *  Values off the grid are the edge values.
 */
typedef struct gfdtd_problem {
    uint32_t struct_size;
    int32_t kind;                /* GFDTD_MODULATION / GFDTD_MATTER        */
    int32_t precision;           /* GFDTD_F32 / GFDTD_F64                  */
    int32_t abc;                 /* GFDTD_ABC_*                            */
    uint32_t flags;              /* GFDTD_FLAG_*                           */
    int32_t nprobe;              /* 0..GFDTD_MAX_PROBES                    */
    int32_t nfreq;               /* >= 0                                   */
    int32_t reserved0;
    int64_t nz;                  /* E nodes, 8 <= nz < 2^31 - 2^20         */
    double courant;              /* S = dt/dz, > 0                         */
    double beta;                 /* v/c, |beta| < 1 and |beta| S <= 0.9    */
    const double *eps_rest;      /* host, nz, > 0 and finite               */
    const double *mu_rest;       /* host, nz, > 0 and finite               */
    int64_t src_cell;            /* 1..nz-2 (ring: 0..nz-1)                */
    double src_amp, src_omega, src_t0, src_tau, src_phase, src_t_off;
    const int64_t *probe_cells;  /* host, nprobe, each in 0..nz-1          */
    const double *omegas;        /* host, nfreq                            */
    const double *init_d;        /* host, nz finite values, or NULL        */
    const double *init_b;        /* host, nz finite values (entry nz-1 is
                                    read on a ring only), or NULL          */
    double t_on, t_off;          /* GFDTD_FLAG_TIME_WINDOW: not NaN (may be
                                    infinite), else ignored                */
    double eps_bg, mu_bg;        /* GFDTD_FLAG_TIME_WINDOW: > 0, finite    */
} gfdtd_problem;

/*
 * Results of one solve, in caller-allocated host buffers (any pointer may
 * be NULL to skip that output).  Sizes from gfdtd_result_sizes().
 *  trace    nprobe*steps doubles, probe q at row q (needs
 *           GFDTD_FLAG_RECORD_TRACE);
 *  dft_re/im nprobe*nfreq doubles, probe q at row q;
 *  final_d  nz doubles: D^{steps+1/2} (converted from the run precision);
 *  final_b  nz doubles: B^{steps} at H nodes 0..nz-2, last entry 0
 *           (on a ring all nz H nodes).
 */
typedef struct gfdtd_result {
    uint32_t struct_size;
    int32_t run_status;          /* GFDTD_OK or GFDTD_E_BLOWUP             */
    int64_t steps_done;
    double *trace;
    double *dft_re;
    double *dft_im;
    double *final_d;
    double *final_b;
} gfdtd_result;

/*
 * Validate a problem and run the stability pre-flight: the von Neumann
 * amplification matrix of one step (Section 5, App. A) is evaluated for
 * every distinct medium of the rest profile, theta in (0, pi]; the larger
 * of the two roots (co- and contra-moving, Section 5) must not exceed 1.
 * Writes the largest modulus to *max_growth (may be NULL).
 * Returns GFDTD_E_INVALID for a malformed problem, GFDTD_E_UNSTABLE when
 * the growth exceeds 1 + 1e-9 and GFDTD_FLAG_ALLOW_UNSTABLE is not set.
 * Host only; does not touch the GPU.
 */
gfdtd_status gfdtd_check(const gfdtd_problem *p, double *max_growth);

/* Lengths (in doubles) of the trace and DFT outputs of one solve. */
gfdtd_status gfdtd_result_sizes(const gfdtd_problem *p, int64_t steps,
                                size_t *trace_len, size_t *dft_len);

/* Device workspace needed by gfdtd_solve (one problem) and by a batch. */
gfdtd_status gfdtd_workspace_bytes(const gfdtd_problem *p, int64_t steps,
                                   size_t *bytes);
gfdtd_status gfdtd_batch_workspace_bytes(const gfdtd_problem *probs,
                                         const int64_t *steps, int32_t count,
                                         size_t *bytes);

/* ------------------------------------------------------------- execution */
#define GFDTD_VARIANT_AUTO 0
#define GFDTD_VARIANT_STEP 1     /* one launch per time step               */
#define GFDTD_VARIANT_TILED 2    /* register tiles, several steps a launch */

/*
 * Execution options (NULL = automatic).  cells_per_lane in {4, 8, 12, 16}
 * (0 = auto), block_steps = temporal block depth, steps per launch
 * (0 = auto; 1 for GFDTD_VARIANT_STEP), use_graph: -1 auto, 0 plain
 * launches, 1 capture the launch sequence in a hipGraph (a captured pass
 * runs every launch on one stream, so use_graph = 1 also keeps groups
 * whole; automatic never captures a group split over two streams).
 * tile_waves in 0..4 (0 = auto): waves that step one tile side by side,
 * sharing overlap cells through LDS (rings always use 1);
 * exchange_steps in 0..16 (0 = auto, 8): steps between the overlap
 * refreshes of multi-wave tiles.
 * The result does not depend on these options (bit for bit).
 */
typedef struct gfdtd_exec {
    uint32_t struct_size;
    int32_t variant;
    int32_t cells_per_lane;
    int32_t block_steps;
    int32_t use_graph;
    int32_t tile_waves;
    int32_t exchange_steps;
    int32_t reserved0;
} gfdtd_exec;

/*
 * Plain single solve: validate, pre-flight, upload, step, collect.
 * Synchronous: on return the results are in *out.  ws/ws_bytes is device
 * memory of at least gfdtd_workspace_bytes().
 */
gfdtd_status gfdtd_solve(const gfdtd_problem *p, int64_t steps, void *ws,
                         size_t ws_bytes, void *stream, gfdtd_result *out);

/*
 * Allocation-free single solve, for callers that cannot allocate device
 * memory (serving loops and harnesses that forbid allocation): the same
 * validation, pre-flight, kernels and results as gfdtd_solve (bit for bit),
 * with the workspace taken from a fixed device array of
 * GFDTD_STATIC_WORKSPACE_BYTES that the library holds on every GPU it runs
 * on until the process ends.  The call makes no device allocation and
 * creates no events, streams or graphs; it is synchronous on `stream`
 * (so it cannot be captured into a graph).
 * Returns GFDTD_E_NOMEM, before any device call, when the problem's
 * workspace (gfdtd_workspace_bytes) exceeds the array.  All calls on one
 * GPU share its array: calls from one process are serialised per device;
 * concurrent use of the array from outside this entry point would race.
 * Each call rewrites every part of the array it reads, so nothing carries
 * over from the previous call.
 */
#define GFDTD_STATIC_WORKSPACE_BYTES ((size_t)32 << 20)
gfdtd_status gfdtd_solve_static(const gfdtd_problem *p, int64_t steps,
                                void *stream, gfdtd_result *out);

/*
 * Many independent solves in one pass: the runs are packed into one run
 * table and every launch advances all live runs by one temporal block.
 * outs[i] receives run i's results; its run_status reports a blow-up of
 * that run alone.  Synchronous.
 */
gfdtd_status gfdtd_solve_batch(const gfdtd_problem *probs, const int64_t *steps,
                               int32_t count, void *ws, size_t ws_bytes,
                               void *stream, gfdtd_result *outs);

/* Split form of a batch: prepare once, run (possibly many times), collect. */
typedef struct gfdtd_batch gfdtd_batch;

/*
 * Validate and pre-flight every problem, carve the workspace, upload rest
 * profiles, probes and frequencies, and build the launch plan (and the
 * hipGraph if requested).  Enqueues uploads on `stream`.  A group of two or
 * more runs and at least 2^18 cells (not with use_graph = 1) is split into
 * two halves; the batch then creates a second, non-blocking stream of
 * default priority, owned by it and destroyed with it.
 */
gfdtd_status gfdtd_batch_prepare(const gfdtd_problem *probs,
                                 const int64_t *steps, int32_t count,
                                 const gfdtd_exec *exec, void *ws,
                                 size_t ws_bytes, void *stream,
                                 gfdtd_batch **out);
/*
 * Enqueue one complete pass on the stream: zero the fields, time-step
 * every run to its step count, then form the probe DFTs.  Device work
 * only; returns without waiting.  Each pass recomputes from zero fields.
 * With a split group, the second half's stepping launches run on the
 * batch's second stream, which waits (by an event) for the work already
 * enqueued on `stream` and which `stream` waits for before the DFTs: work
 * the caller enqueues on `stream` afterwards is ordered after the whole
 * pass, as without the split.
 */
gfdtd_status gfdtd_batch_run(gfdtd_batch *b);
/* Wait for the stream, then copy run i's results to outs[i]. */
gfdtd_status gfdtd_batch_collect(gfdtd_batch *b, gfdtd_result *outs);

typedef struct gfdtd_stats {
    uint32_t struct_size;
    int32_t cells_per_lane;      /* chosen tiling                          */
    int32_t block_steps;         /* temporal block depth                   */
    int32_t graph;               /* 1 if passes replay a hipGraph          */
    int64_t launches;            /* stepping launches per pass             */
    int64_t tiles;               /* wave tiles summed over launches        */
    double cell_updates;         /* sum over runs of nz * steps            */
    double step_ms;              /* device time of the last pass's stepping
                                    launches (HIP events on the stream)    */
    double pass_ms;              /* device time of the whole last pass     */
    int32_t tile_waves;          /* waves per tile                         */
    int32_t exchange_steps;      /* steps between overlap refreshes        */
    int32_t streams;             /* streams the stepping launches use: 2
                                    when a group of two or more runs and
                                    at least 2^18 cells is split into two
                                    halves whose launches overlap
                                    (launches and tiles count both; not
                                    with use_graph = 1), else 1            */
    int32_t reserved;
} gfdtd_stats;

gfdtd_status gfdtd_batch_stats(const gfdtd_batch *b, gfdtd_stats *s);

/*
 * Autotuner: for each (precision, kind) group of the batch, time every
 * valid (cells per lane in {4, 8, 12, 16}, steps per launch in {8, 16, 24,
 * 32, 48, 64}, 1 or 4 waves per tile off rings) on the prepared runs over
 * about trial_blocks * 48 steps (trial_blocks 0 = 4; eight times that for a
 * group under 4M cells, whose launches are short; from the middle of the
 * run for a group of one run, from the start otherwise), and keep the
 * fastest per cell-update.  A group split over two streams (see streams in
 * gfdtd_stats) is timed with both halves' launches on their streams, as a
 * pass issues them, and both take the same choice.  Results of a pass do
 * not depend on the choice.  Choices are cached in the process by precision, kind, sign
 * mix and the size scales of the group.  Writes the first group's choice to
 * *chosen (may be NULL).  Synchronous; leaves the fields to be re-zeroed by
 * the next gfdtd_batch_run.
 */
gfdtd_status gfdtd_batch_autotune(gfdtd_batch *b, int32_t trial_blocks,
                                  gfdtd_exec *chosen);
void gfdtd_batch_destroy(gfdtd_batch *b);

/* --------------------------------------------------------------- serving */
/*
 * Continuous-batching server.  Requests are admitted while their device
 * state fits in the pool (the HBM budget) and a slot is free; every
 * progress block advances all admitted runs by block_steps steps in one
 * launch per precision and kind; finished runs are retired (DFT, copy-out)
 * between blocks and queued requests admitted in their place.  A result
 * does not depend on which other requests shared its blocks.
 */
typedef struct gfdtd_server_config {
    uint32_t struct_size;
    int32_t max_slots;           /* admitted runs at once, >= 1            */
    int32_t block_steps;         /* steps per progress block (0 = auto)    */
    int32_t max_ahead;           /* blocks enqueued beyond the last block
                                    the GPU has finished, at most (0 = 8):
                                    bounds how long a new request waits
                                    behind work already enqueued           */
    void *pool;                  /* device memory for run state            */
    size_t pool_bytes;           /* the HBM budget                         */
    void *stream;
} gfdtd_server_config;

typedef struct gfdtd_server gfdtd_server;

gfdtd_status gfdtd_server_create(const gfdtd_server_config *cfg,
                                 gfdtd_server **out);
/* Queue a request.  GFDTD_E_NOMEM only if the request alone can never fit
 * the pool; GFDTD_E_INVALID / GFDTD_E_UNSTABLE as gfdtd_check. */
gfdtd_status gfdtd_server_submit(gfdtd_server *s, const gfdtd_problem *p,
                                 int64_t steps, uint64_t *id);
/* Admit what fits, enqueue up to max_blocks progress blocks on the stream
 * and retire the runs whose last block is enqueued (their DFT and result
 * copies are enqueued too).  Returns without waiting for the GPU; enqueues
 * fewer blocks (possibly none) once max_ahead blocks are outstanding, so a
 * serving loop calls it repeatedly.  *live gets the number of admitted runs
 * afterwards, *queued the waiting ones (either may be NULL). */
gfdtd_status gfdtd_server_progress(gfdtd_server *s, int32_t max_blocks,
                                   int32_t *live, int32_t *queued);
/* GFDTD_E_NOT_READY until the request has finished.  With out == NULL,
 * only reports readiness (GFDTD_OK once finished) and keeps the results;
 * with a result struct, copies them and releases the request's record
 * (results can be collected once). */
gfdtd_status gfdtd_server_poll(gfdtd_server *s, uint64_t id, gfdtd_result *out);
void gfdtd_server_destroy(gfdtd_server *s);

/* ------------------------------------------------ transfer-matrix sweeps */
/*
 * Frequency-domain scattering of moving multilayers by the transfer-matrix
 * method of App. B.3, batched over stacks and frequencies: the closed-form
 * companion of the time-domain solver for parameter sweeps (uniform
 * space-time slabs only).  Layers 0..N-1 all move at beta; layers 0 and N-1
 * are semi-infinite and the wave is incident from layer 0 at lab angular
 * frequency omega.  Within layer m (index n_m = sqrt(eps mu), impedance
 * eta_m = sqrt(mu/eps)) the forward and backward waves have the Doppler
 * frequencies omega (1 - n_0 beta)/(1 -/+ n_m beta) (the phase invariant
 * of a moving boundary); interfaces match E* and H* (the star amplitudes).
 * For each (stack, omega) the lab-frame E-field transmission T (layer N-1)
 * and reflection Gamma (layer 0) are returned.  All in FP64.
 */
typedef struct gfdtd_tmm_stack {
    uint32_t struct_size;
    int32_t nlayers;             /* N >= 2                                 */
    double beta;                 /* |beta| n_m < 1 in every layer          */
    const double *eps;           /* host, N values > 0                     */
    const double *mu;            /* host, N values > 0, or NULL for all 1  */
    const double *widths;        /* host, N-2 lab-frame widths >= 0 of the
                                    inner layers (NULL if N == 2)          */
} gfdtd_tmm_stack;

/* Device workspace for gfdtd_tmm. */
gfdtd_status gfdtd_tmm_workspace_bytes(const gfdtd_tmm_stack *stacks,
                                       int32_t nstacks, int32_t nomega,
                                       size_t *bytes);
/* Evaluate every stack at every omega (host array, nomega finite values).
 * t and gamma are caller-allocated host arrays of 2 * nstacks * nomega
 * doubles, (re, im) pairs, stack-major: entry [s][f].  Synchronous.
 * GFDTD_E_INVALID for a malformed stack (it names the stack). */
gfdtd_status gfdtd_tmm(const gfdtd_tmm_stack *stacks, int32_t nstacks,
                       const double *omegas, int32_t nomega, void *ws,
                       size_t ws_bytes, void *stream, double *t, double *gamma);
/* Device time in ms of the transfer-matrix kernel alone in the calling
 * thread's last successful gfdtd_tmm (HIP events around the launch, on its
 * stream; the call itself also packs the stacks on the host and copies them
 * and the results).  GFDTD_E_INVALID if there is none. */
gfdtd_status gfdtd_tmm_kernel_ms(double *ms);

#ifdef __cplusplus
}
#endif

#endif /* GFDTD_H */
