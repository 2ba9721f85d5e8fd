// Host-side structures of the generalized-FDTD runtime (not part of the
// C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "gfdtd.h"
#include "gfdtd_internal.h"

namespace gfdtd {

gfdtd_status fail(gfdtd_status s, const char *fmt, ...);
gfdtd_status hip_fail(hipError_t e, const char *what);
void clear_error();
const char *last_error();

gfdtd_status validate(const gfdtd_problem *p, int64_t steps);
gfdtd_status preflight(const gfdtd_problem *p, double *growth);

// Bump allocator over a workspace, 256-byte aligned.
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes);
};

// Byte offsets of one run's device arrays inside a workspace.
struct RunLayout {
    size_t eps = 0, mu = 0, cE = 0, cH = 0, gB = 0, murL = 0, murR = 0;
    size_t src = 0, probes = 0, omegas = 0, trace = 0, dft = 0;
    size_t field[4] = {0, 0, 0, 0};   // D0, D1, B0, B1 (padded)
    size_t init_d = 0, init_b = 0;    // FP64 initial fields, if given
    bool has_init_d = false, has_init_b = false;
    int64_t nsrc = 0;
};

int64_t source_samples(const gfdtd_problem *p, int64_t steps);
int64_t field_cells(int64_t nz);
void carve_run(Carver &cv, const gfdtd_problem *p, int64_t steps, RunLayout &L);
size_t table_bytes(int nruns, int64_t max_tiles);
int64_t max_tiles_of(int64_t nz);
void choose_tiling(int precision, const gfdtd_exec *ex, int64_t max_steps,
                   int64_t total_cells, bool ring, int &C, int &T, int &G, int &K);
bool halo_lanes(double beta, int C, int T, int &hl, int &hr);

// Lane geometry of the tiles of one run: outer halos hl, hr for a T-step
// block; for G-wave tiles the overlaps xl, xr refreshed every K steps;
// own = cells a tile stores.
struct TileGeom {
    int G = 1, hl = 1, hr = 1, xl = 0, xr = 0, xk = 1;
    int64_t own = 0;
};
bool tile_geometry(double beta, int C, int T, int G, int K, TileGeom &g);
// One tile holding a whole open grid (no field halo for the block depth;
// the upwind side holds the block's profile moves); false if the grid does
// not fit.
bool whole_grid_geometry(const gfdtd_problem &p, int C, int T, int G, int K, TileGeom &g);
// The geometry a run gets: a whole-grid tile when it fits, else tile_geometry.
bool run_geometry(const gfdtd_problem &p, int C, int T, int G, int K, TileGeom &g);

// A run with host copies of its inputs.
struct RunHost {
    gfdtd_problem p{};
    int64_t steps = 0;
    int T = 1;                  // block depth of its group
    std::vector<double> eps, mu, omegas, init_d, init_b;
    std::vector<int64_t> probes;
    RunLayout L;
};

// Host copies of a (validated) problem's inputs; r.p points into them.
RunHost make_run_host(const gfdtd_problem &p, int64_t steps);
// Asynchronous uploads of a carved run's inputs (rest profile, probes,
// frequencies, initial fields) into the workspace at base.
hipError_t upload_run_inputs(char *base, const RunHost &r, hipStream_t stream);

void fill_run_desc(char *base, const RunHost &r, int precision, const TileGeom &g,
                   int64_t start_block, RunDesc &rd, PrepDesc &pd, DftDesc &dd);

// The tile reference of tile t of run m: bit w of probe_waves is set when
// wave w of the tile (G waves of C cells per lane) owns one of the run's
// probes, by the owned ranges the stepping kernel uses.
TileRef make_tile_ref(const RunHost &r, const RunDesc &rd, int m, int C, int G, int64_t t);

// The state a run of zero steps returns: its initial fields (or zeros),
// rounded to the run precision; either pointer may be null.
void initial_fields(const RunHost &r, double *d, double *b);

gfdtd_status copy_results(const char *ws, const RunHost &r, const gfdtd_result *unused,
                          hipStream_t stream, gfdtd_result *out);

// Runs of one precision and kind, stepped by one kernel instantiation.
struct Group {
    int precision = 0, kind = 0, C = 16, T = 16;
    int Gw = 1, K = 8;                // waves per tile, steps per refresh
    bool ring = false;                // periodic ends
    bool has_window = false;          // holds finite-duration modulations
    int part = 0;                     // stream its launches go to (0: the batch's)
    std::vector<int> members;         // run indices, longest first
    std::vector<int64_t> blocks_of;   // blocks per member
    std::vector<int64_t> tiles_prefix;
    int64_t nblocks = 0;
    int64_t max_cells = 0, max_field = 0, max_init = 0;
    int max_pf = 0;
    size_t table_off = 0, runs_off = 0, tiles_off = 0, prep_off = 0, dft_off = 0;
    std::vector<RunDesc> host_rd;
    std::vector<PrepDesc> host_pd;
    std::vector<DftDesc> host_dd;
    std::vector<TileRef> host_tiles;
};

struct Batch {
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<RunHost> runs;
    std::vector<Group> groups;
    int use_graph = -1;
    bool graph_on = false;
    // No events, graphs or streams are created (the allocation-free entry
    // point); stats then report no device times.
    bool no_alloc = false;
    bool ran = false;
    hipStream_t cap_stream = nullptr;
    // second stream for the launches of groups with part 1, forked from and
    // joined back to the batch's stream around the stepping launches
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    hipGraph_t graphs[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t execs[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t launches = 0, tiles_total = 0;
    double cell_updates = 0.0;

    gfdtd_status prepare(const gfdtd_problem *probs, const int64_t *steps,
                         int32_t count, const gfdtd_exec *ex, void *ws,
                         size_t ws_bytes, hipStream_t stream);
    void fill_desc(RunHost &r, const Group &G, const TileGeom &g, int64_t start_block,
                   RunDesc &rd, PrepDesc &pd, DftDesc &dd);
    int live_tiles(const Group &G, int64_t b) const;
    bool auto_graph() const;
    gfdtd_status enqueue_zero(hipStream_t s);
    gfdtd_status enqueue_steps(hipStream_t s, bool fork);
    gfdtd_status enqueue_dft(hipStream_t s);
    gfdtd_status build_graphs();
    gfdtd_status build_tiles(Group &G);
    void count_launches();
    gfdtd_status autotune(int trial, gfdtd_exec *chosen);
    gfdtd_status run();
    gfdtd_status collect(gfdtd_result *outs);
    void stats(gfdtd_stats *s) const;
    ~Batch();
};

}  // namespace gfdtd
