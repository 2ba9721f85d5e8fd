// Continuous-batching server of the generalized-FDTD library.
//
// Requests wait in a FIFO queue until their device state fits in the pool
// (the caller's HBM budget) and a slot is free.  Admitted runs share
// progress blocks: one block advances every admitted run by T steps with
// one k_tiles launch per (precision, kind, ring) group.
//
// Each (precision, kind) pair runs on a stream of its own, so launches of
// different pairs overlap; they fork from the caller's stream at every
// progress call.  Everything is stream-ordered, so the host never waits for
// the GPU in steady state:
//  - admission copies a request's inputs into a pinned host buffer, then
//    asynchronously into its pool region (which also holds its own run,
//    set-up and DFT descriptors), and enqueues its set-up and zero fill;
//  - the run and tile tables of the live set are double-buffered in the
//    pool and refreshed from pinned staging only when the set changes;
//  - a run whose last block has been enqueued is retired at once: its DFT
//    kernel and the copies of its results into its pinned buffer are
//    enqueued and followed by an event; its pool region is released (any
//    later use of that memory is ordered after those copies);
//  - a run admitted into memory released by runs of other groups first
//    waits for those runs' retirement events;
//  - poll() checks the event.
// A run's arithmetic depends only on its own cells and on its own start
// block, so its results are the same bits alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gfdtd.h"
#include "gfdtd_internal.h"
#include "runtime.h"

namespace gfdtd {

namespace {

// First-fit allocator over [0, size) with a coalescing free list.
struct Pool {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length

    void init(size_t n)
    {
        size = n;
        free_.clear();
        if (n)
            free_[0] = n;
    }
    bool alloc(size_t n, size_t &off)
    {
        n = (n + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest)
                    free_[off + n] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + 255) / 256 * 256;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Pinned host memory owned by one request or staging slot.
struct Pinned {
    void *p = nullptr;
    size_t n = 0;
    ~Pinned()
    {
        if (p)
            (void)hipHostFree(p);
    }
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= n)
            return hipSuccess;
        // grown geometrically from 1 MiB: pinning is slow, and tables grow
        // as requests join
        const size_t want = std::max({bytes, 2 * n, size_t(1) << 20});
        if (p)
            (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e == hipSuccess)
            n = want;
        return e;
    }
};

// Reusable pinned blocks in power-of-two size classes.  Pinning memory is
// slow (tens of milliseconds for tens of MiB), and pinning in the progress
// call would hold up every live request: a class above kSyncBytes is pinned
// by a helper thread, and the request that needs it waits at the head of
// the queue meanwhile (try_get reports not ready).
struct PinnedPool {
    static constexpr size_t kSyncBytes = size_t(1) << 22;   // 4 MiB
    std::mutex mu;
    std::condition_variable cv;
    std::map<size_t, std::vector<void *>> free_;
    std::deque<size_t> todo;          // classes the helper is to pin
    std::map<size_t, int> pending;    // blocks being pinned, by class
    hipError_t failed = hipSuccess;   // the helper's first error
    bool stop = false;
    std::thread helper;

    ~PinnedPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        if (helper.joinable())
            helper.join();
        for (auto &kv : free_)
            for (void *p : kv.second)
                (void)hipHostFree(p);
    }
    static size_t klass(size_t n)
    {
        size_t k = 4096;
        while (k < n)
            k <<= 1;
        return k;
    }
    void run()
    {
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            cv.wait(lk, [&] { return stop || !todo.empty(); });
            if (stop)
                return;
            const size_t k = todo.front();
            todo.pop_front();
            lk.unlock();
            void *p = nullptr;
            const hipError_t e = hipHostMalloc(&p, k, hipHostMallocDefault);
            lk.lock();
            pending[k] -= 1;
            if (e == hipSuccess)
                free_[k].push_back(p);
            else if (failed == hipSuccess)
                failed = e;
        }
    }
    // A block of at least n bytes in *p (capacity *cap) with *ready = true;
    // or *ready = false while the helper pins one (ask again later).
    hipError_t try_get(size_t n, void **p, size_t *cap, bool *ready)
    {
        const size_t k = klass(n);
        *cap = k;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (failed != hipSuccess)
                return failed;
            auto &v = free_[k];
            if (!v.empty()) {
                *p = v.back();
                v.pop_back();
                *ready = true;
                return hipSuccess;
            }
            if (k > kSyncBytes) {
                if (pending[k] == 0) {
                    pending[k] += 1;
                    todo.push_back(k);
                    if (!helper.joinable())
                        helper = std::thread(&PinnedPool::run, this);
                    cv.notify_one();
                }
                *ready = false;
                return hipSuccess;
            }
        }
        *ready = true;
        return hipHostMalloc(p, k, hipHostMallocDefault);
    }
    void put(void *p, size_t cap)
    {
        if (p) {
            std::lock_guard<std::mutex> lk(mu);
            free_[cap].push_back(p);
        }
    }
};

enum State { QUEUED, LIVE, RETIRING, DONE };

struct Request {
    uint64_t id = 0;
    RunHost r;
    State state = QUEUED;
    size_t off = 0, bytes = 0;       // pool region
    size_t desc_off = 0;             // RunDesc, PrepDesc, DftDesc of the run
    int group = 0;                   // group_of(precision, kind, abc)
    TileGeom geom;                   // one-wave tiles at its group's tiling
    int64_t ntiles = 0;              // tiles at that tiling
    int64_t ntiles_cap = 0;          // tiles at the narrowest tiling (bound)
    int64_t start_block = 0, end_block = 0;
    // pinned host block: inputs at admission, results at retirement
    void *host = nullptr;
    size_t host_cap = 0;
    size_t host_bytes = 0;           // 0 until laid out (host_layout)
    size_t h_eps = 0, h_mu = 0, h_pr = 0, h_om = 0, h_id = 0, h_ib = 0, h_desc = 0;
    size_t h_dft = 0, h_trace = 0, h_d = 0, h_b = 0;
    hipEvent_t done_ev = nullptr;
    int32_t status = GFDTD_OK;
    PinnedPool *pins = nullptr;
    ~Request()
    {
        if (done_ev)
            (void)hipEventDestroy(done_ev);
        if (pins)
            pins->put(host, host_cap);
    }
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

struct Server {
    hipStream_t stream = nullptr;    // the caller's stream
    hipStream_t gs[4] = {nullptr, nullptr, nullptr, nullptr};   // by g >> 1
    hipEvent_t fork_ev = nullptr;
    // per group: retirements (releases of pool memory) its stream has not
    // yet been ordered after
    std::vector<std::shared_ptr<void>> released[kGroups];
    PinnedPool pins;
    char *pool_base = nullptr;
    size_t pool_bytes = 0;
    int max_slots = 1;
    // Cells per lane, by tiling level and precision.  Level 0 is the
    // throughput tiling; deeper levels use narrower lanes, so more waves
    // share the same cells and each steps faster (a step's latency grows
    // with the cells per lane).  The level is the first one at which the
    // live runs fill kTargetTiles one-wave tiles (all tiles resident and
    // several waves per SIMD), else the last: while the GPU is under-filled,
    // narrower lanes cost nothing and shorten every request's latency.
    static constexpr int kLevels = 3;
    static constexpr int64_t kTargetTiles = 4096;    // 4 waves per SIMD
    int Clev[kLevels][2] = {{16, 8}, {8, 4}, {4, 4}};
    int level = 0;
    int Cgrp[kGroups] = {};          // cells per lane of each group's tables
    int T = 32;
    Pool pool;
    size_t tables_bytes = 0;
    int64_t tile_cap = 0;
    uint64_t next_id = 1;
    int64_t gblock = 0;              // global block counter
    std::deque<uint64_t> queue;
    std::vector<uint64_t> live;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    bool gdirty[kGroups] = {true, true, true, true, true, true, true, true};
    int cur[kGroups] = {};           // table buffer in use, per group
    size_t runs_off[2][kGroups], tiles_off[2][kGroups];
    int ntiles[kGroups] = {};        // tiles in each group's current table
    int64_t cap_tiles[kGroups] = {}; // live tiles at the narrowest tiling
    int nwin[kGroups] = {};          // live requests with a time window
    // run-ahead tracking: events recorded on every group stream after each
    // run of block launches, with the global block count reached
    struct Inflight {
        int64_t gblock_end;
        hipEvent_t ev[4];
    };
    std::deque<Inflight> inflight;
    std::vector<hipEvent_t> spare_ev;
    int64_t done_block = 0;          // blocks below this have finished
    int max_ahead = 8;

    gfdtd_status mark_inflight()
    {
        Inflight f;
        f.gblock_end = gblock;
        for (int k = 0; k < 4; ++k) {
            hipError_t e;
            if (spare_ev.empty()) {
                hipEvent_t ev;
                if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)))
                    return hip_fail(e, "create events");
                spare_ev.push_back(ev);
            }
            f.ev[k] = spare_ev.back();
            spare_ev.pop_back();
            if ((e = hipEventRecord(f.ev[k], gs[k])))
                return hip_fail(e, "record progress");
        }
        inflight.push_back(f);
        return GFDTD_OK;
    }

    gfdtd_status reap()
    {
        while (!inflight.empty()) {
            Inflight &f = inflight.front();
            for (int k = 0; k < 4; ++k) {
                const hipError_t e = hipEventQuery(f.ev[k]);
                if (e == hipErrorNotReady)
                    return GFDTD_OK;
                if (e != hipSuccess)
                    return hip_fail(e, "query progress");
            }
            done_block = f.gblock_end;
            for (int k = 0; k < 4; ++k)
                spare_ev.push_back(f.ev[k]);
            inflight.pop_front();
        }
        return GFDTD_OK;
    }
    Pinned stage[2][kGroups];        // host staging of the table buffers
    hipEvent_t stage_ev[2][kGroups] = {};
    bool stage_used[2][kGroups] = {};

    ~Server()
    {
        for (int g = 0; g < 4; ++g)
            if (gs[g])
                (void)hipStreamSynchronize(gs[g]);
        reqs.clear();
        for (auto &v : released)
            v.clear();
        for (auto &row : stage_ev)
            for (auto &e : row)
                if (e)
                    (void)hipEventDestroy(e);
        for (hipStream_t s : gs)
            if (s)
                (void)hipStreamDestroy(s);
        if (fork_ev)
            (void)hipEventDestroy(fork_ev);
        for (auto &f : inflight)
            for (hipEvent_t e : f.ev)
                (void)hipEventDestroy(e);
        for (hipEvent_t e : spare_ev)
            (void)hipEventDestroy(e);
    }

    gfdtd_status create(const gfdtd_server_config *cfg)
    {
        if (!cfg || cfg->struct_size < sizeof(gfdtd_server_config))
            return fail(GFDTD_E_INVALID, "bad server config");
        if (cfg->max_slots < 1)
            return fail(GFDTD_E_INVALID, "max_slots must be >= 1");
        if (!cfg->pool || cfg->pool_bytes == 0)
            return fail(GFDTD_E_INVALID, "pool missing");
        if (cfg->block_steps < 0 || cfg->block_steps > 256)
            return fail(GFDTD_E_INVALID, "block_steps outside 0..256");
        stream = static_cast<hipStream_t>(cfg->stream);
        pool_base = static_cast<char *>(cfg->pool);
        pool_bytes = cfg->pool_bytes;
        max_slots = cfg->max_slots;
        // Tiling on the serving mix (measured, saturated rate): FP32 16
        // cells per lane, FP64 8 (twice the registers per cell), 48 steps
        // per block; 12 cells and 32 steps served 7 % less, 8 and 24 a
        // further 17 % less.
        T = cfg->block_steps > 0 ? cfg->block_steps : 48;
        if (cfg->max_ahead < 0)
            return fail(GFDTD_E_INVALID, "max_ahead must be >= 0");
        max_ahead = cfg->max_ahead > 0 ? cfg->max_ahead : 8;
        // two copies of the run and tile tables at the front of the pool;
        // a tile stores at least 64 cells and a run costs more than 32
        // bytes per cell, which bounds the tiles the pool can hold
        tile_cap = (int64_t)(pool_bytes / (64 * 32)) + 8 * (int64_t)max_slots;
        Carver cv;
        for (int k = 0; k < 2; ++k)
            for (int g = 0; g < kGroups; ++g) {
                runs_off[k][g] = cv.take((size_t)max_slots * sizeof(RunDesc));
                tiles_off[k][g] = cv.take((size_t)tile_cap * sizeof(TileRef));
            }
        tables_bytes = cv.off;
        if (tables_bytes >= pool_bytes)
            return fail(GFDTD_E_NOMEM, "pool of %zu bytes too small for the run tables "
                        "(%zu bytes)", pool_bytes, tables_bytes);
        pool.init(pool_bytes - tables_bytes);
        hipError_t e;
        for (int k = 0; k < 2; ++k)
            for (int g = 0; g < kGroups; ++g)
                if ((e = hipEventCreateWithFlags(&stage_ev[k][g], hipEventDisableTiming)))
                    return hip_fail(e, "create events");
        for (int g = 0; g < 4; ++g)
            if ((e = hipStreamCreateWithFlags(&gs[g], hipStreamNonBlocking)))
                return hip_fail(e, "create group streams");
        if ((e = hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming)))
            return hip_fail(e, "create events");
        return GFDTD_OK;
    }

    // Pool bytes of one request: its arrays plus its three descriptors.
    size_t footprint(const gfdtd_problem *p, int64_t steps, RunLayout &L,
                     size_t &desc_rel) const
    {
        Carver cv;
        carve_run(cv, p, steps, L);
        desc_rel = cv.take(sizeof(RunDesc) + sizeof(PrepDesc) + sizeof(DftDesc));
        return cv.off;
    }

    gfdtd_status submit(const gfdtd_problem *p, int64_t steps, uint64_t *id)
    {
        gfdtd_status st = validate(p, steps);
        if (st != GFDTD_OK)
            return st;
        if ((st = preflight(p, nullptr)) != GFDTD_OK)
            return st;
        std::unique_ptr<Request> rq(new Request);
        RunHost &r = rq->r;
        r = make_run_host(*p, steps);
        r.T = T;
        rq->bytes = footprint(&r.p, steps, r.L, rq->desc_off);
        if (rq->bytes > pool.size)
            return fail(GFDTD_E_NOMEM, "request needs %zu bytes, pool holds %zu",
                        rq->bytes, pool.size);
        rq->group = group_of(p->precision, p->kind, p->abc);
        if (!tile_geometry(p->beta, Clev[0][p->precision], T, 1, 1, rq->geom))
            return fail(GFDTD_E_INVALID, "block depth too large");
        rq->ntiles = (p->nz + rq->geom.own - 1) / rq->geom.own;
        rq->ntiles_cap = rq->ntiles;
        for (int l = 1; l < kLevels; ++l) {
            TileGeom g;
            if (tile_geometry(p->beta, Clev[l][p->precision], T, 1, 1, g))
                rq->ntiles_cap = std::max<int64_t>(rq->ntiles_cap, (p->nz + g.own - 1) / g.own);
        }
        if (rq->ntiles_cap > tile_cap)
            return fail(GFDTD_E_NOMEM, "request needs %lld tiles, tables hold %lld",
                        (long long)rq->ntiles_cap, (long long)tile_cap);
        rq->id = next_id++;
        *id = rq->id;
        queue.push_back(rq->id);
        reqs[rq->id] = std::move(rq);
        return GFDTD_OK;
    }

    // Admit waiting requests in arrival order while they fit.
    // Offsets of a request's pinned block: inputs (rest profile, probes,
    // frequencies, initial fields, descriptors) and results (spectra,
    // trace, final fields).
    static void host_layout(Request *rq)
    {
        const RunHost &r = rq->r;
        const gfdtd_problem &p = r.p;
        const RunLayout &L = r.L;
        const size_t nz = (size_t)p.nz;
        const size_t w = p.precision == GFDTD_F32 ? 4 : 8;
        size_t o = 0;
        rq->h_eps = o;  o += align256(nz * 8);
        rq->h_mu = o;   o += align256(nz * 8);
        rq->h_pr = o;   o += align256(std::max<size_t>(r.probes.size(), 1) * 8);
        rq->h_om = o;   o += align256(std::max<size_t>(r.omegas.size(), 1) * 8);
        rq->h_id = o;   o += L.has_init_d ? align256(nz * 8) : 0;
        rq->h_ib = o;   o += L.has_init_b ? align256(nz * 8) : 0;
        rq->h_desc = o; o += align256(sizeof(RunDesc) + sizeof(PrepDesc) + sizeof(DftDesc));
        rq->h_dft = o;  o += align256((size_t)std::max(p.nprobe * p.nfreq, 1) * 16);
        rq->h_trace = o;
        if (p.flags & GFDTD_FLAG_RECORD_TRACE)
            o += align256((size_t)std::max<int64_t>((int64_t)p.nprobe * r.steps, 1) * 8);
        rq->h_d = o;
        rq->h_b = o;
        if (p.flags & GFDTD_FLAG_KEEP_FIELDS) {
            o += align256(nz * w);
            rq->h_b = o;
            o += align256(nz * w);
        }
        rq->host_bytes = o;
    }

    gfdtd_status admit()
    {
        hipError_t e;
        while (!queue.empty() && (int)live.size() < max_slots) {
            Request *rq = reqs[queue.front()].get();
            // its pinned block (inputs now, results at retirement) first:
            // a large one is pinned by a helper thread meanwhile
            if (!rq->host) {
                if (!rq->host_bytes)
                    host_layout(rq);
                bool ready = false;
                if ((e = pins.try_get(rq->host_bytes, &rq->host, &rq->host_cap, &ready)))
                    return hip_fail(e, "pinned host buffer");
                if (!ready)
                    break;
                rq->pins = &pins;
            }
            if (cap_tiles[rq->group] + rq->ntiles_cap > tile_cap)
                break;
            size_t off;
            if (!pool.alloc(rq->bytes, off))
                break;
            queue.pop_front();
            rq->off = tables_bytes + off;
            RunLayout &L = rq->r.L;
            size_t *fields[] = {&L.eps, &L.mu, &L.cE, &L.cH, &L.gB, &L.murL, &L.murR,
                                &L.src, &L.probes, &L.omegas, &L.trace, &L.dft,
                                &L.field[0], &L.field[1], &L.field[2], &L.field[3],
                                &L.init_d, &L.init_b};
            for (size_t *f : fields)
                *f += rq->off;
            rq->desc_off += rq->off;
            rq->state = LIVE;
            rq->start_block = gblock;
            rq->end_block = gblock + (rq->r.steps + T - 1) / T - 1;
            live.push_back(rq->id);
            cap_tiles[rq->group] += rq->ntiles_cap;
            if (rq->r.p.flags & GFDTD_FLAG_TIME_WINDOW)
                nwin[rq->group] += 1;
            gdirty[rq->group] = true;
            hipStream_t st = gs[rq->group >> 1];
            // memory released by retirements on other streams is reused
            // only after those retirements
            for (auto &ev : released[rq->group])
                if ((e = hipStreamWaitEvent(st, static_cast<hipEvent_t>(ev.get()), 0)))
                    return hip_fail(e, "order memory reuse");
            released[rq->group].clear();

            // the pinned block's inputs
            RunHost &r = rq->r;
            const gfdtd_problem &p = r.p;
            const size_t nz = (size_t)p.nz;
            const size_t h_eps = rq->h_eps, h_mu = rq->h_mu, h_pr = rq->h_pr,
                         h_om = rq->h_om, h_id = rq->h_id, h_ib = rq->h_ib,
                         h_desc = rq->h_desc;
            char *h = static_cast<char *>(rq->host);
            std::memcpy(h + h_eps, r.eps.data(), nz * 8);
            std::memcpy(h + h_mu, r.mu.data(), nz * 8);
            if (!r.probes.empty())
                std::memcpy(h + h_pr, r.probes.data(), r.probes.size() * 8);
            if (!r.omegas.empty())
                std::memcpy(h + h_om, r.omegas.data(), r.omegas.size() * 8);
            if (L.has_init_d)
                std::memcpy(h + h_id, r.init_d.data(), nz * 8);
            if (L.has_init_b)
                std::memcpy(h + h_ib, r.init_b.data(), nz * 8);
            RunDesc rd;
            PrepDesc pd;
            DftDesc dd;
            fill_run_desc(pool_base, r, p.precision, rq->geom, rq->start_block, rd, pd, dd);
            std::memcpy(h + h_desc, &rd, sizeof rd);
            std::memcpy(h + h_desc + sizeof rd, &pd, sizeof pd);
            std::memcpy(h + h_desc + sizeof rd + sizeof pd, &dd, sizeof dd);
            const size_t desc_bytes = sizeof rd + sizeof pd + sizeof dd;
            if ((e = hipMemcpyAsync(pool_base + L.eps, h + h_eps, nz * 8,
                                    hipMemcpyHostToDevice, st)) ||
                (e = hipMemcpyAsync(pool_base + L.mu, h + h_mu, nz * 8,
                                    hipMemcpyHostToDevice, st)) ||
                (e = hipMemcpyAsync(pool_base + rq->desc_off, h + h_desc, desc_bytes,
                                    hipMemcpyHostToDevice, st)))
                return hip_fail(e, "upload request");
            if (!r.probes.empty() &&
                (e = hipMemcpyAsync(pool_base + L.probes, h + h_pr, r.probes.size() * 8,
                                    hipMemcpyHostToDevice, st)))
                return hip_fail(e, "upload probes");
            if (!r.omegas.empty() &&
                (e = hipMemcpyAsync(pool_base + L.omegas, h + h_om, r.omegas.size() * 8,
                                    hipMemcpyHostToDevice, st)))
                return hip_fail(e, "upload omegas");
            if ((L.has_init_d &&
                 (e = hipMemcpyAsync(pool_base + L.init_d, h + h_id, nz * 8,
                                     hipMemcpyHostToDevice, st))) ||
                (L.has_init_b &&
                 (e = hipMemcpyAsync(pool_base + L.init_b, h + h_ib, nz * 8,
                                     hipMemcpyHostToDevice, st))))
                return hip_fail(e, "upload initial fields");
            const PrepDesc *dp =
                reinterpret_cast<const PrepDesc *>(pool_base + rq->desc_off + sizeof(RunDesc));
            if ((e = launch_prep(dp, 1, (int)std::min<int64_t>(std::max(p.nz, L.nsrc), 1 << 30),
                                 st)) ||
                (e = launch_zero(dp, 1, field_cells(p.nz), p.precision, st)) ||
                ((L.has_init_d || L.has_init_b) &&
                 (e = launch_init(dp, 1, p.nz, p.precision, st))))
                return hip_fail(e, "launch set-up");
        }
        return GFDTD_OK;
    }

    // Write a group's tables into its spare buffer (stream-ordered after
    // every launch that used it) and switch to it.
    // Tiles of request rq at cells per lane C (false: no valid geometry).
    bool tiles_at(const Request *rq, int C, TileGeom &g, int64_t &n) const
    {
        if (!tile_geometry(rq->r.p.beta, C, T, 1, 1, g))
            return false;
        n = (rq->r.p.nz + g.own - 1) / g.own;
        return true;
    }

    // Tiling level for the current live set (see Clev).
    int choose_level() const
    {
        for (int l = 0; l < kLevels; ++l) {
            int64_t n = 0;
            bool ok = true;
            for (uint64_t id : live) {
                const Request *rq = reqs.at(id).get();
                TileGeom g;
                int64_t k = 0;
                ok = ok && tiles_at(rq, Clev[l][rq->r.p.precision], g, k);
                n += k;
            }
            if (!ok)
                return l > 0 ? l - 1 : 0;
            if (n >= kTargetTiles || l == kLevels - 1)
                return l;
        }
        return 0;
    }

    gfdtd_status rebuild_tables(int g)
    {
        hipError_t e;
        const int nxt = cur[g] ^ 1;
        std::vector<RunDesc> rd;
        std::vector<TileRef> tl;
        Cgrp[g] = Clev[level][group_precision(g)];
        for (uint64_t id : live) {
            Request *rq = reqs[id].get();
            if (rq->group != g)
                continue;
            if (!tiles_at(rq, Cgrp[g], rq->geom, rq->ntiles))
                return fail(GFDTD_E_INVALID, "no tiling at %d cells per lane", Cgrp[g]);
            RunDesc d;
            PrepDesc pd;
            DftDesc dd;
            fill_run_desc(pool_base, rq->r, rq->r.p.precision, rq->geom, rq->start_block, d,
                          pd, dd);
            const int m = (int)rd.size();
            rd.push_back(d);
            for (int64_t t = 0; t < rq->ntiles; ++t)
                tl.push_back(make_tile_ref(rq->r, d, m, Cgrp[g], 1, t));
        }
        ntiles[g] = (int)tl.size();
        gdirty[g] = false;
        cur[g] = nxt;
        if (rd.empty())
            return GFDTD_OK;
        const size_t a = rd.size() * sizeof(RunDesc);
        const size_t b = tl.size() * sizeof(TileRef);
        // the staging buffer's previous copies must have been consumed
        if (stage_used[nxt][g] && (e = hipEventSynchronize(stage_ev[nxt][g])))
            return hip_fail(e, "table staging");
        if ((e = stage[nxt][g].ensure(align256(a) + align256(b))))
            return hip_fail(e, "pinned table staging");
        char *h = static_cast<char *>(stage[nxt][g].p);
        std::memcpy(h, rd.data(), a);
        std::memcpy(h + align256(a), tl.data(), b);
        hipStream_t gst = gs[g >> 1];
        if ((e = hipMemcpyAsync(pool_base + runs_off[nxt][g], h, a, hipMemcpyHostToDevice,
                                gst)) ||
            (e = hipMemcpyAsync(pool_base + tiles_off[nxt][g], h + align256(a), b,
                                hipMemcpyHostToDevice, gst)) ||
            (e = hipEventRecord(stage_ev[nxt][g], gst)))
            return hip_fail(e, "upload tables");
        stage_used[nxt][g] = true;
        return GFDTD_OK;
    }

    // Enqueue the DFT and result copies of a run whose last block has been
    // enqueued, release its pool region and drop it from the live set.
    gfdtd_status retire(Request *rq)
    {
        hipError_t e;
        const gfdtd_problem &p = rq->r.p;
        const RunLayout &L = rq->r.L;
        char *h = static_cast<char *>(rq->host);
        hipStream_t stream = gs[rq->group >> 1];
        const DftDesc *dd = reinterpret_cast<const DftDesc *>(
            pool_base + rq->desc_off + sizeof(RunDesc) + sizeof(PrepDesc));
        if ((e = launch_dft(dd, 1, p.nprobe * p.nfreq, stream)))
            return hip_fail(e, "launch DFT");
        if (p.nprobe * p.nfreq > 0 &&
            (e = hipMemcpyAsync(h + rq->h_dft, pool_base + L.dft,
                                (size_t)p.nprobe * p.nfreq * 16, hipMemcpyDeviceToHost,
                                stream)))
            return hip_fail(e, "copy DFT");
        if ((p.flags & GFDTD_FLAG_RECORD_TRACE) && p.nprobe > 0 && rq->r.steps > 0 &&
            (e = hipMemcpyAsync(h + rq->h_trace, pool_base + L.trace,
                                (size_t)p.nprobe * rq->r.steps * 8, hipMemcpyDeviceToHost,
                                stream)))
            return hip_fail(e, "copy trace");
        if ((p.flags & GFDTD_FLAG_KEEP_FIELDS) && rq->r.steps > 0) {
            const size_t w = p.precision == GFDTD_F32 ? 4 : 8;
            const int fin = (int)(((rq->r.steps + T - 1) / T) & 1);
            if ((e = hipMemcpyAsync(h + rq->h_d, pool_base + L.field[fin] + kPad * w,
                                    (size_t)p.nz * w, hipMemcpyDeviceToHost, stream)) ||
                (e = hipMemcpyAsync(h + rq->h_b, pool_base + L.field[2 + fin] + kPad * w,
                                    (size_t)p.nz * w, hipMemcpyDeviceToHost, stream)))
                return hip_fail(e, "copy fields");
        }
        if ((e = hipEventCreateWithFlags(&rq->done_ev, hipEventDisableTiming)) ||
            (e = hipEventRecord(rq->done_ev, stream)))
            return hip_fail(e, "record retirement");
        // a server-owned event orders later reuse of the region on other
        // streams (the request's own event lives only until it is polled)
        hipEvent_t rel = nullptr;
        if ((e = hipEventCreateWithFlags(&rel, hipEventDisableTiming)) ||
            (e = hipEventRecord(rel, stream)))
            return hip_fail(e, "record release");
        std::shared_ptr<void> ev(rel, [](void *x) {
            (void)hipEventDestroy(static_cast<hipEvent_t>(x));
        });
        for (int g = 0; g < kGroups; ++g)
            if ((g >> 1) != (rq->group >> 1))
                released[g].push_back(ev);
        rq->state = RETIRING;
        pool.release(rq->off - tables_bytes, rq->bytes);
        cap_tiles[rq->group] -= rq->ntiles_cap;
        if (rq->r.p.flags & GFDTD_FLAG_TIME_WINDOW)
            nwin[rq->group] -= 1;
        live.erase(std::find(live.begin(), live.end(), rq->id));
        gdirty[rq->group] = true;
        return GFDTD_OK;
    }

    gfdtd_status progress(int32_t max_blocks, int32_t *nlive, int32_t *nqueued)
    {
        hipError_t e;
        int32_t left = max_blocks < 0 ? 0 : max_blocks;
        gfdtd_status st;
        // order the server's work after what the caller has enqueued
        if ((e = hipEventRecord(fork_ev, stream)))
            return hip_fail(e, "fork");
        for (hipStream_t g : gs)
            if ((e = hipStreamWaitEvent(g, fork_ev, 0)))
                return hip_fail(e, "fork");
        while (true) {
            if ((st = admit()) != GFDTD_OK)
                return st;
            bool retired = false;
            for (size_t i = 0; i < live.size();) {
                Request *rq = reqs[live[i]].get();
                if (rq->r.steps == 0) {      // nothing to step
                    if ((st = retire(rq)) != GFDTD_OK)
                        return st;
                    retired = true;
                } else {
                    ++i;
                }
            }
            if (retired)
                continue;
            if (live.empty() || left <= 0)
                break;
            bool changed = false;
            for (int g = 0; g < kGroups; ++g)
                changed = changed || gdirty[g];
            if (changed) {
                const int l = choose_level();
                if (l != level) {
                    level = l;
                    for (int g = 0; g < kGroups; ++g)
                        gdirty[g] = gdirty[g] || ntiles[g] > 0;
                }
            }
            for (int g = 0; g < kGroups; ++g)
                if (gdirty[g] && (st = rebuild_tables(g)) != GFDTD_OK)
                    return st;
            int64_t next_end = INT64_MAX;
            for (uint64_t id : live)
                next_end = std::min(next_end, reqs[id]->end_block);
            // run-ahead limit: at most max_ahead blocks enqueued beyond the
            // last block the GPU has finished (a request admitted now then
            // waits behind at most that many)
            if ((st = reap()) != GFDTD_OK)
                return st;
            const int64_t room = (int64_t)max_ahead - (gblock - done_block);
            if (room <= 0)
                break;
            const int64_t nb = std::min<int64_t>(std::min<int64_t>(next_end - gblock + 1, left),
                                                 room);
            for (int64_t b = 0; b < nb; ++b, ++gblock)
                for (int g = 0; g < kGroups; ++g) {
                    if (!ntiles[g])
                        continue;
                    const int pr = group_precision(g);
                    for (int w = 0; w < (nwin[g] ? 2 : 1); ++w) {
                        e = launch_tiles(pr, group_kind(g), group_ring(g), w == 1, Cgrp[g], 1,
                                         reinterpret_cast<const RunDesc *>(pool_base + runs_off[cur[g]][g]),
                                         reinterpret_cast<const TileRef *>(pool_base + tiles_off[cur[g]][g]),
                                         gblock, T, ntiles[g], gs[g >> 1]);
                        if (e)
                            return hip_fail(e, "launch step kernel");
                    }
                }
            left -= (int32_t)nb;
            if ((st = mark_inflight()) != GFDTD_OK)
                return st;
            for (size_t i = 0; i < live.size();) {
                Request *rq = reqs[live[i]].get();
                if (rq->end_block < gblock) {
                    if ((st = retire(rq)) != GFDTD_OK)
                        return st;
                } else {
                    ++i;
                }
            }
        }
        if (nlive)
            *nlive = (int32_t)live.size();
        if (nqueued)
            *nqueued = (int32_t)queue.size();
        return GFDTD_OK;
    }

    gfdtd_status poll(uint64_t id, gfdtd_result *out)
    {
        auto it = reqs.find(id);
        if (it == reqs.end())
            return fail(GFDTD_E_INVALID, "unknown request %llu", (unsigned long long)id);
        Request *rq = it->second.get();
        if (rq->state == QUEUED || rq->state == LIVE)
            return GFDTD_E_NOT_READY;
        if (rq->state == RETIRING) {
            hipError_t q = hipEventQuery(rq->done_ev);
            if (q == hipErrorNotReady)
                return GFDTD_E_NOT_READY;
            if (q != hipSuccess)
                return hip_fail(q, "retirement");
            rq->state = DONE;
            const gfdtd_problem &p = rq->r.p;
            const char *h = static_cast<const char *>(rq->host);
            bool finite = true;
            const double *dft = reinterpret_cast<const double *>(h + rq->h_dft);
            for (int i = 0; i < 2 * p.nprobe * p.nfreq; ++i)
                finite = finite && std::isfinite(dft[i]);
            if (p.flags & GFDTD_FLAG_RECORD_TRACE) {
                const double *tr = reinterpret_cast<const double *>(h + rq->h_trace);
                for (int64_t i = 0; i < (int64_t)p.nprobe * rq->r.steps; ++i)
                    finite = finite && std::isfinite(tr[i]);
            }
            rq->status = finite ? GFDTD_OK : GFDTD_E_BLOWUP;
        }
        if (!out)                    // readiness query only
            return GFDTD_OK;
        if (out->struct_size < sizeof(gfdtd_result))
            return fail(GFDTD_E_INVALID, "bad result struct");
        const gfdtd_problem &p = rq->r.p;
        const char *h = static_cast<const char *>(rq->host);
        out->run_status = rq->status;
        out->steps_done = rq->r.steps;
        const double *dft = reinterpret_cast<const double *>(h + rq->h_dft);
        if (out->dft_re && out->dft_im)
            for (int i = 0; i < p.nprobe * p.nfreq; ++i) {
                out->dft_re[i] = dft[2 * i];
                out->dft_im[i] = dft[2 * i + 1];
            }
        if (out->trace && (p.flags & GFDTD_FLAG_RECORD_TRACE) && p.nprobe > 0)
            std::memcpy(out->trace, h + rq->h_trace, (size_t)p.nprobe * rq->r.steps * 8);
        const bool keep = (p.flags & GFDTD_FLAG_KEEP_FIELDS) != 0;
        const bool f32 = p.precision == GFDTD_F32;
        auto field = [&](size_t o, double *dst, int64_t n) {
            for (int64_t i = 0; i < n; ++i)
                dst[i] = f32 ? (double)reinterpret_cast<const float *>(h + o)[i]
                             : reinterpret_cast<const double *>(h + o)[i];
        };
        if (keep && rq->r.steps == 0) {
            initial_fields(rq->r, out->final_d, out->final_b);
        } else if (keep) {
            const bool ring = p.abc == GFDTD_ABC_PERIODIC;
            if (out->final_d)
                field(rq->h_d, out->final_d, p.nz);
            if (out->final_b) {
                field(rq->h_b, out->final_b, ring ? p.nz : p.nz - 1);
                if (!ring)
                    out->final_b[p.nz - 1] = 0.0;
            }
        }
        reqs.erase(it);
        return GFDTD_OK;
    }
};

}  // namespace gfdtd

using namespace gfdtd;

extern "C" {

gfdtd_status gfdtd_server_create(const gfdtd_server_config *cfg, gfdtd_server **out)
{
    clear_error();
    if (!out)
        return fail(GFDTD_E_INVALID, "out is NULL");
    *out = nullptr;
    std::unique_ptr<Server> s(new Server);
    gfdtd_status st = s->create(cfg);
    if (st != GFDTD_OK)
        return st;
    *out = reinterpret_cast<gfdtd_server *>(s.release());
    return GFDTD_OK;
}

gfdtd_status gfdtd_server_submit(gfdtd_server *s, const gfdtd_problem *p, int64_t steps,
                                 uint64_t *id)
{
    clear_error();
    if (!s || !id)
        return fail(GFDTD_E_INVALID, "bad arguments");
    return reinterpret_cast<Server *>(s)->submit(p, steps, id);
}

gfdtd_status gfdtd_server_progress(gfdtd_server *s, int32_t max_blocks, int32_t *live,
                                   int32_t *queued)
{
    clear_error();
    if (!s)
        return fail(GFDTD_E_INVALID, "server is NULL");
    return reinterpret_cast<Server *>(s)->progress(max_blocks, live, queued);
}

gfdtd_status gfdtd_server_poll(gfdtd_server *s, uint64_t id, gfdtd_result *out)
{
    clear_error();
    if (!s)
        return fail(GFDTD_E_INVALID, "server is NULL");
    return reinterpret_cast<Server *>(s)->poll(id, out);
}

void gfdtd_server_destroy(gfdtd_server *s)
{
    if (s) {
        Server *sv = reinterpret_cast<Server *>(s);
        delete sv;      // waits for the group streams
    }
}

}  // extern "C"
