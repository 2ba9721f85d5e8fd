// Continuous-batching server of the generalized-FDTD library.
//
// Requests wait in a FIFO queue until their device state fits in the pool
// (the caller's HBM budget) and a slot is free.  Admitted runs share
// progress blocks: one block advances every admitted run by T steps with
// one k_tiles launch per (precision, kind) group.  The host knows each
// run's last block in advance, so it enqueues blocks back to back up to the
// next retirement, then waits once, forms the DFTs of the finished runs,
// copies their results out, frees their memory and admits waiting
// requests.  A run's arithmetic depends only on its own cells, so its
// results are the same alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <unordered_map>
#include <vector>

#include "gfdtd.h"
#include "gfdtd_internal.h"
#include "runtime.h"

namespace gfdtd {

namespace {

// First-fit allocator over [0, size) with coalescing free list.
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

enum State { QUEUED, LIVE, DONE };

struct Request {
    uint64_t id = 0;
    RunHost r;
    State state = QUEUED;
    size_t off = 0, bytes = 0;       // pool region
    int group = 0;                   // precision * 2 + kind
    int hl = 0, hr = 0;
    int64_t own = 0, ntiles = 0;
    int64_t start_block = 0, end_block = 0;
    // results
    int32_t status = GFDTD_OK;
    std::vector<double> trace, dft_re, dft_im, final_d, final_b;
};

}  // namespace

struct Server {
    hipStream_t stream = nullptr;
    char *pool_base = nullptr;
    size_t pool_bytes = 0;
    int max_slots = 1;
    int Cg[2] = {16, 8};             // cells per lane by precision
    int T = 16;
    Pool pool;
    size_t tables_off = 0, tables_bytes = 0;
    int64_t tile_cap = 0;
    uint64_t next_id = 1;
    int64_t gblock = 0;              // global block counter
    std::deque<uint64_t> queue;
    std::vector<uint64_t> live;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    bool dirty = true;
    // per group device tables (offsets in the pool)
    size_t runs_off[4] = {0, 0, 0, 0}, tiles_off[4] = {0, 0, 0, 0};
    size_t aux_off = 0;              // PrepDesc / DftDesc staging
    int ntiles[4] = {0, 0, 0, 0};
    std::vector<RunDesc> h_rd[4];
    std::vector<TileRef> h_tiles[4];
    std::vector<PrepDesc> h_pd;
    std::vector<DftDesc> h_dd;

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
        gfdtd_exec ex{};
        ex.struct_size = sizeof ex;
        ex.block_steps = cfg->block_steps;
        choose_tiling(GFDTD_F32, &ex, 0, INT64_MAX, Cg[0], T);
        choose_tiling(GFDTD_F64, &ex, 0, INT64_MAX, Cg[1], T);
        // descriptor tables at the front of the pool: run tables for every
        // slot and group, tile tables sized to the pool (a tile stores at
        // least 64 cells and a run costs more than 32 bytes per cell)
        tile_cap = (int64_t)(pool_bytes / (64 * 32)) + 8 * (int64_t)max_slots;
        Carver cv;
        for (int g = 0; g < 4; ++g) {
            runs_off[g] = cv.take((size_t)max_slots * sizeof(RunDesc));
            tiles_off[g] = cv.take((size_t)tile_cap * sizeof(TileRef));
        }
        aux_off = cv.take((size_t)max_slots * std::max(sizeof(PrepDesc), sizeof(DftDesc)));
        tables_bytes = cv.off;
        if (tables_bytes >= pool_bytes)
            return fail(GFDTD_E_NOMEM, "pool of %zu bytes too small for the run tables "
                        "(%zu bytes)", pool_bytes, tables_bytes);
        pool.init(pool_bytes - tables_bytes);
        return GFDTD_OK;
    }

    size_t footprint(const gfdtd_problem *p, int64_t steps, RunLayout &L) const
    {
        Carver cv;
        carve_run(cv, p, steps, L);
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
        r.p = *p;
        r.steps = steps;
        r.T = T;
        r.eps.assign(p->eps_rest, p->eps_rest + p->nz);
        r.mu.assign(p->mu_rest, p->mu_rest + p->nz);
        r.probes.assign(p->probe_cells, p->probe_cells + p->nprobe);
        r.omegas.assign(p->omegas, p->omegas + p->nfreq);
        r.p.eps_rest = r.eps.data();
        r.p.mu_rest = r.mu.data();
        r.p.probe_cells = r.probes.data();
        r.p.omegas = r.omegas.data();
        rq->bytes = footprint(&r.p, steps, r.L);
        if (rq->bytes > pool.size)
            return fail(GFDTD_E_NOMEM, "request needs %zu bytes, pool holds %zu",
                        rq->bytes, pool.size);
        rq->group = p->precision * 2 + p->kind;
        if (!halo_lanes(p->beta, Cg[p->precision], T, rq->hl, rq->hr))
            return fail(GFDTD_E_INVALID, "block depth too large");
        rq->own = (int64_t)(kWave - rq->hl - rq->hr) * Cg[p->precision];
        rq->ntiles = (p->nz + rq->own - 1) / rq->own;
        rq->id = next_id++;
        *id = rq->id;
        queue.push_back(rq->id);
        reqs[rq->id] = std::move(rq);
        return GFDTD_OK;
    }

    // Admit waiting requests in arrival order while they fit.
    gfdtd_status admit()
    {
        std::vector<Request *> adm;
        while (!queue.empty() && (int)live.size() < max_slots) {
            Request *rq = reqs[queue.front()].get();
            if (ntiles[rq->group] + rq->ntiles > tile_cap)
                break;
            size_t off;
            if (!pool.alloc(rq->bytes, off))
                break;
            queue.pop_front();
            rq->off = tables_bytes + off;
            // offsets of the run's arrays relative to the pool base
            RunLayout &L = rq->r.L;
            size_t *fields[] = {&L.eps, &L.mu, &L.cE, &L.cH, &L.gB, &L.murL, &L.murR,
                                &L.src, &L.probes, &L.omegas, &L.trace, &L.dft,
                                &L.field[0], &L.field[1], &L.field[2], &L.field[3]};
            for (size_t *f : fields)
                *f += rq->off;
            rq->state = LIVE;
            rq->start_block = gblock;
            rq->end_block = gblock + (rq->r.steps + T - 1) / T - 1;
            live.push_back(rq->id);
            ntiles[rq->group] += (int)rq->ntiles;
            adm.push_back(rq);
            dirty = true;
        }
        if (adm.empty())
            return GFDTD_OK;
        hipError_t e;
        h_pd.resize(adm.size());
        for (size_t i = 0; i < adm.size(); ++i) {
            Request *rq = adm[i];
            RunHost &r = rq->r;
            const size_t nz = (size_t)r.p.nz;
            if ((e = hipMemcpyAsync(pool_base + r.L.eps, r.eps.data(), nz * 8,
                                    hipMemcpyHostToDevice, stream)) ||
                (e = hipMemcpyAsync(pool_base + r.L.mu, r.mu.data(), nz * 8,
                                    hipMemcpyHostToDevice, stream)))
                return hip_fail(e, "upload rest profile");
            if (r.p.nprobe &&
                (e = hipMemcpyAsync(pool_base + r.L.probes, r.probes.data(),
                                    r.probes.size() * 8, hipMemcpyHostToDevice, stream)))
                return hip_fail(e, "upload probes");
            if (r.p.nfreq &&
                (e = hipMemcpyAsync(pool_base + r.L.omegas, r.omegas.data(),
                                    r.omegas.size() * 8, hipMemcpyHostToDevice, stream)))
                return hip_fail(e, "upload omegas");
            RunDesc rd;
            DftDesc dd;
            fill_run_desc(pool_base, r, r.p.precision, rq->hl, rq->hr, rq->own,
                          rq->start_block, rd, h_pd[i], dd);
        }
        // set-up and zero fill, grouped by precision (word size)
        for (int prec = 0; prec < 2; ++prec) {
            std::vector<PrepDesc> sel;
            int64_t maxc = 0, maxf = 0;
            for (size_t i = 0; i < adm.size(); ++i)
                if (adm[i]->r.p.precision == prec) {
                    sel.push_back(h_pd[i]);
                    maxc = std::max<int64_t>(maxc, std::max(adm[i]->r.p.nz, adm[i]->r.L.nsrc));
                    maxf = std::max<int64_t>(maxf, field_cells(adm[i]->r.p.nz));
                }
            if (sel.empty())
                continue;
            if ((e = hipMemcpyAsync(pool_base + aux_off, sel.data(),
                                    sel.size() * sizeof(PrepDesc), hipMemcpyHostToDevice,
                                    stream)))
                return hip_fail(e, "upload set-up table");
            const PrepDesc *dp = reinterpret_cast<const PrepDesc *>(pool_base + aux_off);
            if ((e = launch_prep(dp, (int)sel.size(), (int)std::min<int64_t>(maxc, 1 << 30),
                                 stream)) ||
                (e = launch_zero(dp, (int)sel.size(), maxf, prec, stream)))
                return hip_fail(e, "launch set-up");
            // the staging table is reused: finish before the next upload
            if ((e = hipStreamSynchronize(stream)))
                return hip_fail(e, "set-up");
        }
        return GFDTD_OK;
    }

    gfdtd_status rebuild_tables()
    {
        hipError_t e;
        for (int g = 0; g < 4; ++g) {
            h_rd[g].clear();
            h_tiles[g].clear();
        }
        for (uint64_t id : live) {
            Request *rq = reqs[id].get();
            const int g = rq->group;
            RunDesc rd;
            PrepDesc pd;
            DftDesc dd;
            fill_run_desc(pool_base, rq->r, rq->r.p.precision, rq->hl, rq->hr, rq->own,
                          rq->start_block, rd, pd, dd);
            const int m = (int)h_rd[g].size();
            h_rd[g].push_back(rd);
            for (int64_t t = 0; t < rq->ntiles; ++t)
                h_tiles[g].push_back(TileRef{m, (int32_t)t});
        }
        for (int g = 0; g < 4; ++g) {
            ntiles[g] = (int)h_tiles[g].size();
            if (h_rd[g].empty())
                continue;
            if ((e = hipMemcpyAsync(pool_base + runs_off[g], h_rd[g].data(),
                                    h_rd[g].size() * sizeof(RunDesc),
                                    hipMemcpyHostToDevice, stream)) ||
                (e = hipMemcpyAsync(pool_base + tiles_off[g], h_tiles[g].data(),
                                    h_tiles[g].size() * sizeof(TileRef),
                                    hipMemcpyHostToDevice, stream)))
                return hip_fail(e, "upload run tables");
        }
        dirty = false;
        return GFDTD_OK;
    }

    gfdtd_status retire(const std::vector<Request *> &done)
    {
        hipError_t e;
        h_dd.resize(done.size());
        for (size_t i = 0; i < done.size(); ++i) {
            RunDesc rd;
            PrepDesc pd;
            fill_run_desc(pool_base, done[i]->r, done[i]->r.p.precision, done[i]->hl,
                          done[i]->hr, done[i]->own, done[i]->start_block, rd, pd,
                          h_dd[i]);
        }
        int max_pf = 0;
        for (auto *rq : done)
            max_pf = std::max(max_pf, rq->r.p.nprobe * rq->r.p.nfreq);
        if (!done.empty()) {
            if ((e = hipMemcpyAsync(pool_base + aux_off, h_dd.data(),
                                    h_dd.size() * sizeof(DftDesc), hipMemcpyHostToDevice,
                                    stream)))
                return hip_fail(e, "upload DFT table");
            if ((e = launch_dft(reinterpret_cast<const DftDesc *>(pool_base + aux_off),
                                (int)done.size(), max_pf, stream)))
                return hip_fail(e, "launch DFT");
        }
        for (auto *rq : done) {
            const gfdtd_problem &p = rq->r.p;
            rq->dft_re.assign((size_t)p.nprobe * p.nfreq, 0.0);
            rq->dft_im.assign((size_t)p.nprobe * p.nfreq, 0.0);
            if (p.flags & GFDTD_FLAG_RECORD_TRACE)
                rq->trace.assign((size_t)p.nprobe * rq->r.steps, 0.0);
            if (p.flags & GFDTD_FLAG_KEEP_FIELDS) {
                rq->final_d.assign((size_t)p.nz, 0.0);
                rq->final_b.assign((size_t)p.nz, 0.0);
            }
            gfdtd_result out{};
            out.struct_size = sizeof out;
            out.trace = rq->trace.empty() ? nullptr : rq->trace.data();
            out.dft_re = rq->dft_re.data();
            out.dft_im = rq->dft_im.data();
            out.final_d = rq->final_d.empty() ? nullptr : rq->final_d.data();
            out.final_b = rq->final_b.empty() ? nullptr : rq->final_b.data();
            gfdtd_status st = copy_results(pool_base, rq->r, nullptr, stream, &out);
            if (st != GFDTD_OK)
                return st;
            rq->status = out.run_status;
            rq->state = DONE;
            pool.release(rq->off - tables_bytes, rq->bytes);
            ntiles[rq->group] -= (int)rq->ntiles;
            live.erase(std::find(live.begin(), live.end(), rq->id));
            dirty = true;
        }
        return GFDTD_OK;
    }

    gfdtd_status progress(int32_t max_blocks, int32_t *nlive, int32_t *nqueued)
    {
        hipError_t e;
        int32_t left = max_blocks < 0 ? 0 : max_blocks;
        gfdtd_status st;
        // zero-step requests finish on admission
        while (left > 0) {
            if ((st = admit()) != GFDTD_OK)
                return st;
            std::vector<Request *> done;
            for (uint64_t id : live)
                if (reqs[id]->r.steps == 0)
                    done.push_back(reqs[id].get());
            if (!done.empty()) {
                if ((st = retire(done)) != GFDTD_OK)
                    return st;
                continue;
            }
            if (live.empty())
                break;
            if (dirty && (st = rebuild_tables()) != GFDTD_OK)
                return st;
            int64_t next_end = INT64_MAX;
            for (uint64_t id : live)
                next_end = std::min(next_end, reqs[id]->end_block);
            const int64_t nb = std::min<int64_t>(next_end - gblock + 1, left);
            for (int64_t b = 0; b < nb; ++b, ++gblock)
                for (int g = 0; g < 4; ++g) {
                    if (!ntiles[g])
                        continue;
                    e = launch_tiles(g >> 1, g & 1, Cg[g >> 1],
                                     reinterpret_cast<const RunDesc *>(pool_base + runs_off[g]),
                                     reinterpret_cast<const TileRef *>(pool_base + tiles_off[g]),
                                     gblock, T, ntiles[g], stream);
                    if (e)
                        return hip_fail(e, "launch step kernel");
                }
            left -= (int32_t)nb;
            for (uint64_t id : live)
                if (reqs[id]->end_block < gblock)
                    done.push_back(reqs[id].get());
            if (!done.empty() && (st = retire(done)) != GFDTD_OK)
                return st;
        }
        if ((e = hipStreamSynchronize(stream)))
            return hip_fail(e, "progress");
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
        if (rq->state != DONE)
            return GFDTD_E_NOT_READY;
        if (!out || out->struct_size < sizeof(gfdtd_result))
            return fail(GFDTD_E_INVALID, "bad result struct");
        out->run_status = rq->status;
        out->steps_done = rq->r.steps;
        if (out->dft_re && out->dft_im && !rq->dft_re.empty()) {
            std::memcpy(out->dft_re, rq->dft_re.data(), rq->dft_re.size() * 8);
            std::memcpy(out->dft_im, rq->dft_im.data(), rq->dft_im.size() * 8);
        }
        if (out->trace && !rq->trace.empty())
            std::memcpy(out->trace, rq->trace.data(), rq->trace.size() * 8);
        if (out->final_d && !rq->final_d.empty())
            std::memcpy(out->final_d, rq->final_d.data(), rq->final_d.size() * 8);
        if (out->final_b && !rq->final_b.empty())
            std::memcpy(out->final_b, rq->final_b.data(), rq->final_b.size() * 8);
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
        (void)hipStreamSynchronize(sv->stream);
        delete sv;
    }
}

}  // extern "C"
