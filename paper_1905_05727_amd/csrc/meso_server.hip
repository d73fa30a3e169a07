// meso_server.hip -- continuous-batching server of independent solves
// (host side of the mf_server_* calls in include/meso.h).
//
// Device memory: one arena of hbm_budget bytes allocated at creation; every
// admitted solve holds one block of it: control block, two state copies and a
// dense FP64 read-back area (6 planes; 7 for a reactive liquid).  A first-fit free list with
// coalescing manages the blocks, so admission can never exceed the budget.
//
// Per tick: finished read-backs are harvested (non-blocking event queries),
// queued requests are admitted while a slot and a block are free (their
// initial state is uploaded and converted on the compute stream, so they join
// the very next batched launch), and one batched dt kernel plus one batched
// state-update kernel advance every admitted solve by one step.  A solve whose
// last step has been enqueued is converted to dense FP64 on the compute stream
// and copied to pinned host memory on the read-back stream, overlapping the
// following ticks.
//
// Host memory: a submitted request's primitive planes are copied once, into a
// pinned upload buffer from a pool, and go to the device straight from it; a
// finished request keeps its pinned read-back buffer until mf_server_result
// copies it into the caller's array.  Pooled buffers are reused by later
// requests, so a steady stream of requests neither allocates nor page-faults
// host memory.

#include "meso.h"
#include "meso_internal.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

using meso::Control;
using meso::Desc;

namespace {

// Rows per workgroup segment of a served solve at admission; the tile tables
// then choose the height per class of solves (class_seg_h).
constexpr int kServerSegH = 32;

struct Request {
    uint64_t id;
    mf_grid grid;
    mf_material mat[2];
    mf_options opt;
    int up;                       // pinned upload buffer (primitive planes) until admitted
    int64_t nsteps;
    int state;                    // MF_REQ_*
    int rb;                       // pinned read-back buffer (nc planes + control) once done
    int nc;                       // conserved planes: 6, or 7 for a reactive liquid
    double t_final;
    int64_t steps_final;
};

struct Pinned {                   // reusable pinned host buffer
    double *p;
    size_t bytes;
    hipEvent_t ev;                // last async copy that used it
};

struct Slot {
    bool used;
    uint64_t req;
    size_t off, bytes;            // arena block
    Desc d;
    int64_t steps_enq;            // steps enqueued so far
    int64_t nsteps;
    bool draining;
    int pin;                      // pinned buffer holding the read-back
    hipEvent_t done;              // read-back copy finished
};

struct FreeList {                 // first-fit arena allocator with coalescing
    std::map<size_t, size_t> free_;   // offset -> length
    size_t in_use = 0, peak = 0;
    void init(size_t n) {
        free_.clear();
        free_[0] = n;
    }
    bool alloc(size_t n, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t o2 = it->first + n;
                free_.erase(it);
                if (rest) free_[o2] = rest;
                in_use += n;
                peak = std::max(peak, in_use);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        in_use -= n;
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

size_t readback_bytes(const mf_grid *g, int nc) {
    return meso::round_up((size_t)nc * g->nx * (size_t)g->ny * sizeof(double), meso::kAlign);
}

}  // namespace

struct mf_server {
    mf_server_config cfg;
    hipStream_t st;               // compute stream
    hipStream_t rb;               // read-back stream
    bool own_st;
    char *arena;
    FreeList fl;
    std::vector<Slot> slots;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    std::deque<uint64_t> finished;    // tickets done or failed, not yet reported
    uint64_t next_id;
    // batched launch tables
    Desc *d_descs;
    int4 *d_tiles;
    size_t tiles_cap;
    std::vector<Pinned> tab_pins;     // pinned staging of the tables, ring
    size_t tab_next;
    bool dirty;
    int n_active;
    int n_tiles;
    // tiles per class, in this order: stiffened-gas liquid, inert Cochran-Chan
    // liquid, reactive Cochran-Chan liquid (one batched launch each)
    int n_tiles_cls[3];
    int n_cu;                     // compute units of the device (0: unknown)
    int64_t active_cells;
    // uploads of initial states: pinned buffers, filled at submission, free
    // again once their copy to the device has been enqueued
    double *d_stage;
    size_t stage_bytes;
    std::vector<Pinned> up_pins;
    std::vector<int> up_free;
    // read-back pinned buffers, held by a finished request until its result
    // is taken
    std::vector<Pinned> rb_pins;
    std::vector<int> rb_free;
    // in-flight tick events
    std::deque<hipEvent_t> inflight;
    std::vector<hipEvent_t> ev_pool;
    // stats
    int64_t ticks, cell_updates, completed;
};

namespace {

int32_t dev_err(hipError_t e) { return e == hipSuccess ? MF_OK : MF_E_DEVICE; }

hipEvent_t take_event(mf_server *s) {
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// A pinned buffer of at least `bytes` from a ring: waits for its last copy.
int32_t ring_pinned(std::vector<Pinned> &ring, size_t &next, size_t bytes, Pinned **out) {
    Pinned &p = ring[next];
    next = (next + 1) % ring.size();
    if (hipEventSynchronize(p.ev) != hipSuccess) return MF_E_DEVICE;
    if (p.bytes < bytes) {
        if (p.p) (void)hipHostFree(p.p);
        p.p = nullptr;
        p.bytes = 0;
        if (hipHostMalloc((void **)&p.p, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return MF_E_OUT_OF_MEMORY;
        }
        p.bytes = bytes;
    }
    *out = &p;
    return MF_OK;
}

// A pinned buffer of at least `bytes` from a pool: the smallest free one that
// fits (after its last asynchronous copy), else a new one.
int32_t pool_pinned(std::vector<Pinned> &pool, std::vector<int> &freel, size_t bytes, int *out) {
    int best = -1;
    for (size_t i = 0; i < freel.size(); ++i) {
        const Pinned &p = pool[freel[i]];
        if (p.bytes >= bytes && (best < 0 || p.bytes < pool[freel[best]].bytes)) best = (int)i;
    }
    if (best >= 0) {
        const int k = freel[best];
        freel.erase(freel.begin() + best);
        if (pool[k].ev && hipEventSynchronize(pool[k].ev) != hipSuccess) return MF_E_DEVICE;
        *out = k;
        return MF_OK;
    }
    Pinned p{nullptr, 0, nullptr};
    if (hipHostMalloc((void **)&p.p, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return MF_E_OUT_OF_MEMORY;
    }
    if (hipEventCreateWithFlags(&p.ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(p.p);
        return MF_E_DEVICE;
    }
    p.bytes = bytes;
    pool.push_back(p);
    *out = (int)pool.size() - 1;
    return MF_OK;
}

size_t request_bytes(const mf_grid *g, int prec, int nc) {
    return meso::kAlign + 2 * meso::state_bytes(g, prec, nc) + readback_bytes(g, nc);
}

// Upload and convert a request's initial state into a free slot.
int32_t admit_one(mf_server *s, Request &r, Slot &sl) {
    const size_t n = (size_t)r.grid.nx * r.grid.ny * r.nc;
    const size_t bytes = n * sizeof(double);
    if (bytes > s->stage_bytes) {
        if (s->d_stage) {
            if (hipStreamSynchronize(s->st) != hipSuccess) return MF_E_DEVICE;
            (void)hipFree(s->d_stage);
        }
        s->d_stage = nullptr;
        s->stage_bytes = 0;
        if (hipMalloc((void **)&s->d_stage, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return MF_E_OUT_OF_MEMORY;
        }
        s->stage_bytes = bytes;
    }
    Pinned &pp = s->up_pins[r.up];
    hipError_t e = hipMemcpyAsync(s->d_stage, pp.p, bytes, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipEventRecord(pp.ev, s->st);
    s->up_free.push_back(r.up);   // reusable once that copy has run
    r.up = -1;
    if (e == hipSuccess) e = meso::launch_init_control(sl.d, 0.0, 0, s->st);
    if (e == hipSuccess) e = meso::launch_prim_to_cons(sl.d, s->cfg.precision, 0, s->d_stage, s->st);
    if (e == hipSuccess) e = meso::launch_reduce(sl.d, s->cfg.precision, 0, s->st);
    return dev_err(e);
}

int32_t admit(mf_server *s) {
    while (!s->queue.empty()) {
        int free_slot = -1;
        for (size_t i = 0; i < s->slots.size(); ++i)
            if (!s->slots[i].used) {
                free_slot = (int)i;
                break;
            }
        if (free_slot < 0) return MF_OK;
        Request &r = s->reqs[s->queue.front()];
        const size_t need = request_bytes(&r.grid, s->cfg.precision, r.nc);
        size_t off = 0;
        if (!s->fl.alloc(need, &off)) return MF_OK;   // wait for memory
        Slot &sl = s->slots[free_slot];
        sl.used = true;
        sl.req = r.id;
        sl.off = off;
        sl.bytes = need;
        sl.steps_enq = 0;
        sl.nsteps = r.nsteps;
        sl.draining = false;
        sl.pin = -1;
        meso::fill_desc(sl.d, &r.grid, r.mat, &r.opt, s->arena + off, kServerSegH);
        s->queue.pop_front();
        r.state = MF_REQ_RUNNING;
        const int32_t rc = admit_one(s, r, sl);
        if (rc != MF_OK) return rc;
        s->dirty = true;
    }
    return MF_OK;
}

// Rows per segment for the tiles of one class of solves: the same model as a
// lone solve's, over all the class's grids (few solves get short segments and
// more workgroups in flight, a full device taller ones and less halo work).
// No stored value depends on the height.  MESO_SERVE_SEG_H (>= 1) fixes it.
int class_seg_h(mf_server *s, const std::vector<Slot *> &members) {
    if (const char *env = getenv("MESO_SERVE_SEG_H")) {
        const int v = atoi(env);
        if (v >= 1) return v;
    }
    std::vector<int> strips, rows;
    for (const Slot *sl : members) {
        strips.push_back(sl->d.nstrips);
        rows.push_back(sl->d.ny);
    }
    return meso::seg_h_model(strips.data(), rows.data(), (int)members.size(), s->n_cu);
}

// Rebuild the descriptor and tile tables of the advancing solves.
int32_t rebuild_tables(mf_server *s) {
    std::vector<Desc> descs;
    std::vector<int4> tiles, tail_tiles;
    int64_t cells = 0;
    // tiles grouped by class (liquid EoS, reaction): one batched launch each
    std::vector<Slot *> members;
    for (int cls = 0; cls < 3; ++cls) {
        const size_t before = tiles.size();
        members.clear();
        for (auto &sl : s->slots) {
            if (!sl.used || sl.draining) continue;
            const int c = sl.d.nc == 7 ? 2 : sl.d.eos2;
            if (c == cls) members.push_back(&sl);
        }
        if (members.empty()) {
            s->n_tiles_cls[cls] = 0;
            continue;
        }
        const int h = class_seg_h(s, members);
        // Under load (segments of 12 rows or more) each solve's last h rows
        // go into h/4-row segments dispatched after all the class's leading
        // ones, which evens out the end of the launch: a warm burst of the
        // serving workload measured 5 % faster on MI355X, p99 6 % lower.
        // MESO_SERVE_TAPER = "h2,rows" sets the tail ("0,0": none); a height
        // fixed by MESO_SERVE_SEG_H stays uniform.
        const char *fixed = getenv("MESO_SERVE_SEG_H");
        int h2 = 0, tail = 0;
        if (!(fixed && atoi(fixed) >= 1) && h >= 12) {
            h2 = h / 4;
            tail = h;
        }
        if (const char *env = getenv("MESO_SERVE_TAPER")) {
            if (sscanf(env, "%d,%d", &h2, &tail) != 2) h2 = tail = 0;
        }
        tail_tiles.clear();
        for (Slot *psl : members) {
            Slot &sl = *psl;
            meso::set_segments(sl.d, sl.d.ny, h, h2, tail);
            const int k = (int)descs.size();
            descs.push_back(sl.d);
            for (int by = 0; by < sl.d.nsegs; ++by)
                for (int bx = 0; bx < sl.d.nstrips; ++bx)
                    (by < sl.d.seg_n1 ? tiles : tail_tiles).push_back(make_int4(k, bx, by, 0));
            cells += (int64_t)sl.d.nx * sl.d.ny;
        }
        // every solve's tail segments after all the class's leading ones
        tiles.insert(tiles.end(), tail_tiles.begin(), tail_tiles.end());
        s->n_tiles_cls[cls] = (int)(tiles.size() - before);
    }
    s->n_active = (int)descs.size();
    s->n_tiles = (int)tiles.size();
    s->active_cells = cells;
    s->dirty = false;
    if (descs.empty()) return MF_OK;
    if (tiles.size() > s->tiles_cap) {
        if (hipStreamSynchronize(s->st) != hipSuccess) return MF_E_DEVICE;
        if (s->d_tiles) (void)hipFree(s->d_tiles);
        s->d_tiles = nullptr;
        size_t cap = std::max(tiles.size(), 2 * s->tiles_cap);
        if (hipMalloc((void **)&s->d_tiles, cap * sizeof(int4)) != hipSuccess) {
            (void)hipGetLastError();
            s->tiles_cap = 0;
            return MF_E_OUT_OF_MEMORY;
        }
        s->tiles_cap = cap;
    }
    const size_t bd = descs.size() * sizeof(Desc), bt = tiles.size() * sizeof(int4);
    Pinned *pp = nullptr;
    int32_t rc = ring_pinned(s->tab_pins, s->tab_next, bd + bt, &pp);
    if (rc != MF_OK) return rc;
    memcpy(pp->p, descs.data(), bd);
    memcpy((char *)pp->p + bd, tiles.data(), bt);
    hipError_t e = hipMemcpyAsync(s->d_descs, pp->p, bd, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_tiles, (char *)pp->p + bd, bt, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipEventRecord(pp->ev, s->st);
    return dev_err(e);
}

// The solve in `sl` has all its steps enqueued: convert and copy it back.
int32_t start_drain(mf_server *s, Slot &sl) {
    Request &r = s->reqs[sl.req];
    const size_t n = (size_t)r.grid.nx * r.grid.ny;
    const int nc = r.nc;
    const size_t bytes = nc * n * sizeof(double) + sizeof(Control);
    // a free pinned read-back buffer
    int pin = -1;
    int32_t rc = pool_pinned(s->rb_pins, s->rb_free, bytes, &pin);
    if (rc != MF_OK) return rc;
    sl.pin = pin;
    sl.draining = true;
    double *dense = (double *)(s->arena + sl.off + meso::kAlign +
                               2 * meso::state_bytes(&r.grid, s->cfg.precision, nc));
    const int src = (int)(sl.nsteps & 1);
    hipError_t e = hipSuccess;
    for (int f = 0; f < nc && e == hipSuccess; ++f)
        e = meso::launch_read_field(sl.d, s->cfg.precision, src, f < 6 ? f : MF_Z2RHO2LAM,
                                    dense + f * n, s->st);
    hipEvent_t conv = take_event(s);
    if (!conv) return MF_E_DEVICE;
    if (e == hipSuccess) e = hipEventRecord(conv, s->st);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->rb, conv, 0);
    double *hp = s->rb_pins[pin].p;
    if (e == hipSuccess)
        e = hipMemcpyAsync(hp, dense, nc * n * sizeof(double), hipMemcpyDeviceToHost, s->rb);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hp + nc * n, sl.d.ctl, sizeof(Control), hipMemcpyDeviceToHost, s->rb);
    sl.done = take_event(s);
    if (!sl.done) return MF_E_DEVICE;
    if (e == hipSuccess) e = hipEventRecord(sl.done, s->rb);
    s->ev_pool.push_back(conv);   // reusable once recorded again later (stream order)
    s->dirty = true;
    return dev_err(e);
}

// Collect finished read-backs; wait = true blocks on each.
int32_t harvest(mf_server *s, bool wait) {
    for (auto &sl : s->slots) {
        if (!sl.used || !sl.draining) continue;
        hipError_t q = wait ? hipEventSynchronize(sl.done) : hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return MF_E_DEVICE;
        Request &r = s->reqs[sl.req];
        const size_t n = (size_t)r.grid.nx * r.grid.ny;
        const double *hp = s->rb_pins[sl.pin].p;
        Control c;
        memcpy(&c, hp + (size_t)r.nc * n, sizeof(Control));
        r.t_final = c.t;
        r.steps_final = c.step;
        r.state = c.err ? MF_REQ_FAILED : MF_REQ_DONE;
        s->finished.push_back(sl.req);
        if (c.err) s->rb_free.push_back(sl.pin);   // nothing to hand back
        else r.rb = sl.pin;                          // held until the result is taken
        s->ev_pool.push_back(sl.done);
        s->fl.release(sl.off, sl.bytes);
        sl.used = false;
        sl.draining = false;
        s->completed++;
    }
    return MF_OK;
}

void count(const mf_server *s, int32_t *active, int32_t *queued) {
    int a = 0;
    for (auto &sl : s->slots)
        if (sl.used && !sl.draining) ++a;
    if (active) *active = a;
    if (queued) *queued = (int32_t)s->queue.size();
}

}  // namespace

extern "C" {

size_t mf_server_request_bytes(const mf_grid *grid, const mf_material mat[2], int32_t precision) {
    if (!meso::valid_grid(grid) || precision < MF_FP64 || precision > MF_FP64_FAST) return 0;
    if (mat && !meso::valid_materials(mat)) return 0;
    return request_bytes(grid, precision, meso::planes_of(mat));
}

int32_t mf_server_create(const mf_server_config *cfg, void *hip_stream, mf_server **out) {
    if (!out) return MF_E_INVALID_ARG;
    *out = nullptr;
    if (!cfg || cfg->hbm_budget < meso::kAlign || cfg->max_slots < 1 || cfg->max_slots > 65536 ||
        cfg->precision < MF_FP64 || cfg->precision > MF_FP64_FAST ||
        (cfg->limiter != MF_LIM_VANLEER && cfg->limiter != MF_LIM_MINMOD) ||
        cfg->max_inflight < 1 || cfg->max_inflight > 64)
        return MF_E_INVALID_ARG;
    mf_server *s = new (std::nothrow) mf_server();
    if (!s) return MF_E_OUT_OF_MEMORY;
    s->cfg = *cfg;
    s->cfg.hbm_budget = cfg->hbm_budget / meso::kAlign * meso::kAlign;
    s->next_id = 1;
    s->own_st = hip_stream == nullptr;
    hipError_t e = hipSuccess;
    if (s->own_st) e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
    else s->st = (hipStream_t)hip_stream;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->rb, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void **)&s->arena, s->cfg.hbm_budget);
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_descs, sizeof(Desc) * cfg->max_slots);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (s->arena) (void)hipFree(s->arena);
        if (s->d_descs) (void)hipFree(s->d_descs);
        if (s->rb) (void)hipStreamDestroy(s->rb);
        if (s->own_st && s->st) (void)hipStreamDestroy(s->st);
        delete s;
        return e == hipErrorOutOfMemory ? MF_E_OUT_OF_MEMORY : MF_E_DEVICE;
    }
    s->n_cu = meso::device_cus();
    s->fl.init(s->cfg.hbm_budget);
    s->slots.assign(cfg->max_slots, Slot());
    for (auto &sl : s->slots) sl.used = false;
    const int ring = cfg->max_inflight + 2;
    for (int i = 0; i < ring; ++i) {
        Pinned a{nullptr, 0, nullptr};
        (void)hipEventCreateWithFlags(&a.ev, hipEventDisableTiming);
        s->tab_pins.push_back(a);
    }
    *out = s;
    return MF_OK;
}

int32_t mf_server_submit(mf_server *s, const mf_grid *grid, const mf_material mat[2],
                         const mf_options *opt, const double *prim, int64_t nsteps,
                         uint64_t *ticket) {
    if (!s || !prim || !ticket || nsteps < 1) return MF_E_INVALID_ARG;
    if (!meso::valid_grid(grid) || !meso::valid_materials(mat) || !meso::valid_scheme(opt))
        return MF_E_INVALID_ARG;
    if (opt->precision != s->cfg.precision || opt->limiter != s->cfg.limiter)
        return MF_E_INVALID_ARG;
    if (grid->nx > 1 << 15 || grid->ny > 1 << 15) return MF_E_INVALID_ARG;
    const int nc = meso::planes_of(mat);
    if (request_bytes(grid, s->cfg.precision, nc) > s->cfg.hbm_budget) return MF_E_OUT_OF_MEMORY;
    Request r;
    r.id = s->next_id++;
    r.grid = *grid;
    r.mat[0] = mat[0];
    r.mat[1] = mat[1];
    r.opt = *opt;
    r.opt.fused = 1;
    const size_t n = (size_t)grid->nx * grid->ny * nc;
    int up = -1;
    const int32_t rc = pool_pinned(s->up_pins, s->up_free, n * sizeof(double), &up);
    if (rc != MF_OK) return rc;
    memcpy(s->up_pins[up].p, prim, n * sizeof(double));
    r.up = up;
    r.rb = -1;
    r.nc = nc;
    r.nsteps = nsteps;
    r.state = MF_REQ_QUEUED;
    r.t_final = 0.0;
    r.steps_final = 0;
    *ticket = r.id;
    s->queue.push_back(r.id);
    s->reqs.emplace(r.id, std::move(r));
    return MF_OK;
}

int32_t mf_server_tick(mf_server *s, int32_t *active, int32_t *queued) {
    if (!s) return MF_E_INVALID_ARG;
    int32_t rc = harvest(s, false);
    if (rc == MF_OK) rc = admit(s);
    if (rc != MF_OK) return rc;
    if (s->dirty) {
        rc = rebuild_tables(s);
        if (rc != MF_OK) return rc;
    }
    if (s->n_active > 0) {
        if ((int)s->inflight.size() >= s->cfg.max_inflight) {
            hipEvent_t old = s->inflight.front();
            s->inflight.pop_front();
            if (hipEventSynchronize(old) != hipSuccess) return MF_E_DEVICE;
            s->ev_pool.push_back(old);
        }
        hipError_t e = meso::launch_batched_dt(s->d_descs, s->n_active, s->st);
        int first = 0;
        for (int cls = 0; cls < 3 && e == hipSuccess; ++cls) {
            e = meso::launch_batched_step(s->d_descs, s->d_tiles + first, s->n_tiles_cls[cls],
                                          s->cfg.precision, s->cfg.limiter, cls == 0 ? 0 : 1,
                                          cls == 2 ? 7 : 6, s->st);
            first += s->n_tiles_cls[cls];
        }
        hipEvent_t ev = take_event(s);
        if (!ev) return MF_E_DEVICE;
        if (e == hipSuccess) e = hipEventRecord(ev, s->st);
        if (e != hipSuccess) return MF_E_DEVICE;
        s->inflight.push_back(ev);
        s->ticks++;
        s->cell_updates += s->active_cells;
        for (auto &sl : s->slots) {
            if (!sl.used || sl.draining) continue;
            if (++sl.steps_enq == sl.nsteps) {
                rc = start_drain(s, sl);
                if (rc != MF_OK) return rc;
            }
        }
    }
    count(s, active, queued);
    return MF_OK;
}

int32_t mf_server_poll(mf_server *s, uint64_t ticket, int32_t *state) {
    if (!s || !state) return MF_E_INVALID_ARG;
    int32_t rc = harvest(s, false);
    if (rc != MF_OK) return rc;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return MF_E_INVALID_ARG;
    *state = it->second.state;
    return MF_OK;
}

int32_t mf_server_finished(mf_server *s, uint64_t *tickets, int32_t capacity, int32_t *count_out) {
    if (!s || !count_out || capacity < 0 || (capacity > 0 && !tickets)) return MF_E_INVALID_ARG;
    int32_t rc = harvest(s, false);
    if (rc != MF_OK) return rc;
    int32_t n = 0;
    while (n < capacity && !s->finished.empty()) {
        tickets[n++] = s->finished.front();
        s->finished.pop_front();
    }
    *count_out = n;
    return MF_OK;
}

int32_t mf_server_result(mf_server *s, uint64_t ticket, double *out_cons, size_t count_,
                         double *t, int64_t *steps) {
    if (!s) return MF_E_INVALID_ARG;
    int32_t rc = harvest(s, false);
    if (rc != MF_OK) return rc;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return MF_E_INVALID_ARG;
    Request &r = it->second;
    if (r.state == MF_REQ_QUEUED || r.state == MF_REQ_RUNNING) return MF_E_NOT_READY;
    if (r.state == MF_REQ_FAILED) {
        s->reqs.erase(it);
        return MF_E_NONFINITE_STATE;
    }
    const size_t n = (size_t)r.grid.nx * r.grid.ny * r.nc;
    if (!out_cons || count_ != n) return MF_E_INVALID_ARG;
    memcpy(out_cons, s->rb_pins[r.rb].p, n * sizeof(double));
    s->rb_free.push_back(r.rb);
    if (t) *t = r.t_final;
    if (steps) *steps = r.steps_final;
    s->reqs.erase(it);
    return MF_OK;
}

int32_t mf_server_drain(mf_server *s) {
    if (!s) return MF_E_INVALID_ARG;
    for (;;) {
        int32_t a = 0, q = 0;
        int32_t rc = mf_server_tick(s, &a, &q);
        if (rc != MF_OK) return rc;
        if (a == 0 && q == 0) break;
    }
    return harvest(s, true);
}

int32_t mf_server_get_stats(mf_server *s, mf_server_stats *st) {
    if (!s || !st) return MF_E_INVALID_ARG;
    memset(st, 0, sizeof(*st));
    st->ticks = s->ticks;
    st->cell_updates = s->cell_updates;
    st->completed = s->completed;
    st->peak_bytes = (int64_t)s->fl.peak;
    st->bytes_in_use = (int64_t)s->fl.in_use;
    count(s, &st->active, &st->queued);
    int dr = 0;
    for (auto &sl : s->slots)
        if (sl.used && sl.draining) ++dr;
    st->draining = dr;
    return MF_OK;
}

int32_t mf_server_destroy(mf_server *s) {
    if (!s) return MF_E_INVALID_ARG;
    hipError_t e = hipStreamSynchronize(s->st);
    (void)hipStreamSynchronize(s->rb);
    for (auto ev : s->inflight) (void)hipEventDestroy(ev);
    for (auto ev : s->ev_pool) (void)hipEventDestroy(ev);
    for (auto &sl : s->slots)
        if (sl.used && sl.draining) (void)hipEventDestroy(sl.done);
    for (auto *ring : {&s->tab_pins, &s->up_pins, &s->rb_pins})
        for (auto &p : *ring) {
            if (p.p) (void)hipHostFree(p.p);
            if (p.ev) (void)hipEventDestroy(p.ev);
        }
    if (s->d_stage) (void)hipFree(s->d_stage);
    if (s->d_tiles) (void)hipFree(s->d_tiles);
    (void)hipFree(s->d_descs);
    (void)hipFree(s->arena);
    (void)hipStreamDestroy(s->rb);
    if (s->own_st) (void)hipStreamDestroy(s->st);
    delete s;
    return dev_err(e);
}

}  // extern "C"
