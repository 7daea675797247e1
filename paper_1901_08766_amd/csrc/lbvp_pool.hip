// lbvp_pool.hip -- the serving pool of include/lbvp.h: admission by device
// footprint into a chunked first-fit arena, set-up of new solves on a private
// stream, epochs of batched steps on the serving stream, completion events and
// result hand-off that never waits for running epochs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lbvp.h"
#include "lbvp_internal.h"

using namespace lbvp;

namespace {

constexpr size_t ARENA_ALIGN = 256;
constexpr size_t DEFAULT_CHUNK = size_t(1) << 30;
constexpr int32_t MAX_SLOTS = 65536;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Device memory in chunks reserved on demand, each split first-fit; a freed
// range merges with free neighbours. Chunks go back only when the pool is
// destroyed, so no hipFree (which waits for the whole device) runs between
// epochs.
class Arena {
  public:
    Arena() = default;
    Arena(const Arena&) = delete;
    Arena& operator=(const Arena&) = delete;
    ~Arena()
    {
        for (Chunk& c : chunks_) (void)hipFree(c.base);
    }

    lbvp_status alloc(size_t n, size_t cap, size_t chunk, char** out, std::string& err)
    {
        n = round_up(n, ARENA_ALIGN);
        for (Chunk& c : chunks_)
            if (take(c, n, out)) return LBVP_OK;
        if (reserved_ + n > cap) {
            err = "no free range large enough and the cap allows no further chunk";
            return LBVP_E_NOMEM;
        }
        const size_t size = std::max(n, std::min(round_up(chunk, ARENA_ALIGN), cap - reserved_) / ARENA_ALIGN * ARENA_ALIGN);
        void* m = nullptr;
        const hipError_t e = hipMalloc(&m, size);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            err = std::string("hipMalloc of a pool chunk: ") + hipGetErrorString(e);
            return LBVP_E_NOMEM;
        }
        chunks_.push_back(Chunk{static_cast<char*>(m), size, {}});
        chunks_.back().free.emplace(0, size);
        reserved_ += size;
        take(chunks_.back(), n, out);
        return LBVP_OK;
    }

    void release(char* p, size_t n)
    {
        n = round_up(n, ARENA_ALIGN);
        for (Chunk& c : chunks_) {
            if (p < c.base || p >= c.base + c.size) continue;
            size_t off = (size_t)(p - c.base), len = n;
            auto next = c.free.lower_bound(off);
            if (next != c.free.end() && off + len == next->first) {
                len += next->second;
                next = c.free.erase(next);
            }
            if (next != c.free.begin()) {
                auto prev = std::prev(next);
                if (prev->first + prev->second == off) {
                    prev->second += len;
                    return;
                }
            }
            c.free.emplace(off, len);
            return;
        }
    }

    size_t reserved() const { return reserved_; }

  private:
    struct Chunk {
        char* base;
        size_t size;
        std::map<size_t, size_t> free;   // offset -> length
    };
    static bool take(Chunk& c, size_t n, char** out)
    {
        for (auto it = c.free.begin(); it != c.free.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            c.free.erase(it);
            if (len > n) c.free.emplace(off + n, len - n);
            *out = c.base + off;
            return true;
        }
        return false;
    }
    std::vector<Chunk> chunks_;
    size_t reserved_ = 0;
};

enum class State { FREE, WAITING, RUNNING, FINISHED, DONE };

struct Solve {
    State state = State::FREE;
    lbvp_ctx* ctx = nullptr;
    char* mem = nullptr;
    size_t bytes = 0;
    int64_t remaining = 0;
    int64_t nodes = 0;
    uint64_t id = 0;                 // admission number: tells reused slots apart
    hipEvent_t done_ev = nullptr;    // recorded after the solve's last step
    bool reported = false;
};

thread_local std::string g_pool_error;

}  // namespace

struct lbvp_pool {
    lbvp_pool_config cfg{};
    hipStream_t stream = nullptr;    // borrowed: epochs
    hipStream_t admin = nullptr;     // owned: set-up and result copies
    Arena arena;
    std::vector<Solve> slots;
    std::vector<int32_t> free_slots;
    lbvp_batch* batch = nullptr;
    std::vector<uint64_t> batch_ids; // admission numbers of the batch's members, in order
    std::deque<hipEvent_t> in_flight;
    std::vector<hipEvent_t> spare;
    size_t used = 0;
    uint64_t next_id = 1;
    int64_t epochs = 0, node_updates = 0;
    std::string err;

    lbvp_status fail(lbvp_status st, const std::string& m)
    {
        err = m;
        return st;
    }
    lbvp_status hip_fail(hipError_t e, const char* what)
    {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LBVP_E_DEVICE;
    }
    hipError_t event(hipEvent_t* ev)
    {
        if (!spare.empty()) {
            *ev = spare.back();
            spare.pop_back();
            return hipSuccess;
        }
        return hipEventCreateWithFlags(ev, hipEventDisableTiming);
    }
    ~lbvp_pool()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        if (admin) (void)hipStreamSynchronize(admin);
        if (batch) lbvp_batch_destroy(batch);
        for (Solve& s : slots) {
            if (s.ctx) {
                ctx_rebind_stream(s.ctx, admin);
                lbvp_destroy(s.ctx);
            }
            if (s.done_ev) (void)hipEventDestroy(s.done_ev);
        }
        for (hipEvent_t e : in_flight) (void)hipEventDestroy(e);
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
        if (admin) (void)hipStreamDestroy(admin);
    }
};

namespace {

bool valid_slot(const lbvp_pool* p, int32_t slot)
{
    return slot >= 0 && slot < (int32_t)p->slots.size();
}

// All steps of a solve are enqueued: note the point on the stream where it completes.
lbvp_status mark_finished(lbvp_pool* p, Solve& s)
{
    hipEvent_t ev = nullptr;
    hipError_t e = p->event(&ev);
    if (e == hipSuccess) e = hipEventRecord(ev, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "recording a completion event");
    s.done_ev = ev;
    s.state = State::FINISHED;
    return LBVP_OK;
}

// Finished solves whose last step has run become DONE; their contexts move to
// the private stream so that result copies never wait for later epochs.
lbvp_status collect(lbvp_pool* p)
{
    for (Solve& s : p->slots) {
        if (s.state != State::FINISHED) continue;
        const hipError_t e = hipEventQuery(s.done_ev);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return p->hip_fail(e, "hipEventQuery");
        p->spare.push_back(s.done_ev);
        s.done_ev = nullptr;
        ctx_rebind_stream(s.ctx, p->admin);
        s.state = State::DONE;
    }
    return LBVP_OK;
}

}  // namespace

extern "C" {

lbvp_status lbvp_pool_create(const lbvp_pool_config* cfg, void* hip_stream, lbvp_pool** out)
{
    if (!cfg || !out) {
        g_pool_error = "cfg and out are required";
        return LBVP_E_ARG;
    }
    *out = nullptr;
    lbvp_pool_config c = *cfg;
    const int vw = vector_width(c.storage);
    const bool two_byte_aa = (c.layout_flags & LBVP_LAYOUT_AA) && (c.storage == LBVP_F16_DEV || c.storage == LBVP_BF16_DEV);
    std::string why;
    if (!hip_stream) why = "the pool needs a stream other than the null stream";
    else if (c.cap_bytes == 0) why = "cap_bytes must be > 0";
    else if (c.max_slots < 1 || c.max_slots > MAX_SLOTS) why = "max_slots must be in 1..65536";
    else if (c.storage < LBVP_F64 || c.storage > LBVP_BF16_DEV) why = "unknown storage type";
    else if (c.layout_flags & ~LBVP_LAYOUT_AA) why = "layout_flags must be 0 or LBVP_LAYOUT_AA";
    else if (c.max_in_flight < 0) why = "max_in_flight must be >= 0";
    else if (c.block != 0 && c.block != 64 && c.block != 128 && c.block != 256) why = "block must be 0, 64, 128 or 256";
    if (why.empty()) {
        if (c.vec == 0) c.vec = two_byte_aa ? 1 : vw;
        if (c.block == 0) c.block = 256;
        const bool two_byte = c.storage == LBVP_F16_DEV || c.storage == LBVP_BF16_DEV;
        const bool ok = c.vec == 1 || (!two_byte_aa && (c.vec == vw || (two_byte && c.vec == 4)));
        if (!ok) why = "vec must be 1, the storage type's vector width or, for 2-byte storage, 4";
    }
    if (!why.empty()) {
        g_pool_error = why;
        return LBVP_E_ARG;
    }
    if (c.chunk_bytes == 0) c.chunk_bytes = DEFAULT_CHUNK;
    if (c.max_in_flight == 0) c.max_in_flight = 2;
    lbvp_pool* p = new (std::nothrow) lbvp_pool();
    if (!p) {
        g_pool_error = "host allocation failed";
        return LBVP_E_NOMEM;
    }
    p->cfg = c;
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->slots.resize((size_t)c.max_slots);
    for (int32_t i = c.max_slots - 1; i >= 0; --i) p->free_slots.push_back(i);
    hipError_t e = hipStreamCreateWithFlags(&p->admin, hipStreamNonBlocking);
    if (e != hipSuccess) {
        g_pool_error = std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e);
        p->admin = nullptr;
        delete p;
        return LBVP_E_DEVICE;
    }
    if (batch_new(p->stream, c.storage, c.layout_flags, 1, c.vec, c.block, &p->batch) != LBVP_OK) {
        g_pool_error = "host allocation failed";
        delete p;
        return LBVP_E_NOMEM;
    }
    *out = p;
    return LBVP_OK;
}

lbvp_status lbvp_pool_admit(lbvp_pool* p, const lbvp_params* prm, const uint8_t* body_id, int32_t n_bodies,
                            const lbvp_body* bodies, const double* rho, const double* ux, const double* uy,
                            int64_t n_steps, int32_t* slot)
{
    if (!p) return LBVP_E_ARG;
    if (!prm || !slot) return p->fail(LBVP_E_ARG, "params and slot are required");
    if (n_steps < 1) return p->fail(LBVP_E_ARG, "n_steps must be >= 1");
    if (n_steps > (int64_t(1) << 26)) return p->fail(LBVP_E_ARG, "n_steps larger than the force ring allows");
    if (prm->storage != p->cfg.storage || (prm->flags & LBVP_LAYOUT_AA) != p->cfg.layout_flags)
        return p->fail(LBVP_E_ARG, "the solve's storage and layout must be the pool's");
    if (prm->bc_west == LBVP_BC_NEIGHBOR || prm->bc_east == LBVP_BC_NEIGHBOR)
        return p->fail(LBVP_E_ARG, "a slab of a decomposed domain needs its halo exchanges: step it outside the pool");
    if (n_bodies < 0 || n_bodies > 255) return p->fail(LBVP_E_ARG, "n_bodies must be in 0..255");
    if (p->free_slots.empty()) return p->fail(LBVP_E_BUSY, "no free slot");
    lbvp_params q = *prm;
    q.force_every = 1;
    q.force_capacity = n_steps + 1;
    q.max_bodies = std::max(1, n_bodies);
    const size_t fp = lbvp_footprint_bytes(&q);
    if (fp == 0) return p->fail(LBVP_E_ARG, "invalid solve parameters");
    const size_t bytes = round_up(fp, ARENA_ALIGN);
    if (p->used + bytes > p->cfg.cap_bytes) return p->fail(LBVP_E_NOMEM, "the footprint does not fit under the cap now");
    char* mem = nullptr;
    std::string why;
    lbvp_status st = p->arena.alloc(bytes, p->cfg.cap_bytes, p->cfg.chunk_bytes, &mem, why);
    if (st != LBVP_OK) return p->fail(st, why);
    lbvp_ctx* c = nullptr;
    st = lbvp_create(&q, p->admin, mem, bytes, &c);
    if (st != LBVP_OK) {
        p->arena.release(mem, bytes);
        return p->fail(st, std::string("creating the solve: ") + lbvp_last_error(nullptr));
    }
    st = lbvp_set_launch(c, p->cfg.vec, p->cfg.block);
    if (st == LBVP_OK) st = lbvp_set_mask(c, body_id, n_bodies, bodies);
    if (st == LBVP_OK) st = lbvp_init_equilibrium(c, rho, ux, uy);   // waits for the private stream
    if (st != LBVP_OK) {
        const std::string m = lbvp_last_error(c);
        lbvp_destroy(c);
        p->arena.release(mem, bytes);
        return p->fail(st, "setting up the solve: " + m);
    }
    ctx_rebind_stream(c, p->stream);
    const int32_t k = p->free_slots.back();
    p->free_slots.pop_back();
    Solve& s = p->slots[(size_t)k];
    s.state = State::WAITING;
    s.ctx = c;
    s.mem = mem;
    s.bytes = bytes;
    s.remaining = n_steps;
    s.nodes = (int64_t)prm->nx * prm->ny;
    s.id = p->next_id++;
    s.reported = false;
    p->used += bytes;
    *slot = k;
    return LBVP_OK;
}

lbvp_status lbvp_pool_run_epoch(lbvp_pool* p, int64_t max_steps, int64_t* steps_run)
{
    if (!p) return LBVP_E_ARG;
    if (max_steps < 1 || !steps_run) return p->fail(LBVP_E_ARG, "max_steps >= 1 and steps_run are required");
    *steps_run = 0;
    const bool aa = (p->cfg.layout_flags & LBVP_LAYOUT_AA) != 0;
    std::vector<int32_t> run;
    bool any = false;
    for (int32_t i = 0; i < (int32_t)p->slots.size(); ++i) {
        Solve& s = p->slots[(size_t)i];
        if (s.state != State::WAITING && s.state != State::RUNNING) continue;
        if (aa && s.remaining == 1) {   // an odd last step runs alone: batched AA epochs are even
            const lbvp_status st = lbvp_step(s.ctx, 1, LBVP_KEEP_FIELDS);
            if (st != LBVP_OK) return p->fail(st, std::string("last step of a solve: ") + lbvp_last_error(s.ctx));
            s.remaining = 0;
            p->node_updates += s.nodes;
            const lbvp_status f = mark_finished(p, s);
            if (f != LBVP_OK) return f;
            any = true;
            *steps_run = 1;
            continue;
        }
        run.push_back(i);
    }
    if (!run.empty()) {
        int64_t e = aa ? std::max<int64_t>(2, max_steps & ~int64_t(1)) : max_steps;
        for (int32_t i : run) {
            const int64_t r = p->slots[(size_t)i].remaining;
            e = std::min(e, aa ? (r & ~int64_t(1)) : r);
        }
        std::vector<uint64_t> ids;
        std::vector<lbvp_ctx*> ctxs;
        bool keep = false;
        int64_t nodes = 0;
        for (int32_t i : run) {
            const Solve& s = p->slots[(size_t)i];
            ids.push_back(s.id);
            ctxs.push_back(s.ctx);
            keep = keep || s.remaining == e;
            nodes += s.nodes;
        }
        if (ids != p->batch_ids) {
            const lbvp_status st = batch_set_members(p->batch, ctxs.data(), (int32_t)ctxs.size());
            if (st != LBVP_OK) {
                p->batch_ids.clear();
                return p->fail(st, std::string("batch members: ") + lbvp_batch_last_error(p->batch));
            }
            p->batch_ids = ids;
        }
        const lbvp_status st = lbvp_batch_step(p->batch, e, keep ? LBVP_KEEP_FIELDS : 0);
        if (st != LBVP_OK) return p->fail(st, std::string("epoch: ") + lbvp_batch_last_error(p->batch));
        for (int32_t i : run) {
            Solve& s = p->slots[(size_t)i];
            s.state = State::RUNNING;
            s.remaining -= e;
            if (s.remaining == 0) {
                const lbvp_status f = mark_finished(p, s);
                if (f != LBVP_OK) return f;
            }
        }
        p->node_updates += e * nodes;
        *steps_run = e;
        any = true;
    }
    if (!any) return LBVP_OK;
    p->epochs += 1;
    hipEvent_t ev = nullptr;
    hipError_t he = p->event(&ev);
    if (he == hipSuccess) he = hipEventRecord(ev, p->stream);
    if (he != hipSuccess) return p->hip_fail(he, "recording an epoch event");
    p->in_flight.push_back(ev);
    while ((int32_t)p->in_flight.size() > p->cfg.max_in_flight) {
        he = hipEventSynchronize(p->in_flight.front());
        if (he != hipSuccess) return p->hip_fail(he, "waiting for an epoch");
        p->spare.push_back(p->in_flight.front());
        p->in_flight.pop_front();
    }
    return LBVP_OK;
}

lbvp_status lbvp_pool_poll(lbvp_pool* p, int32_t wait, int32_t* slots, int32_t cap, int32_t* n_done)
{
    if (!p) return LBVP_E_ARG;
    if (!n_done || cap < 0 || (cap > 0 && !slots)) return p->fail(LBVP_E_ARG, "slots[cap] and n_done are required");
    *n_done = 0;
    lbvp_status st = collect(p);
    if (st != LBVP_OK) return st;
    auto report = [&]() {
        for (int32_t i = 0; i < (int32_t)p->slots.size() && *n_done < cap; ++i) {
            Solve& s = p->slots[(size_t)i];
            if (s.state == State::DONE && !s.reported) {
                s.reported = true;
                slots[(*n_done)++] = i;
            }
        }
    };
    report();
    if (wait && *n_done == 0 && cap > 0) {
        for (Solve& s : p->slots)
            if (s.state == State::FINISHED) {
                const hipError_t e = hipEventSynchronize(s.done_ev);
                if (e != hipSuccess) return p->hip_fail(e, "waiting for a solve");
                break;
            }
        st = collect(p);
        if (st != LBVP_OK) return st;
        report();
    }
    return LBVP_OK;
}

lbvp_status lbvp_pool_forces(lbvp_pool* p, int32_t slot, double* out, double* mass, int64_t cap, int64_t* n_out,
                             int64_t* first_step)
{
    if (!p) return LBVP_E_ARG;
    if (!valid_slot(p, slot)) return p->fail(LBVP_E_ARG, "no such slot");
    Solve& s = p->slots[(size_t)slot];
    if (s.state != State::DONE) return p->fail(LBVP_E_STATE, "the solve is not complete (poll first)");
    const lbvp_status st = lbvp_forces(s.ctx, out, mass, cap, n_out, first_step);
    if (st != LBVP_OK) return p->fail(st, lbvp_last_error(s.ctx));
    return LBVP_OK;
}

lbvp_status lbvp_pool_read_fields(lbvp_pool* p, int32_t slot, double* rho, double* ux, double* uy, double* fx,
                                  double* fy)
{
    if (!p) return LBVP_E_ARG;
    if (!valid_slot(p, slot)) return p->fail(LBVP_E_ARG, "no such slot");
    Solve& s = p->slots[(size_t)slot];
    if (s.state != State::DONE) return p->fail(LBVP_E_STATE, "the solve is not complete (poll first)");
    const lbvp_status st = lbvp_read_fields(s.ctx, rho, ux, uy, fx, fy);
    if (st != LBVP_OK) return p->fail(st, lbvp_last_error(s.ctx));
    return LBVP_OK;
}

lbvp_status lbvp_pool_release(lbvp_pool* p, int32_t slot)
{
    if (!p) return LBVP_E_ARG;
    if (!valid_slot(p, slot)) return p->fail(LBVP_E_ARG, "no such slot");
    Solve& s = p->slots[(size_t)slot];
    if (s.state != State::DONE && s.state != State::WAITING)
        return p->fail(LBVP_E_STATE, "only a complete or not yet started solve can be released");
    ctx_rebind_stream(s.ctx, p->admin);   // a waiting solve has no work on the serving stream
    const lbvp_status st = lbvp_destroy(s.ctx);
    p->arena.release(s.mem, s.bytes);
    p->used -= s.bytes;
    s = Solve{};
    p->free_slots.push_back(slot);
    if (st != LBVP_OK) return p->fail(st, "destroying the solve's context");
    return LBVP_OK;
}

lbvp_status lbvp_pool_get_stats(const lbvp_pool* p, lbvp_pool_stats* out)
{
    if (!p || !out) return LBVP_E_ARG;
    lbvp_pool_stats r{};
    for (const Solve& s : p->slots) {
        if (s.state == State::WAITING) r.waiting += 1;
        else if (s.state == State::RUNNING) r.running += 1;
        else if (s.state == State::FINISHED) r.finished += 1;
        else if (s.state == State::DONE) r.done += 1;
    }
    r.free_slots = (int32_t)p->free_slots.size();
    r.used_bytes = p->used;
    r.reserved_bytes = p->arena.reserved();
    r.epochs = p->epochs;
    r.node_updates = p->node_updates;
    *out = r;
    return LBVP_OK;
}

lbvp_status lbvp_pool_destroy(lbvp_pool* p)
{
    if (!p) return LBVP_OK;
    lbvp_status st = LBVP_OK;
    if (hipStreamSynchronize(p->stream) != hipSuccess) st = LBVP_E_DEVICE;
    delete p;
    return st;
}

const char* lbvp_pool_last_error(const lbvp_pool* p)
{
    return p ? p->err.c_str() : g_pool_error.c_str();
}

}  // extern "C"
