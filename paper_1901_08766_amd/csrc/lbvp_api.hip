// lbvp_api.hip -- host side of the C ABI declared in include/lbvp.h.
//
// A context owns (or borrows) one device arena holding, in order: the two
// population lattices, the mask, the body table, the field planes, the force
// and mass reduction partials and their index tables, the force ring and a
// staging area for host<->device conversions. Every launch goes to the
// context's stream; only lbvp_forces / lbvp_read_* / lbvp_synchronize wait.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "lbvp.h"
#include "lbvp_graph.h"
#include "lbvp_internal.h"

using namespace lbvp;
using lbvp_host::GraphCache;
using lbvp_host::GraphKey;

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t STAGE_MIN_BYTES = size_t(16) << 20;
constexpr int64_t DEFAULT_CAPACITY = 16384;
constexpr int32_t DEFAULT_MAX_BODIES = 8;
constexpr int32_t MAX_BODIES = 255;
constexpr uint32_t KNOWN_PARAM_FLAGS = LBVP_LAYOUT_AA | LBVP_MOVING_BODIES;
constexpr uint32_t KNOWN_STEP_FLAGS = LBVP_KEEP_FIELDS | LBVP_GRAPH;
constexpr int64_t GRAPH_CHUNK = 512;   // steps per captured graph; longer calls replay it
static_assert(GRAPH_CHUNK <= POSE_ROWS, "a captured chunk reads one pose table");

thread_local std::string g_create_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t storage_bytes(int32_t st) { return st == LBVP_F64 ? 8 : st == LBVP_F32 ? 4 : 2; }
size_t arith_bytes(int32_t st) { return st == LBVP_F64 ? 8 : 4; }

// Device arena layout. Tile tables are sized for the finest tiling any launch
// configuration uses (one node per thread, 64-thread blocks).
struct Layout {
    int64_t pitch = 0, plane = 0, lstride = 0, plane_f = 0;
    int32_t max_tiles = 0, max_waves = 0;
    int64_t slot_cap = 0, capacity = 0;
    int32_t max_bodies = 0;
    int64_t stage_rows = 0;
    size_t lat[2] = {0, 0}, mask = 0, bodies = 0, fields = 0, mass_part = 0, slot_force = 0,
           tile_slot_ptr = 0, slot_body = 0, body_slot_ptr = 0, body_slots = 0, ring_force = 0,
           ring_mass = 0, rec_count = 0, stage = 0, ghost_w = 0, ghost_e = 0, pose = 0, pose_base = 0, total = 0;
};

// Launch configuration of the step kernel and the tiling it implies.
struct Launch {
    int32_t vec = 1, block = MAX_BLOCK, tile_w = MAX_BLOCK, tile_rows = 1;
    int32_t tiles_x = 0, n_tiles = 0, tiles_per_xcd = 0;
    int32_t band = 0;   // block -> tile order: 0 = one eighth per XCD, else bands of `band` tiles
};

// band_log2 of the kernel arguments: -1 for eighths, else log2(band).
int32_t band_log2(int32_t band)
{
    int32_t k = -1;
    while (band > 0) {
        band >>= 1;
        ++k;
    }
    return k;
}

bool band_allowed(int32_t band) { return band >= 0 && band <= MAX_TILE_BAND && (band & (band - 1)) == 0; }

int32_t pow2_ceil(int32_t v)
{
    int32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// A tile is tile_rows rows of tile_w nodes, vec * block nodes in all: full rows
// of vec * block nodes on wide grids, several shorter rows on narrow ones.
Launch make_launch(int32_t nx, int32_t ny, int32_t vec, int32_t block)
{
    Launch l;
    l.vec = vec;
    l.block = block;
    l.tile_w = std::min(vec * block, std::max(vec, pow2_ceil(nx)));
    l.tile_rows = vec * block / l.tile_w;
    l.tiles_x = (nx + l.tile_w - 1) / l.tile_w;
    l.n_tiles = l.tiles_x * ((ny + l.tile_rows - 1) / l.tile_rows);
    l.tiles_per_xcd = (l.n_tiles + N_XCD - 1) / N_XCD;
    return l;
}

// Vector widths a launch may use: 1 always; the 16-byte width, and for 2-byte
// storage also 4 nodes (8 bytes), except in the AA layout with 2-byte storage
// (its push step moves single elements).
std::vector<int32_t> vec_options(int32_t storage, uint32_t flags)
{
    const bool two_byte = storage == LBVP_F16_DEV || storage == LBVP_BF16_DEV;
    if (two_byte && (flags & LBVP_LAYOUT_AA)) return {1};
    if (two_byte) return {1, 4, vector_width(storage)};
    return {1, vector_width(storage)};
}

bool vec_allowed(int32_t storage, uint32_t flags, int32_t vec)
{
    for (int32_t v : vec_options(storage, flags))
        if (v == vec) return true;
    return false;
}

// Default launch: the 16-byte vector form (for 2-byte types 8 bytes if 16 are
// too many) when it still gives at least 8 wavefronts per SIMD (1024 SIMDs:
// 256 CUs x 4), else one node per thread; small grids use 64-thread blocks to
// spread over more CUs. Vector launches of the pull layout take tiles in bands
// (lbvp_set_tile_band). The shapes and bands are the fastest measured on MI355X
// for an 8192 x 4096 domain, recording every step: FP32 128 threads, bands of 8
// tiles (0.394-0.399 ms against 0.407 for 256 threads and one eighth per XCD);
// FP64 128 threads, bands of 2 (0.789-0.792 against 0.812); FP16 and BF16 256
// threads of 4 nodes (8-byte accesses), bands of 16 (FP16 0.208 ms, BF16 0.209,
// against 0.210 and 0.213 for 8 nodes in bands of 2 and 0.221 for 128 threads).
Launch default_launch(int32_t nx, int32_t ny, int32_t storage, uint32_t flags)
{
    const int64_t n = (int64_t)nx * ny;
    const bool two_byte = storage == LBVP_F16_DEV || storage == LBVP_BF16_DEV;
    int32_t vec = 1;
    for (int32_t v : {two_byte ? 4 : vector_width(storage), two_byte ? vector_width(storage) : 1})
        if (vec == 1 && v > 1 && vec_allowed(storage, flags, v) && n / (64 * v) >= 8 * 1024) vec = v;
    const int64_t waves = n / (64 * vec);
    int32_t block = two_byte ? 128 : MAX_BLOCK;
    if (waves < 4096) block = MIN_BLOCK;
    else if (vec > 1) block = two_byte ? MAX_BLOCK : 128;
    Launch l = make_launch(nx, ny, vec, block);
    if (vec > 1 && !(flags & LBVP_LAYOUT_AA)) l.band = storage == LBVP_F32 ? 8 : (two_byte && vec == 4) ? 16 : 2;
    return l;
}

// Returns an empty string if the parameters are valid.
std::string validate(const lbvp_params* p)
{
    if (!p) return "params is NULL";
    if (p->nx < 3 || p->ny < 3) return "nx and ny must be >= 3";
    if ((int64_t)p->nx * p->ny > (int64_t(1) << 34)) return "grid too large";
    if (!std::isfinite(p->tau_plus) || !(p->tau_plus > 0.5)) return "tau_plus must be finite and > 1/2";
    if (!std::isfinite(p->magic_lambda) || !(p->magic_lambda > 0.0)) return "magic_lambda must be finite and > 0";
    if (!std::isfinite(p->eta) || !(p->eta > 0.0)) return "eta must be finite and > 0";
    if (!std::isfinite(p->rho0) || !(p->rho0 > 0.0)) return "rho0 must be finite and > 0";
    const double vals[] = {p->rho_in, p->u_in[0], p->u_in[1], p->body_force[0], p->body_force[1]};
    for (double v : vals)
        if (!std::isfinite(v)) return "non-finite inflow state or body force";
    auto side_ok = [](int32_t s) {
        return s == LBVP_BC_PERIODIC || s == LBVP_BC_INFLOW_EQ || s == LBVP_BC_OUTFLOW_ZERO_GRAD || s == LBVP_BC_NEIGHBOR;
    };
    if (!side_ok(p->bc_west) || !side_ok(p->bc_east)) return "unknown x side";
    const bool cut = p->bc_west == LBVP_BC_NEIGHBOR || p->bc_east == LBVP_BC_NEIGHBOR;
    if (cut && (p->flags & (LBVP_LAYOUT_AA | LBVP_MOVING_BODIES)))
        return "LBVP_BC_NEIGHBOR sides need the two-lattice layout and a fixed mask";
    if ((p->bc_west == LBVP_BC_PERIODIC) != (p->bc_east == LBVP_BC_PERIODIC))
        return "x sides must be both periodic or both non-periodic";
    if (p->bc_south != LBVP_BC_PERIODIC || p->bc_north != LBVP_BC_PERIODIC) return "y sides must be periodic";
    if (p->storage < LBVP_F64 || p->storage > LBVP_BF16_DEV) return "unknown storage type";
    if (p->force_every < 0) return "force_every must be >= 0";
    if (p->force_capacity < 0 || p->force_capacity > (int64_t(1) << 26)) return "force_capacity out of range";
    if (p->max_bodies < 0 || p->max_bodies > MAX_BODIES) return "max_bodies must be in 0..255";
    if (p->flags & ~KNOWN_PARAM_FLAGS) return "unknown or unsupported params flag";
    if ((p->flags & LBVP_MOVING_BODIES) && p->max_bodies > MAX_MOVING)
        return "moving bodies: max_bodies must be at most 8";
    return "";
}

Layout make_layout(const lbvp_params* p)
{
    Layout L;
    const size_t es = storage_bytes(p->storage), rs = arith_bytes(p->storage);
    // a cut side keeps its halo column in the lattice's padding: room for two
    const bool cut = p->bc_west == LBVP_BC_NEIGHBOR || p->bc_east == LBVP_BC_NEIGHBOR;
    L.pitch = (int64_t)align_up((size_t)p->nx + (cut ? 2 : 0), 64);
    L.plane = L.pitch;          // population rows of a lattice row back to back
    L.lstride = 9 * L.pitch;
    L.plane_f = (int64_t)p->ny * L.pitch;
    for (int vec : vec_options(p->storage, p->flags))
        for (int block : {64, 128, 256}) {
            const Launch l = make_launch(p->nx, p->ny, vec, block);
            L.max_tiles = std::max(L.max_tiles, l.n_tiles);
            L.max_waves = std::max(L.max_waves, l.n_tiles * (block / 64));
        }
    L.capacity = p->force_capacity > 0 ? p->force_capacity : DEFAULT_CAPACITY;
    L.max_bodies = p->max_bodies > 0 ? p->max_bodies : DEFAULT_MAX_BODIES;
    L.slot_cap = 2 * (int64_t)L.max_tiles + 1024;
    if (p->flags & LBVP_MOVING_BODIES)   // a slot for every (tile, body): bodies can reach any tile
        L.slot_cap = std::max<int64_t>(L.slot_cap, (int64_t)L.max_tiles * L.max_bodies);
    const size_t row_bytes = (size_t)p->nx * 9 * sizeof(double);
    const size_t stage_bytes = std::max(STAGE_MIN_BYTES, row_bytes);
    L.stage_rows = std::max<int64_t>(1, (int64_t)(stage_bytes / row_bytes));
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, ALIGN); return at; };
    const size_t lat_bytes = (size_t)p->ny * (size_t)L.lstride * es;
    const bool aa = (p->flags & LBVP_LAYOUT_AA) != 0;
    L.lat[0] = take(lat_bytes);
    L.lat[1] = aa ? L.lat[0] : take(lat_bytes);   // the AA pattern streams in place
    L.mask = take((size_t)p->ny * L.pitch);
    L.bodies = take((size_t)(L.max_bodies + 1) * BODY_STRIDE * rs);
    L.fields = take(5 * (size_t)L.plane_f * rs);
    L.mass_part = take(2 * (size_t)L.max_waves * sizeof(double));          // double-buffered
    L.slot_force = take(2 * (size_t)L.slot_cap * 2 * sizeof(double));
    L.tile_slot_ptr = take((size_t)(L.max_tiles + 1) * sizeof(int32_t));
    L.slot_body = take((size_t)L.slot_cap * sizeof(int32_t));
    L.body_slot_ptr = take((size_t)(MAX_BODIES + 2) * sizeof(int32_t));
    L.body_slots = take((size_t)L.slot_cap * sizeof(int32_t));
    L.ring_force = take((size_t)L.capacity * L.max_bodies * 2 * sizeof(double));
    L.ring_mass = take((size_t)L.capacity * sizeof(double));
    L.rec_count = take(sizeof(int64_t));
    L.ghost_w = take(3 * (size_t)p->ny * es);
    L.ghost_e = take(3 * (size_t)p->ny * es);
    L.stage = take(stage_bytes);
    L.pose = take((p->flags & LBVP_MOVING_BODIES) ? (size_t)POSE_ROWS * MAX_MOVING * POSE_STRIDE * sizeof(double) : 0);
    L.pose_base = take((p->flags & LBVP_MOVING_BODIES) ? sizeof(int64_t) : 0);
    L.total = o;
    return L;
}

// Pinned host buffers for uploads that must not wait for the stream: a
// pageable source would make hipMemcpyAsync wait for the copy. A buffer is
// reused once the event recorded after its copy has fired.
class PinnedRing {
  public:
    PinnedRing() = default;
    PinnedRing(const PinnedRing&) = delete;
    PinnedRing& operator=(const PinnedRing&) = delete;
    ~PinnedRing()
    {
        for (Slot& x : s_) {
            if (x.ev) {
                (void)hipEventSynchronize(x.ev);
                (void)hipEventDestroy(x.ev);
            }
            if (x.p) (void)hipHostFree(x.p);
        }
    }
    hipError_t upload(void* dst, const void* src, size_t n, hipStream_t st)
    {
        Slot& x = s_[next_];
        next_ = (next_ + 1) % SLOTS;
        hipError_t e = hipSuccess;
        if (!x.ev) e = hipEventCreateWithFlags(&x.ev, hipEventDisableTiming);
        else e = hipEventSynchronize(x.ev);
        if (e != hipSuccess) return e;
        if (x.cap < n) {
            if (x.p) (void)hipHostFree(x.p);
            x.p = nullptr;
            x.cap = 0;
            const size_t want = std::max(n, size_t(64) << 10);
            void* m = nullptr;
            e = hipHostMalloc(&m, want, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            x.p = static_cast<char*>(m);
            x.cap = want;
        }
        std::memcpy(x.p, src, n);
        e = hipMemcpyAsync(dst, x.p, n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(x.ev, st);
        return e;
    }

  private:
    static constexpr int SLOTS = 4;
    struct Slot {
        char* p = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
    };
    Slot s_[SLOTS];
    int next_ = 0;
};

}  // namespace

struct lbvp_ctx {
    lbvp_params p{};
    Layout L;
    hipStream_t stream = nullptr;
    char* mem = nullptr;
    bool owns = false;
    int cur = 0;                // lattice holding the current post-collision state
    int64_t step = 0;
    int64_t rec_head = 0, rec_tail = 0;
    bool pending = false;       // a recorded step whose sums are not yet in the ring
    int32_t pending_buf = 0;
    bool fields_valid = false;
    int32_t n_bodies = 0;
    double tau_minus = 0.0;
    Launch launch;
    std::vector<uint8_t> mask_host;         // [ny][nx], kept to rebuild the tile tables
    std::vector<lbvp_body> bodies_host;
    std::vector<double> mov_r2;             // moving bodies: squared reach about the centre
    // moving bodies: each body's mask rows as (row, first column, last column),
    // the span between its first and last node of the row
    std::vector<std::vector<std::array<int32_t, 3>>> mov_runs;
    std::vector<double> pose_host;          // moving bodies: the uploaded pose table
    int64_t pose_first = -1;                // its first time level (-1: none)
    uint64_t gen = 0;                       // kernel-argument generation (graph keys)
    GraphCache graphs;
    StepArgs<double> a64{};
    StepArgs<float> a32{};
    FinalizeArgs fin{};
    std::string err;

    template <typename T> T* at(size_t off) { return reinterpret_cast<T*>(mem + off); }
    bool aa() const { return (p.flags & LBVP_LAYOUT_AA) != 0; }
    bool moving() const { return (p.flags & LBVP_MOVING_BODIES) != 0; }
    int32_t storage() const { return p.storage; }
    bool is_f64() const { return p.storage == LBVP_F64; }
    size_t esize() const { return storage_bytes(p.storage); }
    size_t rsize() const { return arith_bytes(p.storage); }

    lbvp_status fail(lbvp_status s, const std::string& m) { err = m; return s; }
    lbvp_status hip_fail(hipError_t e, const char* what)
    {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LBVP_E_DEVICE;
    }
};

namespace {

#define LBVP_HIP(ctx, call)                                               \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) return (ctx)->hip_fail(e_, #call);          \
    } while (0)

// The inflow ghost populations (f^eq(rho_in, u_in) - w rho0) / w (eq. feq), in FP64.
void inflow_ghost(const lbvp_params& p, double out[9])
{
    static const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double r = p.rho_in, ux = p.u_in[0], uy = p.u_in[1], uu = ux * ux + uy * uy;
    for (int q = 0; q < 9; ++q) {
        const double eu = ex[q] * ux + ey[q] * uy;
        out[q] = (r - p.rho0) + r * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

template <typename R>
void fill_step_args(lbvp_ctx* c, StepArgs<R>& a)
{
    const lbvp_params& p = c->p;
    const Layout& L = c->L;
    const Launch& l = c->launch;
    a.nx = p.nx;
    a.ny = p.ny;
    a.vec = l.vec;
    a.block = l.block;
    a.tile_w = l.tile_w;
    a.tile_rows = l.tile_rows;
    a.tiles_x = l.tiles_x;
    a.n_tiles = l.n_tiles;
    a.tiles_per_xcd = l.tiles_per_xcd;
    a.band_log2 = band_log2(l.band);
    a.west = p.bc_west;
    a.east = p.bc_east;
    a.pitch = L.pitch;
    a.plane = L.plane;
    a.lstride = L.lstride;
    a.plane_f = L.plane_f;
    a.off32 = (uint64_t)p.ny * (uint64_t)L.lstride * storage_bytes(p.storage) <= 0xFFFFFFFFull ? 1 : 0;
    a.rho0 = (R)p.rho0;
    a.om_p = (R)(1.0 / p.tau_plus);
    a.om_m = (R)(1.0 / c->tau_minus);
    a.k_p = (R)(1.0 - 0.5 / p.tau_plus);
    a.k_m = (R)(1.0 - 0.5 / c->tau_minus);
    a.vp_c = (R)(1.0 / (2.0 * p.eta + 1.0));
    {
        const double om_p = 1.0 / p.tau_plus, om_m = 1.0 / c->tau_minus;
        const double k_p = 1.0 - 0.5 / p.tau_plus, k_m = 1.0 - 0.5 / c->tau_minus;
        a.c1 = (R)(1.0 - 0.5 * (om_p + om_m));
        a.c2 = (R)(0.5 * (om_m - om_p));
        a.om_p1 = (R)(1.0 - om_p);
        a.om_p45 = (R)(4.5 * om_p);
        a.om_p15 = (R)(1.5 * om_p);
        a.om_m3 = (R)(3.0 * om_m);
        a.k_p9 = (R)(9.0 * k_p);
        a.k_p3 = (R)(3.0 * k_p);
        a.k_m3 = (R)(3.0 * k_m);
    }
    a.fbx = (R)p.body_force[0];
    a.fby = (R)p.body_force[1];
    a.fbx18 = (R)(18.0 * p.body_force[0]);
    a.fby18 = (R)(18.0 * p.body_force[1]);
    double fin[9];
    inflow_ghost(p, fin);
    for (int q = 0; q < 9; ++q) a.feq_in[q] = (R)fin[q];
    a.mask = c->at<uint8_t>(L.mask);
    a.bodies = c->at<R>(L.bodies);
    a.tile_slot_ptr = c->at<int32_t>(L.tile_slot_ptr);
    a.slot_body = c->at<int32_t>(L.slot_body);
    a.slot_force = c->at<double>(L.slot_force);
    a.mass_part = c->at<double>(L.mass_part);
    a.fields = c->at<R>(L.fields);
    a.part_buf = 0;
    a.fin_buf = -1;
    a.ghost_w = c->at<char>(L.ghost_w);
    a.ghost_e = c->at<char>(L.ghost_e);
    a.fin = c->fin;
    a.n_moving = c->moving() ? c->n_bodies : 0;
    a.pose_k = 0;
    a.pose_base = c->at<int64_t>(L.pose_base);
    a.pose = c->at<double>(L.pose);
}

// Moving bodies: each body's pose at time level t into a pose row (one
// rounding per operation, as the kernels and the reference evaluate it).
void moving_pose(const lbvp_ctx* c, int64_t t_level, double* row)
{
    const double t = (double)t_level;
    for (int32_t b = 0; b < c->n_bodies; ++b) {
        const lbvp_body& B = c->bodies_host[b];
        const double th = B.omega * t;
        const double vxt = B.vx * t;
        const double vyt = B.vy * t;
        double* m = row + (size_t)b * POSE_STRIDE;
        m[0] = std::cos(th);
        m[1] = std::sin(th);
        m[2] = B.cx + vxt;
        m[3] = B.cy + vyt;
        m[4] = B.cx;
        m[5] = B.cy;
        m[6] = c->mov_r2[b];
        m[7] = 0.0;
    }
}

template <typename R>
std::vector<char> body_table_bytes(const lbvp_body* bodies, int32_t n, int32_t max_bodies)
{
    std::vector<R> t((size_t)(max_bodies + 1) * BODY_STRIDE, R(0));
    for (int32_t k = 0; k < n; ++k) {
        const double cxi = std::nearbyint(bodies[k].cx), cyi = std::nearbyint(bodies[k].cy);
        const double v[BODY_STRIDE] = {cxi, cyi, bodies[k].cx - cxi, bodies[k].cy - cyi,   // exact splits
                                       bodies[k].vx, bodies[k].vy, bodies[k].omega};
        for (int q = 0; q < BODY_STRIDE; ++q) t[(size_t)(k + 1) * BODY_STRIDE + q] = (R)v[q];
    }
    std::vector<char> out(t.size() * sizeof(R));
    std::memcpy(out.data(), t.data(), out.size());
    return out;
}

// The (tile, body) reduction tables for the current tiling and mask: a slot per
// body present in each tile, numbered in tile order, and each body's slots.
// Moving bodies: with a pose window on the device (time levels pose_first ..
// pose_first + POSE_ROWS - 1), a tile lists body b when one of b's nodes can lie
// in it at one of the window's time levels; before any window, every body in
// every tile. The kernels test only the bodies a tile lists. A node x belongs to
// b at time t when R(-theta) (x - c(t)) + c0 rounds to a node y of b's mask:
// then x lies within 1/sqrt(2) of c(t) + R(theta) d, d = y - c0. Over the
// window c(t) stays in the box of its two ends, and R(theta) d within |d| |dtheta|
// of its value at the first level; the points d of one mask row's span between
// its first and last node rotate onto the segment between the rotated ends. So
// each row span, its ends rotated to the first level, boxed, widened by the
// centre's path, |d|max |dtheta|, 1/sqrt(2) and two nodes, holds every tile
// its nodes reach.
lbvp_status build_tile_tables(lbvp_ctx* c)
{
    const lbvp_params& p = c->p;
    const Layout& L = c->L;
    const Launch& l = c->launch;
    const int32_t nb = c->n_bodies;
    const uint8_t* body_id = c->mask_host.data();
    std::vector<int32_t> tile_ptr((size_t)l.n_tiles + 1, 0), slot_body;
    std::vector<std::vector<int32_t>> per_body((size_t)nb);
    std::vector<uint8_t> seen((size_t)nb + 1, 0);
    const bool windowed = c->moving() && c->pose_first >= 0;
    std::vector<uint8_t> reach;   // windowed: bit b - 1 of tile t when body b can reach t
    if (windowed) {
        reach.assign((size_t)l.n_tiles, 0);
        const int32_t tiles_y = l.n_tiles / l.tiles_x;
        const double ta = (double)c->pose_first, tb = (double)(c->pose_first + POSE_ROWS - 1);
        auto span = [](double lo, double hi, int32_t size, int32_t count, int32_t* first, int32_t* last) {
            *first = (int32_t)std::max(0.0, std::floor(lo / size));
            *last = (int32_t)std::min((double)count - 1.0, std::floor(hi / size));
        };
        for (int32_t b = 0; b < nb; ++b) {
            const lbvp_body& B = c->bodies_host[b];
            const double xa = B.cx + B.vx * ta, xb = B.cx + B.vx * tb;
            const double ya = B.cy + B.vy * ta, yb = B.cy + B.vy * tb;
            const double th = B.omega * ta, dth = std::fabs(B.omega) * (tb - ta);
            const double co = std::cos(th), si = std::sin(th);
            for (const auto& run : c->mov_runs[b]) {
                const double dy = run[0] - B.cy, dx0 = run[1] - B.cx, dx1 = run[2] - B.cx;
                const double px0 = co * dx0 - si * dy, py0 = si * dx0 + co * dy;
                const double px1 = co * dx1 - si * dy, py1 = si * dx1 + co * dy;
                const double rho = std::sqrt(std::max(dx0 * dx0, dx1 * dx1) + dy * dy);
                const double w = rho * dth + 0.7072 + 2.0;
                int32_t c0, c1, r0, r1;
                span(std::min(xa, xb) + std::min(px0, px1) - w, std::max(xa, xb) + std::max(px0, px1) + w,
                     l.tile_w, l.tiles_x, &c0, &c1);
                span(std::min(ya, yb) + std::min(py0, py1) - w, std::max(ya, yb) + std::max(py0, py1) + w,
                     l.tile_rows, tiles_y, &r0, &r1);
                for (int32_t ty = r0; ty <= r1; ++ty)
                    for (int32_t tx = c0; tx <= c1; ++tx) reach[(size_t)ty * l.tiles_x + tx] |= (uint8_t)(1u << b);
            }
        }
    }
    for (int32_t t = 0; t < l.n_tiles; ++t) {
        tile_ptr[t] = (int32_t)slot_body.size();
        if (nb == 0) continue;
        if (c->moving()) {   // in body order
            for (int32_t b = 1; b <= nb; ++b) {
                if (windowed && !((reach[t] >> (b - 1)) & 1u)) continue;
                per_body[b - 1].push_back((int32_t)slot_body.size());
                slot_body.push_back(b);
            }
            continue;
        }
        const int32_t ty = t / l.tiles_x, i0 = (t % l.tiles_x) * l.tile_w, i1 = std::min(p.nx, i0 + l.tile_w);
        const int32_t j0 = ty * l.tile_rows, j1 = std::min(p.ny, j0 + l.tile_rows);
        std::fill(seen.begin(), seen.end(), 0);
        for (int32_t j = j0; j < j1; ++j) {
            const uint8_t* row = body_id + (int64_t)j * p.nx;
            for (int32_t i = i0; i < i1; ++i) seen[row[i]] = 1;
        }
        for (int32_t b = 1; b <= nb; ++b) {
            if (!seen[b]) continue;
            if ((int64_t)slot_body.size() >= L.slot_cap) {
                (void)hipStreamSynchronize(c->stream);  // copies from the caller's host buffers
                return c->fail(LBVP_E_NOMEM, "mask has more (tile, body) pairs than the reduction tables hold");
            }
            per_body[b - 1].push_back((int32_t)slot_body.size());
            slot_body.push_back(b);
        }
    }
    tile_ptr[l.n_tiles] = (int32_t)slot_body.size();
    std::vector<int32_t> body_ptr((size_t)nb + 1, 0), body_slots;
    for (int32_t b = 0; b < nb; ++b) {
        body_ptr[b] = (int32_t)body_slots.size();
        body_slots.insert(body_slots.end(), per_body[b].begin(), per_body[b].end());
    }
    body_ptr[nb] = (int32_t)body_slots.size();
    hipStream_t s = c->stream;
    LBVP_HIP(c, hipMemcpyAsync(c->at<int32_t>(L.tile_slot_ptr), tile_ptr.data(), tile_ptr.size() * 4,
                               hipMemcpyHostToDevice, s));
    if (!slot_body.empty()) {
        LBVP_HIP(c, hipMemcpyAsync(c->at<int32_t>(L.slot_body), slot_body.data(), slot_body.size() * 4,
                                   hipMemcpyHostToDevice, s));
        LBVP_HIP(c, hipMemcpyAsync(c->at<int32_t>(L.body_slots), body_slots.data(), body_slots.size() * 4,
                                   hipMemcpyHostToDevice, s));
    }
    LBVP_HIP(c, hipMemcpyAsync(c->at<int32_t>(L.body_slot_ptr), body_ptr.data(), body_ptr.size() * 4,
                               hipMemcpyHostToDevice, s));
    LBVP_HIP(c, hipStreamSynchronize(s));  // the host tables above go out of scope
    return LBVP_OK;
}

// Adopt a launch configuration: kernel arguments, finalize arguments, tile tables.
lbvp_status apply_launch(lbvp_ctx* c, const Launch& l)
{
    c->launch = l;
    c->gen += 1;
    c->fin.n_mass = l.n_tiles * (l.block / 64);
    fill_step_args(c, c->a64);
    fill_step_args(c, c->a32);
    return build_tile_tables(c);
}

ConvArgs conv_args(lbvp_ctx* c, int32_t row0, int32_t rows)
{
    ConvArgs a{};
    a.nx = c->p.nx;
    a.rows = rows;
    a.row0 = row0;
    a.pitch = c->L.pitch;
    a.plane = c->L.plane;
    a.lstride = c->L.lstride;
    a.plane_f = c->L.plane_f;
    a.rho0 = c->p.rho0;
    a.swap = c->aa() ? 1 : 0;
    a.pops = c->at<double>(c->L.stage);
    return a;
}

lbvp_status check_ctx(const lbvp_ctx* c) { return c ? LBVP_OK : LBVP_E_ARG; }

// AA layout after an even step count: refresh the outflow ghost columns.
hipError_t refresh_aa_ghosts(lbvp_ctx* c)
{
    if (!c->aa()) return hipSuccess;
    GhostArgs g{};
    g.nx = c->p.nx;
    g.ny = c->p.ny;
    g.west_outflow = c->p.bc_west == LBVP_BC_OUTFLOW_ZERO_GRAD;
    g.east_outflow = c->p.bc_east == LBVP_BC_OUTFLOW_ZERO_GRAD;
    if (!g.west_outflow && !g.east_outflow) return hipSuccess;
    g.pitch = c->L.pitch;
    g.plane = c->L.plane;
    g.lstride = c->L.lstride;
    g.ghost_w = c->at<char>(c->L.ghost_w);
    g.ghost_e = c->at<char>(c->L.ghost_e);
    return launch_aa_ghosts(c->p.storage, c->at<char>(c->L.lat[0]), g, c->stream);
}

// The host bookkeeping that a run of steps advances.
struct CtxClock {
    int cur;
    int64_t step, rec_head;
    bool pending, fields_valid;
    int32_t pending_buf;
};

CtxClock save_clock(const lbvp_ctx* c)
{
    return CtxClock{c->cur, c->step, c->rec_head, c->pending, c->fields_valid, c->pending_buf};
}

void restore_clock(lbvp_ctx* c, const CtxClock& k)
{
    c->cur = k.cur;
    c->step = k.step;
    c->rec_head = k.rec_head;
    c->pending = k.pending;
    c->fields_valid = k.fields_valid;
    c->pending_buf = k.pending_buf;
    c->pose_first = -1;   // a failed run may have left the device pose row anywhere
}

// Moving bodies: make the device pose table hold the time levels next .. next +
// n - 1 (n <= POSE_ROWS; next is the count after the coming step). If it does
// not, the table is refilled from `next` on and the device base row reset to 0;
// either way the base row is then the coming step's (every run advances it by
// its length when it ends).
lbvp_status pose_window(lbvp_ctx* c, int64_t next, int64_t n)
{
    if (c->pose_first >= 0 && next >= c->pose_first && next + n <= c->pose_first + POSE_ROWS) return LBVP_OK;
    // the previous upload must have been read from its host buffer first
    LBVP_HIP(c, hipStreamSynchronize(c->stream));
    const size_t row = (size_t)MAX_MOVING * POSE_STRIDE;
    c->pose_host.assign(row * POSE_ROWS, 0.0);
    for (int32_t r = 0; r < POSE_ROWS; ++r) moving_pose(c, next + r, c->pose_host.data() + r * row);
    LBVP_HIP(c, hipMemcpyAsync(c->at<double>(c->L.pose), c->pose_host.data(), c->pose_host.size() * sizeof(double),
                               hipMemcpyHostToDevice, c->stream));
    LBVP_HIP(c, launch_set_i64(c->at<int64_t>(c->L.pose_base), 0, c->stream));
    c->pose_first = next;
    // the force slots of the window's reach (after the previous run's last
    // record was summed: same stream)
    const lbvp_status st = build_tile_tables(c);
    if (st != LBVP_OK) c->pose_first = -1;
    return st;
}

// n steps from the current state, one launch each, then the standalone sum of
// the last record. With launch == false only the bookkeeping advances (the
// same launches were replayed from a graph). Moving bodies: the pose table
// must hold the run's time levels (pose_window).
lbvp_status enqueue_steps(lbvp_ctx* c, int64_t n_steps, bool keep_last, bool launch)
{
    const int64_t fe = c->p.force_every;
    c->a64.fin = c->fin;
    c->a32.fin = c->fin;
    for (int64_t k = 0; k < n_steps; ++k) {
        const int64_t next = c->step + 1;
        const bool record = fe > 0 && next % fe == 0;
        const bool keep = keep_last && k == n_steps - 1;
        const int32_t part_buf = (int32_t)(c->rec_head & 1);
        if (launch) {
            const int32_t fin_buf = c->pending ? c->pending_buf : -1;
            c->a64.part_buf = c->a32.part_buf = part_buf;
            c->a64.fin_buf = c->a32.fin_buf = fin_buf;
            const void* args = c->is_f64() ? (const void*)&c->a64 : (const void*)&c->a32;
            const int32_t mode = !c->aa() ? MODE_PULL : (c->step % 2 == 0 ? MODE_AA_PUSH : MODE_AA_LOCAL);
            hipError_t e;
            if (c->moving()) {   // row *pose_base + k: the poses at the time level this step computes
                c->a64.pose_k = c->a32.pose_k = (int32_t)k;
                e = launch_step_moving(c->p.storage, mode, record, keep, c->at<char>(c->L.lat[c->cur]),
                                       c->at<char>(c->L.lat[c->cur ^ 1]), args, c->stream);
            } else {
                e = launch_step(c->p.storage, mode, record, keep, c->at<char>(c->L.lat[c->cur]),
                                c->at<char>(c->L.lat[c->cur ^ 1]), args, c->stream);
            }
            if (e != hipSuccess) return c->hip_fail(e, "step kernel launch");
        }
        c->pending = record;
        if (record) {
            c->pending_buf = part_buf;
            c->rec_head += 1;
        }
        if (keep) c->fields_valid = true;
        if (!c->aa()) c->cur ^= 1;
        c->step = next;
    }
    if (c->pending) {  // the last record of the run is summed on its own
        if (launch) {
            hipError_t e = launch_finalize(c->fin, c->pending_buf, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "finalize kernel launch");
        }
        c->pending = false;
    }
    if (launch && c->moving() && n_steps > 0) {   // the next run's first pose row
        hipError_t e = launch_pose_advance(c->at<int64_t>(c->L.pose_base), n_steps, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "pose advance launch");
    }
    return LBVP_OK;
}

}  // namespace


// A set of contexts advanced together, one launch per step over all their
// tiles. The contexts stay ordinary contexts: their forces, fields and
// populations are read through the usual calls.
struct lbvp_batch {
    std::vector<lbvp_ctx*> members;
    hipStream_t stream = nullptr;
    int32_t storage = 0, vec = 1, block = MAX_BLOCK;
    bool aa = false;
    int32_t force_every = 0;
    char* dev = nullptr;                 // owned: [step args | finalize args | tile map]
    size_t dev_cap = 0;
    size_t arg_size = 0, off_fins = 0, off_tile_domain = 0, off_tile_start = 0, bytes = 0;
    int32_t total_tiles = 0, tiles_per_xcd = 0;
    int32_t band = 0;                    // block -> tile order over the concatenated tiles (lbvp_batch_set_tile_band)
    std::vector<char> image;             // host image of the device block
    std::vector<char> uploaded;          // the image as last enqueued for upload
    PinnedRing ring;
    GraphCache graphs;
    uint64_t gen = 0;                    // bumped whenever the members or the block change
    std::vector<int32_t> halo_w, halo_e; // cuts between members (lbvp_batch_set_halo)
    std::string err;

    lbvp_status fail(lbvp_status st, const std::string& m) { err = m; return st; }
    lbvp_status hip_fail(hipError_t e, const char* what)
    {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LBVP_E_DEVICE;
    }
    ~lbvp_batch()
    {
        graphs.clear(stream);
        if (dev) {
            (void)hipStreamSynchronize(stream);
            (void)hipFree(dev);
        }
    }
};

namespace {

thread_local std::string g_batch_error;

// Some member has moving bodies: the batch runs the kernels that evaluate a
// moving mask (members with fixed masks take their mask as usual).
bool batch_moving(const lbvp_batch* b)
{
    for (const lbvp_ctx* c : b->members)
        if (c->moving()) return true;
    return false;
}

// The batch requires one step kind, one record cadence and one stream for all
// its members at every call.
std::string batch_consistency(const lbvp_batch* b, const std::vector<lbvp_ctx*>& m)
{
    if (m.empty()) return "";
    const lbvp_ctx* c0 = m[0];
    for (const lbvp_ctx* c : m) {
        if (!c) return "a member is NULL";
        if (c->p.storage != b->storage) return "members differ in storage type";
        if (c->aa() != b->aa) return "members differ in layout";
        if (c->stream != b->stream) return "members use different streams";
        if (c->p.force_every != b->force_every) return "members differ in force_every";
        if (c->aa() && (c->step % 2) != (c0->step % 2)) return "AA members must be at the same step parity";
        const int64_t fe = c->p.force_every;
        if (fe > 1 && (c->step % fe) != (c0->step % fe)) return "members must be at the same force-record phase";
        if (c->pending) return "a member has an unsummed record";
    }
    return "";
}

// The member list's tables in the host image: offsets of the argument blocks,
// the finalize arguments and the tile map, and the tile map itself. The members
// must already have the batch's launch shape. No device memory is touched.
void batch_layout(lbvp_batch* b, const std::vector<lbvp_ctx*>& m)
{
    const size_t n = m.size();
    std::vector<int32_t> tile_start(n), tile_domain;
    for (size_t d = 0; d < n; ++d) {
        tile_start[d] = (int32_t)tile_domain.size();
        tile_domain.insert(tile_domain.end(), (size_t)m[d]->launch.n_tiles, (int32_t)d);
    }
    b->arg_size = b->storage == LBVP_F64 ? sizeof(StepArgs<double>) : sizeof(StepArgs<float>);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, ALIGN); return at; };
    take(b->arg_size * std::max<size_t>(n, 1));
    b->off_fins = take(sizeof(FinalizeArgs) * std::max<size_t>(n, 1));
    b->off_tile_domain = take(std::max<size_t>(tile_domain.size(), 1) * sizeof(int32_t));
    b->off_tile_start = take(std::max<size_t>(n, 1) * sizeof(int32_t));
    b->bytes = o;
    b->image.assign(b->bytes, 0);
    b->uploaded.clear();
    std::memcpy(b->image.data() + b->off_tile_domain, tile_domain.data(), tile_domain.size() * sizeof(int32_t));
    std::memcpy(b->image.data() + b->off_tile_start, tile_start.data(), n * sizeof(int32_t));
    b->members = m;
    b->halo_w.clear();   // member indices no longer mean the same contexts
    b->halo_e.clear();
    b->total_tiles = (int32_t)tile_domain.size();
    b->tiles_per_xcd = (b->total_tiles + N_XCD - 1) / N_XCD;
}

// Adopt a member list: launch shapes, the tables in the host image and a
// device block large enough for them.
lbvp_status batch_assign(lbvp_batch* b, const std::vector<lbvp_ctx*>& m)
{
    const std::string why = batch_consistency(b, m);
    if (!why.empty()) return b->fail(LBVP_E_ARG, why);
    for (lbvp_ctx* c : m) {
        const lbvp_status st = lbvp_set_launch(c, b->vec, b->block);
        if (st != LBVP_OK) return b->fail(st, std::string("setting a member's launch shape: ") + c->err);
    }
    batch_layout(b, m);
    if (b->bytes > b->dev_cap) {   // rare: grow, after the stream has finished with the old block
        b->graphs.clear(b->stream);
        if (b->dev) {
            LBVP_HIP(b, hipStreamSynchronize(b->stream));
            LBVP_HIP(b, hipFree(b->dev));
            b->dev = nullptr;
            b->dev_cap = 0;
        }
        const size_t want = std::max(b->bytes, b->dev_cap * 2);
        void* d = nullptr;
        hipError_t e = hipMalloc(&d, want);
        if (e != hipSuccess) return b->fail(LBVP_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        b->dev = static_cast<char*>(d);
        b->dev_cap = want;
    }
    b->graphs.clear(b->stream);
    b->gen += 1;
    return LBVP_OK;
}

// The members' step and finalize arguments as of now (lattice parity, record
// tables) in the host image.
void batch_fill_args(lbvp_batch* b)
{
    for (size_t d = 0; d < b->members.size(); ++d) {
        lbvp_ctx* c = b->members[d];
        c->fin.n_bodies = c->n_bodies;
        char* dst = b->image.data() + d * b->arg_size;
        if (c->is_f64()) {
            StepArgs<double> a = c->a64;
            a.fin = c->fin;
            a.lat0 = c->at<char>(c->L.lat[0]);
            a.lat1 = c->at<char>(c->L.lat[1]);
            a.cur = c->cur;
            a.part_buf = 0;
            a.fin_buf = -1;
            std::memcpy(dst, &a, sizeof(a));
        } else {
            StepArgs<float> a = c->a32;
            a.fin = c->fin;
            a.lat0 = c->at<char>(c->L.lat[0]);
            a.lat1 = c->at<char>(c->L.lat[1]);
            a.cur = c->cur;
            a.part_buf = 0;
            a.fin_buf = -1;
            std::memcpy(dst, &a, sizeof(a));
        }
        std::memcpy(b->image.data() + b->off_fins + d * sizeof(FinalizeArgs), &c->fin, sizeof(FinalizeArgs));
    }
}

// The same, uploaded if they differ from what the device block holds.
lbvp_status batch_refresh_args(lbvp_batch* b)
{
    batch_fill_args(b);
    if (b->image == b->uploaded) return LBVP_OK;
    LBVP_HIP(b, b->ring.upload(b->dev, b->image.data(), b->bytes, b->stream));
    b->uploaded = b->image;
    return LBVP_OK;
}

// Steps k0 .. k0 + n - 1 of a call that started at step step0, one launch
// each, then the standalone sum of the run's last record. *recs counts the
// records of the call so far (its parity picks the partial buffer).
lbvp_status batch_run(lbvp_batch* b, int64_t step0, int64_t k0, int64_t n, bool keep_last, int64_t* recs)
{
    const int64_t fe = b->force_every;
    BatchLaunch L{};
    L.total_tiles = b->total_tiles;
    L.tiles_per_xcd = b->tiles_per_xcd;
    L.band_log2 = band_log2(b->band);
    L.tile_domain = reinterpret_cast<const int32_t*>(b->dev + b->off_tile_domain);
    L.tile_start = reinterpret_cast<const int32_t*>(b->dev + b->off_tile_start);
    L.args = b->dev;
    L.off32 = 1;
    for (const lbvp_ctx* c : b->members) L.off32 &= c->a32.off32;   // off32 does not depend on the precision
    bool pending = false;
    int32_t pending_buf = 0;
    for (int64_t k = k0; k < k0 + n; ++k) {
        const int64_t next = step0 + k + 1;
        const bool record = fe > 0 && next % fe == 0;
        const bool keep = keep_last && k == k0 + n - 1;
        const int32_t mode = !b->aa ? MODE_PULL : ((step0 + k) % 2 == 0 ? MODE_AA_PUSH : MODE_AA_LOCAL);
        L.flip = b->aa ? 0 : (int32_t)(k & 1);
        L.part_buf = (int32_t)(*recs & 1);
        L.fin_buf = pending ? pending_buf : -1;
        L.n_domains = (int32_t)b->members.size();
        L.n_fin = L.fin_buf >= 0 ? (L.n_domains + N_XCD - 1) / N_XCD * N_XCD : 0;
        L.pose_k = (int32_t)(k - k0);
        if (!b->halo_w.empty()) {   // the cuts' halo columns for this step
            BatchHalo H{};
            H.n_links = (int32_t)b->halo_w.size();
            H.ny = b->members[0]->p.ny;
            H.flip = L.flip;
            H.args = b->dev;
            for (int32_t i = 0; i < H.n_links; ++i) {
                H.w[i] = b->halo_w[i];
                H.e[i] = b->halo_e[i];
            }
            hipError_t he = launch_halo_batch(b->storage, H, b->stream);
            if (he != hipSuccess) return b->hip_fail(he, "halo exchange launch");
        }
        hipError_t e = launch_step_batch(b->storage, b->vec, b->block, mode, record, keep, batch_moving(b), L,
                                         b->stream);
        if (e != hipSuccess) return b->hip_fail(e, "batched step launch");
        pending = record;
        if (record) {
            pending_buf = L.part_buf;
            *recs += 1;
        }
    }
    if (pending) {
        hipError_t e = launch_finalize_batch(reinterpret_cast<const FinalizeArgs*>(b->dev + b->off_fins),
                                             (int32_t)b->members.size(), pending_buf, b->stream);
        if (e != hipSuccess) return b->hip_fail(e, "batched finalize launch");
    }
    if (batch_moving(b) && n > 0) {   // the moving members' next pose rows
        hipError_t e = launch_pose_advance_batch(b->storage, b->dev, (int32_t)b->members.size(), n, b->stream);
        if (e != hipSuccess) return b->hip_fail(e, "pose advance launch");
    }
    return LBVP_OK;
}

// Moving members: every one's pose table holds the time levels of the call's
// steps k0 + 1 .. k0 + n, counted from the member's own step count (outside any
// capture; n <= POSE_ROWS).
lbvp_status batch_pose_windows(lbvp_batch* b, int64_t k0, int64_t n)
{
    for (lbvp_ctx* c : b->members)
        if (c->moving()) {
            const lbvp_status st = pose_window(c, c->step + k0 + 1, n);
            if (st != LBVP_OK) return b->fail(st, "pose table of a moving member: " + c->err);
        }
    return LBVP_OK;
}

// Until disarmed, forgets the members' pose windows when it goes out of scope:
// a run that failed part way may have left their device pose rows anywhere.
struct PoseWindowGuard {
    const std::vector<lbvp_ctx*>& members;
    bool armed = true;
    ~PoseWindowGuard()
    {
        if (armed)
            for (lbvp_ctx* c : members) c->pose_first = -1;
    }
};

// After a run of n_steps: the members' step counts, lattice parity, records
// and fields, as lbvp_step would leave them.
void batch_advance_members(lbvp_batch* b, int64_t n_steps, int64_t recs, bool keep)
{
    for (lbvp_ctx* c : b->members) {
        c->step += n_steps;
        if (!c->aa() && (n_steps & 1)) c->cur ^= 1;
        c->rec_head += recs;
        if (keep) c->fields_valid = true;
    }
}

// ---- the static device array of lbvp_batch_step_static
// For callers that cannot allocate device memory, the batch tables (argument
// blocks, finalize arguments, tile map) of that call live in this array, one
// copy per GPU, held until the process ends. Host code never passes the array's
// name to a kernel or a copy: it is a host-side stand-in there. Each device's
// address comes from hipGetSymbolAddress, taken once with that device current.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(4) << 20;
__device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

struct StaticScratch {
    char* dev = nullptr;                 // this device's copy of `scratch`
    std::vector<char> host;              // pageable staging of the tables, STATIC_SCRATCH_BYTES
    hipEvent_t copied = nullptr;         // recorded after the last upload from `host`
};
constexpr int MAX_STATIC_DEVICES = 64;
std::mutex g_static_mu;
StaticScratch g_static[MAX_STATIC_DEVICES];

// The current device's entry, set up on its first use; "" or the reason it failed.
std::string static_scratch(StaticScratch** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return std::string("hipGetDevice: ") + hipGetErrorString(e);
    if (dev < 0 || dev >= MAX_STATIC_DEVICES) return "device index beyond the static table";
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticScratch& s = g_static[dev];
    if (!s.dev) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        if (!s.copied) {
            e = hipEventCreateWithFlags(&s.copied, hipEventDisableTiming);
            if (e != hipSuccess) return std::string("hipEventCreate: ") + hipGetErrorString(e);
        }
        s.host.assign(STATIC_SCRATCH_BYTES, 0);
        s.dev = static_cast<char*>(p);
    }
    *out = &s;
    return "";
}

lbvp_status batch_static_fail(lbvp_status st, const std::string& why)
{
    g_batch_error = "lbvp_batch_step_static: " + why;
    return st;
}

}  // namespace

namespace lbvp {

lbvp_status batch_new(hipStream_t stream, int32_t storage, uint32_t layout_flags, int32_t force_every, int32_t vec,
                      int32_t block, lbvp_batch** out)
{
    lbvp_batch* b = new (std::nothrow) lbvp_batch();
    if (!b) return LBVP_E_NOMEM;
    b->stream = stream;
    b->storage = storage;
    b->aa = (layout_flags & LBVP_LAYOUT_AA) != 0;
    b->force_every = force_every;
    b->vec = vec;
    b->block = block;
    *out = b;
    return LBVP_OK;
}

lbvp_status batch_set_members(lbvp_batch* b, lbvp_ctx* const* members, int32_t n)
{
    return batch_assign(b, std::vector<lbvp_ctx*>(members, members + n));
}

void ctx_rebind_stream(lbvp_ctx* c, hipStream_t s)
{
    c->graphs.clear(c->stream);
    c->stream = s;
}

}  // namespace lbvp

namespace {

thread_local std::string g_tune_error;
std::mutex g_tune_mu;
std::map<std::string, std::pair<std::vector<lbvp_tune_row>, int32_t>> g_tune_cache;

std::string tune_signature(const std::vector<lbvp_ctx*>& m, int32_t steps, uint32_t flags)
{
    // a domain's size and whether it runs the moving-body kernels
    std::vector<std::array<int32_t, 3>> shapes;
    for (const lbvp_ctx* c : m) shapes.push_back({c->p.nx, c->p.ny, c->moving() ? c->n_bodies : 0});
    std::sort(shapes.begin(), shapes.end());
    std::ostringstream o;
    const lbvp_ctx* c0 = m[0];
    o << c0->p.storage << '/' << (c0->p.flags & LBVP_LAYOUT_AA) << '/' << c0->p.force_every << '/' << steps << '/'
      << (flags & LBVP_TUNE_LAYOUTS);
    for (auto& x : shapes) o << ';' << x[0] << 'x' << x[1] << (x[2] ? "m" + std::to_string(x[2]) : "");
    return o.str();
}

// Tile bands the tuner tries for vector launches: eighths, and the bands measured
// fastest for single domains (2 for 2-byte and FP64 storage, 8 to 16 for FP32).
constexpr int32_t TUNE_BANDS[] = {0, 2, 16};

// Time every launch shape in one layout on scratch copies of the members'
// problems (parameters, mask, bodies; fluid at rest).
lbvp_status tune_layout(const std::vector<lbvp_ctx*>& m, uint32_t layout, int32_t steps,
                        std::vector<lbvp_tune_row>& rows)
{
    std::vector<lbvp_ctx*> s;
    lbvp_batch* b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto finish = [&](lbvp_status st, const std::string& why) {
        if (b) lbvp_batch_destroy(b);
        for (lbvp_ctx* x : s) lbvp_destroy(x);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st != LBVP_OK) g_tune_error = why;
        return st;
    };
    const hipStream_t stream = m[0]->stream;
    double nodes = 0.0;
    for (const lbvp_ctx* c : m) {
        lbvp_params p = c->p;
        p.flags = (p.flags & ~LBVP_LAYOUT_AA) | layout;
        p.force_capacity = std::max<int64_t>(p.force_capacity, 2 * (int64_t)steps + 16);
        lbvp_ctx* x = nullptr;
        lbvp_status st = lbvp_create(&p, stream, nullptr, 0, &x);
        if (st != LBVP_OK) return finish(st, "scratch context: " + g_create_error);
        s.push_back(x);
        st = lbvp_set_mask(x, c->mask_host.data(), c->n_bodies, c->bodies_host.data());
        if (st != LBVP_OK) return finish(st, "scratch mask: " + x->err);
        nodes += (double)c->p.nx * c->p.ny;
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return finish(LBVP_E_DEVICE, "hipEventCreate failed");
    const int32_t storage = m[0]->p.storage;
    for (int32_t vec : vec_options(storage, layout))
        for (int32_t block : {64, 128, 256})
            for (int32_t band : TUNE_BANDS) {
                if (vec == 1 && band != 0) continue;   // one node per thread: eighths only
                lbvp_status st = LBVP_OK;
                if (s.size() == 1) {
                    st = lbvp_set_launch(s[0], vec, block);
                    if (st == LBVP_OK) st = lbvp_set_tile_band(s[0], band);
                } else {
                    st = lbvp_batch_create(s.data(), (int32_t)s.size(), vec, block, &b);
                    if (st == LBVP_OK) st = lbvp_batch_set_tile_band(b, band);
                }
                if (st != LBVP_OK) return finish(st, "launch shape: " + (s.size() == 1 ? s[0]->err : g_batch_error));
                auto run = [&](int64_t k) { return b ? lbvp_batch_step(b, k, 0) : lbvp_step(s[0], k, 0); };
                double best = 1e300;
                st = run(std::max(2, steps / 4));
                for (lbvp_ctx* x : s) x->rec_tail = x->rec_head;   // records are not needed
                for (int rep = 0; rep < 3 && st == LBVP_OK; ++rep) {
                    if (hipEventRecord(e0, stream) != hipSuccess) return finish(LBVP_E_DEVICE, "hipEventRecord");
                    st = run(steps);
                    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                        return finish(LBVP_E_DEVICE, "timing events failed");
                    float ms = 0.0f;
                    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return finish(LBVP_E_DEVICE, "hipEventElapsedTime");
                    best = std::min(best, (double)ms);
                    for (lbvp_ctx* x : s) x->rec_tail = x->rec_head;   // records are not needed
                }
                if (st != LBVP_OK) return finish(st, "timed steps failed");
                if (b) {
                    lbvp_batch_destroy(b);
                    b = nullptr;
                }
                lbvp_tune_row r{};
                r.layout_flags = layout;
                r.vec = vec;
                r.block = block;
                r.band = band;
                r.ms_per_step = best / steps;
                r.mlups = nodes * steps / (best * 1e3);
                rows.push_back(r);
            }
    return finish(LBVP_OK, "");
}

}  // namespace

extern "C" {

size_t lbvp_footprint_bytes(const lbvp_params* p)
{
    if (!validate(p).empty()) return 0;
    return make_layout(p).total;
}

lbvp_status lbvp_create(const lbvp_params* p, void* hip_stream, void* dev_mem, size_t dev_bytes,
                        lbvp_ctx** out)
{
    if (!out) {
        g_create_error = "out is NULL";
        return LBVP_E_ARG;
    }
    *out = nullptr;
    const std::string why = validate(p);
    if (!why.empty()) {
        g_create_error = why;
        return LBVP_E_ARG;
    }
    lbvp_ctx* c = new (std::nothrow) lbvp_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return LBVP_E_NOMEM;
    }
    c->p = *p;
    c->L = make_layout(p);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->tau_minus = 0.5 + p->magic_lambda / (p->tau_plus - 0.5);
    if (dev_mem) {
        if (dev_bytes < c->L.total) {
            g_create_error = "dev_mem smaller than lbvp_footprint_bytes";
            delete c;
            return LBVP_E_NOMEM;
        }
        if (reinterpret_cast<uintptr_t>(dev_mem) % ALIGN) {
            g_create_error = "dev_mem must be 256-byte aligned";
            delete c;
            return LBVP_E_ARG;
        }
        c->mem = static_cast<char*>(dev_mem);
    } else {
        void* m = nullptr;
        hipError_t e = hipMalloc(&m, c->L.total);
        if (e != hipSuccess) {
            g_create_error = std::string("hipMalloc: ") + hipGetErrorString(e);
            delete c;
            return LBVP_E_NOMEM;
        }
        c->mem = static_cast<char*>(m);
        c->owns = true;
    }
    c->launch = default_launch(p->nx, p->ny, p->storage, p->flags);
    c->fin.max_bodies = c->L.max_bodies;
    c->fin.n_mass = c->launch.n_tiles * (c->launch.block / 64);
    c->fin.capacity = c->L.capacity;
    c->fin.mass_offset = p->rho0 * (double)p->nx * (double)p->ny;
    c->fin.body_slot_ptr = c->at<int32_t>(c->L.body_slot_ptr);
    c->fin.body_slots = c->at<int32_t>(c->L.body_slots);
    c->fin.slot_force = c->at<double>(c->L.slot_force);
    c->fin.mass_part = c->at<double>(c->L.mass_part);
    c->fin.slot_stride = c->L.slot_cap * 2;
    c->fin.mass_stride = c->L.max_waves;
    c->fin.ring_force = c->at<double>(c->L.ring_force);
    c->fin.ring_mass = c->at<double>(c->L.ring_mass);
    c->fin.rec_count = c->at<int64_t>(c->L.rec_count);
    fill_step_args(c, c->a64);
    fill_step_args(c, c->a32);
    if (p->bc_west == LBVP_BC_NEIGHBOR || p->bc_east == LBVP_BC_NEIGHBOR) {
        // the halo columns (lattice padding) hold zero deviations, the state at
        // rest, until the first halo exchange
        const size_t lat_bytes = (size_t)p->ny * (size_t)c->L.lstride * c->esize();
        hipError_t e = hipMemsetAsync(c->at<char>(c->L.lat[0]), 0, lat_bytes, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->at<char>(c->L.lat[1]), 0, lat_bytes, c->stream);
        if (e != hipSuccess) {
            g_create_error = std::string("hipMemsetAsync: ") + hipGetErrorString(e);
            lbvp_destroy(c);
            return LBVP_E_DEVICE;
        }
    }
    // empty mask, fluid at rest
    std::vector<uint8_t> zero((size_t)p->nx * p->ny, 0);
    lbvp_status s = lbvp_set_mask(c, zero.data(), 0, nullptr);
    if (s == LBVP_OK) s = lbvp_init_equilibrium(c, nullptr, nullptr, nullptr);
    if (s != LBVP_OK) {
        g_create_error = c->err;
        lbvp_destroy(c);
        return s;
    }
    *out = c;
    return LBVP_OK;
}

lbvp_status lbvp_set_mask(lbvp_ctx* c, const uint8_t* body_id, int32_t n_bodies, const lbvp_body* bodies)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    const lbvp_params& p = c->p;
    const Layout& L = c->L;
    if (!body_id) return c->fail(LBVP_E_ARG, "body_id is NULL");
    if (n_bodies < 0 || n_bodies > L.max_bodies) return c->fail(LBVP_E_ARG, "n_bodies out of range (see max_bodies)");
    if (n_bodies > 0 && !bodies) return c->fail(LBVP_E_ARG, "bodies is NULL");
    for (int32_t k = 0; k < n_bodies; ++k) {
        const double v[5] = {bodies[k].cx, bodies[k].cy, bodies[k].vx, bodies[k].vy, bodies[k].omega};
        for (double x : v)
            if (!std::isfinite(x)) return c->fail(LBVP_E_ARG, "non-finite body value");
    }
    const int64_t n = (int64_t)p.nx * p.ny;
    for (int64_t k = 0; k < n; ++k)
        if (body_id[k] > n_bodies) return c->fail(LBVP_E_ARG, "body_id larger than n_bodies");

    std::vector<char> table = c->is_f64() ? body_table_bytes<double>(bodies, n_bodies, L.max_bodies)
                                          : body_table_bytes<float>(bodies, n_bodies, L.max_bodies);
    if (c->moving() && n_bodies > MAX_MOVING) return c->fail(LBVP_E_ARG, "moving bodies: at most 8");
    c->graphs.clear(c->stream);
    c->mask_host.assign(body_id, body_id + n);
    c->bodies_host.assign(bodies, bodies + n_bodies);
    c->mov_r2.assign((size_t)n_bodies, 0.0);
    c->mov_runs.assign((size_t)n_bodies, {});
    c->pose_first = -1;   // the poses follow the new bodies
    c->a64.n_moving = c->a32.n_moving = c->moving() ? n_bodies : 0;
    if (c->moving()) {   // reach of each body about its centre: farthest node + 1
        std::vector<double> rmax((size_t)n_bodies, 0.0);
        std::vector<std::array<int32_t, 2>> span((size_t)n_bodies);
        for (int32_t j = 0; j < p.ny; ++j) {
            for (auto& q : span) q = {INT32_MAX, -1};
            for (int32_t i = 0; i < p.nx; ++i) {
                const int b = body_id[(int64_t)j * p.nx + i];
                if (!b) continue;
                const double dx = i - bodies[b - 1].cx, dy = j - bodies[b - 1].cy;
                rmax[b - 1] = std::max(rmax[b - 1], std::sqrt(dx * dx + dy * dy));
                span[b - 1][0] = std::min(span[b - 1][0], i);
                span[b - 1][1] = i;
            }
            for (int32_t b = 0; b < n_bodies; ++b)
                if (span[b][1] >= 0) c->mov_runs[b].push_back({j, span[b][0], span[b][1]});
        }
        for (int32_t b = 0; b < n_bodies; ++b) c->mov_r2[b] = (rmax[b] + 1.0) * (rmax[b] + 1.0);
    }
    c->n_bodies = n_bodies;
    c->fin.n_bodies = n_bodies;
    c->gen += 1;

    hipStream_t s = c->stream;
    LBVP_HIP(c, hipMemcpy2DAsync(c->at<uint8_t>(L.mask), (size_t)L.pitch, body_id, (size_t)p.nx,
                                 (size_t)p.nx, (size_t)p.ny, hipMemcpyHostToDevice, s));
    LBVP_HIP(c, hipMemcpyAsync(c->at<char>(L.bodies), table.data(), table.size(), hipMemcpyHostToDevice, s));
    return build_tile_tables(c);  // synchronizes
}

lbvp_status lbvp_init_equilibrium(lbvp_ctx* c, const double* rho, const double* ux, const double* uy)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    const lbvp_params& p = c->p;
    const Layout& L = c->L;
    hipStream_t s = c->stream;
    const int64_t stage_nodes = L.stage_rows * 9 * p.nx / 3;  // three staged planes
    const int32_t rows_per = (int32_t)std::max<int64_t>(1, std::min<int64_t>(p.ny, stage_nodes / p.nx));
    for (int32_t r0 = 0; r0 < p.ny; r0 += rows_per) {
        const int32_t rows = std::min(rows_per, p.ny - r0);
        ConvArgs a = conv_args(c, r0, rows);
        const size_t nn = (size_t)rows * p.nx;
        double* st = c->at<double>(L.stage);
        const double* src[3] = {rho, ux, uy};
        const double* dst[3] = {nullptr, nullptr, nullptr};
        for (int q = 0; q < 3; ++q) {
            if (!src[q]) continue;
            LBVP_HIP(c, hipMemcpyAsync(st + q * nn, src[q] + (size_t)r0 * p.nx, nn * sizeof(double),
                                       hipMemcpyHostToDevice, s));
            dst[q] = st + q * nn;
        }
        a.rho = dst[0];
        a.ux = dst[1];
        a.uy = dst[2];
        LBVP_HIP(c, launch_init(p.storage, c->at<char>(L.lat[0]), c->at<char>(L.fields), a, s));
    }
    LBVP_HIP(c, refresh_aa_ghosts(c));
    LBVP_HIP(c, launch_set_i64(c->fin.rec_count, 0, s));
    LBVP_HIP(c, hipStreamSynchronize(s));
    c->cur = 0;
    c->step = 0;
    c->pose_first = -1;   // the step count starts again: so do the poses
    c->rec_head = c->rec_tail = 0;
    c->pending = false;
    c->fields_valid = true;
    return LBVP_OK;
}

lbvp_status lbvp_step(lbvp_ctx* c, int64_t n_steps, uint32_t flags)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    if (n_steps < 0) return c->fail(LBVP_E_ARG, "n_steps < 0");
    if (flags & ~KNOWN_STEP_FLAGS) return c->fail(LBVP_E_ARG, "unknown step flag");
    const int64_t fe = c->p.force_every;
    if (fe > 0) {
        const int64_t new_recs = (c->step + n_steps) / fe - c->step / fe;
        if (c->rec_head + new_recs - c->rec_tail > c->L.capacity)
            return c->fail(LBVP_E_STATE, "force records would overflow the device ring; call lbvp_forces first");
    }
    const bool keep = (flags & LBVP_KEEP_FIELDS) != 0;
    if (!(flags & LBVP_GRAPH)) {
        if (!c->moving()) return enqueue_steps(c, n_steps, keep, true);
        for (int64_t done = 0; done < n_steps;) {   // runs that fit the pose table
            const int64_t n = std::min<int64_t>(POSE_ROWS, n_steps - done);
            lbvp_status st = pose_window(c, c->step + 1, n);
            if (st == LBVP_OK) st = enqueue_steps(c, n, keep && done + n == n_steps, true);
            if (st != LBVP_OK) return st;
            done += n;
        }
        return LBVP_OK;
    }
    if (!c->stream) return c->fail(LBVP_E_ARG, "LBVP_GRAPH needs a stream other than the null stream");
    for (int64_t done = 0; done < n_steps;) {
        const int64_t n = std::min(GRAPH_CHUNK, n_steps - done);
        const bool keep_here = keep && done + n == n_steps;
        if (c->moving()) {   // outside any capture: the chunk's poses on the device
            const lbvp_status st = pose_window(c, c->step + 1, n);
            if (st != LBVP_OK) return st;
        }
        GraphKey key;
        key.n = n;
        key.keep = keep_here;
        key.cur = c->cur;
        key.par = c->aa() ? (int32_t)(c->step & 1) : 0;
        key.phase = fe > 0 ? c->step % fe : 0;
        key.rec = (int32_t)(c->rec_head & 1);
        key.gen = c->gen;
        hipGraphExec_t x = c->graphs.find(key);
        if (x) {
            LBVP_HIP(c, hipGraphLaunch(x, c->stream));
            enqueue_steps(c, n, keep_here, false);
        } else {
            const CtxClock saved = save_clock(c);
            LBVP_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            const lbvp_status st = enqueue_steps(c, n, keep_here, true);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(c->stream, &g);
            if (st != LBVP_OK || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                restore_clock(c, saved);
                return st != LBVP_OK ? st : c->hip_fail(e, "hipStreamEndCapture");
            }
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                restore_clock(c, saved);
                return c->hip_fail(e, "hipGraphInstantiate");
            }
            c->graphs.put(key, x, c->stream);
            e = hipGraphLaunch(x, c->stream);
            if (e != hipSuccess) {
                restore_clock(c, saved);
                return c->hip_fail(e, "hipGraphLaunch");
            }
        }
        done += n;
    }
    return LBVP_OK;
}

lbvp_status lbvp_forces(lbvp_ctx* c, double* out, double* mass, int64_t cap, int64_t* n_out, int64_t* first_step)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    if (cap < 0) return c->fail(LBVP_E_ARG, "cap < 0");
    LBVP_HIP(c, hipStreamSynchronize(c->stream));
    const int64_t avail = c->rec_head - c->rec_tail;
    const int64_t n = std::min(avail, cap);
    const int64_t C = c->L.capacity, mb = c->L.max_bodies, nb = c->n_bodies;
    std::vector<double> rf((size_t)std::max<int64_t>(n, 1) * mb * 2), rm((size_t)std::max<int64_t>(n, 1));
    int64_t done = 0;
    while (done < n) {
        const int64_t r = (c->rec_tail + done) % C;
        const int64_t len = std::min(n - done, C - r);
        LBVP_HIP(c, hipMemcpyAsync(rf.data() + done * mb * 2, c->at<double>(c->L.ring_force) + r * mb * 2,
                                   (size_t)(len * mb * 2) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        LBVP_HIP(c, hipMemcpyAsync(rm.data() + done, c->at<double>(c->L.ring_mass) + r,
                                   (size_t)len * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        done += len;
    }
    LBVP_HIP(c, hipStreamSynchronize(c->stream));
    bool finite = true;
    for (int64_t k = 0; k < n; ++k) {
        if (out)
            for (int64_t b = 0; b < nb; ++b) {
                out[(k * nb + b) * 2] = rf[(k * mb + b) * 2];
                out[(k * nb + b) * 2 + 1] = rf[(k * mb + b) * 2 + 1];
            }
        if (mass) mass[k] = rm[k];
        if (!std::isfinite(rm[k])) finite = false;
    }
    if (n_out) *n_out = n;
    if (first_step) *first_step = n > 0 ? (c->rec_tail + 1) * c->p.force_every : 0;
    c->rec_tail += n;
    if (!finite) return c->fail(LBVP_E_UNSTABLE, "non-finite global mass: the run went unstable");
    return LBVP_OK;
}

lbvp_status lbvp_read_fields_rows(lbvp_ctx* c, int32_t y0, int32_t n_rows, double* rho, double* ux, double* uy,
                                  double* fx, double* fy)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    const lbvp_params& p = c->p;
    if (y0 < 0 || n_rows < 1 || n_rows > p.ny - y0) return c->fail(LBVP_E_ARG, "row range outside the grid");
    if (!c->fields_valid) return c->fail(LBVP_E_STATE, "no fields kept since the last init");
    LBVP_HIP(c, hipStreamSynchronize(c->stream));
    double* dst[5] = {rho, ux, uy, fx, fy};
    const size_t rs = c->rsize();
    const size_t n = (size_t)p.nx * n_rows;
    std::vector<char> tmp(n * rs);
    for (int q = 0; q < 5; ++q) {
        if (!dst[q]) continue;
        const char* srcp = c->at<char>(c->L.fields) + ((size_t)q * c->L.plane_f + (size_t)y0 * c->L.pitch) * rs;
        LBVP_HIP(c, hipMemcpy2DAsync(tmp.data(), (size_t)p.nx * rs, srcp, (size_t)c->L.pitch * rs,
                                     (size_t)p.nx * rs, (size_t)n_rows, hipMemcpyDeviceToHost, c->stream));
        LBVP_HIP(c, hipStreamSynchronize(c->stream));
        if (c->is_f64()) std::memcpy(dst[q], tmp.data(), n * sizeof(double));
        else {
            const float* f = reinterpret_cast<const float*>(tmp.data());
            for (size_t k = 0; k < n; ++k) dst[q][k] = (double)f[k];
        }
    }
    return LBVP_OK;
}

lbvp_status lbvp_read_fields(lbvp_ctx* c, double* rho, double* ux, double* uy, double* fx, double* fy)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    return lbvp_read_fields_rows(c, 0, c->p.ny, rho, ux, uy, fx, fy);
}

lbvp_status lbvp_read_populations_rows(lbvp_ctx* c, int32_t y0, int32_t n_rows, double* g)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    if (!g) return c->fail(LBVP_E_ARG, "g is NULL");
    const lbvp_params& p = c->p;
    if (y0 < 0 || n_rows < 1 || n_rows > p.ny - y0) return c->fail(LBVP_E_ARG, "row range outside the grid");
    if (c->aa() && c->step % 2)
        return c->fail(LBVP_E_STATE, "the AA layout holds the post-collision populations after an even step count");
    hipStream_t s = c->stream;
    const int32_t rows_per = (int32_t)std::min<int64_t>(n_rows, c->L.stage_rows);
    const size_t N = (size_t)p.nx * n_rows;
    for (int32_t r0 = 0; r0 < n_rows; r0 += rows_per) {
        const int32_t rows = std::min(rows_per, n_rows - r0);
        ConvArgs a = conv_args(c, y0 + r0, rows);
        LBVP_HIP(c, launch_decode(p.storage, c->at<char>(c->L.lat[c->cur]), a, s));
        const size_t nn = (size_t)rows * p.nx;
        for (int q = 0; q < 9; ++q)
            LBVP_HIP(c, hipMemcpyAsync(g + q * N + (size_t)r0 * p.nx, a.pops + q * nn, nn * sizeof(double),
                                       hipMemcpyDeviceToHost, s));
        LBVP_HIP(c, hipStreamSynchronize(s));
    }
    return LBVP_OK;
}

lbvp_status lbvp_read_populations(lbvp_ctx* c, double* g)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    return lbvp_read_populations_rows(c, 0, c->p.ny, g);
}

lbvp_status lbvp_write_populations(lbvp_ctx* c, const double* g)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    if (!g) return c->fail(LBVP_E_ARG, "g is NULL");
    if (c->aa() && c->step % 2)
        return c->fail(LBVP_E_STATE, "the AA layout takes populations after an even step count");
    const lbvp_params& p = c->p;
    hipStream_t s = c->stream;
    const int32_t rows_per = (int32_t)std::min<int64_t>(p.ny, c->L.stage_rows);
    const size_t N = (size_t)p.nx * p.ny;
    for (int32_t r0 = 0; r0 < p.ny; r0 += rows_per) {
        const int32_t rows = std::min(rows_per, p.ny - r0);
        ConvArgs a = conv_args(c, r0, rows);
        const size_t nn = (size_t)rows * p.nx;
        for (int q = 0; q < 9; ++q)
            LBVP_HIP(c, hipMemcpyAsync(a.pops + q * nn, g + q * N + (size_t)r0 * p.nx, nn * sizeof(double),
                                       hipMemcpyHostToDevice, s));
        LBVP_HIP(c, launch_encode(p.storage, c->at<char>(c->L.lat[c->cur]), a, s));
    }
    LBVP_HIP(c, refresh_aa_ghosts(c));
    LBVP_HIP(c, hipStreamSynchronize(s));
    return LBVP_OK;
}

}  // extern "C"

namespace {

// Checkpoint blob: this header, then the stored lattice, the two ghost columns,
// the mask (ny x nx bytes), the bodies, the five field planes (pitched, as stored).
struct StateHeader {
    char magic[8];
    uint32_t version, header_bytes;
    int32_t nx, ny, storage;
    uint32_t layout;
    int32_t n_bodies, cur, fields_valid, pad;
    int64_t step, records;
    uint64_t lat_bytes, ghost_bytes, mask_bytes, body_bytes, field_bytes;
};
constexpr char STATE_MAGIC[8] = {'L', 'B', 'V', 'P', 'S', 'T', 'A', 'T'};
constexpr uint32_t STATE_VERSION = 1;

StateHeader state_header(const lbvp_ctx* c)
{
    StateHeader h{};
    std::memcpy(h.magic, STATE_MAGIC, 8);
    h.version = STATE_VERSION;
    h.header_bytes = sizeof(StateHeader);
    h.nx = c->p.nx;
    h.ny = c->p.ny;
    h.storage = c->p.storage;
    h.layout = c->p.flags & LBVP_LAYOUT_AA;
    h.n_bodies = c->n_bodies;
    h.cur = c->cur;
    h.fields_valid = c->fields_valid ? 1 : 0;
    h.step = c->step;
    h.records = c->rec_head;
    h.lat_bytes = (uint64_t)c->p.ny * (uint64_t)c->L.lstride * c->esize();
    h.ghost_bytes = 3 * (uint64_t)c->p.ny * c->esize();
    h.mask_bytes = (uint64_t)c->p.nx * c->p.ny;
    h.body_bytes = (uint64_t)c->n_bodies * sizeof(lbvp_body);
    h.field_bytes = 5 * (uint64_t)c->L.plane_f * c->rsize();
    return h;
}

uint64_t state_bytes(const StateHeader& h)
{
    return h.header_bytes + h.lat_bytes + 2 * h.ghost_bytes + h.mask_bytes + h.body_bytes + h.field_bytes;
}

}  // namespace

extern "C" {

lbvp_status lbvp_save_state(lbvp_ctx* c, void* buf, size_t cap, size_t* size)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    if (!size) return c->fail(LBVP_E_ARG, "size is NULL");
    if (c->rec_head != c->rec_tail) return c->fail(LBVP_E_STATE, "drain the force records first");
    const StateHeader h = state_header(c);
    *size = (size_t)state_bytes(h);
    if (!buf || cap < *size) return c->fail(LBVP_E_NOMEM, "buffer too small for the state (see *size)");
    hipStream_t s = c->stream;
    char* o = static_cast<char*>(buf);
    std::memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    LBVP_HIP(c, hipMemcpyAsync(o, c->at<char>(c->L.lat[c->cur]), h.lat_bytes, hipMemcpyDeviceToHost, s));
    o += h.lat_bytes;
    LBVP_HIP(c, hipMemcpyAsync(o, c->at<char>(c->L.ghost_w), h.ghost_bytes, hipMemcpyDeviceToHost, s));
    o += h.ghost_bytes;
    LBVP_HIP(c, hipMemcpyAsync(o, c->at<char>(c->L.ghost_e), h.ghost_bytes, hipMemcpyDeviceToHost, s));
    o += h.ghost_bytes;
    LBVP_HIP(c, hipMemcpyAsync(o + h.mask_bytes + h.body_bytes, c->at<char>(c->L.fields), h.field_bytes,
                               hipMemcpyDeviceToHost, s));
    std::memcpy(o, c->mask_host.data(), h.mask_bytes);
    o += h.mask_bytes;
    if (h.body_bytes) std::memcpy(o, c->bodies_host.data(), h.body_bytes);
    LBVP_HIP(c, hipStreamSynchronize(s));
    return LBVP_OK;
}

lbvp_status lbvp_load_state(lbvp_ctx* c, const void* buf, size_t size)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    if (!buf || size < sizeof(StateHeader)) return c->fail(LBVP_E_ARG, "not a state blob");
    StateHeader h;
    std::memcpy(&h, buf, sizeof(h));
    const StateHeader mine = state_header(c);
    if (std::memcmp(h.magic, STATE_MAGIC, 8) != 0 || h.version != STATE_VERSION || h.header_bytes != sizeof(h))
        return c->fail(LBVP_E_ARG, "not a state blob of this version");
    if (h.nx != mine.nx || h.ny != mine.ny || h.storage != mine.storage || h.layout != mine.layout)
        return c->fail(LBVP_E_ARG, "the state is of another grid, storage type or layout");
    if (h.n_bodies < 0 || h.n_bodies > c->L.max_bodies) return c->fail(LBVP_E_ARG, "the state holds more bodies than max_bodies");
    if (h.cur < 0 || h.cur > 1 || (mine.layout && h.cur != 0) || h.step < 0 || h.records < 0)
        return c->fail(LBVP_E_ARG, "damaged state counters");
    if (h.lat_bytes != mine.lat_bytes || h.ghost_bytes != mine.ghost_bytes || h.mask_bytes != mine.mask_bytes ||
        h.body_bytes != (uint64_t)h.n_bodies * sizeof(lbvp_body) || h.field_bytes != mine.field_bytes ||
        size < state_bytes(h))
        return c->fail(LBVP_E_ARG, "damaged state sizes");
    const char* o = static_cast<const char*>(buf) + sizeof(h);
    const char* lat = o;
    const char* gw = lat + h.lat_bytes;
    const char* ge = gw + h.ghost_bytes;
    const uint8_t* mask = reinterpret_cast<const uint8_t*>(ge + h.ghost_bytes);
    std::vector<lbvp_body> bodies((size_t)h.n_bodies);
    if (h.body_bytes) std::memcpy(bodies.data(), mask + h.mask_bytes, h.body_bytes);
    const char* fields = reinterpret_cast<const char*>(mask) + h.mask_bytes + h.body_bytes;
    lbvp_status st = lbvp_set_mask(c, mask, h.n_bodies, bodies.data());   // validates and synchronizes
    if (st != LBVP_OK) return st;
    hipStream_t s = c->stream;
    LBVP_HIP(c, hipMemcpyAsync(c->at<char>(c->L.lat[h.cur]), lat, h.lat_bytes, hipMemcpyHostToDevice, s));
    LBVP_HIP(c, hipMemcpyAsync(c->at<char>(c->L.ghost_w), gw, h.ghost_bytes, hipMemcpyHostToDevice, s));
    LBVP_HIP(c, hipMemcpyAsync(c->at<char>(c->L.ghost_e), ge, h.ghost_bytes, hipMemcpyHostToDevice, s));
    LBVP_HIP(c, hipMemcpyAsync(c->at<char>(c->L.fields), fields, h.field_bytes, hipMemcpyHostToDevice, s));
    LBVP_HIP(c, launch_set_i64(c->fin.rec_count, h.records, s));
    LBVP_HIP(c, hipStreamSynchronize(s));
    c->graphs.clear(s);
    c->cur = h.cur;
    c->step = h.step;
    c->pose_first = -1;
    c->rec_head = c->rec_tail = h.records;
    c->pending = false;
    c->fields_valid = h.fields_valid != 0;
    c->gen += 1;
    return LBVP_OK;
}

}  // extern "C"

extern "C" {

lbvp_status lbvp_set_launch(lbvp_ctx* c, int32_t vec, int32_t block)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    if (!vec_allowed(c->p.storage, c->p.flags, vec))
        return c->fail(LBVP_E_ARG, "vec must be 1, the storage type's 16-byte vector width or, for "
                                   "2-byte storage, 4 (1 only for 2-byte storage in the AA layout)");
    if (block != 64 && block != 128 && block != 256) return c->fail(LBVP_E_ARG, "block must be 64, 128 or 256");
    if (c->launch.vec == vec && c->launch.block == block) return LBVP_OK;
    if (c->rec_head != c->rec_tail) return c->fail(LBVP_E_STATE, "drain the force records first");
    LBVP_HIP(c, hipStreamSynchronize(c->stream));
    c->graphs.clear(c->stream);
    Launch l = make_launch(c->p.nx, c->p.ny, vec, block);
    l.band = c->launch.band;
    return apply_launch(c, l);
}

lbvp_status lbvp_get_launch(const lbvp_ctx* c, int32_t* vec, int32_t* block)
{
    if (!c || !vec || !block) return LBVP_E_ARG;
    *vec = c->launch.vec;
    *block = c->launch.block;
    return LBVP_OK;
}

lbvp_status lbvp_set_tile_band(lbvp_ctx* c, int32_t band)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    if (!band_allowed(band)) return c->fail(LBVP_E_ARG, "band must be 0 or a power of two up to 65536");
    if (c->launch.band == band) return LBVP_OK;
    c->launch.band = band;
    c->gen += 1;   // captured graphs hold the old kernel arguments
    fill_step_args(c, c->a64);
    fill_step_args(c, c->a32);
    return LBVP_OK;
}

lbvp_status lbvp_get_tile_band(const lbvp_ctx* c, int32_t* band)
{
    if (!c || !band) return LBVP_E_ARG;
    *band = c->launch.band;
    return LBVP_OK;
}

lbvp_status lbvp_halo_exchange(lbvp_ctx* const* west, lbvp_ctx* const* east, int32_t n)
{
    if (!west || !east || n < 1 || n > MAX_HALO_LINKS || !west[0]) return LBVP_E_ARG;
    lbvp_ctx* c0 = west[0];
    HaloArgs h{};
    h.n_links = n;
    h.ny = c0->p.ny;
    for (int32_t i = 0; i < n; ++i) {
        lbvp_ctx* w = west[i];
        lbvp_ctx* e = east[i];
        if (!w || !e) return c0->fail(LBVP_E_ARG, "lbvp_halo_exchange: NULL context");
        if (w->p.bc_east != LBVP_BC_NEIGHBOR || e->p.bc_west != LBVP_BC_NEIGHBOR)
            return c0->fail(LBVP_E_ARG, "lbvp_halo_exchange: linked sides must be LBVP_BC_NEIGHBOR");
        if (w->p.ny != h.ny || e->p.ny != h.ny || w->p.storage != c0->p.storage || e->p.storage != c0->p.storage)
            return c0->fail(LBVP_E_ARG, "lbvp_halo_exchange: linked slabs need equal ny and storage type");
        if (w->stream != c0->stream || e->stream != c0->stream)
            return c0->fail(LBVP_E_ARG, "lbvp_halo_exchange: all slabs must share one stream");
        HaloLink& L = h.link[i];
        L.w_lat = L.w_lat_w = w->at<char>(w->L.lat[w->cur]);
        L.e_lat = L.e_lat_w = e->at<char>(e->L.lat[e->cur]);
        L.w_lstride = w->L.lstride;
        L.w_plane = w->L.plane;
        L.e_lstride = e->L.lstride;
        L.e_plane = e->L.plane;
        L.e_pitch = e->L.pitch;
        L.w_nx = w->p.nx;
    }
    LBVP_HIP(c0, launch_halo(c0->p.storage, h, c0->stream));
    return LBVP_OK;
}

int64_t lbvp_step_count(const lbvp_ctx* c) { return c ? c->step : -1; }

lbvp_status lbvp_device_copy(const void* src, void* dst, size_t bytes, void* hip_stream)
{
    if (!src || !dst || bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return LBVP_E_ARG;
    if (bytes == 0) return LBVP_OK;
    return launch_copy16(src, dst, (int64_t)(bytes / 16), static_cast<hipStream_t>(hip_stream)) == hipSuccess
               ? LBVP_OK : LBVP_E_DEVICE;
}

lbvp_status lbvp_synchronize(lbvp_ctx* c)
{
    if (check_ctx(c)) return LBVP_E_ARG;
    LBVP_HIP(c, hipStreamSynchronize(c->stream));
    return LBVP_OK;
}

lbvp_status lbvp_destroy(lbvp_ctx* c)
{
    if (!c) return LBVP_OK;
    lbvp_status st = LBVP_OK;
    if (c->mem) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) st = LBVP_E_DEVICE;
        if (c->owns && hipFree(c->mem) != hipSuccess) st = LBVP_E_DEVICE;
    }
    delete c;
    return st;
}

const char* lbvp_last_error(const lbvp_ctx* c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

lbvp_status lbvp_batch_create(lbvp_ctx* const* members, int32_t n, int32_t vec, int32_t block, lbvp_batch** out)
{
    if (!out || !members || n < 1) {
        g_batch_error = "members, n >= 1 and out are required";
        return LBVP_E_ARG;
    }
    *out = nullptr;
    for (int32_t d = 0; d < n; ++d)
        if (!members[d]) {
            g_batch_error = "a member is NULL";
            return LBVP_E_ARG;
        }
    const lbvp_ctx* c0 = members[0];
    if (vec == 0) vec = vec_allowed(c0->p.storage, c0->p.flags, vector_width(c0->p.storage)) ? vector_width(c0->p.storage) : 1;
    if (block == 0) block = MAX_BLOCK;
    lbvp_batch* b = nullptr;
    if (batch_new(c0->stream, c0->p.storage, c0->p.flags, c0->p.force_every, vec, block, &b) != LBVP_OK) {
        g_batch_error = "host allocation failed";
        return LBVP_E_NOMEM;
    }
    const lbvp_status st = batch_assign(b, std::vector<lbvp_ctx*>(members, members + n));
    if (st != LBVP_OK) {
        g_batch_error = b->err;
        delete b;
        return st;
    }
    *out = b;
    return LBVP_OK;
}

lbvp_status lbvp_batch_step(lbvp_batch* b, int64_t n_steps, uint32_t flags)
{
    if (!b) return LBVP_E_ARG;
    if (n_steps < 0) return b->fail(LBVP_E_ARG, "n_steps < 0");
    if (flags & ~KNOWN_STEP_FLAGS) return b->fail(LBVP_E_ARG, "unknown step flag");
    if (n_steps == 0) return LBVP_OK;
    if (b->members.empty()) return b->fail(LBVP_E_STATE, "the batch has no members");
    std::string why = batch_consistency(b, b->members);
    if (!why.empty()) return b->fail(LBVP_E_STATE, why);
    const int64_t fe = b->force_every;
    const int64_t step0 = b->members[0]->step;
    const int64_t new_recs = fe > 0 ? (step0 + n_steps) / fe - step0 / fe : 0;
    for (lbvp_ctx* c : b->members) {
        if (c->launch.vec != b->vec || c->launch.block != b->block)
            return b->fail(LBVP_E_STATE, "a member's launch shape was changed after the batch was made");
        if (c->rec_head + new_recs - c->rec_tail > c->L.capacity)
            return b->fail(LBVP_E_STATE, "a member's force ring would overflow; drain it with lbvp_forces first");
    }
    const lbvp_status up = batch_refresh_args(b);
    if (up != LBVP_OK) return up;
    const bool keep = (flags & LBVP_KEEP_FIELDS) != 0;
    int64_t recs = 0;
    const bool moving = batch_moving(b);
    PoseWindowGuard guard{b->members};
    if (!(flags & LBVP_GRAPH)) {
        // one run, or runs that fit the moving members' pose tables
        const int64_t seg = moving ? (int64_t)POSE_ROWS : n_steps;
        for (int64_t k0 = 0; k0 < n_steps;) {
            const int64_t n = std::min(seg, n_steps - k0);
            lbvp_status st = moving ? batch_pose_windows(b, k0, n) : LBVP_OK;
            if (st == LBVP_OK) st = batch_run(b, step0, k0, n, keep && k0 + n == n_steps, &recs);
            if (st != LBVP_OK) return st;
            k0 += n;
        }
    } else {
        if (!b->stream) return b->fail(LBVP_E_ARG, "LBVP_GRAPH needs a stream other than the null stream");
        for (int64_t k0 = 0; k0 < n_steps;) {
            const int64_t n = std::min(GRAPH_CHUNK, n_steps - k0);
            const bool keep_here = keep && k0 + n == n_steps;
            if (moving) {   // outside any capture: the chunk's poses on the device
                const lbvp_status st = batch_pose_windows(b, k0, n);
                if (st != LBVP_OK) return st;
            }
            GraphKey key;
            key.n = n;
            key.keep = keep_here;
            key.cur = (int32_t)(k0 & 1);
            key.par = b->aa ? (int32_t)((step0 + k0) & 1) : 0;
            key.phase = fe > 0 ? (step0 + k0) % fe : 0;
            key.rec = (int32_t)(recs & 1);
            key.gen = b->gen;
            hipGraphExec_t x = b->graphs.find(key);
            if (x) {
                LBVP_HIP(b, hipGraphLaunch(x, b->stream));
                if (fe > 0) recs += (step0 + k0 + n) / fe - (step0 + k0) / fe;
            } else {
                LBVP_HIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
                const lbvp_status st = batch_run(b, step0, k0, n, keep_here, &recs);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(b->stream, &g);
                if (st != LBVP_OK || e != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return st != LBVP_OK ? st : b->hip_fail(e, "hipStreamEndCapture");
                }
                e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return b->hip_fail(e, "hipGraphInstantiate");
                b->graphs.put(key, x, b->stream);
                LBVP_HIP(b, hipGraphLaunch(x, b->stream));
            }
            k0 += n;
        }
    }
    guard.armed = false;
    batch_advance_members(b, n_steps, recs, keep);
    return LBVP_OK;
}

lbvp_status lbvp_batch_step_static(lbvp_ctx* const* members, int32_t n, int64_t n_steps, uint32_t flags)
{
    g_batch_error.clear();
    if (!members || n < 1) return batch_static_fail(LBVP_E_ARG, "members[n] with n >= 1 required");
    if (n_steps < 0) return batch_static_fail(LBVP_E_ARG, "n_steps < 0");
    if (flags & ~KNOWN_STEP_FLAGS) return batch_static_fail(LBVP_E_ARG, "unknown step flag");
    if (flags & LBVP_GRAPH) return batch_static_fail(LBVP_E_ARG, "LBVP_GRAPH instantiates graphs, which allocates");
    for (int32_t i = 0; i < n; ++i)
        if (check_ctx(members[i])) return batch_static_fail(LBVP_E_ARG, "a member is NULL or not a context");
    const lbvp_ctx* c0 = members[0];
    for (int32_t i = 0; i < n; ++i)
        if (members[i]->launch.vec != c0->launch.vec || members[i]->launch.block != c0->launch.block)
            return batch_static_fail(LBVP_E_ARG, "members need the first member's launch shape (lbvp_set_launch)");
    // a batch object on the host only: its device block is the static array
    lbvp_batch b;
    b.stream = c0->stream;
    b.storage = c0->p.storage;
    b.aa = c0->aa();
    b.force_every = c0->p.force_every;
    b.vec = c0->launch.vec;
    b.block = c0->launch.block;
    const std::vector<lbvp_ctx*> m(members, members + n);
    const std::string why = batch_consistency(&b, m);
    if (!why.empty()) return batch_static_fail(LBVP_E_ARG, why);
    if (n_steps == 0) return LBVP_OK;
    const int64_t fe = b.force_every;
    const int64_t step0 = c0->step;
    const int64_t new_recs = fe > 0 ? (step0 + n_steps) / fe - step0 / fe : 0;
    for (lbvp_ctx* c : m)
        if (c->rec_head + new_recs - c->rec_tail > c->L.capacity)
            return batch_static_fail(LBVP_E_STATE, "a member's force ring would overflow; drain it with lbvp_forces first");
    batch_layout(&b, m);
    if (b.bytes > STATIC_SCRATCH_BYTES) {
        std::ostringstream os;
        os << "the members' tables need " << b.bytes << " bytes, more than the " << STATIC_SCRATCH_BYTES
           << "-byte static array (fewer members, or fewer tiles: a wider launch shape)";
        return batch_static_fail(LBVP_E_ARG, os.str());
    }
    StaticScratch* sc = nullptr;
    const std::string setup = static_scratch(&sc);
    if (!setup.empty()) return batch_static_fail(LBVP_E_DEVICE, setup);
    batch_fill_args(&b);
    // the previous call's copy must have read the host staging block before it
    // is overwritten; every byte of the tables is rewritten, none is left over
    hipError_t e = hipSuccess;
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        e = hipEventSynchronize(sc->copied);
        if (e == hipSuccess) {
            std::memcpy(sc->host.data(), b.image.data(), b.bytes);
            e = hipMemcpyAsync(sc->dev, sc->host.data(), b.bytes, hipMemcpyHostToDevice, b.stream);
        }
        if (e == hipSuccess) e = hipEventRecord(sc->copied, b.stream);
    }
    if (e != hipSuccess) return batch_static_fail(LBVP_E_DEVICE, std::string("uploading the tables: ") + hipGetErrorString(e));
    b.dev = sc->dev;
    b.dev_cap = STATIC_SCRATCH_BYTES;
    int64_t recs = 0;
    lbvp_status st = LBVP_OK;
    const bool moving = batch_moving(&b);
    const int64_t seg = moving ? (int64_t)POSE_ROWS : n_steps;
    for (int64_t k0 = 0; k0 < n_steps && st == LBVP_OK;) {
        const int64_t n = std::min(seg, n_steps - k0);
        if (moving) st = batch_pose_windows(&b, k0, n);
        if (st == LBVP_OK) st = batch_run(&b, step0, k0, n, (flags & LBVP_KEEP_FIELDS) != 0 && k0 + n == n_steps, &recs);
        k0 += n;
    }
    b.dev = nullptr;   // not the batch's to free
    if (st != LBVP_OK) {
        for (lbvp_ctx* c : m) c->pose_first = -1;   // the device pose rows may be anywhere
        return batch_static_fail(st, b.err);
    }
    batch_advance_members(&b, n_steps, recs, (flags & LBVP_KEEP_FIELDS) != 0);
    return LBVP_OK;
}

lbvp_status lbvp_batch_set_halo(lbvp_batch* b, const int32_t* west, const int32_t* east, int32_t n)
{
    if (!b) return LBVP_E_ARG;
    if (n < 0 || n > MAX_HALO_LINKS || (n > 0 && (!west || !east)))
        return b->fail(LBVP_E_ARG, "lbvp_batch_set_halo: 0..32 links with both index arrays");
    const int32_t nm = (int32_t)b->members.size();
    for (int32_t i = 0; i < n; ++i) {
        if (west[i] < 0 || west[i] >= nm || east[i] < 0 || east[i] >= nm)
            return b->fail(LBVP_E_ARG, "lbvp_batch_set_halo: member index out of range");
        const lbvp_ctx* w = b->members[west[i]];
        const lbvp_ctx* e = b->members[east[i]];
        if (w->p.bc_east != LBVP_BC_NEIGHBOR || e->p.bc_west != LBVP_BC_NEIGHBOR)
            return b->fail(LBVP_E_ARG, "lbvp_batch_set_halo: linked sides must be LBVP_BC_NEIGHBOR");
        if (w->p.ny != b->members[0]->p.ny || e->p.ny != b->members[0]->p.ny)
            return b->fail(LBVP_E_ARG, "lbvp_batch_set_halo: linked members need equal ny");
    }
    b->halo_w.assign(west, west + n);
    b->halo_e.assign(east, east + n);
    b->graphs.clear(b->stream);
    b->gen += 1;
    return LBVP_OK;
}

lbvp_status lbvp_batch_set_tile_band(lbvp_batch* b, int32_t band)
{
    if (!b) return LBVP_E_ARG;
    if (!band_allowed(band)) return b->fail(LBVP_E_ARG, "band must be 0 or a power of two up to 65536");
    if (b->band == band) return LBVP_OK;
    b->band = band;
    b->gen += 1;   // captured graphs hold the old launch arguments
    return LBVP_OK;
}

lbvp_status lbvp_batch_get_tile_band(const lbvp_batch* b, int32_t* band)
{
    if (!b || !band) return LBVP_E_ARG;
    *band = b->band;
    return LBVP_OK;
}

lbvp_status lbvp_batch_destroy(lbvp_batch* b)
{
    if (!b) return LBVP_OK;
    lbvp_status st = LBVP_OK;
    if (b->dev && hipStreamSynchronize(b->stream) != hipSuccess) st = LBVP_E_DEVICE;
    delete b;
    return st;
}

const char* lbvp_batch_last_error(const lbvp_batch* b)
{
    return b ? b->err.c_str() : g_batch_error.c_str();
}

lbvp_status lbvp_tune(lbvp_ctx* const* members, int32_t n, int32_t steps, uint32_t flags, lbvp_tune_row* rows,
                      int32_t cap, int32_t* n_rows, int32_t* best)
{
    if (!members || n < 1 || steps < 1 || cap < 0 || (cap > 0 && !rows) || !n_rows || !best ||
        (flags & ~(LBVP_TUNE_LAYOUTS | LBVP_TUNE_FRESH))) {
        g_tune_error = "members, n >= 1, steps >= 1, rows[cap], n_rows, best and known flags are required";
        return LBVP_E_ARG;
    }
    std::vector<lbvp_ctx*> m(members, members + n);
    for (lbvp_ctx* c : m)
        if (!c) {
            g_tune_error = "a member is NULL";
            return LBVP_E_ARG;
        }
    const lbvp_ctx* c0 = m[0];
    for (const lbvp_ctx* c : m) {
        if (c->p.storage != c0->p.storage || c->aa() != c0->aa() || c->stream != c0->stream ||
            c->p.force_every != c0->p.force_every) {
            g_tune_error = "members differ in storage, layout, stream or force_every";
            return LBVP_E_ARG;
        }
    }
    const std::string key = tune_signature(m, steps, flags);
    std::vector<lbvp_tune_row> table;
    int32_t pick = 0;
    bool cached = false;
    if (!(flags & LBVP_TUNE_FRESH)) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            table = it->second.first;
            pick = it->second.second;
            cached = true;
        }
    }
    if (!cached) {
        const uint32_t own = c0->p.flags & LBVP_LAYOUT_AA;
        std::vector<uint32_t> layouts{own};
        if (flags & LBVP_TUNE_LAYOUTS) layouts.push_back(own ^ LBVP_LAYOUT_AA);
        for (uint32_t layout : layouts) {
            const lbvp_status st = tune_layout(m, layout, steps, table);
            if (st != LBVP_OK) return st;
        }
        for (int32_t i = 1; i < (int32_t)table.size(); ++i)
            if (table[i].ms_per_step < table[pick].ms_per_step) pick = i;
        if (flags & LBVP_TUNE_LAYOUTS) {
            int32_t aa = -1;
            for (int32_t i = 0; i < (int32_t)table.size(); ++i)
                if ((table[i].layout_flags & LBVP_LAYOUT_AA) && (aa < 0 || table[i].ms_per_step < table[aa].ms_per_step))
                    aa = i;
            if (aa >= 0 && table[aa].ms_per_step <= 1.03 * table[pick].ms_per_step) pick = aa;
        }
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = {table, pick};
    }
    const int32_t k = std::min<int32_t>(cap, (int32_t)table.size());
    for (int32_t i = 0; i < k; ++i) rows[i] = table[i];
    *n_rows = (int32_t)table.size();
    *best = pick;
    return LBVP_OK;
}

const char* lbvp_tune_last_error(void) { return g_tune_error.c_str(); }

}  // extern "C"
