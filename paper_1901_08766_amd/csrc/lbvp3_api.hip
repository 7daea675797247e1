// lbvp3_api.hip -- host side of the D3Q19 C ABI (include/lbvp3.h): validation,
// the device memory layout, tiling and record tables, and the step sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lbvp3.h"
#include "lbvp3_internal.h"
#include "lbvp_graph.h"

using namespace lbvp3;

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t STAGE_MIN_BYTES = size_t(64) << 20;
constexpr int64_t DEFAULT_CAPACITY = 4096;
constexpr int32_t DEFAULT_MAX_BODIES = 8;
constexpr int32_t MAX_BODIES = 255;
constexpr uint32_t KNOWN_STEP_FLAGS = LBVP_KEEP_FIELDS | LBVP_GRAPH;
constexpr int64_t GRAPH_CHUNK = 512;   // steps per captured graph; longer calls replay it
constexpr int32_t VECS[3] = {1, 2, 4};
constexpr int32_t BLOCKS[3] = {64, 128, 256};

thread_local std::string g_create_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
size_t storage_bytes(int32_t st) { return st == LBVP_F64 ? 8 : st == LBVP_F32 ? 4 : 2; }
size_t arith_bytes(int32_t st) { return st == LBVP_F64 ? 8 : 4; }

struct Launch3 {
    int32_t vec = 1, block = 256, tile_w = 256, tile_rows = 1;
    int32_t tiles_x = 0, n_tiles = 0, tiles_per_xcd = 0;
    int32_t band = 0;   // block -> tile order: 0 = one eighth per XCD, else bands of `band` tiles
};

int32_t band_log2(int32_t band)
{
    int32_t k = -1;
    while (band > 0) {
        band >>= 1;
        ++k;
    }
    return k;
}

// A tile is tile_rows lattice rows of tile_w nodes: full rows of vec * block
// nodes on wide grids; on narrow ones, as many whole rows of nx nodes (rounded
// up to vec) as a block holds, the block's remaining threads idle (a 96- or
// 160-node row then idles 6% of a 512-node block, not the 25% or 37.5% of rows
// padded to a power of two).
Launch3 make_launch(int32_t nx, int64_t rows, int32_t vec, int32_t block)
{
    Launch3 l;
    l.vec = vec;
    l.block = block;
    l.tile_w = std::min(vec * block, (std::max(nx, 1) + vec - 1) / vec * vec);
    l.tile_rows = vec * block / l.tile_w;
    l.tiles_x = (nx + l.tile_w - 1) / l.tile_w;
    l.n_tiles = (int32_t)(l.tiles_x * ((rows + l.tile_rows - 1) / l.tile_rows));
    l.tiles_per_xcd = (l.n_tiles + N_XCD - 1) / N_XCD;
    return l;
}

// Defaults measured on a 512 x 256 x 256 domain: one node per thread for FP32
// (256-thread blocks) and FP64 (128): the 19 loads of a node already keep enough
// bytes in flight, and the narrow form keeps ~70 VGPRs and 7 waves per SIMD,
// against ~150 VGPRs and 3 waves for 16-byte vectors. The 2-byte types take four
// nodes per thread (8-byte loads, lane shuffles) in 128-thread blocks, 7% ahead
// of single 2-byte elements. Tiles go to the XCDs in bands (lbvp3_set_tile_band):
// 128 tiles (a quarter plane there) for FP32 and FP64, 0.874 and 1.736 ms per
// step against 0.890 and 1.758 with one eighth per XCD; 4 tiles for the 2-byte
// types, 0.445 ms against 0.468 with one eighth per XCD and 0.458 for bands of
// 2 tiles of 256-thread blocks. Grids too small to fill the chip: one node per
// thread, 64-thread blocks, one eighth per XCD.
Launch3 default_launch(const lbvp3_params& p)
{
    const int64_t rows = (int64_t)p.ny * p.nz, n = rows * p.nx;
    const bool two_byte = p.storage == LBVP_F16_DEV || p.storage == LBVP_BF16_DEV;
    const int32_t vec = two_byte && n / (64 * 4) >= 8 * 1024 ? 4 : 1;
    const int32_t wide = (p.storage == LBVP_F64 || two_byte) ? 128 : 256;
    const bool large = n / (64 * vec) >= 4096;
    Launch3 l = make_launch(p.nx, rows, vec, large ? wide : 64);
    if (large) l.band = two_byte ? 4 : 128;
    return l;
}

std::string validate(const lbvp3_params* p)
{
    if (!p) return "params is NULL";
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return "nx, ny and nz must be >= 3";
    const int64_t rows = (int64_t)p->ny * p->nz;
    if (rows > (int64_t(1) << 30) || rows * p->nx > (int64_t(1) << 34)) return "grid too large";
    if (!std::isfinite(p->tau_plus) || !(p->tau_plus > 0.5)) return "tau_plus must be finite and > 1/2";
    if (!std::isfinite(p->magic_lambda) || !(p->magic_lambda > 0.0)) return "magic_lambda must be finite and > 0";
    if (!std::isfinite(p->eta) || !(p->eta > 0.0)) return "eta must be finite and > 0";
    if (!std::isfinite(p->rho0) || !(p->rho0 > 0.0)) return "rho0 must be finite and > 0";
    const double vals[] = {p->rho_in, p->u_in[0], p->u_in[1], p->u_in[2], p->body_force[0], p->body_force[1],
                           p->body_force[2]};
    for (double v : vals)
        if (!std::isfinite(v)) return "non-finite inflow state or body force";
    const int32_t sides[2] = {p->bc_west, p->bc_east};
    for (int32_t s : sides)
        if (s != LBVP_BC_PERIODIC && s != LBVP_BC_INFLOW_EQ && s != LBVP_BC_OUTFLOW_ZERO_GRAD) return "unknown side";
    if ((p->bc_west == LBVP_BC_PERIODIC) != (p->bc_east == LBVP_BC_PERIODIC))
        return "x sides must be both periodic or both non-periodic";
    if (p->storage < LBVP_F64 || p->storage > LBVP_BF16_DEV) return "unknown storage";
    if (p->force_every < 0) return "force_every < 0";
    if (p->force_capacity < 0) return "force_capacity < 0";
    if (p->max_bodies < 0 || p->max_bodies > MAX_BODIES) return "max_bodies out of range";
    if (p->flags != 0) return "unknown flag";
    return "";
}

// Device memory of a context: every table sized for the finest tiling any
// launch configuration uses.
struct Layout3 {
    int64_t pitch = 0, lstride = 0, plane_f = 0, rows = 0;
    int32_t max_tiles = 0, max_waves = 0, max_bodies = 0;
    int64_t slot_cap = 0, capacity = 0, stage_planes = 0;
    size_t lat[2] = {0, 0}, mask = 0, bodies = 0, fields = 0, mass_part = 0, slot_force = 0, tile_slot_ptr = 0,
           slot_body = 0, body_slot_ptr = 0, body_slots = 0, ring_force = 0, ring_mass = 0, rec_count = 0,
           arrivals = 0, fin_stage = 0, stage = 0, total = 0;
};

Layout3 make_layout(const lbvp3_params& p)
{
    Layout3 L;
    L.pitch = (int64_t)align_up((size_t)p.nx, 64);
    L.lstride = (int64_t)Q * L.pitch;
    L.rows = (int64_t)p.ny * p.nz;
    L.plane_f = L.rows * L.pitch;
    for (int32_t v : VECS)
        for (int32_t b : BLOCKS) {
            const Launch3 l = make_launch(p.nx, L.rows, v, b);
            L.max_tiles = std::max(L.max_tiles, l.n_tiles);
            L.max_waves = std::max(L.max_waves, l.n_tiles * (b / 64));
        }
    L.max_bodies = p.max_bodies > 0 ? p.max_bodies : DEFAULT_MAX_BODIES;
    L.capacity = p.force_capacity > 0 ? p.force_capacity : DEFAULT_CAPACITY;
    // (tile, body) pairs: one body per tile, two where bodies meet, plus headroom
    L.slot_cap = 2 * (int64_t)L.max_tiles + 4096;
    const size_t es = storage_bytes(p.storage), rs = arith_bytes(p.storage);
    const size_t plane_pops = (size_t)Q * 8 * (size_t)p.nx * (size_t)p.ny;
    const size_t stage_bytes = std::max(STAGE_MIN_BYTES, plane_pops);
    L.stage_planes = std::max<int64_t>(1, std::min<int64_t>(p.nz, (int64_t)(stage_bytes / plane_pops)));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, ALIGN);
        return o;
    };
    const size_t lat_bytes = (size_t)L.rows * L.lstride * es;
    L.lat[0] = take(lat_bytes);
    L.lat[1] = take(lat_bytes);
    L.mask = take((size_t)L.rows * L.pitch);
    L.bodies = take((size_t)(L.max_bodies + 1) * BODY3_STRIDE * rs);
    L.fields = take((size_t)7 * L.plane_f * rs);
    L.mass_part = take((size_t)2 * L.max_waves * 8);       // double-buffered partials
    L.slot_force = take((size_t)2 * L.slot_cap * 3 * 8);
    L.tile_slot_ptr = take((size_t)(L.max_tiles + 1) * 4);
    L.slot_body = take((size_t)L.slot_cap * 4);
    L.body_slot_ptr = take((size_t)(L.max_bodies + 1) * 4);
    L.body_slots = take((size_t)L.slot_cap * 4);
    L.ring_force = take((size_t)L.capacity * L.max_bodies * 3 * 8);
    L.ring_mass = take((size_t)L.capacity * 8);
    L.rec_count = take(8);
    L.arrivals = take(8);
    L.fin_stage = take((size_t)N_LEAD * (1 + 3 * L.max_bodies) * 8);
    L.stage = take((size_t)L.stage_planes * plane_pops);
    L.total = off;
    return L;
}

}  // namespace

struct lbvp3_ctx {
    lbvp3_params p{};
    Layout3 L;
    Launch3 launch;
    hipStream_t stream = nullptr;
    char* mem = nullptr;
    int cur = 0;
    int64_t step = 0, rec_head = 0, rec_tail = 0;
    bool pending = false;       // a recorded step whose sums are not yet in the ring
    int32_t pending_buf = 0;
    bool fields_valid = false;
    int32_t n_bodies = 0;
    double tau_minus = 0.0;
    std::vector<uint8_t> mask_host;   // [nz][ny][nx], kept to rebuild the tile tables
    std::vector<lbvp3_body> bodies_host;   // the bodies as given, kept for checkpoints
    Step3Args<double> a64{};
    Step3Args<float> a32{};
    Fin3Args fin{};
    lbvp_host::GraphCache graphs;   // captured chunks of steps (LBVP_GRAPH)
    uint64_t gen = 0;               // kernel-argument generation (graph keys)
    std::string err;

    template <typename T> T* at(size_t off) { return reinterpret_cast<T*>(mem + off); }
    // captured graphs hold the old kernel arguments
    void args_changed()
    {
        graphs.clear(stream);
        gen += 1;
    }
    bool is_f64() const { return p.storage == LBVP_F64; }
    size_t rsize() const { return arith_bytes(p.storage); }
    lbvp_status fail(lbvp_status s, const std::string& m)
    {
        err = m;
        return s;
    }
    lbvp_status hip_fail(hipError_t e, const char* what)
    {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LBVP_E_DEVICE;
    }
};

// Contexts advanced together, one launch per step over all their tiles. The
// members stay ordinary contexts (their records, fields and populations are read
// through the usual calls) and step in lockstep.
struct lbvp3_batch {
    std::vector<lbvp3_ctx*> members;
    hipStream_t stream = nullptr;
    int32_t storage = 0, vec = 1, block = 256, band = 0;
    int32_t total_tiles = 0, tiles_per_xcd = 0;
    char* dev = nullptr;             // owned: [member images | tile_domain | tile_start]
    size_t member_bytes = 0, off_domain = 0, off_start = 0;
    std::vector<char> image;         // host image of the member block, as last uploaded
    lbvp_host::GraphCache graphs;    // captured chunks of batched steps (LBVP_GRAPH)
    int64_t gen = 0;                 // bumped when something a captured launch bakes in changes
    std::string err;

    lbvp_status fail(lbvp_status s, const std::string& m)
    {
        err = m;
        return s;
    }
    lbvp_status hip_fail(hipError_t e, const char* what)
    {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LBVP_E_DEVICE;
    }
    ~lbvp3_batch()
    {
        graphs.clear(stream);
        if (dev) {
            (void)hipStreamSynchronize(stream);
            (void)hipFree(dev);
        }
    }
};

thread_local std::string g_batch3_error;
thread_local std::string g_tune3_error;
std::mutex g_tune3_mu;
std::map<std::string, std::pair<std::vector<lbvp3_tune_row>, int32_t>> g_tune3_cache;

namespace {

#define LBVP3_HIP(ctx, call)                                              \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) return (ctx)->hip_fail(e_, #call);          \
    } while (0)

template <typename R>
void fill_args(lbvp3_ctx* c, Step3Args<R>& a)
{
    const lbvp3_params& p = c->p;
    const Layout3& L = c->L;
    const Launch3& l = c->launch;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
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
    a.lstride = L.lstride;
    a.plane_f = L.plane_f;
    a.rho0 = (R)p.rho0;
    a.om_p = (R)(1.0 / p.tau_plus);
    a.om_m = (R)(1.0 / c->tau_minus);
    a.k_p = (R)(1.0 - 0.5 / p.tau_plus);
    a.k_m = (R)(1.0 - 0.5 / c->tau_minus);
    a.vp_c = (R)(1.0 / (2.0 * p.eta + 1.0));
    for (int d = 0; d < 3; ++d) {
        a.fb[d] = (R)p.body_force[d];
        a.fb18[d] = (R)(18.0 * p.body_force[d]);
    }
    // the inflow populations (f^eq(rho_in, u_in) - w rho0) / w (eq. feq), in FP64
    const double* u = p.u_in;
    const double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    for (int q = 0; q < Q; ++q) {
        const double eu = (CX[q] * u[0] + CY[q] * u[1]) + CZ[q] * u[2];
        a.feq_in[q] = (R)((p.rho_in - p.rho0) + p.rho_in * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
    }
    a.mask = c->at<uint8_t>(L.mask);
    a.bodies = c->at<R>(L.bodies);
    a.tile_slot_ptr = c->at<int32_t>(L.tile_slot_ptr);
    a.slot_body = c->at<int32_t>(L.slot_body);
    a.slot_force = c->at<double>(L.slot_force);
    a.mass_part = c->at<double>(L.mass_part);
    a.fields = c->at<R>(L.fields);
    a.part_buf = 0;
    a.fin_buf = -1;
    a.fin = c->fin;
}

// The (tile, body) tables for the current tiling and mask: a slot per body
// present in each tile, numbered in tile order, and the slots of each body.
lbvp_status build_tile_tables(lbvp3_ctx* c)
{
    const lbvp3_params& p = c->p;
    const Launch3& l = c->launch;
    const int32_t nb = c->n_bodies;
    const int64_t rows = c->L.rows;
    std::vector<int32_t> tile_ptr((size_t)l.n_tiles + 1, 0), slot_body;
    std::vector<std::vector<int32_t>> per_body((size_t)nb);
    std::vector<uint8_t> seen((size_t)nb + 1, 0);
    for (int32_t t = 0; t < l.n_tiles; ++t) {
        tile_ptr[t] = (int32_t)slot_body.size();
        if (nb == 0) continue;
        const int32_t ty = t / l.tiles_x, i0 = (t % l.tiles_x) * l.tile_w, i1 = std::min(p.nx, i0 + l.tile_w);
        const int64_t r0 = (int64_t)ty * l.tile_rows, r1 = std::min(rows, r0 + l.tile_rows);
        std::fill(seen.begin(), seen.end(), 0);
        for (int64_t r = r0; r < r1; ++r) {
            const uint8_t* row = c->mask_host.data() + r * p.nx;
            for (int32_t i = i0; i < i1; ++i) seen[row[i]] = 1;
        }
        for (int32_t b = 1; b <= nb; ++b) {
            if (!seen[b]) continue;
            if ((int64_t)slot_body.size() >= c->L.slot_cap) {
                (void)hipStreamSynchronize(c->stream);   // copies from the caller's host buffers
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
    const Layout3& L = c->L;
    LBVP3_HIP(c, hipMemcpyAsync(c->at<int32_t>(L.tile_slot_ptr), tile_ptr.data(), tile_ptr.size() * 4,
                                hipMemcpyHostToDevice, s));
    if (!slot_body.empty()) {
        LBVP3_HIP(c, hipMemcpyAsync(c->at<int32_t>(L.slot_body), slot_body.data(), slot_body.size() * 4,
                                    hipMemcpyHostToDevice, s));
        LBVP3_HIP(c, hipMemcpyAsync(c->at<int32_t>(L.body_slots), body_slots.data(), body_slots.size() * 4,
                                    hipMemcpyHostToDevice, s));
    }
    LBVP3_HIP(c, hipMemcpyAsync(c->at<int32_t>(L.body_slot_ptr), body_ptr.data(), body_ptr.size() * 4,
                                hipMemcpyHostToDevice, s));
    LBVP3_HIP(c, hipStreamSynchronize(s));   // the host tables above go out of scope
    c->fin.n_bodies = nb;
    return LBVP_OK;
}

lbvp_status apply_launch(lbvp3_ctx* c, const Launch3& l)
{
    c->launch = l;
    c->fin.n_mass = l.n_tiles * (l.block / 64);
    fill_args(c, c->a64);
    fill_args(c, c->a32);
    return build_tile_tables(c);
}

Conv3Args conv_args(lbvp3_ctx* c, int32_t plane0, int32_t planes)
{
    Conv3Args a{};
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.plane0 = plane0;
    a.planes = planes;
    a.pitch = c->L.pitch;
    a.lstride = c->L.lstride;
    a.plane_f = c->L.plane_f;
    a.rho0 = c->p.rho0;
    a.pops = c->at<double>(c->L.stage);
    return a;
}

bool bad_range(const lbvp3_ctx* c, int32_t z0, int32_t n) { return z0 < 0 || n < 0 || (int64_t)z0 + n > c->p.nz; }

// The member block a batch step reads: each member's step arguments (with its
// finalize arguments), lattices and current lattice, as now.
template <typename R>
void write_member_images(lbvp3_batch* b)
{
    for (size_t d = 0; d < b->members.size(); ++d) {
        lbvp3_ctx* c = b->members[d];
        Member3<R> m{};
        if constexpr (std::is_same<R, double>::value) m.a = c->a64;
        else m.a = c->a32;
        m.a.fin = c->fin;
        m.lat0 = c->at<char>(c->L.lat[0]);
        m.lat1 = c->at<char>(c->L.lat[1]);
        m.cur = c->cur;
        std::memcpy(b->image.data() + d * sizeof(Member3<R>), &m, sizeof(m));
    }
}

// Checkpoint blob: this header, then the current lattice as stored (pitched
// rows of 19 populations), the mask ([nz][ny][nx] bytes), the bodies, the seven
// field planes (pitched, as stored).
struct State3Header {
    char magic[8];
    uint32_t version, header_bytes;
    int32_t nx, ny, nz, storage;
    int32_t n_bodies, cur, fields_valid, pad;
    int64_t step, records;
    uint64_t lat_bytes, mask_bytes, body_bytes, field_bytes;
};
constexpr char STATE3_MAGIC[8] = {'L', 'B', 'V', 'P', '3', 'S', 'T', 'A'};
constexpr uint32_t STATE3_VERSION = 1;

State3Header state3_header(const lbvp3_ctx* c)
{
    State3Header h{};
    std::memcpy(h.magic, STATE3_MAGIC, 8);
    h.version = STATE3_VERSION;
    h.header_bytes = sizeof(State3Header);
    h.nx = c->p.nx;
    h.ny = c->p.ny;
    h.nz = c->p.nz;
    h.storage = c->p.storage;
    h.n_bodies = c->n_bodies;
    h.cur = c->cur;
    h.fields_valid = c->fields_valid ? 1 : 0;
    h.step = c->step;
    h.records = c->rec_head;
    h.lat_bytes = (uint64_t)c->L.rows * (uint64_t)c->L.lstride * storage_bytes(c->p.storage);
    h.mask_bytes = (uint64_t)c->L.rows * (uint64_t)c->p.nx;
    h.body_bytes = (uint64_t)c->n_bodies * sizeof(lbvp3_body);
    h.field_bytes = 7 * (uint64_t)c->L.plane_f * c->rsize();
    return h;
}

uint64_t state3_bytes(const State3Header& h)
{
    return h.header_bytes + h.lat_bytes + h.mask_bytes + h.body_bytes + h.field_bytes;
}

}  // namespace

extern "C" {

size_t lbvp3_footprint_bytes(const lbvp3_params* p)
{
    if (!validate(p).empty()) return 0;
    return make_layout(*p).total;
}

lbvp_status lbvp3_create(const lbvp3_params* p, void* hip_stream, lbvp3_ctx** out)
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
    lbvp3_ctx* c = new (std::nothrow) lbvp3_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return LBVP_E_NOMEM;
    }
    c->p = *p;
    c->L = make_layout(*p);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->tau_minus = 0.5 + p->magic_lambda / (p->tau_plus - 0.5);
    void* m = nullptr;
    hipError_t e = hipMalloc(&m, c->L.total);
    if (e != hipSuccess) {
        g_create_error = std::string("hipMalloc: ") + hipGetErrorString(e);
        delete c;
        return LBVP_E_NOMEM;
    }
    c->mem = static_cast<char*>(m);
    const Layout3& L = c->L;
    c->fin.max_bodies = L.max_bodies;
    c->fin.capacity = L.capacity;
    c->fin.mass_offset = p->rho0 * (double)p->nx * (double)p->ny * (double)p->nz;
    c->fin.body_slot_ptr = c->at<int32_t>(L.body_slot_ptr);
    c->fin.body_slots = c->at<int32_t>(L.body_slots);
    c->fin.slot_force = c->at<double>(L.slot_force);
    c->fin.mass_part = c->at<double>(L.mass_part);
    c->fin.slot_stride = L.slot_cap * 3;
    c->fin.mass_stride = L.max_waves;
    c->fin.ring_force = c->at<double>(L.ring_force);
    c->fin.ring_mass = c->at<double>(L.ring_mass);
    c->fin.rec_count = c->at<int64_t>(L.rec_count);
    c->fin.arrivals = c->at<int64_t>(L.arrivals);
    c->fin.stage = c->at<double>(L.fin_stage);
    c->launch = default_launch(*p);
    c->mask_host.assign((size_t)L.rows * p->nx, 0);
    lbvp_status s = lbvp3_set_mask(c, c->mask_host.data(), 0, nullptr);
    if (s == LBVP_OK) s = lbvp3_init_equilibrium(c, nullptr, nullptr, nullptr, nullptr);
    if (s != LBVP_OK) {
        g_create_error = c->err;
        lbvp3_destroy(c);
        return s;
    }
    *out = c;
    return LBVP_OK;
}

lbvp_status lbvp3_set_mask(lbvp3_ctx* c, const uint8_t* body_id, int32_t n_bodies, const lbvp3_body* bodies)
{
    if (!c) return LBVP_E_ARG;
    const lbvp3_params& p = c->p;
    const Layout3& L = c->L;
    if (!body_id) return c->fail(LBVP_E_ARG, "body_id is NULL");
    if (n_bodies < 0 || n_bodies > L.max_bodies) return c->fail(LBVP_E_ARG, "n_bodies out of range (see max_bodies)");
    if (n_bodies > 0 && !bodies) return c->fail(LBVP_E_ARG, "bodies is NULL");
    for (int32_t b = 0; b < n_bodies; ++b)
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(bodies[b].c[d]) || !std::isfinite(bodies[b].v[d]) || !std::isfinite(bodies[b].omega[d]))
                return c->fail(LBVP_E_ARG, "non-finite body value");
    const int64_t n = L.rows * p.nx;
    for (int64_t k = 0; k < n; ++k)
        if (body_id[k] > n_bodies) return c->fail(LBVP_E_ARG, "body_id larger than n_bodies");
    // accepted: from here the body count and the tables the graphs hold change
    // (a rejected call above leaves the context, its stream and its graphs alone)
    c->args_changed();
    // body table: row 0 all zero (fluid), row b = c_int, c_frac, v, omega of body
    // b, in the arithmetic type (the centre's split is exact in FP64)
    const size_t rs = c->rsize();
    std::vector<char> table((size_t)(L.max_bodies + 1) * BODY3_STRIDE * rs, 0);
    for (int32_t b = 0; b < n_bodies; ++b)
        for (int d = 0; d < 3; ++d) {
            const double ci = std::nearbyint(bodies[b].c[d]);
            const double vals[4] = {ci, bodies[b].c[d] - ci, bodies[b].v[d], bodies[b].omega[d]};
            for (int g = 0; g < 4; ++g) {
                const size_t idx = (size_t)(b + 1) * BODY3_STRIDE + 3 * g + d;
                if (c->is_f64()) reinterpret_cast<double*>(table.data())[idx] = vals[g];
                else reinterpret_cast<float*>(table.data())[idx] = (float)vals[g];
            }
        }
    if (body_id != c->mask_host.data()) c->mask_host.assign(body_id, body_id + n);
    c->bodies_host.assign(bodies, bodies + n_bodies);
    c->n_bodies = n_bodies;
    hipStream_t s = c->stream;
    LBVP3_HIP(c, hipMemcpy2DAsync(c->at<uint8_t>(L.mask), (size_t)L.pitch, c->mask_host.data(), (size_t)p.nx,
                                  (size_t)p.nx, (size_t)L.rows, hipMemcpyHostToDevice, s));
    LBVP3_HIP(c, hipMemcpyAsync(c->at<char>(L.bodies), table.data(), table.size(), hipMemcpyHostToDevice, s));
    return apply_launch(c, c->launch);   // synchronizes
}

lbvp_status lbvp3_init_equilibrium(lbvp3_ctx* c, const double* rho, const double* ux, const double* uy,
                                   const double* uz)
{
    if (!c) return LBVP_E_ARG;
    const lbvp3_params& p = c->p;
    const Layout3& L = c->L;
    hipStream_t s = c->stream;
    const size_t plane_nodes = (size_t)p.nx * p.ny;
    // four staged FP64 arrays per node fit the 19 the stage holds
    const int32_t per = (int32_t)std::max<int64_t>(1, std::min<int64_t>(p.nz, L.stage_planes * Q / 4));
    for (int32_t z0 = 0; z0 < p.nz; z0 += per) {
        const int32_t planes = std::min(per, p.nz - z0);
        Conv3Args a = conv_args(c, z0, planes);
        const size_t nn = (size_t)planes * plane_nodes;
        double* st = c->at<double>(L.stage);
        const double* src[4] = {rho, ux, uy, uz};
        const double* dst[4] = {nullptr, nullptr, nullptr, nullptr};
        for (int q = 0; q < 4; ++q) {
            if (!src[q]) continue;
            LBVP3_HIP(c, hipMemcpyAsync(st + q * nn, src[q] + (size_t)z0 * plane_nodes, nn * sizeof(double),
                                        hipMemcpyHostToDevice, s));
            dst[q] = st + q * nn;
        }
        a.rho = dst[0];
        for (int d = 0; d < 3; ++d) a.u[d] = dst[1 + d];
        LBVP3_HIP(c, launch_init3(p.storage, c->at<char>(L.lat[0]), c->at<char>(L.fields), a, s));
        LBVP3_HIP(c, hipStreamSynchronize(s));   // the next chunk reuses the stage
    }
    LBVP3_HIP(c, launch_zero_i64(c->fin.rec_count, s));
    LBVP3_HIP(c, launch_zero_i64(c->fin.arrivals, s));
    LBVP3_HIP(c, hipStreamSynchronize(s));
    c->cur = 0;
    c->step = 0;
    c->rec_head = c->rec_tail = 0;
    c->pending = false;
    c->fields_valid = true;
    return LBVP_OK;
}

lbvp_status lbvp3_step(lbvp3_ctx* c, int64_t n_steps, uint32_t flags)
{
    if (!c) return LBVP_E_ARG;
    if (n_steps < 0) return c->fail(LBVP_E_ARG, "n_steps < 0");
    if (flags & ~KNOWN_STEP_FLAGS) return c->fail(LBVP_E_ARG, "unknown step flag");
    const int64_t fe = c->p.force_every;
    if (fe > 0) {
        const int64_t new_recs = (c->step + n_steps) / fe - c->step / fe;
        if (c->rec_head + new_recs - c->rec_tail > c->L.capacity)
            return c->fail(LBVP_E_STATE, "force records would overflow the device ring; call lbvp3_forces first");
    }
    const bool keep = (flags & LBVP_KEEP_FIELDS) != 0;
    const void* args = c->is_f64() ? (const void*)&c->a64 : (const void*)&c->a32;
    c->a64.fin = c->fin;
    c->a32.fin = c->fin;
    // n steps, the last keeping the fields if asked, and the call's last record summed
    auto enqueue = [&](int64_t n, bool keep_last) -> lbvp_status {
        for (int64_t k = 0; k < n; ++k) {
            const int64_t next = c->step + 1;
            const bool record = fe > 0 && next % fe == 0;
            const bool keep_here = keep_last && k == n - 1;
            const int32_t part_buf = (int32_t)(c->rec_head & 1);
            c->a64.part_buf = c->a32.part_buf = part_buf;
            c->a64.fin_buf = c->a32.fin_buf = c->pending ? c->pending_buf : -1;
            hipError_t e = launch_step3(c->p.storage, record, keep_here, c->at<char>(c->L.lat[c->cur]),
                                        c->at<char>(c->L.lat[c->cur ^ 1]), args, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "step kernel launch");
            c->pending = record;
            if (record) {
                c->pending_buf = part_buf;
                c->rec_head += 1;
            }
            if (keep_here) c->fields_valid = true;
            c->cur ^= 1;
            c->step = next;
        }
        if (c->pending) {   // the last record of the call is summed on its own
            hipError_t e = launch_finalize3(c->fin, c->pending_buf, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "finalize kernel launch");
            c->pending = false;
        }
        return LBVP_OK;
    };
    if (!(flags & LBVP_GRAPH)) return enqueue(n_steps, keep);
    if (!c->stream) return c->fail(LBVP_E_ARG, "LBVP_GRAPH needs a stream other than the null stream");
    for (int64_t done = 0; done < n_steps;) {
        const int64_t n = std::min(GRAPH_CHUNK, n_steps - done);
        const bool keep_here = keep && done + n == n_steps;
        lbvp_host::GraphKey key;   // every call starts with its records summed
        key.n = n;
        key.keep = keep_here;
        key.cur = c->cur;
        key.phase = fe > 0 ? c->step % fe : 0;
        key.rec = (int32_t)(c->rec_head & 1);
        key.gen = c->gen;
        hipGraphExec_t x = c->graphs.find(key);
        if (x) {
            LBVP3_HIP(c, hipGraphLaunch(x, c->stream));
            // advance the host bookkeeping exactly as the captured launches did
            const int cur0 = c->cur;
            const int64_t step0 = c->step, head0 = c->rec_head;
            const int64_t recs = fe > 0 ? (step0 + n) / fe - step0 / fe : 0;
            c->cur = (int)((cur0 + n) & 1);
            c->step = step0 + n;
            c->rec_head = head0 + recs;
            c->pending = false;
            if (recs > 0) c->pending_buf = (int32_t)((c->rec_head - 1) & 1);
            if (keep_here) c->fields_valid = true;
        } else {
            const int cur0 = c->cur;
            const int64_t step0 = c->step, head0 = c->rec_head;
            const bool pend0 = c->pending, fields0 = c->fields_valid;
            const int32_t buf0 = c->pending_buf;
            auto restore = [&]() {
                c->cur = cur0;
                c->step = step0;
                c->rec_head = head0;
                c->pending = pend0;
                c->fields_valid = fields0;
                c->pending_buf = buf0;
            };
            LBVP3_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            const lbvp_status st = enqueue(n, keep_here);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(c->stream, &g);
            if (st != LBVP_OK || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                restore();
                return st != LBVP_OK ? st : c->hip_fail(e, "hipStreamEndCapture");
            }
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                restore();
                return c->hip_fail(e, "hipGraphInstantiate");
            }
            c->graphs.put(key, x, c->stream);
            e = hipGraphLaunch(x, c->stream);
            if (e != hipSuccess) {
                restore();
                return c->hip_fail(e, "hipGraphLaunch");
            }
        }
        done += n;
    }
    return LBVP_OK;
}

lbvp_status lbvp3_forces(lbvp3_ctx* c, double* out, double* mass, int64_t cap, int64_t* n_out, int64_t* first_step)
{
    if (!c) return LBVP_E_ARG;
    if (cap < 0) return c->fail(LBVP_E_ARG, "cap < 0");
    LBVP3_HIP(c, hipStreamSynchronize(c->stream));
    const int64_t n = std::min(c->rec_head - c->rec_tail, cap);
    const int64_t C = c->L.capacity, mb = c->L.max_bodies, nb = c->n_bodies;
    std::vector<double> rf((size_t)std::max<int64_t>(n, 1) * mb * 3), rm((size_t)std::max<int64_t>(n, 1));
    for (int64_t done = 0; done < n;) {
        const int64_t r = (c->rec_tail + done) % C;
        const int64_t len = std::min(n - done, C - r);
        LBVP3_HIP(c, hipMemcpyAsync(rf.data() + done * mb * 3, c->at<double>(c->L.ring_force) + r * mb * 3,
                                    (size_t)(len * mb * 3) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        LBVP3_HIP(c, hipMemcpyAsync(rm.data() + done, c->at<double>(c->L.ring_mass) + r, (size_t)len * sizeof(double),
                                    hipMemcpyDeviceToHost, c->stream));
        done += len;
    }
    LBVP3_HIP(c, hipStreamSynchronize(c->stream));
    bool finite = true;
    for (int64_t k = 0; k < n; ++k) {
        if (out)
            for (int64_t b = 0; b < nb; ++b)
                for (int d = 0; d < 3; ++d) out[(k * nb + b) * 3 + d] = rf[(k * mb + b) * 3 + d];
        if (mass) mass[k] = rm[k];
        if (!std::isfinite(rm[k])) finite = false;
    }
    if (n_out) *n_out = n;
    if (first_step) *first_step = n > 0 ? (c->rec_tail + 1) * c->p.force_every : 0;
    c->rec_tail += n;
    if (!finite) return c->fail(LBVP_E_UNSTABLE, "non-finite global mass: the run went unstable");
    return LBVP_OK;
}

lbvp_status lbvp3_read_fields(lbvp3_ctx* c, int32_t z0, int32_t n_planes, double* out)
{
    if (!c) return LBVP_E_ARG;
    if (!out) return c->fail(LBVP_E_ARG, "out is NULL");
    if (bad_range(c, z0, n_planes)) return c->fail(LBVP_E_ARG, "plane range outside the grid");
    if (!c->fields_valid) return c->fail(LBVP_E_STATE, "no fields kept since the last init");
    const lbvp3_params& p = c->p;
    const size_t rs = c->rsize();
    const size_t rows = (size_t)n_planes * p.ny, n = rows * p.nx;
    std::vector<char> tmp(std::max<size_t>(n, 1) * rs);
    for (int f = 0; f < 7; ++f) {
        const char* srcp = c->at<char>(c->L.fields) + ((size_t)f * c->L.plane_f + (size_t)z0 * p.ny * c->L.pitch) * rs;
        if (n) {
            LBVP3_HIP(c, hipMemcpy2DAsync(tmp.data(), (size_t)p.nx * rs, srcp, (size_t)c->L.pitch * rs,
                                          (size_t)p.nx * rs, rows, hipMemcpyDeviceToHost, c->stream));
        }
        LBVP3_HIP(c, hipStreamSynchronize(c->stream));
        double* dst = out + (size_t)f * n;
        if (c->is_f64()) std::memcpy(dst, tmp.data(), n * sizeof(double));
        else {
            const float* v = reinterpret_cast<const float*>(tmp.data());
            for (size_t k = 0; k < n; ++k) dst[k] = (double)v[k];
        }
    }
    return LBVP_OK;
}

lbvp_status lbvp3_read_populations(lbvp3_ctx* c, int32_t z0, int32_t n_planes, double* g)
{
    if (!c) return LBVP_E_ARG;
    if (!g) return c->fail(LBVP_E_ARG, "g is NULL");
    if (bad_range(c, z0, n_planes)) return c->fail(LBVP_E_ARG, "plane range outside the grid");
    const lbvp3_params& p = c->p;
    hipStream_t s = c->stream;
    const size_t plane_nodes = (size_t)p.nx * p.ny, N = (size_t)n_planes * plane_nodes;
    for (int32_t k0 = 0; k0 < n_planes; k0 += (int32_t)c->L.stage_planes) {
        const int32_t planes = std::min<int32_t>((int32_t)c->L.stage_planes, n_planes - k0);
        Conv3Args a = conv_args(c, z0 + k0, planes);
        LBVP3_HIP(c, launch_decode3(p.storage, c->at<char>(c->L.lat[c->cur]), a, s));
        const size_t nn = (size_t)planes * plane_nodes;
        for (int q = 0; q < Q; ++q)
            LBVP3_HIP(c, hipMemcpyAsync(g + q * N + (size_t)k0 * plane_nodes, a.pops + q * nn, nn * sizeof(double),
                                        hipMemcpyDeviceToHost, s));
        LBVP3_HIP(c, hipStreamSynchronize(s));
    }
    return LBVP_OK;
}

lbvp_status lbvp3_write_populations(lbvp3_ctx* c, int32_t z0, int32_t n_planes, const double* g)
{
    if (!c) return LBVP_E_ARG;
    if (!g) return c->fail(LBVP_E_ARG, "g is NULL");
    if (bad_range(c, z0, n_planes)) return c->fail(LBVP_E_ARG, "plane range outside the grid");
    const lbvp3_params& p = c->p;
    hipStream_t s = c->stream;
    const size_t plane_nodes = (size_t)p.nx * p.ny, N = (size_t)n_planes * plane_nodes;
    for (int32_t k0 = 0; k0 < n_planes; k0 += (int32_t)c->L.stage_planes) {
        const int32_t planes = std::min<int32_t>((int32_t)c->L.stage_planes, n_planes - k0);
        Conv3Args a = conv_args(c, z0 + k0, planes);
        const size_t nn = (size_t)planes * plane_nodes;
        for (int q = 0; q < Q; ++q)
            LBVP3_HIP(c, hipMemcpyAsync(a.pops + q * nn, g + q * N + (size_t)k0 * plane_nodes, nn * sizeof(double),
                                        hipMemcpyHostToDevice, s));
        LBVP3_HIP(c, launch_encode3(p.storage, c->at<char>(c->L.lat[c->cur]), a, s));
        LBVP3_HIP(c, hipStreamSynchronize(s));
    }
    return LBVP_OK;
}

lbvp_status lbvp3_set_launch(lbvp3_ctx* c, int32_t vec, int32_t block)
{
    if (!c) return LBVP_E_ARG;
    if (!vec_supported(c->p.storage, vec)) return c->fail(LBVP_E_ARG, "vec not built for this storage type");
    if (block != 64 && block != 128 && block != 256) return c->fail(LBVP_E_ARG, "block must be 64, 128 or 256");
    LBVP3_HIP(c, hipStreamSynchronize(c->stream));   // running steps still read the old tables
    Launch3 l = make_launch(c->p.nx, c->L.rows, vec, block);
    l.band = c->launch.band;
    c->args_changed();
    return apply_launch(c, l);
}

lbvp_status lbvp3_get_launch(const lbvp3_ctx* c, int32_t* vec, int32_t* block)
{
    if (!c) return LBVP_E_ARG;
    if (vec) *vec = c->launch.vec;
    if (block) *block = c->launch.block;
    return LBVP_OK;
}

lbvp_status lbvp3_set_tile_band(lbvp3_ctx* c, int32_t band)
{
    if (!c) return LBVP_E_ARG;
    if (band < 0 || band > MAX_TILE_BAND || (band & (band - 1)) != 0)
        return c->fail(LBVP_E_ARG, "band must be 0 or a power of two up to 65536");
    c->launch.band = band;
    fill_args(c, c->a64);
    fill_args(c, c->a32);
    c->args_changed();
    return LBVP_OK;
}

lbvp_status lbvp3_get_tile_band(const lbvp3_ctx* c, int32_t* band)
{
    if (!c || !band) return LBVP_E_ARG;
    *band = c->launch.band;
    return LBVP_OK;
}

int64_t lbvp3_step_count(const lbvp3_ctx* c) { return c ? c->step : -1; }

lbvp_status lbvp3_synchronize(lbvp3_ctx* c)
{
    if (!c) return LBVP_E_ARG;
    LBVP3_HIP(c, hipStreamSynchronize(c->stream));
    return LBVP_OK;
}

lbvp_status lbvp3_destroy(lbvp3_ctx* c)
{
    if (!c) return LBVP_E_ARG;
    (void)hipStreamSynchronize(c->stream);
    if (c->mem) (void)hipFree(c->mem);
    delete c;
    return LBVP_OK;
}

const char* lbvp3_last_error(const lbvp3_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

lbvp_status lbvp3_save_state(lbvp3_ctx* c, void* buf, size_t cap, size_t* size)
{
    if (!c) return LBVP_E_ARG;
    if (!size) return c->fail(LBVP_E_ARG, "size is NULL");
    if (c->rec_head != c->rec_tail) return c->fail(LBVP_E_STATE, "drain the force records first");
    const State3Header h = state3_header(c);
    *size = (size_t)state3_bytes(h);
    if (!buf || cap < *size) return c->fail(LBVP_E_NOMEM, "buffer too small for the state (see *size)");
    hipStream_t s = c->stream;
    char* o = static_cast<char*>(buf);
    std::memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    LBVP3_HIP(c, hipMemcpyAsync(o, c->at<char>(c->L.lat[c->cur]), h.lat_bytes, hipMemcpyDeviceToHost, s));
    o += h.lat_bytes;
    LBVP3_HIP(c, hipMemcpyAsync(o + h.mask_bytes + h.body_bytes, c->at<char>(c->L.fields), h.field_bytes,
                                hipMemcpyDeviceToHost, s));
    std::memcpy(o, c->mask_host.data(), h.mask_bytes);
    o += h.mask_bytes;
    if (h.body_bytes) std::memcpy(o, c->bodies_host.data(), h.body_bytes);
    LBVP3_HIP(c, hipStreamSynchronize(s));
    return LBVP_OK;
}

lbvp_status lbvp3_load_state(lbvp3_ctx* c, const void* buf, size_t size)
{
    if (!c) return LBVP_E_ARG;
    if (!buf || size < sizeof(State3Header)) return c->fail(LBVP_E_ARG, "not a state blob");
    State3Header h;
    std::memcpy(&h, buf, sizeof(h));
    const State3Header mine = state3_header(c);
    if (std::memcmp(h.magic, STATE3_MAGIC, 8) != 0 || h.version != STATE3_VERSION || h.header_bytes != sizeof(h))
        return c->fail(LBVP_E_ARG, "not a D3Q19 state blob of this version");
    if (h.nx != mine.nx || h.ny != mine.ny || h.nz != mine.nz || h.storage != mine.storage)
        return c->fail(LBVP_E_ARG, "the state is of another grid or storage type");
    if (h.n_bodies < 0 || h.n_bodies > c->L.max_bodies)
        return c->fail(LBVP_E_ARG, "the state holds more bodies than max_bodies");
    if (h.cur < 0 || h.cur > 1 || h.step < 0 || h.records < 0) return c->fail(LBVP_E_ARG, "damaged state counters");
    if (h.lat_bytes != mine.lat_bytes || h.mask_bytes != mine.mask_bytes ||
        h.body_bytes != (uint64_t)h.n_bodies * sizeof(lbvp3_body) || h.field_bytes != mine.field_bytes ||
        size < state3_bytes(h))
        return c->fail(LBVP_E_ARG, "damaged state sizes");
    const char* lat = static_cast<const char*>(buf) + sizeof(h);
    const uint8_t* mask = reinterpret_cast<const uint8_t*>(lat + h.lat_bytes);
    std::vector<lbvp3_body> bodies((size_t)h.n_bodies);
    if (h.body_bytes) std::memcpy(bodies.data(), mask + h.mask_bytes, h.body_bytes);
    const char* fields = reinterpret_cast<const char*>(mask) + h.mask_bytes + h.body_bytes;
    const lbvp_status st = lbvp3_set_mask(c, mask, h.n_bodies, bodies.data());   // validates, synchronizes
    if (st != LBVP_OK) return st;
    hipStream_t s = c->stream;
    const int64_t records = h.records;
    LBVP3_HIP(c, hipMemcpyAsync(c->at<char>(c->L.lat[h.cur]), lat, h.lat_bytes, hipMemcpyHostToDevice, s));
    LBVP3_HIP(c, hipMemcpyAsync(c->at<char>(c->L.fields), fields, h.field_bytes, hipMemcpyHostToDevice, s));
    LBVP3_HIP(c, hipMemcpyAsync(c->fin.rec_count, &records, sizeof(records), hipMemcpyHostToDevice, s));
    LBVP3_HIP(c, launch_zero_i64(c->fin.arrivals, s));
    LBVP3_HIP(c, hipStreamSynchronize(s));
    c->cur = h.cur;
    c->step = h.step;
    c->rec_head = c->rec_tail = h.records;
    c->pending = false;
    c->fields_valid = h.fields_valid != 0;
    return LBVP_OK;
}

lbvp_status lbvp3_batch_create(lbvp3_ctx* const* members, int32_t n, int32_t vec, int32_t block, lbvp3_batch** out)
{
    if (!out || !members || n < 1) {
        g_batch3_error = "members, n >= 1 and out are required";
        return LBVP_E_ARG;
    }
    *out = nullptr;
    for (int32_t d = 0; d < n; ++d)
        if (!members[d]) {
            g_batch3_error = "a member is NULL";
            return LBVP_E_ARG;
        }
    lbvp3_ctx* c0 = members[0];
    for (int32_t d = 0; d < n; ++d) {
        const lbvp3_ctx* c = members[d];
        if (c->p.storage != c0->p.storage || c->stream != c0->stream || c->p.force_every != c0->p.force_every ||
            c->step != c0->step || c->rec_head != c0->rec_head) {
            g_batch3_error = "members differ in storage, stream, force_every or step count";
            return LBVP_E_ARG;
        }
        for (int32_t e = 0; e < d; ++e)
            if (members[e] == c) {
                g_batch3_error = "a context appears twice";
                return LBVP_E_ARG;
            }
    }
    if (vec == 0) vec = c0->launch.vec;
    if (block == 0) block = c0->launch.block;
    if (!vec_supported(c0->p.storage, vec) || (block != 64 && block != 128 && block != 256)) {
        g_batch3_error = "vec or block not built for this storage type (see lbvp3_set_launch)";
        return LBVP_E_ARG;
    }
    for (int32_t d = 0; d < n; ++d) {   // every member tiled for the batch's shape
        lbvp3_ctx* c = members[d];
        if (c->launch.vec != vec || c->launch.block != block) {
            const lbvp_status st = lbvp3_set_launch(c, vec, block);
            if (st != LBVP_OK) {
                g_batch3_error = "launch shape: " + c->err;
                return st;
            }
        }
    }
    lbvp3_batch* b = new (std::nothrow) lbvp3_batch();
    if (!b) {
        g_batch3_error = "host allocation failed";
        return LBVP_E_NOMEM;
    }
    b->members.assign(members, members + n);
    b->stream = c0->stream;
    b->storage = c0->p.storage;
    b->vec = vec;
    b->block = block;
    std::vector<int32_t> tile_domain, tile_start((size_t)n);
    for (int32_t d = 0; d < n; ++d) {
        tile_start[d] = (int32_t)tile_domain.size();
        tile_domain.insert(tile_domain.end(), (size_t)members[d]->launch.n_tiles, d);
    }
    b->total_tiles = (int32_t)tile_domain.size();
    b->tiles_per_xcd = (b->total_tiles + N_XCD - 1) / N_XCD;
    b->member_bytes = (b->storage == LBVP_F64 ? sizeof(Member3<double>) : sizeof(Member3<float>)) * (size_t)n;
    b->off_domain = align_up(b->member_bytes, 256);
    b->off_start = align_up(b->off_domain + tile_domain.size() * 4, 256);
    const size_t bytes = b->off_start + tile_start.size() * 4;
    b->image.assign(b->member_bytes, 0);
    hipError_t e = hipMalloc(&b->dev, bytes);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->dev + b->off_domain, tile_domain.data(), tile_domain.size() * 4, hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->dev + b->off_start, tile_start.data(), tile_start.size() * 4, hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);   // the host tables go out of scope
    if (e != hipSuccess) {
        g_batch3_error = std::string("device tables: ") + hipGetErrorString(e);
        delete b;
        return e == hipErrorOutOfMemory ? LBVP_E_NOMEM : LBVP_E_DEVICE;
    }
    *out = b;
    return LBVP_OK;
}

lbvp_status lbvp3_batch_step(lbvp3_batch* b, int64_t n_steps, uint32_t flags)
{
    if (!b) return LBVP_E_ARG;
    if (n_steps < 0) return b->fail(LBVP_E_ARG, "n_steps < 0");
    if (flags & ~KNOWN_STEP_FLAGS) return b->fail(LBVP_E_ARG, "unknown step flag");
    if ((flags & LBVP_GRAPH) && !b->stream) return b->fail(LBVP_E_ARG, "LBVP_GRAPH needs a stream other than the null stream");
    if (n_steps == 0) return LBVP_OK;
    lbvp3_ctx* c0 = b->members[0];
    const int64_t fe = c0->p.force_every;
    for (lbvp3_ctx* c : b->members) {
        if (c->step != c0->step || c->rec_head != c0->rec_head)
            return b->fail(LBVP_E_STATE, "members went out of step (one was stepped alone)");
        if (c->launch.vec != b->vec || c->launch.block != b->block)
            return b->fail(LBVP_E_STATE, "a member's launch shape was changed after the batch was made");
        if (fe > 0) {
            const int64_t new_recs = (c->step + n_steps) / fe - c->step / fe;
            if (c->rec_head + new_recs - c->rec_tail > c->L.capacity)
                return b->fail(LBVP_E_STATE, "a member's force records would overflow its ring; drain them first");
        }
    }
    // the member block: rewritten once the previous call's steps (which read it) are done
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return b->hip_fail(e, "hipStreamSynchronize");
    for (lbvp3_ctx* c : b->members) {
        c->a64.fin = c->fin;
        c->a32.fin = c->fin;
    }
    if (b->storage == LBVP_F64) write_member_images<double>(b);
    else write_member_images<float>(b);
    e = hipMemcpyAsync(b->dev, b->image.data(), b->member_bytes, hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return b->hip_fail(e, "member upload");
    const bool keep = (flags & LBVP_KEEP_FIELDS) != 0;
    const int32_t n = (int32_t)b->members.size();
    Batch3Launch L{};
    L.total_tiles = b->total_tiles;
    L.tiles_per_xcd = b->tiles_per_xcd;
    L.band_log2 = band_log2(b->band);
    L.tile_domain = reinterpret_cast<const int32_t*>(b->dev + b->off_domain);
    L.tile_start = reinterpret_cast<const int32_t*>(b->dev + b->off_start);
    L.members = b->dev;
    L.n_members = n;
    // steps k0 .. k0 + n - 1 of the call (the members' parity flips with k),
    // then the run's last record summed in one launch
    auto run = [&](int64_t k0, int64_t n_run, bool keep_last) -> lbvp_status {
    for (int64_t k = k0; k < k0 + n_run; ++k) {
        const int64_t next = c0->step + 1;
        const bool record = fe > 0 && next % fe == 0;
        const bool keep_here = keep_last && k == k0 + n_run - 1;
        const int32_t part_buf = (int32_t)(c0->rec_head & 1);
        L.flip = (int32_t)(k & 1);
        L.part_buf = part_buf;
        L.fin_buf = c0->pending ? c0->pending_buf : -1;
        L.n_fin = L.fin_buf >= 0 ? (n + N_XCD - 1) / N_XCD * N_XCD : 0;
        e = launch_step3_batch(b->storage, b->vec, b->block, record, keep_here, L, b->stream);
        if (e != hipSuccess) return b->hip_fail(e, "batch step kernel launch");
        for (lbvp3_ctx* c : b->members) {
            c->pending = record;
            if (record) {
                c->pending_buf = part_buf;
                c->rec_head += 1;
            }
            if (keep_here) c->fields_valid = true;
            c->cur ^= 1;
            c->step = next;
        }
    }
    if (c0->pending) {   // the last record of the run, every member's in one launch
        L.fin_buf = c0->pending_buf;
        e = launch_finalize3_members(b->storage, L, b->stream);
        if (e != hipSuccess) return b->hip_fail(e, "finalize kernel launch");
        for (lbvp3_ctx* c : b->members) c->pending = false;
    }
    return LBVP_OK;
    };
    if (!(flags & LBVP_GRAPH)) return run(0, n_steps, keep);
    // through graphs: runs of up to GRAPH_CHUNK steps, each captured once per
    // distinct launch sequence (length, parity within the call, record phase and
    // buffer) and replayed; the member block was uploaded above, outside any
    // capture, and is read by the replayed kernels
    for (int64_t done = 0; done < n_steps;) {
        const int64_t n_run = std::min(GRAPH_CHUNK, n_steps - done);
        const bool keep_here = keep && done + n_run == n_steps;
        lbvp_host::GraphKey key;   // every run starts with its records summed
        key.n = n_run;
        key.keep = keep_here;
        key.cur = (int32_t)(done & 1);
        key.phase = fe > 0 ? c0->step % fe : 0;
        key.rec = (int32_t)(c0->rec_head & 1);
        key.gen = b->gen;
        hipGraphExec_t x = b->graphs.find(key);
        if (x) {
            e = hipGraphLaunch(x, b->stream);
            if (e != hipSuccess) return b->hip_fail(e, "hipGraphLaunch");
            // the members' bookkeeping exactly as the captured launches advanced it
            const int64_t step0 = c0->step;
            const int64_t recs = fe > 0 ? (step0 + n_run) / fe - step0 / fe : 0;
            for (lbvp3_ctx* c : b->members) {
                c->cur = (c->cur + (int)(n_run & 1)) & 1;
                c->step = step0 + n_run;
                c->rec_head += recs;
                c->pending = false;
                if (recs > 0) c->pending_buf = (int32_t)((c->rec_head - 1) & 1);
                if (keep_here) c->fields_valid = true;
            }
        } else {
            struct Saved { int cur; int64_t step, head; bool pending, fields; int32_t buf; };
            std::vector<Saved> saved;
            for (lbvp3_ctx* c : b->members)
                saved.push_back({c->cur, c->step, c->rec_head, c->pending, c->fields_valid, c->pending_buf});
            auto restore = [&]() {
                for (size_t i = 0; i < b->members.size(); ++i) {
                    lbvp3_ctx* c = b->members[i];
                    c->cur = saved[i].cur;
                    c->step = saved[i].step;
                    c->rec_head = saved[i].head;
                    c->pending = saved[i].pending;
                    c->fields_valid = saved[i].fields;
                    c->pending_buf = saved[i].buf;
                }
            };
            e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return b->hip_fail(e, "hipStreamBeginCapture");
            const lbvp_status st = run(done, n_run, keep_here);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->stream, &g);
            if (st != LBVP_OK || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                restore();
                return st != LBVP_OK ? st : b->hip_fail(e, "hipStreamEndCapture");
            }
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                restore();
                return b->hip_fail(e, "hipGraphInstantiate");
            }
            b->graphs.put(key, x, b->stream);
            e = hipGraphLaunch(x, b->stream);
            if (e != hipSuccess) {
                restore();
                return b->hip_fail(e, "hipGraphLaunch");
            }
        }
        done += n_run;
    }
    return LBVP_OK;
}

lbvp_status lbvp3_batch_set_tile_band(lbvp3_batch* b, int32_t band)
{
    if (!b) return LBVP_E_ARG;
    if (band < 0 || band > MAX_TILE_BAND || (band & (band - 1)) != 0)
        return b->fail(LBVP_E_ARG, "band must be 0 or a power of two up to 65536");
    if (band != b->band) {   // the band is baked into captured launches
        b->graphs.clear(b->stream);
        b->gen += 1;
    }
    b->band = band;
    return LBVP_OK;
}

lbvp_status lbvp3_batch_get_tile_band(const lbvp3_batch* b, int32_t* band)
{
    if (!b || !band) return LBVP_E_ARG;
    *band = b->band;
    return LBVP_OK;
}

lbvp_status lbvp3_batch_destroy(lbvp3_batch* b)
{
    if (!b) return LBVP_OK;
    delete b;
    return LBVP_OK;
}

const char* lbvp3_batch_last_error(const lbvp3_batch* b) { return b ? b->err.c_str() : g_batch3_error.c_str(); }


// Scratch contexts of the members' parameters, masks and bodies (fluid at rest),
// destroyed with this object.
struct Tune3Scratch {
    std::vector<lbvp3_ctx*> ctx;
    ~Tune3Scratch()
    {
        for (lbvp3_ctx* c : ctx) (void)lbvp3_destroy(c);
    }
};

lbvp_status tune3_fail(lbvp_status st, const std::string& m)
{
    g_tune3_error = m;
    return st;
}

lbvp_status lbvp3_tune(lbvp3_ctx* const* members, int32_t n, int32_t steps, uint32_t flags, lbvp3_tune_row* rows,
                       int32_t cap, int32_t* n_rows, int32_t* best)
{
    if (!members || n < 1 || steps < 1 || cap < 0 || (cap > 0 && !rows) || !n_rows || !best ||
        (flags & ~LBVP_TUNE_FRESH))
        return tune3_fail(LBVP_E_ARG, "members, n >= 1, steps >= 1, rows[cap], n_rows, best and known flags are required");
    for (int32_t d = 0; d < n; ++d)
        if (!members[d]) return tune3_fail(LBVP_E_ARG, "a member is NULL");
    const lbvp3_ctx* c0 = members[0];
    std::string key = std::to_string(c0->p.storage) + "/" + std::to_string(c0->p.force_every) + "/" +
                      std::to_string(steps);
    for (int32_t d = 0; d < n; ++d) {
        const lbvp3_ctx* c = members[d];
        if (c->p.storage != c0->p.storage || c->stream != c0->stream || c->p.force_every != c0->p.force_every)
            return tune3_fail(LBVP_E_ARG, "members differ in storage, stream or force_every");
        // the pick is kept per grid shape, body count and mask (FNV-1a of the
        // body ids): members with other solids may tune differently
        uint64_t h = 1469598103934665603ull;
        for (uint8_t v : c->mask_host) h = (h ^ v) * 1099511628211ull;
        key += "/" + std::to_string(c->p.nx) + "x" + std::to_string(c->p.ny) + "x" + std::to_string(c->p.nz) + ":" +
               std::to_string(c->n_bodies) + ":" + std::to_string(h);
    }
    std::vector<lbvp3_tune_row> table;
    int32_t pick = 0;
    bool cached = false;
    if (!(flags & LBVP_TUNE_FRESH)) {
        std::lock_guard<std::mutex> g(g_tune3_mu);
        auto it = g_tune3_cache.find(key);
        if (it != g_tune3_cache.end()) {
            table = it->second.first;
            pick = it->second.second;
            cached = true;
        }
    }
    if (!cached) {
        hipStream_t stream = c0->stream;
        const int64_t warm = std::max(1, steps / 4), per_run = warm + 3 * (int64_t)steps;
        Tune3Scratch sc;
        int64_t nodes = 0;
        for (int32_t d = 0; d < n; ++d) {
            const lbvp3_ctx* c = members[d];
            lbvp3_params p = c->p;
            p.force_capacity = p.force_every > 0 ? per_run / p.force_every + 16 : 0;
            lbvp3_ctx* s = nullptr;
            lbvp_status st = lbvp3_create(&p, stream, &s);
            if (st != LBVP_OK) return tune3_fail(st, "scratch context: " + g_create_error);
            sc.ctx.push_back(s);
            if (!c->mask_host.empty())   // else all fluid, as the member
                st = lbvp3_set_mask(s, c->mask_host.data(), c->n_bodies,
                                    c->bodies_host.empty() ? nullptr : c->bodies_host.data());
            if (st == LBVP_OK) st = lbvp3_init_equilibrium(s, nullptr, nullptr, nullptr, nullptr);
            if (st != LBVP_OK) return tune3_fail(st, "scratch context: " + s->err);
            nodes += (int64_t)p.nx * p.ny * p.nz;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            return tune3_fail(LBVP_E_DEVICE, "hipEventCreate failed");
        }
        lbvp_status st = LBVP_OK;
        std::string skipped;   // candidates a member's grid does not admit
        for (int32_t vec : {1, 2, 4, 8}) {
            if (!vec_supported(c0->p.storage, vec)) continue;
            for (int32_t block : BLOCKS)
                for (int32_t band : {0, 2, 4, 16}) {
                    lbvp3_batch* b = nullptr;
                    std::string why;
                    for (lbvp3_ctx* s : sc.ctx) {
                        if (st == LBVP_OK) st = lbvp3_set_launch(s, vec, block);
                        if (st == LBVP_OK && n == 1) st = lbvp3_set_tile_band(s, band);
                        if (st != LBVP_OK && why.empty()) why = s->err;
                    }
                    if (st == LBVP_OK && n > 1) {
                        st = lbvp3_batch_create(sc.ctx.data(), n, vec, block, &b);
                        if (st == LBVP_OK) st = lbvp3_batch_set_tile_band(b, band);
                        if (st != LBVP_OK) why = lbvp3_batch_last_error(b);
                    }
                    if (st == LBVP_E_ARG) {   // not a failure of the run: skip the candidate
                        if (b) (void)lbvp3_batch_destroy(b);
                        skipped += " (" + std::to_string(vec) + ", " + std::to_string(block) + ", " +
                                   std::to_string(band) + "): " + why + ";";
                        st = LBVP_OK;
                        continue;
                    }
                    auto run = [&](int64_t k) {
                        return n > 1 ? lbvp3_batch_step(b, k, 0) : lbvp3_step(sc.ctx[0], k, 0);
                    };
                    float best_ms = 0.0f;
                    if (st == LBVP_OK) st = run(warm);
                    for (int rep = 0; rep < 3 && st == LBVP_OK; ++rep) {
                        float ms = 0.0f;
                        if (hipEventRecord(e0, stream) != hipSuccess) st = LBVP_E_DEVICE;
                        if (st == LBVP_OK) st = run(steps);
                        if (st == LBVP_OK && (hipEventRecord(e1, stream) != hipSuccess ||
                                              hipEventSynchronize(e1) != hipSuccess ||
                                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                            st = LBVP_E_DEVICE;
                        if (st == LBVP_OK && (rep == 0 || ms < best_ms)) best_ms = ms;
                    }
                    if (b) (void)lbvp3_batch_destroy(b);
                    for (lbvp3_ctx* s : sc.ctx)   // drain the records of this candidate
                        if (st == LBVP_OK) {
                            int64_t got = 0, first = 0;
                            const lbvp_status fs = lbvp3_forces(s, nullptr, nullptr, per_run, &got, &first);
                            if (fs != LBVP_OK && fs != LBVP_E_UNSTABLE) st = fs;
                        }
                    if (st != LBVP_OK) break;
                    const double ms_step = (double)best_ms / steps;
                    table.push_back(lbvp3_tune_row{vec, block, band, ms_step, (double)nodes / (ms_step * 1e3)});
                }
            if (st != LBVP_OK) break;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != LBVP_OK) return tune3_fail(st, "tuning run failed");
        if (table.empty()) return tune3_fail(LBVP_E_ARG, "no launch shape admitted by every member:" + skipped);
        g_tune3_error = skipped.empty() ? "" : "skipped:" + skipped;
        for (int32_t i = 1; i < (int32_t)table.size(); ++i)
            if (table[i].ms_per_step < table[pick].ms_per_step) pick = i;
        std::lock_guard<std::mutex> g(g_tune3_mu);
        g_tune3_cache[key] = {table, pick};
    }
    const int32_t k = std::min<int32_t>(cap, (int32_t)table.size());
    for (int32_t i = 0; i < k; ++i) rows[i] = table[i];
    *n_rows = (int32_t)table.size();
    *best = pick;
    return LBVP_OK;
}

const char* lbvp3_tune_last_error(void) { return g_tune3_error.c_str(); }

}  // extern "C"
