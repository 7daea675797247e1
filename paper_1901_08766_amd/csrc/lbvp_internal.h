// lbvp_internal.h -- kernel argument blocks and launchers shared by the host
// side of liblbvp (lbvp_api.hip, lbvp_pool.hip) and its kernels
// (lbvp_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbvp.h"

namespace lbvp {

// One workgroup of `block` threads updates one tile of block * vec consecutive
// nodes of a row, vec nodes per thread. Workgroups are dealt to the 8 XCDs
// round-robin by block id; the launch maps blocks to tiles (xcd_tile) so that
// each XCD sweeps runs of neighbouring tiles, which then share its L2: one
// contiguous eighth of the domain per XCD (band_log2 = -1) or bands of
// 2^band_log2 tiles.
constexpr int N_XCD = 8;
constexpr int MAX_BLOCK = 256;
constexpr int MIN_BLOCK = 64;
constexpr int MAX_TILE_BAND = 1 << 16;
// Body table row: the centre split into its nearest integer and the remainder
// (cx_int, cy_int, cx_frac, cy_frac), then vx, vy, omega, all in the arithmetic
// type: x - c is then (x - c_int) - c_frac, exact up to one rounding of a
// remainder of at most 1/2, at any coordinate below 2^24.
constexpr int BODY_STRIDE = 7;
constexpr int FIN_THREADS = 256;
constexpr int MAX_MOVING = 8;       // bodies of a domain with moving masks
constexpr int POSE_STRIDE = 8;      // doubles per body pose row
constexpr int POSE_ROWS = 1024;     // time levels per uploaded pose table

enum Side : int32_t { SIDE_PERIODIC = 0, SIDE_INFLOW_EQ = 1, SIDE_OUTFLOW = 2, SIDE_NEIGHBOR = 3 };

// Storage codes (match lbvp_storage).
enum Storage : int32_t { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

// Sums one force record: the per-wavefront mass partials and the (tile, body)
// force partials of partial buffer `buf`, in a fixed order, into ring slot
// rec_count % capacity. The partials are double-buffered so that the record of
// step k can be summed while step k + 1 writes its own.
struct FinalizeArgs {
    int32_t n_bodies, max_bodies, n_mass;   // n_mass: wavefronts of a launch
    int64_t capacity;
    double mass_offset;             // rho0 * nx * ny
    const int32_t* body_slot_ptr;   // [n_bodies + 1]
    const int32_t* body_slots;      // slots of each body in tile order
    const double* slot_force;       // [2][slot_stride / 2][2]
    const double* mass_part;        // [2][mass_stride]
    int64_t slot_stride, mass_stride;
    double* ring_force;             // [capacity][max_bodies][2]
    double* ring_mass;              // [capacity]
    int64_t* rec_count;             // records written so far
};

template <typename R>
struct StepArgs {
    int32_t nx, ny;
    int32_t vec, block;             // nodes per thread, threads per block
    int32_t tile_w, tile_rows;      // a tile: tile_rows rows of tile_w nodes (tile_w * tile_rows = vec * block)
    int32_t tiles_x, n_tiles, tiles_per_xcd;
    int32_t band_log2;  // block -> tile order (xcd_tile): -1 eighths, else bands of 2^band_log2 tiles
    int32_t west, east;
    int32_t part_buf;   // partial buffer a recording step writes
    int32_t fin_buf;    // partial buffer whose record a leading block of the launch sums, or -1
    int32_t off32;      // a lattice spans fewer than 2^32 bytes: per-lane offsets fit 32 bits
    int64_t pitch;      // elements per row of one population, of the mask and of a field
    int64_t plane;      // elements between the rows of populations q and q + 1 (= pitch)
    int64_t lstride;    // elements between lattice rows j and j + 1 (= 9 pitch)
    int64_t plane_f;    // elements between field planes
    R rho0;
    R om_p, om_m;       // 1/tau_plus, 1/tau_minus
    R k_p, k_m;         // 1 - 1/(2 tau_plus), 1 - 1/(2 tau_minus)
    R vp_c;             // 1 / (2 eta + 1): the chi = 1 value of chi / (2 eta + chi)
    // the collision of the 2-byte storage types, regrouped per population pair
    // (collide_node_lowp): g_a = c1 h_a + c2 h_opp(a) + E+ + E-
    R c1, c2;           // 1 - (om_p + om_m) / 2, (om_m - om_p) / 2
    R om_p1;            // 1 - om_p
    R om_p45, om_p15;   // 9/2 om_p, 3/2 om_p
    R om_m3;            // 3 om_m
    R k_p9, k_p3, k_m3; // 9 k_p, 3 k_p, 3 k_m
    R fbx, fby;         // body force
    R fbx18, fby18;     // 18 F_b: the body-force half step in units of 36 j
    R feq_in[9];        // (f^eq(rho_in, u_in) - w rho0) / w of an INFLOW_EQ side
    const uint8_t* mask;
    const R* bodies;    // [(n_bodies + 1)][BODY_STRIDE] (body_table_bytes); row 0 all zero (fluid)
    const int32_t* tile_slot_ptr;   // [n_tiles + 1]
    const int32_t* slot_body;       // [n_slots]
    double* slot_force;             // [2][n_slots][2]
    double* mass_part;              // [2][n_tiles * block / 64]
    R* fields;                      // [5][plane_f]
    void* ghost_w;                  // AA layout: [3][ny] zero-gradient ghost columns (storage type)
    void* ghost_e;
    void* lat0;                     // batched launches: the domain's lattices and which one is
    void* lat1;                     // current (two-lattice pull; the AA layout uses lat0 only)
    int32_t cur;
    FinalizeArgs fin;
    // moving bodies: pose[(row * MAX_MOVING + b) * POSE_STRIDE + k] holds body b's
    // pose at the time level of table row `row`, k = 0..6: cos th, sin th, cx(t),
    // cy(t), cx(0), cy(0) with th = omega t, c(t) = c(0) + V t, and the square
    // of a radius about c(t) outside which no node can belong to the body. A
    // launch that is the k-th step of a run takes row *pose_base + k, with k =
    // pose_k (single-domain launches) or BatchLaunch::pose_k; the device value
    // pose_base is advanced after every run, so captured runs replay correctly.
    // n_moving = 0 for fixed masks
    int32_t n_moving;
    int32_t pose_k;
    const int64_t* pose_base;
    const double* pose;
};

// A launch over many domains (k_step_batch).
struct BatchLaunch {
    int32_t total_tiles, tiles_per_xcd;
    int32_t band_log2;              // block -> tile order over all tiles (xcd_tile)
    int32_t flip;                   // lattice parity of this step relative to StepArgs::cur
    int32_t part_buf, fin_buf;      // as in StepArgs, for every domain of the batch
    int32_t n_domains;
    int32_t n_fin;                  // leading blocks that sum the fin_buf records: n_domains
                                    // rounded up to a multiple of 8, or 0 if fin_buf < 0
    int32_t pose_k;                 // this launch's step within the run (moving bodies)
    int32_t off32;                  // every member's StepArgs::off32
    const int32_t* tile_domain;     // [total_tiles] domain of each tile
    const int32_t* tile_start;      // [n_domains] first tile of each domain
    const void* args;               // StepArgs<R>[n_domains]
};

// One cut between two slabs (lbvp_halo_exchange): west's column nx - 1
// populations with e_x = +1 into east's west halo (its lattice's column
// pitch - 1), east's column 0 populations with e_x = -1 into west's east halo
// (column nx); both in the slabs' current lattices.
struct HaloLink {
    const void* w_lat;
    const void* e_lat;
    void* e_lat_w;      // = e_lat, written
    void* w_lat_w;      // = w_lat, written
    int64_t w_lstride, w_plane, e_lstride, e_plane, e_pitch;
    int32_t w_nx;
};
constexpr int MAX_HALO_LINKS = 32;   // HaloArgs stays within the 4 KB of kernel arguments
struct HaloArgs {
    int32_t n_links, ny;
    HaloLink link[MAX_HALO_LINKS];
};

// The cuts of a batch (lbvp_batch_set_halo): member indices of each link; the
// lattices, halos and strides come from the members' step arguments in the
// batch's device block, with the lattice parity `flip` of the coming step.
struct BatchHalo {
    int32_t n_links, ny, flip;
    int32_t w[MAX_HALO_LINKS], e[MAX_HALO_LINKS];
    const void* args;   // StepArgs<R>[members]
};

struct GhostArgs {
    int32_t nx, ny;
    int32_t west_outflow, east_outflow;
    int64_t pitch, plane, lstride;
    void* ghost_w;
    void* ghost_e;
};

// Step kinds (see lbvp_kernels.hip): two-lattice pull, AA push (even step
// count), AA local (odd step count).
enum StepMode : int32_t { MODE_PULL = 0, MODE_AA_PUSH = 1, MODE_AA_LOCAL = 2 };

struct ConvArgs {
    int32_t nx, rows, row0;
    int64_t pitch, plane, lstride, plane_f;
    double rho0;
    int32_t swap;       // AA layout: population q lives in slot opp(q)
    const double* rho;  // staged [rows][nx] or null
    const double* ux;
    const double* uy;
    double* pops;       // staged [9][rows][nx]
};

// nodes per thread of the vector form of the step for a storage type (16 bytes)
int vector_width(int32_t storage);

// launchers (lbvp_kernels.hip); all return the launch status
hipError_t launch_step(int32_t storage, int32_t mode, bool record, bool fields, const void* src, void* dst,
                       const void* step_args, hipStream_t s);
// the same with the mask moved to the step's time level (one node per thread)
hipError_t launch_step_moving(int32_t storage, int32_t mode, bool record, bool fields, const void* src, void* dst,
                              const void* step_args, hipStream_t s);
hipError_t launch_aa_ghosts(int32_t storage, const void* lat, const GhostArgs& a, hipStream_t s);
hipError_t launch_step_batch(int32_t storage, int32_t vec, int32_t block, int32_t mode, bool record, bool fields,
                             bool moving, const BatchLaunch& b, hipStream_t s);
// moving bodies: advance the pose table row of a context (base) or of every
// moving member of a batch (their StepArgs in args) by n steps
hipError_t launch_pose_advance(int64_t* base, int64_t n, hipStream_t s);
hipError_t launch_pose_advance_batch(int32_t storage, const void* args, int32_t n_domains, int64_t n, hipStream_t s);
hipError_t launch_finalize_batch(const FinalizeArgs* fin_dev, int32_t n, int32_t buf, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, int32_t buf, hipStream_t s);
hipError_t launch_init(int32_t storage, void* lat, void* fields, const ConvArgs& a, hipStream_t s);
hipError_t launch_decode(int32_t storage, const void* lat, const ConvArgs& a, hipStream_t s);
hipError_t launch_encode(int32_t storage, void* lat, const ConvArgs& a, hipStream_t s);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);
hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s);
hipError_t launch_halo(int32_t storage, const HaloArgs& h, hipStream_t s);
hipError_t launch_halo_batch(int32_t storage, const BatchHalo& h, hipStream_t s);

// host-side pieces the serving pool builds on (lbvp_api.hip)
// An empty batch of the given kind on a stream; members come with batch_set_members.
lbvp_status batch_new(hipStream_t stream, int32_t storage, uint32_t layout_flags, int32_t force_every, int32_t vec,
                      int32_t block, lbvp_batch** out);
// Replace a batch's members (same checks as lbvp_batch_create); no stream wait
// unless the batch's device block has to grow.
lbvp_status batch_set_members(lbvp_batch* b, lbvp_ctx* const* members, int32_t n);
// Move an idle context to another stream (no work of it may be pending).
void ctx_rebind_stream(lbvp_ctx* c, hipStream_t s);

}  // namespace lbvp
