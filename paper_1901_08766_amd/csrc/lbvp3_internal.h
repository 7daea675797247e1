// lbvp3_internal.h -- argument blocks and launchers of the D3Q19 step, shared by
// its host side (lbvp3_api.hip) and its kernels (lbvp3_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbvp3.h"

namespace lbvp3 {

constexpr int Q = 19;
constexpr int N_XCD = 8;
constexpr int FIN_THREADS = 256;
constexpr int N_LEAD = 32;   // blocks that sum one record, a multiple of the 8 XCDs
constexpr int MAX_TILE_BAND = 1 << 16;
// Body table row, in the arithmetic type: the centre split into its nearest
// integer and the remainder (x - c = (x - c_int) - c_frac, exact up to one
// rounding of a remainder of at most 1/2), then v and omega.
constexpr int BODY3_STRIDE = 12;

// Velocity components of the 19 directions in the interface order: rest, the
// faces +x -x +y -y +z -z, then the edges as (opposite) pairs in the xy, xz and
// yz planes. Device code indexes them with compile-time indices only.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// Sums one force record: the per-wavefront mass partials and the (tile, body)
// force partials of partial buffer `buf`, in a fixed order, into ring slot
// rec_count % capacity. N_LEAD blocks each sum a fixed slice into a row of
// `stage`; the last to arrive (counted in `arrivals`) adds the rows in block
// order. The partials are double-buffered so that the record of one step is
// summed by leading blocks of the next step's launch while that step writes the
// other buffer.
struct Fin3Args {
    int32_t n_bodies, max_bodies, n_mass;   // n_mass: wavefronts of a step launch
    int64_t capacity;
    double mass_offset;             // rho0 * nx * ny * nz
    const int32_t* body_slot_ptr;   // [n_bodies + 1]
    const int32_t* body_slots;      // slots of each body in tile order
    const double* slot_force;       // [2][slot_stride]: [n_slots][3] per buffer
    const double* mass_part;        // [2][mass_stride]
    int64_t slot_stride, mass_stride;
    double* ring_force;             // [capacity][max_bodies][3]
    double* ring_mass;              // [capacity]
    int64_t* rec_count;             // records written so far
    double* stage;                  // [N_LEAD][1 + 3 max_bodies] slice sums
    int64_t* arrivals;              // slices summed of the record in progress (0 between records)
};

// One workgroup updates one tile: tile_rows consecutive lattice rows of tile_w
// nodes (vec nodes per thread), a lattice row being the nx nodes of one (y, z);
// rows are numbered r = z * ny + y.
template <typename R>
struct Step3Args {
    int32_t nx, ny, nz;
    int32_t vec, block, tile_w, tile_rows;
    int32_t tiles_x, n_tiles, tiles_per_xcd;
    int32_t band_log2;              // block -> tile order (xcd_tile): -1 eighths, else bands of 2^band_log2 tiles
    int32_t west, east;             // lbvp_bc of the x sides
    int64_t pitch;                  // elements per population row, mask row and field row
    int64_t lstride;                // elements between lattice rows r and r + 1 (= 19 pitch)
    int64_t plane_f;                // elements between field planes (= ny nz pitch)
    R rho0;
    R om_p, om_m;                   // 1/tau_plus, 1/tau_minus
    R k_p, k_m;                     // 1 - 1/(2 tau_plus), 1 - 1/(2 tau_minus)
    R vp_c;                         // 1 / (2 eta + 1)
    R fb[3];                        // body force
    R fb18[3];                      // 18 F_b: the half step in units of 36 j
    R feq_in[Q];                    // (f^eq(rho_in, u_in) - w rho0) / w of an INFLOW_EQ side
    const uint8_t* mask;            // [ny nz][pitch]
    const R* bodies;                // [(max_bodies + 1)][BODY3_STRIDE]: c_int, c_frac, v, omega; row 0 all zero
    const int32_t* tile_slot_ptr;   // [n_tiles + 1]
    const int32_t* slot_body;       // [n_slots]
    double* slot_force;             // [2][fin.slot_stride]
    double* mass_part;              // [2][fin.mass_stride]
    R* fields;                      // [7][plane_f]
    int32_t part_buf;               // partial buffer a recording step writes
    int32_t fin_buf;                // partial buffer whose record a leading block sums, or -1
    Fin3Args fin;
};

struct Conv3Args {
    int32_t nx, ny, plane0, planes;
    int64_t pitch, lstride, plane_f;
    double rho0;
    const double* rho;   // staged [planes][ny][nx] or null
    const double* u[3];
    double* pops;        // staged [19][planes][ny][nx]
};

// A batch member as the batch kernel sees it: its step arguments and lattices,
// and its current lattice when the batch wrote this image (Batch3Launch::flip
// gives each step's parity relative to it).
template <typename R>
struct Member3 {
    Step3Args<R> a;
    void* lat0;
    void* lat1;
    int32_t cur;
};

// One step of every member of a batch: block -> (member, tile) through the tile
// map (tiles of member d are tile_start[d] .. tile_start[d + 1] - 1).
struct Batch3Launch {
    int32_t total_tiles, tiles_per_xcd, band_log2;
    int32_t flip;                   // this step's lattice parity relative to Member3::cur
    int32_t part_buf, fin_buf;      // as in Step3Args, for every member
    int32_t n_members;
    int32_t n_fin;                  // leading blocks, one per member (rounded up to a multiple of
                                    // the 8 XCDs), or 0 if fin_buf < 0
    const int32_t* tile_domain;     // [total_tiles] member of each tile
    const int32_t* tile_start;      // [n_members] first tile of each member
    const void* members;            // Member3<R>[n_members]
};

// nodes per thread the step kernel is built for, per storage type
bool vec_supported(int32_t storage, int32_t vec);

hipError_t launch_step3(int32_t storage, bool record, bool fields, const void* src, void* dst, const void* step_args,
                        hipStream_t s);
hipError_t launch_step3_batch(int32_t storage, int32_t vec, int32_t block, bool record, bool fields,
                              const Batch3Launch& b, hipStream_t s);
hipError_t launch_finalize3(const Fin3Args& a, int32_t buf, hipStream_t s);
// every member's record in partial buffer b.fin_buf summed by one block each
hipError_t launch_finalize3_members(int32_t storage, const Batch3Launch& b, hipStream_t s);
hipError_t launch_init3(int32_t storage, void* lat, void* fields, const Conv3Args& a, hipStream_t s);
hipError_t launch_decode3(int32_t storage, const void* lat, const Conv3Args& a, hipStream_t s);
hipError_t launch_encode3(int32_t storage, void* lat, const Conv3Args& a, hipStream_t s);
hipError_t launch_zero_i64(int64_t* p, hipStream_t s);

}  // namespace lbvp3
