/*
 * lbvp3.h -- C ABI of the three-dimensional (D3Q19) TRT-LBM-VP step in liblbvp.so.
 *
 * The paper (Cui, Wang, Yao, Liu, Yu, arXiv 1901.08766) states its scheme on
 * D2Q9 and names the 3-D extension as its next step (Sec. 4). This interface
 * runs the same algorithm (Sec. 2.2, steps (1)-(7)) on the D3Q19 lattice: pull
 * streaming (eq. streaming), density and intermediate velocity (eqs. rho,
 * rho*velocity-star), the implicit penalization (eqs. d-V, force-density,
 * velocity-r) taken per component, and the TRT collision with split Guo forcing
 * (eqs. TRT-collision, feq, external-force-term, collision-modified) with the
 * D3Q19 velocities and weights 1/3, 1/18, 1/36. One time step is one fused HIP
 * kernel on the device. Lattice units: dx = dy = dz = dt = 1.
 *
 * Conventions (as in lbvp.h, whose status codes, sides and storage types these
 * calls share):
 *  - Every call returns lbvp_status; messages per context (lbvp3_last_error(ctx))
 *    or, for a failed lbvp3_create, per calling thread (lbvp3_last_error(NULL)).
 *  - Host arrays are [nz][ny][nx] with x fastest; node (i, j, k) sits at
 *    x = i, y = j, z = k. Host inputs are caller-owned and copied before the call
 *    returns; host outputs are caller-allocated with the stated sizes.
 *  - Population order: a = 0 rest; 1..6 the faces (+x, -x, +y, -y, +z, -z);
 *    7..18 the edges (+x+y, -x-y, +x-y, -x+y, +x+z, -x-z, +x-z, -x+z, +y+z,
 *    -y-z, +y-z, -y+z); every odd a >= 1 is followed by its opposite.
 *  - The context allocates and owns its device memory. The HIP stream given to
 *    lbvp3_create is borrowed; lbvp3_step only enqueues work on it, and faults
 *    surface at the next synchronizing call.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBVP3_H
#define LBVP3_H

#include <stddef.h>
#include <stdint.h>

#include "lbvp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The problem statement of the 3-D step.
 *   nx, ny, nz    grid (each >= 3)
 *   tau_plus      symmetric relaxation time (> 1/2); nu = (tau_plus - 1/2)/3
 *   magic_lambda  Lambda = (tau_plus - 1/2)(tau_minus - 1/2) (> 0)
 *   eta           penalization parameter (> 0)
 *   rho0          reference density (deviation storage offset, initial density)
 *   bc_west/east  x sides (lbvp_bc; both or neither periodic); y and z are periodic
 *   rho_in, u_in  state of an INFLOW_EQ side
 *   body_force    uniform body force F_b
 *   storage       lbvp_storage: F64 computes in double; F32, F16_DEV, BF16_DEV in float;
 *                 every type stores the weight-normalized deviation (f_a - w_a rho0)/w_a
 *   force_every   record forces and mass every k steps (0: never)
 *   force_capacity records held on the device between lbvp3_forces calls (0: 4096)
 *   max_bodies    largest n_bodies lbvp3_set_mask accepts (0: 8; at most 255)
 *   flags         must be 0
 */
typedef struct lbvp3_params {
    int32_t nx, ny, nz;
    double tau_plus;
    double magic_lambda;
    double eta;
    double rho0;
    int32_t bc_west, bc_east;
    double rho_in;
    double u_in[3];
    double body_force[3];
    int32_t storage;
    int32_t force_every;
    int64_t force_capacity;
    int32_t max_bodies;
    uint32_t flags;
} lbvp3_params;

/* A rigid obstacle: U_O(x) = v + omega x (x - c) (eq. boundary-condition with a
 * vector angular velocity). */
typedef struct lbvp3_body {
    double c[3];
    double v[3];
    double omega[3];
} lbvp3_body;

typedef struct lbvp3_ctx lbvp3_ctx;

/* Device bytes a context with these parameters allocates. 0 if invalid. */
size_t lbvp3_footprint_bytes(const lbvp3_params* p);

/* Create a context on hip_stream (a hipStream_t, NULL = the null stream; borrowed).
 * Errors: E_ARG (a parameter out of range, non-finite, or an unknown flag),
 * E_NOMEM, E_DEVICE. The populations start at rest, f = f^eq(rho0, 0), with no
 * obstacle. */
lbvp_status lbvp3_create(const lbvp3_params* p, void* hip_stream, lbvp3_ctx** out);

/* The mask function chi and the obstacle motions. body_id: host [nz][ny][nx],
 * 0 = fluid, b in 1..n_bodies = node in body b (chi = 1). bodies: host
 * [n_bodies] (NULL if n_bodies = 0). Errors: E_ARG (n_bodies out of range, a
 * body_id > n_bodies, a non-finite body value), E_NOMEM (more (tile, body) pairs
 * than the reduction tables hold). Synchronizes the stream. */
lbvp_status lbvp3_set_mask(lbvp3_ctx* ctx, const uint8_t* body_id, int32_t n_bodies, const lbvp3_body* bodies);

/* Algorithm step (1): populations set to f^eq(rho, u) (eq. feq), computed on the
 * device in FP64 and rounded to the storage type. Host arrays [nz][ny][nx];
 * rho NULL = rho0, a velocity component NULL = 0. Resets the step counter and
 * the force records; the fields of step 0 are (rho, u, F_VP = 0). */
lbvp_status lbvp3_init_equilibrium(lbvp3_ctx* ctx, const double* rho, const double* ux, const double* uy,
                                   const double* uz);

/* Enqueue n_steps time steps. flags: LBVP_KEEP_FIELDS (store rho, u, F_VP of the
 * call's last step); LBVP_GRAPH (as for lbvp_step: each run of up to 512 steps is
 * captured once per distinct launch sequence, at most 8 kept per context, and
 * replayed; bitwise the plain call's results; a new launch shape, tile band,
 * mask or loaded state drops the kept graphs; needs a stream other than the
 * null stream). Asynchronous. Errors: E_ARG (n_steps < 0, unknown flag, graph on
 * the null stream), E_STATE (the records this call would produce do not fit the
 * undrained ring), E_DEVICE. */
lbvp_status lbvp3_step(lbvp3_ctx* ctx, int64_t n_steps, uint32_t flags);

/* Drain the force records produced since the last call, oldest first.
 * out: host [cap][n_bodies][3] = force on each body, - sum of F_VP over its
 * nodes, FP64, summed in an order fixed by the data (bitwise reproducible for a
 * given launch configuration). mass: host [cap] or NULL = sum of rho over all
 * nodes. *n_out gets the count, *first_step the step number of the first record.
 * Synchronizes the stream. E_UNSTABLE (data still written) if a mass is not
 * finite. */
lbvp_status lbvp3_forces(lbvp3_ctx* ctx, double* out, double* mass, int64_t cap, int64_t* n_out,
                         int64_t* first_step);

/* Fields of planes z0 .. z0 + n_planes - 1 of the last step that ran with
 * LBVP_KEEP_FIELDS (or of the initialisation), host out [7][n_planes][ny][nx]
 * FP64: rho, u_x, u_y, u_z (the corrected velocity of eq. velocity-r), F_VP x,
 * y, z (eq. force-density). Synchronizes the stream. E_ARG (plane range outside
 * the grid), E_STATE (no such step since the last init). */
lbvp_status lbvp3_read_fields(lbvp3_ctx* ctx, int32_t z0, int32_t n_planes, double* out);

/* Post-collision populations g_a of planes z0 .. z0 + n_planes - 1 as host
 * [19][n_planes][ny][nx] FP64 (full values, w_a rho0 added back), in the order
 * stated above. Synchronizes the stream. */
lbvp_status lbvp3_read_populations(lbvp3_ctx* ctx, int32_t z0, int32_t n_planes, double* g);

/* Overwrite the populations of planes z0 .. z0 + n_planes - 1 with host
 * [19][n_planes][ny][nx] FP64 values (rounded to the storage type). Keeps the
 * step counter. Synchronizes the stream. */
lbvp_status lbvp3_write_populations(lbvp3_ctx* ctx, int32_t z0, int32_t n_planes, const double* g);

/* Launch configuration of the step kernel: vec nodes per thread (1, 2 or 4 for
 * F32; 1 or 2 for F64; 1, 4 or 8 for F16_DEV and BF16_DEV) and block threads per workgroup
 * (64, 128 or 256). Results are bitwise independent of it, except the order in
 * which force and mass records are summed. E_ARG for other values. */
lbvp_status lbvp3_set_launch(lbvp3_ctx* ctx, int32_t vec, int32_t block);
lbvp_status lbvp3_get_launch(const lbvp3_ctx* ctx, int32_t* vec, int32_t* block);

/* Order in which the step kernel's workgroups take the tiles, as lbvp_set_tile_band
 * states it for the 2-D step (a tile is vec * block nodes of consecutive lattice
 * rows r = k * ny + j). Results and records do not depend on it; lbvp3_set_launch
 * keeps the band. E_ARG for values other than 0 and powers of two up to 65536. */
lbvp_status lbvp3_set_tile_band(lbvp3_ctx* ctx, int32_t band);
lbvp_status lbvp3_get_tile_band(const lbvp3_ctx* ctx, int32_t* band);

/* Checkpoint and resume, as lbvp_save_state / lbvp_load_state for the 2-D step:
 * lbvp3_save_state writes the context's exact state (the current lattice as
 * stored, the mask and bodies, the fields, the step and record counters) into a
 * caller-allocated host buffer; *size gets the bytes needed, and with buf NULL
 * or cap too small nothing is written and E_NOMEM is returned. E_STATE if force
 * records are undrained (call lbvp3_forces first). lbvp3_load_state restores
 * such a state into a context of the same grid and storage type (launch shape,
 * tile band and parameters are the context's own): stepping it gives bitwise
 * the results the saved context would have given. E_ARG for another grid or
 * storage type, too many bodies, or a damaged blob. Both synchronize the stream. */
lbvp_status lbvp3_save_state(lbvp3_ctx* ctx, void* buf, size_t cap, size_t* size);
lbvp_status lbvp3_load_state(lbvp3_ctx* ctx, const void* buf, size_t size);

/* Batches: many contexts advanced together, one launch per step over all their
 * tiles (as lbvp_batch_* for the 2-D step). lbvp3_batch_create: members[n]
 * (borrowed; they must outlive the batch; same storage type, stream, force_every
 * and step count), vec / block as in lbvp3_set_launch (0: member 0's), applied
 * to every member. lbvp3_batch_step: every member advances n_steps (flags as
 * lbvp3_step: with LBVP_GRAPH each run of up to 512 batched steps is captured
 * once per distinct launch sequence and replayed, bitwise equal to the plain
 * call; it needs a stream other than the null stream); each member's
 * populations, fields and force and mass records are bitwise those of the
 * member stepped alone with the same launch shape.
 * Asynchronous, apart from waiting for the batch's previous steps. E_STATE if a
 * member was stepped alone or given another launch shape since, or a member's
 * records would overflow its ring. The batch's tile band (lbvp3_batch_set_tile_band,
 * 0 at creation) orders the tiles of all members together. */
typedef struct lbvp3_batch lbvp3_batch;
lbvp_status lbvp3_batch_create(lbvp3_ctx* const* members, int32_t n, int32_t vec, int32_t block,
                               lbvp3_batch** out);
lbvp_status lbvp3_batch_step(lbvp3_batch* batch, int64_t n_steps, uint32_t flags);
lbvp_status lbvp3_batch_set_tile_band(lbvp3_batch* batch, int32_t band);
lbvp_status lbvp3_batch_get_tile_band(const lbvp3_batch* batch, int32_t* band);
lbvp_status lbvp3_batch_destroy(lbvp3_batch* batch);
const char* lbvp3_batch_last_error(const lbvp3_batch* batch);

/* Tuner: times the step for every launch shape built for the members' storage
 * (vec x block as in lbvp3_set_launch) and tile bands 0, 2, 4 and 16, on scratch
 * contexts made from the members' parameters, masks and bodies at rest (the
 * members themselves are not stepped; the scratch contexts need as much device
 * memory again). One member runs alone, several as one batch, as lbvp3_step and
 * lbvp3_batch_step would. Each candidate: steps / 4 warm-up steps, then the best
 * of three timed runs of `steps` steps (HIP events on the members' stream).
 * rows[cap] receives one row per candidate and *best the index of the fastest.
 * A candidate that a member's grid does not admit (lbvp3_set_launch or
 * lbvp3_batch_create answers E_ARG) is skipped, and lbvp3_tune_last_error lists
 * it with the reason. Results are cached per process, keyed by storage, record
 * cadence, steps and each member's grid size, body count and mask, unless flags
 * holds LBVP_TUNE_FRESH (no other flag is known). Errors (message from
 * lbvp3_tune_last_error): E_ARG (NULL or mixed members, or no candidate admitted
 * by every member), E_NOMEM, E_DEVICE. */
typedef struct lbvp3_tune_row {
    int32_t vec, block, band;
    double ms_per_step;
    double mlups;            /* million node updates per second over all members */
} lbvp3_tune_row;
lbvp_status lbvp3_tune(lbvp3_ctx* const* members, int32_t n, int32_t steps, uint32_t flags, lbvp3_tune_row* rows,
                       int32_t cap, int32_t* n_rows, int32_t* best);
const char* lbvp3_tune_last_error(void);

/* Steps taken since the last init; -1 for a NULL context. */
int64_t lbvp3_step_count(const lbvp3_ctx* ctx);

/* Wait for the context's stream. */
lbvp_status lbvp3_synchronize(lbvp3_ctx* ctx);

/* Free the context and its device memory (after waiting for its stream). */
lbvp_status lbvp3_destroy(lbvp3_ctx* ctx);

/* Message of the last failure on ctx, or of the calling thread's last failed
 * lbvp3_create if ctx is NULL. Never NULL. */
const char* lbvp3_last_error(const lbvp3_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBVP3_H */
