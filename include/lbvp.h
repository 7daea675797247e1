/*
 * lbvp.h -- C ABI of the MI355X (gfx950) TRT-LBM-VP solver library (liblbvp.so).
 *
 * The library advances a 2-D D2Q9 lattice-Boltzmann domain with the
 * two-relaxation-time collision and the volume-penalization obstacle force of
 * Cui, Wang, Yao, Liu, Yu, "A Coupled Two-relaxation-time Lattice
 * Boltzmann-Volume Penalization method for Flows Past Obstacles" (arXiv
 * 1901.08766). One time step is one fused HIP kernel on the device: pull
 * streaming (eq. streaming), density and intermediate velocity (eqs. rho,
 * rho*velocity-star), the implicit velocity correction and penalization force
 * (eqs. d-V, force-density), the corrected velocity (eq. velocity-r) and the
 * TRT collision with split Guo forcing (eqs. TRT-collision, feq,
 * external-force-term, collision-modified). Lattice units: dx = dy = dt = 1.
 *
 * Conventions
 *  - Every call returns lbvp_status; no C++ exception crosses this boundary.
 *    On failure a message is kept per context (lbvp_last_error(ctx)) or, for a
 *    failed lbvp_create, per calling thread (lbvp_last_error(NULL)).
 *  - Host arrays are row-major [ny][nx] with x fastest; node (i, j) sits at
 *    x = i, y = j. Host inputs are caller-owned and copied before the call
 *    returns; host outputs are caller-allocated with the stated sizes.
 *  - Device memory is either borrowed (dev_mem given to lbvp_create: never freed
 *    by the library) or allocated and owned by the context.
 *  - The HIP stream passed to lbvp_create is borrowed. lbvp_step only enqueues
 *    work on it; faults surface at the next synchronizing call (lbvp_forces,
 *    lbvp_read_fields, lbvp_read_populations, lbvp_synchronize).
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LBVP_H
#define LBVP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbvp_status {
    LBVP_OK = 0,
    LBVP_E_ARG = 1,      /* invalid argument */
    LBVP_E_NOMEM = 2,    /* device memory (or the given dev_mem) too small */
    LBVP_E_BUSY = 3,     /* no free slot (pool) */
    LBVP_E_DEVICE = 4,   /* a HIP runtime call or kernel launch failed */
    LBVP_E_STATE = 5,    /* call not valid in the context's current state */
    LBVP_E_UNSTABLE = 6  /* a non-finite value was detected in the global mass */
} lbvp_status;

/* Domain sides. The paper only draws them (Sec. 3, computational-domain figure):
 * an equilibrium inflow, a zero-gradient outflow and periodic sides.
 * INFLOW_EQ: populations entering from outside are f^eq(rho_in, u_in).
 * OUTFLOW_ZERO_GRAD: populations entering from outside repeat the post-collision
 * populations of the adjacent boundary column. x sides take any of the three
 * (both or neither periodic); y sides are periodic only. */
typedef enum lbvp_bc {
    LBVP_BC_PERIODIC = 0,
    LBVP_BC_INFLOW_EQ = 1,
    LBVP_BC_OUTFLOW_ZERO_GRAD = 2
} lbvp_bc;

/* Storage type of the nine populations in device memory. All types store the
 * weight-normalized deviation (f_a - w_a rho0) / w_a. F64 computes in double;
 * F32, F16_DEV and BF16_DEV compute in float (F16/BF16 encode with
 * round-to-nearest-even). */
typedef enum lbvp_storage {
    LBVP_F64 = 0,
    LBVP_F32 = 1,
    LBVP_F16_DEV = 2,
    LBVP_BF16_DEV = 3
} lbvp_storage;

/* lbvp_params.flags
 * LBVP_LAYOUT_AA: one lattice updated in place with the AA pattern (alternate
 * steps pull from and push to the neighbours' opposite slots, or read and write
 * a node's own slots), half the lattice memory of the default two-lattice pull
 * at the same traffic and the same per-node arithmetic (results are bitwise
 * equal). lbvp_read_populations / lbvp_write_populations need an even step
 * count; F16_DEV and BF16_DEV run with one node per thread. */
#define LBVP_LAYOUT_AA 0x1u

/* lbvp_step flags */
#define LBVP_KEEP_FIELDS 0x1u      /* store rho, u, F_VP of the last step of the call */

/* The problem statement (paper Sec. 2): grid, relaxation, penalization and sides.
 *   tau_plus      symmetric relaxation time tau_s (> 1/2); the viscosity is
 *                 nu = (tau_plus - 1/2)/3 (Sec. 2.1, below eq. feq, read with the
 *                 standard + 1/2)
 *   magic_lambda  Lambda = (tau_s - 1/2)(tau_a - 1/2) (> 0), which fixes tau_a
 *   eta           penalization parameter (> 0), eq. (N-S-modified)
 *   rho0          reference density (deviation storage offset and initial density)
 *   rho_in, u_in  state of an INFLOW_EQ side
 *   body_force    uniform body force F_b of eq. (N-S-modified)
 *   force_every   record forces and mass every k steps (0: never)
 *   force_capacity records held on the device between lbvp_forces calls (0: 16384)
 *   max_bodies    largest n_bodies lbvp_set_mask accepts (0: 8; at most 255)
 */
typedef struct lbvp_params {
    int32_t nx, ny;
    double tau_plus;
    double magic_lambda;
    double eta;
    double rho0;
    int32_t bc_west, bc_east, bc_south, bc_north;   /* lbvp_bc */
    double rho_in;
    double u_in[2];
    double body_force[2];
    int32_t storage;                                /* lbvp_storage */
    int32_t force_every;
    int64_t force_capacity;
    int32_t max_bodies;
    uint32_t flags;
} lbvp_params;

/* A rigid obstacle: U_O(x) = (vx, vy) + omega z x (x - (cx, cy)) (eq. boundary-condition;
 * the paper's experiments rotate bodies, Secs. 3.1 and 3.4). */
typedef struct lbvp_body {
    double cx, cy, vx, vy, omega;
} lbvp_body;

typedef struct lbvp_ctx lbvp_ctx;

/* Device bytes a context with these parameters needs (lattice(s), mask, fields,
 * reduction partials, force ring, staging). 0 if the parameters are invalid. */
size_t lbvp_footprint_bytes(const lbvp_params* p);

/* Create a context. hip_stream: a hipStream_t (NULL = the null stream), borrowed.
 * dev_mem: NULL (the context allocates and owns its memory) or a device buffer of
 * dev_bytes >= lbvp_footprint_bytes(p), 256-byte aligned, borrowed.
 * Errors: E_ARG (nx or ny < 3, tau_plus <= 1/2, magic_lambda <= 0, eta <= 0,
 * exactly one x side periodic, a non-periodic y side, unknown storage or flag,
 * non-finite value), E_NOMEM, E_DEVICE. The populations start at rest,
 * f = f^eq(rho0, 0), with no obstacle. */
lbvp_status lbvp_create(const lbvp_params* p, void* hip_stream, void* dev_mem, size_t dev_bytes,
                        lbvp_ctx** out);

/* The mask function chi of eq. (mask function) and the obstacle velocities.
 * body_id: host [ny][nx], 0 = fluid, k in 1..n_bodies = node belongs to body k
 * (chi = 1). bodies: host [n_bodies] rigid motions (NULL if n_bodies = 0).
 * Errors: E_ARG (n_bodies < 0 or > max_bodies, a body_id > n_bodies, non-finite
 * body values), E_NOMEM (more (tile, body) pairs than the reduction tables hold). */
lbvp_status lbvp_set_mask(lbvp_ctx* ctx, const uint8_t* body_id, int32_t n_bodies,
                          const lbvp_body* bodies);

/* Algorithm step (1) of Sec. 2.2: populations set to f^eq(rho, u) (eq. feq), which
 * is also the state after the first collision, taken with F = 0. Host arrays
 * [ny][nx]; rho NULL = rho0, ux/uy NULL = 0. Resets the step counter and the
 * force records. The fields of step 0 are (rho, u, F_VP = 0). */
lbvp_status lbvp_init_equilibrium(lbvp_ctx* ctx, const double* rho, const double* ux,
                                  const double* uy);

/* Enqueue n_steps time steps (algorithm steps (2)-(7)). flags: LBVP_KEEP_FIELDS.
 * Asynchronous. Errors: E_ARG (n_steps < 0), E_STATE (the force records this
 * call would produce do not fit the undrained ring: call lbvp_forces first),
 * E_DEVICE (launch failure). */
lbvp_status lbvp_step(lbvp_ctx* ctx, int64_t n_steps, uint32_t flags);

/* Drain the force records produced since the last call, oldest first.
 * out: host [cap][n_bodies][2] = force on each body, - sum of F_VP over its nodes
 * (eq. hydrodynamic force; Sec. 3 sums F_VP dx dy), FP64. mass: host [cap] or
 * NULL = sum of rho over all nodes. At most cap records are returned; *n_out gets
 * the count and *first_step the step number of the first one (records are
 * force_every steps apart). Synchronizes the stream. Returns E_UNSTABLE (data
 * still written) if a drained mass is not finite. */
lbvp_status lbvp_forces(lbvp_ctx* ctx, double* out, double* mass, int64_t cap, int64_t* n_out,
                        int64_t* first_step);

/* Fields of the last step that ran with LBVP_KEEP_FIELDS (or of the
 * initialisation): rho (eq. rho), corrected velocity u = u* + du (eq. velocity-r)
 * and F_VP (eq. force-density), each host [ny][nx] FP64, any may be NULL.
 * Synchronizes the stream. E_STATE if no such step ran since the last init. */
lbvp_status lbvp_read_fields(lbvp_ctx* ctx, double* rho, double* ux, double* uy, double* fx,
                             double* fy);

/* Current post-collision populations g_a (eq. collision-modified) as host
 * [9][ny][nx] FP64 (full values, w_a rho0 added back), in the D2Q9 order of
 * eq. (D2Q9). Synchronizes the stream. E_STATE in the AA layout after an odd
 * step count (the lattice then holds streamed, not post-collision, values). */
lbvp_status lbvp_read_populations(lbvp_ctx* ctx, double* g);

/* Overwrite the populations with host [9][ny][nx] FP64 values g_a (rounded to
 * the storage type). Keeps the step counter. E_STATE in the AA layout after an
 * odd step count. */
lbvp_status lbvp_write_populations(lbvp_ctx* ctx, const double* g);

/* Launch configuration of the step kernel: vec nodes per thread (1, or the
 * storage type's 16-byte width: 2 for F64, 4 for F32, 8 for F16/BF16) and block
 * threads per workgroup (64, 128 or 256). Results do not depend on it except
 * through the order of the force and mass sums. A default is chosen from the
 * grid size at lbvp_create; a tuner may set another. Errors: E_ARG (other
 * values), E_STATE (undrained force records). Synchronizes the stream. */
lbvp_status lbvp_set_launch(lbvp_ctx* ctx, int32_t vec, int32_t block);
lbvp_status lbvp_get_launch(const lbvp_ctx* ctx, int32_t* vec, int32_t* block);

/* ---- Batches: many contexts advanced by one launch per step -------------------
 * A batch holds contexts of one storage type and layout on one stream. Each step
 * of lbvp_batch_step is a single launch over the tiles of every member (block ->
 * (domain, tile) through a tile map), so domains of any size, parameters and mask
 * share the device. Every member must be at the same force-record phase (and, in
 * the AA layout, step parity); the members stay ordinary contexts and keep their
 * own force rings, fields and populations, read with the usual calls. Results
 * are bitwise those of stepping each member alone with the same launch shape.
 *
 * lbvp_batch_create: members[n] (borrowed; they must outlive the batch), vec /
 * block as in lbvp_set_launch (0: the storage type's vector width, 256), applied
 * to every member. E_ARG (mixed storage, layout, stream, force cadence or phase),
 * E_STATE (a member has undrained force records), E_NOMEM, E_DEVICE.
 * lbvp_batch_step: every member advances n_steps (flags as lbvp_step);
 * asynchronous; E_STATE if members went out of phase or a ring would overflow. */
typedef struct lbvp_batch lbvp_batch;
lbvp_status lbvp_batch_create(lbvp_ctx* const* members, int32_t n, int32_t vec, int32_t block, lbvp_batch** out);
lbvp_status lbvp_batch_step(lbvp_batch* batch, int64_t n_steps, uint32_t flags);
lbvp_status lbvp_batch_destroy(lbvp_batch* batch);
const char* lbvp_batch_last_error(const lbvp_batch* batch);

/* Number of steps taken since the last lbvp_init_equilibrium. */
int64_t lbvp_step_count(const lbvp_ctx* ctx);

/* Wait for all work enqueued by the context; E_DEVICE if a kernel failed. */
lbvp_status lbvp_synchronize(lbvp_ctx* ctx);

/* Free the context (and its memory if it owns it). NULL is accepted. */
lbvp_status lbvp_destroy(lbvp_ctx* ctx);

/* Last error message of ctx, or of the calling thread's last failed
 * lbvp_create if ctx is NULL. Never NULL; valid until the next call on ctx. */
const char* lbvp_last_error(const lbvp_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBVP_H */
