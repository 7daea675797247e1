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
    LBVP_BC_OUTFLOW_ZERO_GRAD = 2,
    /* a cut through one larger domain (slab decomposition along x): the
     * populations entering through this side are the neighbouring slab's
     * post-collision boundary column, delivered by lbvp_halo_exchange before
     * each step. Not with LBVP_LAYOUT_AA or LBVP_MOVING_BODIES. */
    LBVP_BC_NEIGHBOR = 3
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
/* LBVP_MOVING_BODIES: the mask function chi(x, t) follows each body's rigid
 * motion (eq. mask function with a time-dependent chi; eq. boundary-condition):
 * at the step that takes the counter to k, body b has moved to
 * c_b(t) = c_b + V_b t and turned by omega_b t (t = k), and node x belongs to it
 * when the mask given to lbvp_set_mask (the bodies at t = 0) holds b at the node
 * nearest to R(-omega_b t)(x - c_b(t)) + c_b (first such body wins); U_O uses
 * c_b(t). At most 8 bodies. Every launch shape, LBVP_GRAPH, batches (moving
 * and fixed members mixed), the pool and the tuner take such contexts: the
 * poses are evaluated on the host in double for up to 1024 coming time levels
 * at a time and read on the device at a row that the device itself advances
 * after each run, so a captured graph replays correctly at any later time.
 * Results are bitwise equal across launch shapes, alone or in a batch, plain or
 * through graphs. */
#define LBVP_MOVING_BODIES 0x2u

/* lbvp_step / lbvp_batch_step flags
 * LBVP_KEEP_FIELDS: store rho, u, F_VP of the last step of the call.
 * LBVP_GRAPH: enqueue the call through HIP graphs: each run of up to 512 steps is
 * captured once per distinct launch sequence (at most 8 kept per context or
 * batch) and replayed, which removes the per-launch host cost. Results are
 * bitwise those of the plain call. Needs a stream other than the null stream. */
#define LBVP_KEEP_FIELDS 0x1u
#define LBVP_GRAPH 0x2u

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

/* lbvp_read_fields and lbvp_read_populations for rows y0 .. y0 + n_rows - 1 only:
 * each field host [n_rows][nx], populations host [9][n_rows][nx], so that a large
 * domain can be read a band at a time. E_ARG (a row range outside the grid),
 * otherwise as the whole-domain calls. */
lbvp_status lbvp_read_fields_rows(lbvp_ctx* ctx, int32_t y0, int32_t n_rows, double* rho, double* ux,
                                  double* uy, double* fx, double* fy);
lbvp_status lbvp_read_populations_rows(lbvp_ctx* ctx, int32_t y0, int32_t n_rows, double* g);

/* Overwrite the populations with host [9][ny][nx] FP64 values g_a (rounded to
 * the storage type). Keeps the step counter. E_STATE in the AA layout after an
 * odd step count. */
lbvp_status lbvp_write_populations(lbvp_ctx* ctx, const double* g);

/* Checkpoint and resume. lbvp_save_state writes the context's exact state into
 * a caller-allocated host buffer: the lattice as stored (any step parity, any
 * layout), the AA outflow ghost columns, the mask and bodies, the fields, the
 * step and record counters. *size gets the bytes needed; with buf NULL or cap
 * too small nothing is written and E_NOMEM is returned (call once to size).
 * E_STATE if force records are undrained (call lbvp_forces first).
 * Synchronizes the stream.
 * lbvp_load_state restores such a blob into a context created with the same
 * grid, storage type and layout (E_ARG otherwise, or for a damaged blob); the
 * context's own relaxation, penalization and side parameters apply from then
 * on. Stepping a restored context gives bitwise the results the saved one
 * would have given. Synchronizes the stream. */
lbvp_status lbvp_save_state(lbvp_ctx* ctx, void* buf, size_t cap, size_t* size);
lbvp_status lbvp_load_state(lbvp_ctx* ctx, const void* buf, size_t size);

/* Launch configuration of the step kernel: vec nodes per thread (1, the
 * storage type's 16-byte width: 2 for F64, 4 for F32, 8 for F16/BF16, or 4 for
 * F16/BF16; 2-byte types in the AA layout take 1 only) and block
 * threads per workgroup (64, 128 or 256). Populations and fields do not depend
 * on it; the force and mass records do only through the per-tile partial sums
 * (each record is then summed in an order fixed by the data, independent of the
 * block size and of how steps are split over calls). A default is chosen from
 * the grid size at lbvp_create; lbvp_tune measures the others. Errors: E_ARG
 * (other values), E_STATE (undrained force records when the shape changes).
 * Synchronizes the stream when the shape changes. */
lbvp_status lbvp_set_launch(lbvp_ctx* ctx, int32_t vec, int32_t block);
lbvp_status lbvp_get_launch(const lbvp_ctx* ctx, int32_t* vec, int32_t* block);

/* Order in which the step kernel's workgroups take the tiles of the domain (a
 * tile is the vec * block nodes one workgroup updates, in row order). The GPU
 * deals workgroups to its 8 XCDs round robin, and each XCD has its own L2.
 *   band = 0: each XCD sweeps one contiguous eighth of the tiles;
 *   band = 2^k (1 .. 65536): the tiles form groups of 8 bands of `band`
 *     consecutive tiles and each XCD takes one band of every group, so the
 *     chip moves through a window of 8 * band tiles at a time (band = 1 is
 *     plain dispatch order).
 * Populations, fields and force and mass records do not depend on it. A default
 * is chosen with the launch shape at lbvp_create; lbvp_set_launch keeps the
 * band. Batches have their own (lbvp_batch_set_tile_band); the pool uses 0.
 * Errors: E_ARG (other values). */
lbvp_status lbvp_set_tile_band(lbvp_ctx* ctx, int32_t band);
lbvp_status lbvp_get_tile_band(const lbvp_ctx* ctx, int32_t* band);

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
 * E_STATE (a member whose launch shape changes has undrained force records),
 * E_NOMEM, E_DEVICE.
 * lbvp_batch_step: every member advances n_steps (flags as lbvp_step);
 * asynchronous (the members' arguments go through pinned host buffers, so the
 * call does not wait for earlier work); E_STATE if members went out of phase or
 * a ring would overflow. */
typedef struct lbvp_batch lbvp_batch;
lbvp_status lbvp_batch_create(lbvp_ctx* const* members, int32_t n, int32_t vec, int32_t block, lbvp_batch** out);
lbvp_status lbvp_batch_step(lbvp_batch* batch, int64_t n_steps, uint32_t flags);
lbvp_status lbvp_batch_destroy(lbvp_batch* batch);
const char* lbvp_batch_last_error(const lbvp_batch* batch);
/* The slabs of one decomposed domain as members of a batch: before every step,
 * lbvp_batch_step exchanges the halo columns of the n cuts (member west[i]'s east
 * side to member east[i]'s west side, as lbvp_halo_exchange does) in one kernel,
 * so a run of steps needs one call. n = 0 removes the cuts; replacing the
 * members removes them too. E_ARG (n > 32, an index out of range, a linked side
 * that is not LBVP_BC_NEIGHBOR, unequal ny). */
lbvp_status lbvp_batch_set_halo(lbvp_batch* batch, const int32_t* west, const int32_t* east, int32_t n);
/* Block -> tile order of the batch's step launches over the members' tiles, taken
 * in member order, as lbvp_set_tile_band states it (0 at lbvp_batch_create; the
 * members' own bands do not apply to batch steps). Results and records do not
 * depend on it. E_ARG for values other than 0 and powers of two up to 65536. */
lbvp_status lbvp_batch_set_tile_band(lbvp_batch* batch, int32_t band);
lbvp_status lbvp_batch_get_tile_band(const lbvp_batch* batch, int32_t* band);

/* ---- A batched step that allocates nothing ---------------------------------------
 * For callers that cannot allocate device or pinned host memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid it): one call of
 * lbvp_batch_create + lbvp_batch_step + lbvp_batch_destroy on members[n]
 * (borrowed contexts, as for a batch), with the batch's tables (each member's step
 * and finalize arguments and the tile map) kept in a file-scope device array of
 * 4 MiB (one copy per GPU, held until the process ends) instead of memory the
 * library allocates. The same kernels run in the same order, so populations,
 * fields and force records are bitwise those of lbvp_batch_step at band 0.
 * Members must share the first member's launch shape (set beforehand with
 * lbvp_set_launch, which may allocate) and the conditions of lbvp_batch_create.
 * The tables go up with one host-to-device copy on the members' stream from a
 * pageable staging block; the call returns without waiting for the steps.
 * Every call on a GPU shares its array and rewrites all of the tables it uses,
 * so calls that overlap on one GPU (other streams, other host threads) race.
 * flags: LBVP_KEEP_FIELDS (LBVP_GRAPH is rejected: instantiating a graph
 * allocates). E_ARG (tables larger than 4 MiB, with the size in the message; NULL
 * members; mixed storage, layout, stream, cadence, phase or launch shape),
 * E_STATE (a ring would overflow), E_DEVICE. Messages: lbvp_batch_last_error(NULL). */
lbvp_status lbvp_batch_step_static(lbvp_ctx* const* members, int32_t n, int64_t n_steps, uint32_t flags);

/* ---- Tuner ----------------------------------------------------------------------
 * Times the step kernel for every launch shape (vec x block, and for vec > 1 the
 * tile bands 0, 2 and 16 of lbvp_set_tile_band) and, with LBVP_TUNE_LAYOUTS, in
 * both layouts, on scratch contexts made from the members'
 * parameters and masks (the members themselves are not stepped; the scratch
 * contexts need as much device memory again). n > 1 members run as one batch, as
 * they would in lbvp_batch_step. Each candidate: steps/4 warm-up steps, then the
 * best of three timed runs of `steps` steps (HIP events on the members' stream).
 * rows[cap] receives one row per candidate and *best the index of the fastest;
 * when layouts are compared, the fastest AA row wins if within 3% of the
 * fastest row, for its halved lattice memory. Results are cached per process,
 * keyed by storage, layout, record cadence, steps and the members' grid sizes,
 * unless LBVP_TUNE_FRESH. Errors (message from lbvp_tune_last_error): E_ARG,
 * E_NOMEM, E_DEVICE. */
#define LBVP_TUNE_LAYOUTS 0x1u
#define LBVP_TUNE_FRESH 0x2u
typedef struct lbvp_tune_row {
    uint32_t layout_flags;   /* 0 or LBVP_LAYOUT_AA */
    int32_t vec, block;
    int32_t band;            /* tile band (lbvp_set_tile_band, lbvp_batch_set_tile_band) */
    double ms_per_step;
    double mlups;            /* million node updates per second over all members */
} lbvp_tune_row;
lbvp_status lbvp_tune(lbvp_ctx* const* members, int32_t n, int32_t steps, uint32_t flags, lbvp_tune_row* rows,
                      int32_t cap, int32_t* n_rows, int32_t* best);
const char* lbvp_tune_last_error(void);

/* ---- Serving pool: continuous batching of independent solves ---------------------
 * A pool keeps many solves (a domain, its mask and bodies, its parameters and a
 * step count) resident on one stream and advances all running ones together, an
 * epoch at a time, one batched launch per step. lbvp_pool_admit takes a solve
 * when a slot is free and its footprint fits under cap_bytes; it is set up on a
 * private stream while earlier epochs run and joins at the next epoch. An epoch
 * runs up to max_steps steps, fewer if a solve would otherwise overshoot its
 * count (AA layout: an even number, a solve's odd last step running on its
 * own), so each solve stops exactly at its count with its final fields kept.
 * Every solve's populations, fields and force records are bitwise those of the
 * same problem stepped alone (lbvp_step) with the pool's launch shape.
 * Device memory comes from chunks of chunk_bytes reserved as needed (never
 * returned before lbvp_pool_destroy), split first-fit among solves.
 *
 * Solve parameters: storage and layout are the pool's; force_every must be 0 or
 * 1; force_capacity is set by the pool to hold every record of the solve.
 * Thread use: one host thread per pool. */
typedef struct lbvp_pool lbvp_pool;
typedef struct lbvp_pool_config {
    size_t cap_bytes;        /* admission limit on the summed footprints (and on reserved memory) */
    size_t chunk_bytes;      /* device memory reserved at a time (0: 1 GiB) */
    int32_t max_slots;       /* most solves admitted at once (1 .. 65536) */
    int32_t storage;         /* lbvp_storage of every solve */
    uint32_t layout_flags;   /* 0 or LBVP_LAYOUT_AA */
    int32_t vec, block;      /* launch shape as in lbvp_set_launch (0, 0: the storage width, 256) */
    int32_t max_in_flight;   /* epochs enqueued ahead of the host (0: 2) */
} lbvp_pool_config;

typedef struct lbvp_pool_stats {
    int32_t waiting;         /* admitted, not yet stepped */
    int32_t running;         /* in the batch */
    int32_t finished;        /* all steps enqueued, not yet complete on the device */
    int32_t done;            /* complete; results readable until released */
    int32_t free_slots;
    size_t used_bytes;       /* summed footprints of admitted solves */
    size_t reserved_bytes;   /* device memory held by the pool */
    int64_t epochs;
    int64_t node_updates;    /* nx * ny * steps summed over every step enqueued */
} lbvp_pool_stats;

/* hip_stream: borrowed, the stream every epoch runs on (not the null stream).
 * E_ARG (bad config), E_DEVICE. */
lbvp_status lbvp_pool_create(const lbvp_pool_config* cfg, void* hip_stream, lbvp_pool** out);
/* Admit one solve. p, body_id, n_bodies, bodies as lbvp_create / lbvp_set_mask;
 * rho, ux, uy as lbvp_init_equilibrium (nullable); n_steps >= 1. *slot gets the
 * handle. E_BUSY (no free slot), E_NOMEM (the footprint does not fit now; retry
 * after a release), E_ARG. The host arrays are copied before return. */
lbvp_status lbvp_pool_admit(lbvp_pool* pool, const lbvp_params* p, const uint8_t* body_id, int32_t n_bodies,
                            const lbvp_body* bodies, const double* rho, const double* ux, const double* uy,
                            int64_t n_steps, int32_t* slot);
/* Enqueue one epoch of at most max_steps steps (>= 1) over the admitted solves
 * and return; waits only while more than max_in_flight epochs are enqueued.
 * *steps_run: the epoch length (0 if nothing is running). */
lbvp_status lbvp_pool_run_epoch(lbvp_pool* pool, int64_t max_steps, int64_t* steps_run);
/* Slots whose solve completed on the device since the last poll (cap at most).
 * wait != 0: block until at least one completes if any is still finishing. */
lbvp_status lbvp_pool_poll(lbvp_pool* pool, int32_t wait, int32_t* slots, int32_t cap, int32_t* n_done);
/* Results of a completed solve, as lbvp_forces / lbvp_read_fields of a context
 * (fields of its last step). E_STATE if the solve is not complete. These wait
 * on the pool's private stream only, never on running epochs. */
lbvp_status lbvp_pool_forces(lbvp_pool* pool, int32_t slot, double* out, double* mass, int64_t cap,
                             int64_t* n_out, int64_t* first_step);
lbvp_status lbvp_pool_read_fields(lbvp_pool* pool, int32_t slot, double* rho, double* ux, double* uy,
                                  double* fx, double* fy);
/* Free a completed (or not yet started) solve's slot and memory. E_STATE otherwise. */
lbvp_status lbvp_pool_release(lbvp_pool* pool, int32_t slot);
lbvp_status lbvp_pool_get_stats(const lbvp_pool* pool, lbvp_pool_stats* out);
/* Waits for the pool's work, frees everything. NULL is accepted. */
lbvp_status lbvp_pool_destroy(lbvp_pool* pool);
const char* lbvp_pool_last_error(const lbvp_pool* pool);

/* Measurement aid, not part of the method: copy bytes (a multiple of 16) from
 * src to dst, both device pointers 16-byte aligned, one 16-byte non-temporal
 * load and store per thread (the fastest copy form measured on MI355X), on
 * hip_stream (asynchronous). Its rate is the copy bandwidth the step is
 * compared with.
 * E_ARG on misaligned pointers or sizes, E_DEVICE on a launch failure. */
lbvp_status lbvp_device_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Slab decomposition of one domain along x (the decomposition the method's
 * two-lattice streaming, eq. streaming, allows: per step only the populations
 * crossing a cut move). For each i, link i joins west[i]'s east side to
 * east[i]'s west side (both LBVP_BC_NEIGHBOR; west[i] == east[i] closes one slab
 * on itself): east[i]'s west halo column receives west[i]'s current populations
 * with e_x = +1 at its column nx - 1, and west[i]'s east halo column receives
 * east[i]'s populations with e_x = -1 at its column 0. Call it before every step
 * of the slabs; one kernel, enqueued on west[0]'s stream, which must be the
 * stream of every slab (one device: the slabs stand for the shares of several
 * GPUs, where this is the halo transfer over xGMI). Linked slabs need equal ny
 * and storage type. Errors: E_ARG (NULL, n < 1 or > 32, a side that is not
 * LBVP_BC_NEIGHBOR, unequal ny, storage or stream), E_DEVICE. */
lbvp_status lbvp_halo_exchange(lbvp_ctx* const* west, lbvp_ctx* const* east, int32_t n);

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
