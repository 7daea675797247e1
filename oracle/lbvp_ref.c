/*
 * lbvp_ref.c -- plain FP64 CPU reference of the coupled TRT-LBM-VP method.
 *
 * TEST INFRASTRUCTURE. This file is the oracle that the HIP library is checked
 * against. Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no code, header, table or helper with the HIP path.
 *
 * It is deliberately slow and literal: two full lattices (post-collision g at
 * time t_n and the next one), every node updated by the same function, in the
 * order the paper's algorithm gives (Sec. 2.2, steps (1)-(7)):
 *
 *   (1)   initial values; the first collision has F = 0, so the state after it
 *         is g = f^eq(rho0, u0) exactly;
 *   (3)   streaming, eq. (streaming), pull form: f_a(x) = g_a(x - e_a);
 *   (4)   rho, eq. (rho), and the intermediate velocity, eq. (rho*velocity-star);
 *   (5)   velocity correction and force density, eqs. (d-V), (force-density);
 *   (6)   corrected velocity, eq. (velocity-r), and the TRT collision with the
 *         split Guo forcing, eqs. (TRT-collision), (collision-modified);
 *   (2)/(7) the result is the next post-collision lattice; repeat.
 *
 * Lattice units: dx = dy = dt = 1.
 *
 * Readings where the paper is silent, garbled or inconsistent:
 *  - tau_s: the printed tau_s = nu/(c_s^2 dt) lacks the + 1/2 of the standard
 *    relation; callers pass tau_plus directly, and tau_minus comes from the
 *    magic parameter, Lambda = (tau_s - 1/2)(tau_a - 1/2).
 *  - Guo term, eq. (external-force-term), carries a factor (1 - 1/(2 lambda))
 *    with lambda undefined, while eq. (collision-modified) applies (1 - 1/(2 tau))
 *    per part. The factor of eq. (external-force-term) is dropped (applying
 *    both would count it twice); with tau_s = tau_a this is the SRT Guo scheme.
 *  - The velocity inside f^eq and inside the Guo term is the corrected
 *    u = u* + du, and the force is the total F = F_b + F_VP.
 *  - A uniform body force F_b (eq. (N-S-modified)) enters u* with its half step,
 *    rho u* = sum e f + F_b/2, so that rho u = sum e f + F/2 (eq. rho*velocity-ex).
 *  - The obstacle velocity is a per-body rigid motion, U_O = V + omega z x (x - c).
 *  - Force on a body = - sum over its nodes of F_VP (eq. (hydrodynamic force);
 *    the drag formula of Sec. 3 drops this sign).
 *  - Domain sides (only drawn in a missing figure): PERIODIC, INFLOW_EQ (ghost
 *    populations are f^eq(rho_in, u_in)) and OUTFLOW_ZERO_GRAD (ghost = the
 *    post-collision populations of the adjacent boundary column). y sides are
 *    periodic only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9

/* eq. (D2Q9): alpha = 0 rest; alpha = 1..4 at angle (alpha-1) pi/2;
 * alpha = 5..8 of length sqrt(2) at angle (2 alpha - 9) pi/4. */
static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* weights of eq. (feq) */
static const double WGT[Q] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* the direction opposite to alpha ("-alpha" in Sec. 2.1): f_{-1} = f_3, f_{-0} = f_0 */
static const int OPPOSITE[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0; /* c_s = 1/sqrt(3) */

enum { REF_PERIODIC = 0, REF_INFLOW_EQ = 1, REF_OUTFLOW_ZERO_GRAD = 2 };

typedef struct ref_params {
    int32_t nx, ny;
    double tau_plus;      /* tau_s */
    double magic_lambda;  /* Lambda */
    double eta;           /* penalization parameter */
    double rho0;
    int32_t bc_west, bc_east, bc_south, bc_north;
    double rho_in, u_in_x, u_in_y;
    double fb_x, fb_y;    /* uniform body force F_b */
    int32_t moving;       /* bodies move rigidly: chi(x, t) follows them */
} ref_params;

typedef struct ref_ctx {
    ref_params p;
    double tau_minus;
    int64_t n;            /* nx * ny */
    double *g, *g_next;   /* [Q][ny][nx] post-collision populations */
    uint8_t *body_id;     /* [ny][nx] */
    int32_t n_bodies;
    double *bodies;       /* [n_bodies][5] = cx, cy, vx, vy, omega */
    double *fields;       /* [5][ny][nx] = rho, ux, uy, FVPx, FVPy of the last step */
    double *row_force;    /* [ny][n_bodies][2] per-row partials */
    double *row_mass;     /* [ny] */
    int64_t step;
} ref_ctx;

/* ---------------------------------------------------------------- pieces --- */

void lbvp_ref_lattice(int32_t ex[Q], int32_t ey[Q], double w[Q], int32_t opp[Q])
{
    for (int a = 0; a < Q; ++a) {
        ex[a] = EX[a];
        ey[a] = EY[a];
        w[a] = WGT[a];
        opp[a] = OPPOSITE[a];
    }
}

/* tau_a from the magic parameter: Lambda = (tau_s - 1/2)(tau_a - 1/2). */
double lbvp_ref_tau_minus(double tau_plus, double magic_lambda)
{
    return 0.5 + magic_lambda / (tau_plus - 0.5);
}

/* eq. (feq) */
static double feq_one(int a, double rho, double ux, double uy)
{
    double eu = EX[a] * ux + EY[a] * uy;
    double uu = ux * ux + uy * uy;
    return rho * WGT[a] * (1.0 + eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2));
}

void lbvp_ref_feq(double rho, double ux, double uy, double out[Q])
{
    for (int a = 0; a < Q; ++a) out[a] = feq_one(a, rho, ux, uy);
}

/* eq. (external-force-term) without the (1 - 1/(2 lambda)) factor:
 * F_a = w_a [ (e_a - u)/c_s^2 + (e_a . u) e_a / c_s^4 ] . F */
void lbvp_ref_guo(double ux, double uy, double Fx, double Fy, double out[Q])
{
    for (int a = 0; a < Q; ++a) {
        double eu = EX[a] * ux + EY[a] * uy;
        double vx = (EX[a] - ux) / CS2 + eu * EX[a] / (CS2 * CS2);
        double vy = (EY[a] - uy) / CS2 + eu * EY[a] / (CS2 * CS2);
        out[a] = WGT[a] * (vx * Fx + vy * Fy);
    }
}

/* eqs. (TRT-collision) and (collision-modified): the distributions, their
 * equilibria and the forcing are split into symmetric and antisymmetric parts
 * about the opposite direction and relaxed with tau_s and tau_a. */
void lbvp_ref_trt_collide(const double f[Q], const double feq[Q], const double F[Q],
                          double tau_s, double tau_a, double g[Q])
{
    for (int a = 0; a < Q; ++a) {
        int b = OPPOSITE[a];
        double fs = 0.5 * (f[a] + f[b]), fa = 0.5 * (f[a] - f[b]);
        double es = 0.5 * (feq[a] + feq[b]), ea = 0.5 * (feq[a] - feq[b]);
        double Fs = 0.5 * (F[a] + F[b]), Fa = 0.5 * (F[a] - F[b]);
        double omega = -(fs - es) / tau_s - (fa - ea) / tau_a;
        g[a] = f[a] + omega + (1.0 - 1.0 / (2.0 * tau_s)) * Fs + (1.0 - 1.0 / (2.0 * tau_a)) * Fa;
    }
}

/* eqs. (d-V) and (force-density) with dt = 1:
 *   du    = chi (U_O - u*) / (2 eta + chi)
 *   F_VP  = 2 rho chi (U_O - u*) / (2 eta + chi)                              */
void lbvp_ref_vp(double rho, double usx, double usy, int chi, double UOx, double UOy,
                 double eta, double out[4] /* dux, duy, FVPx, FVPy */)
{
    double c = chi ? 1.0 : 0.0;
    out[0] = c * (UOx - usx) / (2.0 * eta + c);
    out[1] = c * (UOy - usy) / (2.0 * eta + c);
    out[2] = 2.0 * rho * c * (UOx - usx) / (2.0 * eta + c);
    out[3] = 2.0 * rho * c * (UOy - usy) / (2.0 * eta + c);
}

/* Steps (4)-(6) at one node, given the streamed populations f. Writes the
 * post-collision populations g and the node's fields (rho, ux, uy, FVPx, FVPy). */
void lbvp_ref_collide_node(const double f[Q], double tau_s, double tau_a, double eta,
                           int chi, double UOx, double UOy, double fbx, double fby,
                           double g[Q], double fields[5])
{
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < Q; ++a) {           /* eq. (rho), eq. (rho*velocity-star) */
        rho += f[a];
        jx += EX[a] * f[a];
        jy += EY[a] * f[a];
    }
    double usx = (jx + 0.5 * fbx) / rho;    /* half step of the body force */
    double usy = (jy + 0.5 * fby) / rho;
    double vp[4];
    lbvp_ref_vp(rho, usx, usy, chi, UOx, UOy, eta, vp);
    double ux = usx + vp[0];                /* eq. (velocity-r) */
    double uy = usy + vp[1];
    double Fx = fbx + vp[2];
    double Fy = fby + vp[3];
    double feq[Q], F[Q];
    lbvp_ref_feq(rho, ux, uy, feq);
    lbvp_ref_guo(ux, uy, Fx, Fy, F);
    lbvp_ref_trt_collide(f, feq, F, tau_s, tau_a, g);
    fields[0] = rho;
    fields[1] = ux;
    fields[2] = uy;
    fields[3] = vp[2];
    fields[4] = vp[3];
}

/* ------------------------------------------------------------ the solver --- */

static int valid_side(int32_t s) { return s == REF_PERIODIC || s == REF_INFLOW_EQ || s == REF_OUTFLOW_ZERO_GRAD; }

ref_ctx *lbvp_ref_create(const ref_params *p)
{
    if (p->nx < 3 || p->ny < 3) return NULL;
    if (!(p->tau_plus > 0.5) || !(p->magic_lambda > 0.0) || !(p->eta > 0.0)) return NULL;
    if (!valid_side(p->bc_west) || !valid_side(p->bc_east)) return NULL;
    if ((p->bc_west == REF_PERIODIC) != (p->bc_east == REF_PERIODIC)) return NULL;
    if (p->bc_south != REF_PERIODIC || p->bc_north != REF_PERIODIC) return NULL;
    ref_ctx *c = (ref_ctx *)calloc(1, sizeof(ref_ctx));
    if (!c) return NULL;
    c->p = *p;
    c->tau_minus = lbvp_ref_tau_minus(p->tau_plus, p->magic_lambda);
    c->n = (int64_t)p->nx * p->ny;
    c->g = (double *)calloc((size_t)(Q * c->n), sizeof(double));
    c->g_next = (double *)calloc((size_t)(Q * c->n), sizeof(double));
    c->body_id = (uint8_t *)calloc((size_t)c->n, 1);
    c->fields = (double *)calloc((size_t)(5 * c->n), sizeof(double));
    c->row_mass = (double *)calloc((size_t)p->ny, sizeof(double));
    if (!c->g || !c->g_next || !c->body_id || !c->fields || !c->row_mass) {
        free(c->g); free(c->g_next); free(c->body_id); free(c->fields); free(c->row_mass); free(c);
        return NULL;
    }
    return c;
}

void lbvp_ref_destroy(ref_ctx *c)
{
    if (!c) return;
    free(c->g); free(c->g_next); free(c->body_id); free(c->fields);
    free(c->bodies); free(c->row_force); free(c->row_mass);
    free(c);
}

int lbvp_ref_set_mask(ref_ctx *c, const uint8_t *body_id, int32_t n_bodies, const double *bodies)
{
    if (n_bodies < 0 || n_bodies > 255) return 1;
    for (int64_t k = 0; k < c->n; ++k)
        if (body_id[k] > n_bodies) return 1;
    memcpy(c->body_id, body_id, (size_t)c->n);
    free(c->bodies);
    free(c->row_force);
    c->n_bodies = n_bodies;
    c->bodies = (double *)calloc((size_t)(5 * (n_bodies > 0 ? n_bodies : 1)), sizeof(double));
    c->row_force = (double *)calloc((size_t)(2 * c->p.ny * (n_bodies > 0 ? n_bodies : 1)), sizeof(double));
    if (n_bodies > 0) memcpy(c->bodies, bodies, sizeof(double) * 5 * (size_t)n_bodies);
    return 0;
}

/* Centre of body b (1-based) at time level t: fixed, or c(t) = c + V t for
 * moving bodies. */
static void body_centre(const ref_ctx *c, int b, double t, double *cx, double *cy)
{
    const double *B = c->bodies + 5 * (b - 1);
    if (!c->p.moving) {
        *cx = B[0];
        *cy = B[1];
        return;
    }
    *cx = B[0] + B[2] * t;
    *cy = B[1] + B[3] * t;
}

/* rigid-body velocity of body b at node (x, y) and time level t (eq.
 * boundary-condition): U_O = V + omega z x (x - c(t)) */
static void obstacle_velocity(const ref_ctx *c, int b, double x, double y, double t, double *UOx, double *UOy)
{
    const double *B = c->bodies + 5 * (b - 1);
    double cx, cy;
    body_centre(c, b, t, &cx, &cy);
    *UOx = B[2] - B[4] * (y - cy);
    *UOy = B[3] + B[4] * (x - cx);
}

/* The mask function chi(x, t) as the body id at node (i, j), time level t. A
 * fixed mask is the one given. A moving body b, translated to c(t) and turned
 * by omega t, covers the nodes whose position carried back by that motion,
 * R(-omega t) (x - c(t)) + c, lands (to the nearest node, halves rounded up)
 * on a node of the given t = 0 mask holding b; the first such body wins. */
static int body_at(const ref_ctx *c, int i, int j, double t)
{
    if (!c->p.moving) return c->body_id[(int64_t)j * c->p.nx + i];
    for (int b = 1; b <= c->n_bodies; ++b) {
        const double *B = c->bodies + 5 * (b - 1);
        double cx, cy;
        body_centre(c, b, t, &cx, &cy);
        const double th = B[4] * t;
        const double cs = cos(th), sn = sin(th);
        const double dx = (double)i - cx, dy = (double)j - cy;
        const double xr = cs * dx + sn * dy + B[0];
        const double yr = cs * dy - sn * dx + B[1];
        const double ir = floor(xr + 0.5), jr = floor(yr + 0.5);
        if (ir < 0.0 || jr < 0.0 || ir >= (double)c->p.nx || jr >= (double)c->p.ny) continue;
        if (c->body_id[(int64_t)jr * c->p.nx + (int64_t)ir] == b) return b;
    }
    return 0;
}

int lbvp_ref_body_at(const ref_ctx *c, int32_t i, int32_t j, int64_t t_level)
{
    if (i < 0 || j < 0 || i >= c->p.nx || j >= c->p.ny) return -1;
    return body_at(c, i, j, (double)t_level);
}

/* Step (1): g = f^eq(rho0(x), u0(x)); fields(0) = (rho0, u0, 0). */
int lbvp_ref_init_equilibrium(ref_ctx *c, const double *rho, const double *ux, const double *uy)
{
    for (int64_t k = 0; k < c->n; ++k) {
        double r = rho ? rho[k] : c->p.rho0;
        double vx = ux ? ux[k] : 0.0;
        double vy = uy ? uy[k] : 0.0;
        double feq[Q];
        lbvp_ref_feq(r, vx, vy, feq);
        for (int a = 0; a < Q; ++a) c->g[a * c->n + k] = feq[a];
        c->fields[k] = r;
        c->fields[c->n + k] = vx;
        c->fields[2 * c->n + k] = vy;
        c->fields[3 * c->n + k] = 0.0;
        c->fields[4 * c->n + k] = 0.0;
    }
    c->step = 0;
    return 0;
}

/* eq. (streaming), pull form, with the domain sides resolved:
 * f_a(i, j) = g_a(i - ex_a, j - ey_a). */
static double pull(const ref_ctx *c, const double *g, int a, int i, int j)
{
    const int nx = c->p.nx, ny = c->p.ny;
    int si = i - EX[a];
    int sj = j - EY[a];
    sj = (sj % ny + ny) % ny; /* y sides are periodic */
    if (si < 0 || si >= nx) {
        int side = si < 0 ? c->p.bc_west : c->p.bc_east;
        if (side == REF_PERIODIC) {
            si = (si % nx + nx) % nx;
        } else if (side == REF_INFLOW_EQ) {
            return feq_one(a, c->p.rho_in, c->p.u_in_x, c->p.u_in_y);
        } else { /* zero gradient: the ghost column repeats the boundary column */
            si = si < 0 ? 0 : nx - 1;
        }
    }
    return g[(int64_t)a * c->n + (int64_t)sj * nx + si];
}

/* One node of the step that produces time level t (the step count after it);
 * returns the node's body id. */
static int node_update(const ref_ctx *c, const double *g, int i, int j, double t, double gout[Q], double fl[5])
{
    double f[Q];
    for (int a = 0; a < Q; ++a) f[a] = pull(c, g, a, i, j);
    int b = body_at(c, i, j, t);
    double UOx = 0.0, UOy = 0.0;
    if (b > 0) obstacle_velocity(c, b, (double)i, (double)j, t, &UOx, &UOy);
    lbvp_ref_collide_node(f, c->p.tau_plus, c->tau_minus, c->p.eta, b > 0, UOx, UOy,
                          c->p.fb_x, c->p.fb_y, gout, fl);
    return b;
}

/* Advance n steps. If forces is non-NULL it receives [n][n_bodies][2] (force on
 * each body, - sum F_VP, in fixed row order); mass receives [n] sum rho. */
int lbvp_ref_step(ref_ctx *c, int64_t n_steps, double *forces, double *mass)
{
    const int nx = c->p.nx, ny = c->p.ny, nb = c->n_bodies;
    for (int64_t s = 0; s < n_steps; ++s) {
        const double *g = c->g;
        double *gn = c->g_next;
        const double t = (double)(c->step + 1);
        /* rows in parallel only when the grid is big enough to pay for the fork */
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny >= 65536)
        for (int j = 0; j < ny; ++j) {
            double *rf = c->row_force + (int64_t)2 * nb * j;
            for (int k = 0; k < 2 * nb; ++k) rf[k] = 0.0;
            double rm = 0.0;
            for (int i = 0; i < nx; ++i) {
                double gout[Q], fl[5];
                int b = node_update(c, g, i, j, t, gout, fl);
                int64_t k = (int64_t)j * nx + i;
                for (int a = 0; a < Q; ++a) gn[(int64_t)a * c->n + k] = gout[a];
                for (int q = 0; q < 5; ++q) c->fields[(int64_t)q * c->n + k] = fl[q];
                if (b > 0) {
                    rf[2 * (b - 1)] -= fl[3];
                    rf[2 * (b - 1) + 1] -= fl[4];
                }
                rm += fl[0];
            }
            c->row_mass[j] = rm;
        }
        if (forces) {
            double *out = forces + 2 * nb * s;
            for (int k = 0; k < 2 * nb; ++k) out[k] = 0.0;
            for (int j = 0; j < ny; ++j)
                for (int k = 0; k < 2 * nb; ++k) out[k] += c->row_force[(int64_t)2 * nb * j + k];
        }
        if (mass) {
            double m = 0.0;
            for (int j = 0; j < ny; ++j) m += c->row_mass[j];
            mass[s] = m;
        }
        c->g_next = c->g;
        c->g = gn;
        c->step += 1;
    }
    return 0;
}

/* One step evaluated only at sampled nodes, from a caller-supplied lattice
 * g [Q][ny][nx] (for checking a large run node by node). */
int lbvp_ref_step_nodes(const ref_ctx *c, const double *g, int64_t n_nodes, const int32_t *xs,
                        const int32_t *ys, double *gout /* [n][Q] */, double *fields /* [n][5] */)
{
    for (int64_t k = 0; k < n_nodes; ++k) {
        if (xs[k] < 0 || xs[k] >= c->p.nx || ys[k] < 0 || ys[k] >= c->p.ny) return 1;
        double fl[5];
        node_update(c, g, xs[k], ys[k], (double)(c->step + 1), gout + Q * k, fl);
        if (fields)
            for (int q = 0; q < 5; ++q) fields[5 * k + q] = fl[q];
    }
    return 0;
}

int64_t lbvp_ref_step_count(const ref_ctx *c) { return c->step; }

/* The populations (lbvp_ref_write_populations) are those of time level `step`:
 * the next step, whole or sampled, computes level step + 1 (which is where
 * moving bodies stand). */
int lbvp_ref_set_step_count(ref_ctx *c, int64_t step)
{
    if (step < 0) return 1;
    c->step = step;
    return 0;
}

void lbvp_ref_read_fields(const ref_ctx *c, double *rho, double *ux, double *uy, double *fx, double *fy)
{
    double *dst[5] = {rho, ux, uy, fx, fy};
    for (int q = 0; q < 5; ++q)
        if (dst[q]) memcpy(dst[q], c->fields + (int64_t)q * c->n, sizeof(double) * (size_t)c->n);
}

void lbvp_ref_read_populations(const ref_ctx *c, double *g)
{
    memcpy(g, c->g, sizeof(double) * (size_t)(Q * c->n));
}

void lbvp_ref_write_populations(ref_ctx *c, const double *g)
{
    memcpy(c->g, g, sizeof(double) * (size_t)(Q * c->n));
}

int lbvp_ref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the row loops from now on (timing only; results do not depend on it). */
void lbvp_ref_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
