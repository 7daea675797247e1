/*
 * lbvp3_ref.c -- plain FP64 CPU reference of the TRT-LBM-VP method on the
 * three-dimensional D3Q19 lattice.
 *
 * TEST INFRASTRUCTURE. This file is the oracle that the HIP library's 3-D step
 * is checked against. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it. It shares no code, header, table or helper
 * with the HIP path (nor with the 2-D oracle).
 *
 * The paper's scheme (Sec. 2.2, steps (1)-(7)) is written for D2Q9 and names
 * the 3-D extension as future work (Sec. 4). Here the same steps run on D3Q19:
 * the equilibrium of eq. (feq) and the Guo term of eq. (external-force-term)
 * are the same expressions in e.u, u.u, e.F with the D3Q19 velocities and
 * weights (1/3, 1/18, 1/36), the TRT split of eqs. (TRT-collision),
 * (collision-modified) pairs each velocity with its opposite, and the
 * penalization of eqs. (d-V), (force-density), (velocity-r) is taken per
 * component. Two full lattices, every node updated by one function:
 *
 *   (3)   f_a(x) = g_a(x - e_a)                                     (streaming)
 *   (4)   rho = sum f, rho u* = sum e f + F_b/2
 *   (5)   du = chi (U_O - u*)/(2 eta + chi), F_VP = 2 rho du
 *   (6)   u = u* + du, F = F_b + F_VP, TRT collision with split forcing.
 *
 * Readings as in the 2-D oracle: tau_plus passed directly and tau_minus from
 * Lambda; the (1 - 1/(2 lambda)) factor of eq. (external-force-term) dropped;
 * corrected u in f^eq and in the Guo term; force on a body = - sum F_VP; the
 * obstacle velocity a rigid motion U_O = V + omega x (x - c) with a vector omega.
 * Sides: x sides PERIODIC, INFLOW_EQ or OUTFLOW_ZERO_GRAD (as in 2-D); y and z
 * sides periodic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define Q3 19

/* D3Q19: rest; the six face neighbours; the twelve edge neighbours, each
 * direction followed by its opposite. */
static const int EX3[Q3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY3[Q3] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ3[Q3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double W3[Q3] = {1.0 / 3.0,
                              1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP3[Q3] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
static const double CS2 = 1.0 / 3.0;

enum { R3_PERIODIC = 0, R3_INFLOW_EQ = 1, R3_OUTFLOW_ZERO_GRAD = 2 };

typedef struct ref3_params {
    int32_t nx, ny, nz;
    double tau_plus, magic_lambda, eta, rho0;
    int32_t bc_west, bc_east;             /* x sides; y and z sides are periodic */
    double rho_in, u_in[3];
    double fb[3];                         /* uniform body force F_b */
} ref3_params;

typedef struct ref3_ctx {
    ref3_params p;
    double tau_minus;
    int64_t n;                            /* nx ny nz */
    double *g, *g_next;                   /* [Q3][nz][ny][nx] */
    uint8_t *body_id;                     /* [nz][ny][nx] */
    int32_t n_bodies;
    double *bodies;                       /* [n][9]: cx cy cz vx vy vz wx wy wz */
    double *fields;                       /* [7][n]: rho ux uy uz FVPx FVPy FVPz */
    double *plane_force;                  /* [nz][n_bodies][3] */
    double *plane_mass;                   /* [nz] */
    int64_t step;
} ref3_ctx;

void lbvp3_ref_lattice(int32_t ex[Q3], int32_t ey[Q3], int32_t ez[Q3], double w[Q3], int32_t opp[Q3])
{
    for (int a = 0; a < Q3; ++a) {
        ex[a] = EX3[a];
        ey[a] = EY3[a];
        ez[a] = EZ3[a];
        w[a] = W3[a];
        opp[a] = OPP3[a];
    }
}

/* eq. (feq) on D3Q19 */
static double feq3_one(int a, double rho, const double u[3])
{
    double eu = EX3[a] * u[0] + EY3[a] * u[1] + EZ3[a] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return rho * W3[a] * (1.0 + eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2));
}

void lbvp3_ref_feq(double rho, const double u[3], double out[Q3])
{
    for (int a = 0; a < Q3; ++a) out[a] = feq3_one(a, rho, u);
}

/* eq. (external-force-term) without the (1 - 1/(2 lambda)) factor */
void lbvp3_ref_guo(const double u[3], const double F[3], double out[Q3])
{
    for (int a = 0; a < Q3; ++a) {
        const double e[3] = {EX3[a], EY3[a], EZ3[a]};
        double eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s += ((e[d] - u[d]) / CS2 + eu * e[d] / (CS2 * CS2)) * F[d];
        out[a] = W3[a] * s;
    }
}

/* eqs. (TRT-collision), (collision-modified) with opposite pairs */
void lbvp3_ref_trt_collide(const double f[Q3], const double feq[Q3], const double F[Q3], double tau_s,
                           double tau_a, double g[Q3])
{
    for (int a = 0; a < Q3; ++a) {
        int b = OPP3[a];
        double fs = 0.5 * (f[a] + f[b]), fa = 0.5 * (f[a] - f[b]);
        double es = 0.5 * (feq[a] + feq[b]), ea = 0.5 * (feq[a] - feq[b]);
        double Fs = 0.5 * (F[a] + F[b]), Fa = 0.5 * (F[a] - F[b]);
        double omega = -(fs - es) / tau_s - (fa - ea) / tau_a;
        g[a] = f[a] + omega + (1.0 - 1.0 / (2.0 * tau_s)) * Fs + (1.0 - 1.0 / (2.0 * tau_a)) * Fa;
    }
}

/* Steps (4)-(6) at one node: fields = rho, ux, uy, uz, FVPx, FVPy, FVPz */
void lbvp3_ref_collide_node(const double f[Q3], double tau_s, double tau_a, double eta, int chi,
                            const double UO[3], const double fb[3], double g[Q3], double fields[7])
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < Q3; ++a) {
        rho += f[a];
        j[0] += EX3[a] * f[a];
        j[1] += EY3[a] * f[a];
        j[2] += EZ3[a] * f[a];
    }
    double c = chi ? 1.0 : 0.0;
    double u[3], F[3], fvp[3];
    for (int d = 0; d < 3; ++d) {
        double us = (j[d] + 0.5 * fb[d]) / rho;
        double du = c * (UO[d] - us) / (2.0 * eta + c);
        fvp[d] = 2.0 * rho * c * (UO[d] - us) / (2.0 * eta + c);
        u[d] = us + du;
        F[d] = fb[d] + fvp[d];
    }
    double feq[Q3], Fa[Q3];
    lbvp3_ref_feq(rho, u, feq);
    lbvp3_ref_guo(u, F, Fa);
    lbvp3_ref_trt_collide(f, feq, Fa, tau_s, tau_a, g);
    fields[0] = rho;
    for (int d = 0; d < 3; ++d) {
        fields[1 + d] = u[d];
        fields[4 + d] = fvp[d];
    }
}

/* ------------------------------------------------------------ the solver --- */

static int valid3_side(int32_t s) { return s == R3_PERIODIC || s == R3_INFLOW_EQ || s == R3_OUTFLOW_ZERO_GRAD; }

ref3_ctx *lbvp3_ref_create(const ref3_params *p)
{
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || !(p->tau_plus > 0.5) || !(p->magic_lambda > 0.0) ||
        !(p->eta > 0.0) || !valid3_side(p->bc_west) || !valid3_side(p->bc_east) ||
        ((p->bc_west == R3_PERIODIC) != (p->bc_east == R3_PERIODIC)))
        return NULL;
    ref3_ctx *c = (ref3_ctx *)calloc(1, sizeof(ref3_ctx));
    if (!c) return NULL;
    c->p = *p;
    c->tau_minus = 0.5 + p->magic_lambda / (p->tau_plus - 0.5);
    c->n = (int64_t)p->nx * p->ny * p->nz;
    c->g = (double *)calloc((size_t)(Q3 * c->n), sizeof(double));
    c->g_next = (double *)calloc((size_t)(Q3 * c->n), sizeof(double));
    c->body_id = (uint8_t *)calloc((size_t)c->n, 1);
    c->fields = (double *)calloc((size_t)(7 * c->n), sizeof(double));
    c->plane_mass = (double *)calloc((size_t)p->nz, sizeof(double));
    c->bodies = (double *)calloc(9, sizeof(double));
    c->plane_force = (double *)calloc((size_t)(3 * p->nz), sizeof(double));
    if (!c->g || !c->g_next || !c->body_id || !c->fields || !c->plane_mass || !c->bodies || !c->plane_force) {
        free(c->g); free(c->g_next); free(c->body_id); free(c->fields); free(c->plane_mass);
        free(c->bodies); free(c->plane_force); free(c);
        return NULL;
    }
    return c;
}

void lbvp3_ref_destroy(ref3_ctx *c)
{
    if (!c) return;
    free(c->g); free(c->g_next); free(c->body_id); free(c->fields); free(c->plane_mass);
    free(c->bodies); free(c->plane_force); free(c);
}

int lbvp3_ref_set_mask(ref3_ctx *c, const uint8_t *body_id, int32_t n_bodies, const double *bodies)
{
    if (n_bodies < 0 || n_bodies > 255) return 1;
    for (int64_t k = 0; k < c->n; ++k)
        if (body_id[k] > n_bodies) return 1;
    memcpy(c->body_id, body_id, (size_t)c->n);
    free(c->bodies);
    free(c->plane_force);
    c->n_bodies = n_bodies;
    c->bodies = (double *)calloc((size_t)(9 * (n_bodies > 0 ? n_bodies : 1)), sizeof(double));
    c->plane_force = (double *)calloc((size_t)(3 * c->p.nz * (n_bodies > 0 ? n_bodies : 1)), sizeof(double));
    if (!c->bodies || !c->plane_force) return 2;
    if (n_bodies > 0) memcpy(c->bodies, bodies, sizeof(double) * 9 * (size_t)n_bodies);
    return 0;
}

/* U_O = V + omega x (x - c) of body b (1-based) at node (x, y, z) */
static void obstacle3_velocity(const ref3_ctx *c, int b, double x, double y, double z, double UO[3])
{
    const double *B = c->bodies + 9 * (b - 1);
    double r[3] = {x - B[0], y - B[1], z - B[2]};
    UO[0] = B[3] + (B[7] * r[2] - B[8] * r[1]);
    UO[1] = B[4] + (B[8] * r[0] - B[6] * r[2]);
    UO[2] = B[5] + (B[6] * r[1] - B[7] * r[0]);
}

int lbvp3_ref_init_equilibrium(ref3_ctx *c, const double *rho, const double *ux, const double *uy, const double *uz)
{
    for (int64_t k = 0; k < c->n; ++k) {
        double r = rho ? rho[k] : c->p.rho0;
        double u[3] = {ux ? ux[k] : 0.0, uy ? uy[k] : 0.0, uz ? uz[k] : 0.0};
        double feq[Q3];
        lbvp3_ref_feq(r, u, feq);
        for (int a = 0; a < Q3; ++a) c->g[a * c->n + k] = feq[a];
        c->fields[k] = r;
        for (int d = 0; d < 3; ++d) {
            c->fields[(1 + d) * c->n + k] = u[d];
            c->fields[(4 + d) * c->n + k] = 0.0;
        }
    }
    c->step = 0;
    return 0;
}

/* eq. (streaming), pull form, with the x sides resolved */
static double pull3(const ref3_ctx *c, const double *g, int a, int i, int j, int k)
{
    const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
    int si = i - EX3[a];
    int sj = ((j - EY3[a]) % ny + ny) % ny;
    int sk = ((k - EZ3[a]) % nz + nz) % nz;
    if (si < 0 || si >= nx) {
        int side = si < 0 ? c->p.bc_west : c->p.bc_east;
        if (side == R3_PERIODIC) {
            si = (si % nx + nx) % nx;
        } else if (side == R3_INFLOW_EQ) {
            return feq3_one(a, c->p.rho_in, c->p.u_in);
        } else {
            si = si < 0 ? 0 : nx - 1;
        }
    }
    return g[(int64_t)a * c->n + ((int64_t)sk * ny + sj) * nx + si];
}

static int node3_update(const ref3_ctx *c, const double *g, int i, int j, int k, double gout[Q3], double fl[7])
{
    double f[Q3];
    for (int a = 0; a < Q3; ++a) f[a] = pull3(c, g, a, i, j, k);
    int b = c->body_id[((int64_t)k * c->p.ny + j) * c->p.nx + i];
    double UO[3] = {0.0, 0.0, 0.0};
    if (b > 0) obstacle3_velocity(c, b, (double)i, (double)j, (double)k, UO);
    lbvp3_ref_collide_node(f, c->p.tau_plus, c->tau_minus, c->p.eta, b > 0, UO, c->p.fb, gout, fl);
    return b;
}

/* Advance n steps; forces [n][n_bodies][3] (force on each body, - sum F_VP, summed
 * plane by plane in a fixed order) and mass [n] (sum rho), each nullable. */
int lbvp3_ref_step(ref3_ctx *c, int64_t n_steps, double *forces, double *mass)
{
    const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz, nb = c->n_bodies;
    for (int64_t s = 0; s < n_steps; ++s) {
        const double *g = c->g;
        double *gn = c->g_next;
#pragma omp parallel for schedule(static) if (c->n >= 4096)
        for (int k = 0; k < nz; ++k) {
            double *pf = c->plane_force + (int64_t)3 * nb * k;
            for (int q = 0; q < 3 * nb; ++q) pf[q] = 0.0;
            double pm = 0.0;
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    double gout[Q3], fl[7];
                    int b = node3_update(c, g, i, j, k, gout, fl);
                    int64_t x = ((int64_t)k * ny + j) * nx + i;
                    for (int a = 0; a < Q3; ++a) gn[(int64_t)a * c->n + x] = gout[a];
                    for (int q = 0; q < 7; ++q) c->fields[(int64_t)q * c->n + x] = fl[q];
                    if (b > 0)
                        for (int d = 0; d < 3; ++d) pf[3 * (b - 1) + d] -= fl[4 + d];
                    pm += fl[0];
                }
            c->plane_mass[k] = pm;
        }
        if (forces) {
            double *out = forces + 3 * nb * s;
            for (int q = 0; q < 3 * nb; ++q) out[q] = 0.0;
            for (int k = 0; k < nz; ++k)
                for (int q = 0; q < 3 * nb; ++q) out[q] += c->plane_force[(int64_t)3 * nb * k + q];
        }
        if (mass) {
            double m = 0.0;
            for (int k = 0; k < nz; ++k) m += c->plane_mass[k];
            mass[s] = m;
        }
        c->g_next = c->g;
        c->g = gn;
        c->step += 1;
    }
    return 0;
}

int64_t lbvp3_ref_step_count(const ref3_ctx *c) { return c->step; }

void lbvp3_ref_read_fields(const ref3_ctx *c, double *out /* [7][n] */)
{
    memcpy(out, c->fields, sizeof(double) * 7 * (size_t)c->n);
}

void lbvp3_ref_read_populations(const ref3_ctx *c, double *g)
{
    memcpy(g, c->g, sizeof(double) * (size_t)(Q3 * c->n));
}

void lbvp3_ref_write_populations(ref3_ctx *c, const double *g)
{
    memcpy(c->g, g, sizeof(double) * (size_t)(Q3 * c->n));
}

/* One step at selected nodes from a given population array g [Q3][nz][ny][nx]
 * (the context's own lattice is untouched): gout [n][Q3], fields [n][7]. */
int lbvp3_ref_step_nodes(const ref3_ctx *c, const double *g, int64_t n_nodes, const int32_t *xs,
                         const int32_t *ys, const int32_t *zs, double *gout, double *fields)
{
    for (int64_t k = 0; k < n_nodes; ++k) {
        if (xs[k] < 0 || xs[k] >= c->p.nx || ys[k] < 0 || ys[k] >= c->p.ny || zs[k] < 0 || zs[k] >= c->p.nz)
            return 1;
        double fl[7];
        node3_update(c, g, xs[k], ys[k], zs[k], gout + Q3 * k, fl);
        if (fields)
            for (int q = 0; q < 7; ++q) fields[7 * k + q] = fl[q];
    }
    return 0;
}

int lbvp3_ref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void lbvp3_ref_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
