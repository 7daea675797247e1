// lbvp_kernels.hip -- gfx950 kernels of the fused D2Q9 TRT-VP time step.
//
// Data layout in HBM (rows of structures of arrays): population a of node (i, j)
// lives at lattice[j * lstride + a * plane + i] with plane = pitch and
// lstride = 9 pitch: the nine population rows of a lattice row lie back to back.
// pitch is a multiple of 64 elements, so every population row starts on a
// 128-byte (2-byte types) or 256-byte boundary. A tile's loads and stores then
// stay within a few neighbouring lattice rows of memory instead of touching
// nine planes a whole domain apart, which HBM serves measurably faster. All storage types hold the
// weight-normalized deviation h_a = (f_a - w_a rho0) / w_a. Its size is set by
// the flow (|h| ~ 3|u|) and is the same for every direction, and the equilibrium
// in these units carries no weight at all,
//   h^eq_a = drho + rho (3 eu + 9/2 eu^2 - 3/2 u.u),
// while the moments use the exact integers 36 w_a = 16, 4, 1:
//   36 drho = 16 h_0 + 4 sum_axis h + sum_diag h,  36 j = 4 sum_axis e h + sum_diag e h.
// In FP32 the inexact weights 1/9 and 1/36 would otherwise bias every collision's
// momentum by ~1e-8, which a freely decaying flow accumulates step after step.
//
// One step (Sec. 2.2, steps (2)-(6)), per node, fused:
//   pull   f_a(x) = g_a(x - e_a)                      eq. (streaming)
//   rho = rho0 + sum w_a h_a,  rho u* = sum e_a w_a h_a + F_b/2   eqs. (rho), (rho*velocity-star)
//   chi from the mask, U_O = V + omega z x (x - c) of the node's body
//   du = chi (U_O - u*) / (2 eta + chi),  F_VP = 2 rho du    eqs. (d-V), (force-density)
//   u = u* + du,  F = F_b + F_VP                       eq. (velocity-r)
//   g_a = f_a - (f+_a - f^eq+_a)/tau+ - (f-_a - f^eq-_a)/tau-
//         + (1 - 1/(2 tau+)) F+_a + (1 - 1/(2 tau-)) F-_a        eqs. (TRT-collision), (collision-modified)
// with f^eq of eq. (feq) and F_a of eq. (external-force-term), both taken at the
// corrected u and split into parts even (+) and odd (-) under a -> opposite(a).
// For a pair (a, opposite a) with eu = e_a.u and eF = e_a.F the parts are, in
// units of w_a,
//   h^eq+ = drho + rho (9/2 eu^2 - 3/2 u.u),  h^eq- = 3 rho eu = e.(36 j + 18 F)/12,
//   F+/w  = 9 eu eF - 3 u.F,                 F-/w  = 3 eF.
//
// The step is bound by HBM traffic: 9 loads, 9 stores and one mask byte per node
// against ~200 flops, so there is no matrix-core work here. What limits it is
// the bytes in flight: each thread owns V consecutive nodes of a row and moves
// every population with one aligned V-wide (16-byte) load and store. The pull
// from x -/+ 1 takes the missing end element from the neighbouring lane of the
// wavefront (a lane shuffle); the two lanes at a wavefront's ends load it
// themselves, with the domain sides resolved there.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lbvp_device.h"
#include "lbvp_internal.h"

namespace lbvp {
namespace {


template <typename R>
struct NodeResult {
    R drho, rho, ux, uy, fvx, fvy;
};

// One row of the body table (see StepArgs::bodies): the centre split into its
// nearest integer and the remainder, then V and omega.
template <typename R>
struct BodyRow {
    R cxi, cyi, cxf, cyf, vx, vy, om;
};

template <typename R>
__device__ __forceinline__ BodyRow<R> body_row(const R* B)
{
    return {B[0], B[1], B[2], B[3], B[4], B[5], B[6]};
}

// Where a solid node finds its body's row: `uniform` when every solid node of
// the tile belongs to one body, whose row was then read once per tile (scalar
// loads, before any store); otherwise each node reads its own row.
template <typename R>
struct BodySource {
    bool uniform;
    BodyRow<R> row;
    const double* pose;   // moving bodies: the poses at this step's time level, else null
    uint32_t near;        // moving bodies whose reach meets the tile (bit b - 1 for body b)
};

// Volume penalization of a solid node (eqs. d-V, force-density): U_O = V +
// omega z x (x - c), du = (U_O - u*) / (2 eta + 1), F_VP = 2 rho du, u = u* + du.
// x - c comes from the split centre (a centre rounded to FP32 whole would be off
// by up to half an FP32 spacing, 1/512 node near x = 32768, the same for every
// node of the body); a moving body's centre at time t is FP64.
template <typename R, bool MOVING>
__device__ __forceinline__ void penalize(const BodySource<R>& src, int body, int i, int j, const StepArgs<R>& a,
                                         R rho, R& ux, R& uy, R& fvx, R& fvy)
{
    BodyRow<R> B;
    if (src.uniform) B = src.row;
    else B = body_row(a.bodies + BODY_STRIDE * body);
    R rx, ry;
    if (MOVING && src.pose) {
        const double* m = src.pose + (body - 1) * POSE_STRIDE;
        rx = (R)((double)i - m[2]);
        ry = (R)((double)j - m[3]);
    } else {
        rx = ((R)i - B.cxi) - B.cxf;
        ry = ((R)j - B.cyi) - B.cyf;
    }
    const R uox = B.vx - B.om * ry;
    const R uoy = B.vy + B.om * rx;
    const R dux = a.vp_c * (uox - ux);
    const R duy = a.vp_c * (uoy - uy);
    fvx = R(2) * rho * dux;
    fvy = R(2) * rho * duy;
    ux += dux;
    uy += duy;
}

// Steps (4)-(6) of the algorithm at node (i, j) with streamed populations f;
// overwrites f with the post-collision populations.
// EXACT_MOM: the odd equilibrium from the momentum (momentum3); the 2-byte
// storage types take 3 rho u as (3 rho) u instead, whose ~1e-8 momentum bias is
// far below their own rounding, for two fewer quotients per node.
template <typename R, bool MOVING = false, bool EXACT_MOM = true>
__device__ __forceinline__ NodeResult<R> collide_node(R (&f)[9], int body, int i, int j, const StepArgs<R>& a,
                                                    const BodySource<R>& bs)
{
    // moments with the integers 36 w_a = 16, 4, 1 (sum w_a rho0 = rho0 and
    // sum e_a w_a = 0 drop out); 1/36 and 1/rho through div36 / recip
    const R s36 = R(16) * f[0] + (R(4) * ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
    const R drho = div36(s36);
    const R rho = a.rho0 + drho;
    const R d57 = f[5] - f[7], d86 = f[8] - f[6];
    const R inv_36rho = recip(R(36) * rho);
    // u* = (j + F_b/2) / rho with 36 j = 4 (h1 - h3) + ... (eq. rho*velocity-star)
    const R jx36 = R(4) * (f[1] - f[3]) + (d57 + d86) + a.fbx18;
    const R jy36 = R(4) * (f[2] - f[4]) + (d57 - d86) + a.fby18;
    R ux = jx36 * inv_36rho;
    R uy = jy36 * inv_36rho;

    // volume penalization (eqs. d-V, force-density) on solid nodes only
    R fvx = R(0), fvy = R(0);
    if (body) penalize<R, MOVING>(bs, body, i, j, a, rho, ux, uy, fvx, fvy);
    const R Fx = a.fbx + fvx, Fy = a.fby + fvy;
    R px, py;   // 3 rho u
    if constexpr (EXACT_MOM) {
        px = momentum3(jx36, fvx);
        py = momentum3(jy36, fvy);
    } else {
        const R rho3 = R(3) * rho;
        px = rho3 * ux;
        py = rho3 * uy;
    }

    NodeTerms<R> n;
    const R uu = ux * ux + uy * uy;
    n.A = drho - (R(1.5) * rho) * uu;
    n.rho45 = R(4.5) * rho;
    n.uF3 = R(-3) * (ux * Fx + uy * Fy);
    const R g0 = a.om_p * (n.A - f[0]) + f[0] + a.k_p * n.uF3;
    const Pair<R> p13 = collide_pair(f[1], f[3], ux, px, Fx, n, a);
    const Pair<R> p24 = collide_pair(f[2], f[4], uy, py, Fy, n, a);
    const Pair<R> p57 = collide_pair(f[5], f[7], ux + uy, px + py, Fx + Fy, n, a);
    const Pair<R> p68 = collide_pair(f[6], f[8], uy - ux, py - px, Fy - Fx, n, a);
    f[0] = g0;
    f[1] = p13.ga;
    f[3] = p13.gb;
    f[2] = p24.ga;
    f[4] = p24.gb;
    f[5] = p57.ga;
    f[7] = p57.gb;
    f[6] = p68.ga;
    f[8] = p68.gb;
    return {drho, rho, ux, uy, fvx, fvy};
}

// The same steps for the 2-byte storage types, whose stored values carry a
// rounding error (~1e-3 relative) far above any FP32 arithmetic detail, in the
// fewest operations: 1/36 and 1/rho as single roundings, the odd equilibrium as
// (3 rho) e.u, and each pair's two relaxations regrouped into
//   g_a     = c1 h_a + c2 h_opp + (E+ + E-),
//   g_opp   = c2 h_a + c1 h_opp + (E+ - E-),
//   E+ = om_p h^eq+ + k_p F+/w = eu (9/2 om_p rho eu + 9 k_p eF) + B,
//   E- = om_m h^eq- + k_m F-/w = 3 om_m rho eu + 3 k_m eF,
//   B  = om_p (drho - 3/2 rho u.u) - 3 k_p u.F,
// with c1 = 1 - (om_p + om_m)/2, c2 = (om_m - om_p)/2 (algebraically the
// relaxation of collide_pair); the rest population is g_0 = (1 - om_p) h_0 + B.
// About 85 operations per node instead of about 125.
template <typename R, bool MOVING = false>
__device__ __forceinline__ NodeResult<R> collide_node_lowp(R (&f)[9], int body, int i, int j, const StepArgs<R>& a,
                                                         const BodySource<R>& bs)
{
    const R s36 = R(16) * f[0] + (R(4) * ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
    const R drho = s36 * R(1.0 / 36.0);
    const R rho = a.rho0 + drho;
    const R d57 = f[5] - f[7], d86 = f[8] - f[6];
    const R inv_36rho = __builtin_amdgcn_rcpf(R(36) * rho);
    const R jx36 = R(4) * (f[1] - f[3]) + (d57 + d86) + a.fbx18;
    const R jy36 = R(4) * (f[2] - f[4]) + (d57 - d86) + a.fby18;
    R ux = jx36 * inv_36rho;
    R uy = jy36 * inv_36rho;
    R fvx = R(0), fvy = R(0);
    if (body) penalize<R, MOVING>(bs, body, i, j, a, rho, ux, uy, fvx, fvy);
    const R Fx = a.fbx + fvx, Fy = a.fby + fvy;
    const R uu = ux * ux + uy * uy;
    const R uF = ux * Fx + uy * Fy;
    const R B0 = a.om_p * drho - (a.om_p15 * (rho * uu) + a.k_p3 * uF);
    const R a1 = a.om_p45 * rho;
    const R r3m = a.om_m3 * rho;
    const R g0 = a.om_p1 * f[0] + B0;
    auto pair = [&](R& ha, R& hb, R eu, R eF) {
        const R t = a1 * eu + a.k_p9 * eF;
        const R ep = eu * t + B0;
        const R em = r3m * eu + a.k_m3 * eF;
        const R sum = ep + em, dif = ep - em;
        const R ga = a.c1 * ha + (a.c2 * hb + sum);
        const R gb = a.c2 * ha + (a.c1 * hb + dif);
        ha = ga;
        hb = gb;
    };
    pair(f[1], f[3], ux, Fx);
    pair(f[2], f[4], uy, Fy);
    pair(f[5], f[7], ux + uy, Fx + Fy);
    pair(f[6], f[8], uy - ux, Fy - Fx);
    f[0] = g0;
    return {drho, rho, ux, uy, fvx, fvy};
}

// Moving masks: the body occupying node (i, j) at the step's time level. Node
// x belongs to body b when the reference (t = 0) mask holds b at the node
// nearest to R(-th) (x - c(t)) + c(0), the node carried back by the body's
// rigid motion; the first such body in order wins. Evaluated in FP64 one
// operation per statement (no fused multiply-adds), so that membership does
// not depend on the storage type. Only the bodies in `near` are tried (the
// tile's, see tile_near_bodies); nodes outside a body's radius skip it.
template <typename R>
__device__ __forceinline__ int moving_body(const StepArgs<R>& a, const double* row, uint32_t near, int i, int j)
{
    for (uint32_t bits = near; bits; bits &= bits - 1) {
        const int b = __builtin_ctz(bits);
        const double* m = row + b * POSE_STRIDE;
        const double dx = (double)i - m[2];
        const double dy = (double)j - m[3];
        const double dx2 = dx * dx;
        const double dy2 = dy * dy;
        if (dx2 + dy2 > m[6]) continue;
        const double a1 = m[0] * dx;
        const double a2 = m[1] * dy;
        const double s1 = a1 + a2;
        const double xr = s1 + m[4];
        const double b1 = m[0] * dy;
        const double b2 = m[1] * dx;
        const double s2 = b1 - b2;
        const double yr = s2 + m[5];
        const double fx = floor(xr + 0.5);
        const double fy = floor(yr + 0.5);
        if (fx < 0.0 || fy < 0.0 || fx >= (double)a.nx || fy >= (double)a.ny) continue;
        if (a.mask[(int64_t)fy * a.pitch + (int64_t)fx] == b + 1) return b + 1;
    }
    return 0;
}

// The moving bodies whose radius reaches the rectangle [x0, x1] x [y0, y1] (a
// tile), as bits. Skipping the others for the tile's nodes changes nothing:
// rounding is monotone, so a node's FP64 squared distance to a centre, computed
// as in moving_body, is never below the rectangle's computed the same way.
template <typename R>
__device__ __forceinline__ uint32_t tile_near_bodies(const StepArgs<R>& a, const double* row, double x0, double x1,
                                                     double y0, double y1)
{
    uint32_t near = 0;
    for (int b = 0; b < a.n_moving; ++b) {
        const double* m = row + b * POSE_STRIDE;
        const double ex = m[2] < x0 ? x0 - m[2] : (m[2] > x1 ? m[2] - x1 : 0.0);
        const double ey = m[3] < y0 ? y0 - m[3] : (m[3] > y1 ? m[3] - y1 : 0.0);
        const double ex2 = ex * ex;
        const double ey2 = ey * ey;
        if (!(ex2 + ey2 > m[6])) near |= 1u << b;
    }
    return near;
}

// D2Q9 directions (eq. D2Q9) and the opposite map (Sec. 2.1: f_{-1} = f_3).
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr int EXQ[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
// Directions by x component, with rows ey = 0, +1, -1 for m = 0, 1, 2.
constexpr int EXP[3] = {1, 5, 8};   // ex = +1: pulled from column i - 1
constexpr int EXM[3] = {3, 6, 7};   // ex = -1: pulled from column i + 1

// Step kinds. PULL: two lattices, g(n) -> g(n + 1), every node pulls its nine
// populations from its neighbours' slots of the source lattice. The AA pattern
// runs on one lattice in two alternating kinds:
//   AA_PUSH  (n even) reads g_q(x - e_q) from slot opp(q) of the neighbour and
//            writes g_q(x) into slot q of the neighbour x + e_q, so that the
//            lattice then holds the streamed populations in place;
//   AA_LOCAL (n odd) reads its own slots q and writes its own slots opp(q).
// Each slot is read and written by one node only, so one buffer suffices. The
// domain sides: in AA_PUSH populations leaving through a non-periodic side are
// dropped and the ones entering are written into the boundary node's slots
// (inflow: the equilibrium; zero-gradient outflow: the boundary column's own
// outgoing value); the outflow values that AA_PUSH pulls come from a ghost
// column that AA_LOCAL writes, because the lattice slot holding them is
// overwritten by a neighbour in the same kernel.
enum Mode { PULL = 0, AA_PUSH = 1, AA_LOCAL = 2 };

// Population q pulled from column c (-1 and nx are outside the domain) of plane
// `plane_q` in the row starting at row_off (row index `row`): the domain sides
// are resolved here. A NEIGHBOR side (a cut of a slab decomposition) reads the
// halo column that lbvp_halo_exchange wrote into the current lattice's padding
// (column nx for the east side, pitch - 1 for the west; a context with a cut has
// pitch >= nx + 2), so it is one more column choice, like a periodic side, with
// the same single load. Ghost populations are values of the storage type, like
// every other population (the AA push step stores the inflow ones in the
// lattice), so the inflow equilibrium is rounded to it.
template <int MODE, typename S, typename R>
__device__ __forceinline__ R pull_column(const S* src, int q, int plane_q, int64_t row_off, int row, int c,
                                         const StepArgs<R>& a)
{
    if (c < 0) {
        if (a.west == SIDE_INFLOW_EQ) return dec(enc<S>(a.feq_in[q]));
        if (MODE == AA_PUSH && a.west == SIDE_OUTFLOW)
            return dec(static_cast<const S*>(a.ghost_w)[(q == 1 ? 0 : q == 5 ? 1 : 2) * (int64_t)a.ny + row]);
        // a cut's west halo lives in the row's last padding column
        c = (a.west == SIDE_PERIODIC) ? a.nx - 1 : (a.west == SIDE_NEIGHBOR ? (int)a.pitch - 1 : 0);
    } else if (c >= a.nx) {
        if (a.east == SIDE_INFLOW_EQ) return dec(enc<S>(a.feq_in[q]));
        if (MODE == AA_PUSH && a.east == SIDE_OUTFLOW)
            return dec(static_cast<const S*>(a.ghost_e)[(q == 3 ? 0 : q == 6 ? 1 : 2) * (int64_t)a.ny + row]);
        // a cut's east halo lives in column nx, the first padding column
        c = (a.east == SIDE_PERIODIC) ? 0 : (a.east == SIDE_NEIGHBOR ? a.nx : a.nx - 1);
    }
    return dec(src[(int64_t)plane_q * a.plane + row_off + c]);
}



__device__ __forceinline__ void finalize_record(const FinalizeArgs& f, int buf, double* lds)
{
    const double* pm = f.mass_part + buf * f.mass_stride;
    const double* sf = f.slot_force + buf * f.slot_stride;
    double* sx = lds;
    double* sy = lds + FIN_LANES;
    for (int v = (int)threadIdx.x; v < FIN_LANES; v += (int)blockDim.x) sx[v] = lane_sum(pm, f.n_mass, v);
    const double m = tree_sum(sx);
    const int64_t r = *f.rec_count % f.capacity;
    for (int b = 0; b < f.n_bodies; ++b) {
        const int s0 = f.body_slot_ptr[b], s1 = f.body_slot_ptr[b + 1];
        for (int v = (int)threadIdx.x; v < FIN_LANES; v += (int)blockDim.x) {
            double x = 0.0, y = 0.0;
            int k = s0 + v;
            // four slots' loads in flight at a time, added in the same order
            for (; k + 3 * FIN_LANES < s1; k += 4 * FIN_LANES) {
                int sl[4];
                double px[4], py[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) sl[u] = f.body_slots[k + u * FIN_LANES];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    px[u] = sf[2 * sl[u]];
                    py[u] = sf[2 * sl[u] + 1];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    x += px[u];
                    y += py[u];
                }
            }
            for (; k < s1; k += FIN_LANES) {
                const int sl = f.body_slots[k];
                x += sf[2 * sl];
                y += sf[2 * sl + 1];
            }
            sx[v] = x;
            sy[v] = y;
        }
        const double x = tree_sum(sx);
        const double y = tree_sum(sy);
        if (threadIdx.x == 0) {
            f.ring_force[(r * f.max_bodies + b) * 2] = x;
            f.ring_force[(r * f.max_bodies + b) * 2 + 1] = y;
        }
    }
    if (threadIdx.x == 0) {
        f.ring_mass[r] = f.mass_offset + m;
        *f.rec_count += 1;
    }
}

// ------------------------------------------------------------ the step --

// One block updates tile t of a domain: tile_rows rows of tile_w nodes, V
// consecutive nodes per thread. part_buf: the partial buffer this step's record
// writes (the previous record is summed by leading blocks of the same launch).
// lds: the kernel's 2 FIN_LANES doubles.
// OFF32 (2-byte storage, vector pull form, a lattice under 4 GiB): the main
// loads and stores address a uniform population-row base plus a 32-bit per-lane
// byte offset, which the scalar-base addressing mode takes directly.
template <typename S, int V, int MODE, bool RECORD, bool FIELDS, bool MOVING = false, bool OFF32 = false>
__device__ __forceinline__ void step_body(const S* src, S* dst, const StepArgs<typename Arith<S>::R>& a, int t,
                                          int part_buf, double* lds, int pose_k = 0)
{
    using R = typename Arith<S>::R;
    int s0 = 0, s1 = 0;          // this tile's (tile, body) force slots
    BodySource<R> bs;
    bs.uniform = false;
    bs.pose = nullptr;
    bs.near = 0;
    if constexpr (MOVING) {      // the poses at this step's time level (a domain with moving bodies)
        if (a.n_moving > 0) bs.pose = a.pose + (*a.pose_base + pose_k) * (int64_t)(MAX_MOVING * POSE_STRIDE);
    }
    {
        s0 = a.tile_slot_ptr[t];
        s1 = a.tile_slot_ptr[t + 1];
        // the slots list every body with a node in the tile: with none, the
        // tile's mask is not read at all; with one, its row serves every solid
        // node of the tile (read here, before any store)
        if (s1 - s0 == 1) {
            bs.uniform = true;
            bs.row = body_row(a.bodies + BODY_STRIDE * a.slot_body[s0]);
        }
    }
    const int ty = t / a.tiles_x, tx = t - ty * a.tiles_x;
    const int tpr = a.tile_w / V;                       // threads per tile row (tile_w and V are powers of two)
    const int lr = (int)threadIdx.x >> __builtin_ctz((unsigned)tpr), lc = (int)threadIdx.x & (tpr - 1);
    const int j = min(ty * a.tile_rows + lr, a.ny - 1); // rows past ny idle (clamped for addressing)
    const int i0 = tx * a.tile_w + lc * V;
    const int lane = (int)(threadIdx.x & 63);
    const bool act = i0 < a.nx && ty * a.tile_rows + lr < a.ny;   // owns at least one real node
    const int n_own = act ? min(V, a.nx - i0) : 0;
    if constexpr (MOVING) {
        if (bs.pose) {   // once per tile: most tiles meet no moving body
            // only the bodies the tile's slots list can reach it during the
            // pose window (none for most tiles); of those, the ones whose
            // radius about this step's centre meets the tile
            uint32_t listed = 0;
            for (int s = s0; s < s1; ++s) listed |= 1u << (a.slot_body[s] - 1);
            if (listed) {
                const double x0 = (double)(tx * a.tile_w), y0 = (double)(ty * a.tile_rows);
                bs.near = listed & __builtin_amdgcn_readfirstlane(tile_near_bodies(
                                       a, bs.pose, x0, x0 + (double)(a.tile_w - 1), y0, y0 + (double)(a.tile_rows - 1)));
            }
        }
    }

    const int jm = (j == 0) ? a.ny - 1 : j - 1;     // rows are periodic
    const int jp = (j == a.ny - 1) ? 0 : j + 1;
    const int64_t r0 = (int64_t)j * a.pitch;   // mask and fields
    const int64_t l0 = (int64_t)j * a.lstride, lm = (int64_t)jm * a.lstride, lp = (int64_t)jp * a.lstride;
    // lattice pull source row of each direction (ey = 0 -> j, +1 -> j - 1,
    // -1 -> j + 1) and push target row (the opposite)
    const int64_t row_of[9] = {l0, l0, lm, l0, lp, lm, lm, lp, lp};
    const int row_idx[9] = {j, j, jm, j, jp, jm, jm, jp, jp};
    const int64_t row_to[9] = {l0, l0, lp, l0, lm, lp, lp, lm, lm};
    const int64_t P = a.plane;

    // Source plane of direction q: the pull and the AA local step read plane q,
    // the AA push step the neighbour's opposite slot. FP32 vectors, single
    // nodes and the AA steps take the x-shifted directions as single accesses
    // one element off alignment (columns i0 - 1 .. or i0 + 1 ..; both stay
    // inside the allocation: population 0 of row 0 is never shifted left, the
    // last population row (8 of row ny - 1) is never shifted right, and every
    // other population row is preceded and followed by another). FP64 and
    // FP16/BF16 vectors of the pull step load aligned and shift through lane
    // moves (FP64: 0.787 -> 0.783 ms and no line-straddling reads; FP32 measured
    // the same either way).
    constexpr bool kShifted = sizeof(S) == 4 || V == 1 || MODE != PULL;
    static_assert(MODE == PULL || kShifted, "the AA pattern needs dword-or-wider elements or one node per thread");
    // The lane-shuffle form (FP64 and 2-byte types, V > 1, pull) keeps the
    // loaded values in the storage type and decodes each node's nine just before
    // its collision, so that the packed loads, not 9 V decoded floats, stay live
    // across the tile.
    using LV = typename std::conditional<kShifted, R, S>::type;
    LV v[9][V];
    int body[V];
    // Threads without a node of their own (past the last column or row) load
    // column 0 of their (clamped) row instead: every access stays inside the
    // lattice, no branch or register clearing is needed, and their results are
    // never stored, summed or shuffled into an owned node.
    const int il = act ? i0 : 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        S raw[V];
        if constexpr (MODE == AA_LOCAL) {
            load_vec<S, V>(src + q * P + l0 + il, raw);
        } else {
            const int pq = (MODE == AA_PUSH) ? OPP[q] : q;
            if constexpr (OFF32) {
                static_assert(!kShifted && MODE == PULL, "the 32-bit form is the lane-shuffle pull form");
                load_vec<S, V>(at_off32(src + pq * P, (uint32_t)row_idx[q] * (uint32_t)a.lstride + (uint32_t)il),
                               raw);
            } else if constexpr (kShifted) {
                if (EXQ[q] == 1) load_vec_shifted<S, V>(src + pq * P + row_of[q] + (il - 1), raw);
                else if (EXQ[q] == -1) load_vec_shifted<S, V>(src + pq * P + row_of[q] + (il + 1), raw);
                else load_vec<S, V>(src + pq * P + row_of[q] + il, raw);
            } else {
                load_vec<S, V>(src + pq * P + row_of[q] + il, raw);
            }
        }
#pragma unroll
        for (int k = 0; k < V; ++k) v[q][k] = as_lv<LV>(raw[k]);
    }
    if (MOVING && bs.pose) {
#pragma unroll
        for (int k = 0; k < V; ++k) body[k] = (k < n_own) ? moving_body(a, bs.pose, bs.near, i0 + k, j) : 0;
    } else if (s1 > s0) {
        load_mask<V>(a.mask + r0 + il, body);
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) body[k] = 0;
    }

    // the end elements of the x-shifted directions (lane-shuffle form only)
    R left[3], right[3];
    if constexpr (!kShifted) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            left[m] = wave_shift_up1(dec(v[EXP[m]][V - 1]));
            right[m] = wave_shift_down1(dec(v[EXM[m]][0]));
        }
        // lanes that start a wavefront or a tile row load the end element
        // themselves: a plain load inside the domain, the side resolution only
        // where the column lies outside it
        if (act && (lane == 0 || lc == 0)) {
            if (i0 > 0) {
#pragma unroll
                for (int m = 0; m < 3; ++m) left[m] = dec(src[EXP[m] * P + row_of[EXP[m]] + (i0 - 1)]);
            } else {
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    left[m] = pull_column<MODE, S, R>(src, EXP[m], EXP[m], row_of[EXP[m]], row_idx[EXP[m]], -1, a);
            }
        }
        if (act && (lane == 63 || lc == tpr - 1)) {
            if (i0 + V < a.nx) {
#pragma unroll
                for (int m = 0; m < 3; ++m) right[m] = dec(src[EXM[m] * P + row_of[EXM[m]] + (i0 + V)]);
            } else {
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    right[m] = pull_column<MODE, S, R>(src, EXM[m], EXM[m], row_of[EXM[m]], row_idx[EXM[m]], i0 + V, a);
            }
        }
    } else {
        if (MODE != AA_LOCAL && act && i0 == 0) {  // the west side: column -1 is outside
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const int q = EXP[m];
                v[q][0] = pull_column<MODE, S, R>(src, q, MODE == AA_PUSH ? OPP[q] : q, row_of[q], row_idx[q], -1, a);
            }
        }
    }

    R fl_rho[V], fl_ux[V], fl_uy[V], fl_fx[V], fl_fy[V];
    double tile_drho = 0.0;
    S out[9][V];
    R prev[9];   // 2-byte storage: the even node's results, converted with the odd node's
#pragma unroll
    for (int k = 0; k < V; ++k) {
        R f[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q] = dec(v[q][k]);
        if constexpr (!kShifted) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                f[EXP[m]] = (k == 0) ? left[m] : dec(v[EXP[m]][k > 0 ? k - 1 : 0]);
                f[EXM[m]] = (k == V - 1) ? right[m] : dec(v[EXM[m]][k < V - 1 ? k + 1 : 0]);
            }
        }
        const int i = i0 + k;
        if (MODE != AA_LOCAL && i == a.nx - 1) {  // the east side: the neighbour column is outside
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const int q = EXM[m];
                f[q] = pull_column<MODE, S, R>(src, q, MODE == AA_PUSH ? OPP[q] : q, row_of[q], row_idx[q], a.nx, a);
            }
        }
        NodeResult<R> n;
        if constexpr (sizeof(S) == 2) {
            n = collide_node_lowp<R, MOVING>(f, body[k], i, j, a, bs);
            if constexpr (V >= 2) {
                // two nodes' populations at a time, one packed conversion each
                if (k & 1) {
#pragma unroll
                    for (int q = 0; q < 9; ++q) enc2<S>(prev[q], f[q], &out[q][k - 1]);
                } else {
#pragma unroll
                    for (int q = 0; q < 9; ++q) prev[q] = f[q];
                }
            } else {
                // the packed conversion here too: a scalar one may be fused with
                // the collision's last multiply-add into a single rounding to the
                // storage type, which rounds some values differently from the
                // two roundings (to FP32, then to storage) of the vector forms
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    S two[2];
                    enc2<S>(f[q], R(0), two);
                    out[q][k] = two[0];
                }
            }
        } else {
            n = collide_node<R, MOVING, true>(f, body[k], i, j, a, bs);
#pragma unroll
            for (int q = 0; q < 9; ++q) out[q][k] = enc<S>(f[q]);
        }
        fl_rho[k] = n.rho;
        fl_ux[k] = n.ux;
        fl_uy[k] = n.uy;
        fl_fx[k] = n.fvx;
        fl_fy[k] = n.fvy;
        if constexpr (RECORD) {
            // penalization force of every node to LDS (tiles holding solid nodes
            // only), summed per body after the stores
            if (s1 > s0) {
                R* fv = dyn_lds<R>();
                fv[k * a.block + (int)threadIdx.x] = n.fvx;
                fv[(V + k) * a.block + (int)threadIdx.x] = n.fvy;
            }
        }
        if (k < n_own) tile_drho += (double)n.drho;
    }

    // ---- stores
    if constexpr (MODE == PULL || MODE == AA_LOCAL) {
        // own node: plane q (pull) or plane opp(q) (AA local)
        if (n_own == V) {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                if constexpr (OFF32)
                    store_vec<S, V>(at_off32(dst + q * P, (uint32_t)j * (uint32_t)a.lstride + (uint32_t)i0), out[q]);
                else
                    store_vec<S, V>(dst + (MODE == PULL ? q : OPP[q]) * P + l0 + i0, out[q]);
            }
        } else if (n_own > 0) {  // ragged end of a row
#pragma unroll
            for (int k = 0; k < V; ++k)
                if (k < n_own)
#pragma unroll
                    for (int q = 0; q < 9; ++q) store_one<S>(dst + (MODE == PULL ? q : OPP[q]) * P + l0 + i0 + k, out[q][k]);
        }
        if constexpr (MODE == AA_LOCAL) {
            // the zero-gradient ghost columns that the next push step pulls from
            if (a.west == SIDE_OUTFLOW && act && i0 == 0)
#pragma unroll
                for (int m = 0; m < 3; ++m) static_cast<S*>(a.ghost_w)[m * (int64_t)a.ny + j] = out[EXP[m]][0];
            if (a.east == SIDE_OUTFLOW && act && i0 + n_own == a.nx)
#pragma unroll
                for (int k = 0; k < V; ++k)
                    if (k == n_own - 1)
#pragma unroll
                        for (int m = 0; m < 3; ++m)
                            static_cast<S*>(a.ghost_e)[m * (int64_t)a.ny + j] = out[EXM[m]][k];
        }
    } else {  // AA push: g_q(x) -> slot q of x + e_q
        const bool edge = (i0 == 0) || (i0 + V >= a.nx);
        if (act && !edge) {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                if (EXQ[q] == 0) {
                    store_vec<S, V>(dst + q * P + row_to[q] + i0, out[q]);
                } else if constexpr (sizeof(S) >= 4) {
                    if (EXQ[q] == 1) store_vec_shifted<S, V>(dst + q * P + row_to[q] + (i0 + 1), out[q]);
                    else store_vec_shifted<S, V>(dst + q * P + row_to[q] + (i0 - 1), out[q]);
                } else {
#pragma unroll
                    for (int k = 0; k < V; ++k) store_one<S>(dst + q * P + row_to[q] + i0 + k + EXQ[q], out[q][k]);
                }
            }
        } else if (act) {
            // node by node, with the domain sides resolved
#pragma unroll
            for (int k = 0; k < V; ++k) {
                if (k < n_own) {
                    const int i = i0 + k;
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        int c = i + EXQ[q];
                        bool keep = true;
                        if (c < 0) {
                            keep = (a.west == SIDE_PERIODIC);   // else it leaves the domain
                            c = a.nx - 1;
                        } else if (c >= a.nx) {
                            keep = (a.east == SIDE_PERIODIC);
                            c = 0;
                        }
                        if (keep) store_one<S>(dst + q * P + row_to[q] + c, out[q][k]);
                    }
                    // populations entering through a non-periodic side, for the next step
                    if (i == 0 && a.west != SIDE_PERIODIC) {
#pragma unroll
                        for (int m = 0; m < 3; ++m) {
                            const int q = EXP[m];
                            if (a.west == SIDE_INFLOW_EQ) store_one<S>(dst + q * P + l0, enc<S>(a.feq_in[q]));
                            else store_one<S>(dst + q * P + row_to[q], out[q][k]);
                        }
                    }
                    if (i == a.nx - 1 && a.east != SIDE_PERIODIC) {
#pragma unroll
                        for (int m = 0; m < 3; ++m) {
                            const int q = EXM[m];
                            if (a.east == SIDE_INFLOW_EQ) store_one<S>(dst + q * P + l0 + i, enc<S>(a.feq_in[q]));
                            else store_one<S>(dst + q * P + row_to[q] + i, out[q][k]);
                        }
                    }
                }
            }
        }
    }

    if constexpr (FIELDS) {
        R* fb = a.fields + r0 + i0;
        const int64_t F = a.plane_f;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (k < n_own) {
                fb[k] = fl_rho[k];
                fb[F + k] = fl_ux[k];
                fb[2 * F + k] = fl_uy[k];
                fb[3 * F + k] = fl_fx[k];
                fb[4 * F + k] = fl_fy[k];
            }
        }
    }

    if constexpr (RECORD) {
        // mass: one partial per wavefront (DPP moves only, no block barrier)
        double* mass_part = a.mass_part + part_buf * a.fin.mass_stride;
        double* slot_force = a.slot_force + part_buf * a.fin.slot_stride;
        const double wm = wave_sum_lane63(tile_drho);
        if (lane == 63) mass_part[(int64_t)t * (a.block >> 6) + (threadIdx.x >> 6)] = wm;
        // forces: only tiles that hold solid nodes (uniform across the block);
        // the body ids are read again (cache hit) rather than kept live
        int bid[V];
#pragma unroll
        for (int k = 0; k < V; ++k) bid[k] = 0;
        if (s1 > s0 && act) {
            if (MOVING && bs.pose) {
#pragma unroll
                for (int k = 0; k < V; ++k) bid[k] = (k < n_own) ? moving_body(a, bs.pose, bs.near, i0 + k, j) : 0;
            } else {
                load_mask<V>(a.mask + r0 + i0, bid);
            }
        }
        // each (tile, body) slot: every wavefront sums its lanes with DPP moves
        // into lane 63, which parks the sum in LDS; after one barrier per batch
        // of slots the block's first threads add the wavefronts in order
        const R* fv = dyn_lds<R>();
        const int nw = a.block >> 6, wid = (int)threadIdx.x >> 6;
        const int per_pass = FIN_LANES / nw;          // slots whose wave sums fit lds[2 FIN_LANES]
        for (int c0 = s0; c0 < s1; c0 += per_pass) {
            const int c1 = min(s1, c0 + per_pass);
            for (int s = c0; s < c1; ++s) {
                const int b = a.slot_body[s];
                // slots of moving bodies are dense (every tile, every body): a body
                // whose radius misses this tile adds zero, without the wave sums
                // (uniform across the block)
                const bool skip = MOVING && bs.pose && !((bs.near >> (b - 1)) & 1u);
                double wx = 0.0, wy = 0.0;
                if (!skip) {
                    double px = 0.0, py = 0.0;
#pragma unroll
                    for (int k = 0; k < V; ++k) {
                        if (k < n_own && bid[k] == b) {
                            px -= (double)fv[k * a.block + (int)threadIdx.x];
                            py -= (double)fv[(V + k) * a.block + (int)threadIdx.x];
                        }
                    }
                    wx = wave_sum_lane63(px);
                    wy = wave_sum_lane63(py);
                }
                if (lane == 63) {
                    lds[2 * ((s - c0) * nw + wid)] = wx;
                    lds[2 * ((s - c0) * nw + wid) + 1] = wy;
                }
            }
            __syncthreads();
            for (int s = c0 + (int)threadIdx.x; s < c1; s += a.block) {
                double x = 0.0, y = 0.0;
                for (int w = 0; w < nw; ++w) {
                    x += lds[2 * ((s - c0) * nw + w)];
                    y += lds[2 * ((s - c0) * nw + w) + 1];
                }
                slot_force[2 * s] = x;
                slot_force[2 * s + 1] = y;
            }
            __syncthreads();   // lds is reused by the next batch of slots
        }
    }
}

// Two lattices: source and destination never alias.
template <typename S, int V, bool RECORD, bool FIELDS, bool MOVING = false, bool OFF32 = false>
__global__ void __launch_bounds__(256)
k_step(const S* __restrict__ src, S* __restrict__ dst, StepArgs<typename Arith<S>::R> a)
{
    __shared__ double lds[2 * FIN_LANES];   // the record sums, then the per-wavefront sums
    // block 0 of the first 8 sums the previous step's record (no block waits on it)
    const int lead = a.fin_buf >= 0 ? N_XCD : 0;
    if ((int)blockIdx.x < lead) {
        if (blockIdx.x == 0) finalize_record(a.fin, a.fin_buf, lds);
        return;
    }
    const int t = xcd_tile(a.tiles_per_xcd, a.band_log2, lead);
    if (t >= a.n_tiles) return;  // whole block
    step_body<S, V, PULL, RECORD, FIELDS, MOVING, OFF32>(src, dst, a, t, a.part_buf, lds, a.pose_k);
}

// One lattice, read and written in place (no restrict).
template <typename S, int V, int MODE, bool RECORD, bool FIELDS, bool MOVING = false>
__global__ void __launch_bounds__(256) k_step_aa(S* lat, StepArgs<typename Arith<S>::R> a)
{
    __shared__ double lds[2 * FIN_LANES];
    const int lead = a.fin_buf >= 0 ? N_XCD : 0;
    if ((int)blockIdx.x < lead) {
        if (blockIdx.x == 0) finalize_record(a.fin, a.fin_buf, lds);
        return;
    }
    const int t = xcd_tile(a.tiles_per_xcd, a.band_log2, lead);
    if (t >= a.n_tiles) return;  // whole block
    step_body<S, V, MODE, RECORD, FIELDS, MOVING>(lat, lat, a, t, a.part_buf, lds, a.pose_k);
}

// Many domains in one launch: block -> (domain, tile) through the tile map;
// every domain's arguments (geometry, parameters, lattices) live in device
// memory. All domains take the same step kind, record flag and partial buffers.
template <typename S, int V, int MODE, bool RECORD, bool FIELDS, bool MOVING = false, bool OFF32 = false>
__global__ void __launch_bounds__(256) k_step_batch(BatchLaunch b)
{
    using R = typename Arith<S>::R;
    __shared__ double lds[2 * FIN_LANES];
    const StepArgs<R>* args = static_cast<const StepArgs<R>*>(b.args);
    // the first n_fin blocks sum the previous step's record of one domain each:
    // dispatched first and spread over the XCDs, they overlap the streaming
    // tiles instead of trailing them (n_fin is a multiple of 8)
    if ((int)blockIdx.x < b.n_fin) {
        if ((int)blockIdx.x < b.n_domains) finalize_record(args[blockIdx.x].fin, b.fin_buf, lds);
        return;
    }
    const int g = xcd_tile(b.tiles_per_xcd, b.band_log2, b.n_fin);
    if (g >= b.total_tiles) return;  // whole block
#if defined(__HIP_DEVICE_COMPILE__)
    // the tile map and the members' arguments do not change during a launch:
    // read through the constant address space they are scalar loads that no
    // store of the step can alias, and the arguments are copied once, up front
    // (through a generic reference every later use reloaded them)
    using CI = const __attribute__((address_space(4))) int32_t;
    using CA = const __attribute__((address_space(4))) StepArgs<R>;
    const int d = ((CI*)b.tile_domain)[g];
    const StepArgs<R> a = ((CA*)args)[d];
    const int t = g - ((CI*)b.tile_start)[d];
#else
    const int d = b.tile_domain[g];
    const StepArgs<R>& a = args[d];
    const int t = g - b.tile_start[d];
#endif
    const int cur = a.cur ^ b.flip;
    S* lat_cur = static_cast<S*>(cur ? a.lat1 : a.lat0);
    S* lat_next = static_cast<S*>(cur ? a.lat0 : a.lat1);
    step_body<S, V, MODE, RECORD, FIELDS, MOVING, OFF32>(lat_cur, MODE == PULL ? lat_next : lat_cur, a, t, b.part_buf,
                                                         lds, b.pose_k);
}

// The last record of an lbvp_step call, summed on its own.
__global__ void __launch_bounds__(FIN_THREADS) k_finalize(FinalizeArgs a, int32_t buf)
{
    __shared__ double lds[2 * FIN_LANES];
    finalize_record(a, buf, lds);
}

// The same for every domain of a batch, one block each.
__global__ void __launch_bounds__(FIN_THREADS) k_finalize_batch(const FinalizeArgs* fins, int32_t buf)
{
    __shared__ double lds[2 * FIN_LANES];
    finalize_record(fins[blockIdx.x], buf, lds);
}

// Moving bodies: after a run of n steps, the pose table row of the next step.
__global__ void k_pose_advance(int64_t* base, int64_t n) { *base += n; }

template <typename R>
__global__ void __launch_bounds__(256) k_pose_advance_batch(const StepArgs<R>* args, int32_t n_domains, int64_t n)
{
    const int d = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (d < n_domains && args[d].n_moving > 0) *const_cast<int64_t*>(args[d].pose_base) += n;
}

// ------------------------------------------------------------ conversions --
__constant__ double W_ALL[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
__constant__ int EX_ALL[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int EY_ALL[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__constant__ int OPP_ALL[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Algorithm step (1): populations at equilibrium (eq. feq) for staged rows, in
// FP64, stored as normalized deviations; the fields of step 0 are (rho, u, 0, 0).
// In the AA layout the post-collision population q of a node lives in its slot
// opp(q) after an even number of steps (a.swap).
template <typename S>
__global__ void __launch_bounds__(256) k_init(S* lat, typename Arith<S>::R* fields, ConvArgs a)
{
    using R = typename Arith<S>::R;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)a.rows * a.nx) return;
    const int jl = (int)(k / a.nx), i = (int)(k - (int64_t)jl * a.nx);
    const double rho = a.rho ? a.rho[k] : a.rho0;
    const double ux = a.ux ? a.ux[k] : 0.0;
    const double uy = a.uy ? a.uy[k] : 0.0;
    const double uu = ux * ux + uy * uy;
    const int64_t o = (int64_t)(a.row0 + jl) * a.pitch + i;
    const int64_t lo = (int64_t)(a.row0 + jl) * a.lstride + i;
    for (int q = 0; q < 9; ++q) {
        const double eu = EX_ALL[q] * ux + EY_ALL[q] * uy;
        const double h = (rho - a.rho0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        lat[(a.swap ? OPP_ALL[q] : q) * a.plane + lo] = enc<S>((R)h);
    }
    if (fields) {
        fields[o] = (R)rho;
        fields[a.plane_f + o] = (R)ux;
        fields[2 * a.plane_f + o] = (R)uy;
        fields[3 * a.plane_f + o] = R(0);
        fields[4 * a.plane_f + o] = R(0);
    }
}

template <typename S>
__global__ void __launch_bounds__(256) k_decode(const S* lat, ConvArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)a.rows * a.nx;
    if (k >= n) return;
    const int jl = (int)(k / a.nx), i = (int)(k - (int64_t)jl * a.nx);
    const int64_t lo = (int64_t)(a.row0 + jl) * a.lstride + i;
    for (int q = 0; q < 9; ++q)
        a.pops[q * n + k] = W_ALL[q] * ((double)dec(lat[(a.swap ? OPP_ALL[q] : q) * a.plane + lo]) + a.rho0);
}

template <typename S>
__global__ void __launch_bounds__(256) k_encode(S* lat, ConvArgs a)
{
    using R = typename Arith<S>::R;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)a.rows * a.nx;
    if (k >= n) return;
    const int jl = (int)(k / a.nx), i = (int)(k - (int64_t)jl * a.nx);
    const int64_t lo = (int64_t)(a.row0 + jl) * a.lstride + i;
    for (int q = 0; q < 9; ++q)
        lat[(a.swap ? OPP_ALL[q] : q) * a.plane + lo] = enc<S>((R)(a.pops[q * n + k] / W_ALL[q] - a.rho0));
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

// A plain device copy: one 16-byte non-temporal load and store per thread in
// 64-thread blocks, the fastest of the copy forms measured (6.6-6.7 TB/s against
// 6.1 for four elements per thread in 256-thread blocks, XCD-ordered or not):
// the bandwidth the memory system gives a streaming read-and-write, against
// which the steps are measured.
__global__ void __launch_bounds__(64) k_copy16(const u32x4_t* __restrict__ src, u32x4_t* __restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// AA layout after an even number of steps: copy the outflow sides' outgoing
// post-collision populations into the ghost columns the next push step reads.
template <typename S>
__global__ void __launch_bounds__(256) k_aa_ghosts(const S* lat, GhostArgs a)
{
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= a.ny) return;
    const int64_t row = (int64_t)y * a.lstride;
    const int exp_q[3] = {1, 5, 8}, exm_q[3] = {3, 6, 7};
    for (int m = 0; m < 3; ++m) {
        if (a.west_outflow)
            static_cast<S*>(a.ghost_w)[m * (int64_t)a.ny + y] = lat[OPP_ALL[exp_q[m]] * a.plane + row];
        if (a.east_outflow)
            static_cast<S*>(a.ghost_e)[m * (int64_t)a.ny + y] = lat[OPP_ALL[exm_q[m]] * a.plane + row + a.nx - 1];
    }
}

// The halo columns of every cut of a slab decomposition (one thread per row and
// direction of each link): plain copies of the storage values, so that a
// decomposed domain steps bitwise like the whole one.
template <typename S>
__global__ void __launch_bounds__(256) k_halo(HaloArgs h)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_link = 3 * (int64_t)h.ny;
    if (k >= per_link * h.n_links) return;
    const int l = (int)(k / per_link);
    const int r = (int)(k - (int64_t)l * per_link);
    const int m = r / h.ny, j = r - m * h.ny;
    const HaloLink& L = h.link[l];
    const int q_in = m == 0 ? 1 : (m == 1 ? 5 : 8);    // e_x = +1 (1, 5, 8): leave west through its east side
    const int q_out = m == 0 ? 3 : (m == 1 ? 6 : 7);   // e_x = -1 (3, 6, 7): leave east through its west side
    const S* wl = static_cast<const S*>(L.w_lat);
    const S* el = static_cast<const S*>(L.e_lat);
    // east slab's west halo: its last padding column; west slab's east halo: column nx
    static_cast<S*>(L.e_lat_w)[j * L.e_lstride + q_in * L.e_plane + (L.e_pitch - 1)] =
        wl[j * L.w_lstride + q_in * L.w_plane + (L.w_nx - 1)];
    static_cast<S*>(L.w_lat_w)[j * L.w_lstride + q_out * L.w_plane + L.w_nx] = el[j * L.e_lstride + q_out * L.e_plane];
}

// The same for the cuts of a batch, before one of its steps: each member's
// current lattice is read from its step arguments (so a captured graph replays
// correctly whatever the members' lattice parity when it is launched).
template <typename S>
__global__ void __launch_bounds__(256) k_halo_batch(BatchHalo h)
{
    using R = typename Arith<S>::R;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_link = 3 * (int64_t)h.ny;
    if (k >= per_link * h.n_links) return;
    const int l = (int)(k / per_link);
    const int r = (int)(k - (int64_t)l * per_link);
    const int m = r / h.ny, j = r - m * h.ny;
    const StepArgs<R>* args = static_cast<const StepArgs<R>*>(h.args);
    const StepArgs<R>& aw = args[h.w[l]];
    const StepArgs<R>& ae = args[h.e[l]];
    S* wl = static_cast<S*>((aw.cur ^ h.flip) ? aw.lat1 : aw.lat0);
    S* el = static_cast<S*>((ae.cur ^ h.flip) ? ae.lat1 : ae.lat0);
    const int q_in = m == 0 ? 1 : (m == 1 ? 5 : 8);
    const int q_out = m == 0 ? 3 : (m == 1 ? 6 : 7);
    el[j * ae.lstride + q_in * ae.plane + (ae.pitch - 1)] = wl[j * aw.lstride + q_in * aw.plane + (aw.nx - 1)];
    wl[j * aw.lstride + q_out * aw.plane + aw.nx] = el[j * ae.lstride + q_out * ae.plane];
}

template <typename R>
size_t record_lds_bytes(int v, int block)
{
    return 2 * (size_t)v * (size_t)block * sizeof(R);
}

template <typename S, int V, bool MOVING = false>
hipError_t step_v(int mode, bool record, bool fields, const S* in, S* out, const StepArgs<typename Arith<S>::R>& a,
                  hipStream_t s)
{
    const dim3 grid((unsigned)(a.tiles_per_xcd * N_XCD + (a.fin_buf >= 0 ? N_XCD : 0))), block((unsigned)a.block);
    const size_t lds = record_lds_bytes<typename Arith<S>::R>(V, a.block);
    if (mode == PULL) {
        if constexpr (sizeof(S) == 2 && V > 1) {
            if (a.off32) {
                if (record) {
                    if (fields) hipLaunchKernelGGL((k_step<S, V, true, true, MOVING, true>), grid, block, lds, s, in, out, a);
                    else hipLaunchKernelGGL((k_step<S, V, true, false, MOVING, true>), grid, block, lds, s, in, out, a);
                } else {
                    if (fields) hipLaunchKernelGGL((k_step<S, V, false, true, MOVING, true>), grid, block, 0, s, in, out, a);
                    else hipLaunchKernelGGL((k_step<S, V, false, false, MOVING, true>), grid, block, 0, s, in, out, a);
                }
                return hipGetLastError();
            }
        }
        if (record) {
            if (fields) hipLaunchKernelGGL((k_step<S, V, true, true, MOVING>), grid, block, lds, s, in, out, a);
            else hipLaunchKernelGGL((k_step<S, V, true, false, MOVING>), grid, block, lds, s, in, out, a);
        } else {
            if (fields) hipLaunchKernelGGL((k_step<S, V, false, true, MOVING>), grid, block, 0, s, in, out, a);
            else hipLaunchKernelGGL((k_step<S, V, false, false, MOVING>), grid, block, 0, s, in, out, a);
        }
        return hipGetLastError();
    }
    if constexpr (sizeof(S) >= 4 || V == 1) {
        if (mode == AA_PUSH) {
            if (record) {
                if (fields) hipLaunchKernelGGL((k_step_aa<S, V, AA_PUSH, true, true, MOVING>), grid, block, lds, s, out, a);
                else hipLaunchKernelGGL((k_step_aa<S, V, AA_PUSH, true, false, MOVING>), grid, block, lds, s, out, a);
            } else {
                if (fields) hipLaunchKernelGGL((k_step_aa<S, V, AA_PUSH, false, true, MOVING>), grid, block, 0, s, out, a);
                else hipLaunchKernelGGL((k_step_aa<S, V, AA_PUSH, false, false, MOVING>), grid, block, 0, s, out, a);
            }
        } else {
            if (record) {
                if (fields) hipLaunchKernelGGL((k_step_aa<S, V, AA_LOCAL, true, true, MOVING>), grid, block, lds, s, out, a);
                else hipLaunchKernelGGL((k_step_aa<S, V, AA_LOCAL, true, false, MOVING>), grid, block, lds, s, out, a);
            } else {
                if (fields) hipLaunchKernelGGL((k_step_aa<S, V, AA_LOCAL, false, true, MOVING>), grid, block, 0, s, out, a);
                else hipLaunchKernelGGL((k_step_aa<S, V, AA_LOCAL, false, false, MOVING>), grid, block, 0, s, out, a);
            }
        }
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;  // AA with sub-dword vectors: not built (one node per thread is)
    }
}

template <typename S>
hipError_t step_typed(int mode, bool record, bool fields, const void* src, void* dst, const void* args_v,
                      hipStream_t s)
{
    using R = typename Arith<S>::R;
    const StepArgs<R>& a = *static_cast<const StepArgs<R>*>(args_v);
    const S* in = static_cast<const S*>(src);
    S* out = static_cast<S*>(dst);
    constexpr int VW = 16 / (int)sizeof(S);
    if (a.vec == VW) return step_v<S, VW>(mode, record, fields, in, out, a, s);
    if (a.vec == 1) return step_v<S, 1>(mode, record, fields, in, out, a, s);
    if constexpr (sizeof(S) == 2) {   // 2-byte types also run 4 nodes (8 bytes) per thread
        if (a.vec == 4) return step_v<S, 4>(mode, record, fields, in, out, a, s);
    }
    return hipErrorInvalidValue;
}

template <typename S>
hipError_t step_typed_moving(int mode, bool record, bool fields, const void* src, void* dst, const void* args_v,
                             hipStream_t s)
{
    using R = typename Arith<S>::R;
    const StepArgs<R>& a = *static_cast<const StepArgs<R>*>(args_v);
    const S* in = static_cast<const S*>(src);
    S* out = static_cast<S*>(dst);
    constexpr int VW = 16 / (int)sizeof(S);
    if (a.vec == VW) return step_v<S, VW, true>(mode, record, fields, in, out, a, s);
    if (a.vec == 1) return step_v<S, 1, true>(mode, record, fields, in, out, a, s);
    if constexpr (sizeof(S) == 2) {
        if (a.vec == 4) return step_v<S, 4, true>(mode, record, fields, in, out, a, s);
    }
    return hipErrorInvalidValue;
}

template <typename S, int V, int MODE, bool MOVING>
hipError_t batch_mode(bool record, bool fields, const BatchLaunch& b, int32_t block, hipStream_t s)
{
    const dim3 grid((unsigned)(b.tiles_per_xcd * N_XCD + b.n_fin)), blk((unsigned)block);
    const size_t lds = record_lds_bytes<typename Arith<S>::R>(V, block);
    if constexpr (sizeof(S) == 2 && V > 1 && MODE == PULL) {
        if (b.off32) {
            if (record) {
                if (fields) hipLaunchKernelGGL((k_step_batch<S, V, MODE, true, true, MOVING, true>), grid, blk, lds, s, b);
                else hipLaunchKernelGGL((k_step_batch<S, V, MODE, true, false, MOVING, true>), grid, blk, lds, s, b);
            } else {
                if (fields) hipLaunchKernelGGL((k_step_batch<S, V, MODE, false, true, MOVING, true>), grid, blk, 0, s, b);
                else hipLaunchKernelGGL((k_step_batch<S, V, MODE, false, false, MOVING, true>), grid, blk, 0, s, b);
            }
            return hipGetLastError();
        }
    }
    if (record) {
        if (fields) hipLaunchKernelGGL((k_step_batch<S, V, MODE, true, true, MOVING>), grid, blk, lds, s, b);
        else hipLaunchKernelGGL((k_step_batch<S, V, MODE, true, false, MOVING>), grid, blk, lds, s, b);
    } else {
        if (fields) hipLaunchKernelGGL((k_step_batch<S, V, MODE, false, true, MOVING>), grid, blk, 0, s, b);
        else hipLaunchKernelGGL((k_step_batch<S, V, MODE, false, false, MOVING>), grid, blk, 0, s, b);
    }
    return hipGetLastError();
}

template <typename S, int V, bool MOVING>
hipError_t batch_v(int32_t mode, bool record, bool fields, const BatchLaunch& b, int32_t block, hipStream_t s)
{
    if (mode == PULL) return batch_mode<S, V, PULL, MOVING>(record, fields, b, block, s);
    if constexpr (sizeof(S) >= 4 || V == 1) {
        if (mode == AA_PUSH) return batch_mode<S, V, AA_PUSH, MOVING>(record, fields, b, block, s);
        return batch_mode<S, V, AA_LOCAL, MOVING>(record, fields, b, block, s);
    } else {
        return hipErrorInvalidValue;
    }
}

// moving: some member has moving bodies (every member then runs the kernel
// that evaluates a moving mask where a domain has one)
template <typename S, bool MOVING>
hipError_t batch_typed(int32_t vec, int32_t mode, bool record, bool fields, const BatchLaunch& b, int32_t block,
                       hipStream_t s)
{
    constexpr int VW = 16 / (int)sizeof(S);
    if (vec == VW) return batch_v<S, VW, MOVING>(mode, record, fields, b, block, s);
    if (vec == 1) return batch_v<S, 1, MOVING>(mode, record, fields, b, block, s);
    if constexpr (sizeof(S) == 2) {
        if (vec == 4) return batch_v<S, 4, MOVING>(mode, record, fields, b, block, s);
    }
    return hipErrorInvalidValue;
}

unsigned conv_blocks(const ConvArgs& a) { return (unsigned)(((int64_t)a.rows * a.nx + 255) / 256); }

}  // namespace

int vector_width(int32_t storage)
{
    switch (storage) {
    case ST_F64: return 2;
    case ST_F32: return 4;
    default: return 8;
    }
}

hipError_t launch_step(int32_t storage, int32_t mode, bool record, bool fields, const void* src, void* dst,
                       const void* step_args, hipStream_t s)
{
    switch (storage) {
    case ST_F64: return step_typed<double>(mode, record, fields, src, dst, step_args, s);
    case ST_F32: return step_typed<float>(mode, record, fields, src, dst, step_args, s);
    case ST_F16: return step_typed<_Float16>(mode, record, fields, src, dst, step_args, s);
    case ST_BF16: return step_typed<__bf16>(mode, record, fields, src, dst, step_args, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_moving(int32_t storage, int32_t mode, bool record, bool fields, const void* src, void* dst,
                              const void* step_args, hipStream_t s)
{
    switch (storage) {
    case ST_F64: return step_typed_moving<double>(mode, record, fields, src, dst, step_args, s);
    case ST_F32: return step_typed_moving<float>(mode, record, fields, src, dst, step_args, s);
    case ST_F16: return step_typed_moving<_Float16>(mode, record, fields, src, dst, step_args, s);
    case ST_BF16: return step_typed_moving<__bf16>(mode, record, fields, src, dst, step_args, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_batch(int32_t storage, int32_t vec, int32_t block, int32_t mode, bool record, bool fields,
                             bool moving, const BatchLaunch& b, hipStream_t s)
{
    if (moving) {
        switch (storage) {
        case ST_F64: return batch_typed<double, true>(vec, mode, record, fields, b, block, s);
        case ST_F32: return batch_typed<float, true>(vec, mode, record, fields, b, block, s);
        case ST_F16: return batch_typed<_Float16, true>(vec, mode, record, fields, b, block, s);
        case ST_BF16: return batch_typed<__bf16, true>(vec, mode, record, fields, b, block, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (storage) {
    case ST_F64: return batch_typed<double, false>(vec, mode, record, fields, b, block, s);
    case ST_F32: return batch_typed<float, false>(vec, mode, record, fields, b, block, s);
    case ST_F16: return batch_typed<_Float16, false>(vec, mode, record, fields, b, block, s);
    case ST_BF16: return batch_typed<__bf16, false>(vec, mode, record, fields, b, block, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pose_advance(int64_t* base, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_pose_advance, dim3(1), dim3(1), 0, s, base, n);
    return hipGetLastError();
}

hipError_t launch_pose_advance_batch(int32_t storage, const void* args, int32_t n_domains, int64_t n, hipStream_t s)
{
    const dim3 g((unsigned)((n_domains + 255) / 256)), b(256);
    if (storage == ST_F64)
        hipLaunchKernelGGL(k_pose_advance_batch<double>, g, b, 0, s, static_cast<const StepArgs<double>*>(args),
                           n_domains, n);
    else
        hipLaunchKernelGGL(k_pose_advance_batch<float>, g, b, 0, s, static_cast<const StepArgs<float>*>(args),
                           n_domains, n);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const FinalizeArgs* fin_dev, int32_t n, int32_t buf, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_batch, dim3((unsigned)n), dim3(FIN_THREADS), 0, s, fin_dev, buf);
    return hipGetLastError();
}

hipError_t launch_aa_ghosts(int32_t storage, const void* lat, const GhostArgs& a, hipStream_t s)
{
    const dim3 g((unsigned)((a.ny + 255) / 256)), b(256);
    switch (storage) {
    case ST_F64: hipLaunchKernelGGL(k_aa_ghosts<double>, g, b, 0, s, (const double*)lat, a); break;
    case ST_F32: hipLaunchKernelGGL(k_aa_ghosts<float>, g, b, 0, s, (const float*)lat, a); break;
    case ST_F16: hipLaunchKernelGGL(k_aa_ghosts<_Float16>, g, b, 0, s, (const _Float16*)lat, a); break;
    case ST_BF16: hipLaunchKernelGGL(k_aa_ghosts<__bf16>, g, b, 0, s, (const __bf16*)lat, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, int32_t buf, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, s, a, buf);
    return hipGetLastError();
}

hipError_t launch_init(int32_t storage, void* lat, void* fields, const ConvArgs& a, hipStream_t s)
{
    const dim3 g(conv_blocks(a)), b(256);
    switch (storage) {
    case ST_F64: hipLaunchKernelGGL(k_init<double>, g, b, 0, s, (double*)lat, (double*)fields, a); break;
    case ST_F32: hipLaunchKernelGGL(k_init<float>, g, b, 0, s, (float*)lat, (float*)fields, a); break;
    case ST_F16: hipLaunchKernelGGL(k_init<_Float16>, g, b, 0, s, (_Float16*)lat, (float*)fields, a); break;
    case ST_BF16: hipLaunchKernelGGL(k_init<__bf16>, g, b, 0, s, (__bf16*)lat, (float*)fields, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_decode(int32_t storage, const void* lat, const ConvArgs& a, hipStream_t s)
{
    const dim3 g(conv_blocks(a)), b(256);
    switch (storage) {
    case ST_F64: hipLaunchKernelGGL(k_decode<double>, g, b, 0, s, (const double*)lat, a); break;
    case ST_F32: hipLaunchKernelGGL(k_decode<float>, g, b, 0, s, (const float*)lat, a); break;
    case ST_F16: hipLaunchKernelGGL(k_decode<_Float16>, g, b, 0, s, (const _Float16*)lat, a); break;
    case ST_BF16: hipLaunchKernelGGL(k_decode<__bf16>, g, b, 0, s, (const __bf16*)lat, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_encode(int32_t storage, void* lat, const ConvArgs& a, hipStream_t s)
{
    const dim3 g(conv_blocks(a)), b(256);
    switch (storage) {
    case ST_F64: hipLaunchKernelGGL(k_encode<double>, g, b, 0, s, (double*)lat, a); break;
    case ST_F32: hipLaunchKernelGGL(k_encode<float>, g, b, 0, s, (float*)lat, a); break;
    case ST_F16: hipLaunchKernelGGL(k_encode<_Float16>, g, b, 0, s, (_Float16*)lat, a); break;
    case ST_BF16: hipLaunchKernelGGL(k_encode<__bf16>, g, b, 0, s, (__bf16*)lat, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s)
{
    const int64_t blocks = (n16 + 63) / 64;
    if (blocks > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(64), 0, s, static_cast<const u32x4_t*>(src),
                       static_cast<u32x4_t*>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_halo(int32_t storage, const HaloArgs& h, hipStream_t s)
{
    const int64_t n = 3 * (int64_t)h.ny * h.n_links;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    switch (storage) {
    case ST_F64: hipLaunchKernelGGL(k_halo<double>, g, b, 0, s, h); break;
    case ST_F32: hipLaunchKernelGGL(k_halo<float>, g, b, 0, s, h); break;
    case ST_F16: hipLaunchKernelGGL(k_halo<_Float16>, g, b, 0, s, h); break;
    case ST_BF16: hipLaunchKernelGGL(k_halo<__bf16>, g, b, 0, s, h); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_halo_batch(int32_t storage, const BatchHalo& h, hipStream_t s)
{
    const int64_t n = 3 * (int64_t)h.ny * h.n_links;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    switch (storage) {
    case ST_F64: hipLaunchKernelGGL(k_halo_batch<double>, g, b, 0, s, h); break;
    case ST_F32: hipLaunchKernelGGL(k_halo_batch<float>, g, b, 0, s, h); break;
    case ST_F16: hipLaunchKernelGGL(k_halo_batch<_Float16>, g, b, 0, s, h); break;
    case ST_BF16: hipLaunchKernelGGL(k_halo_batch<__bf16>, g, b, 0, s, h); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace lbvp
