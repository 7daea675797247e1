// lbvp3_kernels.hip -- gfx950 kernels of the fused D3Q19 TRT-VP time step.
//
// The 3-D extension of the scheme (the paper states it on D2Q9, Sec. 2.2, and
// names 3-D as its next step, Sec. 4). Layout in HBM: lattice rows of
// structures of arrays, population a of node (i, j, k) at
//   lattice[r * lstride + a * pitch + i],  r = k * ny + j,  lstride = 19 pitch,
// so that the 19 population rows of one lattice row lie back to back and a
// tile's loads and stores stay within a few neighbouring rows of memory. pitch
// is a multiple of 64 elements. Every storage type holds the weight-normalized
// deviation h_a = (f_a - w_a rho0) / w_a; the moments use the integers
// 36 w_a = 12 (rest), 2 (faces), 1 (edges):
//   36 drho = 12 h_0 + 2 sum_faces h + sum_edges h,   36 j = sum e_a (36 w_a) h_a,
// and in these units the equilibrium is h^eq_a = drho + rho (3 eu + 9/2 eu^2 - 3/2 u.u)
// and the Guo term F_a / w_a = 3 (e_a - u).F + 9 (e_a.u)(e_a.F) (eqs. feq,
// external-force-term with the D3Q19 weights; c_s^2 = 1/3). The odd part of the
// equilibrium, 3 rho e.u, is formed as e.(36 j + 18 F)/12 from the momentum.
//
// One step per node, fused (Sec. 2.2, steps (2)-(6)):
//   pull     f_a(x) = g_a(x - e_a)                                   eq. (streaming)
//   rho = rho0 + sum w_a h_a,  u* = (j + F_b/2) / rho                eqs. (rho), (rho*velocity-star)
//   du = chi (U_O - u*) / (2 eta + chi),  F_VP = 2 rho du            eqs. (d-V), (force-density)
//   u = u* + du,  F = F_b + F_VP                                     eq. (velocity-r)
//   TRT collision of the nine (a, opposite a) pairs and the rest population with
//   the even/odd split of f^eq and of the Guo term          eqs. (TRT-collision), (collision-modified)
// with U_O = v + omega x (x - c) of the node's body.
//
// The step is bound by HBM traffic: 19 loads, 19 stores and a mask byte per node
// against ~350 flops. Each thread owns V consecutive nodes of a row and moves
// each population with one V-wide access; the directions with an x component
// load V elements one element off alignment (a single dword-aligned vector
// load), or, for 2-byte vectors, aligned with the end element from a lane shuffle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lbvp3_internal.h"
#include "lbvp_device.h"

namespace lbvp3 {
namespace {

using lbvp::Arith;
using lbvp::as_lv;
using lbvp::block_sum;
using lbvp::collide_pair;
using lbvp::dec;
using lbvp::div36;
using lbvp::enc;
using lbvp::FIN_LANES;
using lbvp::lane_sum;
using lbvp::load_mask;
using lbvp::load_vec;
using lbvp::load_vec_shifted;
using lbvp::momentum3;
using lbvp::NodeTerms;
using lbvp::Pair;
using lbvp::recip;
using lbvp::store_one;
using lbvp::store_vec;
using lbvp::tree_sum;
using lbvp::wave_sum_lane63;
using lbvp::xcd_tile;

template <typename R>
struct Node3 {
    R drho, rho, u[3], fv[3];
};

// Steps (4)-(6) at node (i, j, k) with streamed populations f (weight-normalized);
// overwrites f with the post-collision populations.
// EXACT_MOM as in the 2-D step: the 2-byte storage types take 3 rho u as (3 rho) u.
template <typename R, bool EXACT_MOM = true>
__device__ __forceinline__ Node3<R> collide3(R (&f)[Q], int body, int i, int j, int k, const Step3Args<R>& a)
{
    const R faces = ((f[1] + f[2]) + (f[3] + f[4])) + (f[5] + f[6]);
    const R edges = (((f[7] + f[8]) + (f[9] + f[10])) + ((f[11] + f[12]) + (f[13] + f[14]))) +
                    ((f[15] + f[16]) + (f[17] + f[18]));
    const R drho = div36(R(12) * f[0] + (R(2) * faces + edges));
    const R rho = a.rho0 + drho;
    const R inv_36rho = recip(R(36) * rho);
    const R d78 = f[7] - f[8], d910 = f[9] - f[10], d1112 = f[11] - f[12], d1314 = f[13] - f[14];
    const R d1516 = f[15] - f[16], d1718 = f[17] - f[18];
    // 36 j from the odd parts of the pairs, plus 18 F_b (eq. rho*velocity-star)
    R j36[3], u[3];
    j36[0] = R(2) * (f[1] - f[2]) + ((d78 + d910) + (d1112 + d1314)) + a.fb18[0];
    j36[1] = R(2) * (f[3] - f[4]) + ((d78 - d910) + (d1516 + d1718)) + a.fb18[1];
    j36[2] = R(2) * (f[5] - f[6]) + ((d1112 - d1314) + (d1516 - d1718)) + a.fb18[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = j36[d] * inv_36rho;

    R fv[3] = {R(0), R(0), R(0)};
    if (body) {
        const R* B = a.bodies + BODY3_STRIDE * body;
        // x - c from the split centre (a centre rounded to FP32 whole would be off
        // by up to half an FP32 spacing, the same for every node of the body)
        const R rx = ((R)i - B[0]) - B[3], ry = ((R)j - B[1]) - B[4], rz = ((R)k - B[2]) - B[5];
        R uo[3];
        uo[0] = B[6] + (B[10] * rz - B[11] * ry);
        uo[1] = B[7] + (B[11] * rx - B[9] * rz);
        uo[2] = B[8] + (B[9] * ry - B[10] * rx);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const R du = a.vp_c * (uo[d] - u[d]);
            fv[d] = R(2) * rho * du;
            u[d] += du;
        }
    }
    R F[3], P[3];   // total force; 3 rho u formed from the momentum
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        F[d] = a.fb[d] + fv[d];
        if constexpr (EXACT_MOM) P[d] = momentum3(j36[d], fv[d]);
        else P[d] = (R(3) * rho) * u[d];
    }

    NodeTerms<R> n;
    const R uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    n.A = drho - (R(1.5) * rho) * uu;
    n.rho45 = R(4.5) * rho;
    n.uF3 = R(-3) * ((u[0] * F[0] + u[1] * F[1]) + u[2] * F[2]);
    const R g0 = a.om_p * (n.A - f[0]) + f[0] + a.k_p * n.uF3;
    // pair (a, a + 1) for odd a: e_a.u and e_a.F
    const Pair<R> p1 = collide_pair(f[1], f[2], u[0], P[0], F[0], n, a);
    const Pair<R> p3 = collide_pair(f[3], f[4], u[1], P[1], F[1], n, a);
    const Pair<R> p5 = collide_pair(f[5], f[6], u[2], P[2], F[2], n, a);
    const Pair<R> p7 = collide_pair(f[7], f[8], u[0] + u[1], P[0] + P[1], F[0] + F[1], n, a);
    const Pair<R> p9 = collide_pair(f[9], f[10], u[0] - u[1], P[0] - P[1], F[0] - F[1], n, a);
    const Pair<R> p11 = collide_pair(f[11], f[12], u[0] + u[2], P[0] + P[2], F[0] + F[2], n, a);
    const Pair<R> p13 = collide_pair(f[13], f[14], u[0] - u[2], P[0] - P[2], F[0] - F[2], n, a);
    const Pair<R> p15 = collide_pair(f[15], f[16], u[1] + u[2], P[1] + P[2], F[1] + F[2], n, a);
    const Pair<R> p17 = collide_pair(f[17], f[18], u[1] - u[2], P[1] - P[2], F[1] - F[2], n, a);
    f[0] = g0;
    f[1] = p1.ga;
    f[2] = p1.gb;
    f[3] = p3.ga;
    f[4] = p3.gb;
    f[5] = p5.ga;
    f[6] = p5.gb;
    f[7] = p7.ga;
    f[8] = p7.gb;
    f[9] = p9.ga;
    f[10] = p9.gb;
    f[11] = p11.ga;
    f[12] = p11.gb;
    f[13] = p13.ga;
    f[14] = p13.gb;
    f[15] = p15.ga;
    f[16] = p15.gb;
    f[17] = p17.ga;
    f[18] = p17.gb;
    Node3<R> out;
    out.drho = drho;
    out.rho = rho;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        out.u[d] = u[d];
        out.fv[d] = fv[d];
    }
    return out;
}

// Population q pulled from column c of the lattice row at row_off, with the x
// sides resolved (c = -1 or nx lies outside the domain). Inflow populations are
// rounded to the storage type like every stored population.
template <typename S, typename R>
__device__ __forceinline__ R pull_col(const S* src, int q, int64_t row_off, int c, const Step3Args<R>& a)
{
    if (c < 0) {
        if (a.west == LBVP_BC_INFLOW_EQ) return dec(enc<S>(a.feq_in[q]));
        c = (a.west == LBVP_BC_PERIODIC) ? a.nx - 1 : 0;
    } else if (c >= a.nx) {
        if (a.east == LBVP_BC_INFLOW_EQ) return dec(enc<S>(a.feq_in[q]));
        c = (a.east == LBVP_BC_PERIODIC) ? 0 : a.nx - 1;
    }
    return dec(src[row_off + (int64_t)q * a.pitch + c]);
}

template <typename R>
__device__ __forceinline__ R* force_lds()
{
    extern __shared__ __align__(16) unsigned char lds3_dyn[];
    return reinterpret_cast<R*>(lds3_dyn);
}

// Tile t: tile_rows lattice rows of tile_w nodes, V consecutive nodes per thread.
template <typename S, int V, bool RECORD, bool FIELDS>
__device__ __forceinline__ void step3_body(const S* __restrict__ src, S* __restrict__ dst,
                                           const Step3Args<typename Arith<S>::R>& a, int t, int part_buf,
                                           double* lds)
{
    using R = typename Arith<S>::R;
    const int n_rows = a.ny * a.nz;
    const int ty = t / a.tiles_x, tx = t - ty * a.tiles_x;
    const int tpr = a.tile_w / V;
    const int lr = (int)threadIdx.x / tpr, lc = (int)threadIdx.x - lr * tpr;
    const int row_u = ty * a.tile_rows + lr;
    const int row = min(row_u, n_rows - 1);          // rows past the grid idle (clamped for addressing)
    const int k = row / a.ny, j = row - k * a.ny;
    const int i0 = tx * a.tile_w + lc * V;
    const bool act = i0 < a.nx && row_u < n_rows && lr < a.tile_rows;   // threads past the tile's rows idle
    const int n_own = act ? min(V, a.nx - i0) : 0;

    const int jm = (j == 0) ? a.ny - 1 : j - 1, jp = (j == a.ny - 1) ? 0 : j + 1;   // y and z periodic
    const int km = (k == 0) ? a.nz - 1 : k - 1, kp = (k == a.nz - 1) ? 0 : k + 1;
    // the lattice row each direction pulls from: (y - e_y, z - e_z)
    int64_t src_row[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int y = CY[q] == 1 ? jm : (CY[q] == -1 ? jp : j);
        const int z = CZ[q] == 1 ? km : (CZ[q] == -1 ? kp : k);
        src_row[q] = ((int64_t)z * a.ny + y) * a.lstride;
    }
    const int64_t own_row = (int64_t)row * a.lstride;
    const int64_t r0 = (int64_t)row * a.pitch;       // mask and fields

    // this tile's (tile, body) force slots: loaded first, so that waiting for them
    // never waits for the stores (a vector-memory wait covers every earlier
    // access); a tile without slots holds no solid node and reads no mask
    const int s0 = a.tile_slot_ptr[t];
    const int s1 = a.tile_slot_ptr[t + 1];
    // Dword-or-wider elements (and single nodes) fetch the x-shifted directions
    // as one vector access one element off alignment. 2-byte vectors load aligned
    // and take the missing end element from the neighbouring lane (lanes that
    // start or end a wavefront or a tile row load it themselves), keeping the
    // loaded values packed in the storage type until each node's collision.
    constexpr bool kShifted = sizeof(S) >= 4 || V == 1;
    using LV = typename std::conditional<kShifted, R, S>::type;
    const int lane = (int)(threadIdx.x & 63);
    LV v[Q][V];
    int body[V];
    // 2-byte storage: threads without a node of their own load column 0 of
    // their (clamped) row instead (every access stays inside the lattice; their
    // results are never stored, summed or shuffled into an owned node), which
    // spares the register clearing (1.5% faster); the wider types keep the branch
    const int il = act ? i0 : 0;
    if (sizeof(S) == 2 || act) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            S raw[V];
            const S* p = src + src_row[q] + (int64_t)q * a.pitch;
            if constexpr (kShifted) {
                if (CX[q] == 1) load_vec_shifted<S, V>(p + (il - 1), raw);
                else if (CX[q] == -1) load_vec_shifted<S, V>(p + (il + 1), raw);
                else load_vec<S, V>(p + il, raw);
            } else {
                load_vec<S, V>(p + il, raw);
            }
#pragma unroll
            for (int e = 0; e < V; ++e) v[q][e] = as_lv<LV>(raw[e]);
        }
        if (s1 > s0) {
            load_mask<V>(a.mask + r0 + il, body);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) body[e] = 0;
        }
        if constexpr (kShifted) {
            if (il == 0) {   // the west side: column -1 lies outside
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    if (CX[q] == 1) v[q][0] = pull_col<S, R>(src, q, src_row[q], -1, a);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int e = 0; e < V; ++e) v[q][e] = LV{};
#pragma unroll
        for (int e = 0; e < V; ++e) body[e] = 0;
    }

    // the end elements of the x-shifted directions (lane-shuffle form only)
    R left[Q], right[Q];
    if constexpr (!kShifted) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (CX[q] == 1) left[q] = __shfl_up(dec(v[q][V - 1]), 1, 64);
            if (CX[q] == -1) right[q] = __shfl_down(dec(v[q][0]), 1, 64);
        }
        if (act && (lane == 0 || lc == 0)) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (CX[q] == 1) left[q] = pull_col<S, R>(src, q, src_row[q], i0 - 1, a);
        }
        if (act && (lane == 63 || lc == tpr - 1)) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (CX[q] == -1) right[q] = pull_col<S, R>(src, q, src_row[q], i0 + V, a);
        }
    }

    R fl[7][V];
    double tile_drho = 0.0;
    S out[Q][V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        R f[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if constexpr (kShifted) {
                f[q] = v[q][e];
            } else {
                if (CX[q] == 1) f[q] = (e == 0) ? left[q] : dec(v[q][e > 0 ? e - 1 : 0]);
                else if (CX[q] == -1) f[q] = (e == V - 1) ? right[q] : dec(v[q][e < V - 1 ? e + 1 : 0]);
                else f[q] = dec(v[q][e]);
            }
        }
        const int i = i0 + e;
        if (i == a.nx - 1) {   // the east side: column nx lies outside
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (CX[q] == -1) f[q] = pull_col<S, R>(src, q, src_row[q], a.nx, a);
        }
        const Node3<R> n = collide3<R, (sizeof(S) >= 4)>(f, body[e], i, j, k, a);
#pragma unroll
        for (int q = 0; q < Q; ++q) out[q][e] = enc<S>(f[q]);
        fl[0][e] = n.rho;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            fl[1 + d][e] = n.u[d];
            fl[4 + d][e] = n.fv[d];
        }
        if constexpr (RECORD) {
            // the penalization force of every node of a tile holding solid nodes
            // goes to LDS at once, summed per body after the stores
            if (s1 > s0) {
                R* fv = force_lds<R>();
#pragma unroll
                for (int c = 0; c < 3; ++c) fv[(c * V + e) * (int)blockDim.x + (int)threadIdx.x] = n.fv[c];
            }
        }
        if (e < n_own) tile_drho += (double)n.drho;
    }

    if (n_own == V) {
#pragma unroll
        for (int q = 0; q < Q; ++q) store_vec<S, V>(dst + own_row + (int64_t)q * a.pitch + i0, out[q]);
    } else if (n_own > 0) {   // the ragged end of a row
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (e < n_own)
#pragma unroll
                for (int q = 0; q < Q; ++q) store_one<S>(dst + own_row + (int64_t)q * a.pitch + i0 + e, out[q][e]);
    }

    if constexpr (FIELDS) {
        R* fb = a.fields + r0 + i0;
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (e < n_own)
#pragma unroll
                for (int c = 0; c < 7; ++c) fb[c * a.plane_f + e] = fl[c][e];
    }

    if constexpr (RECORD) {
        // mass: one partial per wavefront (DPP moves only, no block barrier)
        const int lane = (int)(threadIdx.x & 63);
        const double wm = wave_sum_lane63(tile_drho);
        double* mass_part = a.mass_part + part_buf * a.fin.mass_stride;
        double* slot_force = a.slot_force + part_buf * a.fin.slot_stride;
        if (lane == 63) mass_part[(int64_t)t * (a.block >> 6) + (threadIdx.x >> 6)] = wm;
        if (s1 > s0) {   // tiles that hold solid nodes (uniform across the block)
            const R* fv = force_lds<R>();
            const int nt = (int)blockDim.x;
            for (int s = s0; s < s1; ++s) {
                const int b = a.slot_body[s];
                double p[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if (e < n_own && body[e] == b)
#pragma unroll
                        for (int c = 0; c < 3; ++c) p[c] -= (double)fv[(c * V + e) * nt + (int)threadIdx.x];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double sum = block_sum(p[c], lds);
                    if (threadIdx.x == 0) slot_force[3 * s + c] = sum;
                }
            }
        }
    }
}

// tree_sum's binary tree over FIN_LANES virtual lanes, with the same pairwise
// additions (lane v takes lane v + w, w = FIN_LANES / 2 .. 1), where thread t
// holds lanes t + k * blockDim in h[k]: levels w >= blockDim inside each thread,
// levels 64 <= w < blockDim through lds, the last six by wave shuffles. The sum
// is bitwise tree_sum's and lands in thread 0 only.
constexpr int SERIAL_H = FIN_LANES / 64;
__device__ __forceinline__ double serial_tree(double (&h)[SERIAL_H], double* lds)
{
    const int bd = (int)blockDim.x, t = (int)threadIdx.x;
    const int nh = FIN_LANES / bd;
#pragma unroll
    for (int k = SERIAL_H / 2; k > 0; k >>= 1)
        if (k < nh)
#pragma unroll
            for (int i = 0; i < k; ++i) h[i] += h[i + k];
    for (int w = bd / 2; w >= 64; w >>= 1) {
        __syncthreads();   // lds free from the previous level or sum
        if (t >= w && t < 2 * w) lds[t - w] = h[0];
        __syncthreads();
        if (t < w) h[0] += lds[t];
    }
    double v = h[0];
#pragma unroll
    for (int w = 32; w > 0; w >>= 1) v += __shfl_down(v, w, 64);
    return v;
}

// One record: mass and the force on each body, each summed in an order fixed by
// the partials alone, so that neither the block size of the launch that runs it
// nor the way steps are split over calls changes a record by one bit. Block
// `part` of N_LEAD sums its fixed slice of every partial list (FIN_LANES virtual
// lanes, then their binary tree, serial_tree) into its stage row; the last
// block to arrive adds the N_LEAD rows in block order.
__device__ __forceinline__ void finalize3(const Fin3Args& f, int buf, int part, double* lds, int* flag)
{
    const double* pm = f.mass_part + buf * f.mass_stride;
    const double* sf = f.slot_force + buf * f.slot_stride;
    const int row_len = 1 + 3 * f.max_bodies;
    double* row = f.stage + (int64_t)part * row_len;
    const int bd = (int)blockDim.x, t = (int)threadIdx.x, nh = FIN_LANES / bd;
    const int m0 = (int)((int64_t)f.n_mass * part / N_LEAD), m1 = (int)((int64_t)f.n_mass * (part + 1) / N_LEAD);
    {
        double h[SERIAL_H];
#pragma unroll
        for (int k = 0; k < SERIAL_H; ++k) h[k] = k < nh ? lane_sum(pm + m0, m1 - m0, t + k * bd) : 0.0;
        const double m = serial_tree(h, lds);
        if (t == 0) row[0] = m;
    }
    for (int b = 0; b < f.n_bodies; ++b) {   // one pass over the slice serves three components
        const int s0 = f.body_slot_ptr[b], n = f.body_slot_ptr[b + 1] - s0;
        const int a0 = s0 + (int)((int64_t)n * part / N_LEAD), a1 = s0 + (int)((int64_t)n * (part + 1) / N_LEAD);
        double h[3][SERIAL_H];
#pragma unroll
        for (int k = 0; k < SERIAL_H; ++k) {
            double y0 = 0.0, y1 = 0.0, y2 = 0.0;
            if (k < nh)
                for (int kk = a0 + t + k * bd; kk < a1; kk += FIN_LANES) {
                    const double* p = sf + 3 * f.body_slots[kk];
                    y0 += p[0];
                    y1 += p[1];
                    y2 += p[2];
                }
            h[0][k] = y0;
            h[1][k] = y1;
            h[2][k] = y2;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double X = serial_tree(h[c], lds);
            if (t == 0) row[1 + 3 * b + c] = X;
        }
    }
    __threadfence();   // publish the row before counting in
    if (threadIdx.x == 0)
        *flag = atomicAdd(reinterpret_cast<unsigned long long*>(f.arrivals), 1ull) == (unsigned long long)(N_LEAD - 1);
    __syncthreads();
    if (!*flag) return;
    __threadfence();   // the other blocks' rows are visible from here on
    // each column of the N_LEAD rows fetched at once into lds, then added in
    // row order by one thread
    int64_t r = 0;
    if (threadIdx.x == 0) r = *f.rec_count % f.capacity;
    double mass = 0.0;
    for (int col = 0; col < 1 + 3 * f.n_bodies; ++col) {
        __syncthreads();   // lds free from the previous column
        if ((int)threadIdx.x < N_LEAD) lds[threadIdx.x] = f.stage[(int64_t)threadIdx.x * row_len + col];
        __syncthreads();
        if (threadIdx.x == 0) {
            double x = 0.0;
            for (int p = 0; p < N_LEAD; ++p) x += lds[p];
            if (col == 0) mass = x;
            else f.ring_force[(r * f.max_bodies + (col - 1) / 3) * 3 + (col - 1) % 3] = x;
        }
    }
    if (threadIdx.x == 0) {
        f.ring_mass[r] = f.mass_offset + mass;
        *f.rec_count += 1;
        *f.arrivals = 0;
    }
}

// The same record by one block: the N_LEAD slice sums of finalize3 formed in
// turn, each with the same virtual lanes and tree, and added in slice order as
// its last block adds the stage rows, so the result is bitwise the same; no
// stage rows, fences or arrival counter. For small domains, where the partial
// lists are short. One pass over a body's slots serves its three components.
__device__ __forceinline__ void finalize3_serial(const Fin3Args& f, int buf, double* lds)
{
    const double* pm = f.mass_part + buf * f.mass_stride;
    const double* sf = f.slot_force + buf * f.slot_stride;
    const int bd = (int)blockDim.x, t = (int)threadIdx.x, nh = FIN_LANES / bd;
    int64_t r = 0;
    if (t == 0) r = *f.rec_count % f.capacity;
    double mass = 0.0;
    for (int part = 0; part < N_LEAD; ++part) {
        const int m0 = (int)((int64_t)f.n_mass * part / N_LEAD), m1 = (int)((int64_t)f.n_mass * (part + 1) / N_LEAD);
        double h[SERIAL_H];
#pragma unroll
        for (int k = 0; k < SERIAL_H; ++k) h[k] = k < nh ? lane_sum(pm + m0, m1 - m0, t + k * bd) : 0.0;
        mass += serial_tree(h, lds);
    }
    for (int b = 0; b < f.n_bodies; ++b) {
        const int s0 = f.body_slot_ptr[b], n = f.body_slot_ptr[b + 1] - s0;
        double x[3] = {0.0, 0.0, 0.0};
        for (int part = 0; part < N_LEAD; ++part) {
            const int a0 = s0 + (int)((int64_t)n * part / N_LEAD), a1 = s0 + (int)((int64_t)n * (part + 1) / N_LEAD);
            double h[3][SERIAL_H];
#pragma unroll
            for (int k = 0; k < SERIAL_H; ++k) {
                double y0 = 0.0, y1 = 0.0, y2 = 0.0;
                if (k < nh)
                    for (int kk = a0 + t + k * bd; kk < a1; kk += FIN_LANES) {
                        const double* p = sf + 3 * f.body_slots[kk];
                        y0 += p[0];
                        y1 += p[1];
                        y2 += p[2];
                    }
                h[0][k] = y0;
                h[1][k] = y1;
                h[2][k] = y2;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) x[c] += serial_tree(h[c], lds);
        }
        if (t == 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) f.ring_force[(r * f.max_bodies + b) * 3 + c] = x[c];
    }
    if (t == 0) {
        f.ring_mass[r] = f.mass_offset + mass;
        *f.rec_count += 1;
    }
}

// A step launch: when the previous step recorded (fin_buf >= 0), N_LEAD leading
// blocks sum that record while the other blocks stream their tiles.
template <typename S, int V, bool RECORD, bool FIELDS>
__global__ void __launch_bounds__(256)
k_step3(const S* __restrict__ src, S* __restrict__ dst, Step3Args<typename Arith<S>::R> a)
{
    __shared__ double lds[FIN_LANES];   // the record sums; per-wavefront sums of block_sum
    const int lead = a.fin_buf >= 0 ? N_LEAD : 0;
    if ((int)blockIdx.x < lead) {
        __shared__ int last;
        finalize3(a.fin, a.fin_buf, (int)blockIdx.x, lds, &last);
        return;
    }
    const int t = xcd_tile(a.tiles_per_xcd, a.band_log2, lead);
    if (t >= a.n_tiles) return;   // whole block
    step3_body<S, V, RECORD, FIELDS>(src, dst, a, t, a.part_buf, lds);
}

// Many domains in one launch: block -> (member, tile) through the tile map; each
// member's arguments and lattices live in device memory. The members step in
// lockstep: one step kind, record flag and partial buffer for all; one leading
// block per member sums that member's previous record (finalize3_serial).
template <typename S, int V, bool RECORD, bool FIELDS>
__global__ void __launch_bounds__(256) k_step3_batch(Batch3Launch b)
{
    using R = typename Arith<S>::R;
    __shared__ double lds[FIN_LANES];
    const Member3<R>* m = static_cast<const Member3<R>*>(b.members);
    if ((int)blockIdx.x < b.n_fin) {
        if ((int)blockIdx.x < b.n_members) finalize3_serial(m[blockIdx.x].a.fin, b.fin_buf, lds);
        return;
    }
    const int g = xcd_tile(b.tiles_per_xcd, b.band_log2, b.n_fin);
    if (g >= b.total_tiles) return;   // whole block
#if defined(__HIP_DEVICE_COMPILE__)
    // the tile map and the members do not change during a launch: read through
    // the constant address space (scalar loads no store of the step can alias),
    // the member copied once, up front
    using CI = const __attribute__((address_space(4))) int32_t;
    using CM = const __attribute__((address_space(4))) Member3<R>;
    const int d = ((CI*)b.tile_domain)[g];
    const Member3<R> md = ((CM*)m)[d];
    const int t = g - ((CI*)b.tile_start)[d];
#else
    const int d = b.tile_domain[g];
    const Member3<R>& md = m[d];
    const int t = g - b.tile_start[d];
#endif
    const int cur = md.cur ^ b.flip;
    const S* src = static_cast<const S*>(cur ? md.lat1 : md.lat0);
    S* dst = static_cast<S*>(cur ? md.lat0 : md.lat1);
    step3_body<S, V, RECORD, FIELDS>(src, dst, md.a, t, b.part_buf, lds);
}

// The last record of an lbvp3_batch_step call: one block per member.
template <typename R>
__global__ void __launch_bounds__(FIN_THREADS) k_finalize3_members(Batch3Launch b)
{
    __shared__ double lds[FIN_LANES];
    const Member3<R>* m = static_cast<const Member3<R>*>(b.members);
    finalize3_serial(m[blockIdx.x].a.fin, b.fin_buf, lds);
}

// The last record of an lbvp3_step call, summed on its own (N_LEAD blocks).
__global__ void __launch_bounds__(FIN_THREADS) k_finalize3(Fin3Args f, int32_t buf)
{
    __shared__ double lds[FIN_LANES];
    __shared__ int last;
    finalize3(f, buf, (int)blockIdx.x, lds, &last);
}

// ------------------------------------------------------------ conversions --
__constant__ double W3[Q] = {1.0 / 3.0,
                             1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

__device__ __forceinline__ void conv_node(const Conv3Args& a, int64_t n, int64_t& lat_off, int64_t& fld_off)
{
    const int64_t per_plane = (int64_t)a.ny * a.nx;
    const int kl = (int)(n / per_plane);
    const int64_t rem = n - kl * per_plane;
    const int j = (int)(rem / a.nx), i = (int)(rem - (int64_t)j * a.nx);
    const int64_t row = (int64_t)(a.plane0 + kl) * a.ny + j;
    lat_off = row * a.lstride + i;
    fld_off = row * a.pitch + i;
}

// Algorithm step (1): equilibrium populations (eq. feq) of staged planes, in
// FP64, stored as normalized deviations; the fields of step 0 are (rho, u, 0).
template <typename S>
__global__ void __launch_bounds__(256) k_init3(S* lat, typename Arith<S>::R* fields, Conv3Args a)
{
    using R = typename Arith<S>::R;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)a.planes * a.ny * a.nx) return;
    int64_t lo, fo;
    conv_node(a, n, lo, fo);
    const double rho = a.rho ? a.rho[n] : a.rho0;
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = a.u[d] ? a.u[d][n] : 0.0;
    const double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double eu = (CX[q] * u[0] + CY[q] * u[1]) + CZ[q] * u[2];
        const double h = (rho - a.rho0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        lat[lo + q * a.pitch] = enc<S>((R)h);
    }
    if (fields) {
        fields[fo] = (R)rho;
        for (int d = 0; d < 3; ++d) {
            fields[(1 + d) * a.plane_f + fo] = (R)u[d];
            fields[(4 + d) * a.plane_f + fo] = R(0);
        }
    }
}

template <typename S>
__global__ void __launch_bounds__(256) k_decode3(const S* lat, Conv3Args a)
{
    const int64_t N = (int64_t)a.planes * a.ny * a.nx;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    int64_t lo, fo;
    conv_node(a, n, lo, fo);
    for (int q = 0; q < Q; ++q) a.pops[q * N + n] = W3[q] * ((double)dec(lat[lo + q * a.pitch]) + a.rho0);
}

template <typename S>
__global__ void __launch_bounds__(256) k_encode3(S* lat, Conv3Args a)
{
    using R = typename Arith<S>::R;
    const int64_t N = (int64_t)a.planes * a.ny * a.nx;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    int64_t lo, fo;
    conv_node(a, n, lo, fo);
    for (int q = 0; q < Q; ++q) lat[lo + q * a.pitch] = enc<S>((R)(a.pops[q * N + n] / W3[q] - a.rho0));
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

template <typename S, int V>
hipError_t step_v(bool record, bool fields, const S* in, S* out, const Step3Args<typename Arith<S>::R>& a,
                  hipStream_t s)
{
    using R = typename Arith<S>::R;
    const dim3 grid((unsigned)(a.tiles_per_xcd * N_XCD + (a.fin_buf >= 0 ? N_LEAD : 0))), block((unsigned)a.block);
    const size_t lds = record ? 3 * (size_t)V * (size_t)a.block * sizeof(R) : 0;
    if (record) {
        if (fields) hipLaunchKernelGGL((k_step3<S, V, true, true>), grid, block, lds, s, in, out, a);
        else hipLaunchKernelGGL((k_step3<S, V, true, false>), grid, block, lds, s, in, out, a);
    } else {
        if (fields) hipLaunchKernelGGL((k_step3<S, V, false, true>), grid, block, 0, s, in, out, a);
        else hipLaunchKernelGGL((k_step3<S, V, false, false>), grid, block, 0, s, in, out, a);
    }
    return hipGetLastError();
}

template <typename S>
hipError_t step_typed(bool record, bool fields, const void* src, void* dst, const void* args_v, hipStream_t s)
{
    using R = typename Arith<S>::R;
    const Step3Args<R>& a = *static_cast<const Step3Args<R>*>(args_v);
    const S* in = static_cast<const S*>(src);
    S* out = static_cast<S*>(dst);
    if (a.vec == 1) return step_v<S, 1>(record, fields, in, out, a, s);
    if constexpr (sizeof(S) >= 4) {
        if (a.vec == 2) return step_v<S, 2>(record, fields, in, out, a, s);
    }
    if constexpr (sizeof(S) == 4) {
        if (a.vec == 4) return step_v<S, 4>(record, fields, in, out, a, s);
    }
    if constexpr (sizeof(S) == 2) {   // lane-shuffle forms: 8 and 16 bytes per thread
        if (a.vec == 4) return step_v<S, 4>(record, fields, in, out, a, s);
        if (a.vec == 8) return step_v<S, 8>(record, fields, in, out, a, s);
    }
    return hipErrorInvalidValue;
}

template <typename S, int V>
hipError_t batch_v(bool record, bool fields, const Batch3Launch& b, int32_t block, hipStream_t s)
{
    using R = typename Arith<S>::R;
    const dim3 grid((unsigned)(b.tiles_per_xcd * N_XCD + b.n_fin)), blk((unsigned)block);
    const size_t lds = record ? 3 * (size_t)V * (size_t)block * sizeof(R) : 0;
    if (record) {
        if (fields) hipLaunchKernelGGL((k_step3_batch<S, V, true, true>), grid, blk, lds, s, b);
        else hipLaunchKernelGGL((k_step3_batch<S, V, true, false>), grid, blk, lds, s, b);
    } else {
        if (fields) hipLaunchKernelGGL((k_step3_batch<S, V, false, true>), grid, blk, 0, s, b);
        else hipLaunchKernelGGL((k_step3_batch<S, V, false, false>), grid, blk, 0, s, b);
    }
    return hipGetLastError();
}

template <typename S>
hipError_t batch_typed(int32_t vec, int32_t block, bool record, bool fields, const Batch3Launch& b, hipStream_t s)
{
    if (vec == 1) return batch_v<S, 1>(record, fields, b, block, s);
    if constexpr (sizeof(S) >= 4) {
        if (vec == 2) return batch_v<S, 2>(record, fields, b, block, s);
    }
    if constexpr (sizeof(S) == 4) {
        if (vec == 4) return batch_v<S, 4>(record, fields, b, block, s);
    }
    if constexpr (sizeof(S) == 2) {
        if (vec == 4) return batch_v<S, 4>(record, fields, b, block, s);
        if (vec == 8) return batch_v<S, 8>(record, fields, b, block, s);
    }
    return hipErrorInvalidValue;
}

unsigned conv_blocks(const Conv3Args& a) { return (unsigned)(((int64_t)a.planes * a.ny * a.nx + 255) / 256); }

}  // namespace

bool vec_supported(int32_t storage, int32_t vec)
{
    switch (storage) {
    case LBVP_F64: return vec == 1 || vec == 2;
    case LBVP_F32: return vec == 1 || vec == 2 || vec == 4;
    case LBVP_F16_DEV:
    case LBVP_BF16_DEV: return vec == 1 || vec == 4 || vec == 8;
    default: return false;
    }
}

hipError_t launch_step3(int32_t storage, bool record, bool fields, const void* src, void* dst, const void* step_args,
                        hipStream_t s)
{
    switch (storage) {
    case LBVP_F64: return step_typed<double>(record, fields, src, dst, step_args, s);
    case LBVP_F32: return step_typed<float>(record, fields, src, dst, step_args, s);
    case LBVP_F16_DEV: return step_typed<_Float16>(record, fields, src, dst, step_args, s);
    case LBVP_BF16_DEV: return step_typed<__bf16>(record, fields, src, dst, step_args, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step3_batch(int32_t storage, int32_t vec, int32_t block, bool record, bool fields,
                              const Batch3Launch& b, hipStream_t s)
{
    switch (storage) {
    case LBVP_F64: return batch_typed<double>(vec, block, record, fields, b, s);
    case LBVP_F32: return batch_typed<float>(vec, block, record, fields, b, s);
    case LBVP_F16_DEV: return batch_typed<_Float16>(vec, block, record, fields, b, s);
    case LBVP_BF16_DEV: return batch_typed<__bf16>(vec, block, record, fields, b, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize3_members(int32_t storage, const Batch3Launch& b, hipStream_t s)
{
    if (storage == LBVP_F64) hipLaunchKernelGGL(k_finalize3_members<double>, dim3(b.n_members), dim3(FIN_THREADS), 0, s, b);
    else hipLaunchKernelGGL(k_finalize3_members<float>, dim3(b.n_members), dim3(FIN_THREADS), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_finalize3(const Fin3Args& a, int32_t buf, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize3, dim3(N_LEAD), dim3(FIN_THREADS), 0, s, a, buf);
    return hipGetLastError();
}

hipError_t launch_init3(int32_t storage, void* lat, void* fields, const Conv3Args& a, hipStream_t s)
{
    const dim3 g(conv_blocks(a)), b(256);
    switch (storage) {
    case LBVP_F64: hipLaunchKernelGGL(k_init3<double>, g, b, 0, s, (double*)lat, (double*)fields, a); break;
    case LBVP_F32: hipLaunchKernelGGL(k_init3<float>, g, b, 0, s, (float*)lat, (float*)fields, a); break;
    case LBVP_F16_DEV: hipLaunchKernelGGL(k_init3<_Float16>, g, b, 0, s, (_Float16*)lat, (float*)fields, a); break;
    case LBVP_BF16_DEV: hipLaunchKernelGGL(k_init3<__bf16>, g, b, 0, s, (__bf16*)lat, (float*)fields, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_decode3(int32_t storage, const void* lat, const Conv3Args& a, hipStream_t s)
{
    const dim3 g(conv_blocks(a)), b(256);
    switch (storage) {
    case LBVP_F64: hipLaunchKernelGGL(k_decode3<double>, g, b, 0, s, (const double*)lat, a); break;
    case LBVP_F32: hipLaunchKernelGGL(k_decode3<float>, g, b, 0, s, (const float*)lat, a); break;
    case LBVP_F16_DEV: hipLaunchKernelGGL(k_decode3<_Float16>, g, b, 0, s, (const _Float16*)lat, a); break;
    case LBVP_BF16_DEV: hipLaunchKernelGGL(k_decode3<__bf16>, g, b, 0, s, (const __bf16*)lat, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_encode3(int32_t storage, void* lat, const Conv3Args& a, hipStream_t s)
{
    const dim3 g(conv_blocks(a)), b(256);
    switch (storage) {
    case LBVP_F64: hipLaunchKernelGGL(k_encode3<double>, g, b, 0, s, (double*)lat, a); break;
    case LBVP_F32: hipLaunchKernelGGL(k_encode3<float>, g, b, 0, s, (float*)lat, a); break;
    case LBVP_F16_DEV: hipLaunchKernelGGL(k_encode3<_Float16>, g, b, 0, s, (_Float16*)lat, a); break;
    case LBVP_BF16_DEV: hipLaunchKernelGGL(k_encode3<__bf16>, g, b, 0, s, (__bf16*)lat, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zero_i64(int64_t* p, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}

}  // namespace lbvp3
