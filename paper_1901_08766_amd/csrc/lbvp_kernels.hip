// lbvp_kernels.hip -- gfx950 kernels of the fused D2Q9 TRT-VP time step.
//
// Data layout in HBM (structure of arrays): population a of node (i, j) lives at
// lattice[a * plane + j * pitch + i]; pitch is a multiple of 64 elements, so
// every row starts on a 256-byte boundary (FP32). All storage types hold the
// deviation f_a - w_a rho0, which keeps the stored magnitudes small (|u| ~ 0.1
// gives |deviation| ~ 0.05) and the FP32/FP16/BF16 rounding error with them.
//
// One step (Sec. 2.2, steps (2)-(6)), per node, fused:
//   pull   f_a(x) = g_a(x - e_a)                      eq. (streaming)
//   rho = rho0 + sum f~_a,  rho u* = sum e_a f~_a + F_b/2   eqs. (rho), (rho*velocity-star)
//   chi from the mask, U_O = V + omega z x (x - c) of the node's body
//   du = chi (U_O - u*) / (2 eta + chi),  F_VP = 2 rho du    eqs. (d-V), (force-density)
//   u = u* + du,  F = F_b + F_VP                       eq. (velocity-r)
//   g_a = f_a - (f+_a - f^eq+_a)/tau+ - (f-_a - f^eq-_a)/tau-
//         + (1 - 1/(2 tau+)) F+_a + (1 - 1/(2 tau-)) F-_a        eqs. (TRT-collision), (collision-modified)
// with f^eq of eq. (feq) and F_a of eq. (external-force-term), both taken at the
// corrected u and split into parts even (+) and odd (-) under a -> opposite(a).
// For a pair (a, opposite a) with eu = e_a.u and eF = e_a.F the parts are
//   f^eq+ - w rho0 = w (drho + rho (9/2 eu^2 - 3/2 u.u)),  f^eq- = 3 w rho eu,
//   F+ = w (9 eu eF - 3 u.F),                           F- = 3 w eF.
//
// The step is bound by HBM traffic: 9 loads, 9 stores and one mask byte per node
// against ~200 flops, so there is no matrix-core work here.
#include <hip/hip_runtime.h>

#include "lbvp_internal.h"

namespace lbvp {
namespace {

// ------------------------------------------------------------ storage codecs --
__device__ __forceinline__ double dec(double v) { return v; }
__device__ __forceinline__ float dec(float v) { return v; }
__device__ __forceinline__ float dec(_Float16 v) { return (float)v; }
__device__ __forceinline__ float dec(__bf16 v) { return (float)v; }

template <typename S, typename R>
__device__ __forceinline__ S enc(R v) { return (S)v; }  // round to nearest even

template <typename S> struct Arith { using R = float; };
template <> struct Arith<double> { using R = double; };

// ------------------------------------------------------------ reductions --
// Sum over a 256-thread block in a fixed order (deterministic); result valid in
// thread 0. lds must hold 4 doubles and is reused across calls.
__device__ __forceinline__ double block_sum_256(double v, double* lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// ------------------------------------------------------------ the step --
template <typename R>
struct Pair {
    R ga, gb;
};

// Collision of a population pair (a, opposite a) of weight w.
template <typename R>
__device__ __forceinline__ Pair<R> collide_pair(R fa, R fb, R w, R eu, R eF, R drho, R rho, R uu,
                                                R uF, const StepArgs<R>& a)
{
    const R half = R(0.5);
    const R sp = half * (fa + fb);
    const R sm = half * (fa - fb);
    const R ep = w * (drho + rho * (R(4.5) * eu * eu - R(1.5) * uu));
    const R em = R(3) * w * rho * eu;
    const R Fp = w * (R(9) * eu * eF - R(3) * uF);
    const R Fm = R(3) * w * eF;
    const R gp = sp - a.om_p * (sp - ep) + a.k_p * Fp;
    const R gm = sm - a.om_m * (sm - em) + a.k_m * Fm;
    return {gp + gm, gp - gm};
}

template <typename S, bool RECORD, bool FIELDS>
__global__ void __launch_bounds__(TILE_X)
k_step_pull(const S* __restrict__ src, S* __restrict__ dst, StepArgs<typename Arith<S>::R> a)
{
    using R = typename Arith<S>::R;
    const int blk = blockIdx.x;
    const int t = (blk % N_XCD) * a.tiles_per_xcd + blk / N_XCD;
    if (t >= a.n_tiles) return;  // whole block
    const int j = t / a.tiles_x;
    const int i = (t - j * a.tiles_x) * TILE_X + (int)threadIdx.x;
    const bool on = i < a.nx;

    R drho = 0, fvx = 0, fvy = 0;
    int body = 0;
    if (on) {
        // source rows/columns of the pull, with the domain sides resolved
        const int jm = (j == 0) ? a.ny - 1 : j - 1;        // rows are periodic
        const int jp = (j == a.ny - 1) ? 0 : j + 1;
        int im = i - 1, ip = i + 1;
        bool w_in = false, e_in = false;
        if (i == 0) {
            if (a.west == SIDE_PERIODIC) im = a.nx - 1;
            else { im = 0; w_in = (a.west == SIDE_INFLOW_EQ); }
        }
        if (i == a.nx - 1) {
            if (a.east == SIDE_PERIODIC) ip = 0;
            else { ip = a.nx - 1; e_in = (a.east == SIDE_INFLOW_EQ); }
        }
        const int64_t r0 = (int64_t)j * a.pitch, rm = (int64_t)jm * a.pitch, rp = (int64_t)jp * a.pitch;
        const int64_t P = a.plane;
        const R f0 = dec(src[r0 + i]);
        const R f1 = w_in ? a.feq_in[1] : dec(src[1 * P + r0 + im]);
        const R f2 = dec(src[2 * P + rm + i]);
        const R f3 = e_in ? a.feq_in[3] : dec(src[3 * P + r0 + ip]);
        const R f4 = dec(src[4 * P + rp + i]);
        const R f5 = w_in ? a.feq_in[5] : dec(src[5 * P + rm + im]);
        const R f6 = e_in ? a.feq_in[6] : dec(src[6 * P + rm + ip]);
        const R f7 = e_in ? a.feq_in[7] : dec(src[7 * P + rp + ip]);
        const R f8 = w_in ? a.feq_in[8] : dec(src[8 * P + rp + im]);
        body = a.mask[r0 + i];

        // moments (deviation form: sum w_a rho0 = rho0, sum e_a w_a = 0)
        drho = ((f0 + f1) + (f2 + f3)) + ((f4 + f5) + (f6 + f7)) + f8;
        const R rho = a.rho0 + drho;
        const R jx = (f1 - f3) + (f5 - f7) + (f8 - f6);
        const R jy = (f2 - f4) + (f5 - f7) + (f6 - f8);
        const R inv_rho = R(1) / rho;
        R ux = (jx + R(0.5) * a.fbx) * inv_rho;   // u*
        R uy = (jy + R(0.5) * a.fby) * inv_rho;

        // volume penalization, branch-free: row 0 of the body table is zero
        const R* B = a.bodies + 5 * body;
        const R uox = B[2] - B[4] * ((R)j - B[1]);
        const R uoy = B[3] + B[4] * ((R)i - B[0]);
        const R c = body ? a.vp_c : R(0);
        const R dux = c * (uox - ux);
        const R duy = c * (uoy - uy);
        fvx = R(2) * rho * dux;
        fvy = R(2) * rho * duy;
        ux += dux;
        uy += duy;
        const R Fx = a.fbx + fvx, Fy = a.fby + fvy;

        const R uu = ux * ux + uy * uy;
        const R uF = ux * Fx + uy * Fy;
        const R w0 = R(4.0 / 9.0), w1 = R(1.0 / 9.0), w5 = R(1.0 / 36.0);
        const R g0 = f0 - a.om_p * (f0 - w0 * (drho - R(1.5) * rho * uu)) + a.k_p * (R(-3) * w0 * uF);
        const Pair<R> p13 = collide_pair(f1, f3, w1, ux, Fx, drho, rho, uu, uF, a);
        const Pair<R> p24 = collide_pair(f2, f4, w1, uy, Fy, drho, rho, uu, uF, a);
        const Pair<R> p57 = collide_pair(f5, f7, w5, ux + uy, Fx + Fy, drho, rho, uu, uF, a);
        const Pair<R> p68 = collide_pair(f6, f8, w5, uy - ux, Fy - Fx, drho, rho, uu, uF, a);

        S* d = dst + r0 + i;
        d[0] = enc<S>(g0);
        d[1 * P] = enc<S>(p13.ga);
        d[2 * P] = enc<S>(p24.ga);
        d[3 * P] = enc<S>(p13.gb);
        d[4 * P] = enc<S>(p24.gb);
        d[5 * P] = enc<S>(p57.ga);
        d[6 * P] = enc<S>(p68.ga);
        d[7 * P] = enc<S>(p57.gb);
        d[8 * P] = enc<S>(p68.gb);

        if constexpr (FIELDS) {
            R* fl = a.fields + r0 + i;
            const int64_t F = a.plane_f;
            fl[0] = rho;
            fl[F] = ux;
            fl[2 * F] = uy;
            fl[3 * F] = fvx;
            fl[4 * F] = fvy;
        }
    }

    if constexpr (RECORD) {
        __shared__ double lds[4];
        const double m = block_sum_256((double)drho, lds);
        if (threadIdx.x == 0) a.tile_mass[t] = m;
        const int s0 = a.tile_slot_ptr[t], s1 = a.tile_slot_ptr[t + 1];
        for (int s = s0; s < s1; ++s) {   // uniform across the block
            const int b = a.slot_body[s];
            const bool mine = on && body == b;
            const double sx = block_sum_256(mine ? -(double)fvx : 0.0, lds);
            const double sy = block_sum_256(mine ? -(double)fvy : 0.0, lds);
            if (threadIdx.x == 0) {
                a.slot_force[2 * s] = sx;
                a.slot_force[2 * s + 1] = sy;
            }
        }
    }
}

// Sum the per-tile partials of one record into the ring, in a fixed order.
__global__ void __launch_bounds__(FIN_THREADS) k_finalize(FinalizeArgs a)
{
    __shared__ double sx[FIN_THREADS], sy[FIN_THREADS];
    const int tid = threadIdx.x;
    const int64_t r = *a.rec_count % a.capacity;
    for (int b = 0; b <= a.n_bodies; ++b) {
        double x = 0.0, y = 0.0;
        if (b < a.n_bodies) {
            for (int k = a.body_slot_ptr[b] + tid; k < a.body_slot_ptr[b + 1]; k += FIN_THREADS) {
                const int s = a.body_slots[k];
                x += a.slot_force[2 * s];
                y += a.slot_force[2 * s + 1];
            }
        } else {
            for (int k = tid; k < a.n_tiles; k += FIN_THREADS) x += a.tile_mass[k];
        }
        sx[tid] = x;
        sy[tid] = y;
        __syncthreads();
        for (int w = FIN_THREADS / 2; w > 0; w >>= 1) {
            if (tid < w) {
                sx[tid] += sx[tid + w];
                sy[tid] += sy[tid + w];
            }
            __syncthreads();
        }
        if (tid == 0) {
            if (b < a.n_bodies) {
                a.ring_force[(r * a.max_bodies + b) * 2] = sx[0];
                a.ring_force[(r * a.max_bodies + b) * 2 + 1] = sy[0];
            } else {
                a.ring_mass[r] = a.mass_offset + sx[0];
            }
        }
        __syncthreads();
    }
    if (tid == 0) *a.rec_count += 1;
}

// ------------------------------------------------------------ conversions --
__constant__ double W_ALL[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
__constant__ int EX_ALL[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int EY_ALL[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Algorithm step (1): populations at equilibrium (eq. feq) for staged rows, in
// FP64, stored as deviations; the fields of step 0 are (rho, u, 0, 0).
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
    for (int q = 0; q < 9; ++q) {
        const double eu = EX_ALL[q] * ux + EY_ALL[q] * uy;
        const double dev = W_ALL[q] * ((rho - a.rho0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
        lat[q * a.plane + o] = enc<S>((R)dev);
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
    const int64_t o = (int64_t)(a.row0 + jl) * a.pitch + i;
    for (int q = 0; q < 9; ++q) a.pops[q * n + k] = (double)dec(lat[q * a.plane + o]) + W_ALL[q] * a.rho0;
}

template <typename S>
__global__ void __launch_bounds__(256) k_encode(S* lat, ConvArgs a)
{
    using R = typename Arith<S>::R;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)a.rows * a.nx;
    if (k >= n) return;
    const int jl = (int)(k / a.nx), i = (int)(k - (int64_t)jl * a.nx);
    const int64_t o = (int64_t)(a.row0 + jl) * a.pitch + i;
    for (int q = 0; q < 9; ++q) lat[q * a.plane + o] = enc<S>((R)(a.pops[q * n + k] - W_ALL[q] * a.rho0));
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

template <typename S>
hipError_t step_typed(bool record, bool fields, const void* src, void* dst, const void* args_v,
                      hipStream_t s)
{
    using R = typename Arith<S>::R;
    const StepArgs<R>& a = *static_cast<const StepArgs<R>*>(args_v);
    const dim3 grid((unsigned)(a.tiles_per_xcd * N_XCD)), block(TILE_X);
    const S* in = static_cast<const S*>(src);
    S* out = static_cast<S*>(dst);
    if (record) {
        if (fields) hipLaunchKernelGGL((k_step_pull<S, true, true>), grid, block, 0, s, in, out, a);
        else hipLaunchKernelGGL((k_step_pull<S, true, false>), grid, block, 0, s, in, out, a);
    } else {
        if (fields) hipLaunchKernelGGL((k_step_pull<S, false, true>), grid, block, 0, s, in, out, a);
        else hipLaunchKernelGGL((k_step_pull<S, false, false>), grid, block, 0, s, in, out, a);
    }
    return hipGetLastError();
}

unsigned conv_blocks(const ConvArgs& a) { return (unsigned)(((int64_t)a.rows * a.nx + 255) / 256); }

}  // namespace

hipError_t launch_step(int32_t storage, bool record, bool fields, const void* src, void* dst,
                       const void* step_args, hipStream_t s)
{
    switch (storage) {
    case ST_F64: return step_typed<double>(record, fields, src, dst, step_args, s);
    case ST_F32: return step_typed<float>(record, fields, src, dst, step_args, s);
    case ST_F16: return step_typed<_Float16>(record, fields, src, dst, step_args, s);
    case ST_BF16: return step_typed<__bf16>(record, fields, src, dst, step_args, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, s, a);
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

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

}  // namespace lbvp
