// lbvp_device.h -- device building blocks shared by the D2Q9 and D3Q19 step
// kernels: storage codecs, aligned and one-off vector accesses, deterministic
// block and record sums, the quotients whose rounding must not drift, the
// collision of one population pair, and the XCD-aware tile order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbvp {
namespace {

constexpr int N_XCD_DEV = 8;   // XCDs of an MI355X; workgroups are dealt to them round-robin
// ------------------------------------------------------------ storage codecs --
__device__ __forceinline__ double dec(double v) { return v; }
__device__ __forceinline__ float dec(float v) { return v; }
__device__ __forceinline__ float dec(_Float16 v) { return (float)v; }
__device__ __forceinline__ float dec(__bf16 v) { return (float)v; }

// A loaded element kept in the storage type (LV = S) or decoded (LV = R).
template <typename LV, typename S>
__device__ __forceinline__ LV as_lv(S x)
{
    if constexpr (std::is_same<LV, S>::value) return x;
    else return dec(x);
}

template <typename S, typename R>
__device__ __forceinline__ S enc(R v) { return (S)v; }  // round to nearest even

// Two values of a 2-byte storage type from one packed conversion (round to
// nearest even, as enc), written to out[0], out[1]. The values are first pinned
// as FP32 results (an empty register constraint, no instruction): otherwise the
// compiler may fuse a conversion with the multiply-add that produced its value
// into one mixed-precision operation that rounds once, straight to FP16, which
// rounds some values differently from FP32-then-FP16 and would make launch
// forms of one step disagree bitwise.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
template <typename S>
__device__ __forceinline__ void enc2(float a, float b, S* out)
{
    static_assert(sizeof(S) == 2, "packed conversion of 2-byte storage types");
    asm("" : "+v"(a), "+v"(b));
    const f32x2_t v = {a, b};
    if constexpr (std::is_same<S, _Float16>::value) {
        const f16x2_t h = __builtin_convertvector(v, f16x2_t);
        __builtin_memcpy(out, &h, 4);
    } else {
        const bf16x2_t h = __builtin_convertvector(v, bf16x2_t);
        __builtin_memcpy(out, &h, 4);
    }
}

template <typename S> struct Arith { using R = float; };
template <> struct Arith<double> { using R = double; };

// base + elem elements, the element offset taken as a 32-bit byte offset (the
// caller guarantees it fits): the address is a uniform base plus a zero-extended
// 32-bit lane offset, the form of the scalar-base global access.
template <typename T>
__device__ __forceinline__ T* at_off32(T* base, uint32_t elem)
{
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(base) + elem * (uint32_t)sizeof(T));
}

// The wavefront's values moved one lane up (lane l gets lane l - 1) or down
// (lane l gets lane l + 1) by a DPP wavefront shift, a VALU move rather than a
// trip through the LDS crossbar; the end lane gets 0 (callers load lanes 0 and
// 63's end elements themselves).
__device__ __forceinline__ float wave_shift_up1(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_shift_down1(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double wave_shift_up1(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_shift_down1(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// V consecutive elements moved as one aligned access of V * sizeof(S) bytes.
template <typename S, int V>
__device__ __forceinline__ void load_vec(const S* p, S (&out)[V])
{
    constexpr int B = V * (int)sizeof(S);
    if constexpr (B == 16) {
        const uint4 r = *reinterpret_cast<const uint4*>(p);
        __builtin_memcpy(out, &r, 16);
    } else if constexpr (B == 8) {
        const uint2 r = *reinterpret_cast<const uint2*>(p);
        __builtin_memcpy(out, &r, 8);
    } else if constexpr (B == 4) {
        const uint32_t r = *reinterpret_cast<const uint32_t*>(p);
        __builtin_memcpy(out, &r, 4);
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) out[k] = p[k];
    }
}

// Stores are non-temporal: the new lattice is not read again before the whole
// domain has streamed through the caches, so it should not displace anything.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

template <typename S, int V>
__device__ __forceinline__ void store_vec(S* p, const S (&in)[V])
{
    constexpr int B = V * (int)sizeof(S);
    if constexpr (B == 16) {
        u32x4_t r;
        __builtin_memcpy(&r, in, 16);
        __builtin_nontemporal_store(r, reinterpret_cast<u32x4_t*>(p));
    } else if constexpr (B == 8) {
        u32x2_t r;
        __builtin_memcpy(&r, in, 8);
        __builtin_nontemporal_store(r, reinterpret_cast<u32x2_t*>(p));
    } else if constexpr (B == 4) {
        uint32_t r;
        __builtin_memcpy(&r, in, 4);
        __builtin_nontemporal_store(r, reinterpret_cast<uint32_t*>(p));
    } else if constexpr (B == 2) {
        uint16_t r;
        __builtin_memcpy(&r, in, 2);
        __builtin_nontemporal_store(r, reinterpret_cast<uint16_t*>(p));
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) p[k] = in[k];
    }
}

// One element, non-temporal like the vector stores. Every store of the lattice
// carries the hint: where the compiler merges a vector path and an element path
// into one store, it keeps only the hints both carry, and a plain element store
// there once stripped it from all 19 stores of a 3-D step (7% slower).
template <typename S>
__device__ __forceinline__ void store_one(S* p, S v)
{
    const S tmp[1] = {v};
    store_vec<S, 1>(p, tmp);
}

// The same V elements starting one element off a 16-byte boundary: a single
// vector access that needs only the element's own (dword or wider) alignment.
template <typename S, int V>
__device__ __forceinline__ void load_vec_shifted(const S* p, S (&out)[V])
{
    static_assert(sizeof(S) >= 4 || V == 1, "sub-dword vectors take the lane-shuffle path");
    __builtin_memcpy(out, p, V * sizeof(S));
}

template <int V>
__device__ __forceinline__ void load_mask(const uint8_t* p, int (&out)[V])
{
    uint8_t b[V];
    if constexpr (V == 8) {
        const uint2 r = *reinterpret_cast<const uint2*>(p);
        __builtin_memcpy(b, &r, 8);
    } else if constexpr (V == 4) {
        const uint32_t r = *reinterpret_cast<const uint32_t*>(p);
        __builtin_memcpy(b, &r, 4);
    } else if constexpr (V == 2) {
        const uint16_t r = *reinterpret_cast<const uint16_t*>(p);
        __builtin_memcpy(b, &r, 2);
    } else {
        b[0] = p[0];
    }
#pragma unroll
    for (int k = 0; k < V; ++k) out[k] = b[k];
}

// ------------------------------------------------------------ reductions --
// One DPP move of a double (both 32-bit halves with the same control); lanes
// whose source lies outside the pattern, or whose row is masked off, read 0.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, BANK_MASK, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, BANK_MASK, true);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront, returned in lane 63, in an order fixed
// by the code: running sums over 2, 4, 8, 16 lanes within each row of 16
// (row_shr 1, 2, 4, 8), then row 0's total into row 1 and row 2's into row 3
// (row_bcast 15), then rows 0-1 into rows 2-3 (row_bcast 31). DPP moves are
// ALU operations of a few cycles; a chain of six LDS-permute shuffles at the end
// of every wavefront of a recording step cost ~7% of a 3-D step.
__device__ __forceinline__ double wave_sum_lane63(double x)
{
    x += dpp_f64<0x111, 0xf, 0xf>(x);   // row_shr:1
    x += dpp_f64<0x112, 0xf, 0xf>(x);   // row_shr:2
    x += dpp_f64<0x114, 0xf, 0xf>(x);   // row_shr:4
    x += dpp_f64<0x118, 0xf, 0xf>(x);   // row_shr:8: lane 16 r + 15 holds row r's sum
    x += dpp_f64<0x142, 0xa, 0xf>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp_f64<0x143, 0xc, 0xf>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// Dynamic LDS of a recording step launch: [2][V][blockDim] values of the
// arithmetic type (the penalization force of every node of the tile).
template <typename R>
__device__ __forceinline__ R* dyn_lds()
{
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    return reinterpret_cast<R*>(lds_dyn);
}


// Sum over the block in a fixed order (deterministic): wavefront shuffles, then
// the per-wavefront sums in wavefront order. lds holds one double per wavefront
// and is reused across calls; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6);
    double s = lds[0];
    for (int w = 1; w < nw; ++w) s += lds[w];
    return s;
}

// ------------------------------------------------------------ the collision --
// Quotients that must not carry a fixed relative error (a biased 1/36 or 1/rho
// would bias every collision's momentum, which a decaying flow accumulates): FP64
// divides; FP32 multiplies by the rounded reciprocal and corrects with the exact
// residual (one FMA), which returns the quotient to within a hair of correct
// rounding with no systematic direction, in 3 instructions instead of ~10.
__device__ __forceinline__ double div36(double s) { return s / 36.0; }
__device__ __forceinline__ float div36(float s)
{
    const float r = 1.0f / 36.0f;
    const float q = s * r;
    return __builtin_fmaf(__builtin_fmaf(-36.0f, q, s), r, q);
}
__device__ __forceinline__ double div12(double s) { return s / 12.0; }
__device__ __forceinline__ float div12(float s)
{
    const float r = 1.0f / 12.0f;
    const float q = s * r;
    return __builtin_fmaf(__builtin_fmaf(-12.0f, q, s), r, q);
}
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);            // ~1 ulp
    return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);  // one Newton step
}

template <typename R>
struct Pair {
    R ga, gb;
};

// Per-node terms shared by the pair collisions of a node, in weight-normalized
// units (h_a = (f_a - w_a rho0) / w_a).
template <typename R>
struct NodeTerms {
    R A;        // drho - 3/2 rho u.u : the even equilibrium without its eu^2 part
    R rho45;    // 9/2 rho
    R uF3;      // -3 u.F
};

// The momentum 3 rho u = (36 j + 18 F) / 12 of the corrected velocity, formed
// from the population moments: the odd equilibrium 3 rho e.u is taken as e.(3 rho u)
// so that it carries exactly the momentum the populations hold. Forming it as
// (3 rho)(e.u) instead rounds rho twice (in 36 rho for u and in 3 rho), and near
// rho = 1 those roundings do not average out: every collision then scales the
// momentum by a fixed ~1e-8 in FP32, which a slowly decaying flow accumulates
// into a visible error in its decay rate. j36 = 36 j + 18 F_b, fv = F_VP.
template <typename R>
__device__ __forceinline__ R momentum3(R j36, R fv)
{
    return div12(j36) + R(1.5) * fv;
}

// Collision of a population pair (a, opposite a) with eu = e_a.u, eP = e_a.(3 rho u)
// and eF = e_a.F:
//   even part  s+ + (h^eq+ - s+)/tau+ + (1 - 1/(2 tau+)) F+/w,  h^eq+ = A + 9/2 rho eu^2
//   odd part   s- + (h^eq- - s-)/tau- + (1 - 1/(2 tau-)) F-/w,  h^eq- = 3 rho eu = eP
// (F+/w = 9 eu eF - 3 u.F, F-/w = 3 eF). Relaxing as x + (y - x)/tau keeps the
// fixed point x = y exact in floating point.
template <typename R, typename Args>
__device__ __forceinline__ Pair<R> collide_pair(R ha, R hb, R eu, R eP, R eF, const NodeTerms<R>& n,
                                                const Args& a)
{
    const R sp = R(0.5) * (ha + hb);
    const R sm = R(0.5) * (ha - hb);
    const R ep = n.rho45 * (eu * eu) + n.A;
    const R em = eP;
    const R Fp = (R(9) * eu) * eF + n.uF3;
    const R Fm = R(3) * eF;
    const R gp = a.om_p * (ep - sp) + sp + a.k_p * Fp;
    const R gm = a.om_m * (em - sm) + sm + a.k_m * Fm;
    return {gp + gm, gp - gm};
}

// V elements one element off a 16-byte boundary, stored as one vector access
// that needs only dword alignment.
typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

template <typename S, int V>
__device__ __forceinline__ void store_vec_shifted(S* p, const S (&in)[V])
{
    static_assert(sizeof(S) >= 4 || V == 1, "sub-dword vectors are stored one by one");
    constexpr int B = V * (int)sizeof(S);
    if constexpr (B == 16) {
        u32x4_a4 r;
        __builtin_memcpy(&r, in, 16);
        __builtin_nontemporal_store(r, reinterpret_cast<u32x4_a4*>(p));
    } else if constexpr (B == 8) {
        u32x2_a4 r;
        __builtin_memcpy(&r, in, 8);
        __builtin_nontemporal_store(r, reinterpret_cast<u32x2_a4*>(p));
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) p[k] = in[k];
    }
}

// ------------------------------------------------------------ the record --
// One block sums one force record (see FinalizeArgs) in an order fixed by the
// data alone: the partials are dealt to FIN_LANES virtual lanes (lane v takes
// v, v + FIN_LANES, ...), each lane adds its share with eight interleaved
// accumulators (so that loads overlap), and the lanes meet in a fixed binary
// tree in LDS. Neither the block size of the launch that runs it nor the way
// steps are split over calls changes a record by one bit.
constexpr int FIN_LANES = 256;

__device__ __forceinline__ double lane_sum(const double* x, int n, int v)
{
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int k = v;
    for (; k + 7 * FIN_LANES < n; k += 8 * FIN_LANES) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += x[k + u * FIN_LANES];
    }
#pragma unroll
    for (int u = 0; u < 7; ++u) {   // at most 7 left
        const int kk = k + u * FIN_LANES;
        if (kk < n) acc[u] += x[kk];
    }
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// Sum of the FIN_LANES values in s (LDS), pairwise with halving spans; every
// thread of the block must call it and gets the sum.
__device__ __forceinline__ double tree_sum(double* s)
{
    for (int w = FIN_LANES / 2; w > 0; w >>= 1) {
        __syncthreads();
        for (int v = (int)threadIdx.x; v < w; v += (int)blockDim.x) s[v] += s[v + w];
    }
    __syncthreads();
    const double r = s[0];
    __syncthreads();   // s is reused by the next sum
    return r;
}

// Block -> tile order. Workgroups are dealt to the 8 XCDs round-robin by block
// id, and each XCD has its own L2. Counting blocks from first_block:
//  - band_log2 < 0: block b takes tile (b % 8) * per_xcd + b / 8, so each XCD
//    sweeps one contiguous eighth of the tiles;
//  - band_log2 = k >= 0: the tiles form groups of 8 bands of 2^k consecutive
//    tiles, and XCD x takes band x of every group: each XCD still sweeps runs
//    of neighbouring tiles, while the chip as a whole moves through a window of
//    8 * 2^k tiles (k = 0 is plain dispatch order). Blocks past the last whole
//    group keep dispatch order.
// Either way the map is a permutation of [0, 8 per_xcd); a block whose tile is
// past the domain's last one has nothing to do.
__device__ __forceinline__ int xcd_tile(int per_xcd, int band_log2, int first_block)
{
    const int blk = (int)blockIdx.x - first_block;   // first_block is a multiple of 8
    if (band_log2 < 0) return (blk % N_XCD_DEV) * per_xcd + blk / N_XCD_DEV;
    const int span = N_XCD_DEV << band_log2;
    if (blk >= (per_xcd >> band_log2) * span) return blk;
    const int r = blk & (span - 1);
    return (blk - r) + ((r % N_XCD_DEV) << band_log2) + r / N_XCD_DEV;
}

}  // namespace
}  // namespace lbvp
