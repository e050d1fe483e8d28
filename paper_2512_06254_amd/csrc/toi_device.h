// Device helpers shared by the kernels: deterministic block reductions and
// small numeric routines.
#pragma once

#include <hip/hip_runtime.h>

namespace toi {

// Sum over a 64-lane wavefront with a fixed butterfly order (deterministic).
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// Order LDS accesses of one wavefront that pass data between its lanes: the
// hardware executes a wave's LDS instructions in order; this keeps the
// compiler from moving them across the point.
__device__ inline void lds_order() {
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Eight FP32 values as bf16 pairs x = hi + lo: hi = bf16(x) (round to
// nearest even), lo = bf16(x - hi).  Two values are converted per
// instruction; hi is widened back to FP32 by bit shifts of the packed word
// (element 2w is the low half of word w), so the residual x - hi is exact
// (and fused into an FMA where x is a product).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
__device__ inline void split_bf16x8(const float* x, bf16x8_t& hi, bf16x8_t& lo) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    u4 h, l;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const f2 v = {x[2 * w], x[2 * w + 1]};
        const unsigned p = __builtin_bit_cast(unsigned, __builtin_convertvector(v, b2));
        const f2 r = {x[2 * w] - __uint_as_float(p << 16), x[2 * w + 1] - __uint_as_float(p & 0xffff0000u)};
        h[w] = p;
        l[w] = __builtin_bit_cast(unsigned, __builtin_convertvector(r, b2));
    }
    hi = __builtin_bit_cast(bf16x8_t, h);
    lo = __builtin_bit_cast(bf16x8_t, l);
}

// Products a_i b_i (i = 0, 1) of FP32 values as fp16 pairs a b = hi + lo:
// hi = f16(a b) and lo = f16(a b - hi), each from one fused multiply-add in
// FP32 with the result rounded to fp16 (v_fma_mixlo_f16 / v_fma_mixhi_f16
// write the low / high half of the packed word; for lo the third operand is
// the fp16 hi read from its half of the packed word).  The residual a b - hi
// is exact in the FMA, so hi + lo carries about 22 significant bits of a b
// (lo keeps 11 of the residual's).  Values must lie in fp16's range
// (|a b| < 65504).  The two instructions of each word write disjoint halves,
// so the word is fully defined.
__device__ inline void split_prod_f16x2(float a0, float b0, float a1, float b1, uint32_t& hi, uint32_t& lo) {
    uint32_t h, l;
    asm("v_fma_mixlo_f16 %0, %1, %2, 0\n\t"
        "v_fma_mixhi_f16 %0, %3, %4, 0"
        : "=&v"(h)
        : "v"(a0), "v"(b0), "v"(a1), "v"(b1));
    asm("v_fma_mixlo_f16 %0, %1, %2, -%5 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %0, %3, %4, -%5 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "=&v"(l)
        : "v"(a0), "v"(b0), "v"(a1), "v"(b1), "v"(h));
    hi = h;
    lo = l;
}
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
__device__ inline void split_prod_f16x8(const float* a, const float* b, f16x8_t& hi, f16x8_t& lo) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    u4 h, l;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t hw, lw;
        split_prod_f16x2(a[2 * w], b[2 * w], a[2 * w + 1], b[2 * w + 1], hw, lw);
        h[w] = hw;
        l[w] = lw;
    }
    hi = __builtin_bit_cast(f16x8_t, h);
    lo = __builtin_bit_cast(f16x8_t, l);
}

// Sum over a 64-lane wavefront with DPP row shifts and row broadcasts (fixed
// order); the total is returned to every lane (from lane 63).
template <int CTRL, int ROWS>
__device__ inline float dpp_add(float x) {
    return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xf, false));
}
__device__ inline float wave_total(float v) {
    v = dpp_add<0x111, 0xf>(v);   // row_shr:1
    v = dpp_add<0x112, 0xf>(v);   // row_shr:2
    v = dpp_add<0x114, 0xf>(v);   // row_shr:4
    v = dpp_add<0x118, 0xf>(v);   // row_shr:8   (lane 15 of each row: the row's sum)
    v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 (rows 1, 3)
    v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 (rows 2, 3): lane 63 holds the total
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
template <typename T>
__device__ inline T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Block reductions for blockDim.x a multiple of 64 (<= 1024); `red` holds one
// slot per wavefront.  Every thread receives the result.
template <typename T>
__device__ inline T block_sum(T v, T* red) {
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
}
template <typename T>
__device__ inline T block_max(T v, T* red) {
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    T s = red[0];
    for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
    __syncthreads();
    return s;
}
template <typename T>
__device__ inline T block_min(T v, T* red) {
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6;
    v = wave_min(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    T s = red[0];
    for (int i = 1; i < nw; ++i) s = fmin(s, red[i]);
    __syncthreads();
    return s;
}

// Sums of NV values over a block (blockDim.x a multiple of 64, <= 1024) in one
// LDS round: each wavefront reduces its values (fixed butterfly order), the
// waves' partial sums go to red[NV][16], and every thread adds them in wave
// order.  v is replaced by the block totals.
template <int NV>
__device__ inline void block_sum_n(double (&v)[NV], double (*red)[16]) {
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) red[i][w] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int j = 0; j < nw; ++j) s += red[i][j];
        v[i] = s;
    }
    __syncthreads();
}

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Hardware dispatches workgroup i to XCD i mod 8.  Remap so that each XCD
// receives a contiguous range of logical ids (neighbouring tiles share its L2).
__device__ inline int xcd_block_id(int bid, int nblk) {
    if (nblk % 8) return bid;
    return (bid & 7) * (nblk >> 3) + (bid >> 3);
}

// a / b given rb = 1 / b (correctly rounded): q = a rb, then one correction
// with the exact residual a - q b (an FMA): q + (a - q b) rb, within an ulp
// of the correctly rounded quotient (equal to it in all but rare cases), in
// three FP64 operations instead of a division sequence.
__host__ __device__ inline double div_by(double a, double b, double rb) {
    const double q = a * rb;
    return fma(fma(-q, b, a), rb, q);
}

// Exponential-of-semicircle gridding kernel on |z| <= 1 (beta = 2.30 * 8):
// exp(beta (sqrt(1 - z^2) - 1)) = 2^(beta log2(e) (sqrt(1 - z^2) - 1)), with the
// hardware square root and base-2 exponential (about 1 ulp each).
__device__ inline float es_kernel(float z) {
    constexpr float beta_log2e = 18.4f * 1.4426950408889634f;
    const float a = fmaxf(__builtin_fmaf(-z, z, 1.0f), 0.0f);
    return __builtin_amdgcn_exp2f(__builtin_fmaf(beta_log2e, __builtin_amdgcn_sqrtf(a), -beta_log2e));
}

// Kernel weights of one footprint axis at the eight cells c0 + i (i = 0..7)
// of an aligned 8-cell tile: footprint start s (cell index), offset o of the
// sample from s in (3, 4], grid side M (a power of two).  Cell c lies at
// footprint position d = (c - s) mod M (taken in [-M/2, M/2)) and gets
// psi((d - o) / 4) where |d - o| <= 4, 0 elsewhere.  The footprint cells
// d = 0..7 are exactly those, except at o = 4 exactly (or o rounded to 3),
// where one more cell lies on |z| = 1 and gets psi(1) = e^-beta (about 1e-8).
// No index test: outside |z| <= 1 the square root of 1 - z^2 < 0 is NaN,
// the exponential keeps it, and the maximum with 0 returns 0 (maxNum returns
// the operand that is not NaN).  o must be finite.
__device__ inline void tile_axis_weights(int c0, int s, float o, int M, float w[8]) {
    constexpr float beta_log2e = 18.4f * 1.4426950408889634f;
    int b = (c0 - s) & (M - 1);
    if (b >= (M >> 1)) b -= M;                      // footprint position of cell c0, signed
    const float z0 = ((float)b - o) * 0.25f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float z = z0 + 0.25f * (float)i;
        const float r = __builtin_amdgcn_sqrtf(__builtin_fmaf(-z, z, 1.0f));   // NaN outside |z| <= 1
        w[i] = fmaxf(__builtin_amdgcn_exp2f(__builtin_fmaf(beta_log2e, r, -beta_log2e)), 0.0f);
    }
}

}  // namespace toi
