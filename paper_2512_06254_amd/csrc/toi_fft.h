// Block-wide inverse FFT of length M held in LDS (Stockham auto-sort).
//
// T = M / E threads each hold E complex values in registers.  The length is
// split as M = R1 * E * ... * E (R1 <= E, all powers of two); each stage does
// E / R radix-R butterflies per thread in registers, with one LDS round trip
// between stages.  Before the first stage thread t holds elements
// t + b T + r (M / R1) (b < E / R1, r < R1) in v[b R1 + r]; after the last
// stage it holds outputs t + r T (r < E) in v[r], in natural order.  The sign
// is +i (inverse transform, un-normalised).
#pragma once

#include <hip/hip_runtime.h>

#include "toi_device.h"

namespace toi {

// e^{+2 pi i m / 32} for m < 16
__device__ constexpr float kTwCos32[16] = {
    1.0f, 9.807852804e-01f, 9.238795325e-01f, 8.314696123e-01f, 7.071067812e-01f, 5.555702330e-01f,
    3.826834324e-01f, 1.950903220e-01f, 0.0f, -1.950903220e-01f, -3.826834324e-01f, -5.555702330e-01f,
    -7.071067812e-01f, -8.314696123e-01f, -9.238795325e-01f, -9.807852804e-01f};
__device__ constexpr float kTwSin32[16] = {
    0.0f, 1.950903220e-01f, 3.826834324e-01f, 5.555702330e-01f, 7.071067812e-01f, 8.314696123e-01f,
    9.238795325e-01f, 9.807852804e-01f, 1.0f, 9.807852804e-01f, 9.238795325e-01f, 8.314696123e-01f,
    7.071067812e-01f, 5.555702330e-01f, 3.826834324e-01f, 1.950903220e-01f};

// R-point inverse DFT in registers, natural order in and out (radix-2 DIT).
template <int R>
struct Dft {
    __device__ static inline void run(float2* v) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        Dft<R / 2>::run(e);
        Dft<R / 2>::run(o);
#pragma unroll
        for (int m = 0; m < R / 2; ++m) {
            float2 t;
            if (m == 0) {
                t = o[m];
            } else if (4 * m == R) {                         // w = i
                t = make_float2(-o[m].y, o[m].x);
            } else {
                const float2 w = make_float2(kTwCos32[m * (32 / R)], kTwSin32[m * (32 / R)]);
                t = cmul(w, o[m]);
            }
            v[m] = cadd(e[m], t);
            v[m + R / 2] = csub(e[m], t);
        }
    }
};
template <>
struct Dft<1> {
    __device__ static inline void run(float2*) {}
};
template <>
struct Dft<2> {
    __device__ static inline void run(float2* v) {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

__host__ __device__ constexpr int fft_first_radix(int M, int E) {
    int r = M;
    while (r > E) r /= E;
    return r;
}
__host__ __device__ constexpr int fft_radix_at(int M, int E, int NS) {
    return NS == 1 ? fft_first_radix(M, E) : E;
}

// Twiddles in LDS, one table per stage after the first: the stage with
// stride NS (radix E) multiplies element r of the butterfly of k = j mod NS by
// e^{+2 pi i r k / (NS E)}, kept at k (E - 1) + r - 1.  Consecutive lanes then
// read addresses E - 1 values apart, which spreads them over the banks (a
// single M-entry table read at r k M / (NS E) puts up to 16 lanes in one
// bank).  The tables hold about M entries in total.  In HBM the twiddle
// buffer holds the full-period table e^{+2 pi i n / M} (n < M) followed by
// the stage tables of radix 8, 16 and 32 in this order (built on the host),
// so that a workgroup fills its LDS tables with a plain copy.
__host__ __device__ constexpr int fft_stage_table_size(int M, int E) {
    int o = 0;
    for (int ns = fft_first_radix(M, E); ns < M; ns *= E) o += ns * (E - 1);
    return o;
}
__host__ __device__ constexpr int fft_stage_table_offset(int M, int E) {   // E in {8, 16, 32}; 64: the end
    int o = M;
    for (int e = 8; e < E; e *= 2) o += fft_stage_table_size(M, e);
    return o;
}
__host__ __device__ constexpr int fft_twiddle_entries(int M) { return fft_stage_table_offset(M, 64); }

template <int M, int E>
struct FftTw {
    static constexpr int R1 = fft_first_radix(M, E);
    static constexpr int off(int NS) {   // start of the table of the stage with stride NS (> 1)
        int o = 0;
        for (int ns = R1; ns < NS; ns *= E) o += ns * (E - 1);
        return o;
    }
    static constexpr int size() { return off(M); }
};

// Fill the stage tables in LDS from the twiddle buffer (all threads; ends with
// a barrier).  Offsets and sizes are even: 16-byte reads.
template <int M, int E>
__device__ inline void load_twiddles(float2* tw_s, const float2* __restrict__ tw) {
    static_assert(E == 8 || E == 16 || E == 32, "stage tables exist for radix 8, 16 and 32");
    constexpr int S = FftTw<M, E>::size();
    static_assert(S == fft_stage_table_size(M, E) && S % 2 == 0 && fft_stage_table_offset(M, E) % 2 == 0, "");
    const float4* src = reinterpret_cast<const float4*>(tw + fft_stage_table_offset(M, E));
    for (int i = threadIdx.x; i < S / 2; i += blockDim.x) {
        const float4 a = src[i];
        tw_s[2 * i] = make_float2(a.x, a.y);
        tw_s[2 * i + 1] = make_float2(a.z, a.w);
    }
    __syncthreads();
}

template <int M, int E, int R, int NS>
__device__ inline void fft_stage_regs(float2* v, const float2* tw) {
    constexpr int T = M / E;
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        if constexpr (NS > 1) {
            static_assert(R == E, "every stage after the first has radix E");
            const int j = threadIdx.x + b * T;
            const float2* w = tw + FftTw<M, E>::off(NS) + (j & (NS - 1)) * (E - 1) - 1;
#pragma unroll
            for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], w[r]);
        }
        Dft<R>::run(v + b * R);
    }
}

// Exchange buffer of the stages: M values with one pad slot after every E
// (index i at i + i / E), so that the stride-E writes of a stage fall in
// different banks.  Where a stage's offsets r NS (r M / R2 for the reads) are
// multiples of E, or the base is and r NS < E, the padded address is the
// padded base plus a compile-time offset.
template <int M, int E>
__host__ __device__ constexpr int fft_lds_size() {
    return M + M / E;
}
template <int E>
__device__ inline int fft_pad(int i) {
    return i + i / E;
}
template <int E>
__host__ __device__ constexpr int fft_pad_off(int d) {   // padded offset d (a multiple of E, or below E)
    return d + d / E;
}

template <int M, int E, int NS>
__device__ inline void fft_stages(float2* v, float2* lds, const float2* tw) {
    constexpr int T = M / E;
    constexpr int R = fft_radix_at(M, E, NS);
    fft_stage_regs<M, E, R, NS>(v, tw);
    if constexpr (NS * R < M) {
        constexpr int R2 = fft_radix_at(M, E, NS * R);
        // the base of a write is a multiple of E when NS = 1 and R = E, and the
        // offsets r NS are multiples of E when NS >= E; otherwise pad each
        constexpr bool split_w = (NS >= E && NS % E == 0) || (NS == 1 && R == E);
        constexpr bool split_r = (M / R2) % E == 0;
        __syncthreads();
#pragma unroll
        for (int b = 0; b < E / R; ++b) {
            const int j = threadIdx.x + b * T;
            const int base = (j / NS) * NS * R + (j & (NS - 1));
            if constexpr (split_w) {
                float2* dst = lds + fft_pad<E>(base);
#pragma unroll
                for (int r = 0; r < R; ++r) dst[fft_pad_off<E>(r * NS)] = v[b * R + r];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) lds[fft_pad<E>(base + r * NS)] = v[b * R + r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < E / R2; ++b) {
            const int j = threadIdx.x + b * T;
            if constexpr (split_r) {
                const float2* src = lds + fft_pad<E>(j);
#pragma unroll
                for (int r = 0; r < R2; ++r) v[b * R2 + r] = src[fft_pad_off<E>(r * (M / R2))];
            } else {
#pragma unroll
                for (int r = 0; r < R2; ++r) v[b * R2 + r] = lds[fft_pad<E>(j + r * (M / R2))];
            }
        }
        fft_stages<M, E, NS * R>(v, lds, tw);
    }
}

// Load the stage-1 pattern of one length-M row starting at src.
template <int M, int E>
__device__ inline void fft_load(float2* v, const float2* __restrict__ src) {
    constexpr int T = M / E;
    constexpr int R1 = fft_first_radix(M, E);
#pragma unroll
    for (int b = 0; b < E / R1; ++b)
#pragma unroll
        for (int r = 0; r < R1; ++r) v[b * R1 + r] = src[threadIdx.x + b * T + r * (M / R1)];
}

// As fft_load, with elements whose index fails pred(i) read as zero (not
// loaded); element i of the sequence is src[i S].
template <int M, int E, int S = 1, typename Pred>
__device__ inline void fft_load_masked(float2* v, const float2* __restrict__ src, Pred pred) {
    constexpr int T = M / E;
    constexpr int R1 = fft_first_radix(M, E);
#pragma unroll
    for (int b = 0; b < E / R1; ++b)
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int i = threadIdx.x + b * T + r * (M / R1);
            v[b * R1 + r] = pred(i) ? src[(size_t)i * S] : make_float2(0.f, 0.f);
        }
}

// Bit e (element e of the stage-1 pattern) set where pred holds for the
// element's index: the occupancy of this thread's elements, computed once for
// rows or columns that share it.
template <int M, int E, typename Pred>
__device__ inline uint32_t fft_element_bits(Pred pred) {
    constexpr int T = M / E;
    constexpr int R1 = fft_first_radix(M, E);
    static_assert(E <= 32, "one bit per element");
    uint32_t bits = 0;
#pragma unroll
    for (int b = 0; b < E / R1; ++b)
#pragma unroll
        for (int r = 0; r < R1; ++r)
            if (pred(threadIdx.x + b * T + r * (M / R1))) bits |= 1u << (b * R1 + r);
    return bits;
}

// As fft_load, with the elements whose bit is clear read as zero (not
// loaded); element i of the sequence is src[i S].
template <int M, int E, int S = 1>
__device__ inline void fft_load_bits(float2* v, const float2* __restrict__ src, uint32_t bits) {
    constexpr int T = M / E;
    constexpr int R1 = fft_first_radix(M, E);
#pragma unroll
    for (int b = 0; b < E / R1; ++b)
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int e = b * R1 + r;
            v[e] = ((bits >> e) & 1u) ? src[(size_t)(threadIdx.x + b * T + r * (M / R1)) * S] : make_float2(0.f, 0.f);
        }
}

// Output slot r (0 <= r < E) of thread t is bin k = t + r T.  With M = 2N the
// kept bins are a = k (k < N/2) and a = k - M (k >= M - N/2), a in [-N/2, N/2),
// i.e. the slots r < E/4 and r >= 3E/4.
template <int E>
__device__ constexpr int fft_kept_slot(int q) {  // q < E/2 -> slot r
    return q < E / 4 ? q : q + E / 2;
}

// Image index j = a + N/2 of kept slot q for thread t.
template <int M, int E>
__device__ inline int fft_kept_index(int q) {
    constexpr int T = M / E;
    const int r = fft_kept_slot<E>(q);
    const int k = threadIdx.x + r * T;
    return (k < M / 4) ? k + M / 4 : k - M + M / 4;
}

}  // namespace toi
