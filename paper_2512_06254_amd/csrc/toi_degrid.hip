// S10: adjoint of toi_grid + toi_image for the snapshot last gridded.
//
// The imaging map x -> I is real-linear; under <I, y> = sum I y and
// <x, z> = Re sum conj(z) x its adjoint is applied step by step in reverse:
//   1. re-projection transpose: each output pixel's gradient is scattered with
//      its bilinear weights onto the transformed plane;
//   2. column pass: per image column and plane, the pixel gradients times
//      conj(c_k(alpha) e^{i 2 pi r3p t3}) times the grid correction and
//      1/(omega W) are placed at their FFT bins and transformed with e^{-i}
//      (as conj(F^{-1}(conj(.))) with the inverse FFT);
//   3. row pass: the same along x, giving the gradient of every grid plane in
//      the rows that hold samples;
//   4. degridding: each sample gathers the kernel-weighted plane gradients of
//      its 8 x 8 footprint and sums them with T_k(s) (Romein-style walk);
//   5. visibilities: grad V_k = conj(g_a1 conj(g_a2)) W_k (1 - F_k) grad x;
//      gains: per work item sum_c conj(y_c) grad x_c (y = pre-gain weighted
//      sum), reduced per antenna in FP64 in a fixed order.
// The two scatter steps (1 and 4) add into their targets with 64-bit integer
// atomics on fixed-point values: each sum gets a power-of-two scale from the
// largest magnitude that can reach it (the image gradient's for step 1, the
// plane gradients' for step 4, both measured on the device), so that no sum
// exceeds 2^61, and integer addition makes the result independent of the
// order in which the waves arrive: the gradients are bitwise repeatable.
// The resolution is 2^-51 of the bound, far below FP32 rounding.
// The grid and row-pass workspaces are reused, so toi_grid must run again
// before the next toi_image.
#include <algorithm>

#include "toi_fft.h"
#include "toi_grid.h"
#include "toi_internal.h"

namespace toi {


__global__ __launch_bounds__(256) void k_zero_f32(float* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// Fixed-point sums: value v adds rint(v S) to a 64-bit integer; S = 2^(61 - e)
// where the bound b (largest magnitude times the most terms that can meet in
// one sum) is f 2^e, f in [0.5, 1), so every sum stays below 2^61.
__device__ inline unsigned long long to_fixed(float v, double S) {
    return (unsigned long long)(long long)rint((double)v * S);
}
__device__ inline float from_fixed(unsigned long long q, double inv_S) {
    return (float)((double)(long long)q * inv_S);
}
// Per-workgroup largest |x| of n floats (parts[blockIdx.x]).
__global__ __launch_bounds__(256) void k_absmax_parts(const float* __restrict__ x, size_t n, float* __restrict__ parts) {
    __shared__ float red[4];
    float m = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(x[i]));
    m = block_max(m, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = m;
}
// scale[0] = S, scale[1] = 1 / S for the bound mult * max(parts).
__global__ __launch_bounds__(1024) void k_fixed_scale(const float* __restrict__ parts, int n, double mult,
                                                     double* __restrict__ scale) {
    __shared__ float red[16];
    float m = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, parts[i]);
    m = block_max(m, red);
    if (threadIdx.x == 0) {
        int e = 0;
        if (m > 0.f) (void)frexp((double)m * mult, &e);
        e = max(-900, min(900, e));
        scale[0] = ldexp(1.0, 61 - e);
        scale[1] = ldexp(1.0, e - 61);
    }
}
// Most output pixels whose bilinear stencils can meet in one transformed-plane
// pixel, and most (tile, order) terms of one sample's gradient (4 tiles x 64
// cells x 32 orders), as bounds of the fixed-point sums (generous: the
// resolution stays far below FP32 rounding).
constexpr double kRaMaxTerms = 1024.0, kDegridMaxTerms = 8192.0;

// 1. transpose of the bilinear re-projection (t-plane gradient, j1-major).
// A workgroup takes 16 x 16 output pixels; their bilinear sources cover a
// small box of the t-plane, which is accumulated in LDS and then added to HBM
// once (about 1.3 global atomics per output pixel instead of 4).  A box larger
// than kRaBox x kRaBox (an extreme stretch of the map) falls back to direct
// global atomics.
constexpr int kRaTile = 16, kRaBox = 48;
__global__ __launch_bounds__(256) void k_reproject_adj(const float* __restrict__ gimg,
                                                       unsigned long long* __restrict__ gtp,
                                                       const DevPlan* __restrict__ plan, int N, double cell_rad,
                                                       const double* __restrict__ scale) {
    __shared__ unsigned long long box[kRaBox * kRaBox];
    __shared__ int red[4][4];
    if (plan->status & kStatusFatal) return;
    const double S = scale[0];
    const int j1 = blockIdx.x * kRaTile + (threadIdx.x & (kRaTile - 1));
    const int j2 = blockIdx.y * kRaTile + (threadIdx.x / kRaTile);
    int i1 = 0, i2 = 0;
    float f1 = 0.f, f2 = 0.f, y = 0.f;
    bool ok = j1 < N && j2 < N && reproject_source(plan, N, cell_rad, j1, j2, i1, i2, f1, f2);
    if (ok) y = gimg[(size_t)j2 * N + j1];
    ok = ok && y != 0.f;
    // bounding box of the sources (i1, i2) .. (i1 + 1, i2 + 1)
    int lo1 = ok ? i1 : 0x7fffffff, lo2 = ok ? i2 : 0x7fffffff, hi1 = ok ? i1 : -1, hi2 = ok ? i2 : -1;
    lo1 = wave_min(lo1); lo2 = wave_min(lo2); hi1 = wave_max(hi1); hi2 = wave_max(hi2);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[w][0] = lo1; red[w][1] = lo2; red[w][2] = hi1; red[w][3] = hi2; }
    __syncthreads();
    for (int k = 0; k < 4; ++k) {
        lo1 = min(lo1, red[k][0]); lo2 = min(lo2, red[k][1]);
        hi1 = max(hi1, red[k][2]); hi2 = max(hi2, red[k][3]);
    }
    if (hi1 < 0) return;                                   // no contribution (uniform)
    const int w1 = hi1 - lo1 + 2, w2 = hi2 - lo2 + 2;       // box extent in i1, i2
    const float a00 = (1.f - f1) * (1.f - f2) * y, a10 = f1 * (1.f - f2) * y;
    const float a01 = (1.f - f1) * f2 * y, a11 = f1 * f2 * y;
    if (w1 > kRaBox || w2 > kRaBox) {                       // uniform fallback
        if (ok) {
            unsigned long long* c0 = gtp + (size_t)i1 * N + i2;
            unsigned long long* c1 = c0 + N;
            atomicAdd(c0, to_fixed(a00, S));
            atomicAdd(c1, to_fixed(a10, S));
            atomicAdd(c0 + 1, to_fixed(a01, S));
            atomicAdd(c1 + 1, to_fixed(a11, S));
        }
        return;
    }
    for (int e = threadIdx.x; e < w1 * kRaBox; e += blockDim.x) box[e] = 0ull;
    __syncthreads();
    if (ok) {
        unsigned long long* b0 = box + (i1 - lo1) * kRaBox + (i2 - lo2);
        atomicAdd(b0, to_fixed(a00, S));
        atomicAdd(b0 + kRaBox, to_fixed(a10, S));
        atomicAdd(b0 + 1, to_fixed(a01, S));
        atomicAdd(b0 + kRaBox + 1, to_fixed(a11, S));
    }
    __syncthreads();
    for (int e = threadIdx.x; e < w1 * w2; e += blockDim.x) {
        const int d1 = e / w2, d2 = e % w2;
        const unsigned long long v = box[d1 * kRaBox + d2];
        if (v != 0ull) atomicAdd(gtp + (size_t)(lo1 + d1) * N + lo2 + d2, v);
    }
}

// Miller backward recurrence for J_n(alpha) in FP64 from a per-pixel start
// order (no rescaling needed for |alpha| >= 1e-3 and start <= 76).
__device__ inline int miller_start(int K, double alpha) { return 2 * ((K + 14 + (int)ceil(1.5 * fabs(alpha))) / 2); }

__device__ inline double miller_norm(double alpha, int L) {
    double jp1 = 0.0, j = 1e-100, nrm = 0.0;
    const double ia = 1.0 / alpha;
    for (int n = L; n >= 0; --n) {
        if ((n & 1) == 0) nrm += (n == 0 ? 1.0 : 2.0) * j;
        const double jm1 = 2.0 * n * ia * j - jp1;
        jp1 = j;
        j = jm1;
    }
    return nrm;
}

// 2. column pass of the adjoint
// Launch bounds: workgroups of 512 threads (4096-point columns at radix 8)
// are held to 128 VGPRs, so that two fit on a CU (4 waves per SIMD); the
// 20 registers this spills cost less than the halved occupancy (adjoint leg
// at the 2048^2 / 1024-channel shape 1.64 -> 1.49 ms).
template <int M, int E>
__global__ __launch_bounds__(M / E, (M / E) == 512 ? 4 : (M / E) <= 256 ? 2 : 1) void k_adj_cols(const unsigned long long* __restrict__ gtp,
                                                       float2* __restrict__ gh,
                                                       const float2* __restrict__ tw, const float* __restrict__ corr,
                                                       const DevPlan* __restrict__ plan, float cell_rad, int mode,
                                                       const uint32_t* __restrict__ row_bits,
                                                       const double* __restrict__ scale) {
    constexpr int N = M / 2;
    constexpr int KEEP = E / 2;
    constexpr int T = M / E;
    constexpr int NT = M / kTile, WORDS = (NT + 31) / 32;
    __shared__ float2 lds[fft_lds_size<M, E>()];
    __shared__ float2 tw_s[FftTw<M, E>::size()];
    const int j1 = xcd_block_id(blockIdx.x, gridDim.x);
    if (plan->status & kStatusFatal) return;
    load_twiddles<M, E>(tw_s, tw);
    const int K = plan->K, ns = plan->n_slab;
    int j2[KEEP];
    float y[KEEP];
    const float c1 = corr[j1] * (float)plan->norm;
    const double inv_S = scale[1];
#pragma unroll
    for (int q = 0; q < KEEP; ++q) {
        j2[q] = fft_kept_index<M, E>(q);
        y[q] = from_fixed(gtp[(size_t)j1 * N + j2[q]], inv_S) * c1 * corr[j2[q]];
    }
    // per-pixel geometry (FP64 here: the adjoint runs once per backward pass)
    // ia: 1 / alpha (0 where |alpha| < 1e-3: the power series, from af = alpha);
    // inrm: 1 / Miller normalisation
    double t3[KEEP], ia[KEEP], inrm[KEEP], jp1[KEEP], jc[KEEP];
    float af[KEEP];
    int Lq[KEEP];
    if (mode == 3) {
        const double V13 = plan->V[2], V23 = plan->V[5], V33 = plan->V[8];
        const double sg = V33 >= 0 ? 1.0 : -1.0;
        const double t1 = -(double)cell_rad * (j1 - N / 2);
#pragma unroll
        for (int q = 0; q < KEEP; ++q) {
            const double t2 = (double)cell_rad * (j2[q] - N / 2);
            const double a = 1.0 - (t1 + V13) * (t1 + V13) - (t2 + V23) * (t2 + V23);
            if (a < 0) y[q] = 0.f;
            const double num = t1 * t1 + t2 * t2 + 2.0 * t1 * V13 + 2.0 * t2 * V23;
            t3[q] = a >= 0 ? -sg * num / (sqrt(fmax(a, 0.0)) + fabs(V33)) : 0.0;
            const double al = 2.0 * kPi * plan->dr3 * t3[q];
            const bool series = fabs(al) < 1e-3;
            af[q] = (float)al;
            ia[q] = series ? 0.0 : 1.0 / al;
            Lq[q] = miller_start(K, al);
            inrm[q] = series ? 1.0 : 1.0 / miller_norm(al, Lq[q]);
        }
    }
    int wg = -1;              // plane group whose row mask is in wbits
    uint32_t wbits = 0;
    for (int p = 0; p < ns; ++p) {
        float cs[KEEP], sn[KEEP];
        if (mode == 3) {
            const double r3p = plan->r3min + (2 * p + 1) * plan->dr3;
#pragma unroll
            for (int q = 0; q < KEEP; ++q) {
                double ph = 2.0 * kPi * r3p * t3[q];
                ph -= 2.0 * kPi * rint(ph / (2.0 * kPi));
                sincosf((float)ph, &sn[q], &cs[q]);
                // Miller state at order K (recurrence only above)
                jp1[q] = 0.0;
                jc[q] = 1e-100;
                if (ia[q] != 0.0) {
                    for (int n = Lq[q]; n >= K; --n) {
                        const double jm1 = 2.0 * n * ia[q] * jc[q] - jp1[q];
                        jp1[q] = jc[q];
                        jc[q] = jm1;
                    }
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < KEEP; ++q) { cs[q] = 1.f; sn[q] = 0.f; }
        }
        for (int k = K - 1; k >= 0; --k) {
            // gF = y conj(c_k) e^{-i 2 pi r3p t3}, placed at its bin (conjugated for the inverse-FFT trick)
            float2 v[E];
#pragma unroll
            for (int r = 0; r < E; ++r) v[r] = make_float2(0.f, 0.f);
#pragma unroll
            for (int q = 0; q < KEEP; ++q) {
                float jk = 1.f;
                if (mode == 3) {
                    const double a = af[q];
                    double J;
                    if (ia[q] == 0.0) {
                        J = k == 0 ? 1.0 - 0.25 * a * a
                          : k == 1 ? 0.5 * a * (1.0 - 0.125 * a * a)
                          : k == 2 ? 0.125 * a * a
                          : k == 3 ? a * a * a / 48.0 : 0.0;
                    } else {
                        J = jc[q] * inrm[q];
                        if (k > 0) {   // the recurrence of the prologue, 2 n / alpha from 1 / alpha
                            const double jm1 = 2.0 * k * ia[q] * jc[q] - jp1[q];
                            jp1[q] = jc[q];
                            jc[q] = jm1;
                        }
                    }
                    jk = (float)J * (k == 0 ? 1.f : 2.f);
                }
                // conj(c_k) = jk * conj(i^k); times e^{-i phi}; conj of the whole for the FFT trick:
                // conj(y jk conj(i^k) e^{-i phi}) = y jk i^k e^{i phi}
                float2 e = make_float2(y[q] * jk * cs[q], y[q] * jk * sn[q]);
                switch (k & 3) {
                    case 1: e = make_float2(-e.y, e.x); break;
                    case 2: e = make_float2(-e.x, -e.y); break;
                    case 3: e = make_float2(e.y, -e.x); break;
                    default: break;
                }
                v[fft_kept_slot<E>(q)] = e;
            }
            // natural-order scatter, then the stage-1 pattern (the same
            // pattern when the first radix is E: nothing to move)
            constexpr int R1 = fft_first_radix(M, E);
            if constexpr (R1 != E) {
                __syncthreads();
#pragma unroll
                for (int r = 0; r < E; ++r) lds[threadIdx.x + r * T] = v[r];
                __syncthreads();
#pragma unroll
                for (int b = 0; b < E / R1; ++b)
#pragma unroll
                    for (int r = 0; r < R1; ++r) v[b * R1 + r] = lds[threadIdx.x + b * T + r * (M / R1)];
            }
            fft_stages<M, E, 1>(v, lds, tw_s);
            // output element r is row y = t + r T: written only in tile rows
            // that hold samples (the row pass reads no others)
            const int gk = group_of_plane(p * K + k, plan);
            if (gk != wg) {
                wbits = 0;
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int yy = threadIdx.x + r * T;
                    if ((row_bits[gk * WORDS + (yy >> (kTileShift + 5))] >> ((yy >> kTileShift) & 31)) & 1u)
                        wbits |= 1u << r;
                }
                wg = gk;
            }
            float2* dst = gh + ((size_t)(p * K + k) * N + j1) * M;
#pragma unroll
            for (int r = 0; r < E; ++r)
                if ((wbits >> r) & 1u) dst[threadIdx.x + r * T] = make_float2(v[r].x, -v[r].y);
        }
    }
}

// 3. row pass of the adjoint (rows of tile rows that hold samples; only the
// tiles that hold samples are written, the only ones the gather reads)
// Each workgroup also records the largest magnitude it writes in
// gmax_parts[blockIdx.x] (0 when it writes nothing), for the degridder's
// fixed-point scale.
template <int M, int E, int B>
__global__ __launch_bounds__(M / E, (M / E) <= 256 ? 2 : 1) void k_adj_rows(const float2* __restrict__ gh, float2* __restrict__ gg,
                                                       const float2* __restrict__ tw,
                                                       const DevPlan* __restrict__ plan, int nbands,
                                                       const uint32_t* __restrict__ tile_bits,
                                                       const uint32_t* __restrict__ row_bits,
                                                       float* __restrict__ gmax_parts) {
    constexpr int N = M / 2;
    constexpr int KEEP = E / 2;
    constexpr int T = M / E;
    constexpr int NT = M / kTile, WORDS = (NT + 31) / 32;
    __shared__ float2 lds[fft_lds_size<M, E>()];
    __shared__ float2 tw_s[FftTw<M, E>::size()];
    __shared__ uint32_t tb[WORDS];
    __shared__ float red[16];
    const int id = xcd_block_id(blockIdx.x, gridDim.x);
    const int plane = id / nbands, band = id % nbands;
    if ((plan->status & kStatusFatal) || plane >= plan->planes) {
        if (threadIdx.x == 0) gmax_parts[blockIdx.x] = 0.f;
        return;
    }
    const int g = group_of_plane(plane, plan);
    const int ty = (band * B) / kTile;
    if (!((row_bits[g * WORDS + (ty >> 5)] >> (ty & 31)) & 1u)) {
        if (threadIdx.x == 0) gmax_parts[blockIdx.x] = 0.f;
        return;
    }
    if (threadIdx.x < WORDS) tb[threadIdx.x] = tile_bits[((size_t)g * NT + ty) * WORDS + threadIdx.x];
    load_twiddles<M, E>(tw_s, tw);   // its barrier also publishes tb
    // output element r of this thread is column x = t + r T: written only
    // where its tile holds samples (the band's rows share one tile row)
    static_assert(kTile % B == 0, "a band within one tile row");
    uint32_t wbits = 0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = threadIdx.x + r * T;
        if ((tb[x >> (kTileShift + 5)] >> ((x >> kTileShift) & 31)) & 1u) wbits |= 1u << r;
    }
    float vmax = 0.f;
    float2 in[B][KEEP];
#pragma unroll
    for (int q = 0; q < KEEP; ++q) {
        const float2* src = gh + ((size_t)plane * N + fft_kept_index<M, E>(q)) * M + band * B;
#pragma unroll
        for (int rb = 0; rb < B; ++rb) in[rb][q] = src[rb];
    }
#pragma unroll
    for (int rb = 0; rb < B; ++rb) {
        float2 v[E];
#pragma unroll
        for (int r = 0; r < E; ++r) v[r] = make_float2(0.f, 0.f);
#pragma unroll
        for (int q = 0; q < KEEP; ++q) v[fft_kept_slot<E>(q)] = make_float2(in[rb][q].x, -in[rb][q].y);
        // natural order to the stage-1 pattern (the same pattern when the
        // first radix is E: nothing to move)
        constexpr int R1 = fft_first_radix(M, E);
        if constexpr (R1 != E) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < E; ++r) lds[threadIdx.x + r * T] = v[r];
            __syncthreads();
#pragma unroll
            for (int b = 0; b < E / R1; ++b)
#pragma unroll
                for (int r = 0; r < R1; ++r) v[b * R1 + r] = lds[threadIdx.x + b * T + r * (M / R1)];
        }
        fft_stages<M, E, 1>(v, lds, tw_s);
        float2* dst = gg + ((size_t)plane * M + band * B + rb) * M;
#pragma unroll
        for (int r = 0; r < E; ++r)
            if ((wbits >> r) & 1u) {
                dst[threadIdx.x + r * T] = make_float2(v[r].x, -v[r].y);
                vmax = fmaxf(vmax, fmaxf(fabsf(v[r].x), fabsf(v[r].y)));
            }
    }
    vmax = block_max(vmax, red);
    if (threadIdx.x == 0) gmax_parts[blockIdx.x] = vmax;
}

// 4. Gather degridding on the matrix cores, the transpose of the tile
// gridder, over the forward's bins and gridding records (toi_grid of the same
// snapshot).  One wavefront per 8 x 8 tile holds the tile's plane gradients G
// (64 cells x 32 columns: the group's orders x Re/Im) as A operands of
// v_mfma_f32_32x32x16_f16, split as G sc = Gh + Gl in fp16 (sc a power of two
// that puts the largest plane gradient below 2^13; chunk c covers cells
// 16 c .. 16 c + 15, lane l holds G[16 c + 8 (l / 32) + e][l mod 32],
// e = 0..7).  The samples an item has in the tile are compacted into LDS
// (weights at the tile's 8 columns and 8 rows, T_k(s)); per batch of 32 of
// them the B operands are the weights W[cell][q] (sample q from lane
// q mod 32, products split the same way) and H^T = G^T W = sum over the
// chunks of Gh Wh + Gh Wl + Gl Wh, so that lane l holds sample q = l mod 32
// in all its registers (rows, i.e. columns of G: (r mod 4) + 8 (r / 4) +
// 4 (l / 32), hardware layout).  Then grad x_q += sum_k T_k(s_q)
// (H[q][k, Re] + i H[q][k, Im]): each lane sums its 8 orders in registers, one
// exchange with lane l xor 32 adds the other 8, and the lane adds the result
// to the sample's gradient (fixed-point 64-bit atomics: a sample meets 3.5
// tiles on average).
__global__ __launch_bounds__(64) void k_degrid_tiles(const SampleRec* __restrict__ recs, int n_chan,
                                                     const DevPlan* __restrict__ P, int M, int NT,
                                                     const int32_t* __restrict__ bin_off,
                                                     const int32_t* __restrict__ list, int bin_cap,
                                                     const int32_t* __restrict__ order,
                                                     const int32_t* __restrict__ cnt,
                                                     const int4* __restrict__ units,
                                                     const float2* __restrict__ gg,
                                                     unsigned long long* __restrict__ gx,
                                                     const double* __restrict__ scale) {
    typedef float v16 __attribute__((ext_vector_type(16)));
    __shared__ float sw[64 * 16];      // compacted samples: weights at tile columns 0..7, rows 0..7
    __shared__ float sT[64 * 16];      // T_{k0 + k}(s), zero for k >= nk
    __shared__ int sidx[64];           // sample index r * n_chan + c
    const int tiles = NT * NT;
    const int lane = threadIdx.x;
    if (P->status & kStatusFatal) return;
    const int n_chunks = (n_chan + kItemChans - 1) / kItemChans;
    const int col = lane & 31, pl = col & 15, half = lane >> 5;
    // fp16 scale of the plane gradients: scale[1] = 2^(e - 61) with 2^e above
    // 8192 times their largest magnitude, so sc = 2^(26 - e) keeps G sc below
    // 2^13; the sums are scaled back inside the fixed-point conversion
    int e_g;
    (void)frexp(scale[1], &e_g);
    e_g += 60;                                          // scale[1] = 0.5 2^(e - 60)
    const float sc = ldexpf(1.f, max(-100, min(100, 26 - e_g)));
    const double S = scale[0] / (double)sc;
    // the forward's work units (heavy bins split), heaviest first; normally
    // one per workgroup, handed out by the dispatcher as waves finish
    const int n_units = work_unit_count(cnt);
    for (int ob = blockIdx.x; ob < n_units; ob += gridDim.x) {
        const WorkUnit un = work_unit(ob, units, order, cnt);
        const int bid = un.bin;
        const int g = bid / tiles, tile = bid % tiles;
        if (g >= P->ng) continue;
        int b0, b1;
        work_unit_items(un, bin_off, bin_cap, P->unit_shift, b0, b1);
        if (b1 <= b0) continue;
        int s0, s1, k0, k1;
        group_range(g, P, s0, s1, k0, k1);   // one slab per group
        const int nk = k1 - k0;
        const int tx = tile % NT, ty = tile / NT;
        // the tile's plane gradients as A operands, split into fp16 hi + lo:
        // chunk c covers cells 16 c .. 16 c + 15, lane l elements e = 0..7 are
        // cells 16 c + 8 (l / 32) + e, i.e. tile row 2 c + l / 32, column e
        f16x8_t gh[4], gl[4];
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
            float v[8], scv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                v[e] = 0.f;
                scv[e] = sc;
                if (pl < nk) {
                    const float2 gv = gg[((size_t)(s0 * P->K + k0 + pl) * M + ty * kTile + 2 * c4 + half) * M +
                                         tx * kTile + e];
                    v[e] = col < 16 ? gv.x : gv.y;
                }
            }
            split_prod_f16x8(v, scv, gh[c4], gl[c4]);
        }
        for (int it = b0; it < b1; ++it) {
            const int item = list[it];
            const int c = (item % n_chunks) * kItemChans + lane;
            bool act = false;
            int sample = 0;
            float4 ra = make_float4(0.f, 0.f, 4.f, 4.f), rb = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < n_chan) {
                sample = (item / n_chunks) * n_chan + c;
                const float4* src = reinterpret_cast<const float4*>(recs + sample);
                ra = src[0];
                rb = src[1];
                const int pk = __float_as_int(ra.x), sp = __float_as_int(ra.y);
                const int ddx = ((pk & 8191) - tx * kTile) & (M - 1), ddy = (((pk >> 13) & 8191) - ty * kTile) & (M - 1);
                act = pk >= 0 && sp >= s0 && sp < s1 && (ddx < kTile || ddx >= M - 7) && (ddy < kTile || ddy >= M - 7);
            }
            const uint64_t m = __ballot(act);
            if (m == 0) continue;
            const int n_act = __popcll(m);
            if (act) {   // compact: slot = number of active lanes below this one
                const int slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                const int pk = __float_as_int(ra.x);
                const int ix = pk & 8191, iy = (pk >> 13) & 8191;
                float wxy[16];
                tile_axis_weights(tx * kTile, ix, ra.z, M, wxy);
                tile_axis_weights(ty * kTile, iy, ra.w, M, wxy + 8);
                float4* dw = reinterpret_cast<float4*>(sw + slot * 16);
#pragma unroll
                for (int h = 0; h < 4; ++h) dw[h] = make_float4(wxy[4 * h], wxy[4 * h + 1], wxy[4 * h + 2], wxy[4 * h + 3]);
                float4* dt = reinterpret_cast<float4*>(sT + slot * 16);
                float t, tm1;
                cheb_start(rb.x, k0, t, tm1);
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    float t4[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        t4[j] = 4 * k4 + j < nk ? t : 0.f;
                        const float tn = 2.f * rb.x * t - tm1;
                        tm1 = t;
                        t = tn;
                    }
                    dt[k4] = make_float4(t4[0], t4[1], t4[2], t4[3]);
                }
                sidx[slot] = sample;
            }
            lds_order();                                   // staging writes precede the reads below
            for (int b = 0; b < n_act; b += 32) {
                const int qa = b + col;                     // this lane's A row (sample slot)
                const bool oka = qa < n_act;
                const float4* wq = reinterpret_cast<const float4*>(sw + (oka ? qa : 0) * 16);
                const float4 x0 = wq[0], x1 = wq[1], y0 = wq[2], y1 = wq[3];
                const float wx[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                const float wy[8] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w};
                v16 h = {};
#pragma unroll
                for (int c4 = 0; c4 < 4; ++c4) {            // W[cell][q] = w_x(column e) w_y(row 2 c + half)
                    float wr8[8];
                    const float wr = oka ? wy[2 * c4 + half] : 0.f;
#pragma unroll
                    for (int e = 0; e < 8; ++e) wr8[e] = wr;
                    f16x8_t ah, al;
                    split_prod_f16x8(wx, wr8, ah, al);
                    h = __builtin_amdgcn_mfma_f32_32x32x16_f16(gl[c4], ah, h, 0, 0, 0);
                    h = __builtin_amdgcn_mfma_f32_32x32x16_f16(gh[c4], al, h, 0, 0, 0);
                    h = __builtin_amdgcn_mfma_f32_32x32x16_f16(gh[c4], ah, h, 0, 0, 0);
                }
                // this lane's orders 4 half + 0..3 and 8 + 4 half + 0..3 of sample qa:
                // registers r (Re) and r + 8 (Im), r < 8
                const float4* tq = reinterpret_cast<const float4*>(sT + (oka ? qa : 0) * 16);
                const float4 t0 = tq[half], t1 = tq[2 + half];
                const float tk[8] = {t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z, t1.w};
                float vr = 0.f, vi = 0.f;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    vr += tk[r] * h[r];
                    vi += tk[r] * h[r + 8];
                }
                vr += __shfl_xor(vr, 32, 64);
                vi += __shfl_xor(vi, 32, 64);
                if (oka && half == 0) {
                    atomicAdd(gx + 2 * sidx[qa], to_fixed(vr, S));
                    atomicAdd(gx + 2 * sidx[qa] + 1, to_fixed(vi, S));
                }
            }
            lds_order();                                   // the reads above precede the next staging writes
        }
    }
}

// 5. Visibility gradients and per-item gain partials from grad x (one
// wavefront per work item): grad V_k = conj(g_row) W_k (1 - F_k) grad x on the
// selected correlations; item_gain = sum over the item's channels of
// conj(y) grad x in FP64 (y the pre-gain weighted sum).
__global__ __launch_bounds__(256) void k_degrid_finish(const float2* __restrict__ vis, const float* __restrict__ weight,
                                                       const uint8_t* __restrict__ flag, const int32_t* __restrict__ ant1,
                                                       const int32_t* __restrict__ ant2, const float2* __restrict__ gains,
                                                       int n_ant, int n_chan, int n_corr, uint32_t mask, int n_items,
                                                       const unsigned long long* __restrict__ gxv,
                                                       const double* __restrict__ scale, float2* __restrict__ grad_vis,
                                                       double2* __restrict__ item_gain) {
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= n_items) return;
    const int n_chunks = (n_chan + kItemChans - 1) / kItemChans;
    const int r = item / n_chunks;
    const int c = (item % n_chunks) * kItemChans + lane;
    const bool live = c < n_chan;
    const size_t base = ((size_t)r * n_chan + (live ? c : 0)) * n_corr;
    float yr = 0.f, yi = 0.f, gxr = 0.f, gxi = 0.f;
    if (live) {
        (void)sample_value(vis, weight, flag, base, n_corr, mask, yr, yi);
        const size_t smp = (size_t)r * n_chan + c;
        gxr = from_fixed(gxv[2 * smp], scale[1]);
        gxi = from_fixed(gxv[2 * smp + 1], scale[1]);
    }
    // visibility gradients: conj(g_row) W_k (1 - F_k) grad x on the selected correlations
    const float2 gr = row_gain(gains, ant1, ant2, n_ant, r);
    const float hr = gr.x * gxr + gr.y * gxi, hi = gr.x * gxi - gr.y * gxr;   // conj(g) * gx
    if (live && grad_vis) {
        for (int k = 0; k < n_corr; ++k) {
            float wk = 0.f;
            if ((mask >> k) & 1u) {
                wk = weight ? weight[base + k] : 1.f;
                if (flag && flag[base + k]) wk = 0.f;
            }
            grad_vis[base + k] = make_float2(wk * hr, wk * hi);
        }
    }
    if (item_gain) {   // sum over the item's channels of conj(y) grad x, in FP64
        double sr = (double)yr * gxr + (double)yi * gxi;
        double si = (double)yr * gxi - (double)yi * gxr;
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) item_gain[item] = make_double2(sr, si);
    }
}

// Per-row sums of the items' gain partials (one wavefront per row, items in
// order, a fixed butterfly over the lanes): row_gain[r] = sum_items S.
__global__ __launch_bounds__(256) void k_row_gain(const double2* __restrict__ item_gain, int n_row, int n_chunks,
                                                  double2* __restrict__ row_gain) {
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= n_row) return;
    double sr = 0.0, si = 0.0;
    for (int c = lane; c < n_chunks; c += 64) {
        const double2 S = item_gain[(size_t)r * n_chunks + c];
        sr += S.x;
        si += S.y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) row_gain[r] = make_double2(sr, si);
}

// grad g_a = sum_{rows with ant1 = a} g_ant2 S + sum_{rows with ant2 = a} g_ant1 conj(S), S per row
__global__ __launch_bounds__(256) void k_gain_grad(const double2* __restrict__ row_gain, int n_row,
                                                   const int32_t* __restrict__ ant1, const int32_t* __restrict__ ant2,
                                                   const float2* __restrict__ gains, int n_ant,
                                                   float2* __restrict__ grad_gains) {
    __shared__ double red[2][4];
    const int a = blockIdx.x;
    double sr = 0.0, si = 0.0;
    for (int r = threadIdx.x; r < n_row; r += blockDim.x) {
        const int a1 = ant1[r], a2 = ant2[r];
        if (a1 < 0 || a1 >= n_ant || a2 < 0 || a2 >= n_ant) continue;
        const double2 S = row_gain[r];
        if (a1 == a) {
            const float2 g = gains[a2];
            sr += g.x * S.x - g.y * S.y;
            si += g.x * S.y + g.y * S.x;
        }
        if (a2 == a) {   // g_ant1 conj(S)
            const float2 g = gains[a1];
            sr += g.x * S.x + g.y * S.y;
            si += g.y * S.x - g.x * S.y;
        }
    }
    sr = block_sum(sr, red[0]);
    si = block_sum(si, red[1]);
    if (threadIdx.x == 0) grad_gains[a] = make_float2((float)sr, (float)si);
}

template <int M, int E, int EC>   // row-pass and column-pass radices
static void launch_adj_ffts(toi_ctx* c) {
    constexpr int B = (M >= 8192) ? 2 : 4;
    const float cell = (float)(c->p.cell_deg * kPi / 180.0);
    hipLaunchKernelGGL((k_adj_cols<M, EC>), dim3(M / 2), dim3(M / EC), 0, c->stream,
                       reinterpret_cast<const unsigned long long*>(c->adj_tp), c->hbuf, c->twiddle, c->corr, c->plan,
                       cell, c->p.mode, c->row_bits, c->scratch_d);
    const int nbands = M / B;
    hipLaunchKernelGGL((k_adj_rows<M, E, B>), dim3(nbands * c->P_cap), dim3(M / E), 0, c->stream, c->hbuf, c->grid,
                       c->twiddle, c->plan, nbands, c->tile_bits, c->row_bits, c->adj_parts);
    // the degridder's fixed-point scale from the plane gradients written
    hipLaunchKernelGGL(k_fixed_scale, dim3(1), dim3(1024), 0, c->stream, c->adj_parts, nbands * c->P_cap,
                       kDegridMaxTerms, c->scratch_d + 2);
}

hipError_t launch_degrid(toi_ctx* c, const float* grad_image, const toi_snapshot& s, float2* grad_vis,
                         float2* grad_gains) {
    const toi_params& p = c->p;
    StageTimer timer(c, TOI_STAGE_DEGRID);
    const int N = c->N, M = c->M;
    const double cell = p.cell_deg * kPi / 180.0;
    // transformed-plane gradient as fixed point (2 x 32 bits per pixel), its
    // scale from the largest image gradient
    hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, c->stream, c->adj_tp, 2 * (size_t)N * N);
    hipLaunchKernelGGL(k_absmax_parts, dim3(kAdjAbsmaxParts), dim3(256), 0, c->stream, grad_image, (size_t)N * N,
                       c->adj_parts);
    hipLaunchKernelGGL(k_fixed_scale, dim3(1), dim3(1024), 0, c->stream, c->adj_parts, kAdjAbsmaxParts, kRaMaxTerms,
                       c->scratch_d);
    hipLaunchKernelGGL(k_reproject_adj, dim3((N + kRaTile - 1) / kRaTile, (N + kRaTile - 1) / kRaTile), dim3(256), 0,
                       c->stream, grad_image, reinterpret_cast<unsigned long long*>(c->adj_tp), c->plan, N, cell,
                       c->scratch_d);
    switch (M) {
        case 64: launch_adj_ffts<64, 8, 8>(c); break;
        case 128: launch_adj_ffts<128, 8, 8>(c); break;
        case 256: launch_adj_ffts<256, 16, 16>(c); break;
        case 512: launch_adj_ffts<512, 16, 16>(c); break;
        case 1024: launch_adj_ffts<1024, 16, 16>(c); break;
        case 2048: launch_adj_ffts<2048, 16, 16>(c); break;
        case 4096: launch_adj_ffts<4096, 16, 8>(c); break;
        case 8192: launch_adj_ffts<8192, 16, 8>(c); break;
        default: return hipErrorInvalidValue;
    }
    const int n_chunks = (p.n_chan + kItemChans - 1) / kItemChans;
    const int n_items = s.n_row * n_chunks;
    if (n_items > 0) {
        // the gather walks bins of 8 x 8 cells: bins of the 16 x 16 variants
        // are built again at that size from the same records
        if (c->bins_shift != kTileShift) {
            const hipError_t e = launch_rebin(c, s, kTileShift);
            if (e != hipSuccess) return e;
        }
        const int NT = c->NT;
        const size_t n_samp = (size_t)s.n_row * p.n_chan;
        hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, c->stream, reinterpret_cast<float*>(c->gx),
                           4 * n_samp);
        const int blocks = unit_workgroups(n_items, c->NG_max * NT * NT);
        hipLaunchKernelGGL(k_degrid_tiles, dim3(blocks), dim3(64), 0,
                           c->stream, c->recs, p.n_chan, c->plan, M, NT, c->bin_off, c->bin_list, c->bin_cap,
                           c->bin_order, c->scratch_i, c->units, c->grid,
                           reinterpret_cast<unsigned long long*>(c->gx), c->scratch_d + 2);
        hipLaunchKernelGGL(k_degrid_finish, dim3((n_items + 3) / 4), dim3(256), 0, c->stream, (const float2*)s.vis,
                           s.weight, s.flag, s.ant1, s.ant2, (const float2*)s.gains, p.n_ant, p.n_chan, p.n_corr,
                           p.corr_mask, n_items, reinterpret_cast<const unsigned long long*>(c->gx), c->scratch_d + 2,
                           grad_vis, grad_gains ? c->item_gain : nullptr);
    }
    if (grad_gains) {
        // per-row sums first (in the slots after the items' partials), then per antenna over the rows
        double2* row_gain = c->item_gain + n_items;
        if (s.n_row > 0)
            hipLaunchKernelGGL(k_row_gain, dim3((s.n_row + 3) / 4), dim3(256), 0, c->stream, c->item_gain, s.n_row,
                               n_chunks, row_gain);
        hipLaunchKernelGGL(k_gain_grad, dim3(p.n_ant), dim3(256), 0, c->stream, row_gain, s.n_row, s.ant1, s.ant2,
                           (const float2*)s.gains, p.n_ant, grad_gains);
    }
    return hipGetLastError();
}

}  // namespace toi
