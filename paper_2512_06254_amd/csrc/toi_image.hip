// S5-S7: inverse FFT of every moment plane, grid correction, the Chebyshev /
// slab combination of Section 3.4 (or the single plane of Section 3.2), and
// the re-projection of Section 3.3.
//
// Row pass (per plane, bands of B grid rows): FFT along x, keep the N central
// bins and write them column-major per plane in groups of four columns,
// hbuf[plane][j1 / 4][y][j1 mod 4]: a workgroup's band of 4 rows of a column
// group is one 128-byte line, and the column pass reads a column with a
// 32-byte stride (its neighbours in the group are read by the neighbouring
// workgroups of the same XCD).  Grid tiles the gridder did not write (no
// samples) are read as zero, bands of empty tile rows are skipped and their
// hbuf rows read as zero by the column pass.
// Column pass (one image column j1 per workgroup): for every plane, FFT along
// y, keep the N central bins, and fold the plane into the pixel's combination
// in registers; only the real t-plane image leaves the workgroup.
#include "toi_fft.h"
#include "toi_grid.h"
#include "toi_internal.h"

namespace toi {

// Row-pass output layout: groups of G = kHbufGroup neighbouring image
// columns j1 interleaved per grid row y, hbuf[plane][j1 / G][y][j1 mod G].
// The G columns of a band of B rows are one contiguous block of G B 8 bytes,
// written whole by one workgroup; a column is read with stride G.  Measured
// (MeerKAT-shaped snapshot, row + column pass): G = 1 0.82 ms, 2 0.78 ms,
// 4 0.75 ms, 8 0.77 ms.
constexpr int kHbufGroup = 4;
template <int M>
__device__ inline size_t hbuf_index(int plane, int j1, int y) {
    constexpr int N = M / 2;
    return (((size_t)plane * (N / kHbufGroup) + j1 / kHbufGroup) * M + y) * kHbufGroup + j1 % kHbufGroup;
}

// Launch bounds: two workgroups per CU while a workgroup has at most 256
// (rows) or 512 (columns) threads; larger ones keep the full register budget
// of one (their LDS allows only one per CU anyway).
template <int M, int E, int B>
__global__ __launch_bounds__(M / E, (M / E) <= 256 ? 2 : 1) void k_fft_rows(const float2* __restrict__ grid, float2* __restrict__ hbuf,
                                                    const float2* __restrict__ tw,
                                                    const DevPlan* __restrict__ plan, int nbands,
                                                    const uint32_t* __restrict__ tile_bits,
                                                    const uint32_t* __restrict__ row_bits) {
    constexpr int N = M / 2;
    constexpr int KEEP = E / 2;
    constexpr int NT = M / kTile, WORDS = (NT + 31) / 32;
    __shared__ float2 lds[fft_lds_size<M, E>()];
    __shared__ float2 tw_s[FftTw<M, E>::size()];
    __shared__ uint32_t tb[WORDS];
    const int id = xcd_block_id(blockIdx.x, gridDim.x);
    const int plane = id / nbands, band = id % nbands;
    if ((plan->status & kStatusFatal) || plane >= plan->planes) return;
    const int g = group_of_plane(plane, plan);
    const int ty = (band * B) / kTile;
    if (!((row_bits[g * WORDS + (ty >> 5)] >> (ty & 31)) & 1u)) return;   // empty tile row
    if (threadIdx.x < WORDS) tb[threadIdx.x] = tile_bits[((size_t)g * NT + ty) * WORDS + threadIdx.x];
    load_twiddles<M, E>(tw_s, tw);
    // the band's rows lie in one tile row (B divides the tile side): one
    // occupancy mask of this thread's elements serves all of them
    static_assert(kTile % B == 0, "a band within one tile row");
    const uint32_t occ = fft_element_bits<M, E>(
        [&](int x) { return (tb[x >> (kTileShift + 5)] >> ((x >> kTileShift) & 31)) & 1u; });
    float2 keep[B][KEEP];
    // the next row's loads are issued before this row's transform
    float2 vn[E];
    fft_load_bits<M, E>(vn, grid + ((size_t)plane * M + band * B) * M, occ);
#pragma unroll
    for (int rb = 0; rb < B; ++rb) {
        const int y = band * B + rb;
        float2 v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = vn[e];
        if (rb + 1 < B) fft_load_bits<M, E>(vn, grid + ((size_t)plane * M + y + 1) * M, occ);
        fft_stages<M, E, 1>(v, lds, tw_s);
#pragma unroll
        for (int q = 0; q < KEEP; ++q) keep[rb][q] = v[fft_kept_slot<E>(q)];
        // (the next row's first exchange starts with a barrier: no barrier here)
    }
#pragma unroll
    for (int q = 0; q < KEEP; ++q) {
        const int j1 = fft_kept_index<M, E>(q);
        float2* dst = hbuf + hbuf_index<M>(plane, j1, band * B);
#pragma unroll
        for (int rb = 0; rb < B; ++rb) dst[rb * kHbufGroup] = keep[rb][q];
    }
}

// Per-pixel state of the Chebyshev combination.  The Bessel values J_k(alpha)
// come from Miller's backward recurrence (DLMF 10.74(iii)) run from order L
// down to 0 alongside the planes k = K-1 .. 0, with the normalisation
// J_0 + 2 sum_m J_{2m} = 1 applied once at the end; small |alpha| uses the
// power series.
template <int M, int E>
__global__ __launch_bounds__(M / E, (M / E) <= 512 ? 2 : 1) void k_fft_cols(const float2* __restrict__ hbuf, float* __restrict__ tplane_t,
                                                    const float2* __restrict__ tw, const float* __restrict__ corr,
                                                    const DevPlan* __restrict__ plan, float cell_rad, int mode,
                                                    const uint32_t* __restrict__ row_bits) {
    constexpr int N = M / 2;
    constexpr int KEEP = E / 2;
    constexpr int NT = M / kTile, WORDS = (NT + 31) / 32;
    __shared__ float2 lds[fft_lds_size<M, E>()];
    __shared__ float2 tw_s[FftTw<M, E>::size()];
    const int j1 = xcd_block_id(blockIdx.x, gridDim.x);
    int j2[KEEP];
#pragma unroll
    for (int q = 0; q < KEEP; ++q) j2[q] = fft_kept_index<M, E>(q);
    float* out = tplane_t + (size_t)j1 * N;
    load_twiddles<M, E>(tw_s, tw);
    if (plan->status & kStatusFatal) {
#pragma unroll
        for (int q = 0; q < KEEP; ++q) out[j2[q]] = 0.f;
        return;
    }
    const int K = plan->K, ns = plan->n_slab;
    const float c1 = corr[j1];
    float tr[KEEP], ti[KEEP];
#pragma unroll
    for (int q = 0; q < KEEP; ++q) { tr[q] = 0.f; ti[q] = 0.f; }

    if (mode == 2) {
        float2 v[E];
        fft_load_masked<M, E, kHbufGroup>(v, hbuf + hbuf_index<M>(0, j1, 0), [&](int y) { return (row_bits[y >> (kTileShift + 5)] >> ((y >> kTileShift) & 31)) & 1u; });
        fft_stages<M, E, 1>(v, lds, tw_s);
#pragma unroll
        for (int q = 0; q < KEEP; ++q) tr[q] = v[fft_kept_slot<E>(q)].x;
    } else {
        // transformed-plane geometry of this thread's pixels
        const float V13 = (float)plan->V[2], V23 = (float)plan->V[5], V33 = (float)plan->V[8];
        const float sg = V33 >= 0.f ? 1.f : -1.f;
        const float t1 = -cell_rad * (float)(j1 - N / 2);
        const float dr3 = (float)plan->dr3;
        float t3[KEEP], alpha[KEEP], ialpha[KEEP];
        bool small[KEEP], valid[KEEP];
#pragma unroll
        for (int q = 0; q < KEEP; ++q) {
            const float t2 = cell_rad * (float)(j2[q] - N / 2);
            const float a1 = t1 + V13, a2 = t2 + V23;
            const float arg = 1.f - a1 * a1 - a2 * a2;
            valid[q] = arg >= 0.f;
            // eq. (t3) in a cancellation-free form: 1 - V33^2 = V13^2 + V23^2
            const float num = t1 * t1 + t2 * t2 + 2.f * t1 * V13 + 2.f * t2 * V23;
            t3[q] = valid[q] ? -sg * num / (sqrtf(fmaxf(arg, 0.f)) + fabsf(V33)) : 0.f;
            alpha[q] = 2.f * 3.14159265358979f * dr3 * t3[q];
            small[q] = fabsf(alpha[q]) < 1e-3f;
            ialpha[q] = small[q] ? 0.f : 1.f / alpha[q];
        }
        const int L = max(plan->miller_top, K + 2);
        int occ_g = -1;                                // plane group whose occupancy mask is in occ
        uint32_t occ = 0;
        for (int p = 0; p < ns; ++p) {
            float jp1[KEEP], jc[KEEP], nrm[KEEP], ar[KEEP], ai[KEEP];
#pragma unroll
            for (int q = 0; q < KEEP; ++q) { jp1[q] = 0.f; jc[q] = 1.f; nrm[q] = 0.f; ar[q] = 0.f; ai[q] = 0.f; }
            // orders L .. K: recurrence only (no plane yet, ar = ai = 0).
            // The values grow by at most 2n / |alpha| <= 2e3 n per order
            // (|alpha| >= 1e-3 here; small |alpha| has ialpha = 0 and does
            // not grow), so a rescale by 2^-50 when |J| > 2^50, checked every
            // second order, stays far inside FP32 for any start order below
            // 10^8; the scale is exact and cancels in the normalisation.
            for (int n = L; n >= K; --n) {
#pragma unroll
                for (int q = 0; q < KEEP; ++q) {
                    if ((n & 1) == 0) nrm[q] += 2.f * jc[q];
                    const float jm1 = (2.f * n) * ialpha[q] * jc[q] - jp1[q];
                    jp1[q] = jc[q];
                    jc[q] = jm1;
                    if ((n & 1) == 0 && fabsf(jc[q]) > 0x1p50f) {
                        jc[q] *= 0x1p-50f; jp1[q] *= 0x1p-50f; nrm[q] *= 0x1p-50f;
                    }
                }
            }
            // orders K-1 .. 0 with their planes.  Each plane's column is loaded
            // as soon as the previous plane's kept bins are out of its
            // registers, so that the loads are in flight while that plane is
            // folded into the combination (the same registers; 0.341 ->
            // 0.325 ms against loading each column right before its transform)
            auto plane_occ = [&](int k) {
                const int gk = group_of_plane(p * K + k, plan);
                if (gk != occ_g) {   // planes of one group share the occupancy of their tile rows
                    // the group's words come from L1/L2: a copy of every group's
                    // words in LDS took 17 KB at 272 planes and left one
                    // workgroup per CU instead of two
                    const uint32_t* rbg = row_bits + gk * WORDS;
                    occ = fft_element_bits<M, E>(
                        [&](int y) { return (rbg[y >> (kTileShift + 5)] >> ((y >> kTileShift) & 31)) & 1u; });
                    occ_g = gk;
                }
                return occ;
            };
            float2 v[E];
            fft_load_bits<M, E, kHbufGroup>(v, hbuf + hbuf_index<M>(p * K + K - 1, j1, 0), plane_occ(K - 1));
            for (int k = K - 1; k >= 0; --k) {
                fft_stages<M, E, 1>(v, lds, tw_s);
                float2 Fk[KEEP];
#pragma unroll
                for (int q = 0; q < KEEP; ++q) Fk[q] = v[fft_kept_slot<E>(q)];
                if (k > 0)
                    fft_load_bits<M, E, kHbufGroup>(v, hbuf + hbuf_index<M>(p * K + k - 1, j1, 0), plane_occ(k - 1));
#pragma unroll
                for (int q = 0; q < KEEP; ++q) {
                    float jk;
                    if (small[q]) {
                        const float a = alpha[q];
                        jk = k == 0 ? 1.f - 0.25f * a * a
                           : k == 1 ? 0.5f * a * (1.f - 0.125f * a * a)
                           : k == 2 ? 0.125f * a * a
                           : k == 3 ? a * a * a * (1.f / 48.f) : 0.f;
                    } else {
                        jk = jc[q];
                        if ((k & 1) == 0) nrm[q] += (k == 0 ? 1.f : 2.f) * jk;
                    }
                    const float f = (k == 0 ? 1.f : 2.f) * jk;
                    const float2 F = Fk[q];
                    switch (k & 3) {   // c_k = 2 i^k J_k (c_0 = J_0)
                        case 0: ar[q] += f * F.x; ai[q] += f * F.y; break;
                        case 1: ar[q] -= f * F.y; ai[q] += f * F.x; break;
                        case 2: ar[q] -= f * F.x; ai[q] -= f * F.y; break;
                        default: ar[q] += f * F.y; ai[q] -= f * F.x; break;
                    }
                    if (!small[q] && k > 0) {
                        const float jm1 = (2.f * k) * ialpha[q] * jc[q] - jp1[q];
                        jp1[q] = jc[q];
                        jc[q] = jm1;
                        if ((k & 1) == 0 && fabsf(jc[q]) > 0x1p50f) {
                            jc[q] *= 0x1p-50f; jp1[q] *= 0x1p-50f; nrm[q] *= 0x1p-50f;
                            ar[q] *= 0x1p-50f; ai[q] *= 0x1p-50f;
                        }
                    }
                }
                // (the next plane's first exchange starts with a barrier)
            }
            const float r3p = (float)(plan->r3min + (2 * p + 1) * plan->dr3);
#pragma unroll
            for (int q = 0; q < KEEP; ++q) {
                const float inv = small[q] ? 1.f : 1.f / nrm[q];
                float sn, cs;
                sincosf(2.f * 3.14159265358979f * r3p * t3[q], &sn, &cs);
                const float xr = ar[q] * inv, xi = ai[q] * inv;
                tr[q] += cs * xr - sn * xi;
                ti[q] += cs * xi + sn * xr;
            }
        }
#pragma unroll
        for (int q = 0; q < KEEP; ++q)
            if (!valid[q]) tr[q] = 0.f;
    }
    const float norm = (float)plan->norm;
#pragma unroll
    for (int q = 0; q < KEEP; ++q) out[j2[q]] = tr[q] * c1 * corr[j2[q]] * norm;
}

// Re-projection (Section 3.3): output pixel -> reduced SIN map to the tilted
// plane (x' = x + r0 z xi, y' = y + r0 z eta, z = 1 - n) -> in-plane 2x2 block
// of V -> transformed-plane coordinates -> bilinear gather.  FP64 coordinates.
// kReprojRows output rows per thread: the coordinate chain of a pixel (an
// FP64 square root and three divisions) is long, and independent pixels in
// one thread let it overlap (one pixel per thread left the pass latency-bound).
constexpr int kReprojRows = 4;
__global__ __launch_bounds__(256) void k_reproject(const float* __restrict__ tplane_t, float* __restrict__ img,
                                                   const DevPlan* __restrict__ plan, int N, double cell_rad) {
    const int j1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (j1 >= N) return;
    const bool fatal = plan->status & kStatusFatal;
#pragma unroll
    for (int q = 0; q < kReprojRows; ++q) {
        const int j2 = blockIdx.y * kReprojRows + q;
        float val = 0.f;
        int i1, i2;
        float f1, f2;
        if (j2 < N && !fatal && reproject_source(plan, N, cell_rad, j1, j2, i1, i2, f1, f2)) {
            const float* c0 = tplane_t + (size_t)i1 * N + i2;      // j1-major t-plane
            const float* c1 = c0 + N;
            val = (1.f - f1) * (1.f - f2) * c0[0] + f1 * (1.f - f2) * c1[0] + (1.f - f1) * f2 * c0[1] + f1 * f2 * c1[1];
        }
        if (j2 < N) img[(size_t)j2 * N + j1] = val;
    }
}

__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ src, float* __restrict__ dst, int N) {
    __shared__ float tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8) tile[i][tx] = src[(size_t)(by + i) * N + bx + tx];
    __syncthreads();
    for (int i = ty; i < 32; i += 8) dst[(size_t)(bx + i) * N + by + tx] = tile[tx][i];
}

template <int M, int E, int EC>   // row-pass and column-pass radices
static hipError_t launch_fft_passes(toi_ctx* c) {
    constexpr int B = 4;
    const int nbands = M / B;
    const int P = c->P_cap;
    {
        StageTimer timer(c, TOI_STAGE_FFT_ROWS);
        hipLaunchKernelGGL((k_fft_rows<M, E, B>), dim3(nbands * P), dim3(M / E), 0, c->stream, c->grid,
                           c->hbuf, c->twiddle, c->plan, nbands, c->tile_bits, c->row_bits);
    }
    const float cell = (float)(c->p.cell_deg * kPi / 180.0);
    StageTimer timer(c, TOI_STAGE_FFT_COLS);
    hipLaunchKernelGGL((k_fft_cols<M, EC>), dim3(M / 2), dim3(M / EC), 0, c->stream, c->hbuf, c->tplane_t,
                       c->twiddle, c->corr, c->plan, cell, c->p.mode, c->row_bits);
    return hipGetLastError();
}

hipError_t launch_image(toi_ctx* c, float* image_out, float* tplane_out) {
    hipError_t e;
    switch (c->M) {
        case 64: e = launch_fft_passes<64, 8, 8>(c); break;
        case 128: e = launch_fft_passes<128, 8, 8>(c); break;
        case 256: e = launch_fft_passes<256, 16, 16>(c); break;
        case 512: e = launch_fft_passes<512, 16, 16>(c); break;
        case 1024: e = launch_fft_passes<1024, 16, 16>(c); break;
        case 2048: e = launch_fft_passes<2048, 16, 16>(c); break;
        case 4096: e = launch_fft_passes<4096, 16, 8>(c); break;
        case 8192: e = launch_fft_passes<8192, 16, 8>(c); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    const int N = c->N;
    const double cell = c->p.cell_deg * kPi / 180.0;
    StageTimer timer(c, TOI_STAGE_REPROJECT);
    hipLaunchKernelGGL(k_reproject, dim3((N + 255) / 256, (N + kReprojRows - 1) / kReprojRows), dim3(256), 0,
                       c->stream, c->tplane_t, image_out,
                       c->plan, N, cell);
    if (tplane_out)
        hipLaunchKernelGGL(k_transpose, dim3(N / 32, N / 32), dim3(256), 0, c->stream, c->tplane_t, tplane_out, N);
    return hipGetLastError();
}

}  // namespace toi
