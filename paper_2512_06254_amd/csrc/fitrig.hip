// S8: FITrig tLISI map from the three youngest images (Sections 2 and 4.5).
//
// The FITrig index itself is defined outside the paper; this library computes
// a stand-in with the stated properties: per tile, the similarity of the two
// adjacent difference images X = I_{t-1} - I_{t-2} and Y = I_t - I_{t-1}, in
// [0, 1] with 1 for identical tiles.  It uses the SSIM form (Wang et al.,
// IEEE TIP 13, 2004) with C1 = (0.01 L)^2, C2 = (0.03 L)^2, L the range of
// the pair over the whole image, and population statistics per tile:
//   S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2)),
//   tLISI = clamp((1 + S) / 2, 0, 1)          (1 everywhere when L = 0).
// Pass 1 (one workgroup per tile) forms FP64 sums, minimum and maximum;
// pass 2 (one workgroup) combines the ranges and evaluates each tile.
#include <mutex>
#include <string>

#include "toi_device.h"
#include "toi_internal.h"

namespace toi {

// One wavefront per tile: its sums need no workgroup barrier (a workgroup of
// 256 threads per tile with three block reductions took 22 us per 2048^2
// snapshot).  Lane l adds the pixels l, l + 64, ... of the tile in order,
// kB loads ahead, then the wavefront adds the lanes in a fixed butterfly.
__global__ __launch_bounds__(256) void k_tlisi_tiles(const float* __restrict__ a, const float* __restrict__ b,
                                                     const float* __restrict__ c, int N, int tile,
                                                     TileStat* __restrict__ out) {
    const int T = N / tile;
    const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= T * T) return;
    const int lane = threadIdx.x & 63;
    const int ty = t / T, tx = t % T;
    double sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0, mn = 1e300, mx = -1e300;
    const int n = tile * tile;
    constexpr int kB = 4;
    for (int i0 = lane; i0 < n; i0 += kB * 64) {
        float va[kB], vb[kB], vc[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            const int i = i0 + q * 64;
            va[q] = vb[q] = vc[q] = 0.f;
            if (i < n) {
                const size_t o = (size_t)(ty * tile + i / tile) * N + tx * tile + i % tile;
                va[q] = a[o];
                vb[q] = b[o];
                vc[q] = c[o];
            }
        }
#pragma unroll
        for (int q = 0; q < kB; ++q)
            if (i0 + q * 64 < n) {
                const double X = (double)vb[q] - (double)va[q], Y = (double)vc[q] - (double)vb[q];
                sx += X; sy += Y; sxx += X * X; syy += Y * Y; sxy += X * Y;
                mn = fmin(mn, fmin(X, Y));
                mx = fmax(mx, fmax(X, Y));
            }
    }
    sx = wave_sum(sx); sy = wave_sum(sy); sxx = wave_sum(sxx); syy = wave_sum(syy); sxy = wave_sum(sxy);
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (lane == 0) {
        TileStat s;
        s.sx = sx; s.sy = sy; s.sxx = sxx; s.syy = syy; s.sxy = sxy;
        s.mn = mn; s.mx = mx; s.pad_ = 0;
        out[t] = s;
    }
}

// Every workgroup takes the extremes over all tiles (exact, so the same in
// each) and then the map values of its share of the tiles.
constexpr int kTlisiFinalGroups = 16;
__global__ __launch_bounds__(1024) void k_tlisi_final(const TileStat* __restrict__ st, int n_tiles, int tile,
                                                      float* __restrict__ out) {
    __shared__ double red[2][16];
    double mn = 1e300, mx = -1e300;
    for (int i = threadIdx.x; i < n_tiles; i += blockDim.x) {
        mn = fmin(mn, st[i].mn);
        mx = fmax(mx, st[i].mx);
    }
    mn = block_min(mn, red[0]);
    mx = block_max(mx, red[1]);
    const double L = mx - mn;
    const double C1 = (0.01 * L) * (0.01 * L), C2 = (0.03 * L) * (0.03 * L);
    const double inv_n = 1.0 / ((double)tile * tile);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_tiles; i += gridDim.x * blockDim.x) {
        if (!(L > 0.0)) {
            out[i] = 1.f;
            continue;
        }
        const TileStat s = st[i];
        const double mxx = s.sx * inv_n, myy = s.sy * inv_n;
        const double vx = s.sxx * inv_n - mxx * mxx, vy = s.syy * inv_n - myy * myy;
        const double cxy = s.sxy * inv_n - mxx * myy;
        const double S = ((2 * mxx * myy + C1) * (2 * cxy + C2)) / ((mxx * mxx + myy * myy + C1) * (vx + vy + C2));
        out[i] = (float)fmin(1.0, fmax(0.0, 0.5 * (1.0 + S)));
    }
}

static void tlisi_kernels(hipStream_t stream, const float* a, const float* b, const float* d, int N, int tile,
                          TileStat* stats, float* out) {
    const int T = N / tile;
    hipLaunchKernelGGL(k_tlisi_tiles, dim3((T * T + 3) / 4), dim3(256), 0, stream, a, b, d, N, tile, stats);
    hipLaunchKernelGGL(k_tlisi_final, dim3(std::min(kTlisiFinalGroups, (T * T + 1023) / 1024)), dim3(1024), 0, stream,
                       stats, T * T, tile, out);
}

hipError_t launch_tlisi(toi_ctx* c, const float* a, const float* b, const float* d, float* out) {
    StageTimer timer(c, TOI_STAGE_TLISI);
    tlisi_kernels(c->stream, a, b, d, c->N, c->p.tile, c->tiles, out);
    return hipGetLastError();
}

// tLISI without a context: the per-tile statistics go to this file-scope
// device array instead of a context's workspace.  Every device the library
// runs on holds its own copy for the life of the process.  In host code the
// array's name is not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device on its first call and kept in scratch_dev.
static __device__ __align__(256) TileStat scratch[TOI_TLISI_STATIC_TILES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
TileStat* scratch_dev[kMaxDevices];

toi_status scratch_address(int dev, TileStat** out) {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_check(nullptr, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                      "fitrig_tlisi_noalloc: hipGetSymbolAddress");
        scratch_dev[dev] = static_cast<TileStat*>(ptr);
    }
    *out = scratch_dev[dev];
    return TOI_OK;
}
}  // namespace

}  // namespace toi

extern "C" toi_status fitrig_tlisi_noalloc(const float* img_tm2, const float* img_tm1, const float* img_t,
                                           int32_t n_pix, int32_t tile, float* tlisi_out, void* hip_stream) {
    using namespace toi;
    if (!img_tm2 || !img_tm1 || !img_t || !tlisi_out)
        return fail(nullptr, TOI_EINVAL, "fitrig_tlisi_noalloc: NULL image or output");
    if (n_pix <= 0 || tile <= 0 || n_pix % tile != 0)
        return fail(nullptr, TOI_EINVAL, "fitrig_tlisi_noalloc: n_pix and tile must be > 0 and tile must divide n_pix");
    const long T = n_pix / tile;
    if (T * T > TOI_TLISI_STATIC_TILES)
        return fail(nullptr, TOI_EINVAL,
                    "fitrig_tlisi_noalloc: (n_pix / tile)^2 = " + std::to_string(T * T) +
                        " tiles exceeds the static scratch of " + std::to_string(TOI_TLISI_STATIC_TILES));
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(nullptr, e, "fitrig_tlisi_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, TOI_EUNSUPPORTED, "fitrig_tlisi_noalloc: device index");
    TileStat* stats = nullptr;
    const toi_status st = scratch_address(dev, &stats);
    if (st != TOI_OK) return st;
    tlisi_kernels(static_cast<hipStream_t>(hip_stream), img_tm2, img_tm1, img_t, n_pix, tile, stats, tlisi_out);
    return hip_check(nullptr, hipGetLastError(), "fitrig_tlisi_noalloc");
}

// ---------------------------------------------------------------- S9: window detection
// One workgroup (the window is tile-grid sized): per tile the periodic score
// (DFT power of the mean-removed 16-map window at f = 1..8, harmonic sums over
// h in {1, 2, 4, 8} harmonics divided by sqrt(h), maximum over f and h) and the
// non-periodic score sum(1 - tLISI), both in FP64; z-scores over all tiles
// with the population standard deviation; tiles with z_periodic > 5 or
// z_nonperiodic > 4 are grouped into 8-connected components by min-label
// propagation in LDS; one box per component in pixels, sorted by
// (y0, x0, y1, x1).  All decisions are made in FP64 in a fixed order.
namespace toi {

__device__ inline double periodic_score16(const double* x) {
    double mean = 0.0;
    for (int t = 0; t < kWindow; ++t) mean += x[t];
    mean /= kWindow;
    double P[kWindow / 2 + 1];
    P[0] = 0.0;
    for (int f = 1; f <= kWindow / 2; ++f) {
        double re = 0.0, im = 0.0;
        for (int t = 0; t < kWindow; ++t) {
            double sn, cs;
            sincospi(-2.0 * f * t / kWindow, &sn, &cs);
            re += (x[t] - mean) * cs;
            im += (x[t] - mean) * sn;
        }
        P[f] = re * re + im * im;
    }
    double best = -1e300;
    const int hs[4] = {1, 2, 4, 8};
    for (int f = 1; f <= kWindow / 2; ++f) {
        for (int hi = 0; hi < 4; ++hi) {
            const int h = hs[hi];
            double s = 0.0;
            for (int j = 1; j <= h; ++j)
                if (j * f <= kWindow / 2) s += P[j * f];
            best = fmax(best, s / sqrt((double)h));
        }
    }
    return best;
}

__global__ __launch_bounds__(1024) void k_detect(const float* __restrict__ window, int T, int tile, int t_index,
                                                 double* __restrict__ scores, int4* __restrict__ boxes_tmp,
                                                 int32_t* __restrict__ boxes, int max_boxes,
                                                 int32_t* __restrict__ n_boxes) {
    extern __shared__ int32_t sh[];            // label[T*T], root_id[T*T]
    __shared__ double red[16];
    __shared__ int changed, ncomp;
    const int n = T * T;
    int32_t* label = sh;
    int32_t* root_id = sh + n;
    double* sp = scores;                       // periodic
    double* snp = scores + n;                  // non-periodic
    double s1p = 0, s2p = 0, s1n = 0, s2n = 0;
    if (window) {                              // else the scores are in place (whole-cube detection)
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            double x[kWindow];
            double np = 0.0;
            for (int t = 0; t < kWindow; ++t) {
                x[t] = (double)window[(size_t)t * n + i];
                np += 1.0 - x[t];
            }
            sp[i] = periodic_score16(x);
            snp[i] = np;
        }
    }
    __syncthreads();
    // population mean / std in a fixed order: per-thread strided partial sums, then a tree
    for (int i = threadIdx.x; i < n; i += blockDim.x) { s1p += sp[i]; s1n += snp[i]; }
    s1p = block_sum(s1p, red);
    s1n = block_sum(s1n, red);
    const double mp = s1p / n, mn = s1n / n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        s2p += (sp[i] - mp) * (sp[i] - mp);
        s2n += (snp[i] - mn) * (snp[i] - mn);
    }
    s2p = block_sum(s2p, red);
    s2n = block_sum(s2n, red);
    const double sdp = sqrt(s2p / n), sdn = sqrt(s2n / n);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double zp = sdp > 0 ? (sp[i] - mp) / sdp : 0.0;
        const double zn = sdn > 0 ? (snp[i] - mn) / sdn : 0.0;
        label[i] = (zp > 5.0 || zn > 4.0) ? i : -1;
    }
    if (threadIdx.x == 0) ncomp = 0;
    __syncthreads();
    // 8-connected components: every flagged tile takes the smallest label around it
    for (;;) {
        if (threadIdx.x == 0) changed = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            int l = label[i];
            if (l < 0) continue;
            const int ty = i / T, tx = i % T;
            int m = l;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int yy = ty + dy, xx = tx + dx;
                    if (yy < 0 || yy >= T || xx < 0 || xx >= T) continue;
                    const int ln = label[yy * T + xx];
                    if (ln >= 0 && ln < m) m = ln;
                }
            m = min(m, label[m]);              // pointer jumping
            if (m < l) {
                label[i] = m;
                changed = 1;
            }
        }
        __syncthreads();
        if (!changed) break;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (label[i] == i) root_id[i] = atomicAdd(&ncomp, 1);
    __syncthreads();
    const int nc = ncomp;
    for (int k = threadIdx.x; k < nc; k += blockDim.x) boxes_tmp[k] = make_int4(1 << 30, 1 << 30, -1, -1);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int l = label[i];
        if (l < 0) continue;
        int4* b = boxes_tmp + root_id[l];
        const int ty = i / T, tx = i % T;
        atomicMin(&b->x, tx);
        atomicMin(&b->y, ty);
        atomicMax(&b->z, tx);
        atomicMax(&b->w, ty);
    }
    __syncthreads();
    // rank sort by (y0, x0, y1, x1); boxes are distinct (components are disjoint)
    for (int k = threadIdx.x; k < nc; k += blockDim.x) {
        const int4 a = boxes_tmp[k];
        int rank = 0;
        for (int j = 0; j < nc; ++j) {
            const int4 b = boxes_tmp[j];
            const bool less = b.y != a.y ? b.y < a.y : b.x != a.x ? b.x < a.x : b.w != a.w ? b.w < a.w : b.z < a.z;
            rank += less ? 1 : 0;
        }
        if (rank < max_boxes) {
            int32_t* o = boxes + 5 * rank;
            o[0] = t_index;
            o[1] = tile * a.x;
            o[2] = tile * a.y;
            o[3] = tile * a.z + tile - 1;
            o[4] = tile * a.w + tile - 1;
        }
    }
    if (threadIdx.x == 0) *n_boxes = nc;
}

// Whole-cube scores (the after-the-run statistic over all L maps): one
// wavefront per tile stages the tile's series x_0..x_{L-1} in LDS (FP64) and
// its mean; lane l evaluates the DFT power of the mean-removed series at
// f = 1 + l, 65 + l, ... <= L/2 by Goertzel's recurrence
// s_t = d_t + 2 cos(2 pi f / L) s_{t-1} - s_{t-2}, |X_f|^2 = s_{L-1}^2 +
// s_{L-2}^2 - 2 cos(2 pi f / L) s_{L-1} s_{L-2} (Goertzel, 1958), all in FP64;
// the powers go to LDS, and the lanes take the maximum over f and
// h in {1, 2, 4, 8} of the harmonic sum / sqrt(h).  Also the non-periodic
// sum(1 - x).  LDS: 8 L + 8 (L / 2 + 1) bytes.
__global__ __launch_bounds__(64) void k_cube_scores(const float* __restrict__ cube, int L, int n_tiles,
                                                    double* __restrict__ scores) {
    extern __shared__ double sd[];
    double* x = sd;                            // [L]
    double* P = sd + L;                        // [L / 2 + 1]
    const int i = blockIdx.x, lane = threadIdx.x;
    double sum = 0.0;
    for (int t = lane; t < L; t += 64) {
        const double v = (double)cube[(size_t)t * n_tiles + i];
        x[t] = v;
        sum += v;
    }
    sum = wave_sum(sum);
    const double mean = sum / L;
    double np = 0.0;
    for (int t = lane; t < L; t += 64) np += 1.0 - x[t];
    np = wave_sum(np);
    lds_order();
    const int F = L / 2;
    for (int f = 1 + lane; f <= F; f += 64) {
        double sn, cs;
        sincospi(2.0 * f / L, &sn, &cs);
        const double c2 = 2.0 * cs;
        double s1 = 0.0, s2 = 0.0;
        for (int t = 0; t < L; ++t) {
            const double s0 = (x[t] - mean) + c2 * s1 - s2;
            s2 = s1;
            s1 = s0;
        }
        P[f] = s1 * s1 + s2 * s2 - c2 * s1 * s2;
    }
    lds_order();
    double best = -1e300;
    for (int f = 1 + lane; f <= F; f += 64) {
        double acc = 0.0;
        int j = 1;
        for (int h = 1; h <= 8; h *= 2) {      // h = 1, 2, 4, 8 harmonics
            for (; j <= h; ++j)
                if (j * f <= F) acc += P[j * f];
            best = fmax(best, acc / sqrt((double)h));
        }
    }
    best = wave_max(best);
    if (lane == 0) {
        scores[i] = best;
        scores[n_tiles + i] = np;
    }
}

// ---------------------------------------------------------------- localisation
// Full-resolution localisation of a candidate box in the difference image
// D = img_b - img_a (Sections 2 and 6), one workgroup per box:
//  - background med = the lower median of the box's n values, element
//    (n - 1) / 2, and MAD = the lower median of |D - med|, both by an exact
//    4-pass radix selection (8 bits per pass) on order-preserving keys of the
//    FP32 values; sigma = 1.4826 MAD;
//  - the brightest pixel p*: largest |D - med|, the first in row-major order
//    on ties (one 64-bit maximum of (|r| bits, inverted index)); s = its sign;
//  - source pixels s (D - med) > 5 sigma (FP64) as LDS flags; the component of
//    8-connected source pixels reached from p*, grown by sweeps until none
//    changes;
//  - FP64 intensity-weighted centroid and second moments (fixed-order sums),
//    the Gaussian-like check (>= 3 pixels, axis ratio <= 3, p* within 1.5
//    pixels of the centroid), and RA/Dec of the centroid by the inverse SIN
//    projection about (ra0, dec0) with l = -cell (xc - N/2), m = cell (yc - N/2).
// out[8]: valid, xc, yc, ra (deg), dec (deg), s (D - med) at p*, sigma,
// component pixels (-1: box outside the image or above kLocMaxPixels).
constexpr int kLocMaxPixels = 65536;
constexpr int kLocThreads = 256;

__device__ inline uint32_t float_key(float v) {   // order-preserving
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float key_float(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// k-th smallest key(i), i < n (every thread of the block; ends with a barrier)
template <typename KeyFn>
__device__ uint32_t block_select(int n, int k, KeyFn key, uint32_t* hist, int* sel) {
    uint32_t prefix = 0, mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = threadIdx.x; b < 256; b += blockDim.x) hist[b] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t u = key(i);
            if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0, b = 0;
            for (; b < 255; ++b) {
                if (acc + (int)hist[b] > k) break;
                acc += (int)hist[b];
            }
            sel[0] = b;
            sel[1] = k - acc;
        }
        __syncthreads();
        prefix |= (uint32_t)sel[0] << shift;
        mask |= 255u << shift;
        k = sel[1];
        __syncthreads();
    }
    return prefix;
}

__device__ inline unsigned long long block_max_u64(unsigned long long v, unsigned long long* red) {
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long m = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = red[i] > m ? red[i] : m;
    __syncthreads();
    return m;
}

__global__ __launch_bounds__(kLocThreads) void k_localise(const float* __restrict__ img_a,
                                                          const float* __restrict__ img_b,
                                                          const int32_t* __restrict__ boxes, int N,
                                                          double cell_rad, double ra0, double dec0, int morph,
                                                          double* __restrict__ out) {
    __shared__ uint8_t flag[kLocMaxPixels];   // bit 0: source pixel, bit 1: reached from p*
    __shared__ uint32_t hist[256];
    __shared__ int sel[2];
    __shared__ double red[kLocThreads / 64];
    __shared__ unsigned long long redu[kLocThreads / 64];
    __shared__ int changed;
    const int32_t* bx = boxes + 5 * blockIdx.x;
    double* o = out + 8 * blockIdx.x;
    const int x0 = bx[1], y0 = bx[2], x1 = bx[3], y1 = bx[4];
    const int w = x1 - x0 + 1, h = y1 - y0 + 1;
    if (x0 < 0 || y0 < 0 || x1 >= N || y1 >= N || w <= 0 || h <= 0 || (long)w * h > kLocMaxPixels) {
        if (threadIdx.x == 0) {
            for (int j = 0; j < 8; ++j) o[j] = 0.0;
            o[7] = -1.0;
        }
        return;
    }
    const int n = w * h;
    auto D = [&](int i) { const size_t q = (size_t)(y0 + i / w) * N + x0 + i % w; return img_b[q] - img_a[q]; };
    const float med = key_float(block_select(n, (n - 1) / 2, [&](int i) { return float_key(D(i)); }, hist, sel));
    const float mad = key_float(block_select(n, (n - 1) / 2, [&](int i) { return float_key(fabsf(D(i) - med)); },
                                             hist, sel));
    const double sigma = 1.4826 * (double)mad;
    unsigned long long best = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const unsigned long long kk = ((unsigned long long)__float_as_uint(fabsf(D(i) - med)) << 32) |
                                      (unsigned long long)(0xffffffffu - (uint32_t)i);
        best = kk > best ? kk : best;
    }
    best = block_max_u64(best, redu);
    const int ip = (int)(0xffffffffu - (uint32_t)(best & 0xffffffffull));
    const float rp = D(ip) - med;
    const double sg = rp >= 0.f ? 1.0 : -1.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const bool src = sg * (double)(D(i) - med) > 5.0 * sigma;
        flag[i] = (src ? 1 : 0) | ((src && i == ip) ? 2 : 0);
    }
    __syncthreads();
    for (;;) {                                   // grow the component of p*
        if (threadIdx.x == 0) changed = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            if (flag[i] != 1) continue;          // source pixel not reached yet
            const int yy = i / w, xx = i % w;
            bool near = false;
            for (int dy = -1; dy <= 1 && !near; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int y2 = yy + dy, x2 = xx + dx;
                    if (y2 >= 0 && y2 < h && x2 >= 0 && x2 < w && (flag[y2 * w + x2] & 2)) {
                        near = true;
                        break;
                    }
                }
            if (near) {
                flag[i] = 3;
                changed = 1;
            }
        }
        __syncthreads();
        if (!changed) break;
        __syncthreads();
    }
    double sW = 0, sX = 0, sY = 0, cnt = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (flag[i] == 3) {
            const double wt = sg * (double)(D(i) - med);
            sW += wt;
            sX += wt * (x0 + i % w);
            sY += wt * (y0 + i / w);
            cnt += 1.0;
        }
    sW = block_sum(sW, red);
    sX = block_sum(sX, red);
    sY = block_sum(sY, red);
    cnt = block_sum(cnt, red);
    if (cnt == 0.0) {
        if (threadIdx.x == 0) {
            o[0] = 0.0; o[1] = o[2] = o[3] = o[4] = __builtin_nan("");
            o[5] = sg * (double)rp; o[6] = sigma; o[7] = 0.0;
        }
        return;
    }
    const double xc = sX / sW, yc = sY / sW;
    double cxx = 0, cyy = 0, cxy = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (flag[i] == 3) {
            const double wt = sg * (double)(D(i) - med);
            const double dx = x0 + i % w - xc, dy = y0 + i / w - yc;
            cxx += wt * dx * dx;
            cyy += wt * dy * dy;
            cxy += wt * dx * dy;
        }
    cxx = block_sum(cxx, red) / sW;
    cyy = block_sum(cyy, red) / sW;
    cxy = block_sum(cxy, red) / sW;
    if (threadIdx.x == 0) {
        const double tr = cxx + cyy, det = cxx * cyy - cxy * cxy;
        const double disc = sqrt(fmax(0.0, tr * tr / 4.0 - det));
        const double l1 = tr / 2.0 + disc, l2 = tr / 2.0 - disc;
        const double px = x0 + ip % w, py = y0 + ip / w;
        const bool ok = cnt >= 3.0 && l2 > 0.0 && sqrt(l1 / l2) <= 3.0 && hypot(px - xc, py - yc) <= 1.5;
        const double l = -cell_rad * (xc - N / 2), m = cell_rad * (yc - N / 2);
        const double nn = sqrt(fmax(0.0, 1.0 - l * l - m * m));
        const double dec = asin(m * cos(dec0) + nn * sin(dec0));
        double ra = ra0 + atan2(l, nn * cos(dec0) - m * sin(dec0));
        ra = fmod(ra * (180.0 / kPi), 360.0);
        if (ra < 0.0) ra += 360.0;
        o[0] = (ok || !morph) ? 1.0 : 0.0;
        o[1] = xc;
        o[2] = yc;
        o[3] = ra;
        o[4] = dec * (180.0 / kPi);
        o[5] = sg * (double)rp;
        o[6] = sigma;
        o[7] = cnt;
    }
}

// Index of the tLISI map (cube[k], oldest first) with the smallest sum over
// each box's tiles (the first on ties): one workgroup per box, maps strided
// over the threads (each thread's maps ascending), FP64 sums over the tiles in
// row-major order; the minimum sum, then the smallest index holding it.
__global__ __launch_bounds__(256) void k_strongest_map(const float* __restrict__ cube, int n_maps, int T, int tile,
                                                       const int32_t* __restrict__ boxes,
                                                       int32_t* __restrict__ k_out) {
    __shared__ double red[4];
    __shared__ int redi[4];
    const int32_t* bx = boxes + 5 * blockIdx.x;
    const int tx0 = max(0, bx[1] / tile), ty0 = max(0, bx[2] / tile);
    const int tx1 = min(T - 1, bx[3] / tile), ty1 = min(T - 1, bx[4] / tile);
    double best = 1e300;
    int first = INT_MAX;
    for (int k = threadIdx.x; k < n_maps; k += blockDim.x) {
        double sm = 0.0;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) sm += (double)cube[((size_t)k * T + ty) * T + tx];
        if (sm < best) {
            best = sm;
            first = k;
        }
    }
    const double m = block_min(best, red);
    int cand = best == m ? first : INT_MAX;
    for (int o = 32; o > 0; o >>= 1) cand = min(cand, __shfl_xor(cand, o, 64));
    if ((threadIdx.x & 63) == 0) redi[threadIdx.x >> 6] = cand;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = redi[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = min(r, redi[w]);
        k_out[blockIdx.x] = r;
    }
}

hipError_t launch_localise(toi_ctx* c, const float* a, const float* b, const int32_t* boxes, int n_boxes,
                           double ra0_deg, double dec0_deg, int morph, double* out) {
    if (n_boxes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_localise, dim3(n_boxes), dim3(kLocThreads), 0, c->stream, a, b, boxes, c->N,
                       c->p.cell_deg * kPi / 180.0, ra0_deg * kPi / 180.0, dec0_deg * kPi / 180.0, morph, out);
    return hipGetLastError();
}

hipError_t launch_strongest_map(toi_ctx* c, const float* cube, int n_maps, const int32_t* boxes, int n_boxes,
                                int32_t* k_out) {
    if (n_boxes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_strongest_map, dim3(n_boxes), dim3(256), 0, c->stream, cube, n_maps, c->T, c->p.tile,
                       boxes, k_out);
    return hipGetLastError();
}

hipError_t launch_detect_cube(toi_ctx* c, const float* cube, int L, int t, int32_t* boxes, int max_boxes,
                              int32_t* n_boxes) {
    const int T = c->T;
    const size_t lds = 2 * (size_t)T * T * sizeof(int32_t);
    const size_t slds = (size_t)(L + L / 2 + 1) * sizeof(double);
    if (lds > 128 * 1024 || slds > 64 * 1024) return hipErrorNotSupported;
    StageTimer timer(c, TOI_STAGE_DETECT);
    hipLaunchKernelGGL(k_cube_scores, dim3(T * T), dim3(64), slds, c->stream, cube, L, T * T, c->det_scores);
    hipLaunchKernelGGL(k_detect, dim3(1), dim3(1024), lds, c->stream, nullptr, T, c->p.tile, t, c->det_scores,
                       c->det_boxes, boxes, max_boxes, n_boxes);
    return hipGetLastError();
}

hipError_t launch_detect(toi_ctx* c, const float* window, int t, int32_t* boxes, int max_boxes, int32_t* n_boxes) {
    const int T = c->T;
    const size_t lds = 2 * (size_t)T * T * sizeof(int32_t);
    if (lds > 128 * 1024) return hipErrorNotSupported;
    StageTimer timer(c, TOI_STAGE_DETECT);
    hipLaunchKernelGGL(k_detect, dim3(1), dim3(1024), lds, c->stream, window, T, c->p.tile, t, c->det_scores,
                       c->det_boxes, boxes, max_boxes, n_boxes);
    return hipGetLastError();
}

}  // namespace toi
