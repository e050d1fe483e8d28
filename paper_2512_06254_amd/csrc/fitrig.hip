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
#include "toi_device.h"
#include "toi_internal.h"

namespace toi {

__global__ __launch_bounds__(256) void k_tlisi_tiles(const float* __restrict__ a, const float* __restrict__ b,
                                                     const float* __restrict__ c, int N, int tile,
                                                     TileStat* __restrict__ out) {
    __shared__ double red[8][4];
    const int T = N / tile;
    const int ty = blockIdx.x / T, tx = blockIdx.x % T;
    double sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0, mn = 1e300, mx = -1e300;
    const int n = tile * tile;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const size_t o = (size_t)(ty * tile + i / tile) * N + tx * tile + i % tile;
        const double va = a[o], vb = b[o], vc = c[o];
        const double X = vb - va, Y = vc - vb;
        sx += X; sy += Y; sxx += X * X; syy += Y * Y; sxy += X * Y;
        mn = fmin(mn, fmin(X, Y));
        mx = fmax(mx, fmax(X, Y));
    }
    sx = block_sum(sx, red[0]);
    sy = block_sum(sy, red[1]);
    sxx = block_sum(sxx, red[2]);
    syy = block_sum(syy, red[3]);
    sxy = block_sum(sxy, red[4]);
    mn = block_min(mn, red[5]);
    mx = block_max(mx, red[6]);
    if (threadIdx.x == 0) {
        TileStat s;
        s.sx = sx; s.sy = sy; s.sxx = sxx; s.syy = syy; s.sxy = sxy; s.mn = mn; s.mx = mx; s.pad_ = 0;
        out[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void k_tlisi_final(const TileStat* __restrict__ st, int n_tiles, int tile,
                                                     float* __restrict__ out) {
    __shared__ double red[2][4];
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
    for (int i = threadIdx.x; i < n_tiles; i += blockDim.x) {
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

hipError_t launch_tlisi(toi_ctx* c, const float* a, const float* b, const float* d, float* out) {
    const int T = c->T;
    StageTimer timer(c, TOI_STAGE_TLISI);
    hipLaunchKernelGGL(k_tlisi_tiles, dim3(T * T), dim3(256), 0, c->stream, a, b, d, c->N, c->p.tile, c->tiles);
    hipLaunchKernelGGL(k_tlisi_final, dim3(1), dim3(256), 0, c->stream, c->tiles, T * T, c->p.tile, out);
    return hipGetLastError();
}

}  // namespace toi

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
