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
