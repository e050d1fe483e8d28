// S4: gridding of the Chebyshev moment planes M_{p,k} (Section 3.4) with an
// exponential-of-semicircle kernel of support 8 on a periodic 2N x 2N grid.
//
// Work distribution: one wavefront per (row, channel chunk).  A row's samples
// lie on a radial track (b = uvw nu / c), so consecutive channels land on
// nearby grid cells.  Lane (i, j) of the wavefront owns the cells with
// x = i and y = j modulo 8; for every sample exactly one cell of each lane's
// residue class lies inside the 8 x 8 footprint.  Each lane accumulates its
// current cell's K plane values in registers and adds them to the grid only
// when the track moves its cell (or slab), so one global atomic replaces many
// (Romein, ICS 2012, "An efficient work-distribution strategy for gridding
// radio-telescope data on GPUs").
//
// Coordinates are formed in FP64 (X = M/2 - r1 M Delta, Y = M/2 + r2 M Delta)
// and split into an integer cell and an FP32 offset before the kernel is
// evaluated; values and accumulation are FP32.
#include "toi_internal.h"
#include "toi_device.h"

namespace toi {

__global__ __launch_bounds__(256) void k_fill_zero(float4* __restrict__ p, size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int KMAX>
__global__ __launch_bounds__(256) void k_grid_tracks(
    const double* __restrict__ uvw, const float2* __restrict__ vis, const float* __restrict__ weight,
    const uint8_t* __restrict__ flag, const double* __restrict__ freq, const int32_t* __restrict__ ant1,
    const int32_t* __restrict__ ant2, const float2* __restrict__ gains, int n_ant, int n_row, int n_chan, int n_corr,
    uint32_t mask, int chunk, int mode, const DevPlan* __restrict__ plan, float2* __restrict__ grid, int M,
    double cell_rad) {
    const int lane = threadIdx.x & 63;
    const int n_chunks = (n_chan + chunk - 1) / chunk;
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int r = item / n_chunks;
    if (r >= n_row) return;
    if (plan->status) return;                 // nothing to grid: the planes stay zero
    const int c0 = (item % n_chunks) * chunk;
    const int c1 = min(n_chan, c0 + chunk);
    const int K = plan->K, ns = plan->n_slab;
    const double dr3 = plan->dr3, r3min = plan->r3min;
    const double u0 = uvw[3 * r], u1 = uvw[3 * r + 1], u2 = uvw[3 * r + 2];
    const double* V = plan->V;
    const double sc = (double)M * cell_rad / kCLight;
    const double ax = -(V[0] * u0 + V[1] * u1 + V[2] * u2) * sc;     // X = M/2 + ax nu
    const double ay = (V[3] * u0 + V[4] * u1 + V[5] * u2) * sc;      // Y = M/2 + ay nu
    const double a3 = (V[6] * u0 + V[7] * u1 + V[8] * u2) / kCLight; // r3 = a3 nu
    float2 g = make_float2(1.f, 0.f);
    if (gains) {   // an antenna index outside [0, n_ant) gives the row a zero gain
        const int a1 = ant1[r], a2 = ant2[r];
        if (a1 >= 0 && a1 < n_ant && a2 >= 0 && a2 < n_ant) {
            const float2 g1 = gains[a1], g2 = gains[a2];
            g = cmul(g1, make_float2(g2.x, -g2.y));
        } else {
            g = make_float2(0.f, 0.f);
        }
    }
    const int li = lane & 7, lj = lane >> 3;
    const double half = 0.5 * M;
    const bool cheb = (mode == 3) && (dr3 > 0.0);

    int cur_x = 0, cur_y = 0, cur_p = -1;
    float ar[KMAX], ai[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) { ar[k] = 0.f; ai[k] = 0.f; }

    auto flush = [&]() {
        const size_t cell = (size_t)(cur_y & (M - 1)) * M + (cur_x & (M - 1));
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < K) {
                float* dst = reinterpret_cast<float*>(grid + (size_t)(cur_p * K + k) * M * M + cell);
                unsafeAtomicAdd(dst, ar[k]);
                unsafeAtomicAdd(dst + 1, ai[k]);
            }
        }
    };

    for (int c = c0; c < c1; ++c) {
        const size_t base = ((size_t)r * n_chan + c) * n_corr;
        float w = 0.f, xr = 0.f, xi = 0.f;
        for (int k = 0; k < n_corr; ++k) {
            if (!((mask >> k) & 1u)) continue;
            float wk = weight ? weight[base + k] : 1.f;
            if (flag && flag[base + k]) wk = 0.f;
            const float2 v = vis[base + k];
            w += wk;
            xr += wk * v.x;
            xi += wk * v.y;
        }
        if (!(w > 0.f)) continue;
        const float vr0 = xr * g.x - xi * g.y, vi0 = xr * g.y + xi * g.x;
        const double nu = freq[c];
        const double X = half + ax * nu, Y = half + ay * nu;
        const double fx0 = ceil(X - 4.0), fy0 = ceil(Y - 4.0);
        const int ix0 = (int)fx0, iy0 = (int)fy0;
        const float ox = (float)(X - fx0), oy = (float)(Y - fy0);    // in (3, 4]
        const int dx = (li - ix0) & 7, dy = (lj - iy0) & 7;
        const int cx = ix0 + dx, cy = iy0 + dy;
        const float wgt = es_kernel(((float)dx - ox) * 0.25f) * es_kernel(((float)dy - oy) * 0.25f);
        int p = 0;
        float s = 0.f;
        if (cheb) {
            const double r3 = a3 * nu;
            p = (int)floor((r3 - r3min) / (2.0 * dr3));
            p = max(0, min(ns - 1, p));
            s = (float)((r3 - (r3min + (2 * p + 1) * dr3)) / dr3);
        }
        if (cx != cur_x || cy != cur_y || p != cur_p) {
            if (cur_p >= 0) flush();
            cur_x = cx; cur_y = cy; cur_p = p;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) { ar[k] = 0.f; ai[k] = 0.f; }
        }
        const float vr = wgt * vr0, vi = wgt * vi0;
        ar[0] += vr;
        ai[0] += vi;
        if (KMAX > 1) {
            float tm1 = 1.f, t = s;
#pragma unroll
            for (int k = 1; k < KMAX; ++k) {
                ar[k] += t * vr;
                ai[k] += t * vi;
                const float tn = 2.f * s * t - tm1;
                tm1 = t;
                t = tn;
            }
        }
    }
    if (cur_p >= 0) flush();
}

hipError_t launch_grid(toi_ctx* c, const toi_snapshot& s) {
    const toi_params& p = c->p;
    const size_t M = c->M;
    const size_t n4 = (size_t)c->P_cap * M * M * sizeof(float2) / sizeof(float4);
    {
        StageTimer timer(c, TOI_STAGE_CLEAR);
        hipLaunchKernelGGL(k_fill_zero, dim3(2048), dim3(256), 0, c->stream, (float4*)c->grid, n4);
    }
    if (s.n_row == 0) return hipGetLastError();
    StageTimer timer(c, TOI_STAGE_GRID);
    const int chunk = 64;
    const int n_chunks = (p.n_chan + chunk - 1) / chunk;
    const long items = (long)s.n_row * n_chunks;
    const int blocks = (int)((items + 3) / 4);
    const double cell = p.cell_deg * kPi / 180.0;
#define TOI_GRID_ARGS                                                                                  \
    dim3(blocks), dim3(256), 0, c->stream, s.uvw, (const float2*)s.vis, s.weight, s.flag, s.freq, s.ant1, \
        s.ant2, (const float2*)s.gains, p.n_ant, s.n_row, p.n_chan, p.n_corr, p.corr_mask, chunk, p.mode, c->plan,  \
        c->grid, (int)M, cell
    switch (c->kmax) {
        case 1: hipLaunchKernelGGL(k_grid_tracks<1>, TOI_GRID_ARGS); break;
        case 4: hipLaunchKernelGGL(k_grid_tracks<4>, TOI_GRID_ARGS); break;
        case 8: hipLaunchKernelGGL(k_grid_tracks<8>, TOI_GRID_ARGS); break;
        case 16: hipLaunchKernelGGL(k_grid_tracks<16>, TOI_GRID_ARGS); break;
        default: hipLaunchKernelGGL(k_grid_tracks<32>, TOI_GRID_ARGS); break;
    }
#undef TOI_GRID_ARGS
    return hipGetLastError();
}

}  // namespace toi
