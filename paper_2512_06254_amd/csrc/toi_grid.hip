// S4: gridding of the Chebyshev moment planes M_{p,k} (Section 3.4) with an
// exponential-of-semicircle kernel of support 8 on a periodic 2N x 2N grid.
//
// Tile-owner design, no global float atomics:
//  1. Work items are runs of kItemChans channels of one row.  A row's samples
//     lie on a radial track (b = uvw nu / c), so an item's 8 x 8 footprints
//     cover a small box; k_items computes the box and the slabs it touches and
//     counts the item into every (plane group, 32 x 32 tile) bin it overlaps.
//  2. k_bin_scan turns the counts into list offsets and occupancy bit masks;
//     k_bin_fill writes the item lists.
//  3. k_grid_tiles: one workgroup per (group, tile) accumulates the tile's
//     planes in LDS and writes it to HBM once.  Inside a workgroup each
//     wavefront walks one item at a time: lane (i, j) owns the cells with
//     x = i, y = j (mod 8), exactly one of which lies in every footprint, and
//     keeps that cell's plane values in registers until the track moves it
//     (Romein, ICS 2012), then adds them to LDS.
// Tiles without samples are never written; the FFT passes read the
// occupancy masks and treat them as zero.
//
// Coordinates are formed in FP64 (X = M/2 - r1 M Delta, Y = M/2 + r2 M Delta)
// and split into an integer cell and an FP32 offset before the kernel is
// evaluated; values and accumulation are FP32.
#include <algorithm>

#include "toi_device.h"
#include "toi_grid.h"
#include "toi_internal.h"

namespace toi {

__global__ __launch_bounds__(256) void k_fill_zero_i32(int32_t* __restrict__ p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------- 1. items
__global__ __launch_bounds__(256) void k_items(const double* __restrict__ uvw, const float* __restrict__ weight,
                                               const uint8_t* __restrict__ flag, const double* __restrict__ freq,
                                               int n_chan, int n_corr, uint32_t mask, int mode,
                                               const DevPlan* __restrict__ P, int M, int NT, double cell_rad,
                                               int n_items, ItemBox* __restrict__ items,
                                               int32_t* __restrict__ bin_count) {
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= n_items) return;
    const int n_chunks = (n_chan + kItemChans - 1) / kItemChans;
    const int r = item / n_chunks;
    const int c = (item % n_chunks) * kItemChans + lane;
    ItemBox box;
    box.tx0 = 1; box.tx1 = 0; box.ty0 = 1; box.ty1 = 0; box.g0 = 1; box.g1 = 0;
    box.pad_[0] = box.pad_[1] = 0;
    if (P->status) {
        if (lane == 0) items[item] = box;
        return;
    }
    const Track tr = row_track(uvw, r, P, M, cell_rad);
    double xlo = 1e300, xhi = -1e300, ylo = 1e300, yhi = -1e300, rlo = 1e300, rhi = -1e300;
    if (c < n_chan && sample_kept(weight, flag, ((size_t)r * n_chan + c) * n_corr, n_corr, mask)) {
        const double nu = freq[c];
        xlo = xhi = 0.5 * M + tr.ax * nu;
        ylo = yhi = 0.5 * M + tr.ay * nu;
        rlo = rhi = tr.a3 * nu;
    }
    xlo = wave_min(xlo); xhi = wave_max(xhi);
    ylo = wave_min(ylo); yhi = wave_max(yhi);
    rlo = wave_min(rlo); rhi = wave_max(rhi);
    if (xlo > xhi) {   // no kept sample
        if (lane == 0) items[item] = box;
        return;
    }
    // footprint cells [ceil(X - 4), ceil(X - 4) + 7] -> tiles (floor division)
    box.tx0 = ((int)ceil(xlo - 4.0)) >> 5;
    box.tx1 = ((int)ceil(xhi - 4.0) + 7) >> 5;
    box.ty0 = ((int)ceil(ylo - 4.0)) >> 5;
    box.ty1 = ((int)ceil(yhi - 4.0) + 7) >> 5;
    const int p0 = mode == 3 ? slab_index(rlo, P) : 0, p1 = mode == 3 ? slab_index(rhi, P) : 0;
    box.g0 = group_of_slab(min(p0, p1), P);
    box.g1 = group_of_slab(max(p0, p1), P) + (P->K > P->gp ? P->parts - 1 : 0);
    if (lane == 0) items[item] = box;
    // count into bins, lanes spread over the (group, tile) combinations
    const int nx = box.tx1 - box.tx0 + 1, ny = box.ty1 - box.ty0 + 1, ng = box.g1 - box.g0 + 1;
    const int tiles = NT * NT;
    for (int e = lane; e < nx * ny * ng; e += 64) {
        const int tx = (box.tx0 + e % nx) & (NT - 1);
        const int ty = (box.ty0 + (e / nx) % ny) & (NT - 1);
        const int g = box.g0 + e / (nx * ny);
        atomicAdd(&bin_count[(size_t)g * tiles + ty * NT + tx], 1);
    }
}

// ---------------------------------------------------------------- 2. scan
// One workgroup of 1024 threads: exclusive scan of the counts, bin cursors and
// occupancy masks (tile_bits[g][ty][tx/32], row_bits[g][ty/32]).
__global__ __launch_bounds__(1024) void k_bin_scan(const int32_t* __restrict__ count, int n_bins, int NT,
                                                   int bin_cap, DevPlan* __restrict__ P, int32_t* __restrict__ off,
                                                   int32_t* __restrict__ cursor, uint32_t* __restrict__ tile_bits,
                                                   uint32_t* __restrict__ row_bits, int32_t* __restrict__ order,
                                                   int32_t* __restrict__ n_active) {
    __shared__ int32_t part[1024];
    __shared__ int32_t hist[32];
    const int per = (n_bins + 1023) / 1024;
    const int b0 = min(n_bins, (int)threadIdx.x * per), b1 = min(n_bins, b0 + per);
    int s = 0;
    for (int i = b0; i < b1; ++i) s += count[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan of the partial sums
        const int v = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = part[threadIdx.x] - s;
    for (int i = b0; i < b1; ++i) {
        off[i] = run;
        cursor[i] = run;
        run += count[i];
    }
    if (threadIdx.x == 1023) {
        off[n_bins] = part[1023];
        if (part[1023] > bin_cap) atomicOr(&P->status, (uint32_t)TOI_STATUS_OVERFLOW);
    }
    // launch order of the non-empty bins: heaviest first, bucketed by floor(log2(count))
    if (threadIdx.x < 32) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int i = b0; i < b1; ++i)
        if (count[i] > 0) atomicAdd(&hist[31 - __clz(count[i])], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int b = 31; b >= 0; --b) {
            const int h = hist[b];
            hist[b] = acc;
            acc += h;
        }
        *n_active = acc;
    }
    __syncthreads();
    for (int i = b0; i < b1; ++i)
        if (count[i] > 0) order[atomicAdd(&hist[31 - __clz(count[i])], 1)] = i;
    // occupancy masks
    const int words = (NT + 31) / 32;
    const int n_groups = n_bins / (NT * NT);
    for (int w = threadIdx.x; w < n_groups * NT * words; w += blockDim.x) {
        const int g = w / (NT * words), ty = (w / words) % NT, wd = w % words;
        uint32_t bits = 0;
        for (int b = 0; b < 32 && wd * 32 + b < NT; ++b)
            if (count[(size_t)g * NT * NT + ty * NT + wd * 32 + b] > 0) bits |= 1u << b;
        tile_bits[w] = bits;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < n_groups * words; w += blockDim.x) {
        const int g = w / words, wd = w % words;
        uint32_t bits = 0;
        for (int b = 0; b < 32 && wd * 32 + b < NT; ++b) {
            const int ty = wd * 32 + b;
            uint32_t any = 0;
            for (int x = 0; x < words; ++x) any |= tile_bits[((size_t)g * NT + ty) * words + x];
            if (any) bits |= 1u << b;
        }
        row_bits[w] = bits;
    }
}

// ---------------------------------------------------------------- 2b. fill
__global__ __launch_bounds__(256) void k_bin_fill(const ItemBox* __restrict__ items, int n_items, int NT,
                                                  int bin_cap, int32_t* __restrict__ cursor,
                                                  int32_t* __restrict__ list) {
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= n_items) return;
    const ItemBox box = items[item];
    if (box.tx0 > box.tx1) return;
    const int nx = box.tx1 - box.tx0 + 1, ny = box.ty1 - box.ty0 + 1, ng = box.g1 - box.g0 + 1;
    const int tiles = NT * NT;
    for (int e = lane; e < nx * ny * ng; e += 64) {
        const int tx = (box.tx0 + e % nx) & (NT - 1);
        const int ty = (box.ty0 + (e / nx) % ny) & (NT - 1);
        const int g = box.g0 + e / (nx * ny);
        const int pos = atomicAdd(&cursor[(size_t)g * tiles + ty * NT + tx], 1);
        if (pos < bin_cap) list[pos] = item;
    }
}

// ---------------------------------------------------------------- 3. tiles
// LDS tile layout: planar real and imaginary parts, [plane][ly][swizzled lx],
// the column rotated by 8 (ly / 2 mod 4) so that the 64 cells of one 8 x 8
// footprint fall in distinct banks when they are added together.
__device__ inline int tile_index(int ly, int lx) { return ly * kTile + ((lx + 8 * ((ly >> 1) & 3)) & (kTile - 1)); }

// Variants (chosen by the autotuner): CELLS footprint cells per lane.  With
// CELLS = 1 all 64 lanes serve one sample, lane (i, j) owning x = i (mod 8),
// y = j (mod 8); with CELLS = 2 the two half-waves take alternate samples and
// lane (i, j) of a half owns x = i (mod 4) -- cells dx and dx + 4 -- and
// y = j (mod 8).  Each lane keeps its cells' plane values in registers until
// the track moves them (Romein, ICS 2012), then adds them to LDS.
template <int KACC, int CELLS>
__global__ __launch_bounds__(1024) void k_grid_tiles(
    const double* __restrict__ uvw, const float2* __restrict__ vis, const float* __restrict__ weight,
    const uint8_t* __restrict__ flag, const double* __restrict__ freq, const int32_t* __restrict__ ant1,
    const int32_t* __restrict__ ant2, const float2* __restrict__ gains, int n_ant, int n_chan, int n_corr,
    uint32_t mask, int mode, const DevPlan* __restrict__ P, int M, int NT, double cell_rad,
    const int32_t* __restrict__ bin_off, const int32_t* __restrict__ list, int bin_cap,
    const int32_t* __restrict__ order, const int32_t* __restrict__ n_active, float2* __restrict__ grid) {
    extern __shared__ float lds[];                      // re[gp][kTile*kTile], then im[gp][kTile*kTile]
    constexpr int TT = kTile * kTile;
    constexpr int XM = 8 / CELLS;                       // x residue modulus of a lane
    constexpr int SUBL = 64 / CELLS;                    // lanes per sample
    const int tiles = NT * NT;
    // Non-empty bins in decreasing order of work, dealt round-robin over the
    // XCDs by the dispatcher (tiles with samples cluster around the uv centre,
    // so contiguous ranges per XCD would leave most XCDs idle).
    if ((int)blockIdx.x >= *n_active) return;
    const int bid = order[blockIdx.x];
    const int g = bid / tiles, tile = bid % tiles;
    if (P->status & kStatusFatal) return;
    if (g >= P->ng) return;
    const int b0 = bin_off[(size_t)g * tiles + tile];
    const int b1 = min(bin_off[(size_t)g * tiles + tile + 1], bin_cap);
    if (b1 <= b0) return;
    int s0, s1, k0, k1;
    group_range(g, P, s0, s1, k0, k1);
    const int nk = k1 - k0;
    const int n_planes = (s1 - s0) * nk;
    float* lre = lds;
    float* lim = lds + P->gp * TT;
    for (int i = threadIdx.x; i < n_planes * TT; i += blockDim.x) { lre[i] = 0.f; lim[i] = 0.f; }
    __syncthreads();

    const int tx = tile % NT, ty = tile / NT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    const int sub = lane / SUBL, sl = lane % SUBL;
    const int li = sl % XM, lj = sl / XM;
    const double hM = 0.5 * M;
    const bool cheb = (mode == 3) && (P->dr3 > 0.0);
    const double dr3 = P->dr3, r3min = P->r3min;
    const int n_chunks = (n_chan + kItemChans - 1) / kItemChans;

    for (int it = b0 + wave; it < b1; it += n_waves) {
        const int item = list[it];
        const int r = item / n_chunks;
        const int c0 = (item % n_chunks) * kItemChans, c1 = min(n_chan, c0 + kItemChans);
        const Track trk = row_track(uvw, r, P, M, cell_rad);
        const float2 gr = row_gain(gains, ant1, ant2, n_ant, r);
        // lane-parallel prefetch: lane l prepares channel c0 + l (FP64 coordinates once per sample)
        int ix = 0, iy = 0, sp = 0;
        float ox = 0.f, oy = 0.f, vr0 = 0.f, vi0 = 0.f, ss = 0.f;
        bool act = false;
        {
            const int c = c0 + lane;
            if (c < c1) {
                float xr, xi;
                const float w =
                    sample_value(vis, weight, flag, ((size_t)r * n_chan + c) * n_corr, n_corr, mask, xr, xi);
                if (w > 0.f) {
                    const double nu = freq[c];
                    if (cheb) {
                        const double r3 = trk.a3 * nu;
                        sp = slab_index(r3, P);
                        ss = (float)((r3 - (r3min + (2 * sp + 1) * dr3)) / dr3);
                    }
                    const double X = hM + trk.ax * nu, Y = hM + trk.ay * nu;
                    const double fx0 = ceil(X - 4.0), fy0 = ceil(Y - 4.0);
                    ix = (int)fx0;
                    iy = (int)fy0;
                    ox = (float)(X - fx0);                 // in (3, 4]
                    oy = (float)(Y - fy0);
                    const int ddx = (ix - tx * kTile) & (M - 1), ddy = (iy - ty * kTile) & (M - 1);
                    act = (sp >= s0 && sp < s1) && (ddx < kTile || ddx >= M - 7) && (ddy < kTile || ddy >= M - 7);
                    vr0 = xr * gr.x - xi * gr.y;
                    vi0 = xr * gr.y + xi * gr.x;
                }
            }
        }
        uint64_t pending = __ballot(act);
        int cur_x = 0, cur_y = 0, cur_p = -1;
        bool in[CELLS];
        float ar[CELLS][KACC], ai[CELLS][KACC];
#pragma unroll
        for (int m = 0; m < CELLS; ++m) {
            in[m] = false;
#pragma unroll
            for (int k = 0; k < KACC; ++k) { ar[m][k] = 0.f; ai[m][k] = 0.f; }
        }

        auto flush = [&]() {
            const int ly = cur_y & (kTile - 1);
            const int base = (cur_p - s0) * nk * TT;
#pragma unroll
            for (int m = 0; m < CELLS; ++m) {
                if (!in[m]) continue;
                const int ci = base + tile_index(ly, (cur_x + m * XM) & (kTile - 1));
#pragma unroll
                for (int k = 0; k < KACC; ++k) {
                    if (k < nk) {
                        atomicAdd(lre + ci + k * TT, ar[m][k]);
                        atomicAdd(lim + ci + k * TT, ai[m][k]);
                    }
                }
            }
        };

        while (pending) {                               // wave-uniform walk, CELLS samples per step
            int qs[CELLS];
            bool have[CELLS];
#pragma unroll
            for (int m = 0; m < CELLS; ++m) {
                have[m] = pending != 0;
                qs[m] = have[m] ? __ffsll((unsigned long long)pending) - 1 : 0;
                if (have[m]) pending &= pending - 1;
            }
            bool mine = have[0];
            int qx = __builtin_amdgcn_readlane(ix, qs[0]), qy = __builtin_amdgcn_readlane(iy, qs[0]);
            int p = __builtin_amdgcn_readlane(sp, qs[0]);
            int bx = __builtin_amdgcn_readlane(__float_as_int(ox), qs[0]);
            int by = __builtin_amdgcn_readlane(__float_as_int(oy), qs[0]);
            int br = __builtin_amdgcn_readlane(__float_as_int(vr0), qs[0]);
            int bi = __builtin_amdgcn_readlane(__float_as_int(vi0), qs[0]);
            int bs = __builtin_amdgcn_readlane(__float_as_int(ss), qs[0]);
#pragma unroll
            for (int m = 1; m < CELLS; ++m) {
                if (sub == m) {
                    mine = have[m];
                    qx = __builtin_amdgcn_readlane(ix, qs[m]);
                    qy = __builtin_amdgcn_readlane(iy, qs[m]);
                    p = __builtin_amdgcn_readlane(sp, qs[m]);
                    bx = __builtin_amdgcn_readlane(__float_as_int(ox), qs[m]);
                    by = __builtin_amdgcn_readlane(__float_as_int(oy), qs[m]);
                    br = __builtin_amdgcn_readlane(__float_as_int(vr0), qs[m]);
                    bi = __builtin_amdgcn_readlane(__float_as_int(vi0), qs[m]);
                    bs = __builtin_amdgcn_readlane(__float_as_int(ss), qs[m]);
                }
            }
            if (!mine) continue;
            const float qox = __int_as_float(bx), qoy = __int_as_float(by);
            const float qvr = __int_as_float(br), qvi = __int_as_float(bi), s = __int_as_float(bs);
            const int dx = (li - qx) & (XM - 1), dy = (lj - qy) & 7;
            const int cx = qx + dx, cy = qy + dy;
            if (cx != cur_x || cy != cur_y || p != cur_p) {
                flush();
                cur_x = cx; cur_y = cy; cur_p = p;
                const bool yin = ((cy & (M - 1)) >> 5) == ty;
#pragma unroll
                for (int m = 0; m < CELLS; ++m) {
                    in[m] = yin && ((((cx + m * XM) & (M - 1)) >> 5) == tx);
#pragma unroll
                    for (int k = 0; k < KACC; ++k) { ar[m][k] = 0.f; ai[m][k] = 0.f; }
                }
            }
            bool any = false;
#pragma unroll
            for (int m = 0; m < CELLS; ++m) any |= in[m];
            if (!any) continue;
            const float wy = es_kernel(((float)dy - qoy) * 0.25f);
            float vr[CELLS], vi[CELLS];
#pragma unroll
            for (int m = 0; m < CELLS; ++m) {
                const float w = es_kernel(((float)(dx + m * XM) - qox) * 0.25f) * wy;
                vr[m] = w * qvr;
                vi[m] = w * qvi;
            }
            float t, tm1;
            cheb_start(s, k0, t, tm1);                  // t = T_{k0}(s), tm1 = T_{k0 - 1}(s)
#pragma unroll
            for (int k = 0; k < KACC; ++k) {
#pragma unroll
                for (int m = 0; m < CELLS; ++m) {
                    ar[m][k] += t * vr[m];
                    ai[m][k] += t * vi[m];
                }
                const float tn = 2.f * s * t - tm1;
                tm1 = t;
                t = tn;
            }
        }
        flush();
    }
    __syncthreads();
    // write the tile's planes (only the planes of this group)
    for (int i = threadIdx.x; i < n_planes * TT; i += blockDim.x) {
        const int pl = i / TT, cell = i % TT;
        const int ly = cell / kTile, lx = cell % kTile;
        const int pg = (s0 + pl / nk) * P->K + k0 + pl % nk;   // global plane index
        const int li2 = pl * TT + tile_index(ly, lx);
        grid[((size_t)pg * M + ty * kTile + ly) * M + tx * kTile + lx] = make_float2(lre[li2], lim[li2]);
    }
}

hipError_t launch_grid(toi_ctx* c, const toi_snapshot& s) {
    const toi_params& p = c->p;
    const int M = c->M, NT = c->NT;
    const double cell = p.cell_deg * kPi / 180.0;
    const int n_chunks = (p.n_chan + kItemChans - 1) / kItemChans;
    const int n_items = s.n_row * n_chunks;
    const int n_bins = c->NG_max * NT * NT;
    {
        StageTimer timer(c, TOI_STAGE_CLEAR);   // binning
        hipLaunchKernelGGL(k_fill_zero_i32, dim3(256), dim3(256), 0, c->stream, c->bin_count, n_bins);
        if (n_items > 0)
            hipLaunchKernelGGL(k_items, dim3((n_items + 3) / 4), dim3(256), 0, c->stream, s.uvw, s.weight, s.flag,
                               s.freq, p.n_chan, p.n_corr, p.corr_mask, p.mode, c->plan, M, NT, cell, n_items,
                               c->items, c->bin_count);
        hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, c->stream, c->bin_count, n_bins, NT, c->bin_cap,
                           c->plan, c->bin_off, c->bin_cursor, c->tile_bits, c->row_bits, c->bin_order,
                           c->scratch_i);
        if (n_items > 0)
            hipLaunchKernelGGL(k_bin_fill, dim3((n_items + 3) / 4), dim3(256), 0, c->stream, c->items, n_items, NT,
                               c->bin_cap, c->bin_cursor, c->bin_list);
    }
    if (n_items == 0) return hipGetLastError();
    StageTimer timer(c, TOI_STAGE_GRID);
    const int gp = (c->tuning & kTuneEightPlanes) ? 8 : kGroupPlanes;
    const size_t lds_bytes = (size_t)gp * kTile * kTile * 2 * sizeof(float);
    const int threads = (c->tuning & kTuneWide) ? 1024 : 512;
    const int kacc = std::min(c->kmax, gp);
    const bool two = (c->tuning & kTuneTwoCells) != 0;
    const int blocks = n_bins;
#define TOI_TILE_ARGS                                                                                         \
    dim3(blocks), dim3(threads), lds_bytes, c->stream, s.uvw, (const float2*)s.vis, s.weight, s.flag, s.freq,   \
        s.ant1, s.ant2, (const float2*)s.gains, p.n_ant, p.n_chan, p.n_corr, p.corr_mask, p.mode, c->plan, M, NT, \
        cell, c->bin_off, c->bin_list, c->bin_cap, c->bin_order, c->scratch_i, c->grid
#define TOI_TILE_LAUNCH(KA)                                        \
    do {                                                           \
        if (two)                                                   \
            hipLaunchKernelGGL((k_grid_tiles<KA, 2>), TOI_TILE_ARGS); \
        else                                                       \
            hipLaunchKernelGGL((k_grid_tiles<KA, 1>), TOI_TILE_ARGS); \
    } while (0)
    if (kacc <= 1)
        TOI_TILE_LAUNCH(1);
    else if (kacc <= 4)
        TOI_TILE_LAUNCH(4);
    else if (kacc <= 8)
        TOI_TILE_LAUNCH(8);
    else
        TOI_TILE_LAUNCH(16);
#undef TOI_TILE_LAUNCH
#undef TOI_TILE_ARGS
    return hipGetLastError();
}

}  // namespace toi
