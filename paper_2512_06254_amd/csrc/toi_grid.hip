// S4: gridding of the Chebyshev moment planes M_{p,k} (Section 3.4) with an
// exponential-of-semicircle kernel of support 8 on a periodic 2N x 2N grid.
//
// Tile-owner design, no float atomics on the grid:
//  1. Work items are runs of kItemChans channels of one row.  A row's samples
//     lie on a radial track (b = uvw nu / c), so an item's 8 x 8 footprints
//     cover a small box.  k_items writes each sample's gridding record (cell,
//     offsets, slab, value); k_item_bins computes the box and the slabs it
//     touches and counts the item into every (plane group, 8 x 8 tile) bin it
//     overlaps.
//  2. k_scan_local / k_scan_top / k_scan_apply turn the counts into list
//     offsets, a heaviest-first launch order and occupancy bit masks; k_units
//     splits the heaviest bins into work units of at most 2^unit_shift items;
//     k_bin_fill writes the item lists and k_bin_sort_* put every list in
//     increasing item order, so that the accumulation order, and the image,
//     is the same on every run.
//  3. k_grid_tiles_mfma: one wavefront per work unit keeps the whole tile in
//     matrix-core accumulators and writes it to HBM once (the units of a split
//     bin add their partial tiles in a fixed order first).
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

// ---------------------------------------------------------------- 1. items
// One wavefront per item; lane l writes the gridding record of channel c0 + l
// (FP64 coordinates split into a cell and FP32 offsets once per sample), and
// the item's largest value and extreme kept frequencies go to its ItemBox
// (k_item_bins derives the box and counts the bins from them).
// The counters the bin pass adds to: the bin counts and row words of the
// plan's plane groups (the scan treats the bins of the other groups as empty,
// whatever they hold) and the scan's bucket words, cleared by k_scan_clear
// before the record pass.  (Cleared by the record pass's own threads instead,
// that pass took 94 us against 88 + 4.5 for the two launches.)
struct BinClear {
    int32_t* count;
    int n_bins, tiles;
    int32_t* aux;
    uint32_t* row_bits;
    int n_row_words, words;
};
__device__ inline void clear_bins(const DevPlan* __restrict__ P, const BinClear& bc) {
    const int stride = gridDim.x * blockDim.x;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int ng = P->ng;
    const int nb = min(bc.n_bins, ng * bc.tiles), nw = min(bc.n_row_words, ng * bc.words);
    for (int i = t; i < nb; i += stride) bc.count[i] = 0;
    if (t < kAuxTotals) bc.aux[t] = 0;
    for (int i = t; i < nw; i += stride) bc.row_bits[i] = 0;
}

__global__ __launch_bounds__(256) void k_items(const double* __restrict__ uvw, const float2* __restrict__ vis,
                                               const float* __restrict__ weight, const uint8_t* __restrict__ flag,
                                               const double* __restrict__ freq, const int32_t* __restrict__ ant1,
                                               const int32_t* __restrict__ ant2, const float2* __restrict__ gains,
                                               int n_ant, int n_chan, int n_corr, uint32_t mask, int vec4,
                                               int mode, const DevPlan* __restrict__ P, int M, double cell_rad,
                                               int n_items, ItemBox* __restrict__ items, SampleRec* __restrict__ recs) {
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= n_items) return;
    const int n_chunks = (n_chan + kItemChans - 1) / kItemChans;
    const int r = item / n_chunks;
    const int c = (item % n_chunks) * kItemChans + lane;
    if (P->status) {
        if (lane == 0) {
            items[item].vmax = 0.f;
            items[item].nlo = 1e300;
            items[item].nhi = -1e300;
        }
        return;
    }
    const Track tr = row_track(uvw, r, P, M, cell_rad);
    // gridding record of this lane's sample
    bool kept = false;
    float vabs = 0.f;                  // max(|Re|, |Im|) of g x (the gridder's fp16 operand scale)
    if (c < n_chan) {
        float xr, xi;
        const float w = sample_value(vis, weight, flag, ((size_t)r * n_chan + c) * n_corr, n_corr, mask, xr, xi,
                                     vec4 != 0);
        SampleRec rec;
        rec.pk = -1;
        rec.sp = 0;
        rec.ox = rec.oy = 4.f;
        rec.ss = rec.vr = rec.vi = rec.pad_ = 0.f;
        if (w > 0.f) {
            kept = true;
            const double nu = freq[c];
            if (mode == 3 && P->dr3 > 0.0) {
                const double r3 = tr.a3 * nu;
                rec.sp = slab_index(r3, P);
                rec.ss = (float)div_by(r3 - (P->r3min + (2 * rec.sp + 1) * P->dr3), P->dr3, P->inv_dr3);
            }
            const double X = 0.5 * M + tr.ax * nu, Y = 0.5 * M + tr.ay * nu;
            const double fx0 = ceil(X - 4.0), fy0 = ceil(Y - 4.0);
            rec.pk = ((int)fx0 & (M - 1)) | (((int)fy0 & (M - 1)) << 13);
            rec.ox = (float)(X - fx0);
            rec.oy = (float)(Y - fy0);
            const float2 gr = row_gain(gains, ant1, ant2, n_ant, r);
            rec.vr = xr * gr.x - xi * gr.y;
            rec.vi = xr * gr.y + xi * gr.x;
            vabs = fmaxf(fabsf(rec.vr), fabsf(rec.vi));
        }
        float4* dst = reinterpret_cast<float4*>(recs + (size_t)r * n_chan + c);
        dst[0] = make_float4(__int_as_float(rec.pk), __int_as_float(rec.sp), rec.ox, rec.oy);
        dst[1] = make_float4(rec.ss, rec.vr, rec.vi, 0.f);
    }
    // the item's largest value (reduced over all items by the bin scan: no
    // atomic on one address per item)
    const float vmax = wave_max(vabs);
    // X, Y and r3 are linear in nu along the row: their extremes over the kept
    // channels sit at the extreme kept frequencies
    double nlo = 1e300, nhi = -1e300;
    if (kept) nlo = nhi = freq[c];
    nlo = wave_min(nlo);
    nhi = wave_max(nhi);
    if (lane == 0) {
        items[item].vmax = vmax;
        items[item].nlo = nlo;
        items[item].nhi = nhi;
    }
}

// Per item, kItemLanes lanes (eight items per wavefront): the track box of the
// kept samples from the extreme kept frequencies, and the item counted into
// every (plane group, tile) bin its footprints can touch.  The per-item work
// is the same for every lane of a group, so it was most of the record pass's
// instructions while that pass gave it a whole wavefront per item.
constexpr int kItemLanes = 8;
__global__ __launch_bounds__(256) void k_item_bins(const double* __restrict__ uvw, int n_chan, int mode,
                                                   const DevPlan* __restrict__ P, int M, int NT, int bsh, double cell_rad,
                                                   int n_items, ItemBox* __restrict__ items,
                                                   int32_t* __restrict__ bin_count) {
    const int item = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kItemLanes);
    if (item >= n_items) return;
    const bool writer = (threadIdx.x & (kItemLanes - 1)) == 0;
    const int n_chunks = (n_chan + kItemChans - 1) / kItemChans;
    const double nlo = items[item].nlo, nhi = items[item].nhi;
    ItemBox box;
    box.x0 = box.y0 = box.x1 = box.y1 = 0.0;
    box.ty0 = 1; box.ty1 = 0; box.g0 = 1; box.g1 = 0;
    box.inv_dy = 0.0;
    if (!P->status && nlo <= nhi) {
        const Track tr = row_track(uvw, item / n_chunks, P, M, cell_rad);
        box.x0 = 0.5 * M + tr.ax * nlo;
        box.x1 = 0.5 * M + tr.ax * nhi;
        box.y0 = 0.5 * M + tr.ay * nlo;
        box.y1 = 0.5 * M + tr.ay * nhi;
        // (an extent below 1e-9 cells counts as none: every row then takes the whole X range)
        box.inv_dy = fabs(box.y1 - box.y0) > 1e-9 ? 1.0 / (box.y1 - box.y0) : 0.0;
        const double ra = tr.a3 * nlo, rb = tr.a3 * nhi;
        const double ylo = fmin(box.y0, box.y1), yhi = fmax(box.y0, box.y1);
        // footprint rows [ceil(Y - 4), ceil(Y - 4) + 7] -> bin rows (floor division)
        box.ty0 = ((int)ceil(ylo - 1e-6 - 4.0)) >> bsh;
        box.ty1 = ((int)ceil(yhi + 1e-6 - 4.0) + 7) >> bsh;
        box.ty1 = min(box.ty1, box.ty0 + NT - 1);
        const int p0 = mode == 3 ? slab_index(fmin(ra, rb), P) : 0, p1 = mode == 3 ? slab_index(fmax(ra, rb), P) : 0;
        box.g0 = group_of_slab(p0, P);
        box.g1 = group_of_slab(p1, P) + (P->K > P->gp ? P->parts - 1 : 0);
    }
    if (writer) {   // the box fields (vmax, nlo, nhi stay as the record pass wrote them)
        ItemBox& o = items[item];
        o.x0 = box.x0; o.y0 = box.y0; o.x1 = box.x1; o.y1 = box.y1;
        o.ty0 = box.ty0; o.ty1 = box.ty1; o.g0 = box.g0; o.g1 = box.g1;
        o.inv_dy = box.inv_dy;
    }
    // count into bins (each row's tiles from the track)
    const int tiles = NT * NT;
    for_item_bins<kItemLanes>(box, NT, bsh, [&](int g, int ty, int tx) {
        atomicAdd(&bin_count[(size_t)g * tiles + ty * NT + tx], 1);
    });
}

// ---------------------------------------------------------------- 2. scan
// Three passes over the bin counts, kScanBlock bins per workgroup:
//  local: exclusive scan inside the workgroup, its total, and the global
//         histogram of non-empty bins by floor(log2(count)) with the work
//         units of each bucket;
//  top:   one workgroup scans the workgroup totals, writes the list length
//         (overflow check) and turns the histogram into bucket offsets,
//         heaviest bucket first;
//  apply: adds the workgroup offsets (bin offsets and cursors), lists the
//         non-empty bins in launch order (heaviest bucket first; order inside
//         a bucket is arbitrary) and writes the occupancy masks
//         tile_bits[g][ty][tx/32] and row_bits[g][ty/32].
// aux: layout kAux* (toi_internal.h).
constexpr int kScanPer = kScanBlock / 1024;

__global__ __launch_bounds__(256) void k_scan_clear(const DevPlan* __restrict__ P, BinClear bc) {
    clear_bins(P, bc);
}

__device__ inline int block_exclusive_scan(int v, int& total) {
    __shared__ int32_t wsum[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = 0;
    total = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    __syncthreads();
    return before + incl - v;
}

__global__ __launch_bounds__(1024) void k_scan_local(const int32_t* __restrict__ count, int n_bins,
                                                     const DevPlan* __restrict__ P, int tiles,
                                                     const ItemBox* __restrict__ items, int n_items,
                                                     int32_t* __restrict__ off, int32_t* __restrict__ aux) {
    __shared__ int32_t hist[32], hunits[32];
    __shared__ float red[16];
    {   // largest item value of this workgroup's share of the items
        const int per = (n_items + gridDim.x - 1) / gridDim.x;
        const int i0 = blockIdx.x * per, i1 = min(n_items, i0 + per);
        float v = 0.f;
        for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) v = fmaxf(v, items[i].vmax);
        v = block_max(v, red);
        if (threadIdx.x == 0) aux[kAuxTotals + gridDim.x + blockIdx.x] = __float_as_int(v);
    }
    if (blockIdx.x * kScanBlock >= P->ng * tiles) {   // bins of unused plane groups hold no items
        if (threadIdx.x == 0) aux[kAuxTotals + blockIdx.x] = 0;
        return;
    }
    if (threadIdx.x < 32) {
        hist[threadIdx.x] = 0;
        hunits[threadIdx.x] = 0;
    }
    const int ushift = P->unit_shift;
    const int n_live = min(n_bins, P->ng * tiles);   // bins of the plan's plane groups
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    int c[kScanPer], sum = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        c[j] = base + j < n_live ? count[base + j] : 0;
        sum += c[j];
    }
    int total;
    int run = block_exclusive_scan(sum, total);   // its barriers also order the hist clear
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        if (base + j < n_bins) off[base + j] = run;
        run += c[j];
        if (c[j] > 0) {
            const int k = 31 - __clz(c[j]);
            atomicAdd(&hist[k], 1);
            atomicAdd(&hunits[k], (c[j] + (1 << ushift) - 1) >> ushift);
        }
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        if (hist[threadIdx.x]) atomicAdd(&aux[kAuxBuckets + kAuxStride * threadIdx.x], hist[threadIdx.x]);
        if (hunits[threadIdx.x]) atomicAdd(&aux[kAuxUnits + kAuxStride * threadIdx.x], hunits[threadIdx.x]);
    }
    if (threadIdx.x == 0) aux[kAuxTotals + blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(int n_blocks, int n_bins, int bin_cap, DevPlan* __restrict__ P,
                                                   int32_t* __restrict__ aux, int32_t* __restrict__ off,
                                                   int32_t* __restrict__ n_active) {
    int carry = 0;
    for (int b0 = 0; b0 < n_blocks; b0 += 1024) {
        const int b = b0 + (int)threadIdx.x;
        const int v = b < n_blocks ? aux[kAuxTotals + b] : 0;
        int total;
        const int ex = block_exclusive_scan(v, total);
        if (b < n_blocks) aux[kAuxTotals + b] = carry + ex;
        carry += total;
    }
    __shared__ float red[16];
    float v = 0.f;   // the snapshot's largest value, from the scan workgroups' partial maxima
    for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) v = fmaxf(v, __int_as_float(aux[kAuxTotals + n_blocks + b]));
    v = block_max(v, red);
    if (threadIdx.x == 0) {
        P->vmax_bits = __float_as_uint(v);
        off[n_bins] = carry;
        if (carry > bin_cap) atomicOr(&P->status, (uint32_t)TOI_STATUS_OVERFLOW);
        int acc = 0;
        for (int k = 31; k >= 0; --k) {
            aux[kAuxCursors + kAuxStride * k] = acc;
            acc += aux[kAuxBuckets + kAuxStride * k];
        }
        *n_active = acc;
    }
}

__global__ __launch_bounds__(1024) void k_scan_apply(const int32_t* __restrict__ count, int n_bins, int NT, int bsh,
                                                     int32_t* __restrict__ off, int32_t* __restrict__ cursor,
                                                     int32_t* __restrict__ order, int32_t* __restrict__ aux,
                                                     uint32_t* __restrict__ tile_bits,
                                                     uint32_t* __restrict__ row_bits,
                                                     const DevPlan* __restrict__ P) {
    // NT bins of 2^bsh cells per axis; the masks are per kTile x kTile tile,
    // sub x sub mask tiles per bin (sub = 1 or 2; with sub = 2 at least 16
    // bins per axis).  The workgroup's bins are whole bin rows (NT and
    // kScanBlock are powers of two, NT <= kScanBlock): the occupancy words of
    // their mask rows, at most 512 (one per row when there are fewer than 32
    // mask tiles per row), are gathered in LDS from the counts already loaded,
    // and so are the rows' row_bits words, at most 64 (one per plane group
    // when there are fewer than 32 mask tiles per row, at most 4096 / 8 / 8
    // groups), added with one global atomic per word (an atomic per non-empty
    // tile word on a handful of shared words serialised the workgroups: 33 us
    // per snapshot).
    constexpr int kMaxWords = kScanBlock / 8, kMaxRowWords = kScanBlock / 64;
    __shared__ int32_t hist[32], start[32];
    __shared__ uint32_t tbs[kMaxWords], rbs[kMaxRowWords];
    const int tiles = NT * NT;
    if (blockIdx.x * kScanBlock >= P->ng * tiles) return;   // unused plane groups: never read
    const int sub = 1 << (bsh - kTileShift), NTm = NT * sub;  // mask tiles per bin side, per axis
    const int words = (NTm + 31) / 32;
    const int row0 = blockIdx.x * (kScanBlock / NT);        // the workgroup's bin rows [row0, row0 + nrows)
    const int nrows = min(kScanBlock / NT, n_bins / NT - row0);
    const int mrow0 = row0 * sub;                           // and mask rows [mrow0, mrow0 + nrows sub)
    const int nwords = nrows * sub * words;                 // tile_bits words of those rows (contiguous)
    const int wbase = (mrow0 / NTm) * words + ((mrow0 % NTm) >> 5);   // first row_bits word
    if (threadIdx.x < 32) hist[threadIdx.x] = 0;
    if (threadIdx.x < kMaxRowWords) rbs[threadIdx.x] = 0;
    for (int w = threadIdx.x; w < nwords; w += blockDim.x) tbs[w] = 0;
    __syncthreads();
    const int add = aux[kAuxTotals + blockIdx.x];
    const int n_live = min(n_bins, P->ng * tiles);   // bins of the plan's plane groups
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    int c[kScanPer];
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        c[j] = 0;
        if (base + j < n_bins) {
            c[j] = base + j < n_live ? count[base + j] : 0;
            const int o = off[base + j] + add;
            off[base + j] = o;
            cursor[base + j] = o;
            if (c[j] > 0) {
                atomicAdd(&hist[31 - __clz(c[j])], 1);
                const int r = (base + j) / NT, tx = (base + j) % NT;   // global bin row, column
                const int g = r / NT, ty = r % NT;
                const uint32_t cols = ((1u << sub) - 1u) << ((tx * sub) & 31);   // one word (sub <= 2)
                for (int a = 0; a < sub; ++a) {                        // mask rows r sub + a = g NTm + ty sub + a
                    atomicOr(&tbs[(r * sub + a - mrow0) * words + ((tx * sub) >> 5)], cols);
                    const int mty = ty * sub + a;
                    atomicOr(&rbs[g * words + (mty >> 5) - wbase], 1u << (mty & 31));
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        const int h = hist[threadIdx.x];
        start[threadIdx.x] = h ? atomicAdd(&aux[kAuxCursors + kAuxStride * threadIdx.x], h) : 0;
        hist[threadIdx.x] = 0;
    }
    for (int w = threadIdx.x; w < nwords; w += blockDim.x) tile_bits[(size_t)mrow0 * words + w] = tbs[w];
    if (threadIdx.x < kMaxRowWords && rbs[threadIdx.x]) atomicOr(&row_bits[wbase + threadIdx.x], rbs[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanPer; ++j)
        if (c[j] > 0) {
            const int k = 31 - __clz(c[j]);
            order[start[k] + atomicAdd(&hist[k], 1)] = base + j;
        }
}

// Work units of the matrix-core passes (one workgroup).  The bins of the
// heaviest buckets are listed unit by unit, ceil(count / U) units each
// (U = 2^unit_shift items, from the tuning): every bucket from the top down to
// unit_shift (at least U items per bin) while the units of the buckets taken
// fit in max_units (kSplitSlots partial tiles of 8 x 8 cells: a quarter as
// many units of 16 x 16 bins).
// The cut falls between whole buckets, so which bins are split depends only on
// the bin counts, not on the order of the bins inside a bucket; the bins of
// the buckets below the cut run whole.  The split bins are the first entries
// of the launch order (heaviest bucket first).  cnt[1] = units listed,
// cnt[2] = bins they cover.
__global__ __launch_bounds__(1024) void k_units(const DevPlan* __restrict__ P, const int32_t* __restrict__ count,
                                                const int32_t* __restrict__ order, const int32_t* __restrict__ aux,
                                                int max_units, int4* __restrict__ units, int32_t* __restrict__ cnt) {
    const int ushift = P->unit_shift, U = 1 << ushift;
    int n_big = 0, n_units = 0;
    for (int k = 31; k >= ushift; --k) {       // uniform over the workgroup
        const int u = aux[kAuxUnits + kAuxStride * k];
        if (n_units + u > max_units) break;
        n_units += u;
        n_big += aux[kAuxBuckets + kAuxStride * k];
    }
    int carry = 0;
    for (int i0 = 0; i0 < n_big; i0 += 1024) {
        const int i = i0 + (int)threadIdx.x;
        int bin = 0, u = 0;
        if (i < n_big) {
            bin = order[i];
            u = (count[bin] + U - 1) >> ushift;
        }
        int total;
        const int p0 = carry + block_exclusive_scan(u, total);   // barriers inside
        for (int p = 0; p < u; ++p) units[p0 + p] = make_int4(bin, p, u, p0);
        carry += total;
    }
    if (threadIdx.x == 0) {
        cnt[1] = carry;
        cnt[2] = n_big;
    }
}

// ---------------------------------------------------------------- 2b. fill
// kFillLanes lanes per item: an item has about five bins, and the fill is
// bound by the latency of its returned atomics, so a wavefront serves eight
// items at once (one item per wavefront: 43 us per MeerKAT-shaped snapshot,
// four: 22 us, eight: 20.5 us).
constexpr int kFillLanes = 8;
__global__ __launch_bounds__(256) void k_bin_fill(const ItemBox* __restrict__ items, int n_items, int NT, int bsh,
                                                  int bin_cap, int32_t* __restrict__ cursor,
                                                  int32_t* __restrict__ list) {
    const int item = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kFillLanes);
    if (item >= n_items) return;
    const ItemBox box = items[item];
    const int tiles = NT * NT;
    for_item_bins<kFillLanes>(box, NT, bsh, [&](int g, int ty, int tx) {   // the same bins as the count in k_item_bins
        const int pos = atomicAdd(&cursor[(size_t)g * tiles + ty * NT + tx], 1);
        if (pos < bin_cap) list[pos] = item;
    });
}

// ---------------------------------------------------------------- 2c. order
// The fill leaves each bin's items in the order of the atomic cursor; k_bin_sort
// sorts every bin's list into increasing item order (the items of a
// bin are distinct).  Bins of buckets below kBlockSortShift (fewer than 256
// items; the launch order's entries from the heaviest buckets' total on) are
// sorted by a bitonic network across the lanes: one wavefront per bin of 16 or
// more items (four values per lane from 64 items), 16 lanes per bin below
// that.  The others (the first entries of the launch order) by one workgroup each: a
// bitonic network whose every comparison puts the smaller value at the lower
// index (the first substage of each merge compares mirrored positions), so a
// list of any length sorts as if padded to a power of two with values larger
// than every item, and the padding is never stored.  Up to kSortLds items the
// list is sorted in LDS; longer lists in place in HBM (each substage a pass
// over the list, the workgroup's barrier between passes).
// Non-empty bins of the buckets lo .. hi - 1 (floor(log2(count))).
__device__ inline int bucket_bins(const int32_t* __restrict__ aux, int lo, int hi) {
    int n = 0;
    for (int k = lo; k < hi; ++k) n += aux[kAuxBuckets + kAuxStride * k];
    return n;
}

// Bitonic network over aligned groups of W lanes, ascending; every lane of
// the wavefront runs it (each group sorts its own values).
template <int W>
__device__ inline int sort_lanes(int v) {
    const int l = threadIdx.x & (W - 1);
#pragma unroll
    for (int k = 2; k <= W; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int o = __shfl_xor(v, j, W);
            const bool keep_min = ((l & j) == 0) == ((l & k) == 0);
            v = keep_min ? min(v, o) : max(v, o);
        }
    }
    return v;
}

// Bitonic network over 64 S values held S per lane (value s 64 + lane in
// v[s]), ascending: partners within a slot by lane shuffles, partners 64 or
// more apart by register exchange.
template <int S>
__device__ inline void sort_wave_slots(int (&v)[S]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 2; k <= 64 * S; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            int o[S];
#pragma unroll
            for (int s = 0; s < S; ++s) o[s] = j >= 64 ? v[s ^ (j >> 6)] : __shfl_xor(v[s], j, 64);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int e = s * 64 + lane;
                const bool keep_min = ((e & j) == 0) == ((e & k) == 0);
                v[s] = keep_min ? min(v[s], o[s]) : max(v[s], o[s]);
            }
        }
    }
}

// Bins of 64 to 255 items one per wavefront, four values per lane; bins of
// 16 to 63 items one per wavefront; bins of fewer than 16 items four per
// wavefront (16 lanes each): the pass is bound by the latency of its loads,
// and most bins hold a few items.
__device__ inline void sort_small_bins(const int32_t* __restrict__ order, const int32_t* __restrict__ n_active,
                                       const int32_t* __restrict__ aux, const int32_t* __restrict__ off,
                                       int32_t* __restrict__ list) {
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int n_act = *n_active;
    const int first = bucket_bins(aux, kBlockSortShift, 32);
    const int big_end = first + bucket_bins(aux, kSortShift, kBlockSortShift);
    const int mid_end = big_end + bucket_bins(aux, 4, kSortShift);
    for (int ob = first + wave; ob < big_end; ob += waves) {   // 64 .. 255 items
        const int bin = order[ob];
        const int b0 = off[bin], n = off[bin + 1] - b0;
        int v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = q * 64 + lane < n ? list[b0 + q * 64 + lane] : INT_MAX;
        sort_wave_slots<4>(v);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q * 64 + lane < n) list[b0 + q * 64 + lane] = v[q];
    }
    for (int ob = big_end + wave; ob < mid_end; ob += waves) {   // 16 .. 63 items
        const int bin = order[ob];
        const int b0 = off[bin], n = off[bin + 1] - b0;
        const int v = sort_lanes<64>(lane < n ? list[b0 + lane] : INT_MAX);
        if (lane < n) list[b0 + lane] = v;
    }
    const int l16 = lane & 15;
    for (int ob = mid_end + 4 * wave + (lane >> 4); ob - (lane >> 4) < n_act; ob += 4 * waves) {   // below 16
        const bool have = ob < n_act;
        const int bin = have ? order[ob] : 0;
        const int b0 = have ? off[bin] : 0, n = have ? off[bin + 1] - b0 : 0;
        const int v = sort_lanes<16>(l16 < n ? list[b0 + l16] : INT_MAX);
        if (l16 < n) list[b0 + l16] = v;
    }
}

// The bitonic network of sort_heavy_bins over a[0 .. n): substage (k, j) =
// (2^lk, 2^lj) compares the pair (i, l) of every t < P2 / 2 (shifts and
// masks: all sizes are powers of two).  In LDS (kWaveLocal), a substage whose
// pairs stay inside aligned blocks of 128 elements (j <= 64, or the mirrored
// first substage of k <= 128) touches only the elements of its wavefront's
// own pairs (thread t of wavefront w: elements 128 w + 2048 r + 0..127), so
// between two such substages the wavefront orders its own LDS accesses
// instead of waiting for the workgroup.
template <bool kWaveLocal, typename Buf>
__device__ inline void sort_network(Buf a, int n) {
    int P2 = 1, lp = 0;
    while (P2 < n) {
        P2 <<= 1;
        ++lp;
    }
    const int nt = blockDim.x;
    auto local = [](int lk, int lj) { return lj == lk - 1 ? lk <= 7 : lj <= 6; };
    for (int lk = 1; lk <= lp; ++lk) {
        for (int lj = lk - 1; lj >= 0; --lj) {
            const int j = 1 << lj;
            for (int t = threadIdx.x; t < P2 / 2; t += nt) {
                const int blk = t >> lj, o = t & (j - 1);
                int i, l;
                if (lj == lk - 1) {   // mirrored pair of the k-block
                    i = (blk << lk) + o;
                    l = (blk << lk) + (1 << lk) - 1 - o;
                } else {
                    i = (blk << (lj + 1)) + o;
                    l = i + j;
                }
                if (l < n) {
                    const int x = a[i], y = a[l];
                    if (x > y) {
                        a[i] = y;
                        a[l] = x;
                    }
                }
            }
            const int nk = lj > 0 ? lk : lk + 1, nj = lj > 0 ? lj - 1 : lk;   // the next substage
            if (kWaveLocal && nk <= lp && local(lk, lj) && local(nk, nj))
                lds_order();
            else
                __syncthreads();
        }
    }
}

__device__ inline void sort_heavy_bins(const int32_t* __restrict__ order, const int32_t* __restrict__ aux,
                                       const int32_t* __restrict__ off, int32_t* __restrict__ list, int32_t* s) {
    const int n_heavy = bucket_bins(aux, kBlockSortShift, 32);   // 256 items and more
    for (int ob = blockIdx.x; ob < n_heavy; ob += gridDim.x) {
        const int bin = order[ob];
        const int b0 = off[bin], n = off[bin + 1] - b0;
        if (n <= kSortLds) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] = list[b0 + i];
            __syncthreads();
            sort_network<true>(s, n);
            for (int i = threadIdx.x; i < n; i += blockDim.x) list[b0 + i] = s[i];
        } else {
            sort_network<false>(list + b0, n);
        }
        __syncthreads();   // the write-back precedes the next bin's loads into LDS
    }
}

// Both sorts in one launch (one launch each cost about 4 us more): every
// workgroup first takes its share of the heavy bins, then each of its
// wavefronts its share of the others.
__global__ __launch_bounds__(1024) void k_bin_sort(const DevPlan* __restrict__ P, const int32_t* __restrict__ order,
                                                   const int32_t* __restrict__ n_active,
                                                   const int32_t* __restrict__ aux,
                                                   const int32_t* __restrict__ off, int32_t* __restrict__ list) {
    __shared__ int32_t s[kSortLds];
    if (P->status & kStatusFatal) return;
    sort_heavy_bins(order, aux, off, list, s);
    sort_small_bins(order, n_active, aux, off, list);
}

// ---------------------------------------------------------------- 3. tiles, matrix cores

// Matrix-core gridder.  Tiles are 8 x 8 cells: the tile's 64 cells are the
// rows, the group's planes (order, slab) x {Re, Im} the columns.  The
// contribution of one sample to the tile is the outer product of its kernel
// weights at the 64 cells (zero outside its footprint) and the values
// T_k(s) Re(g x), T_k(s) Im(g x) of the planes of its slab (zero for the
// group's other planes); the tile is the product A B of the weights A (64
// cells x samples) and the values B (samples x NCOL).  NCOL = 32 (16
// planes): v_mfma_f32_32x32x16_f16 on two 32-row halves, 16 samples per
// instruction, each operand an FP32 product split as hi + lo in fp16 by
// fused multiply-adds that round to fp16 (hi = f16(a b), lo = f16(a b - hi),
// about 22 significant bits), and A B formed as Ah Bh + Ah Bl + Al Bh
// (products exact in FP32, the dropped Al Bl about 2^-22 relative),
// accumulated in FP32; the values g x are scaled by an exact power of two
// that puts the snapshot's largest |Re|, |Im| in [2^13, 2^14) (fp16 range;
// the weights lie in [0, 1]) and the tile is scaled back at the write-out.
// The half-precision matrix cores run beside the vector ALU, where FP32
// matrix instructions would share it.
// NCOL = 16 (8 planes): one v_mfma_f32_16x16x1f32 (four 16 x 16 blocks) per
// sample.  The accumulators hold the whole tile in registers: no LDS
// accumulation, no atomics, nothing to flush.  Lane l
// supplies the weight of cell (l mod 8, l / 8) (A operand) and column
// l mod NCOL (B operand); accumulator register r of lane l then holds cell
// (4 (l / 32) + r mod 4, r / 4) (NCOL = 32) or (4 ((l / 16) mod 2) + r mod 4,
// 2 (r / 4) + l / 32) (NCOL = 16), column l mod NCOL (hardware output layout).
// One wavefront per tile.  The samples come as gridding records written by
// k_items (cell, offsets, slab, Chebyshev argument, g x); each next item's
// records are loaded during the current walk.  LDS: staging of the item's
// active samples, compacted (kernel weights at the tile's eight columns and
// eight rows, zero outside the footprint, the NPL Chebyshev values and g x,
// which is 0 in the padding slots; B =
// T_k Re/Im(g x) is formed in the walk, which keeps the staging at 8.5 KB per
// wave), then the write-out buffer.
template <int NCOL>
__global__ __launch_bounds__(64, NCOL == 32 ? 3 : 5) void k_grid_tiles_mfma(
    const SampleRec* __restrict__ recs, int n_chan, const DevPlan* __restrict__ P, int M, int NT,
    const int32_t* __restrict__ bin_off, const int32_t* __restrict__ list, int bin_cap,
    const int32_t* __restrict__ order, const int32_t* __restrict__ cnt, const int4* __restrict__ units,
    float* __restrict__ split_part, float2* __restrict__ grid) {
    static_assert(NCOL == 16 || NCOL == 32, "one 16- or 32-column matrix block");
    static_assert(kTile == 8, "a tile is one 64-row matrix block");
    constexpr int NREG = NCOL;                 // accumulator registers per lane (64 x NCOL / 64)
    constexpr int NPL = NCOL / 2;              // planes per block
    constexpr int kQuad = NCOL == 32 ? 16 : 4; // samples per step of the walk
    typedef float acc_t __attribute__((ext_vector_type(NREG)));
    typedef float f32x16 __attribute__((ext_vector_type(16)));
    auto ld8 = [](const float* p, float* o) __attribute__((always_inline)) {
        const float4 u = reinterpret_cast<const float4*>(p)[0], w = reinterpret_cast<const float4*>(p)[1];
        o[0] = u.x; o[1] = u.y; o[2] = u.z; o[3] = u.w; o[4] = w.x; o[5] = w.y; o[6] = w.z; o[7] = w.w;
    };
    extern __shared__ float lds[];
    const int tiles = NT * NT;
    if (P->status & kStatusFatal) return;
    // staging rows of 64 sample slots (the item's active samples, compacted);
    // four consecutive slots are one 16-byte read.  Rows that different lanes
    // of one read access (x weights, Chebyshev values) are padded to 68
    // floats so that they fall in different banks.
    // (A read of slots 64 .. 67 of a 64-float row lands in the next region.)
    float* sx = lds;                           // 8 rows x 68: kernel weight at tile column i
    float* sy = sx + 8 * 68;                   // 8 rows x 64: kernel weight at tile row i
    float* sV = sy + 8 * 64;                   // 2 rows x 64: Re, Im of g x
    float* sT = sV + 2 * 64;                   // NPL rows x 68: T_{k0 + k}(s)
    const int lane = threadIdx.x;
    const int n_chunks = (n_chan + kItemChans - 1) / kItemChans;
    const int col = lane & (NCOL - 1);
    // fp16 scale of the values (NCOL = 32): 2^(14 - e) for max |g x| = m 2^e,
    // m in [0.5, 1); exact in both directions
    float vs = 1.f, ivs = 1.f;
    if constexpr (NCOL == 32) {
        const float vmax = __uint_as_float(P->vmax_bits);
        if (vmax > 0.f) {
            int ex;
            (void)frexpf(vmax, &ex);
            ex = min(max(ex, -100), 127);
            vs = ldexpf(1.f, 14 - ex);
            ivs = ldexpf(1.f, ex - 14);
        }
    }
    // work units (heavy bins split) in decreasing order of work; normally one
    // per workgroup, handed out by the dispatcher as waves finish
    const int n_units = work_unit_count(cnt);
    for (int ob = blockIdx.x; ob < n_units; ob += gridDim.x) {
    const WorkUnit un = work_unit(ob, units, order, cnt);
    const int bid = un.bin;
    const int g = bid / tiles, tile = bid % tiles;
    if (g >= P->ng) continue;
    int b0, b1;
    work_unit_items(un, bin_off, bin_cap, P->unit_shift, b0, b1);
    if (b1 <= b0 && un.parts == 1) continue;   // every unit of a split bin reports in
    int s0, s1, k0, k1;
    group_range(g, P, s0, s1, k0, k1);         // one slab per group (max_sg = 1)
    const int nk = k1 - k0;                    // <= gp <= NPL planes
    const int tx = tile % NT, ty = tile / NT;
    acc_t acc = {};
    f32x16 acc_lo = {}, acc_hi = {};            // NCOL = 32: cells 0..31, 32..63

    // gridding records, loaded two items ahead (a walk is shorter than the
    // latency of HBM)
    auto load_rec = [&](int item_, float4& ra, float4& rb) __attribute__((always_inline)) {
        const int c = (item_ % n_chunks) * kItemChans + lane;
        if (c < n_chan) {
            const float4* src = reinterpret_cast<const float4*>(recs + (size_t)(item_ / n_chunks) * n_chan + c);
            ra = src[0];
            rb = src[1];
        } else {
            ra = make_float4(__int_as_float(-1), 0.f, 4.f, 4.f);
            rb = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    float4 ra, rb, ra2, rb2;
    if (b0 < b1) load_rec(list[b0], ra, rb);
    if (b0 + 1 < b1) load_rec(list[b0 + 1], ra2, rb2);
    for (int it = b0; it < b1; ++it) {
        const int pk = __float_as_int(ra.x), sp = __float_as_int(ra.y);
        const int ix = pk & 8191, iy = (pk >> 13) & 8191;
        const float ox = ra.z, oy = ra.w, ss = rb.x, vr = rb.y, vi = rb.z;
        const int ddx = (ix - tx * kTile) & (M - 1), ddy = (iy - ty * kTile) & (M - 1);
        const bool act = pk >= 0 && (sp >= s0 && sp < s1) && (ddx < kTile || ddx >= M - 7) &&
                         (ddy < kTile || ddy >= M - 7);
        ra = ra2;
        rb = rb2;
        if (it + 2 < b1) load_rec(list[it + 2], ra2, rb2);   // the records two items ahead
        const uint64_t amask = __ballot(act);
        if (amask == 0) continue;
        // the active samples take slots 0 .. n_act - 1; the walk takes kQuad
        // slots at a time, so inactive lanes fill the slots up to n4 with zeros
        const int n_act = __popcll(amask), n4 = (n_act + kQuad - 1) & ~(kQuad - 1);
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(amask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)amask, 0));
        const int q = act ? below : n_act + (lane - below);
        if (q < n4) {
            // A padding slot (inactive lane) gets g x = 0, which zeroes its B
            // row; its other fields are made finite and are otherwise unused.
            // Chebyshev orders past the group's (k >= nk) fill B columns whose
            // sums are never written out.
            const float oxa = act ? ox : 0.f, oya = act ? oy : 0.f, ssa = act ? ss : 0.f;
            // weights at the tile's columns / rows i = 0..7 (0 outside the footprint)
            float wxy[16];
            tile_axis_weights(tx * kTile, ix, oxa, M, wxy);
            tile_axis_weights(ty * kTile, iy, oya, M, wxy + 8);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                sx[r * 68 + q] = wxy[r];
                sy[r * 64 + q] = wxy[8 + r];
            }
            // Chebyshev values T_{k0 + k}(s) of the group's orders, and g x
            float t, tm1;
            cheb_start(ssa, k0, t, tm1);
#pragma unroll
            for (int k = 0; k < NPL; ++k) {
                sT[k * 68 + q] = t;
                const float tn = 2.f * ssa * t - tm1;
                tm1 = t;
                t = tn;
            }
            sV[q] = act ? vr * vs : 0.f;
            sV[64 + q] = act ? vi * vs : 0.f;
        }
        lds_order();                                        // staging writes precede the walk's reads
        // this lane's operands: A = weight of cell (lane mod 8, lane / 8);
        // B = column c = lane mod NCOL: order k0 + c mod NPL, Re (c < NPL) or Im
        if constexpr (NCOL == 32) {
            // fp16 matrix cores, 16 samples per instruction: each product a b
            // = hi + lo in fp16, and A B = Ah Bh + Ah Bl + Al Bh.
            // Lane l: rows (cells) l mod 32 and 32 + l mod 32 of A, column
            // l mod 32 of B, samples 8 (l / 32) .. + 7 of the group.
            const int h = lane >> 5, c = lane & 31;
            const float* px = sx + (c & 7) * 68 + 8 * h;
            const float* py = sy + (c >> 3) * 64 + 8 * h;
            const float* pt = sT + (c & 15) * 68 + 8 * h;
            const float* pv = sV + (c >> 4) * 64 + 8 * h;
            for (int q0 = 0; q0 < n4; q0 += 16) {
                float x[8], y0[8], y1[8], t[8], v[8];
                ld8(px + q0, x);
                ld8(py + q0, y0);
                ld8(py + 4 * 64 + q0, y1);
                ld8(pt + q0, t);
                ld8(pv + q0, v);
                f16x8_t a0h, a0l, a1h, a1l, bh, bl;
                split_prod_f16x8(x, y0, a0h, a0l);
                split_prod_f16x8(x, y1, a1h, a1l);
                split_prod_f16x8(t, v, bh, bl);
                acc_lo = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0l, bh, acc_lo, 0, 0, 0);
                acc_hi = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1l, bh, acc_hi, 0, 0, 0);
                acc_lo = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0h, bl, acc_lo, 0, 0, 0);
                acc_hi = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1h, bl, acc_hi, 0, 0, 0);
                acc_lo = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0h, bh, acc_lo, 0, 0, 0);
                acc_hi = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1h, bh, acc_hi, 0, 0, 0);
            }
        } else {
            const float* pa = sx + (lane & 7) * 68;
            const float* pb = sy + (lane >> 3) * 64;
            const float* pt = sT + (col % NPL) * 68;
            const float* pv = sV + (col / NPL) * 64;
            struct Ops { float4 a, b, t, v; };
            auto rd4 = [&](Ops& o, int q) __attribute__((always_inline)) {   // slots q .. q + 3 (q <= 64)
                o.a = *reinterpret_cast<const float4*>(pa + q);
                o.b = *reinterpret_cast<const float4*>(pb + q);
                o.t = *reinterpret_cast<const float4*>(pt + q);
                o.v = *reinterpret_cast<const float4*>(pv + q);
            };
            auto outer = [&](float a, float b) __attribute__((always_inline)) {
                if constexpr (NCOL == 32) acc = __builtin_amdgcn_mfma_f32_32x32x1f32(a, b, acc, 0, 0, 0);
                else acc = __builtin_amdgcn_mfma_f32_16x16x1f32(a, b, acc, 0, 0, 0);
            };
            auto four = [&](const Ops& o) __attribute__((always_inline)) {
                outer(o.a.x * o.b.x, o.t.x * o.v.x);
                outer(o.a.y * o.b.y, o.t.y * o.v.y);
                outer(o.a.z * o.b.z, o.t.z * o.v.z);
                outer(o.a.w * o.b.w, o.t.w * o.v.w);
            };
            // two operand sets in turn: the next four samples are read while the
            // current four outer products run (the slots read past n4 are unused)
            Ops o0, o1;
            rd4(o0, 0);
            for (int qq = 0;;) {
                rd4(o1, qq + 4);
                four(o0);
                if ((qq += 4) >= n4) break;
                rd4(o0, qq + 4);
                four(o1);
                if ((qq += 4) >= n4) break;
            }
        }
        lds_order();                                        // the walk's reads precede the next staging writes
    }
    if constexpr (NCOL == 32) {   // the 32 x 32 blocks in the layout of the two-block instruction
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            acc[r] = acc_lo[r];
            acc[16 + r] = acc_hi[r];
        }
    }
    // write-out: accumulators -> LDS [cell][NCOL + 1] -> planes of the group in HBM
    float* wo = lds;
    const int hx = NCOL == 32 ? 4 * (lane >> 5) : 4 * ((lane >> 4) & 1);
    const int hy = NCOL == 32 ? 0 : (lane >> 5);
#pragma unroll
    for (int rg = 0; rg < NREG; ++rg) {
        const int cx = hx + (rg & 3);
        const int cy = NCOL == 32 ? (rg >> 2) : 2 * (rg >> 2) + hy;
        wo[(cy * kTile + cx) * (NCOL + 1) + col] = acc[rg] * ivs;
    }
    lds_order();
    if (un.parts > 1) {   // a split bin's partial tile [plane][cell], added up by k_split_sum
        float2* part = reinterpret_cast<float2*>(split_part + (size_t)ob * kPartFloats);
        for (int i = threadIdx.x; i < nk * 64; i += blockDim.x) {
            const float* e = wo + (i % 64) * (NCOL + 1);
            part[i] = make_float2(e[i / 64], e[NPL + i / 64]);
        }
    } else {
        for (int i = threadIdx.x; i < nk * 64; i += blockDim.x) {
            const int pl = i / 64, cell = i % 64;
            const int ly = cell / kTile, lx = cell % kTile;
            const int pg = s0 * P->K + k0 + pl;    // global plane index
            const float* e = wo + cell * (NCOL + 1);
            grid[((size_t)pg * M + ty * kTile + ly) * M + tx * kTile + lx] = make_float2(e[pl], e[NPL + pl]);
        }
    }
    lds_order();                               // the write-out reads precede the next tile's staging writes
    }
}

// Matrix-core gridder over bins of 16 x 16 cells (the tuning's 16 x 16 bin
// variants; 16 planes per pass, operands split as hi + lo in fp16 and
// accumulated in FP32 exactly as in k_grid_tiles_mfma<32>).  One wavefront per
// bin holds 256 cells x 32 columns in eight 32 x 32 accumulator blocks:
// block (bx, by) covers the cells x in [8 bx, 8 bx + 8), y in [4 by, 4 by + 4),
// its A row i is cell (8 bx + i mod 8, 4 by + i / 8), and its register r of
// lane l holds cell (8 bx + 4 (l / 32) + r mod 4, 4 by + r / 4), column l mod
// 32.  A sample meets about 2.1 bins instead of 3.5 tiles of 8 x 8 cells, so
// its kernel weights and Chebyshev values are staged, and the steps of the
// walk formed, less often; the blocks that none of a step's 16 samples
// touches are skipped (a uniform branch per block).  (Two wavefronts per bin,
// each with half the accumulators and half the staging, allow three
// wavefronts per SIMD instead of two, but the barriers of the shared staging
// made the pass slower: 0.78 against 0.64 ms.)
// Staging in LDS, rows of 68 floats, one column per sample slot: T rows
// 0..15, x rows (bin columns 0..15) at rows 16..31, 7 spare rows, y rows (bin
// rows 0..15) at rows 39..54, Re and Im of g x at rows 55 and 56, 5 spare
// rows, the slots' block masks (bytes) in row 62.  A sample's kernel weights
// are evaluated at its 8 footprint cells only: the footprint start d relative
// to the bin lies in [-7, 15], and the weights are stored at x (y) rows
// d .. d + 7 after rows 0..15 of the slot were set to zero.  Rows below 0 or
// above 15 fall on T rows 9..15 and the spare rows (x), or on the spare rows,
// the g x rows and the spare rows after them (y), all of which the lane
// writes afterwards or nobody reads, and only in its own slot's column.
__global__ __launch_bounds__(64, 2) void k_grid_bins16(
    const SampleRec* __restrict__ recs, int n_chan, const DevPlan* __restrict__ P, int M, int NT,
    const int32_t* __restrict__ bin_off, const int32_t* __restrict__ list, int bin_cap,
    const int32_t* __restrict__ order, const int32_t* __restrict__ cnt, const int4* __restrict__ units,
    float* __restrict__ split_part, float2* __restrict__ grid) {
    constexpr int S = 16, R = kBin16Stride;      // bin side, LDS row stride (floats)
    constexpr int rT = 0, rX = 16, rY = 39, rV = 55, rM = 62;
    static_assert(rM < kBin16Rows, "staging rows");
    typedef float f32x16 __attribute__((ext_vector_type(16)));
    auto ld8 = [](const float* p, float* o) __attribute__((always_inline)) {
        const float4 u = reinterpret_cast<const float4*>(p)[0], w = reinterpret_cast<const float4*>(p)[1];
        o[0] = u.x; o[1] = u.y; o[2] = u.z; o[3] = u.w; o[4] = w.x; o[5] = w.y; o[6] = w.z; o[7] = w.w;
    };
    extern __shared__ float lds[];
    const int tiles = NT * NT;
    if (P->status & kStatusFatal) return;
    const int lane = threadIdx.x;
    const int n_chunks = (n_chan + kItemChans - 1) / kItemChans;
    float vs = 1.f, ivs = 1.f;   // fp16 scale of the values, as in k_grid_tiles_mfma<32>
    {
        const float vmax = __uint_as_float(P->vmax_bits);
        if (vmax > 0.f) {
            int ex;
            (void)frexpf(vmax, &ex);
            ex = min(max(ex, -100), 127);
            vs = ldexpf(1.f, 14 - ex);
            ivs = ldexpf(1.f, ex - 14);
        }
    }
    // walk operands of this lane: A row i = lane mod 32, samples 8 h .. 8 h + 7
    // of a step; B column i: order i mod 16, Re (i < 16) or Im
    const int h = lane >> 5, i = lane & 31;
    const float* pT = lds + (rT + (i & 15)) * R + 8 * h;
    const float* pV = lds + (rV + (i >> 4)) * R + 8 * h;
    const float* pX = lds + (rX + (i & 7)) * R + 8 * h;    // + 8 R for bx = 1
    const float* pY = lds + (rY + (i >> 3)) * R + 8 * h;   // + 4 by R
    const uint8_t* pM = reinterpret_cast<const uint8_t*>(lds + rM * R);
    const int n_units = work_unit_count(cnt);
    for (int ob = blockIdx.x; ob < n_units; ob += gridDim.x) {
    const WorkUnit un = work_unit(ob, units, order, cnt);
    const int bid = un.bin;
    const int g = bid / tiles, tile = bid % tiles;
    if (g >= P->ng) continue;
    int b0, b1;
    work_unit_items(un, bin_off, bin_cap, P->unit_shift, b0, b1);
    if (b1 <= b0 && un.parts == 1) continue;   // every unit of a split bin reports in
    int s0, s1, k0, k1;
    group_range(g, P, s0, s1, k0, k1);         // one slab per group (max_sg = 1)
    const int nk = k1 - k0;                    // <= 16 planes
    const int tx = tile % NT, ty = tile / NT;
    f32x16 acc[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[b] = f32x16{};
    auto load_rec = [&](int item_, float4& ra, float4& rb) __attribute__((always_inline)) {
        const int c = (item_ % n_chunks) * kItemChans + lane;
        if (c < n_chan) {
            const float4* src = reinterpret_cast<const float4*>(recs + (size_t)(item_ / n_chunks) * n_chan + c);
            ra = src[0];
            rb = src[1];
        } else {
            ra = make_float4(__int_as_float(-1), 0.f, 4.f, 4.f);
            rb = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    float4 ra, rb, ra2, rb2;
    if (b0 < b1) load_rec(list[b0], ra, rb);
    if (b0 + 1 < b1) load_rec(list[b0 + 1], ra2, rb2);
    for (int it = b0; it < b1; ++it) {
        const int pk = __float_as_int(ra.x), sp = __float_as_int(ra.y);
        const int ix = pk & 8191, iy = (pk >> 13) & 8191;
        const float ox = ra.z, oy = ra.w, ss = rb.x, vr = rb.y, vi = rb.z;
        const int ddx = (ix - tx * S) & (M - 1), ddy = (iy - ty * S) & (M - 1);
        const bool act = pk >= 0 && (sp >= s0 && sp < s1) && (ddx < S || ddx >= M - 7) && (ddy < S || ddy >= M - 7);
        ra = ra2;
        rb = rb2;
        if (it + 2 < b1) load_rec(list[it + 2], ra2, rb2);   // the records two items ahead
        const uint64_t amask = __ballot(act);
        if (amask == 0) continue;
        const int n_act = __popcll(amask), n4 = (n_act + 15) & ~15;
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(amask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)amask, 0));
        const int q = act ? below : n_act + (lane - below);
        if (q < n4) {
            // footprint starts relative to the bin, in [-7, 15] (padding slots:
            // 0, with finite weights and g x = 0)
            const int dx = act ? (ddx < S ? ddx : ddx - M) : 0, dy = act ? (ddy < S ? ddy : ddy - M) : 0;
            const float oxa = act ? ox : 0.f, oya = act ? oy : 0.f, ssa = act ? ss : 0.f;
            float* col = lds + q;
#pragma unroll
            for (int r = 0; r < S; ++r) {
                col[(rX + r) * R] = 0.f;
                col[(rY + r) * R] = 0.f;
            }
            float* cx = col + (rX + dx) * R;
            float* cy = col + (rY + dy) * R;
#pragma unroll
            for (int p = 0; p < 8; ++p) {   // footprint position p: z = (p - o) / 4 in [-1, 1)
                cx[p * R] = es_kernel(((float)p - oxa) * 0.25f);
                cy[p * R] = es_kernel(((float)p - oya) * 0.25f);
            }
            float t, tm1;
            cheb_start(ssa, k0, t, tm1);
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                col[(rT + k) * R] = t;
                const float tn = 2.f * ssa * t - tm1;
                tm1 = t;
                t = tn;
            }
            col[rV * R] = act ? vr * vs : 0.f;
            col[(rV + 1) * R] = act ? vi * vs : 0.f;
            // blocks touched: x half bx where [dx, dx + 8) meets [8 bx, 8 bx + 8),
            // y quarter by where [dy, dy + 8) meets [4 by, 4 by + 4); bit 4 bx + by
            uint32_t m = 0;
            if (act) {
                uint32_t my = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) my |= (dy <= 4 * b + 3 && dy >= 4 * b - 7) ? (1u << b) : 0u;
                m = (dx < 8 ? my : 0u) | (dx >= 1 ? my << 4 : 0u);
            }
            reinterpret_cast<uint8_t*>(lds + rM * R)[q] = (uint8_t)m;
        }
        lds_order();                                        // staging writes precede the walk's reads
        // the block masks of the item's steps (at most four), uniform; slots
        // past n4 hold older masks and belong to no step
        uint32_t sm[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const uint4 mw = reinterpret_cast<const uint4*>(pM)[s4];
            uint32_t m = mw.x | mw.y | mw.z | mw.w;
            m |= m >> 16;
            m |= m >> 8;
            sm[s4] = __builtin_amdgcn_readfirstlane(m & 0xffu);
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int q0 = 16 * s4;
            if (q0 >= n4) break;
            const uint32_t m = sm[s4];
            // every operand of the step is read up front (one wait for all of
            // them; the blocks below only form products)
            float t[8], v[8], x[2][8], y[4][8];
            ld8(pT + q0, t);
            ld8(pV + q0, v);
#pragma unroll
            for (int bx = 0; bx < 2; ++bx) ld8(pX + bx * 8 * R + q0, x[bx]);
#pragma unroll
            for (int by = 0; by < 4; ++by) ld8(pY + by * 4 * R + q0, y[by]);
            f16x8_t bh, bl;
            split_prod_f16x8(t, v, bh, bl);
#pragma unroll
            for (int bx = 0; bx < 2; ++bx)
#pragma unroll
                for (int by = 0; by < 4; ++by) {
                    if (!(m & (1u << (4 * bx + by)))) continue;
                    f16x8_t ah, al;
                    split_prod_f16x8(x[bx], y[by], ah, al);
                    f32x16& a = acc[4 * bx + by];
                    a = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, a, 0, 0, 0);
                    a = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, a, 0, 0, 0);
                    a = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, a, 0, 0, 0);
                }
        }
        lds_order();                                        // the walk's reads precede the next staging writes
    }
    // write-out, half a bin (rows 8 hb .. 8 hb + 7) at a time: accumulators ->
    // LDS [cell][33] -> planes of the group in HBM (or the partial tile)
    float* wo = lds;
    const int col = lane & 31;
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
#pragma unroll
        for (int bx = 0; bx < 2; ++bx)
#pragma unroll
            for (int byl = 0; byl < 2; ++byl)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int cx = 8 * bx + 4 * (lane >> 5) + (r & 3), cyl = 4 * byl + (r >> 2);
                    wo[(cyl * S + cx) * 33 + col] = acc[4 * bx + 2 * hb + byl][r] * ivs;
                }
        lds_order();
        if (un.parts > 1) {   // partial tile [plane][cell], cell = y 16 + x, added up by k_split_sum
            float2* part = reinterpret_cast<float2*>(split_part + (size_t)ob * (4 * kPartFloats));
            for (int e = threadIdx.x; e < nk * 128; e += blockDim.x) {
                const int pl = e / 128, cell = e % 128;
                const float* w = wo + cell * 33;
                part[pl * 256 + hb * 128 + cell] = make_float2(w[pl], w[16 + pl]);
            }
        } else {
            for (int e = threadIdx.x; e < nk * 128; e += blockDim.x) {
                const int pl = e / 128, cell = e % 128;
                const int ly = cell / S, lx = cell % S;
                const int pg = s0 * P->K + k0 + pl;    // global plane index
                const float* w = wo + cell * 33;
                grid[((size_t)pg * M + ty * S + 8 * hb + ly) * M + tx * S + lx] = make_float2(w[pl], w[16 + pl]);
            }
        }
        lds_order();                               // the write-out reads precede the next writes to LDS
    }
    }
}

// Tiles of split bins: the partial tiles of a bin's units (consecutive unit
// slots from part 0) added in part order, written to the grid.  One workgroup
// per 256 elements (plane, cell) of a split bin at a time, one element per
// thread, whose loads of up to eight parts are issued before it adds them in
// order.  (One workgroup per split bin, each thread adding 16 elements one
// load at a time, took 25 us per MeerKAT-shaped snapshot with 16 x 16 bins.)
constexpr int kSplitSumWorkgroups = 2048;
__global__ __launch_bounds__(256) void k_split_sum(const DevPlan* __restrict__ P, int M, int NT, int bsh,
                                                   const int4* __restrict__ units, const int32_t* __restrict__ cnt,
                                                   const float* __restrict__ split_part, float2* __restrict__ grid) {
    if (P->status & kStatusFatal) return;
    const int n_split = cnt[1], tiles = NT * NT;
    const int S = 1 << bsh, cells = S * S;                                  // a bin of S x S cells
    const size_t part_f2 = ((size_t)kPartFloats << (2 * (bsh - kTileShift))) / 2;   // float2 per partial tile
    const int chunks = kGroupPlanes * cells / 256;                          // 256-element chunks of a partial tile
    for (int w = blockIdx.x; w < n_split * chunks; w += gridDim.x) {
        const int ob = w / chunks, ch = w % chunks;
        const int4 u = units[ob];
        if (u.z <= 1 || u.y != 0) continue;   // whole bins and parts after the first
        const int g = u.x / tiles, tile = u.x % tiles;
        if (g >= P->ng) continue;
        int s0, s1, k0, k1;
        group_range(g, P, s0, s1, k0, k1);
        const int nk = k1 - k0, tx = tile % NT, ty = tile / NT;
        const int i = ch * 256 + (int)threadIdx.x;
        if (i >= nk * cells) continue;
        const float2* src = reinterpret_cast<const float2*>(split_part) + (size_t)ob * part_f2 + i;
        float2 v = make_float2(0.f, 0.f);
        int p = 0;
        for (; p + 8 <= u.z; p += 8) {
            float2 a[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = src[(size_t)(p + j) * part_f2];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                v.x += a[j].x;
                v.y += a[j].y;
            }
        }
        for (; p < u.z; ++p) {
            const float2 a = src[(size_t)p * part_f2];
            v.x += a.x;
            v.y += a.y;
        }
        const int pl = i / cells, cell = i % cells;
        const int pg = s0 * P->K + k0 + pl;
        grid[((size_t)pg * M + ty * S + cell / S) * M + tx * S + cell % S] = v;
    }
}

hipError_t launch_grid(toi_ctx* c, const toi_snapshot& s) {
    const hipError_t e = launch_bin(c, s);
    return e != hipSuccess ? e : launch_gridder(c, s);
}

constexpr int kBinSortBlocks = 512;   // 8192 wavefronts

// The bin pipeline with bins of 2^bsh cells per side; the record pass too when
// records is set (otherwise the records and items of the last launch_bin of
// this snapshot are reused).
static hipError_t bin_pipeline(toi_ctx* c, const toi_snapshot& s, int bsh, bool records) {
    const toi_params& p = c->p;
    const int M = c->M, NB = M >> bsh;
    const double cell = p.cell_deg * kPi / 180.0;
    const int n_chunks = (p.n_chan + kItemChans - 1) / kItemChans;
    const int n_items = s.n_row * n_chunks;
    const int n_bins = c->NG_max * NB * NB;
    const int words = (c->NT + 31) / 32;   // row_bits words per plane group (mask tiles)
    const int n_scan = (n_bins + kScanBlock - 1) / kScanBlock;
    const int max_units = kSplitSlots >> (2 * (bsh - kTileShift));
    c->bins_shift = bsh;
    const BinClear bc{c->bin_count, n_bins, NB * NB, c->bin_aux, c->row_bits, c->NG_max * words, words};
    hipLaunchKernelGGL(k_scan_clear, dim3(256), dim3(256), 0, c->stream, c->plan, bc);
    if (n_items > 0 && records)
        hipLaunchKernelGGL(k_items, dim3((n_items + 3) / 4), dim3(256), 0, c->stream, s.uvw,
                           (const float2*)s.vis, s.weight, s.flag, s.freq, s.ant1, s.ant2,
                           (const float2*)s.gains, p.n_ant, p.n_chan, p.n_corr, p.corr_mask,
                           (int)vec4_ok(s.vis, s.flag, s.weight, p.n_corr), p.mode, c->plan, M,
                           cell, n_items, c->items, c->recs);
    if (n_items > 0)
        hipLaunchKernelGGL(k_item_bins, dim3((n_items + 256 / kItemLanes - 1) / (256 / kItemLanes)), dim3(256), 0,
                           c->stream, s.uvw, p.n_chan, p.mode, c->plan, M, NB, bsh, cell, n_items, c->items,
                           c->bin_count);
    hipLaunchKernelGGL(k_scan_local, dim3(n_scan), dim3(1024), 0, c->stream, c->bin_count, n_bins, c->plan,
                       NB * NB, c->items, n_items, c->bin_off, c->bin_aux);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, c->stream, n_scan, n_bins, c->bin_cap, c->plan,
                       c->bin_aux, c->bin_off, c->scratch_i);
    hipLaunchKernelGGL(k_scan_apply, dim3(n_scan), dim3(1024), 0, c->stream, c->bin_count, n_bins, NB, bsh,
                       c->bin_off, c->bin_cursor, c->bin_order, c->bin_aux, c->tile_bits, c->row_bits,
                       c->plan);
    hipLaunchKernelGGL(k_units, dim3(1), dim3(1024), 0, c->stream, c->plan, c->bin_count, c->bin_order,
                       c->bin_aux, max_units, c->units, c->scratch_i);
    if (n_items > 0) {
        hipLaunchKernelGGL(k_bin_fill, dim3((n_items + 256 / kFillLanes - 1) / (256 / kFillLanes)), dim3(256), 0,
                           c->stream, c->items, n_items, NB, bsh,
                           c->bin_cap, c->bin_cursor, c->bin_list);
        hipLaunchKernelGGL(k_bin_sort, dim3(kBinSortBlocks), dim3(1024), 0, c->stream, c->plan,
                           c->bin_order, c->scratch_i, c->bin_aux, c->bin_off, c->bin_list);
    }
    return hipGetLastError();
}

hipError_t launch_bin(toi_ctx* c, const toi_snapshot& s) {
    StageTimer timer(c, TOI_STAGE_BIN);
    return bin_pipeline(c, s, bin_shift_of(c->tuning, c->M), true);
}

hipError_t launch_rebin(toi_ctx* c, const toi_snapshot& s, int bin_shift) {
    StageTimer timer(c, TOI_STAGE_BIN);
    return bin_pipeline(c, s, bin_shift, false);
}

hipError_t launch_gridder(toi_ctx* c, const toi_snapshot& s) {
    const toi_params& p = c->p;
    const int M = c->M, bsh = c->bins_shift, NB = M >> bsh;
    const int n_chunks = (p.n_chan + kItemChans - 1) / kItemChans;
    const int n_items = s.n_row * n_chunks;
    const int n_bins = c->NG_max * NB * NB;
    if (n_items == 0) return hipGetLastError();
    StageTimer timer(c, TOI_STAGE_GRID);
    const GridShape gs = grid_shape(c->tuning, bsh);
    // a fixed grid of single-wave workgroups takes the work units in turn
    // (a 16 x 16 bin holds about as many items as four 8 x 8 tiles)
    const int mblocks = unit_workgroups(n_items >> (2 * (bsh - kTileShift)), n_bins);
#define TOI_MFMA_ARGS                                                                                      \
    dim3(mblocks), dim3(64), gs.lds_bytes, c->stream, c->recs, p.n_chan, c->plan, M, NB, c->bin_off, c->bin_list, \
        c->bin_cap, c->bin_order, c->scratch_i, c->units, c->split_part, c->grid
    if (bsh > kTileShift)
        hipLaunchKernelGGL(k_grid_bins16, TOI_MFMA_ARGS);
    else if (gs.gp > 8)
        hipLaunchKernelGGL((k_grid_tiles_mfma<32>), TOI_MFMA_ARGS);
    else
        hipLaunchKernelGGL((k_grid_tiles_mfma<16>), TOI_MFMA_ARGS);
#undef TOI_MFMA_ARGS
    hipLaunchKernelGGL(k_split_sum, dim3(kSplitSumWorkgroups), dim3(256), 0, c->stream, c->plan, M, NB, bsh,
                       c->units, c->scratch_i, c->split_part, c->grid);
    return hipGetLastError();
}

}  // namespace toi
