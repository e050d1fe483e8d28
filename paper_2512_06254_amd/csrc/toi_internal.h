// Internal declarations shared by the HIP translation units of libtoi.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/toi.h"

namespace toi {

constexpr double kCLight = 299792458.0;
constexpr double kInvCLight = 1.0 / kCLight;   // correctly rounded at compile time
constexpr double kPi = 3.14159265358979323846;
constexpr int kSupport = 8;                 // ES kernel support W (cells)
constexpr double kEsBetaPerW = 2.30;        // beta = 2.30 W for a 2x oversampled grid
constexpr int kWindow = 16;                 // FITrig sliding window (tLISI maps)

// Plan of the current snapshot, written and read on the device only.
struct DevPlan {
    double V[9];          // rows: e1, e2, e3
    double omega, xi, eta;
    double wsum;          // W = sum of sample weights
    double nvis;          // kept samples
    double r3min, r3max;
    double t3max;         // written through its bit pattern by an atomic max
    double phimax, dr3, alpha_slab;
    double inv_dr3;       // 1 / dr3 (0 when dr3 = 0)
    double norm;          // 1 / (omega W)
    double sum_b[3];
    double sum_bb[6];
    int32_t n_slab, K, planes;
    uint32_t status;
    int32_t miller_top;   // starting order of the Bessel backward recurrence
    int32_t ng;           // plane groups gridded together (at most gp planes each)
    int32_t sg;           // slabs per group when K <= gp
    int32_t kp;           // Chebyshev orders per group when K > gp
    int32_t parts;        // groups per slab when K > gp (1 otherwise)
    int32_t gp;           // planes per group (LDS pass of the gridder)
    int32_t max_sg;       // at most this many slabs share a group (1: the gridders and the adjoint rely on it)
    int32_t unit_shift;   // work units of split bins hold at most 2^unit_shift items (from the tuning)
    uint32_t vmax_bits;   // bits of max(|Re|, |Im|) of g x over the kept samples (non-negative float)
};

// Binned gridding: grid tiles of kTile x kTile cells, work items of kItemChans
// channels of one row, up to kGroupPlanes planes accumulated per tile pass.
// The occupancy masks of the FFT passes are always kept per kTile x kTile
// tile; the bins of the gridder are tiles of 2^bin_shift cells per side,
// bin_shift = kTileShift or kTileShift + 1 (the tuning's 16 x 16 bins, each
// four mask tiles).
constexpr int kTile = 8, kTileShift = 3;
constexpr int kItemChans = 64;
constexpr int kGroupPlanes = 16;   // largest plane group held in LDS
constexpr int kScanBlock = 4096;   // bins per workgroup of the bin scan
// Work units of the matrix-core tile passes: a bin of at least U = 2^unit_shift
// items (U from the tuning: 32 .. 256) is split into units of at most U items
// (bins of bucket unit_shift and above are listed unit by unit); the units of
// one bin add their partial tiles in a fixed order.  At most kSplitSlots
// listed units per snapshot (the heaviest buckets first; the rest run whole).
constexpr int kSplitSlots = 16384;
// Layout of the bin scan's auxiliary array: per floor(log2(count)) bucket the
// number of non-empty bins, the launch-order cursor and the work units of its
// bins (ceil(count / 2^unit_shift) each), then one total per scan workgroup,
// then one partial max(|Re|, |Im|) of g x per scan workgroup (float bits).
// Each bucket's three words sit in a 128-byte line of their own (word
// kAux* + kAuxStride k): every scan workgroup adds to them with device-wide
// atomics, which are applied one at a time per line.
constexpr int kAuxStride = 32;
constexpr int kAuxBuckets = 0, kAuxCursors = 1, kAuxUnits = 2, kAuxTotals = 32 * kAuxStride;
// After the list fill, every bin's items are put in increasing item order:
// bins of fewer than 2^kBlockSortShift items by one wavefront (four values per
// lane from 2^kSortShift items, 16 lanes per bin below 16 items), larger ones
// by a workgroup in LDS up to kSortLds items, beyond that in place in HBM.
constexpr int kSortShift = 6, kBlockSortShift = 8, kSortLds = 16384;
constexpr int kPartFloats = 64 * 32;   // one partial tile: 64 cells x up to 16 complex planes
// (a 16 x 16 bin's partial tile takes four such slots, so at most
// kSplitSlots / 4 of its units are listed)
constexpr int kAdjAbsmaxParts = 1024;  // workgroups of the adjoint's image-gradient maximum

// Gridder variant chosen by the autotuner (toi_tune / toi_set_tuning):
// bits 0-1: work-unit size U = 32 << bits items (split bins are gridded by one
// wavefront per U items; fewer, longer units write fewer partial tiles, more,
// shorter ones balance the heaviest tiles across more wavefronts);
// bit 2: the plane schedule, 8 planes per pass over a tile on the FP32 matrix
// cores (v_mfma_f32_16x16x1f32, one instruction per sample) instead of 16
// planes per pass on the fp16 matrix cores with split operands;
// bit 3 (with bit 2 clear; variants 8 .. 11): bins of 16 x 16 cells, one
// wavefront per bin (each sample visits about 2.1 bins instead of 3.5 tiles
// of 8 x 8; used where the grid has at least 256 cells per side).
constexpr int kTuneUnitMask = 3, kTuneEightPlanes = 4, kTuneBin16 = 8;
constexpr int kTuneDefault = 1;   // 64-item units, 16 planes per pass, 8 x 8 bins
constexpr size_t kLdsBytes = 160 * 1024;   // per workgroup on gfx950

// Bin side of a variant on a grid of side M: 2^bin_shift cells.
inline int bin_shift_of(int tuning, int M) {
    return ((tuning & kTuneBin16) && !(tuning & kTuneEightPlanes) && M >= 256) ? kTileShift + 1 : kTileShift;
}

// Launch shape of the tile gridder for a variant: one wavefront per work unit.
// 8 x 8 bins: LDS for staging (rows 8 x 68, 8 x 64, 2 x 64, gp x 68) and then
// the write-out buffer [64][2 gp + 1]; 16 x 16 bins: 63 staging rows of 68
// floats, then the write-out buffer of half a bin [128][33].
struct GridShape {
    int gp, max_sg, unit_shift;
    size_t lds_bytes;
};
constexpr int kBin16Rows = 63, kBin16Stride = 68;
inline GridShape grid_shape(int tuning, int bin_shift = kTileShift) {
    GridShape g;
    g.gp = (tuning & kTuneEightPlanes) ? 8 : kGroupPlanes;
    g.max_sg = 1;   // one slab per plane group (the gridder and the adjoint gather rely on it)
    g.unit_shift = 5 + (tuning & kTuneUnitMask);
    size_t stage = (size_t)8 * 68 + 8 * 64 + 2 * 64 + (size_t)g.gp * 68, wout = (size_t)64 * (2 * g.gp + 1);
    if (bin_shift > kTileShift) {
        stage = (size_t)kBin16Rows * kBin16Stride;
        wout = (size_t)128 * 33;
    }
    g.lds_bytes = (stage > wout ? stage : wout) * sizeof(float);
    return g;
}

// Bin of one work item: the track of its kept samples (grid coordinates X, Y
// at the lowest and the highest kept frequency; both are linear in the
// frequency along a row), the tile rows and plane groups it touches
// (unwrapped tile indices, wrapped modulo the tiles per axis when used; empty
// when ty1 < ty0), max(|Re|, |Im|) of g x over its kept samples, and the
// reciprocal of the track's extent in Y.  The
// tiles of each tile row follow from the track (item_row_tiles, toi_grid.h).
struct ItemBox {
    double x0, y0, x1, y1;
    int32_t ty0, ty1, g0, g1;
    float vmax;
    int32_t pad_;
    double inv_dy;   // 1 / (y1 - y0), 0 when |y1 - y0| <= 1e-9
    double nlo, nhi; // extreme kept frequencies (nlo > nhi: none kept), from the record pass
};

// One sample prepared for gridding (written by k_items, read by the
// matrix-core gridder at every tile the sample's item visits): footprint
// start ix | iy << 13 (-1: sample not kept), slab, offsets of the sample from
// the start in (3, 4], Chebyshev argument, value g x.
struct SampleRec {
    int32_t pk, sp;
    float ox, oy, ss, vr, vi, pad_;
};

// Per-row partial sums of the kept samples (sample prep).
struct RowStat {
    double cnt;           // kept channels
    double s1;            // sum nu / c
    double s2;            // sum (nu / c)^2
    double wsum;          // sum of sample weights
    double numin, numax;  // extreme kept frequencies (Hz)
    double pad_[2];
};

struct TileStat {         // FITrig per-tile sums (FP64)
    double sx, sy, sxx, syy, sxy, mn, mx, pad_;
};

}  // namespace toi

// Per-snapshot state written by sample prep and binning and read by the
// gridder and the FFT passes.  The context holds one set in its own fields;
// batched execution adds a second (toi_ctx::alt) so that the prep and binning
// of snapshot i + 1 can run while snapshot i is gridded and transformed.
struct toi_front {
    toi::DevPlan* plan;
    toi::RowStat* rows;
    toi::ItemBox* items;
    toi::SampleRec* recs;
    int32_t* bin_count;
    int32_t* bin_off;
    int32_t* bin_cursor;
    int32_t* bin_list;
    int32_t* bin_order;
    int32_t* bin_aux;
    int4* units;
    uint32_t* tile_bits;
    uint32_t* row_bits;
    int32_t* scratch_i;
};

struct toi_ctx {
    toi_params p;
    hipStream_t stream;
    int device;
    int N, M, T;          // image side, grid side, tLISI tiles per axis
    int P_cap;            // plane capacity
    int forced_K;         // 0 when chosen on the device
    int tuning;           // gridder variant (kTune* bits)
    std::string err;

    // workspace (device)
    float2* grid;         // [P_cap][M][M]   only tiles with samples are written
    int NT;               // grid tiles per axis (M / kTile)
    int bins_shift;       // bin side 2^bins_shift of the bins last built (launch_bin)
    int NG_max;           // plane-group capacity
    int n_items_max;      // work items capacity (n_row_max * chunks)
    toi::ItemBox* items;  // [n_items_max]
    toi::SampleRec* recs; // [n_row_max][n_chan] gridding records
    float2* gx;           // [n_row_max][n_chan][2] adjoint: gradient of each sample's value (Re, Im as
                          // 64-bit fixed point; 16 bytes per sample)
    int32_t* bin_count;   // [NG_max][NT*NT]
    int32_t* bin_off;     // [NG_max][NT*NT + 1]
    int32_t* bin_cursor;  // [NG_max][NT*NT]
    int32_t* bin_list;    // [bin capacity]
    int32_t* bin_order;   // [NG_max][NT*NT] non-empty bins, heaviest first (count in scratch_i[0];
                          // scratch_i[1]: units of split bins, scratch_i[2]: bins listed as units)
    int32_t* bin_aux;     // bucket sizes, cursors and unit counts (32 each), one total per scan block
    int4* units;          // [kSplitSlots] listed work units {bin, part, parts, index of part 0}
    float* split_part;    // [kSplitSlots][kPartFloats] partial tiles of split bins ([plane][cell] complex)
    int bin_cap;
    uint32_t* tile_bits;  // [NG_max][NT][NT/32]  nonempty tiles of each tile row
    uint32_t* row_bits;   // [NG_max][NT/32]      nonempty tile rows
    float2* hbuf;         // [P_cap][N/4][M][4] row-pass output: column major per plane in groups of 4 columns
                          // (the adjoint uses it as [P_cap][N][M])
    float* tplane_t;      // [N][N]          transformed-plane image, j1 major
    float* adj_tp;        // [N][N]          adjoint: transformed-plane gradient, j1 major, 64-bit fixed
                          // point (8 bytes per pixel; the autotuner uses it as an f32 image)
    float* adj_parts;     // adjoint: per-workgroup largest magnitudes for the fixed-point scales
    double2* item_gain;   // [n_items_max + n_row_max] adjoint: per-item, then per-row gain partial sums
    toi::DevPlan* plan;
    toi::RowStat* rows;   // [n_row_max]
    float* corr;          // [N]  (-1)^a / psi(a), a = j - N/2
    float2* twiddle;      // [M]  e^{+2 pi i n / M}
    toi::TileStat* tiles; // [T*T]
    double* scratch_d;    // small FP64 scratch (reductions)
    int32_t* scratch_i;   // small integer scratch (detection)
    double* det_scores;   // [2][T*T] detection scores (periodic, non-periodic)
    int4* det_boxes;      // [T*T] component bounding boxes in tiles

    // per-stage timing (measurement only)
    uint32_t prof_mask;   // stages whose launches are timed (bit s = stage s)
    std::vector<hipEvent_t> prof_ev;      // pairs (start, stop)
    std::vector<int> prof_stage;          // stage of each recorded pair
    size_t prof_n;

    // batched execution (a captured graph of the whole batch, cached by descriptor set)
    hipGraph_t batch_graph;
    hipGraphExec_t batch_exec;
    uint64_t batch_key;
    int batch_n;
    hipStream_t cap_stream;   // internal stream the batch is captured on (default priority)
    struct toi_batch_ring* ring;   // context-owned input slots (toi_batch_inputs), or null
    int64_t batch_captures, batch_launches;
    hipStream_t cap_stream2;  // second capture stream: prep and binning of the next snapshot
    hipEvent_t batch_ev[4];   // capture-time fork/join and ordering events
    toi_front alt;            // second per-snapshot set (allocated on the first batch of >= 2)
    bool alt_ready;

    // streaming ingest (toi_ingest.cpp): device staging slots and the copy stream
    struct toi_ingest_state* ingest;
};

namespace toi {

// error helpers (toi_ctx.cpp)
toi_status fail(toi_ctx* ctx, toi_status st, const std::string& msg);
toi_status hip_check(toi_ctx* ctx, hipError_t e, const char* what);

// launchers, one per translation unit
hipError_t launch_prep(toi_ctx* ctx, const toi_snapshot& s);
hipError_t launch_grid(toi_ctx* ctx, const toi_snapshot& s);      // launch_bin + launch_gridder
hipError_t launch_bin(toi_ctx* ctx, const toi_snapshot& s);       // records, bins, work units
// bins (not the records) again, with bins of 2^bin_shift cells per side
hipError_t launch_rebin(toi_ctx* ctx, const toi_snapshot& s, int bin_shift);
hipError_t launch_gridder(toi_ctx* ctx, const toi_snapshot& s);   // the tile gridder (+ split sums)
hipError_t launch_image(toi_ctx* ctx, float* image_out, float* tplane_out);
hipError_t launch_degrid(toi_ctx* ctx, const float* grad_image, const toi_snapshot& s,
                         float2* grad_vis, float2* grad_gains);
hipError_t launch_tlisi(toi_ctx* ctx, const float* a, const float* b, const float* c, float* out);
hipError_t launch_detect(toi_ctx* ctx, const float* window, int t, int32_t* boxes, int max_boxes,
                         int32_t* n_boxes);
hipError_t launch_detect_cube(toi_ctx* ctx, const float* cube, int L, int t, int32_t* boxes, int max_boxes,
                              int32_t* n_boxes);
hipError_t launch_localise(toi_ctx* ctx, const float* a, const float* b, const int32_t* boxes, int n_boxes,
                           double ra0_deg, double dec0_deg, int morph, double* out);
hipError_t launch_strongest_map(toi_ctx* ctx, const float* cube, int n_maps, const int32_t* boxes, int n_boxes,
                                int32_t* k_out);

// RAII stage timer: records a start/stop event pair on the context's stream
// when profiling is enabled (toi_ctx.cpp).
struct StageTimer {
    toi_ctx* c;
    int slot;
    StageTimer(toi_ctx* ctx, int stage);
    ~StageTimer();
};

// Single-wave workgroups launched for the matrix-core tile passes: about one
// per expected work unit (a bin holds some 12 items, an item meets some 5
// tiles), so the hardware dispatcher hands the units out as waves finish;
// each workgroup loops if there are more units.
inline int unit_workgroups(int n_items, int n_bins) {
    const long want = std::max<long>(8192, n_items / 2);
    return (int)std::min<long>(std::min<long>(want, 1 << 20), (long)n_bins + kSplitSlots);
}

// streaming ingest state (toi_ingest.cpp), released by toi_destroy
void ingest_release(toi_ctx* ctx);
// batch input slots (toi_batch.cpp), released by toi_destroy
void ring_release(toi_ctx* ctx);

// Byte sizes of the per-snapshot set's buffers (same order as toi_front's
// fields), and the swap of the context's set with ctx->alt (toi_ctx.cpp).
constexpr int kFrontBuffers = 14;
void front_bytes(const toi_ctx* ctx, size_t out[kFrontBuffers]);
void front_swap(toi_ctx* ctx);

// host-side tables (toi_ctx.cpp)
void es_correction_table(int N, int M, double* out);   // (-1)^a / psi(a)

}  // namespace toi
