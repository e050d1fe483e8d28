/*
 * toi.h - C ABI of the MI355X (gfx950) TOI snapshot imager and FITrig stage.
 *
 * Method: FIP-TOI, "Transient-Oriented Radio Astronomical Imager" (arXiv
 * 2512.06254).  Each call below names the passage of the paper whose
 * operation it computes.  All arrays are caller-owned DEVICE pointers
 * (HIP/PyTorch allocations on the context's device) unless stated otherwise;
 * the context owns only its workspace.  Every call is asynchronous on the
 * context's HIP stream, except toi_plan_info (which synchronises) and
 * toi_create/toi_destroy.  No exception crosses this boundary: failures are
 * returned as toi_status and described by toi_last_error().
 *
 * Data-dependent conditions never abort a call: they produce a defined output
 * (an all-zero image) and set bits of a device status word that
 * toi_plan_info() returns (TOI_STATUS_* below).
 *
 * Layouts follow the Measurement Set columns the paper reads (Section 3.5):
 *   uvw    f64  [n_row][3]               baseline (ant2 - ant1) in metres
 *   vis    c64  [n_row][n_chan][n_corr]  interleaved (re, im) float pairs
 *   flag   u8   [n_row][n_chan][n_corr]  nonzero = flagged        (nullable)
 *   weight f32  [n_row][n_chan][n_corr]  WEIGHT_SPECTRUM           (nullable)
 *   freq   f64  [n_chan]                 CHAN_FREQ in Hz
 * Images are f32 [N][N], row j2 (m / t2 axis) major, column j1 (l / t1 axis)
 * fastest; pixel (j1, j2) has l = -cell (j1 - N/2), m = cell (j2 - N/2)
 * (Section 3.3 with 0-based indices).
 */
#ifndef TOI_H
#define TOI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct toi_ctx toi_ctx;

typedef enum {
    TOI_OK = 0,
    TOI_EINVAL = 1,        /* bad argument: NULL pointer, size out of range */
    TOI_ENOMEM = 2,        /* workspace allocation failed (toi_create only) */
    TOI_EDEVICE = 3,       /* a HIP runtime call failed */
    TOI_EUNSUPPORTED = 4   /* a parameter combination this build does not implement */
} toi_status;

/* device status word bits (toi_plan_info) */
#define TOI_STATUS_NO_SAMPLES 1u   /* every sample flagged or zero-weight: zero image      */
#define TOI_STATUS_DEGENERATE 2u   /* |V33| < 1e-6: transformed plane edge-on, zero image   */
#define TOI_STATUS_PLANES     4u   /* automatic N_slab * K exceeds max_planes: zero image   */
#define TOI_STATUS_OVERFLOW   8u   /* gridding bin lists exceed bin_cap: zero image          */

typedef struct {
    int32_t  n_pix;        /* N, image side: power of two, 32 .. 4096                       */
    double   cell_deg;     /* cell size (degrees)                                           */
    int32_t  mode;         /* 2: coplanar imaging (Section 3.2); 3: near-coplanar (3.4)      */
    int32_t  n_slab;       /* N_slab; 0 = eq. (27) with alpha_target                         */
    int32_t  cheb_k;       /* K; 0 = smallest of {8,16,24,32} meeting cheb_gamma (3.4)       */
    double   alpha_target; /* eq. (27), default 10                                           */
    double   cheb_gamma;   /* Chebyshev sampled-error threshold, default 1e-2                */
    int32_t  max_planes;   /* workspace capacity for N_slab*K (0 = n_slab*cheb_k, or 32)     */
    int32_t  support;      /* gridding kernel support W: 8 only                              */
    uint32_t corr_mask;    /* correlations averaged (bit k = corr k); 0 = parallel hands     */
    int32_t  tile;         /* FITrig tile side in pixels, default 32                         */
    int32_t  n_row_max;    /* largest n_row of any snapshot passed to this context           */
    int32_t  n_chan;
    int32_t  n_corr;       /* 1, 2 or 4                                                      */
    int32_t  n_ant;        /* antennas (gains length), may be 0 when no gains are used       */
    int32_t  bin_cap;      /* capacity of the gridding bin lists in (work item, bin) entries */
                           /* (bins of 8 x 8 or 16 x 16 cells, by the gridder variant);     */
                           /* 0 = 128 per work item (a work item is 64 channels of         */
                           /* one row) + 65536.  A snapshot needing more sets               */
                           /* TOI_STATUS_OVERFLOW and images to zero.                        */
} toi_params;

typedef struct {
    const double*  uvw;
    const void*    vis;
    const uint8_t* flag;    /* NULL: nothing flagged                                       */
    const float*   weight;  /* NULL: unit weights                                          */
    const double*  freq;
    const int32_t* ant1;    /* i32[n_row]; required when gains != NULL                     */
    const int32_t* ant2;
    const void*    gains;   /* c64[n_ant] per-antenna factors g; each row's samples are     */
                            /* multiplied by g[ant1] conj(g[ant2]); NULL = no gains         */
    int32_t        n_row;   /* 0 <= n_row <= n_row_max                                      */
} toi_snapshot;

/* Fill *p with defaults for an N x N image of cell_deg cells (host only). */
toi_status toi_params_default(toi_params* p, int32_t n_pix, double cell_deg,
                              int32_t n_row_max, int32_t n_chan, int32_t n_corr);

/* Allocate the context and its whole workspace on the current HIP device
 * (the only allocating call; Section 4.2's rule of no allocation in the loop).
 * hip_stream: a hipStream_t (NULL = the null stream).  On failure *out = NULL. */
toi_status toi_create(const toi_params* p, void* hip_stream, toi_ctx** out);

/* Free the workspace; ctx may be NULL.  Synchronises the context's stream. */
toi_status toi_destroy(toi_ctx* ctx);

/* Change the stream subsequent calls are ordered on. */
toi_status toi_set_stream(toi_ctx* ctx, void* hip_stream);

/* Sections 3.1, 3.4, 3.5: select and weight samples (flags -> zero weight,
 * weighted average of the parallel hands, each baseline-channel pair one
 * sample, uvw scaled to wavelengths per channel), estimate the snapshot basis
 * V by PCA of the centred baselines (omega of eq. 11, xi/eta of Section 3.3),
 * choose N_slab and K (eqs. 26-27) unless forced, and grid every Chebyshev
 * moment M_{p,k} of Section 3.4 (one plane in 2-D mode) with an ES kernel of
 * support 8 on a 2N x 2N grid.  The snapshot's arrays must stay valid until
 * the stream reaches the end of this call's work.  The planes are kept in the
 * context for toi_image / toi_degrid. */
toi_status toi_grid(toi_ctx* ctx, const toi_snapshot* snap);

/* Sections 3.2-3.4: inverse 2-D FFT of every plane, grid correction, the
 * Chebyshev/slab combination sum_p e^{i2pi r3p t3} sum_k c_k(2pi dr3 t3) M_{p,k}
 * scaled by 1/(omega W) (W = sum of sample weights = N_vis for unit weights),
 * real part, then the re-projection of Section 3.3 (the reduced SIN mapping
 * composed with the in-plane 2x2 block of V) with bilinear interpolation onto
 * the standard grid.  image_out: f32[N][N] (required); tplane_out: f32[N][N]
 * transformed-plane image before re-projection (nullable). */
toi_status toi_image(toi_ctx* ctx, float* image_out, float* tplane_out);

/* Adjoint of toi_grid + toi_image for the snapshot last passed to toi_grid
 * (same arrays): given grad_image = dL/dI (f32[N][N]) returns
 * grad_vis = dL/dRe(vis) + i dL/dIm(vis) (c64 like vis; nullable) and
 * grad_gains (c64[n_ant]; nullable, requires gains).  Reads the snapshot's
 * flags/weights/gains again; overwrites both outputs. */
toi_status toi_degrid(toi_ctx* ctx, const float* grad_image, const toi_snapshot* snap,
                      void* grad_vis, void* grad_gains);

/* FITrig tLISI (Sections 2, 4.5): from the three youngest images, the
 * difference images D_{t-1} = I_{t-1} - I_{t-2} and D_t = I_t - I_{t-1} are
 * compared tile by tile; one value in [0, 1] per tile (1 = identical).
 * tlisi_out: f32[N/tile][N/tile].  The index used is the SSIM-form stand-in
 * documented with the implementation (the FITrig formula is not in the
 * paper). */
toi_status fitrig_tlisi(toi_ctx* ctx, const float* img_tm2, const float* img_tm1,
                        const float* img_t, float* tlisi_out);

/* fitrig_tlisi without a context and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same kernels and results as
 * fitrig_tlisi (bit for bit) on three caller-owned device images
 * f32[n_pix][n_pix] and a caller-owned f32[n_pix/tile][n_pix/tile] output,
 * enqueued on hip_stream (a stream of the current device; NULL = its null
 * stream).  The per-tile statistics live in a static device array of
 * TOI_TLISI_STATIC_TILES entries (64 bytes each, 4 MiB) that every device the
 * library runs on holds until the process ends; its device address is looked
 * up once per device on that device's first call.  Every call on one device
 * shares that array and overwrites it completely before reading it, so
 * nothing needs clearing, but calls that overlap on one device (concurrent
 * streams or threads) race and give undefined results: serialise them.
 * Errors (NULL pointers, tile not dividing n_pix, more than
 * TOI_TLISI_STATIC_TILES tiles) return TOI_EINVAL without launching anything;
 * toi_last_error(NULL) gives the message. */
#define TOI_TLISI_STATIC_TILES 65536
toi_status fitrig_tlisi_noalloc(const float* img_tm2, const float* img_tm1, const float* img_t,
                                int32_t n_pix, int32_t tile, float* tlisi_out, void* hip_stream);

/* FITrig detection (Section 2) over a sliding window of the 16 newest tLISI
 * maps: per tile, the harmonic-summed DFT power of the window and the
 * non-periodic score sum(1 - tLISI), z-scores over tiles, thresholds 5 and 4,
 * 8-connected components -> boxes (t, x0, y0, x1, y1) in pixels, sorted by
 * (y0, x0, y1, x1).  window: f32[16][N/tile][N/tile], oldest first (device).
 * boxes_out: i32[max_boxes][5] (device); n_boxes_out: device i32 (the number
 * found, possibly > max_boxes, in which case only max_boxes are written).
 * TOI_EUNSUPPORTED when (N/tile)^2 > 16384.  The detection details (window,
 * harmonics, significance, connectivity) are documented readings: the paper
 * states the steps but not their parameters. */
toi_status fitrig_detect(toi_ctx* ctx, const float* window, int32_t t,
                         int32_t* boxes_out, int32_t max_boxes, int32_t* n_boxes_out);

/* FITrig detection over the whole run (Section 2: the Fourier transform of
 * the tLISI cube along time, harmonic summing, significance, connected
 * tiles): as fitrig_detect, with the window replaced by the cube of all
 * n_maps tLISI maps, f32[n_maps][N/tile][N/tile] oldest first (device): per
 * tile the DFT power of the mean-removed series at f = 1 .. n_maps / 2
 * (FP64), harmonic sums over h in {1, 2, 4, 8} divided by sqrt(h), maximum
 * over f and h; the non-periodic score sum(1 - tLISI); then the same
 * z-scores, thresholds, components and boxes, with t written into each box.
 * TOI_EINVAL unless 2 <= n_maps <= 5460 (the series and its powers are held in
 * 64 KB of LDS); TOI_EUNSUPPORTED as for
 * fitrig_detect. */
toi_status fitrig_detect_cube(toi_ctx* ctx, const float* cube, int32_t n_maps, int32_t t,
                              int32_t* boxes_out, int32_t max_boxes, int32_t* n_boxes_out);

/* Full-resolution localisation (Sections 2 and 6) of each candidate box
 * (boxes: device i32[n_boxes][5] as written by fitrig_detect, pixels,
 * inclusive) in the difference image img_b - img_a of two time-adjacent
 * snapshots (device f32[N][N]): subtract the box's lower median, sigma =
 * 1.4826 x the lower median of |D - median|, source pixels with
 * s (D - median) > 5 sigma where s is the sign at the pixel of largest
 * |D - median| (first in row-major order on ties), the 8-connected component
 * of source pixels containing that pixel, and, with morph != 0, the
 * Gaussian-like check (>= 3 pixels, intensity-weighted second-moment axis
 * ratio <= 3, brightest pixel within 1.5 pixels of the centroid).  out
 * (device f64[n_boxes][8]): valid (0/1), centroid j1, j2 (0-based pixels,
 * intensity-weighted), RA and Dec in degrees (inverse SIN projection about
 * ra0/dec0 with l = -cell (j1 - N/2), m = cell (j2 - N/2)), the peak
 * s (D - median), sigma, and the component's pixel count (-1 for a box
 * outside the image or above 65536 pixels).  The steps' parameters are
 * documented readings. */
toi_status fitrig_localise(toi_ctx* ctx, const float* img_a, const float* img_b, const int32_t* boxes,
                           int32_t n_boxes, double ra0_deg, double dec0_deg, int32_t morph, double* out);

/* The adjacent pair holding a candidate's strongest change (Section 5.2: the
 * pair is found by analysing the tLISI cube): for each box, the index k of
 * the tLISI map of cube (device f32[n_maps][N/tile][N/tile], oldest first)
 * whose sum over the box's tiles is smallest (FP64, the first k on ties);
 * map k compares the differences (I_{k+1} - I_k) and (I_{k+2} - I_{k+1}) of
 * the images it was made from, and the newer difference is the one to
 * localise.  k_out: device i32[n_boxes]. */
toi_status fitrig_strongest_map(toi_ctx* ctx, const float* cube, int32_t n_maps, const int32_t* boxes,
                                int32_t n_boxes, int32_t* k_out);

/* Several snapshots in one call (uneven sample counts allowed): for each i,
 * toi_grid(snaps[i]) + toi_image(images_out + i*N*N), and for i >= 2 the
 * tLISI map of (i-2, i-1, i) into tlisi_out + (i-2)*(N/tile)^2 (nullable);
 * the pipeline of Section 4.1 as one launch.  snaps is a HOST array of n
 * descriptors.  The whole batch is captured into one HIP graph, cached for
 * the same descriptors and outputs and replayed on the context's stream (a
 * new set recaptures; capture allocates graph resources on first use).  With
 * n >= 2 the graph has two lanes: the sample prep and binning of snapshot
 * i + 1 run while snapshot i is gridded and transformed, into a second set of
 * per-snapshot buffers (plan, records, bins; the size of the first set's,
 * allocated on the first such call and kept by the context; TOI_ENOMEM if it
 * cannot be).  The descriptors' arrays must be ready when the launch starts
 * on the context's stream.  The context's grid workspace holds the last
 * snapshot's planes afterwards; toi_plan_info then reports the plan of the
 * last even-indexed snapshot of the batch. */
toi_status toi_image_batch(toi_ctx* ctx, const toi_snapshot* snaps, int32_t n,
                           float* images_out, float* tlisi_out);

/* Input slots for a stream of batches (the ring of device buffers behind
 * Section 4.1's pipeline): n context-owned sets of snapshot arrays in the
 * layouts above, each sized for n_row_max rows (uvw, vis, freq, ant1, ant2,
 * and flag / weight / gains when `arrays` has TOI_INPUT_FLAG /
 * TOI_INPUT_WEIGHT / TOI_INPUT_GAINS; gains need n_ant > 0).  descs_out[i]
 * (caller-owned host array of n) receives slot i's device pointers with
 * n_row = n_row_max.  The slots are allocated on the first call and kept by
 * the context; a later call with n no larger and the same `arrays` returns
 * the same pointers, otherwise the slots are freed (after the context's
 * stream drains) and reallocated, and earlier descriptors become invalid.
 * Filling the slots (toi_batch_fill, or any copy or kernel ordered before the
 * batch on the context's stream) and passing the same descriptors, outputs
 * and n to toi_image_batch each time replays the captured graph: a stream of
 * new data costs no new capture (a changed n_row in a descriptor does).
 * TOI_ENOMEM if the slots cannot be allocated. */
#define TOI_INPUT_FLAG 1u
#define TOI_INPUT_WEIGHT 2u
#define TOI_INPUT_GAINS 4u
toi_status toi_batch_inputs(toi_ctx* ctx, int32_t n, uint32_t arrays, toi_snapshot* descs_out);

/* Copy one snapshot (src: device or page-locked host arrays, n_row <= n_row_max,
 * the same optional arrays as the slots) into input slot `slot` of
 * toi_batch_inputs, asynchronously on the context's stream (rows beyond
 * src->n_row are left as they were). */
toi_status toi_batch_fill(toi_ctx* ctx, int32_t slot, const toi_snapshot* src);

/* Diagnostics: graphs captured and launched by toi_image_batch so far on ctx. */
toi_status toi_batch_info(toi_ctx* ctx, int64_t* captures, int64_t* launches);

/* Streaming ingest (the paper's host pipeline, Section 4: data read and
 * copied to the device while the GPU images): host_snaps holds n snapshot
 * descriptors whose arrays are HOST pointers, in the layouts above.  For each
 * snapshot the library copies the arrays into one of two device staging
 * slots on an internal copy stream (default priority) and images the slot on
 * the context's stream: the copy of snapshot i + 1 overlaps the imaging of
 * snapshot i, and a slot is refilled once the gridding that read it has
 * finished.  Page-locked host memory (hipHostMalloc, a pinned torch tensor)
 * makes the copies asynchronous DMA; pageable memory works, without overlap.
 * images_out (device f32[n][N][N]) and tlisi_out (device f32[n - 2][T][T],
 * nullable) as in toi_image_batch.  The staging (2 x the largest snapshot's
 * arrays) is allocated on the first call and kept by the context.
 * Asynchronous on the context's stream; the host arrays must stay valid and
 * unchanged until the stream has passed the call's work.  Errors as for
 * toi_image_batch. */
toi_status toi_ingest(toi_ctx* ctx, const toi_snapshot* host_snaps, int32_t n,
                      float* images_out, float* tlisi_out);

/* Autotuning of the gridder (batched use).  The gridder accumulates each
 * bin (grid tile) of a plane group in one wavefront's matrix-core
 * accumulators, over a work unit of the bin's item list; the variants differ
 * in the work-unit size (bits 0-1: bins are split into units of at most
 * 32 << bits items -- the subgrid work granularity), the plane schedule
 * (bit 2: 8 planes per pass over a tile on the FP32 matrix cores, else 16
 * planes per pass on the fp16 matrix cores with operands split as hi + lo)
 * and the bin size (bit 3, variants 8 .. 11, 16 planes per pass: bins of
 * 16 x 16 cells instead of 8 x 8 where the grid side is at least 256; the
 * adjoint then bins the snapshot again at 8 x 8 before its gather).
 * Every variant computes the same image up to FP32 rounding order, and each
 * variant's image is the same from run to run.  toi_tune synchronises, times
 * grid + image of `sample` with every variant (HIP events, after one
 * warm-up), keeps the fastest in the context and returns it in *variant_out;
 * ms_out (host, TOI_TUNE_VARIANTS entries, nullable) receives each variant's
 * time.  It overwrites the context's workspaces.  toi_set_tuning selects a
 * variant directly (default 1: 64-item units, 16 planes per pass). */
#define TOI_TUNE_VARIANTS 12
toi_status toi_tune(toi_ctx* ctx, const toi_snapshot* sample, int32_t* variant_out, float* ms_out);
toi_status toi_set_tuning(toi_ctx* ctx, int32_t variant);

/* Synchronise and report the last gridded snapshot's plan (host outputs, each
 * nullable): V row-major, omega, W (sum of weights), N_slab, K, and the status
 * word.  Diagnostics only: the imaging loop never calls it. */
toi_status toi_plan_info(toi_ctx* ctx, double V_out[9], double* omega, double* wsum,
                         int32_t* n_slab, int32_t* cheb_k, uint32_t* status);

/* Synchronise and report the gridding work of the last gridded snapshot (host
 * outputs, each nullable; diagnostics for measurement, never called by the
 * imaging loop): entries = (work item, bin, plane group) entries of the bin
 * lists (8 x 8 bins, or 16 x 16 for the variants with bit 3); tiles = (plane
 * group, 8 x 8 tile) pairs the gridder writes and the row pass reads, per
 * plane of the group (tiles holding samples, or part of a 16 x 16 bin that
 * does);
 * tile_rows = (plane group, tile row) pairs holding samples (the row pass
 * writes 8 grid rows of N kept bins per plane of the group for each);
 * units = work units of split bins. */
toi_status toi_bin_info(toi_ctx* ctx, int64_t* entries, int64_t* tiles, int64_t* tile_rows, int64_t* units);

/* Measurement support.  Stages timed with HIP events on the context's stream:
 * TOI_STAGE_PREP (sample statistics, basis, plan), TOI_STAGE_BIN (work
 * items, gridding records, bin scan, work units and lists), TOI_STAGE_GRID
 * (gridding), TOI_STAGE_FFT_ROWS, TOI_STAGE_FFT_COLS
 * (column FFT + correction + combination), TOI_STAGE_REPROJECT,
 * TOI_STAGE_TLISI, TOI_STAGE_DEGRID (adjoint), TOI_STAGE_BATCH (one whole
 * toi_image_batch graph launch; its kernels are not timed individually).
 * toi_profile_enable(ctx, stage_mask) times the stages whose bit
 * (1 << TOI_STAGE_x) is set (TOI_PROFILE_ALL: every stage; 0 disables
 * recording; bits past TOI_NSTAGE are ignored); it creates the events on
 * first use and clears the totals.  Each timed launch adds two event records
 * to the stream, so timing fewer stages disturbs the timed work less.
 * toi_profile_read synchronises the stream and writes, per stage, the summed
 * duration in milliseconds and the number of timed launches (host arrays of
 * TOI_NSTAGE entries, each nullable). */
#define TOI_STAGE_PREP 0
#define TOI_STAGE_BIN 1
#define TOI_STAGE_GRID 2
#define TOI_STAGE_FFT_ROWS 3
#define TOI_STAGE_FFT_COLS 4
#define TOI_STAGE_REPROJECT 5
#define TOI_STAGE_TLISI 6
#define TOI_STAGE_DEGRID 7
#define TOI_STAGE_BATCH 8
#define TOI_STAGE_DETECT 9
#define TOI_NSTAGE 10
#define TOI_PROFILE_ALL ((1 << TOI_NSTAGE) - 1)
toi_status toi_profile_enable(toi_ctx* ctx, int32_t stage_mask);
toi_status toi_profile_read(toi_ctx* ctx, double* total_ms, int32_t* launches);

/* Message for the last failing call on ctx (or a global one if ctx is NULL). */
const char* toi_last_error(const toi_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TOI_H */
