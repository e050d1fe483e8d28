// Host runtime of libtoi: context creation (the only allocating call), argument
// validation, the host-built tables and the C ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "toi_fft.h"
#include "toi_internal.h"

namespace {
std::mutex g_err_mu;
std::string g_err;   // message of the last failure without a context

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }
}  // namespace

namespace toi {

toi_status fail(toi_ctx* ctx, toi_status st, const std::string& msg) {
    if (ctx) {
        ctx->err = msg;
    } else {
        std::lock_guard<std::mutex> lk(g_err_mu);
        g_err = msg;
    }
    return st;
}

toi_status hip_check(toi_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return TOI_OK;
    return fail(ctx, TOI_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
}

// Grid correction of the ES kernel: psi(a) = (W/2) int_{-1}^{1} phi(z) cos(pi W z a / M) dz,
// a = j - N/2; stored as (-1)^a / psi(a) so that one real factor per axis also
// undoes the half-grid shift of the FFT origin.
void es_correction_table(int N, int M, double* out) {
    std::vector<double> z, w;
    gauss_legendre(128, z, w);
    const double beta = kEsBetaPerW * kSupport;
    for (int j = 0; j < N; ++j) {
        const double a = j - N / 2;
        double s = 0.0;
        for (size_t q = 0; q < z.size(); ++q) {
            const double phi = std::exp(beta * (std::sqrt(1.0 - z[q] * z[q]) - 1.0));
            s += w[q] * phi * std::cos(kPi * kSupport * z[q] * a / M);
        }
        const double psi = 0.5 * kSupport * s;
        const double sign = ((j - N / 2) % 2 == 0) ? 1.0 : -1.0;
        out[j] = sign / psi;
    }
}

StageTimer::StageTimer(toi_ctx* ctx, int stage) : c(ctx), slot(-1) {
    if (!((c->prof_mask >> stage) & 1u) || c->prof_n >= c->prof_stage.size()) return;
    slot = (int)c->prof_n++;
    c->prof_stage[slot] = stage;
    (void)hipEventRecord(c->prof_ev[2 * slot], c->stream);
}

StageTimer::~StageTimer() {
    if (slot >= 0) (void)hipEventRecord(c->prof_ev[2 * slot + 1], c->stream);
}

void front_bytes(const toi_ctx* c, size_t out[kFrontBuffers]) {
    const toi_params& p = c->p;
    const size_t NT = c->NT, NG = c->NG_max, words = (NT + 31) / 32;
    out[0] = sizeof(DevPlan);
    out[1] = std::max<size_t>(1, p.n_row_max) * sizeof(RowStat);
    out[2] = (size_t)c->n_items_max * sizeof(ItemBox);
    out[3] = std::max<size_t>(1, (size_t)p.n_row_max * p.n_chan) * sizeof(SampleRec);
    out[4] = NG * NT * NT * sizeof(int32_t);                                              // bin_count
    out[5] = (NG * NT * NT + 1) * sizeof(int32_t);                                        // bin_off
    out[6] = NG * NT * NT * sizeof(int32_t);                                              // bin_cursor
    out[7] = (size_t)c->bin_cap * sizeof(int32_t);                                        // bin_list
    out[8] = NG * NT * NT * sizeof(int32_t);                                              // bin_order
    out[9] = (kAuxTotals + 2 * ((NG * NT * NT + kScanBlock - 1) / kScanBlock)) * sizeof(int32_t); // bin_aux
    out[10] = (size_t)kSplitSlots * sizeof(int4);                                         // units
    out[11] = NG * NT * words * sizeof(uint32_t);                                         // tile_bits
    out[12] = NG * words * sizeof(uint32_t);                                              // row_bits
    out[13] = 64 * sizeof(int32_t);                                                       // scratch_i
}

void front_swap(toi_ctx* c) {
    toi_front& a = c->alt;
    std::swap(c->plan, a.plan);
    std::swap(c->rows, a.rows);
    std::swap(c->items, a.items);
    std::swap(c->recs, a.recs);
    std::swap(c->bin_count, a.bin_count);
    std::swap(c->bin_off, a.bin_off);
    std::swap(c->bin_cursor, a.bin_cursor);
    std::swap(c->bin_list, a.bin_list);
    std::swap(c->bin_order, a.bin_order);
    std::swap(c->bin_aux, a.bin_aux);
    std::swap(c->units, a.units);
    std::swap(c->tile_bits, a.tile_bits);
    std::swap(c->row_bits, a.row_bits);
    std::swap(c->scratch_i, a.scratch_i);
}

}  // namespace toi

using namespace toi;

extern "C" {

toi_status toi_params_default(toi_params* p, int32_t n_pix, double cell_deg, int32_t n_row_max,
                              int32_t n_chan, int32_t n_corr) {
    if (!p) return fail(nullptr, TOI_EINVAL, "toi_params_default: p is NULL");
    std::memset(p, 0, sizeof(*p));
    p->n_pix = n_pix;
    p->cell_deg = cell_deg;
    p->mode = 3;
    p->n_slab = 0;
    p->cheb_k = 0;
    p->alpha_target = 10.0;
    p->cheb_gamma = 1e-2;
    p->max_planes = 0;
    p->support = kSupport;
    p->corr_mask = 0;
    p->tile = 32;
    p->n_row_max = n_row_max;
    p->n_chan = n_chan;
    p->n_corr = n_corr;
    p->n_ant = 0;
    return TOI_OK;
}

static uint32_t default_mask(int n_corr) {
    return n_corr == 4 ? 0x9u : (n_corr == 2 ? 0x3u : 0x1u);
}

toi_status toi_create(const toi_params* pin, void* hip_stream, toi_ctx** out) {
    if (!out) return fail(nullptr, TOI_EINVAL, "toi_create: out is NULL");
    *out = nullptr;
    if (!pin) return fail(nullptr, TOI_EINVAL, "toi_create: params is NULL");
    toi_params p = *pin;
    if (!is_pow2(p.n_pix) || p.n_pix < 32 || p.n_pix > 4096)
        return fail(nullptr, TOI_EINVAL, "toi_create: n_pix must be a power of two in [32, 4096]");
    if (!(p.cell_deg > 0.0) || p.cell_deg * p.n_pix >= 180.0)
        return fail(nullptr, TOI_EINVAL, "toi_create: cell_deg must be > 0 and the field < 180 deg");
    if (p.mode != 2 && p.mode != 3) return fail(nullptr, TOI_EINVAL, "toi_create: mode must be 2 or 3");
    if (p.support != kSupport)
        return fail(nullptr, TOI_EUNSUPPORTED, "toi_create: only gridding support 8 is implemented");
    if (p.n_corr != 1 && p.n_corr != 2 && p.n_corr != 4)
        return fail(nullptr, TOI_EINVAL, "toi_create: n_corr must be 1, 2 or 4");
    if (p.n_chan <= 0 || p.n_row_max < 0 || p.n_ant < 0)
        return fail(nullptr, TOI_EINVAL, "toi_create: n_chan must be > 0, n_row_max and n_ant >= 0");
    if (p.corr_mask == 0) p.corr_mask = default_mask(p.n_corr);
    if (p.corr_mask >> p.n_corr)
        return fail(nullptr, TOI_EINVAL, "toi_create: corr_mask selects a correlation >= n_corr");
    if (p.tile <= 0 || p.tile > p.n_pix || (p.n_pix % p.tile))
        return fail(nullptr, TOI_EINVAL, "toi_create: tile must divide n_pix");
    if (p.n_slab < 0 || p.cheb_k < 0 || p.cheb_k > 32 || p.max_planes < 0)
        return fail(nullptr, TOI_EINVAL, "toi_create: n_slab, cheb_k in [0, 32], max_planes must be >= 0");
    if (p.bin_cap < 0) return fail(nullptr, TOI_EINVAL, "toi_create: bin_cap must be >= 0");
    if (!(p.alpha_target > 0.0) || !(p.cheb_gamma > 0.0))
        return fail(nullptr, TOI_EINVAL, "toi_create: alpha_target and cheb_gamma must be > 0");

    toi_ctx* c = new toi_ctx();
    c->p = p;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->N = p.n_pix;
    c->M = 2 * p.n_pix;
    c->T = p.n_pix / p.tile;
    if (p.mode == 2) {
        c->P_cap = 1;
        c->forced_K = 1;
    } else {
        const int fk = p.cheb_k;
        c->forced_K = fk;
        int cap = p.max_planes;
        if (cap == 0) cap = (p.n_slab > 0 && fk > 0) ? p.n_slab * fk : 32;
        if (p.n_slab > 0 && fk > 0 && p.n_slab * fk > cap)
            return delete c, fail(nullptr, TOI_EINVAL, "toi_create: n_slab * cheb_k exceeds max_planes");
        c->P_cap = cap;
    }
    c->tuning = kTuneDefault;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, TOI_EDEVICE, "toi_create: no HIP device");
    }

    const size_t N = c->N, M = c->M, P = c->P_cap, T = c->T;
    c->NT = c->M / kTile;
    c->bins_shift = kTileShift;
    c->NG_max = std::max(1, c->P_cap);   // every group holds at least one plane
    c->n_items_max = std::max(1, p.n_row_max * ((p.n_chan + kItemChans - 1) / kItemChans));
    // default: 128 (tile, plane group) entries per work item on average; an
    // item's box of tiles grows with the track length its 64 channels span
    // (about 5 entries per item at 4096 channels over 856-1712 MHz, some 60-100
    // at 512 channels over the same band on a 8192^2 grid)
    c->bin_cap = p.bin_cap > 0 ? p.bin_cap : c->n_items_max * 128 + 65536;
    size_t fb[kFrontBuffers];
    front_bytes(c, fb);
    struct Alloc { void** ptr; size_t bytes; };
    Alloc allocs[] = {
        {(void**)&c->plan, fb[0]},
        {(void**)&c->rows, fb[1]},
        {(void**)&c->items, fb[2]},
        {(void**)&c->recs, fb[3]},
        {(void**)&c->bin_count, fb[4]},
        {(void**)&c->bin_off, fb[5]},
        {(void**)&c->bin_cursor, fb[6]},
        {(void**)&c->bin_list, fb[7]},
        {(void**)&c->bin_order, fb[8]},
        {(void**)&c->bin_aux, fb[9]},
        {(void**)&c->units, fb[10]},
        {(void**)&c->tile_bits, fb[11]},
        {(void**)&c->row_bits, fb[12]},
        {(void**)&c->scratch_i, fb[13]},
        {(void**)&c->gx, std::max<size_t>(1, (size_t)p.n_row_max * p.n_chan) * 2 * sizeof(uint64_t)},
        {(void**)&c->split_part, (size_t)kSplitSlots * kPartFloats * sizeof(float)},
        {(void**)&c->grid, P * M * M * sizeof(float2)},
        {(void**)&c->hbuf, P * N * M * sizeof(float2)},
        {(void**)&c->tplane_t, N * N * sizeof(float)},
        {(void**)&c->adj_tp, N * N * sizeof(uint64_t)},
        {(void**)&c->adj_parts, std::max<size_t>(kAdjAbsmaxParts, M / 2 * P) * sizeof(float)},
        {(void**)&c->item_gain, ((size_t)c->n_items_max + std::max(1, p.n_row_max)) * sizeof(double2)},
        {(void**)&c->corr, N * sizeof(float)},
        {(void**)&c->twiddle, (size_t)fft_twiddle_entries((int)M) * sizeof(float2)},
        {(void**)&c->tiles, T * T * sizeof(TileStat)},
        {(void**)&c->scratch_d, 64 * sizeof(double)},
        {(void**)&c->det_scores, 2 * T * T * sizeof(double)},
        {(void**)&c->det_boxes, T * T * sizeof(int4)},
    };
    for (auto& a : allocs) {
        if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
            for (auto& b : allocs)
                if (*b.ptr) (void)hipFree(*b.ptr);
            delete c;
            return fail(nullptr, TOI_ENOMEM, "toi_create: workspace allocation failed");
        }
    }
    // host-built tables: ES grid correction and FFT twiddles, computed in FP64
    std::vector<double> corr_d(N);
    es_correction_table((int)N, (int)M, corr_d.data());
    std::vector<float> corr_f(N);
    for (size_t j = 0; j < N; ++j) corr_f[j] = (float)corr_d[j];
    std::vector<float2> tw(M);
    for (size_t n = 0; n < M; ++n) {
        const double a = 2.0 * kPi * (double)n / (double)M;
        tw[n] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    // stage tables of radix 8, 16, 32 after the full-period table: entry
    // (stage NS, k, r) = tw[r k M / (NS E)]
    for (int E = 8; E <= 32; E *= 2)
        for (int ns = fft_first_radix((int)M, E); ns < (int)M; ns *= E)
            for (int k = 0; k < ns; ++k)
                for (int r = 1; r < E; ++r) tw.push_back(tw[(size_t)r * k * (M / ((size_t)ns * E))]);
    if (tw.size() != (size_t)fft_twiddle_entries((int)M)) {
        toi_destroy(c);
        return fail(nullptr, TOI_EINVAL, "toi_create: twiddle table size mismatch");
    }
    DevPlan zero{};
    hipError_t e = hipMemcpy(c->corr, corr_f.data(), N * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->twiddle, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->plan, &zero, sizeof(DevPlan), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        toi_destroy(c);
        return fail(nullptr, TOI_EDEVICE, std::string("toi_create: table upload: ") + hipGetErrorString(e));
    }
    *out = c;
    return TOI_OK;
}

toi_status toi_destroy(toi_ctx* c) {
    if (!c) return TOI_OK;
    (void)hipStreamSynchronize(c->stream);
    ingest_release(c);
    ring_release(c);
    for (auto& e : c->prof_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->cap_stream2) (void)hipStreamDestroy(c->cap_stream2);
    for (hipEvent_t ev : c->batch_ev)
        if (ev) (void)hipEventDestroy(ev);
    {
        toi_front& a = c->alt;
        void* alt_ptrs[] = {a.plan, a.rows, a.items, a.recs, a.bin_count, a.bin_off, a.bin_cursor,
                            a.bin_list, a.bin_order, a.bin_aux, a.units, a.tile_bits, a.row_bits, a.scratch_i};
        for (void* q : alt_ptrs)
            if (q) (void)hipFree(q);
    }
    if (c->batch_exec) (void)hipGraphExecDestroy(c->batch_exec);
    if (c->batch_graph) (void)hipGraphDestroy(c->batch_graph);
    void* ptrs[] = {c->items, c->recs, c->gx, c->bin_order, c->bin_aux, c->units, c->split_part,
                    c->bin_count, c->bin_off, c->bin_cursor, c->bin_list, c->tile_bits, c->row_bits,
                    c->adj_tp, c->adj_parts, c->item_gain, c->grid, c->hbuf, c->tplane_t, c->plan, c->rows, c->corr, c->twiddle, c->tiles,
                    c->scratch_d, c->scratch_i, c->det_scores, c->det_boxes};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete c;
    return TOI_OK;
}

toi_status toi_set_stream(toi_ctx* c, void* s) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_set_stream: ctx is NULL");
    c->stream = reinterpret_cast<hipStream_t>(s);
    return TOI_OK;
}

static toi_status check_snapshot(toi_ctx* c, const toi_snapshot* s, const char* who) {
    if (!s) return fail(c, TOI_EINVAL, std::string(who) + ": snapshot is NULL");
    if (s->n_row < 0 || s->n_row > c->p.n_row_max)
        return fail(c, TOI_EINVAL, std::string(who) + ": n_row outside [0, n_row_max]");
    if (s->n_row > 0 && (!s->uvw || !s->vis || !s->freq))
        return fail(c, TOI_EINVAL, std::string(who) + ": uvw, vis and freq are required");
    if (s->gains && (!s->ant1 || !s->ant2))
        return fail(c, TOI_EINVAL, std::string(who) + ": gains need ant1 and ant2");
    if (s->gains && c->p.n_ant <= 0)
        return fail(c, TOI_EINVAL, std::string(who) + ": gains given but n_ant is 0");
    return TOI_OK;
}

toi_status toi_grid(toi_ctx* c, const toi_snapshot* s) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_grid: ctx is NULL");
    toi_status st = check_snapshot(c, s, "toi_grid");
    if (st != TOI_OK) return st;
    st = hip_check(c, launch_prep(c, *s), "toi_grid: prep");
    if (st != TOI_OK) return st;
    return hip_check(c, launch_grid(c, *s), "toi_grid: gridding");
}

toi_status toi_image(toi_ctx* c, float* image_out, float* tplane_out) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_image: ctx is NULL");
    if (!image_out) return fail(c, TOI_EINVAL, "toi_image: image_out is NULL");
    return hip_check(c, launch_image(c, image_out, tplane_out), "toi_image");
}

toi_status toi_degrid(toi_ctx* c, const float* grad_image, const toi_snapshot* s, void* grad_vis,
                      void* grad_gains) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_degrid: ctx is NULL");
    if (!grad_image) return fail(c, TOI_EINVAL, "toi_degrid: grad_image is NULL");
    toi_status st = check_snapshot(c, s, "toi_degrid");
    if (st != TOI_OK) return st;
    if (grad_gains && !s->gains) return fail(c, TOI_EINVAL, "toi_degrid: grad_gains needs gains");
    return hip_check(c, launch_degrid(c, grad_image, *s, (float2*)grad_vis, (float2*)grad_gains),
                     "toi_degrid");
}

toi_status fitrig_tlisi(toi_ctx* c, const float* a, const float* b, const float* d, float* out) {
    if (!c) return fail(nullptr, TOI_EINVAL, "fitrig_tlisi: ctx is NULL");
    if (!a || !b || !d || !out) return fail(c, TOI_EINVAL, "fitrig_tlisi: NULL image or output");
    return hip_check(c, launch_tlisi(c, a, b, d, out), "fitrig_tlisi");
}

toi_status fitrig_detect(toi_ctx* c, const float* window, int32_t t, int32_t* boxes, int32_t max_boxes,
                         int32_t* n_boxes) {
    if (!c) return fail(nullptr, TOI_EINVAL, "fitrig_detect: ctx is NULL");
    if (!window || !n_boxes || (max_boxes > 0 && !boxes) || max_boxes < 0)
        return fail(c, TOI_EINVAL, "fitrig_detect: NULL window/boxes/count or max_boxes < 0");
    return hip_check(c, launch_detect(c, window, t, boxes, max_boxes, n_boxes), "fitrig_detect");
}

toi_status fitrig_localise(toi_ctx* c, const float* img_a, const float* img_b, const int32_t* boxes,
                           int32_t n_boxes, double ra0_deg, double dec0_deg, int32_t morph, double* out) {
    if (!c) return fail(nullptr, TOI_EINVAL, "fitrig_localise: ctx is NULL");
    if (n_boxes < 0 || (n_boxes > 0 && (!img_a || !img_b || !boxes || !out)))
        return fail(c, TOI_EINVAL, "fitrig_localise: NULL image/boxes/output or n_boxes < 0");
    return hip_check(c, launch_localise(c, img_a, img_b, boxes, n_boxes, ra0_deg, dec0_deg, morph, out),
                     "fitrig_localise");
}

toi_status fitrig_strongest_map(toi_ctx* c, const float* cube, int32_t n_maps, const int32_t* boxes,
                                int32_t n_boxes, int32_t* k_out) {
    if (!c) return fail(nullptr, TOI_EINVAL, "fitrig_strongest_map: ctx is NULL");
    if (n_boxes < 0 || n_maps < 1 || (n_boxes > 0 && (!cube || !boxes || !k_out)))
        return fail(c, TOI_EINVAL, "fitrig_strongest_map: NULL cube/boxes/output, n_boxes < 0 or n_maps < 1");
    return hip_check(c, launch_strongest_map(c, cube, n_maps, boxes, n_boxes, k_out), "fitrig_strongest_map");
}

toi_status fitrig_detect_cube(toi_ctx* c, const float* cube, int32_t n_maps, int32_t t, int32_t* boxes,
                              int32_t max_boxes, int32_t* n_boxes) {
    if (!c) return fail(nullptr, TOI_EINVAL, "fitrig_detect_cube: ctx is NULL");
    if (!cube || !n_boxes || (max_boxes > 0 && !boxes) || max_boxes < 0)
        return fail(c, TOI_EINVAL, "fitrig_detect_cube: NULL cube/boxes/count or max_boxes < 0");
    if (n_maps < 2 || n_maps > 5460)
        return fail(c, TOI_EINVAL, "fitrig_detect_cube: n_maps must be in [2, 5460]");
    return hip_check(c, launch_detect_cube(c, cube, n_maps, t, boxes, max_boxes, n_boxes), "fitrig_detect_cube");
}

toi_status toi_plan_info(toi_ctx* c, double V_out[9], double* omega, double* wsum, int32_t* n_slab,
                         int32_t* cheb_k, uint32_t* status) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_plan_info: ctx is NULL");
    DevPlan h{};
    hipError_t e = hipMemcpyAsync(&h, c->plan, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "toi_plan_info");
    if (V_out) std::memcpy(V_out, h.V, sizeof(h.V));
    if (omega) *omega = h.omega;
    if (wsum) *wsum = h.wsum;
    if (n_slab) *n_slab = h.n_slab;
    if (cheb_k) *cheb_k = h.K;
    if (status) *status = h.status;
    return TOI_OK;
}

toi_status toi_bin_info(toi_ctx* c, int64_t* entries, int64_t* tiles, int64_t* tile_rows, int64_t* units) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_bin_info: ctx is NULL");
    DevPlan h{};
    const int NT = c->NT, words = (NT + 31) / 32, NB = c->M >> c->bins_shift;
    const size_t n_bins = (size_t)c->NG_max * NB * NB;
    int32_t total = 0, cnt[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(&h, c->plan, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&total, c->bin_off + n_bins, sizeof(total), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt, c->scratch_i, sizeof(cnt), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "toi_bin_info");
    const int ng = std::max(0, std::min(h.ng, c->NG_max));
    std::vector<uint32_t> tb((size_t)ng * NT * words), rb((size_t)ng * words);
    if (ng > 0) {
        e = hipMemcpy(tb.data(), c->tile_bits, tb.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(rb.data(), c->row_bits, rb.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_check(c, e, "toi_bin_info");
    }
    int64_t nt = 0, nr = 0;
    for (uint32_t w : tb) nt += __builtin_popcount(w);
    for (uint32_t w : rb) nr += __builtin_popcount(w);
    if (entries) *entries = total;
    if (tiles) *tiles = nt;
    if (tile_rows) *tile_rows = nr;
    if (units) *units = cnt[1];
    return TOI_OK;
}

toi_status toi_profile_enable(toi_ctx* c, int32_t stage_mask) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_profile_enable: ctx is NULL");
    c->prof_mask = (uint32_t)stage_mask & ((1u << TOI_NSTAGE) - 1u);
    c->prof_n = 0;
    if (c->prof_mask && c->prof_ev.empty()) {
        const size_t cap = 8192;
        c->prof_ev.resize(2 * cap);
        c->prof_stage.assign(cap, 0);
        for (auto& e : c->prof_ev) {
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return hip_check(c, err, "toi_profile_enable");
        }
    }
    return TOI_OK;
}

toi_status toi_profile_read(toi_ctx* c, double* total_ms, int32_t* launches) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_profile_read: ctx is NULL");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_check(c, e, "toi_profile_read");
    double tot[TOI_NSTAGE] = {0};
    int32_t cnt[TOI_NSTAGE] = {0};
    for (size_t i = 0; i < c->prof_n; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]);
        if (e != hipSuccess) return hip_check(c, e, "toi_profile_read");
        tot[c->prof_stage[i]] += ms;
        cnt[c->prof_stage[i]] += 1;
    }
    for (int s = 0; s < TOI_NSTAGE; ++s) {
        if (total_ms) total_ms[s] = tot[s];
        if (launches) launches[s] = cnt[s];
    }
    return TOI_OK;
}

toi_status toi_set_tuning(toi_ctx* c, int32_t variant) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_set_tuning: ctx is NULL");
    if (variant < 0 || variant >= TOI_TUNE_VARIANTS) return fail(c, TOI_EINVAL, "toi_set_tuning: variant out of range");
    c->tuning = variant;
    return TOI_OK;
}

toi_status toi_tune(toi_ctx* c, const toi_snapshot* s, int32_t* variant_out, float* ms_out) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_tune: ctx is NULL");
    toi_status st = check_snapshot(c, s, "toi_tune");
    if (st != TOI_OK) return st;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    const uint32_t prof = c->prof_mask;
    c->prof_mask = 0;
    int best = c->tuning;
    float best_ms = 1e30f;
    for (int v = 0; v < TOI_TUNE_VARIANTS && e == hipSuccess; ++v) {
        c->tuning = v;
        float ms = 0.f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {   // first repetition warms up
            if (rep == 1) e = hipEventRecord(a, c->stream);
            if (e == hipSuccess) e = launch_prep(c, *s);
            if (e == hipSuccess) e = launch_grid(c, *s);
            if (e == hipSuccess) e = launch_image(c, c->adj_tp, nullptr);
        }
        if (e == hipSuccess) e = hipEventRecord(b, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        ms *= 0.5f;
        if (ms_out) ms_out[v] = ms;
        if (e == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    c->prof_mask = prof;
    c->tuning = best;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_check(c, e, "toi_tune");
    if (variant_out) *variant_out = best;
    return TOI_OK;
}

const char* toi_last_error(const toi_ctx* c) {
    if (c) return c->err.c_str();
    std::lock_guard<std::mutex> lk(g_err_mu);
    return g_err.c_str();
}

}  // extern "C"
