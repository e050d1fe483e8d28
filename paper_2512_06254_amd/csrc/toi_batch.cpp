// Batched execution: many snapshots (uneven flagged-sample counts allowed) in
// one HIP graph launch.  The per-snapshot kernel chain (sample statistics,
// basis and plan, binning, gridding, FFT passes, re-projection, and the tLISI
// map of the three youngest images) is captured once for a given set of
// snapshot descriptors and outputs, instantiated, cached in the context and
// replayed on the caller's stream; a different descriptor set recaptures.
// With two or more snapshots the chain runs in two lanes, as the pipeline of
// Section 4.1 overlaps its stages: the prep and binning of snapshot i + 1
// (lane B, memory- and latency-bound, writing the other of two per-snapshot
// sets) run while snapshot i is gridded and transformed (lane A, bound by
// vector-ALU issue).  Lane B waits until the transform of snapshot i - 1, the
// last reader of that set, has finished.  (Gridding in lane B as well, beside
// the transforms, measured no faster: the gridder's single-wave workgroups
// take every freed CU slot and the FFT workgroups, which need 67.5 KB of LDS
// at once, wait behind them.)
// No host synchronisation and no allocation happen inside the graph.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "toi_internal.h"

namespace {

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

using namespace toi;

// Input slots of toi_batch_inputs: one set of snapshot arrays per slot, each
// sized for n_row_max rows, allocated once and kept by the context.
struct toi_batch_ring {
    int n = 0;
    uint32_t arrays = 0;
    std::vector<void*> bufs;
    std::vector<toi_snapshot> desc;
};

void toi::ring_release(toi_ctx* c) {
    if (!c || !c->ring) return;
    for (void* q : c->ring->bufs)
        if (q) (void)hipFree(q);
    delete c->ring;
    c->ring = nullptr;
}

extern "C" toi_status toi_batch_inputs(toi_ctx* c, int32_t n, uint32_t arrays, toi_snapshot* descs_out) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_batch_inputs: ctx is NULL");
    if (n < 1 || !descs_out) return fail(c, TOI_EINVAL, "toi_batch_inputs: n >= 1 and descs_out are required");
    if (arrays & ~(uint32_t)(TOI_INPUT_FLAG | TOI_INPUT_WEIGHT | TOI_INPUT_GAINS))
        return fail(c, TOI_EINVAL, "toi_batch_inputs: unknown bit in arrays");
    if ((arrays & TOI_INPUT_GAINS) && c->p.n_ant <= 0)
        return fail(c, TOI_EINVAL, "toi_batch_inputs: gains need n_ant > 0");
    if (!c->ring || c->ring->n < n || c->ring->arrays != arrays) {
        (void)hipStreamSynchronize(c->stream);   // the previous slots may still be read
        ring_release(c);
        toi_batch_ring* r = new toi_batch_ring();
        c->ring = r;
        r->n = n;
        r->arrays = arrays;
        const size_t rows = (size_t)std::max(1, c->p.n_row_max), chan = c->p.n_chan, corr = c->p.n_corr;
        auto get = [&](size_t bytes) -> void* {
            void* q = nullptr;
            if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
            r->bufs.push_back(q);
            return q;
        };
        for (int i = 0; i < n; ++i) {
            toi_snapshot d{};
            d.uvw = static_cast<const double*>(get(rows * 3 * sizeof(double)));
            d.vis = get(rows * chan * corr * 2 * sizeof(float));
            d.freq = static_cast<const double*>(get(chan * sizeof(double)));
            d.ant1 = static_cast<const int32_t*>(get(rows * sizeof(int32_t)));
            d.ant2 = static_cast<const int32_t*>(get(rows * sizeof(int32_t)));
            bool ok = d.uvw && d.vis && d.freq && d.ant1 && d.ant2;
            if (arrays & TOI_INPUT_FLAG) ok = ok && (d.flag = static_cast<const uint8_t*>(get(rows * chan * corr)));
            if (arrays & TOI_INPUT_WEIGHT)
                ok = ok && (d.weight = static_cast<const float*>(get(rows * chan * corr * sizeof(float))));
            if (arrays & TOI_INPUT_GAINS) ok = ok && (d.gains = get((size_t)c->p.n_ant * 2 * sizeof(float)));
            if (!ok) {
                ring_release(c);
                return fail(c, TOI_ENOMEM, "toi_batch_inputs: slot allocation failed");
            }
            d.n_row = c->p.n_row_max;
            r->desc.push_back(d);
        }
    }
    for (int i = 0; i < n; ++i) descs_out[i] = c->ring->desc[i];
    return TOI_OK;
}

extern "C" toi_status toi_batch_fill(toi_ctx* c, int32_t slot, const toi_snapshot* src) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_batch_fill: ctx is NULL");
    if (!c->ring || slot < 0 || slot >= c->ring->n)
        return fail(c, TOI_EINVAL, "toi_batch_fill: slot outside the slots of toi_batch_inputs");
    if (!src || src->n_row < 0 || src->n_row > c->p.n_row_max || (src->n_row > 0 && (!src->uvw || !src->vis || !src->freq)))
        return fail(c, TOI_EINVAL, "toi_batch_fill: src needs uvw, vis, freq and n_row in [0, n_row_max]");
    const toi_snapshot& d = c->ring->desc[slot];
    const uint32_t a = c->ring->arrays;
    if (((a & TOI_INPUT_FLAG) != 0) != (src->flag != nullptr) || ((a & TOI_INPUT_WEIGHT) != 0) != (src->weight != nullptr) ||
        ((a & TOI_INPUT_GAINS) != 0) != (src->gains != nullptr) || (src->gains && (!src->ant1 || !src->ant2)))
        return fail(c, TOI_EINVAL, "toi_batch_fill: src's optional arrays differ from the slots'");
    const size_t rows = src->n_row, chan = c->p.n_chan, corr = c->p.n_corr;
    struct Cp { void* dst; const void* s; size_t bytes; };
    const Cp cps[] = {
        {(void*)d.uvw, src->uvw, rows * 3 * sizeof(double)},
        {(void*)d.vis, src->vis, rows * chan * corr * 2 * sizeof(float)},
        {(void*)d.freq, src->freq, chan * sizeof(double)},
        {(void*)d.ant1, src->ant1, src->ant1 ? rows * sizeof(int32_t) : 0},
        {(void*)d.ant2, src->ant2, src->ant2 ? rows * sizeof(int32_t) : 0},
        {(void*)d.flag, src->flag, src->flag ? rows * chan * corr : 0},
        {(void*)d.weight, src->weight, src->weight ? rows * chan * corr * sizeof(float) : 0},
        {(void*)d.gains, src->gains, src->gains ? (size_t)c->p.n_ant * 2 * sizeof(float) : 0},
    };
    for (const Cp& q : cps) {
        if (!q.bytes) continue;
        const hipError_t e = hipMemcpyAsync(q.dst, q.s, q.bytes, hipMemcpyDefault, c->stream);
        if (e != hipSuccess) return hip_check(c, e, "toi_batch_fill: copy");
    }
    return TOI_OK;
}

extern "C" toi_status toi_batch_info(toi_ctx* c, int64_t* captures, int64_t* launches) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_batch_info: ctx is NULL");
    if (captures) *captures = c->batch_captures;
    if (launches) *launches = c->batch_launches;
    return TOI_OK;
}

extern "C" toi_status toi_image_batch(toi_ctx* c, const toi_snapshot* snaps, int32_t n, float* images_out,
                                      float* tlisi_out) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_image_batch: ctx is NULL");
    if (n < 0) return fail(c, TOI_EINVAL, "toi_image_batch: n < 0");
    if (n == 0) return TOI_OK;
    if (!snaps || !images_out) return fail(c, TOI_EINVAL, "toi_image_batch: snaps and images_out are required");
    for (int i = 0; i < n; ++i) {
        const toi_snapshot& s = snaps[i];
        if (s.n_row < 0 || s.n_row > c->p.n_row_max)
            return fail(c, TOI_EINVAL, "toi_image_batch: a snapshot's n_row is outside [0, n_row_max]");
        if (s.n_row > 0 && (!s.uvw || !s.vis || !s.freq))
            return fail(c, TOI_EINVAL, "toi_image_batch: uvw, vis and freq are required");
        if (s.gains && (!s.ant1 || !s.ant2 || c->p.n_ant <= 0))
            return fail(c, TOI_EINVAL, "toi_image_batch: gains need ant1, ant2 and n_ant > 0");
    }
    uint64_t key = 1469598103934665603ull;
    key = fnv1a(key, snaps, sizeof(toi_snapshot) * (size_t)n);
    key = fnv1a(key, &n, sizeof(n));
    key = fnv1a(key, &images_out, sizeof(images_out));
    key = fnv1a(key, &tlisi_out, sizeof(tlisi_out));

    if (!(c->batch_exec && c->batch_key == key)) {
        const bool two = n >= 2;
        if (!c->cap_stream) {
            hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_check(c, e, "toi_image_batch: capture stream");
        }
        if (two && !c->cap_stream2) {
            hipError_t e = hipStreamCreateWithFlags(&c->cap_stream2, hipStreamNonBlocking);
            for (int k = 0; k < 4 && e == hipSuccess; ++k)
                e = hipEventCreateWithFlags(&c->batch_ev[k], hipEventDisableTiming);
            if (e != hipSuccess) return hip_check(c, e, "toi_image_batch: second lane");
        }
        if (two && !c->alt_ready) {   // the second per-snapshot set, same sizes as the first
            size_t fb[kFrontBuffers];
            front_bytes(c, fb);
            toi_front& a = c->alt;
            void** ptrs[kFrontBuffers] = {(void**)&a.plan, (void**)&a.rows, (void**)&a.items, (void**)&a.recs,
                                          (void**)&a.bin_count, (void**)&a.bin_off, (void**)&a.bin_cursor,
                                          (void**)&a.bin_list, (void**)&a.bin_order, (void**)&a.bin_aux,
                                          (void**)&a.units, (void**)&a.tile_bits, (void**)&a.row_bits,
                                          (void**)&a.scratch_i};
            for (int k = 0; k < kFrontBuffers; ++k)
                if (!*ptrs[k] && hipMalloc(ptrs[k], fb[k]) != hipSuccess)
                    return fail(c, TOI_ENOMEM, "toi_image_batch: second per-snapshot set allocation failed");
            c->alt_ready = true;
        }
        hipStream_t user = c->stream;
        const uint32_t prof = c->prof_mask;
        c->prof_mask = 0;                         // no event records inside the graph
        hipStream_t A = c->cap_stream, B = c->cap_stream2;
        hipEvent_t* ev = c->batch_ev;             // [0] fork / join, [1] set ready, [2 + k] set k free
        c->stream = A;
        hipError_t e = hipStreamBeginCapture(A, hipStreamCaptureModeRelaxed);
        if (two && e == hipSuccess) e = hipEventRecord(ev[0], A);
        if (two && e == hipSuccess) e = hipStreamWaitEvent(B, ev[0], 0);
        const size_t NN = (size_t)c->N * c->N, TT = (size_t)c->T * c->T;
        bool swapped = false;
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            if (two && ((i & 1) != 0) != swapped) {   // odd snapshots use the second set
                front_swap(c);
                swapped = !swapped;
            }
            if (two) {
                c->stream = B;
                if (i >= 2) e = hipStreamWaitEvent(B, ev[2 + (i & 1)], 0);
                if (e == hipSuccess) e = launch_prep(c, snaps[i]);
                if (e == hipSuccess) e = launch_bin(c, snaps[i]);
                if (e == hipSuccess) e = hipEventRecord(ev[1], B);
                c->stream = A;
                if (e == hipSuccess) e = hipStreamWaitEvent(A, ev[1], 0);
            } else {
                e = launch_prep(c, snaps[i]);
                if (e == hipSuccess) e = launch_bin(c, snaps[i]);
            }
            if (e == hipSuccess) e = launch_gridder(c, snaps[i]);
            if (e == hipSuccess) e = launch_image(c, images_out + i * NN, nullptr);
            if (two && e == hipSuccess) e = hipEventRecord(ev[2 + (i & 1)], A);
            if (e == hipSuccess && tlisi_out && i >= 2)
                e = launch_tlisi(c, images_out + (i - 2) * NN, images_out + (i - 1) * NN, images_out + i * NN,
                                 tlisi_out + (i - 2) * TT);
        }
        if (swapped) front_swap(c);
        if (two && e == hipSuccess) e = hipEventRecord(ev[0], B);   // join lane B
        if (two && e == hipSuccess) e = hipStreamWaitEvent(A, ev[0], 0);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
        c->stream = user;
        c->prof_mask = prof;
        if (e == hipSuccess) e = e2;
        if (e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_check(c, e, "toi_image_batch: capture");
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_check(c, e, "toi_image_batch: instantiate");
        }
        if (c->batch_exec) (void)hipGraphExecDestroy(c->batch_exec);
        if (c->batch_graph) (void)hipGraphDestroy(c->batch_graph);
        c->batch_graph = graph;
        c->batch_exec = exec;
        c->batch_key = key;
        c->batch_n = n;
        ++c->batch_captures;
    }
    StageTimer timer(c, TOI_STAGE_BATCH);
    const toi_status st = hip_check(c, hipGraphLaunch(c->batch_exec, c->stream), "toi_image_batch: launch");
    if (st == TOI_OK) ++c->batch_launches;
    return st;
}
