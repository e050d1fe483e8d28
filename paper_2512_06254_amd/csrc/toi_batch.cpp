// Batched execution: many snapshots (uneven flagged-sample counts allowed) in
// one HIP graph launch.  The per-snapshot kernel chain (sample statistics,
// basis and plan, binning, gridding, FFT passes, re-projection, and the tLISI
// map of the three youngest images) is captured once for a given set of
// snapshot descriptors and outputs, instantiated, cached in the context and
// replayed on the caller's stream; a different descriptor set recaptures.
// With two or more snapshots the chain runs in two lanes, as the pipeline of
// Section 4.1 overlaps its stages: the prep and binning of snapshot i + 1
// (lane B, writing the other of two per-snapshot sets) run while snapshot i is
// gridded and transformed (lane A).  Lane B waits until the transform of
// snapshot i - 1, the last reader of that set, has finished.
// No host synchronisation and no allocation happen inside the graph.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

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
            size_t fb[14];
            front_bytes(c, fb);
            toi_front& a = c->alt;
            void** ptrs[14] = {(void**)&a.plan, (void**)&a.rows, (void**)&a.items, (void**)&a.recs,
                               (void**)&a.bin_count, (void**)&a.bin_off, (void**)&a.bin_cursor,
                               (void**)&a.bin_list, (void**)&a.bin_order, (void**)&a.bin_aux, (void**)&a.units,
                               (void**)&a.tile_bits, (void**)&a.row_bits, (void**)&a.scratch_i};
            for (int k = 0; k < 14; ++k)
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
    }
    StageTimer timer(c, TOI_STAGE_BATCH);
    return hip_check(c, hipGraphLaunch(c->batch_exec, c->stream), "toi_image_batch: launch");
}
