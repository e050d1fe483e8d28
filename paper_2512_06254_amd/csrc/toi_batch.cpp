// Batched execution: many snapshots (uneven flagged-sample counts allowed) in
// one HIP graph launch.  The per-snapshot kernel chain (sample statistics,
// basis and plan, binning, gridding, FFT passes, re-projection, and the tLISI
// map of the three youngest images) is captured once for a given set of
// snapshot descriptors and outputs, instantiated, cached in the context and
// replayed on the caller's stream; a different descriptor set recaptures.
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
        if (!c->cap_stream) {
            hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_check(c, e, "toi_image_batch: capture stream");
        }
        hipStream_t user = c->stream;
        const uint32_t prof = c->prof_mask;
        c->prof_mask = 0;                         // no event records inside the graph
        c->stream = c->cap_stream;
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
        const size_t NN = (size_t)c->N * c->N, TT = (size_t)c->T * c->T;
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            e = launch_prep(c, snaps[i]);
            if (e == hipSuccess) e = launch_grid(c, snaps[i]);
            if (e == hipSuccess) e = launch_image(c, images_out + i * NN, nullptr);
            if (e == hipSuccess && tlisi_out && i >= 2)
                e = launch_tlisi(c, images_out + (i - 2) * NN, images_out + (i - 1) * NN, images_out + i * NN,
                                 tlisi_out + (i - 2) * TT);
        }
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
