// Streaming ingest: snapshots whose arrays live in host memory are copied to
// the device on an internal copy stream while the previous snapshot is being
// imaged on the context's stream.  Two device staging slots alternate: the
// copy of snapshot i + 1 runs during the imaging of snapshot i, and a slot is
// refilled once the gridding that read it has finished.  With page-locked
// host arrays the copies are DMA transfers that overlap the kernels; the
// images and tLISI maps are the same as from toi_grid + toi_image + fitrig_tlisi.
#include <hip/hip_runtime.h>

#include <cstring>

#include "toi_internal.h"

using namespace toi;

namespace {

struct Slot {
    double* uvw = nullptr;
    float2* vis = nullptr;
    uint8_t* flag = nullptr;
    float* weight = nullptr;
    double* freq = nullptr;
    int32_t* ant1 = nullptr;
    int32_t* ant2 = nullptr;
    float2* gains = nullptr;
    hipEvent_t copied = nullptr;   // the slot's arrays are on the device
    hipEvent_t free_ = nullptr;    // the gridding that read them has finished
    bool used = false;
};

}  // namespace

struct toi_ingest_state {
    Slot slot[2];
    hipStream_t copy = nullptr;
};

namespace toi {

void ingest_release(toi_ctx* c) {
    toi_ingest_state* st = c->ingest;
    if (!st) return;
    if (st->copy) (void)hipStreamSynchronize(st->copy);
    for (Slot& s : st->slot) {
        void* ptrs[] = {s.uvw, s.vis, s.flag, s.weight, s.freq, s.ant1, s.ant2, s.gains};
        for (void* q : ptrs)
            if (q) (void)hipFree(q);
        if (s.copied) (void)hipEventDestroy(s.copied);
        if (s.free_) (void)hipEventDestroy(s.free_);
    }
    if (st->copy) (void)hipStreamDestroy(st->copy);
    delete st;
    c->ingest = nullptr;
}

}  // namespace toi

static toi_status ingest_setup(toi_ctx* c) {
    if (c->ingest) return TOI_OK;
    const toi_params& p = c->p;
    const size_t rows = std::max(1, p.n_row_max), samples = rows * p.n_chan * p.n_corr;
    toi_ingest_state* st = new toi_ingest_state();
    c->ingest = st;
    hipError_t e = hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking);   // default priority
    for (Slot& s : st->slot) {
        if (e == hipSuccess) e = hipMalloc(&s.uvw, rows * 3 * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&s.vis, samples * sizeof(float2));
        if (e == hipSuccess) e = hipMalloc(&s.flag, samples);
        if (e == hipSuccess) e = hipMalloc(&s.weight, samples * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&s.freq, (size_t)p.n_chan * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&s.ant1, rows * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&s.ant2, rows * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&s.gains, std::max(1, p.n_ant) * sizeof(float2));
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.copied, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.free_, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        ingest_release(c);
        return hip_check(c, e, "toi_ingest: staging");
    }
    return TOI_OK;
}

extern "C" toi_status toi_ingest(toi_ctx* c, const toi_snapshot* host_snaps, int32_t n, float* images_out,
                                 float* tlisi_out) {
    if (!c) return fail(nullptr, TOI_EINVAL, "toi_ingest: ctx is NULL");
    if (n < 0) return fail(c, TOI_EINVAL, "toi_ingest: n < 0");
    if (n == 0) return TOI_OK;
    if (!host_snaps || !images_out) return fail(c, TOI_EINVAL, "toi_ingest: host_snaps and images_out are required");
    const toi_params& p = c->p;
    for (int i = 0; i < n; ++i) {
        const toi_snapshot& s = host_snaps[i];
        if (s.n_row < 0 || s.n_row > p.n_row_max)
            return fail(c, TOI_EINVAL, "toi_ingest: a snapshot's n_row is outside [0, n_row_max]");
        if (s.n_row > 0 && (!s.uvw || !s.vis || !s.freq))
            return fail(c, TOI_EINVAL, "toi_ingest: uvw, vis and freq are required");
        if (s.gains && (!s.ant1 || !s.ant2 || p.n_ant <= 0))
            return fail(c, TOI_EINVAL, "toi_ingest: gains need ant1, ant2 and n_ant > 0");
    }
    toi_status st = ingest_setup(c);
    if (st != TOI_OK) return st;
    toi_ingest_state* ig = c->ingest;
    const size_t NN = (size_t)c->N * c->N, TT = (size_t)c->T * c->T;
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        const toi_snapshot& h = host_snaps[i];
        Slot& sl = ig->slot[i & 1];
        const size_t rows = h.n_row, samples = rows * p.n_chan * p.n_corr;
        // copy stream: wait until the slot's previous gridding is done, then fill it
        if (sl.used) e = hipStreamWaitEvent(ig->copy, sl.free_, 0);
        auto put = [&](void* dst, const void* src, size_t bytes) {
            if (e == hipSuccess && src && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ig->copy);
        };
        put(sl.uvw, h.uvw, rows * 3 * sizeof(double));
        put(sl.vis, h.vis, samples * sizeof(float2));
        put(sl.flag, h.flag, samples);
        put(sl.weight, h.weight, samples * sizeof(float));
        put(sl.freq, h.freq, (size_t)p.n_chan * sizeof(double));
        put(sl.ant1, h.ant1, rows * sizeof(int32_t));
        put(sl.ant2, h.ant2, rows * sizeof(int32_t));
        put(sl.gains, h.gains, (size_t)p.n_ant * sizeof(float2));
        if (e == hipSuccess) e = hipEventRecord(sl.copied, ig->copy);
        // context stream: image the slot's snapshot
        if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, sl.copied, 0);
        toi_snapshot d;
        std::memset(&d, 0, sizeof(d));
        d.n_row = h.n_row;
        d.uvw = h.uvw ? sl.uvw : nullptr;
        d.vis = h.vis ? sl.vis : nullptr;
        d.flag = h.flag ? sl.flag : nullptr;
        d.weight = h.weight ? sl.weight : nullptr;
        d.freq = h.freq ? sl.freq : nullptr;
        d.ant1 = h.ant1 ? sl.ant1 : nullptr;
        d.ant2 = h.ant2 ? sl.ant2 : nullptr;
        d.gains = h.gains ? sl.gains : nullptr;
        if (e == hipSuccess) e = launch_prep(c, d);
        if (e == hipSuccess) e = launch_grid(c, d);
        if (e == hipSuccess) e = hipEventRecord(sl.free_, c->stream);   // the inputs are no longer read
        sl.used = true;
        if (e == hipSuccess) e = launch_image(c, images_out + i * NN, nullptr);
        if (e == hipSuccess && tlisi_out && i >= 2)
            e = launch_tlisi(c, images_out + (i - 2) * NN, images_out + (i - 1) * NN, images_out + i * NN,
                             tlisi_out + (i - 2) * TT);
    }
    return hip_check(c, e, "toi_ingest");
}
