// Device helpers shared by the gridder and the degridder: sample selection,
// per-row track coefficients, slab / plane-group mapping and the Chebyshev
// recurrence start.
#pragma once

#include "toi_device.h"
#include "toi_internal.h"

namespace toi {

// Every status bit is fatal: the gridder, the FFT passes and the
// re-projection then produce an all-zero image (an overflowing bin list would
// leave tiles unwritten).
constexpr uint32_t kStatusFatal =
    TOI_STATUS_NO_SAMPLES | TOI_STATUS_DEGENERATE | TOI_STATUS_PLANES | TOI_STATUS_OVERFLOW;

// Weighted sum of the selected correlations of one (row, channel) sample with
// flags as zero weight (Section 3.5).  Returns the sample weight w.  With
// vec4 (four correlations and arrays aligned for it: vis to 16 bytes, flags
// to 4, weights to 16; see vec4_ok) the sample is read as two 16-byte loads
// (and one word of flags, one 16-byte load of weights) instead of one load
// per correlation; the sums are formed in the same order.
__device__ inline float sample_value(const float2* __restrict__ vis, const float* __restrict__ weight,
                                     const uint8_t* __restrict__ flag, size_t base, int n_corr, uint32_t mask,
                                     float& xr, float& xi, bool vec4 = false) {
    if (vec4) {
        const float4* v4 = reinterpret_cast<const float4*>(vis + base);
        const float4 a = v4[0], b = v4[1];
        float wk[4] = {1.f, 1.f, 1.f, 1.f};
        if (weight) {
            const float4 q = *reinterpret_cast<const float4*>(weight + base);
            wk[0] = q.x; wk[1] = q.y; wk[2] = q.z; wk[3] = q.w;
        }
        if (flag) {
            const uint32_t f = *reinterpret_cast<const uint32_t*>(flag + base);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if ((f >> (8 * k)) & 0xffu) wk[k] = 0.f;
        }
        const float vr[4] = {a.x, a.z, b.x, b.z}, vi[4] = {a.y, a.w, b.y, b.w};
        float w = 0.f;
        xr = 0.f;
        xi = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!((mask >> k) & 1u)) continue;
            w += wk[k];
            xr += wk[k] * vr[k];
            xi += wk[k] * vi[k];
        }
        return w;
    }
    float w = 0.f;
    xr = 0.f;
    xi = 0.f;
    for (int k = 0; k < n_corr; ++k) {
        if (!((mask >> k) & 1u)) continue;
        float wk = weight ? weight[base + k] : 1.f;
        if (flag && flag[base + k]) wk = 0.f;
        const float2 v = vis[base + k];
        w += wk;
        xr += wk * v.x;
        xi += wk * v.y;
    }
    return w;
}

// Whether sample_value may read a snapshot's samples with 16-byte loads.
inline bool vec4_ok(const void* vis, const void* flag, const void* weight, int n_corr) {
    return n_corr == 4 && (reinterpret_cast<uintptr_t>(vis) & 15) == 0 &&
           (reinterpret_cast<uintptr_t>(flag) & 3) == 0 && (reinterpret_cast<uintptr_t>(weight) & 15) == 0;
}

__device__ inline bool sample_kept(const float* __restrict__ weight, const uint8_t* __restrict__ flag, size_t base,
                                   int n_corr, uint32_t mask) {
    float w = 0.f;
    for (int k = 0; k < n_corr; ++k) {
        if (!((mask >> k) & 1u)) continue;
        float wk = weight ? weight[base + k] : 1.f;
        if (flag && flag[base + k]) wk = 0.f;
        w += wk;
    }
    return w > 0.f;
}

// Per-row track: grid coordinates X = M/2 + ax nu, Y = M/2 + ay nu and the
// residual coordinate r3 = a3 nu (r = V b with b = uvw nu / c).
struct Track {
    double ax, ay, a3;
};
__device__ inline Track row_track(const double* __restrict__ uvw, int r, const DevPlan* __restrict__ P, int M,
                                  double cell_rad) {
    const double u0 = uvw[3 * r], u1 = uvw[3 * r + 1], u2 = uvw[3 * r + 2];
    const double* V = P->V;
    const double sc = div_by((double)M * cell_rad, kCLight, kInvCLight);
    Track t;
    t.ax = -(V[0] * u0 + V[1] * u1 + V[2] * u2) * sc;
    t.ay = (V[3] * u0 + V[4] * u1 + V[5] * u2) * sc;
    t.a3 = div_by(V[6] * u0 + V[7] * u1 + V[8] * u2, kCLight, kInvCLight);
    return t;
}

// g[ant1] conj(g[ant2]) of a row; an antenna index outside [0, n_ant) gives 0.
__device__ inline float2 row_gain(const float2* __restrict__ gains, const int32_t* __restrict__ ant1,
                                  const int32_t* __restrict__ ant2, int n_ant, int r) {
    if (!gains) return make_float2(1.f, 0.f);
    const int a1 = ant1[r], a2 = ant2[r];
    if (a1 < 0 || a1 >= n_ant || a2 < 0 || a2 >= n_ant) return make_float2(0.f, 0.f);
    const float2 g1 = gains[a1], g2 = gains[a2];
    return cmul(g1, make_float2(g2.x, -g2.y));
}

// Slab of a residual coordinate: p = min(N_slab - 1, floor((r3 - r3min) / (2 dr3))).
__device__ inline int slab_index(double r3, const DevPlan* __restrict__ P) {
    if (!(P->dr3 > 0.0)) return 0;
    int p = (int)floor(div_by(r3 - P->r3min, 2.0 * P->dr3, 0.5 * P->inv_dr3));
    return max(0, min(P->n_slab - 1, p));
}

// Plane groups (one LDS pass of the gridder each, at most gp planes): whole
// slabs (sg of them) when K <= gp, otherwise `parts` groups per slab holding
// orders [part kp, min(K, (part + 1) kp)).
__device__ inline int group_of_slab(int p, const DevPlan* __restrict__ P) {
    return P->K <= P->gp ? p / P->sg : p * P->parts;
}
__device__ inline int group_of_plane(int plane, const DevPlan* __restrict__ P) {
    const int p = plane / P->K, k = plane % P->K;
    return P->K <= P->gp ? p / P->sg : p * P->parts + k / P->kp;
}
__device__ inline void group_range(int g, const DevPlan* __restrict__ P, int& s0, int& s1, int& k0, int& k1) {
    if (P->K <= P->gp) {
        s0 = g * P->sg;
        s1 = min(P->n_slab, s0 + P->sg);
        k0 = 0;
        k1 = P->K;
    } else {
        s0 = g / P->parts;
        s1 = s0 + 1;
        k0 = (g % P->parts) * P->kp;
        k1 = min(P->K, k0 + P->kp);
    }
}

// Work unit ob of the matrix-core tile passes (toi_grid, toi_degrid).  The
// first cnt[1] units come from the bins listed unit by unit (the heaviest
// cnt[2] non-empty bins, 2^unit_shift items per unit); the rest are the other
// non-empty bins, whole, in their launch order.  Item range [b0, b1) of the
// bin's list; parts > 1 marks a split bin whose part 0 is unit slot0.
struct WorkUnit {
    int bin, part, parts, slot0;
};
__device__ inline int work_unit_count(const int32_t* __restrict__ cnt) { return cnt[0] - cnt[2] + cnt[1]; }
__device__ inline WorkUnit work_unit(int ob, const int4* __restrict__ units, const int32_t* __restrict__ order,
                                     const int32_t* __restrict__ cnt) {
    const int n_split = cnt[1];
    if (ob < n_split) {
        const int4 u = units[ob];
        return WorkUnit{u.x, u.y, u.z, u.w};
    }
    return WorkUnit{order[cnt[2] + ob - n_split], 0, 1, -1};
}
__device__ inline void work_unit_items(const WorkUnit& u, const int32_t* __restrict__ bin_off, int bin_cap,
                                       int unit_shift, int& b0, int& b1) {
    const int e = min(bin_off[u.bin + 1], bin_cap);
    b0 = bin_off[u.bin];
    if (u.parts > 1) {
        b0 += u.part << unit_shift;
        b1 = min(b0 + (1 << unit_shift), e);
    } else {
        b1 = e;
    }
}

// Tiles (bins of S = 2^bsh cells per side) of tile row ty that the footprints
// of an item's kept samples can touch: [tx0, tx1] (unwrapped; empty when
// tx1 < tx0).  A footprint starting at row ceil(Y - 4) overlaps the tile
// row's cells [S ty, S ty + S - 1] exactly when Y lies in
// (S ty - 4, S ty + S + 3]; along the track that is an interval
// of the parameter l in [0, 1] (X, Y = start + l (end - start)), over which
// the footprint start columns ceil(X - 4) give the tiles.  Both windows are
// widened by 1e-6 cells, so that a sample whose coordinates were rounded
// differently (or the interval's ends by the reciprocal of the extent) is
// never left out; a tile too many only costs a visit that finds no sample.  At most nt tiles (one full turn of the periodic grid).
__device__ inline void item_row_tiles(const ItemBox& b, int ty, int nt, int bsh, int& tx0, int& tx1) {
    constexpr double eps = 1e-6;
    const double dx = b.x1 - b.x0;
    const double S = (double)(1 << bsh);
    double l0 = 0.0, l1 = 1.0;
    if (b.inv_dy != 0.0) {
        const double la = (S * ty - 4.0 - eps - b.y0) * b.inv_dy, lb = (S * ty + S + 3.0 + eps - b.y0) * b.inv_dy;
        l0 = fmax(0.0, fmin(la, lb));
        l1 = fmin(1.0, fmax(la, lb));
    }
    if (!(l0 <= l1)) {
        tx0 = 1;
        tx1 = 0;
        return;
    }
    const double xa = b.x0 + l0 * dx, xb = b.x0 + l1 * dx;
    tx0 = ((int)ceil(fmin(xa, xb) - eps - 4.0)) >> bsh;
    tx1 = ((int)ceil(fmax(xa, xb) + eps - 4.0) + 7) >> bsh;
    tx1 = min(tx1, tx0 + nt - 1);
}

// Every (plane group, tile) bin of an item, spread over an aligned group of W
// lanes of the calling wavefront (W = 64: the whole wavefront): f(g, ty, tx)
// is called once per bin (wrapped tile indices).  Lane r of the group first
// takes tile row ty0 + r and its tiles; a prefix sum of the per-row counts
// over the group then deals the (row, tile, group) entries round-robin over
// its lanes.  Items with more than W tile rows take their rows in turn.  All
// lanes of the group must call it; other groups of the wavefront may serve
// other items (the group's shuffles stay inside the group).
template <int W = 64, typename F>
__device__ inline void for_item_bins(const ItemBox& b, int NT, int bsh, F f) {
    static_assert(W >= 2 && W <= 64 && (W & (W - 1)) == 0, "a power-of-two group of lanes");
    const int lane = threadIdx.x & (W - 1);
    const int ny = b.ty1 - b.ty0 + 1, ng = b.g1 - b.g0 + 1;
    if (ny <= 0 || ng <= 0) return;
    for (int r0 = 0; r0 < ny; r0 += W) {
        const int ty = b.ty0 + r0 + lane;
        int tx0 = 1, tx1 = 0;
        if (r0 + lane < ny) item_row_tiles(b, ty, NT, bsh, tx0, tx1);
        const int cnt = max(0, tx1 - tx0 + 1);
        int incl = cnt;   // inclusive prefix sum over the group's lanes
#pragma unroll
        for (int o = 1; o < W; o <<= 1) {
            const int u = __shfl_up(incl, o, W);
            if (lane >= o) incl += u;
        }
        const int total = __shfl(incl, W - 1, W);   // uniform over the group: every lane runs every round
        for (int e0 = 0; e0 < total * ng; e0 += W) {
            const int e = min(e0 + lane, total * ng - 1);
            const int ti = e % total, g = b.g0 + e / total;
            // the lane whose row holds tile entry ti: the first with incl > ti
            int lo = 0;
#pragma unroll
            for (int step = W / 2; step > 0; step >>= 1) {
                const int probe = __shfl(incl, lo + step - 1, W);
                if (probe <= ti) lo += step;
            }
            const int start = __shfl(incl - cnt, lo, W), rtx0 = __shfl(tx0, lo, W);
            if (e0 + lane < total * ng) f(g, (b.ty0 + r0 + lo) & (NT - 1), (rtx0 + ti - start) & (NT - 1));
        }
    }
}

// Chebyshev recurrence T_{k+1} = 2 s T_k - T_{k-1} started at order k0:
// returns t = T_{k0}(s) and tm1 = T_{k0-1}(s) (T_{-1} = T_1).
__device__ inline void cheb_start(float s, int k0, float& t, float& tm1) {
    if (k0 == 0) {
        t = 1.f;
        tm1 = s;
        return;
    }
    tm1 = 1.f;
    t = s;
    for (int k = 1; k < k0; ++k) {
        const float tn = 2.f * s * t - tm1;
        tm1 = t;
        t = tn;
    }
}

// Re-projection (Section 3.3): output pixel (j1, j2) -> reduced SIN map onto the
// tilted plane (x' = x + r0 z xi, y' = y + r0 z eta with z = 1 - n) -> in-plane
// 2x2 block of V -> fractional transformed-plane indices, in FP64.  Returns
// false when the pixel has no valid bilinear source (outside the unit circle
// or a neighbour outside the image); otherwise the lower-left source pixel
// (i1, i2) and the FP32 fractions (f1, f2).
__device__ inline bool reproject_source(const DevPlan* __restrict__ P, int N, double cell_rad, int j1, int j2,
                                        int& i1, int& i2, float& f1, float& f2) {
    const double l = -cell_rad * (j1 - N / 2), m = cell_rad * (j2 - N / 2);
    const double rho2 = l * l + m * m;
    if (!(rho2 < 1.0)) return false;
    const double z = rho2 / (1.0 + sqrt(1.0 - rho2));           // 1 - n, stable near the centre
    const double a = l + P->xi * z, b = m + P->eta * z;
    const double t1 = P->V[0] * a + P->V[1] * b;
    const double t2 = P->V[3] * a + P->V[4] * b;
    const double icr = 1.0 / cell_rad;                            // uniform: one division per thread
    const double u1 = 0.5 * N - div_by(t1, cell_rad, icr), u2 = 0.5 * N + div_by(t2, cell_rad, icr);
    const double f1d = floor(u1), f2d = floor(u2);
    if (!(f1d >= 0.0 && f1d <= N - 2 && f2d >= 0.0 && f2d <= N - 2)) return false;
    i1 = (int)f1d;
    i2 = (int)f2d;
    f1 = (float)(u1 - f1d);
    f2 = (float)(u2 - f2d);
    return true;
}

}  // namespace toi
