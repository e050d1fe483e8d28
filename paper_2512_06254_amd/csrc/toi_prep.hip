// Sample statistics, snapshot basis and Chebyshev/slab plan (Sections 3.1, 3.4, 3.5).
//
// Nothing per sample is materialised: the basis needs only count, sum b and
// sum b b^T over the kept samples, and because b = uvw * nu / c these factor
// per row into sum(nu/c) and sum((nu/c)^2) over the row's kept channels.
#include "toi_internal.h"
#include "toi_device.h"

namespace toi {

// ---------------------------------------------------------------- S1: per-row sums
// One workgroup per row.  Without weights and flags every row keeps every
// channel with the same weight, so every row has the same sums: then one
// workgroup (n_same > 1) computes them once and writes them to the n_same
// rows (the 2016 workgroups of a MeerKAT-shaped snapshot took 19 us).
__global__ __launch_bounds__(256) void k_row_stats(const float* __restrict__ weight,
                                                   const uint8_t* __restrict__ flag,
                                                   const double* __restrict__ freq, int n_chan,
                                                   int n_corr, uint32_t mask, int n_same,
                                                   RowStat* __restrict__ rows) {
    const int r = blockIdx.x;
    double cnt = 0, s1 = 0, s2 = 0, ws = 0;
    double mn = 1e300, mx = -1e300;
    // kB channels per thread per round: their loads are issued before any of
    // them is used (one channel at a time left the row latency-bound)
    constexpr int kB = 4;
    for (int c0 = threadIdx.x; c0 < n_chan; c0 += kB * blockDim.x) {
        double w[kB], nu[kB];
#pragma unroll
        for (int i = 0; i < kB; ++i) {
            const int c = c0 + i * blockDim.x;
            w[i] = 0.0;
            nu[i] = 0.0;
            if (c < n_chan) {
                const size_t base = ((size_t)r * n_chan + c) * n_corr;
                nu[i] = freq[c];
                for (int k = 0; k < n_corr; ++k) {
                    if (!((mask >> k) & 1u)) continue;
                    double wk = weight ? (double)weight[base + k] : 1.0;
                    if (flag && flag[base + k]) wk = 0.0;
                    w[i] += wk;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kB; ++i)
            if (w[i] > 0.0) {
                const double kk = div_by(nu[i], kCLight, kInvCLight);
                cnt += 1.0;
                s1 += kk;
                s2 += kk * kk;
                ws += w[i];
                mn = fmin(mn, nu[i]);
                mx = fmax(mx, nu[i]);
            }
    }
    __shared__ double red[4][16], redm[2][16];
    double sums[4] = {cnt, s1, s2, ws};
    block_sum_n(sums, red);
    mn = block_min(mn, redm[0]);
    mx = block_max(mx, redm[1]);
    RowStat o;
    o.cnt = sums[0]; o.s1 = sums[1]; o.s2 = sums[2]; o.wsum = sums[3]; o.numin = mn; o.numax = mx;
    o.pad_[0] = o.pad_[1] = 0;
    if (n_same > 1) {
        for (int i = threadIdx.x; i < n_same; i += blockDim.x) rows[i] = o;
    } else if (threadIdx.x == 0) {
        rows[r] = o;
    }
}

// ---------------------------------------------------------------- S2: basis
// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix (FP64).
__device__ void jacobi3(double a[3][3], double v[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        const double diag = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]);
        if (off <= 1e-300 || off <= 1e-18 * diag) break;
        for (int p = 0; p < 2; ++p) {
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {          // A <- J^T A J
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = cs * akp - sn * akq;
                    a[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = cs * apk - sn * aqk;
                    a[q][k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 3; ++k) {          // V <- V J (columns = eigenvectors)
                    const double vkp = v[k][p], vkq = v[k][q];
                    v[k][p] = cs * vkp - sn * vkq;
                    v[k][q] = sn * vkp + cs * vkq;
                }
            }
        }
    }
}

__device__ inline void positive_major(double e[3]) {
    int m = 0;
    if (fabs(e[1]) > fabs(e[m])) m = 1;
    if (fabs(e[2]) > fabs(e[m])) m = 2;
    if (e[m] < 0) { e[0] = -e[0]; e[1] = -e[1]; e[2] = -e[2]; }
}

__global__ __launch_bounds__(256) void k_basis(const double* __restrict__ uvw, const RowStat* __restrict__ rows,
                                               int n_row, int mode, int gp, int max_sg, int unit_shift,
                                               DevPlan* __restrict__ plan) {
    __shared__ double red[16][4], red11[11][16];
    __shared__ double V_s[9];
    __shared__ uint32_t status_s;
    double acc[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int r = threadIdx.x; r < n_row; r += blockDim.x) {
        const RowStat s = rows[r];
        if (s.cnt == 0) continue;
        const double u[3] = {uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2]};
        acc[0] += s.cnt;
        acc[1] += s.wsum;
        acc[2] += u[0] * s.s1; acc[3] += u[1] * s.s1; acc[4] += u[2] * s.s1;
        acc[5] += u[0] * u[0] * s.s2; acc[6] += u[0] * u[1] * s.s2; acc[7] += u[0] * u[2] * s.s2;
        acc[8] += u[1] * u[1] * s.s2; acc[9] += u[1] * u[2] * s.s2; acc[10] += u[2] * u[2] * s.s2;
    }
    block_sum_n(acc, red11);
    if (threadIdx.x == 0) {
        DevPlan P{};
        P.nvis = acc[0];
        P.wsum = acc[1];
        for (int i = 0; i < 3; ++i) P.sum_b[i] = acc[2 + i];
        for (int i = 0; i < 6; ++i) P.sum_bb[i] = acc[5 + i];
        uint32_t st = 0;
        if (!(acc[0] > 0) || !(acc[1] > 0)) {
            st |= TOI_STATUS_NO_SAMPLES;
            P.V[0] = P.V[4] = P.V[8] = 1.0;
        } else {
            const double n = acc[0];
            const double m[3] = {acc[2] / n, acc[3] / n, acc[4] / n};
            // centred scatter matrix C = sum b b^T - n mean mean^T
            double C[3][3];
            C[0][0] = acc[5] - n * m[0] * m[0];
            C[0][1] = C[1][0] = acc[6] - n * m[0] * m[1];
            C[0][2] = C[2][0] = acc[7] - n * m[0] * m[2];
            C[1][1] = acc[8] - n * m[1] * m[1];
            C[1][2] = C[2][1] = acc[9] - n * m[1] * m[2];
            C[2][2] = acc[10] - n * m[2] * m[2];
            double ev[3][3];
            jacobi3(C, ev);
            int o[3] = {0, 1, 2};   // order eigenvalues descending
            for (int i = 0; i < 3; ++i)
                for (int j = i + 1; j < 3; ++j)
                    if (C[o[j]][o[j]] > C[o[i]][o[i]]) { int t = o[i]; o[i] = o[j]; o[j] = t; }
            double e1[3] = {ev[0][o[0]], ev[1][o[0]], ev[2][o[0]]};
            double e2[3] = {ev[0][o[1]], ev[1][o[1]], ev[2][o[1]]};
            positive_major(e1);
            positive_major(e2);
            double e3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                            e1[0] * e2[1] - e1[1] * e2[0]};
            if (e3[2] < 0) {
                for (int i = 0; i < 3; ++i) { e2[i] = -e2[i]; e3[i] = -e3[i]; }
            }
            for (int i = 0; i < 3; ++i) { P.V[i] = e1[i]; P.V[3 + i] = e2[i]; P.V[6 + i] = e3[i]; }
            P.omega = fabs(P.V[0] * P.V[4] - P.V[3] * P.V[1]);
            if (fabs(P.V[8]) < 1e-6) {
                st |= TOI_STATUS_DEGENERATE;
            } else {
                P.xi = P.V[6] / P.V[8];
                P.eta = P.V[7] / P.V[8];
            }
            if (P.omega > 0) P.norm = 1.0 / (P.omega * P.wsum);
        }
        P.n_slab = 1;
        P.K = 1;
        P.planes = 1;
        P.ng = 1;
        P.sg = min(gp, max_sg);
        P.kp = 1;
        P.parts = 1;
        P.gp = gp;
        P.max_sg = max_sg;
        P.unit_shift = unit_shift;
        P.status = st;
        *plan = P;
        for (int i = 0; i < 9; ++i) V_s[i] = P.V[i];
        status_s = st;
    }
    __syncthreads();
    if (status_s & TOI_STATUS_NO_SAMPLES) return;
    // r3 range over kept samples: r3 = (e3 . uvw) nu / c is monotonic in nu per row
    double lo = 1e300, hi = -1e300;
    for (int r = threadIdx.x; r < n_row; r += blockDim.x) {
        const RowStat s = rows[r];
        if (s.cnt == 0) continue;
        const double a = div_by(V_s[6] * uvw[3 * r] + V_s[7] * uvw[3 * r + 1] + V_s[8] * uvw[3 * r + 2], kCLight, kInvCLight);
        const double x0 = a * s.numin, x1 = a * s.numax;
        lo = fmin(lo, fmin(x0, x1));
        hi = fmax(hi, fmax(x0, x1));
    }
    lo = block_min(lo, red[12]);
    hi = block_max(hi, red[13]);
    if (threadIdx.x == 0) {
        plan->r3min = lo;
        plan->r3max = hi;
        plan->t3max = 0.0;
    }
}

// ---------------------------------------------------------------- S3: t3max over the t-plane
// |t3| = |sg sqrt(1 - rho^2) - V33| with rho^2 = (t1 + V13)^2 + (t2 + V23)^2
// (eq. t3) depends on the pixel only through rho, falls to 0 at the phase
// centre's rho0 = sqrt(V13^2 + V23^2) and grows with |rho - rho0| on either
// side; rho^2 is a convex quadratic in (t1, t2), separable in j1 and j2.  Over
// the pixel grid its maximum therefore sits at a corner and its minimum at
// one of the four pixels around the point t = (-V13, -V23) (clamped to the
// grid), so when all four corners are valid (then every pixel is), the
// maximum of |t3| over all pixel centres is the maximum over those eight
// pixels (the same expression as the scan, equal to it up to rounding).
// Otherwise every pixel is scanned.
__device__ inline double t3_abs(int j1, int j2, int N, double cell_rad, double V13, double V23, double V33,
                                double sg, bool& valid) {
    const double t1 = -cell_rad * (j1 - N / 2), t2 = cell_rad * (j2 - N / 2);
    const double a = 1.0 - (t1 + V13) * (t1 + V13) - (t2 + V23) * (t2 + V23);
    valid = a >= 0;
    return valid ? fabs(-V33 + sg * sqrt(a)) : 0.0;
}

__global__ __launch_bounds__(256) void k_t3max(int N, double cell_rad, DevPlan* __restrict__ plan) {
    __shared__ double red[4];
    if (plan->status & TOI_STATUS_NO_SAMPLES) return;
    const double V13 = plan->V[2], V23 = plan->V[5], V33 = plan->V[8];
    const double sg = V33 >= 0 ? 1.0 : -1.0;
    {
        bool ok = true, v;
        double m = 0.0;
        const int cj[2] = {0, N - 1};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                m = fmax(m, t3_abs(cj[a], cj[b], N, cell_rad, V13, V23, V33, sg, v));
                ok = ok && v;
            }
        if (ok) {   // corners valid: the corners and the pixels around the stationary point
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                const double c1 = N / 2 + V13 / cell_rad, c2 = N / 2 - V23 / cell_rad;   // t1 = -V13, t2 = -V23
                const int f1 = (int)fmin(fmax(floor(c1), 0.0), N - 1.0), f2 = (int)fmin(fmax(floor(c2), 0.0), N - 1.0);
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        m = fmax(m, t3_abs(min(f1 + a, N - 1), min(f2 + b, N - 1), N, cell_rad, V13, V23, V33, sg, v));
                plan->t3max = m;
            }
            return;
        }
    }
    double m = 0.0;
    const long total = (long)N * N;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int j1 = (int)(i % N), j2 = (int)(i / N);
        const double t1 = -cell_rad * (j1 - N / 2), t2 = cell_rad * (j2 - N / 2);
        const double a = 1.0 - (t1 + V13) * (t1 + V13) - (t2 + V23) * (t2 + V23);
        if (a >= 0) m = fmax(m, fabs(-V33 + sg * sqrt(a)));
    }
    m = block_max(m, red);
    if (threadIdx.x == 0)   // non-negative doubles order like their bit patterns
        atomicMax((unsigned long long*)&plan->t3max, (unsigned long long)__double_as_longlong(m));
}

// Bessel J_0..J_{K-1}(x) by Miller's backward recurrence with the
// normalisation J_0 + 2 sum J_{2m} = 1 (DLMF 10.74(iii)), FP64.
__device__ void bessel_j_fp64(double x, int K, double* J) {
    if (fabs(x) < 1e-12) {
        J[0] = 1.0;
        for (int k = 1; k < K; ++k) J[k] = (k == 1) ? 0.5 * x : 0.0;
        return;
    }
    const int L = 2 * ((K + (int)fabs(x) + 40) / 2);
    double jp1 = 0.0, j = 1e-250, norm = 0.0;
    for (int k = 0; k < K; ++k) J[k] = 0.0;
    for (int n = L; n >= 0; --n) {
        if (n < K) J[n] = j;
        if ((n & 1) == 0) norm += (n == 0) ? j : 2.0 * j;
        if (n > 0) {
            const double jm1 = (2.0 * n / x) * j - jp1;
            jp1 = j;
            j = jm1;
        }
        if (fabs(j) > 1e250) {
            j *= 1e-250; jp1 *= 1e-250; norm *= 1e-250;
            for (int k = n; k < K; ++k) J[k] *= 1e-250;
        }
    }
    for (int k = 0; k < K; ++k) J[k] /= norm;
}

// max over alpha in [0, alpha_slab], s in [-1, 1] (129 x 129) of |e^{i alpha s} - sum_k c_k T_k(s)|
__device__ double cheb_sampled_error(double alpha_slab, int K, double* red) {
    constexpr int G = 129;
    double worst = 0.0;
    for (int ia = threadIdx.x; ia < G; ia += blockDim.x) {
        const double a = alpha_slab * ia / (G - 1);
        double J[32];
        bessel_j_fp64(a, K, J);
        for (int is = 0; is < G; ++is) {
            const double s = -1.0 + 2.0 * is / (G - 1);
            double tm1 = 1.0, t = s, re = J[0], im = 0.0;
            for (int k = 1; k < K; ++k) {
                const double c = 2.0 * J[k] * t;     // 2 i^k J_k T_k
                switch (k & 3) {
                    case 0: re += c; break;
                    case 1: im += c; break;
                    case 2: re -= c; break;
                    default: im -= c; break;
                }
                const double tn = 2.0 * s * t - tm1;
                tm1 = t;
                t = tn;
            }
            const double er = cos(a * s) - re, ei = sin(a * s) - im;
            worst = fmax(worst, sqrt(er * er + ei * ei));
        }
    }
    return block_max(worst, red);
}

__global__ __launch_bounds__(256) void k_plan(double alpha_target, double gamma, int forced_slab,
                                              int forced_k, int p_cap, int ng_cap, DevPlan* __restrict__ plan) {
    __shared__ double red[4];
    __shared__ double a_slab;
    if (plan->status & TOI_STATUS_NO_SAMPLES) return;
    if (threadIdx.x == 0) {
        const double t3max = plan->t3max, r3min = plan->r3min, r3max = plan->r3max;
        const double phimax = 2.0 * kPi * t3max * (r3max - r3min) / 2.0;
        int ns = forced_slab > 0 ? forced_slab : (int)fmax(1.0, ceil(phimax / alpha_target));
        double dr3 = (r3max - r3min) / (2.0 * ns);
        if (!(dr3 > 0.0)) { ns = 1; dr3 = 0.0; }
        plan->phimax = phimax;
        plan->n_slab = ns;
        plan->dr3 = dr3;
        plan->inv_dr3 = dr3 > 0.0 ? 1.0 / dr3 : 0.0;
        plan->alpha_slab = 2.0 * kPi * t3max * dr3;
        a_slab = plan->alpha_slab;
    }
    __syncthreads();
    int K = forced_k;
    if (K <= 0) {
        const int choices[4] = {8, 16, 24, 32};
        K = 32;
        for (int i = 0; i < 4; ++i) {
            const double err = cheb_sampled_error(a_slab, choices[i], red);
            if (err < gamma) { K = choices[i]; break; }
        }
    }
    if (threadIdx.x == 0) {
        plan->K = K;
        plan->planes = plan->n_slab * K;
        plan->miller_top = 2 * ((K + 16 + (int)ceil(1.5 * fabs(a_slab))) / 2);
        const int gp = plan->gp;
        if (K <= gp) {
            plan->sg = min(gp / K, plan->max_sg);
            plan->kp = K;
            plan->parts = 1;
            plan->ng = (plan->n_slab + plan->sg - 1) / plan->sg;
        } else {
            plan->sg = 1;
            plan->parts = (K + gp - 1) / gp;
            plan->kp = (K + plan->parts - 1) / plan->parts;
            plan->ng = plan->parts * plan->n_slab;
        }
        if (plan->planes > p_cap || plan->ng > ng_cap) plan->status |= TOI_STATUS_PLANES;
    }
}

hipError_t launch_prep(toi_ctx* c, const toi_snapshot& s) {
    StageTimer timer(c, TOI_STAGE_PREP);
    const toi_params& p = c->p;
    if (s.n_row > 0)
    {
        const bool same = !s.weight && !s.flag;   // every row keeps every channel
        hipLaunchKernelGGL(k_row_stats, dim3(same ? 1 : s.n_row), dim3(256), 0, c->stream, s.weight, s.flag, s.freq,
                           p.n_chan, p.n_corr, p.corr_mask, same ? s.n_row : 1, c->rows);
    }
    const GridShape gs = grid_shape(c->tuning);
    hipLaunchKernelGGL(k_basis, dim3(1), dim3(256), 0, c->stream, s.uvw, c->rows, s.n_row, p.mode, gs.gp, gs.max_sg,
                       gs.unit_shift,
                       c->plan);
    if (p.mode == 3) {
        const double cell = p.cell_deg * kPi / 180.0;
        const long total = (long)c->N * c->N;
        const int blocks = (int)std::min<long>(1024, (total + 255) / 256);
        hipLaunchKernelGGL(k_t3max, dim3(blocks), dim3(256), 0, c->stream, c->N, cell, c->plan);
        hipLaunchKernelGGL(k_plan, dim3(1), dim3(256), 0, c->stream, p.alpha_target, p.cheb_gamma, p.n_slab,
                           p.cheb_k, c->P_cap, c->NG_max, c->plan);
    }
    return hipGetLastError();
}

}  // namespace toi
