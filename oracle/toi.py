"""FP64 CPU oracle of TOI per-snapshot imaging.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path (the HIP library and its binding) never
does.  Everything here is plain numpy in float64 and follows the paper's
definitions in the paper's order, with no blocking or fusion beyond the
definitions themselves.  Library primitives used as steps: ``numpy.linalg.svd``
(the SVD of §3.1), matrix products (sums over samples), ``scipy.special.jv``
(Bessel functions of App. B2), ``numpy.fft`` (the gridded variant only).

Pixel convention (§3.3 and App. A): pixel ``(p1, p2)`` is 1-based with
``j = p - 1``; images are stored ``img[j2][j1]`` (``j1`` fastest);
``l = -Delta (j1 - N/2)``, ``m = Delta (j2 - N/2)`` with ``Delta`` the cell in
radians.  The transformed plane uses the same map for ``(t1, t2)``.

Readings where the paper is silent (each also listed in the design doc):
  * samples: per (row, channel) the selected parallel hands k give
    ``w = sum_k W_k (1 - F_k)`` and ``x = g_a1 conj(g_a2) sum_k W_k (1 - F_k) V_k``;
    samples with ``w = 0`` are dropped everywhere; the normaliser ``N_vis`` of
    the dirty-image equations becomes ``W = sum_q w_q`` (identical for unit
    weights), so ``(1/(omega W)) sum_q x_q ... = (1/(omega N_vis)) sum_q Vis_q ...``;
  * basis signs: the dominant direction ``e1`` is flipped so that its
    largest-magnitude component is positive; ``e2`` likewise, then the third is
    ``e3 = e1 x e2`` and ``e2, e3`` are negated together when ``e3`` has a
    negative w component (so ``V33 >= 0`` and the handedness rule has the
    last word on the sign of ``e2``);
  * the dirty image is the real part of the complex sum;
  * slab assignment ``p = min(N_slab - 1, floor((r3 - r3min) / (2 Delta r3)))``;
  * the K test samples a 129 x 129 grid of ``alpha in [0, alpha_slab]``,
    ``s in [-1, 1]``;
  * ``t3max`` is the maximum of ``|t3|`` over all transformed-plane pixel
    centres where the square root is real.

Parity pins for every function are in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy import special

C_LIGHT = 299_792_458.0
CHEB_K_CHOICES = (8, 16, 24, 32)


# ----------------------------------------------------------------------------
# §3.5: sample selection, weighting, polarisation averaging, MFS

def default_corr_mask(n_corr: int) -> int:
    """Parallel hands: XX and YY of four correlations, the first of one or two."""
    return {1: 0b1, 2: 0b11, 4: 0b1001}[n_corr]


@dataclasses.dataclass
class Samples:
    b: np.ndarray       # (Nq, 3) baseline coordinates in wavelengths
    x: np.ndarray       # (Nq,) complex weighted visibility sum  sum_k W_k (1-F_k) V_k (times gains)
    w: np.ndarray       # (Nq,) total weight of the sample
    row: np.ndarray     # (Nq,) row index
    chan: np.ndarray    # (Nq,) channel index
    W: float            # sum of weights: the normaliser

    @property
    def n(self):
        return self.x.shape[0]


def row_gains(snap) -> Optional[np.ndarray]:
    g = snap.get("gains")
    if g is None:
        return None
    g = np.asarray(g, dtype=np.complex128)
    return g[snap["ant1"]] * np.conj(g[snap["ant2"]])


def sample_weights(snap, corr_mask: Optional[int] = None):
    """Per correlation effective weight ``W_k (1 - F_k)`` on the selected hands."""
    vis = snap["vis"]
    n_corr = vis.shape[2]
    mask = default_corr_mask(n_corr) if corr_mask is None else corr_mask
    sel = [k for k in range(n_corr) if (mask >> k) & 1]
    wk = np.ones(vis.shape, dtype=np.float64)
    if snap.get("weight") is not None:
        wk = np.asarray(snap["weight"], dtype=np.float64).copy()
    if snap.get("flag") is not None:
        wk = wk * (1.0 - np.asarray(snap["flag"], dtype=np.float64))
    keep = np.zeros(n_corr, dtype=bool)
    keep[sel] = True
    wk[:, :, ~keep] = 0.0
    return wk


def select_samples(snap, corr_mask: Optional[int] = None) -> Samples:
    """Every (row, channel) pair is one sample (MFS); uvw is scaled per channel."""
    vis = np.asarray(snap["vis"]).astype(np.complex128)
    wk = sample_weights(snap, corr_mask)
    w = wk.sum(axis=2)                                  # (rows, chans)
    x = (wk * vis).sum(axis=2)
    g = row_gains(snap)
    if g is not None:
        x = x * g[:, None]
    uvw = np.asarray(snap["uvw"], dtype=np.float64)
    freq = np.asarray(snap["freq"], dtype=np.float64)
    b = uvw[:, None, :] * (freq[None, :, None] / C_LIGHT)  # metres -> wavelengths
    keep = w > 0
    rows, chans = np.nonzero(keep)
    return Samples(b=b[keep], x=x[keep], w=w[keep], row=rows, chan=chans, W=float(w.sum()))


# ----------------------------------------------------------------------------
# §3.1: the snapshot basis

@dataclasses.dataclass
class Basis:
    V: np.ndarray        # rows are the basis vectors
    omega: float         # |V11 V22 - V21 V12|  (eq. 11)
    xi: float            # V31 / V33            (§3.3)
    eta: float           # V32 / V33


def _positive_major(e):
    return e if e[np.argmax(np.abs(e))] > 0 else -e


def snapshot_basis(b: np.ndarray) -> Basis:
    """SVD of the centred baseline matrix; rows of V = two dominant directions + their cross product."""
    bc = b - b.mean(axis=0)
    _, _, vt = np.linalg.svd(bc, full_matrices=False)   # rows of vt: right singular vectors, descending
    e1 = _positive_major(vt[0])
    e2 = _positive_major(vt[1])
    e3 = np.cross(e1, e2)
    if e3[2] < 0:
        e2, e3 = -e2, -e3
    V = np.stack([e1, e2, e3])
    return basis_from_V(V)


def basis_from_V(V: np.ndarray) -> Basis:
    V = np.asarray(V, dtype=np.float64)
    omega = abs(V[0, 0] * V[1, 1] - V[1, 0] * V[0, 1])
    return Basis(V=V, omega=omega, xi=V[2, 0] / V[2, 2], eta=V[2, 1] / V[2, 2])


def rotate(V, b):
    """R = B V^T on the *uncentred* baselines (§3.1)."""
    return b @ np.asarray(V).T


# ----------------------------------------------------------------------------
# pixel grids

def pixel_offsets(n_pix: int, cell_deg: float):
    """(l or t1 per column j1, m or t2 per row j2) in radians."""
    d = math.radians(cell_deg)
    j = np.arange(n_pix, dtype=np.float64) - n_pix / 2
    return -d * j, d * j


# ----------------------------------------------------------------------------
# §3.2: 2-D dirty image

def _phasor_matrix(coord, t):
    """exp(i 2 pi coord_q t_j) as a (Nq, Nt) matrix."""
    return np.exp(2j * math.pi * np.outer(coord, t))


def dft_sum_2d(r1, r2, v, t1, t2, chunk=8192):
    """sum_q v_q exp(i 2 pi (r1 t1 + r2 t2)) on the grid t1 (columns) x t2 (rows)."""
    out = np.zeros((t2.size, t1.size), dtype=np.complex128)
    for q0 in range(0, v.size, chunk):
        q1 = min(v.size, q0 + chunk)
        e1 = _phasor_matrix(r1[q0:q1], t1) * v[q0:q1, None]
        e2 = _phasor_matrix(r2[q0:q1], t2)
        out += e2.T @ e1
    return out


def image_2d(r, x, W, omega, n_pix, cell_deg):
    t1, t2 = pixel_offsets(n_pix, cell_deg)
    return np.real(dft_sum_2d(r[:, 0], r[:, 1], x, t1, t2)) / (omega * W)


# ----------------------------------------------------------------------------
# §3.4: near-coplanar (3-D) imaging

def t3_of(t1, t2, V):
    """Eq. (t3): the celestial-sphere branch nearest the transformed plane; NaN where not real."""
    V = np.asarray(V)
    arg = 1.0 - (t1 + V[0, 2]) ** 2 - (t2 + V[1, 2]) ** 2
    sgn = 1.0 if V[2, 2] >= 0 else -1.0
    with np.errstate(invalid="ignore"):
        return np.where(arg >= 0, -V[2, 2] + sgn * np.sqrt(np.maximum(arg, 0.0)), np.nan)


def t3_grid(V, n_pix, cell_deg):
    t1, t2 = pixel_offsets(n_pix, cell_deg)
    return t3_of(t1[None, :], t2[:, None], V)


def cheb_coeffs(alpha, K):
    """c_0 = J_0(alpha), c_k = 2 i^k J_k(alpha) (Jacobi-Anger, App. B2). Shape alpha.shape + (K,)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    k = np.arange(K)
    jk = special.jv(k, alpha[..., None])
    c = 2.0 * (1j ** k) * jk
    c[..., 0] = jk[..., 0]
    return c


def cheb_T(K, s):
    """T_k(s) = cos(k arccos s) for k < K; shape s.shape + (K,)."""
    s = np.clip(np.asarray(s, dtype=np.float64), -1.0, 1.0)
    return np.cos(np.arange(K) * np.arccos(s)[..., None])


def cheb_sampled_error(alpha_slab, K, n_grid=129):
    """max over alpha in [0, alpha_slab], s in [-1, 1] of |e^{i alpha s} - sum_k c_k T_k(s)|."""
    a = np.linspace(0.0, alpha_slab, n_grid)
    s = np.linspace(-1.0, 1.0, n_grid)
    approx = cheb_coeffs(a, K) @ cheb_T(K, s).T          # (alpha, s)
    exact = np.exp(1j * np.outer(a, s))
    return float(np.max(np.abs(exact - approx)))


def choose_k(alpha_slab, gamma=1e-2, choices=CHEB_K_CHOICES, n_grid=129):
    """Smallest K of the list whose sampled error is below gamma, else the largest."""
    for K in choices:
        if cheb_sampled_error(alpha_slab, K, n_grid) < gamma:
            return K
    return choices[-1]


@dataclasses.dataclass
class Plan:
    t3max: float
    r3min: float
    r3max: float
    phimax: float
    n_slab: int
    dr3: float
    alpha_slab: float
    K: int

    @property
    def planes(self):
        return self.n_slab * self.K

    def centre(self, p):
        return self.r3min + (2 * np.asarray(p) + 1) * self.dr3


def plan_from_scales(t3max, r3min, r3max, alpha_target=10.0, gamma=1e-2,
                     n_slab=0, K=0) -> Plan:
    """Eqs. (26)-(27) and the K rule; ``n_slab``/``K`` > 0 force a value."""
    phimax = 2.0 * math.pi * t3max * (r3max - r3min) / 2.0
    ns = n_slab if n_slab > 0 else max(1, math.ceil(phimax / alpha_target))
    dr3 = (r3max - r3min) / (2.0 * ns)
    if dr3 <= 0.0:
        ns, dr3 = 1, 0.0
    alpha_slab = 2.0 * math.pi * t3max * dr3
    kk = K if K > 0 else choose_k(alpha_slab, gamma)
    return Plan(t3max=t3max, r3min=r3min, r3max=r3max, phimax=phimax, n_slab=ns,
                dr3=dr3, alpha_slab=alpha_slab, K=kk)


def make_plan(r3, V, n_pix, cell_deg, alpha_target=10.0, gamma=1e-2, n_slab=0, K=0) -> Plan:
    t3 = t3_grid(V, n_pix, cell_deg)
    t3max = float(np.nanmax(np.abs(t3)))
    return plan_from_scales(t3max, float(r3.min()), float(r3.max()), alpha_target, gamma, n_slab, K)


def slab_of(r3, plan: Plan):
    if plan.dr3 == 0.0:
        return np.zeros(r3.shape, dtype=np.int64), np.zeros(r3.shape)
    p = np.minimum(plan.n_slab - 1, np.floor((r3 - plan.r3min) / (2.0 * plan.dr3))).astype(np.int64)
    p = np.maximum(p, 0)
    s = (r3 - plan.centre(p)) / plan.dr3
    return p, s


def pixel_subgrid(n_pix: int, cell_deg: float, j1=None, j2=None):
    """(t1 of the pixel columns j1, t2 of the pixel rows j2); every pixel by default."""
    t1a, t2a = pixel_offsets(n_pix, cell_deg)
    if j1 is not None:
        t1a = t1a[np.asarray(j1, dtype=np.int64)]
    if j2 is not None:
        t2a = t2a[np.asarray(j2, dtype=np.int64)]
    return t1a, t2a


def moments(r, x, plan: Plan, n_pix, cell_deg, j1=None, j2=None):
    """M_{p,k}(t1, t2) = sum_{q in S_p} T_k(s_q) x_q e^{i 2 pi (r1 t1 + r2 t2)} at the pixel
    columns j1 and rows j2 (all pixels by default); shape (n_slab, K, len(j2), len(j1)).

    The sum over samples runs in chunks; each chunk's phasors are formed once
    and contracted with every order k in one matrix product over the samples
    (the orders side by side in the columns)."""
    t1, t2 = pixel_subgrid(n_pix, cell_deg, j1, j2)
    p, s = slab_of(r[:, 2], plan)
    T = cheb_T(plan.K, s)
    K, n1, n2 = plan.K, t1.size, t2.size
    out = np.zeros((plan.n_slab, n2, n1, K), dtype=np.complex128)
    chunk = max(256, (1 << 22) // (n1 * K))
    for ps in range(plan.n_slab):
        sel = np.nonzero(p == ps)[0]
        for q0 in range(0, sel.size, chunk):
            q = sel[q0:q0 + chunk]
            e1 = _phasor_matrix(r[q, 0], t1)                         # (nq, columns)
            e2t = _phasor_matrix(r[q, 1], t2).T                      # (rows, nq)
            xt = x[q, None] * T[q]                                   # (nq, K)
            out[ps] += (e2t @ (e1[:, :, None] * xt[:, None, :]).reshape(q.size, n1 * K)).reshape(n2, n1, K)
    return np.ascontiguousarray(out.transpose(0, 3, 1, 2))


def image_3d_cheb(r, x, W, omega, V, plan: Plan, n_pix, cell_deg, M=None, j1=None, j2=None):
    """Chebyshev/slab form of eq. (10) at the pixel columns j1 and rows j2 (all
    pixels by default); zero where t3 is not real.  ``M``: the moments on the
    same pixels, if already computed."""
    if M is None:
        M = moments(r, x, plan, n_pix, cell_deg, j1, j2)
    t1, t2 = pixel_subgrid(n_pix, cell_deg, j1, j2)
    t3 = t3_of(t1[None, :], t2[:, None], V)
    valid = np.isfinite(t3)
    t3z = np.where(valid, t3, 0.0)
    c = cheb_coeffs(2.0 * math.pi * plan.dr3 * t3z, plan.K)          # (rows, columns, K)
    acc = np.zeros(t3.shape, dtype=np.complex128)
    for ps in range(plan.n_slab):
        inner = np.einsum("yxk,kyx->yx", c, M[ps])
        acc += np.exp(2j * math.pi * plan.centre(ps) * t3z) * inner
    return np.where(valid, np.real(acc) / (omega * W), 0.0)


def image_3d_exact(r, x, W, omega, V, n_pix, cell_deg, chunk=4096):
    """Eq. (10) summed directly: Re[(1/(omega W)) sum_q x_q e^{i 2 pi r_q . t}] (zero where t3 not real)."""
    t1, t2 = pixel_offsets(n_pix, cell_deg)
    t3 = t3_grid(V, n_pix, cell_deg)
    valid = np.isfinite(t3)
    t3z = np.where(valid, t3, 0.0)
    out = np.zeros((n_pix, n_pix))
    for j2 in range(n_pix):
        acc = np.zeros(n_pix, dtype=np.complex128)
        for q0 in range(0, x.size, chunk):
            q1 = min(x.size, q0 + chunk)
            ph = (np.outer(r[q0:q1, 0], t1) + r[q0:q1, 1:2] * t2[j2]
                  + np.outer(r[q0:q1, 2], t3z[j2]))
            acc += x[q0:q1] @ np.exp(2j * math.pi * ph)
        out[j2] = np.real(acc) / (omega * W)
    return np.where(valid, out, 0.0)


def tplane_at(r, x, W, omega, t1, t2, t3=None):
    """Eq. (10) (or eq. I_D^(2) with t3 = None) at arbitrary transformed coordinates."""
    t1 = np.atleast_1d(np.asarray(t1, dtype=np.float64))
    t2 = np.atleast_1d(np.asarray(t2, dtype=np.float64))
    ph = np.outer(r[:, 0], t1) + np.outer(r[:, 1], t2)
    if t3 is not None:
        ph = ph + np.outer(r[:, 2], np.atleast_1d(t3))
    return np.real(x @ np.exp(2j * math.pi * ph)) / (omega * W)


# ----------------------------------------------------------------------------
# §3.3 and App. A: re-projection

def reproject_coords(V, n_pix, cell_deg, j1=None, j2=None):
    """For output (standard SIN) pixels, the fractional transformed-plane indices (u1, u2).

    ``t = V s`` with ``s = (l, m, n - 1)`` inverts eq. (9); the transformed-plane
    pixel of ``(t1, t2)`` follows the pixel convention.  Returns (u1, u2, ok)
    where ``ok`` is False outside the unit circle of direction cosines.
    """
    V = np.asarray(V)
    d = math.radians(cell_deg)
    if j1 is None:
        l1, m1 = pixel_offsets(n_pix, cell_deg)
        l, m = np.meshgrid(l1, m1)
    else:
        l = -d * (np.asarray(j1, dtype=np.float64) - n_pix / 2)
        m = d * (np.asarray(j2, dtype=np.float64) - n_pix / 2)
    rho2 = l * l + m * m
    ok = rho2 < 1.0
    n = np.sqrt(np.where(ok, 1.0 - rho2, 1.0))
    nm1 = n - 1.0
    t1 = V[0, 0] * l + V[0, 1] * m + V[0, 2] * nm1
    t2 = V[1, 0] * l + V[1, 1] * m + V[1, 2] * nm1
    return n_pix / 2 - t1 / d, n_pix / 2 + t2 / d, ok


def bilinear(img, u1, u2, ok=None):
    """Bilinear gather img[u2][u1]; 0 and invalid where any neighbour is outside the image."""
    n2, n1 = img.shape
    i1 = np.floor(u1); i2 = np.floor(u2)
    valid = (i1 >= 0) & (i1 + 1 <= n1 - 1) & (i2 >= 0) & (i2 + 1 <= n2 - 1)
    if ok is not None:
        valid &= ok
    f1 = np.where(valid, u1 - i1, 0.0); f2 = np.where(valid, u2 - i2, 0.0)
    a = np.where(valid, i1, 0).astype(np.int64); c = np.where(valid, i2, 0).astype(np.int64)
    a1 = np.minimum(a + 1, n1 - 1); c1 = np.minimum(c + 1, n2 - 1)
    v = ((1 - f1) * (1 - f2) * img[c, a] + f1 * (1 - f2) * img[c, a1]
         + (1 - f1) * f2 * img[c1, a] + f1 * f2 * img[c1, a1])
    return np.where(valid, v, 0.0), valid


def reproject(tplane, V, n_pix, cell_deg):
    u1, u2, ok = reproject_coords(V, n_pix, cell_deg)
    return bilinear(tplane, u1, u2, ok)


def reduced_sin_map(p1, p2, xi, eta, n_pix, cell_deg):
    """§3.3's algebraic mapping from a standard-grid pixel to the tilted-plane pixel.

    The second axis uses ``y' = y + r0 z eta`` (the sign that App. A fixes and
    that maps an untilted plane onto itself); the literal ``h yhat`` of §3.3
    would flip the axis.  Pixels are 1-based as in the paper.
    """
    r0 = 180.0 / math.pi
    beta = cell_deg
    x = -beta * (np.asarray(p1, dtype=np.float64) - (n_pix / 2 + 1))
    y = beta * (np.asarray(p2, dtype=np.float64) - (n_pix / 2 + 1))
    h = np.sqrt(x * x + y * y)
    q = (h / r0) ** 2
    z = q / (1.0 + np.sqrt(1.0 - q))
    xp = x + r0 * z * xi
    yp = y + r0 * z * eta
    return -xp / beta + n_pix / 2 + 1, yp / beta + n_pix / 2 + 1


def wcs_sin_chain(p1, p2, xi, eta, n_pix, cell_deg, eps=1e-10):
    """App. A: pixel -> (x, y) -> native (phi, theta) -> slant-SIN (x, y) -> pixel."""
    p1 = np.atleast_1d(np.asarray(p1, dtype=np.float64))
    p2 = np.atleast_1d(np.asarray(p2, dtype=np.float64))
    x = -math.pi / 180 * cell_deg * (p1 - (n_pix / 2 + 1))
    y = math.pi / 180 * cell_deg * (p2 - (n_pix / 2 + 1))
    out1 = np.empty_like(x); out2 = np.empty_like(x)
    for i in range(x.size):
        xi_, yi_ = x[i], y[i]
        if xi_ == 0 and yi_ <= 0:
            phi = 0.0
        elif xi_ == 0 and yi_ > 0:
            phi = 180.0
        elif yi_ == 0 and xi_ > 0:
            phi = 90.0
        elif yi_ == 0 and xi_ < 0:
            phi = -90.0
        else:
            phi = math.degrees(math.atan2(xi_, -yi_))
        r2 = xi_ * xi_ + yi_ * yi_
        if r2 < 0.5:
            rr = math.sqrt(r2)
            if rr >= 1 and rr - 1 < eps:
                theta = 0.0
            elif rr == 0:
                theta = 90.0
            elif rr <= -1 and rr + 1 > -eps:
                theta = 180.0
            else:
                theta = math.degrees(math.acos(rr))
        else:
            cc = math.sqrt(1 - r2)
            if cc <= -1 and cc + 1 > -eps:
                theta = -90.0
            elif cc == 0:
                theta = 0.0
            elif cc >= 1 and cc - 1 < eps:
                theta = 90.0
            else:
                theta = math.degrees(math.asin(cc))
        ph, th = math.radians(phi), math.radians(theta)
        xo = 180 / math.pi * (math.cos(th) * math.sin(ph) + xi * (1 - math.sin(th)))
        yo = -180 / math.pi * (math.cos(th) * math.cos(ph) - eta * (1 - math.sin(th)))
        out1[i] = -xo / cell_deg + n_pix / 2 + 1
        out2[i] = yo / cell_deg + n_pix / 2 + 1
    return out1, out2


# ----------------------------------------------------------------------------
# the whole per-snapshot imaging path

@dataclasses.dataclass
class Result:
    samples: Samples
    basis: Basis
    r: np.ndarray
    plan: Plan
    tplane: np.ndarray     # transformed-plane image img[j2][j1]
    image: np.ndarray      # re-projected image
    valid: np.ndarray      # re-projection validity mask


def image_snapshot(snap, n_pix, cell_deg, mode=3, n_slab=0, K=0, alpha_target=10.0,
                   gamma=1e-2, corr_mask=None, exact=False) -> Result:
    """§3: samples -> basis -> rotation -> (2-D | Chebyshev 3-D | exact 3-D) image -> re-projection."""
    smp = select_samples(snap, corr_mask)
    bas = snapshot_basis(smp.b)
    r = rotate(bas.V, smp.b)
    if mode == 2:
        plan = Plan(t3max=0.0, r3min=float(r[:, 2].min()), r3max=float(r[:, 2].max()),
                    phimax=0.0, n_slab=1, dr3=0.0, alpha_slab=0.0, K=1)
        tp = image_2d(r, smp.x, smp.W, bas.omega, n_pix, cell_deg)
    else:
        plan = make_plan(r[:, 2], bas.V, n_pix, cell_deg, alpha_target, gamma, n_slab, K)
        if exact:
            tp = image_3d_exact(r, smp.x, smp.W, bas.omega, bas.V, n_pix, cell_deg)
        else:
            tp = image_3d_cheb(r, smp.x, smp.W, bas.omega, bas.V, plan, n_pix, cell_deg)
    img, valid = reproject(tp, bas.V, n_pix, cell_deg)
    return Result(samples=smp, basis=bas, r=r, plan=plan, tplane=tp, image=img, valid=valid)
