"""FP64 adjoint of the snapshot imager and the gradients it yields.  TEST INFRASTRUCTURE ONLY.

The map from the weighted visibility sums ``x`` to the re-projected image is
real-linear: ``I = P(T(x))`` with ``T`` the Chebyshev/slab transformed-plane
image of §3.4 (or the exact sum of eq. 10) and ``P`` the bilinear
re-projection.  Under the real inner products ``<I, y> = sum I y`` and
``<x, z> = Re sum conj(z) x`` its adjoint is

    (G^H y)_q = (1 / (omega W)) sum_t (P^T y)(t) conj(phi_q(t)),

with ``phi_q(t) = e^{i 2 pi r_q . t}`` (exact) or its Chebyshev expansion
``e^{i 2 pi r3p t3} sum_k c_k(alpha(t)) T_k(s_q) e^{i 2 pi (r1 t1 + r2 t2)}``.

Gradient convention: for a real loss, ``dL/dRe z + i dL/dIm z`` (what a
central finite difference measures and what PyTorch returns).  With
``x = g_a1 conj(g_a2) sum_k W_k (1 - F_k) V_k``:
``grad V_k = conj(g_a1 conj(g_a2)) W_k (1 - F_k) grad x``;
``grad g_a1 += g_a2 conj(y) grad x`` and ``grad g_a2 += conj(grad x) g_a1 y``
with ``y = sum_k W_k (1 - F_k) V_k``, summed over the channels of each row.
"""
from __future__ import annotations

import math

import numpy as np

from . import toi


def reproject_transpose(y, V, n_pix, cell_deg):
    """P^T: scatter each output pixel's value with its bilinear weights onto the t-plane."""
    u1, u2, ok = toi.reproject_coords(V, n_pix, cell_deg)
    i1 = np.floor(u1); i2 = np.floor(u2)
    valid = ok & (i1 >= 0) & (i1 + 1 <= n_pix - 1) & (i2 >= 0) & (i2 + 1 <= n_pix - 1)
    f1 = (u1 - i1)[valid]; f2 = (u2 - i2)[valid]
    a = i1[valid].astype(np.int64); c = i2[valid].astype(np.int64)
    v = np.asarray(y, dtype=np.float64)[valid]
    out = np.zeros((n_pix, n_pix))
    np.add.at(out, (c, a), (1 - f1) * (1 - f2) * v)
    np.add.at(out, (c, a + 1), f1 * (1 - f2) * v)
    np.add.at(out, (c + 1, a), (1 - f1) * f2 * v)
    np.add.at(out, (c + 1, a + 1), f1 * f2 * v)
    return out


def tplane_adjoint_cheb(ytp, r, W, omega, V, plan, n_pix, cell_deg):
    """Adjoint of the Chebyshev/slab t-plane image: real (N, N) -> complex (Nq,)."""
    t1, t2 = toi.pixel_offsets(n_pix, cell_deg)
    t3 = toi.t3_grid(V, n_pix, cell_deg)
    valid = np.isfinite(t3)
    t3z = np.where(valid, t3, 0.0)
    y = np.where(valid, ytp, 0.0)
    c = toi.cheb_coeffs(2.0 * math.pi * plan.dr3 * t3z, plan.K)      # (N, N, K)
    p, s = toi.slab_of(r[:, 2], plan)
    T = toi.cheb_T(plan.K, s)
    out = np.zeros(r.shape[0], dtype=np.complex128)
    for ps in range(plan.n_slab):
        sel = np.nonzero(p == ps)[0]
        if sel.size == 0:
            continue
        e1c = np.exp(-2j * math.pi * np.outer(r[sel, 0], t1))          # (nq, N) over j1
        e2c = np.exp(-2j * math.pi * np.outer(r[sel, 1], t2))          # (nq, N) over j2
        ph = np.exp(-2j * math.pi * plan.centre(ps) * t3z)
        acc = np.zeros(sel.size, dtype=np.complex128)
        for k in range(plan.K):
            z = y * np.conj(c[..., k]) * ph                              # (j2, j1)
            a = z @ e1c.T                                                # (j2, nq)
            acc += T[sel, k] * np.sum(e2c.T * a, axis=0)
        out[sel] = acc
    return out / (omega * W)


def tplane_adjoint_exact(ytp, r, W, omega, V, n_pix, cell_deg):
    t1, t2 = toi.pixel_offsets(n_pix, cell_deg)
    t3 = toi.t3_grid(V, n_pix, cell_deg)
    valid = np.isfinite(t3)
    t3z = np.where(valid, t3, 0.0)
    y = np.where(valid, ytp, 0.0)
    out = np.zeros(r.shape[0], dtype=np.complex128)
    for j2 in range(n_pix):
        ph = np.outer(r[:, 0], t1) + r[:, 1:2] * t2[j2] + np.outer(r[:, 2], t3z[j2])
        out += np.exp(-2j * math.pi * ph) @ y[j2]
    return out / (omega * W)


class SnapshotOperator:
    """The linear imaging map of one snapshot (its geometry fixed) and its adjoint."""

    def __init__(self, snap, n_pix, cell_deg, mode=3, n_slab=0, K=0, corr_mask=None):
        res = toi.image_snapshot(snap, n_pix, cell_deg, mode=mode, n_slab=n_slab, K=K,
                                 corr_mask=corr_mask)
        self.snap, self.res = snap, res
        self.n_pix, self.cell_deg, self.mode = n_pix, cell_deg, mode
        self.corr_mask = corr_mask

    def forward(self, x):
        """x (Nq,) -> re-projected image (N, N)."""
        s, b, r, plan = self.res.samples, self.res.basis, self.res.r, self.res.plan
        if self.mode == 2:
            tp = toi.image_2d(r, x, s.W, b.omega, self.n_pix, self.cell_deg)
        else:
            tp = toi.image_3d_cheb(r, x, s.W, b.omega, b.V, plan, self.n_pix, self.cell_deg)
        return toi.reproject(tp, b.V, self.n_pix, self.cell_deg)[0]

    def adjoint(self, y):
        """y (N, N) -> complex (Nq,) = G^H y."""
        s, b, r, plan = self.res.samples, self.res.basis, self.res.r, self.res.plan
        ytp = reproject_transpose(y, b.V, self.n_pix, self.cell_deg)
        if self.mode == 2:
            return _adjoint_2d(ytp, r, s.W, b.omega, self.n_pix, self.cell_deg)
        return tplane_adjoint_cheb(ytp, r, s.W, b.omega, b.V, plan, self.n_pix, self.cell_deg)


def _adjoint_2d(ytp, r, W, omega, n_pix, cell_deg):
    t1, t2 = toi.pixel_offsets(n_pix, cell_deg)
    e1c = np.exp(-2j * math.pi * np.outer(r[:, 0], t1))
    e2c = np.exp(-2j * math.pi * np.outer(r[:, 1], t2))
    a = ytp @ e1c.T
    return np.sum(e2c.T * a, axis=0) / (omega * W)


def vis_gradients(snap, samples, grad_x, corr_mask=None):
    """Gradients w.r.t. the raw visibilities ``[row][chan][corr]`` and the antenna gains."""
    vis = np.asarray(snap["vis"]).astype(np.complex128)
    n_row, n_chan, n_corr = vis.shape
    wk = toi.sample_weights(snap, corr_mask)
    gx = np.zeros((n_row, n_chan), dtype=np.complex128)
    gx[samples.row, samples.chan] = grad_x
    g_row = toi.row_gains(snap)
    gain_fac = np.ones(n_row, dtype=np.complex128) if g_row is None else g_row
    grad_vis = np.conj(gain_fac)[:, None, None] * wk * gx[:, :, None]
    grad_g = None
    if snap.get("gains") is not None:
        g = np.asarray(snap["gains"], dtype=np.complex128)
        a1, a2 = np.asarray(snap["ant1"]), np.asarray(snap["ant2"])
        y = (wk * vis).sum(axis=2)                                       # pre-gain weighted sum
        t1 = (np.conj(y) * gx).sum(axis=1) * g[a2]
        t2 = (np.conj(gx) * y).sum(axis=1) * g[a1]
        grad_g = np.zeros(g.shape, dtype=np.complex128)
        np.add.at(grad_g, a1, t1)
        np.add.at(grad_g, a2, t2)
    return grad_vis, grad_g
