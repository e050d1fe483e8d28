"""Pins of the oracle's sample selection and snapshot basis (§3.1, §3.2, §3.5)."""
import math

import numpy as np
import pytest

import synth_inputs as S
from oracle import toi


def _small(**kw):
    base = dict(n_ant=10, n_chan=8, n_pix=32, n_steady=2)
    base.update(kw)
    return S.scaled(S.WORKLOADS["tiny"], **base)


def test_sample_selection_hand_computed():
    # 1 row, 2 channels, 4 correlations; weights and flags on the parallel hands
    vis = np.array([[[1 + 1j, 5, 7, 3 - 1j], [2, 9, 9, 4j]]], dtype=np.complex64)
    flag = np.zeros(vis.shape, np.uint8); flag[0, 1, 3] = 1
    weight = np.array([[[2, 1, 1, 1], [1, 1, 1, 3]]], np.float32)
    snap = dict(uvw=np.array([[100.0, -50.0, 3.0]]), vis=vis, flag=flag, weight=weight,
                freq=np.array([1e9, 2e9]), ant1=np.array([0]), ant2=np.array([1]), gains=None)
    s = toi.select_samples(snap)
    # channel 0: w = 2 + 1, x = 2(1+1j) + (3-1j); channel 1: XX only (YY flagged): w = 1, x = 2
    np.testing.assert_allclose(s.w, [3.0, 1.0])
    np.testing.assert_allclose(s.x, [2 * (1 + 1j) + (3 - 1j), 2.0])
    assert s.W == 4.0
    lam = toi.C_LIGHT / np.array([1e9, 2e9])
    np.testing.assert_allclose(s.b, np.array([[100.0, -50.0, 3.0]]) / lam[:, None])
    # fully flagged samples disappear from every sum
    flag[0, 0, :] = 1
    s2 = toi.select_samples(snap)
    assert s2.n == 1 and s2.chan[0] == 1


def test_unit_weights_reduce_to_paper_normalisation():
    wl = _small(n_corr=4)
    snap = S.make_snapshot(wl, 0)
    s = toi.select_samples(snap)
    vis = snap["vis"].astype(np.complex128)
    paper_vis = 0.5 * (vis[:, :, 0] + vis[:, :, 3]).ravel()          # average of the parallel hands
    # (1/(omega W)) sum x  ==  (1/(omega N_vis)) sum Vis   for any phase factor
    ph = np.exp(1j * np.arange(s.n))
    assert s.W == 2 * s.n
    np.testing.assert_allclose((s.x * ph).sum() / s.W, (paper_vis * ph).sum() / s.n, rtol=1e-13)


def test_basis_is_orthonormal_right_handed():
    for seed in range(4):
        wl = _small(seed=seed, sigma_h_m=20.0)
        b = toi.select_samples(S.make_snapshot(wl, 0, with_noise=False)).b
        bas = toi.snapshot_basis(b)
        V = bas.V
        np.testing.assert_allclose(V @ V.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(V) - 1.0) < 1e-14
        assert V[2, 2] > 0                                  # e2 (and e3) signed by handedness
        assert V[0, np.argmax(np.abs(V[0]))] > 0            # e1: largest component positive
        assert bas.omega == pytest.approx(abs(V[0, 0] * V[1, 1] - V[1, 0] * V[0, 1]), abs=0)


def test_basis_recovers_known_plane_and_axes():
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    u, v, nrm = Q[:, 0], Q[:, 1], Q[:, 2]
    th = 2 * np.pi * np.arange(4096) / 4096   # exactly uncorrelated, zero-mean in-plane spreads
    a = 1000.0 * np.cos(th)                    # dominant spread along u
    c = 100.0 * np.sin(th)                     # second along v
    b = np.outer(a, u) + np.outer(c, v)
    bas = toi.snapshot_basis(b)
    assert abs(abs(bas.V[0] @ u) - 1) < 1e-12
    assert abs(abs(bas.V[1] @ v) - 1) < 1e-12
    assert abs(abs(bas.V[2] @ nrm) - 1) < 1e-12
    r = toi.rotate(bas.V, b)
    assert np.max(np.abs(r[:, 2])) < 1e-9 * np.max(np.abs(b))


def test_coplanar_array_has_zero_residual_coordinate():
    wl = _small(sigma_h_m=0.0)
    b = toi.select_samples(S.make_snapshot(wl, 0)).b
    bas = toi.snapshot_basis(b)
    r = toi.rotate(bas.V, b)
    assert np.max(np.abs(r[:, 2])) < 1e-9 * np.max(np.abs(b))
    sv = np.linalg.svd(b - b.mean(0), compute_uv=False)
    assert sv[2] < 1e-9 * sv[0]


def test_phase_is_preserved():
    wl = _small(sigma_h_m=10.0)
    b = toi.select_samples(S.make_snapshot(wl, 0)).b
    V = toi.snapshot_basis(b).V
    r = toi.rotate(V, b)
    rng = np.random.default_rng(1)
    t = rng.normal(0, 1e-2, (3, 50))
    s = V.T @ t                              # eq. (9): s = V^T t
    np.testing.assert_allclose(b @ s, r @ t, rtol=1e-12, atol=1e-9)


def test_omega_is_area_ratio_of_the_in_plane_map():
    wl = _small(sigma_h_m=10.0)
    V = toi.snapshot_basis(toi.select_samples(S.make_snapshot(wl, 0)).b).V
    h = 1e-6

    def lm(t1, t2):
        s = V.T @ np.array([t1, t2, 0.0])
        return s[:2]
    J = np.stack([(lm(h, 0) - lm(-h, 0)) / (2 * h), (lm(0, h) - lm(0, -h)) / (2 * h)], axis=1)
    assert abs(abs(np.linalg.det(J)) - toi.basis_from_V(V).omega) < 1e-9
