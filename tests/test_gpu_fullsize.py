"""Parity at the real grid shapes: the MeerKAT-shaped 2048^2 image (4096^2
grid), the full run's 4096^2 image (8192^2 grid) and the AA2-like 272-plane
snapshot (4096^2 grid), imaged by the GPU in the launch configuration the
benchmark times and checked against the FP64 oracle on pixel sub-grids:
32 x 32 = 1024 transformed-plane pixels (the brightest source's pixel and
its neighbours, both image edges, random rows and columns) and four 8 x 8
blocks = 256 re-projected pixels (centred on the two brightest sources and at
two random places), each re-projected oracle value interpolated from oracle
t-plane values at its four bilinear sources.

The oracle's cost is samples x evaluated pixels, so the two 16-plane shapes
keep every baseline, correlation and the band edges but use 512 channels
(eight times wider) instead of 4096; the benchmark's exact 4096-channel
snapshot is checked on basis, plan and a 4 x 4 pixel sub-grid."""
import math

import numpy as np
import pytest

import synth_inputs as S
from oracle import toi as O

from gpu_helpers import IMAGE_TOL

pytestmark = pytest.mark.gpu


def _snapshot_on_device(wl, snap_index):
    from paper_2512_06254_amd import toi as T
    enu, sky = S.antenna_enu(wl), S.make_sky(wl)
    uvw = S.snapshot_uvw(wl, snap_index, enu)
    freq = S.channel_freqs(wl)
    l, m, f = S.sources_at(sky, snap_index)
    vis = S.predict(uvw, freq, l, m, f, wl.n_corr, device="cuda", chunk_rows=32).cpu().numpy()
    vis += S.noise(wl, snap_index, vis.shape)
    a1, a2 = S.baseline_pairs(wl.n_ant)
    host = dict(uvw=uvw, vis=vis, flag=S.flags(wl, snap_index), weight=None, freq=freq, ant1=a1, ant2=a2,
                gains=None)
    order = np.argsort(-f)
    return host, T.to_device(host), [(l[i], m[i]) for i in order[:2]]


# gridder variants checked at the real shapes: 8 x 8 bins (the default) and
# 16 x 16 bins, both with 64-item work units and 16 planes per pass
VARIANTS = (1, 9)


def _gpu_image(wl, dev, n_slab, K, tuning=1):
    from paper_2512_06254_amd import toi as T
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=n_slab, cheb_k=K,
                  max_planes=n_slab * K)
    im.set_tuning(tuning)
    im.grid(dev)
    img, tp = im.image(tplane=True)
    info = im.plan_info()
    out = img.cpu().numpy(), tp.cpu().numpy(), info
    im.close()
    return out


def _tplane_pixel(V, l, m, N, cell_deg):
    """The transformed-plane pixel (j1, j2) nearest the direction (l, m): t = V s."""
    d = math.radians(cell_deg)
    t = V @ np.array([l, m, math.sqrt(1 - l * l - m * m) - 1])
    return int(round(N / 2 - t[0] / d)), int(round(N / 2 + t[1] / d))


def _sampled_parity(wl, n_slab, K, label, n_grid=32, n_blocks=4):
    host, dev, bright = _snapshot_on_device(wl, 0)
    N = wl.n_pix
    runs = {v: _gpu_image(wl, dev, n_slab, K, v) for v in VARIANTS}
    smp = O.select_samples(host)
    bas = O.snapshot_basis(smp.b)
    r = O.rotate(bas.V, smp.b)
    plan = O.make_plan(r[:, 2], bas.V, N, wl.cell_deg, n_slab=n_slab, K=K)
    for _, _, info in runs.values():
        np.testing.assert_allclose(info["V"], bas.V, atol=1e-10)
        assert abs(info["wsum"] - smp.W) <= 1e-12 * smp.W and info["status"] == 0
        assert (info["n_slab"], info["K"]) == (plan.n_slab, plan.K)
    rng = np.random.default_rng(1)
    # transformed plane: a sub-grid through the brightest source
    jb1, jb2 = _tplane_pixel(bas.V, *bright[0], N, wl.cell_deg)
    fixed1 = [jb1 - 1, jb1, jb1 + 1, 0, N - 1]
    fixed2 = [jb2 - 1, jb2, jb2 + 1, 0, N - 1]
    j1 = np.unique(np.concatenate([fixed1, rng.choice(N, n_grid, replace=False)]))[:n_grid]
    j2 = np.unique(np.concatenate([fixed2, rng.choice(N, n_grid, replace=False)]))[:n_grid]
    j1 = np.unique(np.concatenate([fixed1, j1]))
    j2 = np.unique(np.concatenate([fixed2, j2]))
    ref = O.image_3d_cheb(r, smp.x, smp.W, bas.omega, bas.V, plan, N, wl.cell_deg, j1=j1, j2=j2)
    scale = np.abs(ref).max()
    e_tp = {v: np.abs(tp[np.ix_(j2, j1)] - ref).max() / scale for v, (_, tp, _) in runs.items()}
    # re-projected pixels: 8 x 8 output blocks at the two brightest sources and two random places
    d = math.radians(wl.cell_deg)
    centres = [(int(round(N / 2 - l / d)), int(round(N / 2 + m / d))) for l, m in bright]
    centres += [tuple(rng.integers(N // 8, 7 * N // 8, 2)) for _ in range(n_blocks - len(centres))]
    e_im, n_px, n_valid, mismatch = dict.fromkeys(runs, 0.0), 0, dict.fromkeys(runs, 0), dict.fromkeys(runs, 0)
    for c1, c2 in centres:
        o1 = np.arange(c1 - 4, c1 + 4)
        o2 = np.arange(c2 - 4, c2 + 4)
        O1, O2 = np.meshgrid(o1, o2)
        u1, u2, ok = O.reproject_coords(bas.V, N, wl.cell_deg, O1, O2)
        q1 = np.arange(max(0, int(np.floor(u1.min()))), min(N, int(np.floor(u1.max())) + 2))
        q2 = np.arange(max(0, int(np.floor(u2.min()))), min(N, int(np.floor(u2.max())) + 2))
        vals = O.image_3d_cheb(r, smp.x, smp.W, bas.omega, bas.V, plan, N, wl.cell_deg, j1=q1, j2=q2)
        tp_part = np.zeros((N, N))
        tp_part[np.ix_(q2, q1)] = vals
        want, valid = O.bilinear(tp_part, u1, u2, ok)
        n_px += O1.size
        for v, (img, _, _) in runs.items():
            got = img[O2, O1]
            both = valid & (got != 0)
            if both.any():
                e_im[v] = max(e_im[v], np.abs(got[both] - want[both]).max() / scale)
            n_valid[v] += int(both.sum())
            mismatch[v] += int(np.sum(valid != (got != 0)))
    for v, (_, _, info) in runs.items():
        print(f"[{label}, variant {v}] plan ({info['n_slab']},{info['K']}) {j1.size}x{j2.size} t-plane pixels "
              f"err {e_tp[v]:.3e}; {n_px} re-projected pixels ({n_valid[v]} valid) err {e_im[v]:.3e}, validity "
              f"mismatches {mismatch[v]} (scale {scale:.4f} at the brightest source)", flush=True)
    assert j1.size * j2.size >= 1024 and n_px >= 256
    for v in runs:
        assert n_valid[v] >= 200
        assert e_tp[v] <= IMAGE_TOL and e_im[v] <= IMAGE_TOL
        assert mismatch[v] == 0


@pytest.mark.parametrize("name", ["meerkat", "full"])
def test_sampled_parity_at_full_grid_size(name):
    base = S.WORKLOADS[name]
    band = base.n_chan * base.dfreq_hz
    wl = S.scaled(base, n_chan=512, dfreq_hz=band / 512)
    _sampled_parity(wl, *base.forced_planes, f"{name}, 512 channels")


def test_sampled_parity_many_slab_272_planes():
    wl = S.WORKLOADS["aa2"]
    _sampled_parity(wl, *wl.forced_planes, "aa2 272 planes")


def test_benchmark_snapshot_basis_plan_and_pixels():
    """The benchmark's exact MeerKAT-shaped snapshot (2016 x 4096 x 4): basis and
    plan from all 8.26 M samples, and a 4 x 4 sub-grid through the brightest
    source."""
    wl = S.WORKLOADS["meerkat"]
    n_slab, K = wl.forced_planes
    host, dev, bright = _snapshot_on_device(wl, 0)
    N = wl.n_pix
    img, tp, info = _gpu_image(wl, dev, n_slab, K)
    smp = O.select_samples(host)
    bas = O.snapshot_basis(smp.b)
    r = O.rotate(bas.V, smp.b)
    plan = O.make_plan(r[:, 2], bas.V, N, wl.cell_deg, n_slab=n_slab, K=K)
    np.testing.assert_allclose(info["V"], bas.V, atol=1e-10)
    assert abs(info["wsum"] - smp.W) <= 1e-12 * smp.W and info["status"] == 0
    jb1, jb2 = _tplane_pixel(bas.V, *bright[0], N, wl.cell_deg)
    j1 = np.array([0, jb1 - 1, jb1, jb1 + 1])
    j2 = np.array([jb2 - 1, jb2, jb2 + 1, N - 1])
    ref = O.image_3d_cheb(r, smp.x, smp.W, bas.omega, bas.V, plan, N, wl.cell_deg, j1=j1, j2=j2)
    e = np.abs(tp[np.ix_(j2, j1)] - ref).max() / np.abs(ref).max()
    print(f"[meerkat 4096 ch] 16 t-plane pixels err {e:.3e} (peak {np.abs(ref).max():.4f})", flush=True)
    assert e <= IMAGE_TOL
