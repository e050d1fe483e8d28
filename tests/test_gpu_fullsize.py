"""Parity at the real workload shapes (MeerKAT-shaped 2048^2 and the full 4096^2
snapshot): basis and plan against the oracle on all samples, and the t-plane
and re-projected image at sampled pixels evaluated one by one by the oracle."""
import math

import numpy as np
import pytest

import synth_inputs as S
from oracle import toi as O

from gpu_helpers import IMAGE_TOL

pytestmark = pytest.mark.gpu


def _snapshot_on_device(wl, snap_index):
    import torch
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
    brightest = int(np.argmax(f))
    return host, T.to_device(host), (l[brightest], m[brightest])


@pytest.mark.parametrize("name", ["meerkat", "full"])
def test_sampled_parity_at_full_size(name):
    from paper_2512_06254_amd import toi as T
    wl = S.WORKLOADS[name]
    n_slab, K = wl.forced_planes
    host, dev, (lb, mb) = _snapshot_on_device(wl, 0)
    N = wl.n_pix
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=n_slab, cheb_k=K)
    im.grid(dev)
    img, tp = im.image(tplane=True)
    info = im.plan_info()
    img, tp = img.cpu().numpy(), tp.cpu().numpy()
    im.close()
    smp = O.select_samples(host)
    bas = O.snapshot_basis(smp.b)
    r = O.rotate(bas.V, smp.b)
    plan = O.make_plan(r[:, 2], bas.V, N, wl.cell_deg, n_slab=n_slab, K=K)
    np.testing.assert_allclose(info["V"], bas.V, atol=1e-10)
    assert abs(info["wsum"] - smp.W) <= 1e-12 * smp.W and info["status"] == 0
    # t-plane pixels: the brightest source's pixel, its neighbours and random ones (incl. near the edge)
    d = math.radians(wl.cell_deg)
    nb = math.sqrt(1 - lb * lb - mb * mb)
    t = bas.V @ np.array([lb, mb, nb - 1])
    jb1, jb2 = int(round(N / 2 - t[0] / d)), int(round(N / 2 + t[1] / d))
    rng = np.random.default_rng(1)
    j1 = np.concatenate([[jb1, jb1 + 1, jb1 - 1, jb1], rng.integers(0, N, 10), [0, N - 1]])
    j2 = np.concatenate([[jb2, jb2, jb2, jb2 + 1], rng.integers(0, N, 10), [N - 1, 0]])
    ref = O.image_cheb_at(r, smp.x, smp.W, bas.omega, bas.V, plan, j1, j2, N, wl.cell_deg)
    got = tp[j2, j1]
    scale = np.abs(ref).max()
    e_tp = np.abs(got - ref).max() / scale
    # re-projected pixels: bilinear from oracle t-plane values at the four source pixels
    o1 = rng.integers(N // 8, 7 * N // 8, 4)
    o2 = rng.integers(N // 8, 7 * N // 8, 4)
    u1, u2, ok = O.reproject_coords(bas.V, N, wl.cell_deg, o1, o2)
    i1, i2 = np.floor(u1).astype(int), np.floor(u2).astype(int)
    f1, f2 = u1 - i1, u2 - i2
    q1 = np.concatenate([i1, i1 + 1, i1, i1 + 1])
    q2 = np.concatenate([i2, i2, i2 + 1, i2 + 1])
    vals = O.image_cheb_at(r, smp.x, smp.W, bas.omega, bas.V, plan, q1, q2, N, wl.cell_deg).reshape(4, -1)
    ref_img = ((1 - f1) * (1 - f2) * vals[0] + f1 * (1 - f2) * vals[1] + (1 - f1) * f2 * vals[2]
               + f1 * f2 * vals[3])
    e_im = np.abs(img[o2, o1] - ref_img).max() / scale
    print(f"[{name}] plan ({info['n_slab']},{info['K']}) t-plane err {e_tp:.3e} image err {e_im:.3e} "
          f"(scale {scale:.4f} at the brightest source)", flush=True)
    assert e_tp <= IMAGE_TOL and e_im <= IMAGE_TOL
