"""Shared helpers of the GPU tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs."""
import numpy as np

import synth_inputs as S
from oracle import toi as O

IMAGE_TOL = 1e-4        # max |delta| <= 1e-4 of the image peak (FP32 vs the FP64 oracle)

# A compact array seen on a small grid: many work items share each 8 x 8 tile,
# so the heaviest bins are split into several work units.
DENSE = dict(n_ant=32, diameter_m=300.0, sigma_h_m=20.0, n_chan=128, n_pix=64, cell_arcsec=60.0)


def items_per_bin(wl, snap_index=0):
    """Work items (runs of 64 channels of one row) counted into every 8 x 8
    tile their footprints overlap, all channels counted as kept (host-side
    estimate of the gridder's bins, from the oracle's basis)."""
    enu = S.antenna_enu(wl)
    uvw = S.snapshot_uvw(wl, snap_index, enu)
    freq = S.channel_freqs(wl)
    b = (uvw[:, None, :] * (freq[None, :, None] / O.C_LIGHT)).reshape(-1, 3)
    V = O.snapshot_basis(b).V
    M = 2 * wl.n_pix
    r = uvw @ V.T
    ix = np.ceil(M / 2 - r[:, 0:1] * freq[None, :] / O.C_LIGHT * M * wl.cell_rad - 4).astype(int)
    iy = np.ceil(M / 2 + r[:, 1:2] * freq[None, :] / O.C_LIGHT * M * wl.cell_rad - 4).astype(int)
    NT = M // 8
    cnt = np.zeros((NT, NT), int)
    for row in range(ix.shape[0]):
        for c0 in range(0, wl.n_chan, 64):
            xs, ys = ix[row, c0:c0 + 64], iy[row, c0:c0 + 64]
            for ty in range(ys.min() >> 3, ((ys.max() + 7) >> 3) + 1):
                for tx in range(xs.min() >> 3, ((xs.max() + 7) >> 3) + 1):
                    cnt[ty % NT, tx % NT] += 1
    return cnt


def run_gpu(snap, n_pix, cell_deg, *, mode=3, n_slab=0, cheb_k=0, max_planes=0, tile=32, n_ant=0,
            corr_mask=0):
    from paper_2512_06254_amd import toi as T
    n_row, n_chan, n_corr = snap["vis"].shape
    im = T.Imager(n_pix, cell_deg, max(n_row, 1), n_chan, n_corr, mode=mode, n_slab=n_slab,
                  cheb_k=cheb_k, max_planes=max_planes, tile=tile, n_ant=n_ant, corr_mask=corr_mask)
    d = T.to_device(snap)
    im.grid(d)
    img, tp = im.image(tplane=True)
    info = im.plan_info()
    out = img.cpu().numpy(), tp.cpu().numpy(), info
    im.close()
    return out


def max_rel_err(gpu, ref, mask=None):
    peak = np.abs(ref).max()
    diff = np.abs(gpu - ref)
    if mask is not None:
        diff = diff[mask]
    return float(diff.max() / peak) if peak > 0 else float(diff.max())


def compare_basis(info, res):
    V = res.basis.V
    np.testing.assert_allclose(info["V"], V, atol=1e-10)
    assert abs(info["omega"] - res.basis.omega) < 1e-10
    assert abs(info["wsum"] - res.samples.W) <= 1e-12 * res.samples.W
    assert info["n_slab"] == res.plan.n_slab and info["K"] == res.plan.K


def check_snapshot(snap, n_pix, cell_deg, *, mode=3, n_slab=0, cheb_k=0, tol=IMAGE_TOL, label=""):
    res = O.image_snapshot(snap, n_pix, cell_deg, mode=mode, n_slab=n_slab, K=cheb_k)
    n_ant = 0 if snap.get("gains") is None else len(snap["gains"])
    img, tp, info = run_gpu(snap, n_pix, cell_deg, mode=mode, n_slab=n_slab, cheb_k=cheb_k, n_ant=n_ant,
                            max_planes=max(32, res.plan.planes))
    assert info["status"] == 0
    compare_basis(info, res)
    e_tp = max_rel_err(tp, res.tplane)
    both = res.valid & (img != 0)
    e_im = max_rel_err(img, res.image, both)
    # validity may differ only where a bilinear neighbour index sits on the image edge
    mismatch = int(np.sum(res.valid != (img != 0)))
    print(f"[{label}] tplane err {e_tp:.3e}  image err {e_im:.3e}  validity mismatches {mismatch}", flush=True)
    assert e_tp <= tol and e_im <= tol
    assert mismatch <= 2 * n_pix // 100 + 2
    return res, img, tp, info
