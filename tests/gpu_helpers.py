"""Shared helpers of the GPU tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs."""
import numpy as np

import synth_inputs as S
from oracle import toi as O

IMAGE_TOL = 1e-4        # max |delta| <= 1e-4 of the image peak (FP32 vs the FP64 oracle)


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
