"""Streaming ingest (toi_ingest: host-resident snapshots, copies on a copy
stream overlapped with the imaging) against the device-resident path and the
oracle."""
import numpy as np
import pytest

import synth_inputs as S
from oracle import toi as O

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pinned", [True, False])
def test_ingest_matches_device_path_and_oracle(pinned):
    import torch
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["batched"], n_ant=10, n_chan=70, n_pix=128, n_steady=6, cell_arcsec=30.0,
                  diameter_m=2000.0, n_snap=8)
    sky, enu = S.make_sky(wl), S.antenna_enu(wl)
    host = [S.make_snapshot(wl, t, sky=sky, enu=enu) for t in range(5)]
    N, TT = wl.n_pix, wl.n_pix // 32
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=16, tile=32)
    ref = []
    for h in host:                                      # device-resident inputs
        im.grid(T.to_device(h))
        ref.append(im.image().clone())
    ref_tl = [im.tlisi(ref[i - 2], ref[i - 1], ref[i]).clone() for i in range(2, len(host))]
    hs = [T.to_host(h, pinned=pinned) for h in host]
    imgs = torch.zeros((len(host), N, N), device="cuda")
    tls = torch.zeros((len(host) - 2, TT, TT), device="cuda")
    for rep in range(2):                                # the second call reuses the staging slots
        imgs.zero_()
        im.ingest(hs, imgs, tls)
        torch.cuda.synchronize()
        for i in range(len(host)):
            err = (imgs[i] - ref[i]).abs().max().item() / ref[i].abs().max().item()
            assert err < 1e-5, (rep, i, err)
        for i in range(len(host) - 2):
            assert (tls[i] - ref_tl[i]).abs().max().item() < 1e-5
    o = O.image_snapshot(host[4], N, wl.cell_deg, mode=3, n_slab=1, K=16)
    e = np.abs(imgs[4].cpu().numpy() - o.image).max() / np.abs(o.image).max()
    print(f"[ingest pinned={pinned}] oracle err {e:.3e}", flush=True)
    assert e < 1e-4
    im.close()


def test_ingest_rejects_bad_arguments():
    import torch
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=6, n_chan=8, n_pix=64)
    h = T.to_host(S.make_snapshot(wl, 0))
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=4)
    with pytest.raises(TypeError):                      # device tensors are not host arrays
        im.ingest([T.to_device(S.make_snapshot(wl, 0))], torch.zeros((1, 64, 64), device="cuda"))
    big = dict(h)
    big["uvw"] = torch.zeros((wl.n_row + 1, 3), dtype=torch.float64)
    with pytest.raises(T.ToiError):                     # more rows than the context holds
        im.ingest([big], torch.zeros((1, 64, 64), device="cuda"))
    im.close()
