"""Batched execution (toi_image_batch, one captured HIP graph) against the
eager per-snapshot path and the oracle; replays interleaved with eager work."""
import numpy as np
import pytest

import synth_inputs as S
from oracle import fitrig as F
from oracle import toi as O

pytestmark = pytest.mark.gpu


def test_batched_graph_matches_eager_and_oracle():
    import torch
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["batched"], n_ant=10, n_chan=70, n_pix=128, n_steady=6, cell_arcsec=30.0,
                  diameter_m=2000.0, n_snap=8)
    sky, enu = S.make_sky(wl), S.antenna_enu(wl)
    host = [S.make_snapshot(wl, t, sky=sky, enu=enu) for t in range(6)]
    kept = [int((1 - h["flag"][:, :, 0]).sum()) for h in host]
    assert len(set(kept)) == len(kept)                 # uneven sample counts
    dev = [T.to_device(h) for h in host]
    N, TT = wl.n_pix, wl.n_pix // 32
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=16, tile=32)
    eager = []
    for d in dev:
        im.grid(d)
        eager.append(im.image().clone())
    eager_tl = [im.tlisi(eager[i - 2], eager[i - 1], eager[i]).clone() for i in range(2, len(dev))]
    imgs = torch.zeros((len(dev), N, N), device="cuda")
    tls = torch.zeros((len(dev) - 2, TT, TT), device="cuda")
    other = T.to_device(S.make_snapshot(wl, 7, sky=sky, enu=enu))
    for replay in range(3):
        imgs.zero_()
        im.image_batch(dev, imgs, tls)
        torch.cuda.synchronize()
        for i in range(len(dev)):
            peak = eager[i].abs().max().item()
            err = (imgs[i] - eager[i]).abs().max().item() / peak
            assert err < 1e-5, (replay, i, err)
        for i in range(len(dev) - 2):
            assert (tls[i] - eager_tl[i]).abs().max().item() < 1e-5
        im.grid(other)                                 # eager work between replays
        im.image()
        torch.cuda.synchronize()
    # one batched image against the oracle
    ref = O.image_snapshot(host[3], N, wl.cell_deg, mode=3, n_slab=1, K=16)
    e = np.abs(imgs[3].cpu().numpy() - ref.image).max() / np.abs(ref.image).max()
    print(f"[batch] oracle err {e:.3e}; kept samples per snapshot {kept}", flush=True)
    assert e < 1e-4
    im.close()


@pytest.mark.parametrize("n", [1, 2, 5])
def test_batched_lengths_match_eager(n):
    """One lane (n = 1) and two lanes ending on either per-snapshot set (n = 2, 5)."""
    import torch
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["batched"], n_ant=9, n_chan=40, n_pix=64, n_steady=4, cell_arcsec=60.0,
                  diameter_m=1500.0, n_snap=8)
    sky, enu = S.make_sky(wl), S.antenna_enu(wl)
    dev = [T.to_device(S.make_snapshot(wl, t, sky=sky, enu=enu)) for t in range(n)]
    N, TT = wl.n_pix, wl.n_pix // 32
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=8, tile=32)
    print(f"[batch lengths] n={n}", flush=True)
    eager = []
    for d in dev:
        im.grid(d)
        eager.append(im.image().clone())
    imgs = torch.zeros((n, N, N), device="cuda")
    tls = torch.zeros((max(n - 2, 1), TT, TT), device="cuda")
    for _ in range(2):
        imgs.zero_()
        im.image_batch(dev, imgs, tls if n >= 3 else None)
        torch.cuda.synchronize()
        for i in range(n):
            peak = eager[i].abs().max().item()
            assert (imgs[i] - eager[i]).abs().max().item() / peak < 1e-5, (n, i)
    im.grid(dev[0])                                    # the eager path after a batch
    again = im.image()
    torch.cuda.synchronize()
    assert (again - eager[0]).abs().max().item() / eager[0].abs().max().item() < 1e-5
    im.close()


def test_input_slots_replay_without_recapture():
    """A stream of batches through the context's input slots (toi_batch_inputs /
    toi_batch_fill): new data every call, the same descriptors, one capture;
    every batch equals the eager images of the data it was filled with."""
    import torch
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["batched"], n_ant=9, n_chan=40, n_pix=64, n_steady=4, cell_arcsec=60.0,
                  diameter_m=1500.0, n_snap=12)
    sky, enu = S.make_sky(wl), S.antenna_enu(wl)
    n, N, TT = 4, wl.n_pix, wl.n_pix // 32
    im = T.Imager(N, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=8, tile=32)
    im.batch_inputs(n, flags=True)
    imgs = torch.zeros((n, N, N), device="cuda")
    tls = torch.zeros((n - 2, TT, TT), device="cuda")
    for call in range(3):
        dev = [T.to_device(S.make_snapshot(wl, call * n + t, sky=sky, enu=enu)) for t in range(n)]
        eager = []
        for d in dev:
            im.grid(d)
            eager.append(im.image().clone())
        eager_tl = [im.tlisi(eager[i - 2], eager[i - 1], eager[i]).clone() for i in range(2, n)]
        for t, d in enumerate(dev):
            im.batch_fill(t, d)
        imgs.zero_()
        im.image_batch_slots(n, imgs, tls)
        torch.cuda.synchronize()
        for i in range(n):
            peak = eager[i].abs().max().item()
            assert (imgs[i] - eager[i]).abs().max().item() / peak < 1e-5, (call, i)
        for i in range(n - 2):
            assert (tls[i] - eager_tl[i]).abs().max().item() < 1e-5, (call, i)
    captures, launches = im.batch_info()
    print(f"[batch slots] captures {captures}, launches {launches}", flush=True)
    assert (captures, launches) == (1, 3)
    im.close()
