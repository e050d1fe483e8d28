"""fitrig_tlisi_noalloc (the tLISI entry point that allocates nothing) through
the C ABI: bit-identical to fitrig_tlisi on the same images, within the tLISI
tolerance of the FP64 oracle, on two calls in a row (the second smaller, so
the static scratch holds the first call's statistics when it starts), at the
largest size the scratch holds, and rejecting one tile more."""
import numpy as np
import pytest

from oracle import fitrig as F

pytestmark = pytest.mark.gpu

TLISI_TOL = 1e-3


def _images(n, seed):
    rng = np.random.default_rng(seed)
    base = rng.normal(0.0, 1.0, (n, n))
    imgs = [base + 0.1 * rng.normal(0.0, 1.0, (n, n)) for _ in range(3)]
    imgs[2][n // 4:n // 4 + n // 8, n // 2:n // 2 + n // 8] += 3.0   # a change in one corner of the sky
    return [im.astype(np.float32) for im in imgs]


def _ctx_tlisi(dev, n, tile):
    from paper_2512_06254_amd import toi as T
    im = T.Imager(n, 1e-3, 1, 64, 1, tile=tile)
    try:
        return im.tlisi(*dev).clone()
    finally:
        im.close()


def test_noalloc_tlisi_matches_context_entry_point_twice():
    import torch
    from paper_2512_06254_amd import toi as T
    outs = []
    for n, tile, seed in ((512, 32, 5), (128, 16, 6)):   # second call smaller
        host = _images(n, seed)
        dev = [torch.from_numpy(x).cuda() for x in host]
        out = torch.full((n // tile, n // tile), -7.0, device="cuda")
        T.tlisi_noalloc(*dev, tile, out)
        want = _ctx_tlisi(dev, n, tile)
        got = out.cpu().numpy()
        ref = F.tlisi(*host, tile=tile)
        err = np.abs(got - ref).max()
        print(f"noalloc tlisi n={n} tile={tile}: identical to fitrig_tlisi "
              f"{bool(torch.equal(out, want))}, oracle err {err:.2e}", flush=True)
        assert torch.equal(out, want)
        assert err <= TLISI_TOL
        assert got.min() < 0.9          # the planted change is seen
        outs.append(out)
    assert outs[0].shape == (16, 16) and outs[1].shape == (8, 8)


def test_noalloc_tlisi_largest_size_and_rejection():
    import torch
    from paper_2512_06254_amd import toi as T
    n, tile = 8192, 32                  # (8192 / 32)^2 = 65536 tiles: the static scratch exactly
    assert (n // tile) ** 2 == 65536
    host = _images(n, 7)
    dev = [torch.from_numpy(x).cuda() for x in host]
    out = torch.empty((n // tile, n // tile), device="cuda")
    T.tlisi_noalloc(*dev, tile, out)
    ref = F.tlisi(*host, tile=tile)
    err = np.abs(out.cpu().numpy() - ref).max()
    print(f"noalloc tlisi n={n} tile={tile}: oracle err {err:.2e}", flush=True)
    assert err <= TLISI_TOL
    small = torch.empty((n // 16, n // 16), device="cuda")
    with pytest.raises(T.ToiError) as e:
        T.tlisi_noalloc(*dev, 16, small)   # 262144 tiles
    assert e.value.code == T.TOI_EINVAL and "static scratch" in str(e.value)
