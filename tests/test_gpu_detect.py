"""FITrig window detection (fitrig_detect through the C ABI): bit-exact
candidate boxes against the FP64 oracle on the same tLISI windows."""
import math

import numpy as np
import pytest

import synth_inputs as S
from oracle import fitrig as F

pytestmark = pytest.mark.gpu

Z_PER, Z_NONPER = 5.0, 4.0


def _window(seed, T=32, planted=True):
    rng = np.random.default_rng(seed)
    w = 1.0 - np.abs(rng.normal(scale=0.02, size=(16, T, T)))
    tau = np.arange(16)
    if planted:
        for (y, x) in [(3, 4), (4, 5), (20, 7)]:                     # two touching + one lone pulsing tile
            w[:, y, x] = 0.6 + 0.3 * np.cos(2 * math.pi * 4 * tau / 16 + 0.3 * seed)
        w[:, 12, 25] -= 0.25                                         # steady drop (non-periodic)
        w[8:, 28, 2] -= 0.3                                          # a transient half-way through
    return w.astype(np.float32)


def _guard(w):
    zp, zn = F.window_scores(w.astype(np.float64))
    return min(np.abs(zp - Z_PER).min(), np.abs(zn - Z_NONPER).min())


def _gpu_detect(w, t, max_boxes=64, tile=32):
    import torch
    from paper_2512_06254_amd import toi as T
    im = T.Imager(w.shape[1] * tile, 0.001, 1, 1, 1, mode=2, tile=tile)
    boxes, n = im.detect(torch.from_numpy(w).cuda(), t, max_boxes=max_boxes)
    n = int(n.item())
    out = [tuple(int(v) for v in b) for b in boxes.cpu().numpy()[:min(n, max_boxes)]]
    im.close()
    return out, n


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_boxes_bit_exact(seed):
    w = _window(seed)
    g = _guard(w)
    assert g > 1e-3, f"seed {seed}: a z-score lies within {g:.2e} of a threshold"
    want, _, _ = F.detect(w.astype(np.float64), t=100 + seed, tile=32)
    got, n = _gpu_detect(w, 100 + seed)
    print(f"[detect seed {seed}] {n} boxes, guard band {g:.3e}: {got}", flush=True)
    assert got == want and n == len(want)
    assert (100 + seed, 128, 96, 191, 159) in got                     # the touching pair is one box


def test_quiet_window_and_truncation():
    w = _window(5, planted=False)
    want, _, _ = F.detect(w.astype(np.float64), t=7, tile=32)
    got, n = _gpu_detect(w, 7)
    assert got == want
    w = _window(6)
    want, _, _ = F.detect(w.astype(np.float64), t=8, tile=32)
    got, n = _gpu_detect(w, 8, max_boxes=2)
    assert n == len(want) and got == want[:2]


def _cube(seed, L, T, period, tiles):
    rng = np.random.default_rng(seed)
    c = 1.0 - np.abs(rng.normal(scale=0.02, size=(L, T, T)))
    tau = np.arange(L)
    for (y, x) in tiles:                                             # on/off pulsar, 50% duty
        c[:, y, x] = np.where((tau % period) < period // 2, 0.55, 0.95) + rng.normal(scale=0.02, size=L)
    c[:, T - 3, 2] -= 0.15                                           # steady drop (non-periodic)
    return c.astype(np.float32)


def _gpu_detect_cube(c, t, max_boxes=64, tile=32):
    import torch
    from paper_2512_06254_amd import toi as T
    im = T.Imager(c.shape[1] * tile, 0.001, 1, 1, 1, mode=2, tile=tile)
    boxes, n = im.detect_cube(torch.from_numpy(c).cuda(), t, max_boxes=max_boxes)
    n = int(n.item())
    out = [tuple(int(v) for v in b) for b in boxes.cpu().numpy()[:min(n, max_boxes)]]
    im.close()
    return out, n


@pytest.mark.parametrize("seed,L,T,period", [(0, 150, 32, 12), (1, 600, 16, 12), (2, 97, 32, 10)])
def test_whole_cube_boxes_bit_exact(seed, L, T, period):
    # the after-the-run statistic over all L maps (L not a power of two)
    c = _cube(seed, L, T, period, [(3, 4), (4, 5), (T // 2, T // 3)])
    g = _guard(c)
    assert g > 1e-3, f"seed {seed}: a z-score lies within {g:.2e} of a threshold"
    want, _, _ = F.detect(c.astype(np.float64), t=L - 1, tile=32)
    got, n = _gpu_detect_cube(c, L - 1)
    print(f"[cube L={L} T={T}] {n} boxes, guard band {g:.3e}: {got}", flush=True)
    assert got == want and n == len(want)
    assert (L - 1, 128, 96, 191, 159) in got                        # the touching pulsar pair is one box


def test_whole_cube_rejects_bad_lengths():
    import torch
    from paper_2512_06254_amd import toi as T
    im = T.Imager(32 * 16, 0.001, 1, 1, 1, mode=2, tile=32)
    with pytest.raises(T.ToiError):
        im.detect_cube(torch.ones((1, 16, 16), device="cuda"), 0)
    im.close()
