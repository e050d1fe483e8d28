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
