"""Full-resolution localisation (fitrig_localise, fitrig_strongest_map through
the C ABI) against the FP64 oracle: exact selections (median, MAD, brightest
pixel, component) and FP64 positions."""
import math

import numpy as np
import pytest

from oracle import localise as Lz

pytestmark = pytest.mark.gpu


def _scene(N=512, seed=0):
    rng = np.random.default_rng(seed)
    j2, j1 = np.mgrid[0:N, 0:N]
    g = lambda x, y, sx, sy, a: a * np.exp(-0.5 * (((j1 - x) / sx) ** 2 + ((j2 - y) / sy) ** 2))
    a = rng.normal(scale=0.01, size=(N, N))
    b = a + rng.normal(scale=0.01, size=(N, N))
    b += g(100.3, 80.7, 1.6, 1.4, 0.8)            # switches on
    a += g(300.6, 220.2, 1.5, 1.5, 0.6)           # switches off: negative difference
    b += g(420.0, 400.0, 6.0, 0.8, 0.5)           # a streak: not Gaussian-like
    boxes = [(9, 64, 64, 127, 127), (9, 288, 192, 351, 255), (9, 384, 384, 447, 447), (9, 0, 448, 63, 511),
             (9, 480, 0, 543, 63)]             # the last leaves the image
    return a.astype(np.float32), b.astype(np.float32), boxes


@pytest.mark.parametrize("morph", [True, False])
def test_localise_matches_oracle(morph):
    import torch
    from paper_2512_06254_amd import toi as T
    N, cell, ra0, dec0 = 512, 0.0004, 135.37, -40.77
    a, b, boxes = _scene(N)
    im = T.Imager(N, cell, 1, 1, 1, mode=2, tile=32)
    out = im.localise(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(),
                      torch.tensor(boxes, dtype=torch.int32, device="cuda"), ra0, dec0, morph=morph)
    out = out.cpu().numpy()
    for k, bx in enumerate(boxes[:-1]):
        want = Lz.localise(a, b, bx, N, cell, ra0, dec0, morph=morph)
        got = out[k]
        print(f"[localise morph={morph} box {k}] {got.tolist()}", flush=True)
        assert bool(got[0]) == want["valid"] and int(got[7]) == want["n_pix"]
        assert got[5] == want["peak"] and got[6] == want["sigma"]
        if want["n_pix"] > 0:
            assert abs(got[1] - want["xc"]) < 1e-9 and abs(got[2] - want["yc"]) < 1e-9
            assert abs(got[3] - want["ra"]) < 1e-9 and abs(got[4] - want["dec"]) < 1e-9
    assert out[-1][7] == -1 and out[-1][0] == 0                      # outside the image
    # the rising and the falling source are found near their true positions
    assert abs(out[0][1] - 100.3) < 0.1 and abs(out[0][2] - 80.7) < 0.1 and out[0][0] == 1
    assert abs(out[1][1] - 300.6) < 0.1 and abs(out[1][2] - 220.2) < 0.1 and out[1][0] == 1
    assert out[2][0] == (0 if morph else 1)                           # the streak
    im.close()


def test_strongest_map_matches_oracle():
    import torch
    from paper_2512_06254_amd import toi as T
    rng = np.random.default_rng(1)
    L, Tt = 40, 16
    cube = (1.0 - np.abs(rng.normal(scale=0.01, size=(L, Tt, Tt)))).astype(np.float32)
    cube[17, 2:4, 5] -= 0.4
    cube[31, 10, 10:13] -= 0.3
    cube[5, 14, 0] -= 0.2
    boxes = [(39, 160, 64, 191, 127), (39, 320, 320, 415, 351), (39, 0, 448, 31, 479), (39, 0, 0, 511, 511)]
    im = T.Imager(Tt * 32, 0.001, 1, 1, 1, mode=2, tile=32)
    k = im.strongest_map(torch.from_numpy(cube).cuda(), torch.tensor(boxes, dtype=torch.int32, device="cuda"))
    got = k.cpu().numpy().tolist()
    want = [Lz.strongest_map(cube, bx) for bx in boxes]
    print(f"[strongest map] {got}", flush=True)
    assert got == want and got[:3] == [17, 31, 5]
    im.close()
