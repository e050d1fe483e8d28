"""Per-stage HIP-event timing through the C ABI: the stage mask selects which
launches are timed, and timing does not change the image."""
import numpy as np
import pytest

import synth_inputs as S

pytestmark = pytest.mark.gpu


def _imager_and_snapshot():
    from paper_2512_06254_amd import toi as T
    wl = S.WORKLOADS["tiny"]
    snap = T.to_device(S.make_snapshot(wl, 0))
    n_row, n_chan, n_corr = snap["vis"].shape
    im = T.Imager(wl.n_pix, wl.cell_deg, n_row, n_chan, n_corr, mode=3, n_slab=1, cheb_k=4)
    return T, im, snap


def test_stage_mask_times_only_the_selected_stages():
    T, im, snap = _imager_and_snapshot()
    try:
        print("[profile] all stages, then grid only, then off", flush=True)
        im.grid(snap)
        ref = im.image().cpu().numpy()

        im.profile(True)
        for _ in range(3):
            im.grid(snap)
            img = im.image()
        every = im.profile_read()
        for name in ("prep", "bin", "grid", "fft_rows", "fft_cols", "reproject"):
            tot, n = every[name]
            assert n == 3 and tot > 0, (name, every[name])
        assert every["tlisi"][1] == 0 and every["degrid"][1] == 0
        np.testing.assert_allclose(img.cpu().numpy(), ref, rtol=0, atol=1e-6 * np.abs(ref).max())

        im.profile(True, stages=["grid"])            # clears the totals
        for _ in range(2):
            im.grid(snap)
            im.image()
        only = im.profile_read()
        assert only["grid"][1] == 2 and only["grid"][0] > 0
        assert all(n == 0 for name, (_, n) in only.items() if name != "grid"), only

        im.profile(False)
        im.grid(snap)
        im.image()
        after = im.profile_read()                    # disabling clears the totals and records nothing
        assert all(n == 0 for _, n in after.values()), after
    finally:
        im.close()
