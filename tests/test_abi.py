"""The C-ABI library loads and exports every entry point the header declares,
and rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "toi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:toi_status|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2512_06254_amd import toi as T
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtoi.so not built")
    return T.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"toi_create", "toi_grid", "toi_image", "toi_degrid", "fitrig_tlisi"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2512_06254_amd import toi as T
    assert set(_declared()) == set(T._SIGS)


def test_argument_validation_without_device(lib):
    from paper_2512_06254_amd import toi as T
    p = T.Params()
    assert lib.toi_params_default(ctypes.byref(p), 256, 0.01, 10, 16, 4) == T.TOI_OK
    h = ctypes.c_void_p()
    bad = [("n_pix", 100), ("n_pix", 16), ("mode", 4), ("support", 6), ("n_corr", 3), ("tile", 48),
           ("cheb_k", 33), ("corr_mask", 0x10)]
    for field, val in bad:
        q = T.Params.from_buffer_copy(p)
        setattr(q, field, val)
        code = lib.toi_create(ctypes.byref(q), None, ctypes.byref(h))
        assert code in (T.TOI_EINVAL, T.TOI_EUNSUPPORTED), field
        assert h.value is None
        assert lib.toi_last_error(None)
    assert lib.toi_create(None, None, ctypes.byref(h)) == T.TOI_EINVAL
    for fn, args in (("toi_grid", (None, None)), ("toi_image", (None, None, None)),
                     ("fitrig_tlisi", (None, None, None, None, None)), ("toi_destroy", (None,)),
                     ("toi_ingest", (None, None, 1, None, None)),
                     ("fitrig_detect_cube", (None, None, 16, 0, None, 0, None)),
                     ("fitrig_localise", (None, None, None, None, 1, 0.0, 0.0, 1, None)),
                     ("fitrig_strongest_map", (None, None, 4, None, 1, None)),
                     ("toi_batch_inputs", (None, 1, 0, None)), ("toi_batch_fill", (None, 0, None)),
                     ("toi_batch_info", (None, None, None))):
        code = getattr(lib, fn)(*args)
        assert code == (T.TOI_OK if fn == "toi_destroy" else T.TOI_EINVAL), fn


def test_noalloc_tlisi_rejects_arguments_before_any_launch(lib):
    from paper_2512_06254_amd import toi as T
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: every case fails its argument check
    cases = [((None, fake, fake, 256, 32, fake, None), "NULL"),
             ((fake, fake, fake, 256, 0, fake, None), "tile"),
             ((fake, fake, fake, 250, 32, fake, None), "tile"),
             ((fake, fake, fake, 16384, 32, fake, None), "static scratch")]   # 262144 tiles
    for args, word in cases:
        assert lib.fitrig_tlisi_noalloc(*args) == T.TOI_EINVAL
        assert word in lib.toi_last_error(None).decode()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2512_06254_amd import toi as T
    monkeypatch.setattr(T, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(T, "_lib", None)
    with pytest.raises(RuntimeError):
        T.lib()
