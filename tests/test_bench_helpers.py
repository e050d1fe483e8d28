"""Host logic of bench.py: the HBM-traffic record is used only while the
gridder's sources match the digest it was taken with."""
import os
import shutil

import bench


def _tree(tmp_path):
    csrc = tmp_path / "paper_2512_06254_amd" / "csrc"
    csrc.mkdir(parents=True)
    for n in bench.GRIDDER_SOURCES:
        shutil.copy(os.path.join(bench.ROOT, "paper_2512_06254_amd", "csrc", n), csrc / n)
    (tmp_path / "profiles").mkdir()
    return csrc


def test_traffic_record_follows_the_source_digest(tmp_path, monkeypatch):
    csrc = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("k_grid_tiles_mfma") is None          # no record yet
    key = "source_sha256 " + "+".join(bench.GRIDDER_SOURCES)
    (tmp_path / "profiles" / "meerkat_hbm_traffic.md").write_text(
        f"# summary\ntraffic_bytes k_grid_tiles_mfma: 1234567\n{key}: {bench.sources_digest()}\n")
    assert bench.recorded_traffic("k_grid_tiles_mfma") == 1234567
    assert bench.recorded_traffic("k_other") is None                     # no line for that kernel
    with open(csrc / bench.GRIDDER_SOURCES[-1], "a") as f:              # any gridder source edited
        f.write("\n// edited\n")
    assert bench.recorded_traffic("k_grid_tiles_mfma") is None


def test_digest_depends_on_every_source(tmp_path, monkeypatch):
    csrc = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.sources_digest()
    for n in bench.GRIDDER_SOURCES:
        p = csrc / n
        text = p.read_text()
        p.write_text(text + " ")
        assert bench.sources_digest() != d0, n
        p.write_text(text)
    assert bench.sources_digest() == d0


def test_method_bytes_of_the_workloads():
    import synth_inputs as S
    # input once + each plane's M x N row-pass intermediate written and read once + ~6 images
    assert abs(bench.method_bytes(S.WORKLOADS["meerkat"], 16, False) - 2.512e9) < 0.005e9
    assert abs(bench.method_bytes(S.WORKLOADS["full"], 16, False) - 9.257e9) < 0.005e9
    assert abs(bench.method_bytes(S.WORKLOADS["adjoint"], 16, False) - 2.314e9) < 0.005e9
    assert abs(bench.method_bytes(S.WORKLOADS["adjoint"], 16, False, adjoint=True) - 2.281e9) < 0.005e9
    assert bench.hbm_frac(8e9, 1.0) == 1.0


def test_stage_bytes_count_only_occupied_tiles():
    import synth_inputs as S
    wl = S.WORKLOADS["meerkat"]
    NT = 2 * wl.n_pix // 8
    dense = bench.stage_bytes(wl, 16, False, {"tiles": NT * NT, "tile_rows": NT})
    M, N = 2 * wl.n_pix, wl.n_pix
    assert dense["fft_rows"] == 16 * M * M * 8 + 16 * N * M * 8          # every tile: the dense grid
    part = bench.stage_bytes(wl, 16, False, {"tiles": NT * NT // 5, "tile_rows": NT // 2})
    assert part["fft_rows"] < dense["fft_rows"] and part["grid"] < dense["grid"]
    assert bench.planes_per_group(16) == 16 and bench.planes_per_group(24) == 12 and bench.planes_per_group(8) == 8


def test_step_traffic_record_follows_every_source(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2512_06254_amd" / "csrc"
    csrc.mkdir(parents=True)
    for n in bench.ALL_SOURCES:
        shutil.copy(os.path.join(bench.ROOT, "paper_2512_06254_amd", "csrc", n), csrc / n)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles" / "meerkat_hbm_traffic.md").write_text(
        f"traffic_bytes step: 42\nsource_sha256 all: {bench.sources_digest(bench.ALL_SOURCES)}\n")
    assert bench.recorded_traffic("step", bench.ALL_SOURCES) == 42
    with open(csrc / bench.ALL_SOURCES[0], "a") as f:
        f.write("\n// edited\n")
    assert bench.recorded_traffic("step", bench.ALL_SOURCES) is None
