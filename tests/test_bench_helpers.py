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
