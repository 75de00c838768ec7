"""Host-side helpers of bench.py: the algorithmic-byte model (with 16-bit
coordinates), the default launch shape, and the committed traffic summary
being used only for the sources it was measured on."""

import os
import shutil

import bench


def test_algorithmic_bytes_per_mode():
    dims, nnz, R = (200, 150, 100), 1000, 32
    b = bench.algorithmic_bytes(dims, nnz, R)
    # mode 0: indices of 2 inputs + value, row pointers, both input factors, the output
    assert b[0] == nnz * (4 * 2 + 4) + 4 * 201 + (150 + 100) * R * 4 + 200 * R * 4
    b16 = bench.algorithmic_bytes(dims, nnz, R, idx16_modes=0b010)
    assert b16[1] == b[1] - nnz * 2 * 2 and b16[0] == b[0] and b16[2] == b[2]
    bf = bench.algorithmic_bytes(dims, nnz, R, factor_bytes=2)
    assert b[0] - bf[0] == (150 + 100) * R * 2


def test_default_shape_names():
    assert bench.default_shape(3, 16) == (8, 512, 2)
    assert bench.default_shape(3, 32) == (8, 512, 4)
    assert bench.default_shape(4, 32) == (8, 0, 0)


def test_traffic_summary_needs_matching_sources(tmp_path, monkeypatch):
    src = os.path.join(bench.ROOT, "profiles", "mttkrp_zipf1.2-20M-R32.traffic.txt")
    got = bench.profiled_traffic("zipf1.2-20M-R32")
    if got is not None:                           # summary taken on these sources
        bytes_, shape = got
        assert bytes_ > 0 and len(shape.split(",")) == 3
    # a copy with another digest is ignored
    root = tmp_path / "r"
    (root / "profiles").mkdir(parents=True)
    text = open(src).read().replace("sources_sha256 = ", "sources_sha256 = 0")
    (root / "profiles" / "mttkrp_x.traffic.txt").write_text(text)
    shutil.copytree(os.path.join(bench.ROOT, "paper_2503_18198_amd", "csrc"),
                    root / "paper_2503_18198_amd" / "csrc")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.profiled_traffic("x") is None
    assert bench.profiled_traffic("missing") is None
