"""Host-side helpers of bench.py: the algorithmic-byte model (with 16-bit
coordinates), the default launch shape, and the committed traffic summary
being used only for the sources it was measured on, and the fiber statistics
(hand-counted and brute-force)."""

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


def _tensor(idx, dims):
    import numpy as np

    import workloads

    idx = np.asarray(idx, dtype=np.uint32)
    return workloads.SparseTensor(idx=idx, val=np.ones(len(idx), np.float32), dims=tuple(dims), nnz_requested=len(idx))


def test_fiber_stats_hand_counted():
    # mode 0 fibers (i0, i1): (0,1) x5, (0,2) x1, (1,1) x4
    idx = [(0, 1, k) for k in range(5)] + [(0, 2, 0)] + [(1, 1, k) for k in range(4)]
    got = bench.fiber_stats(_tensor(idx, (4, 5, 6)), R=32)
    m0 = got["modes"][0]
    assert m0["fibers"] == 3 and m0["mean_len"] == round(10 / 3, 2)
    assert m0["nnz_weighted_mean_len"] == round((25 + 1 + 16) / 10, 1)
    # one 4-segment each from the 5- and 4-long fibers: 2 * (1 + 4) gathers, 2 singles * 2
    assert m0["split_gathers_per_nnz"] == 1.4
    assert got["groups_per_wave"] == 8
    assert all(v["fraction"] is None for v in m0["whole_wave_skip"].values())   # not one whole wave
    # mode 1 fibers (i1, i2): (1,0)..(1,3) twice, (1,4) and (2,0) once; none reaches 4 nonzeros
    assert got["modes"][1]["fibers"] == 6 and got["modes"][1]["split_gathers_per_nnz"] == 2.0


def test_fiber_stats_wave_skip_brute_force():
    import numpy as np

    rng = np.random.default_rng(3)
    nnz = 3 * 256
    # few distinct (i0, i1) pairs so that long fibers occur
    idx = np.stack([rng.integers(0, 3, nnz), rng.integers(0, 4, nnz), rng.integers(0, 500, nnz)], axis=1)
    t = _tensor(idx, (3, 4, 500))
    got = bench.fiber_stats(t, R=32, shapes=((1, 256),), cus=1)
    for n in range(3):
        m = (n + 1) % 3
        key = sorted(int(a) * t.dims[m] + int(b) for a, b in zip(idx[:, n], idx[:, m]))
        gsz, G = 32, 8
        assert got["modes"][n]["whole_wave_skip"]["1/256"]["gsz"] == gsz
        skips = total = 0
        for w in range(nnz // (G * gsz)):
            for s in range(gsz):
                total += 1
                skips += all(s > 0 and key[w * G * gsz + g * gsz + s] == key[w * G * gsz + g * gsz + s - 1]
                             for g in range(G))
        assert got["modes"][n]["whole_wave_skip"]["1/256"]["fraction"] == round(skips / total, 4)
