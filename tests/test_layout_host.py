"""Host logic of the library, no GPU: the mode copies built by
``mttkrp_layout_build`` (host-only handles), argument validation, the
footprint, and the exported C symbols."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2503_18198_amd import capi
from tests import pins

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mttkrp.h")


def host_layout(idx, val, dims, hot_rows=0):
    return capi.mttkrp_layout_build(idx, val, dims, opts=dict(host_only=1, hot_rows=hot_rows))


def row_of_each_nonzero(v):
    """Output row of each nonzero of a view, decoded from its row-start bits
    and per-word row ordinals."""
    nnz = v["nnz"]
    w = v["winfo"].reshape(-1, 2) if nnz else np.zeros((0, 2), np.uint32)
    k = np.arange(nnz)
    bits = (w[k // 32, 0] >> (k % 32).astype(np.uint32)) & 1
    # ordinal: ordinal of the word's first nonzero plus row starts after it within the word
    ordinal = np.empty(nnz, dtype=np.int64)
    for i in range(nnz):
        if i % 32 == 0:
            o = int(w[i // 32, 1])
        elif bits[i]:
            o += 1
        ordinal[i] = o
    return v["row_id"][ordinal].astype(np.int64), bits, ordinal


def decode(v, j):
    """Coordinates of input mode j with hot slots mapped back to rows."""
    raw = v["idx"][j].astype(np.int64)
    hot = (raw & 0x80000000) != 0
    out = raw.copy()
    out[hot] = v["hot_rows"][j][raw[hot] & 0x7FFFFFFF]
    return out


def check_view(idx, val, dims, v, n):
    N = len(dims)
    nnz = idx.shape[0]
    assert v["nnz"] == nnz and v["nnz_pad"] == (nnz + 31) // 32 * 32
    assert v["in_modes"] == [m for m in range(N) if m != n]
    src = v["src_pos"].astype(np.int64)
    # a permutation of the input, carrying every coordinate and value
    assert np.array_equal(np.sort(src), np.arange(nnz))
    for j, m in enumerate(v["in_modes"]):
        assert np.array_equal(decode(v, j)[:nnz], idx[src, m])
        assert not v["idx"][j][nnz:].any()
        # hot rows: the most frequent rows of mode m (degree >= 2), by degree then row
        deg = np.bincount(idx[:, m].astype(np.int64), minlength=dims[m])
        hot = v["hot_rows"][j]
        used = hot[: min(v["nhot"], int(np.sum(deg >= 2)))]
        order = np.lexsort((np.arange(dims[m]), -deg))
        assert np.array_equal(used, order[: used.shape[0]])
    assert np.array_equal(v["val"][:nnz], val[src])
    assert not v["val"][nnz:].any()
    rows, bits, ordinal = row_of_each_nonzero(v)
    assert np.array_equal(rows, idx[src, n].astype(np.int64))
    # order: output row, then the other modes cyclically, then input position
    cyc = [(n + j) % N for j in range(1, N)]
    keys = [idx[src, n].astype(np.int64)] + [idx[src, m].astype(np.int64) for m in cyc] + [src]
    order = np.lexsort(keys[::-1])
    assert np.array_equal(order, np.arange(nnz))
    # nonempty / empty rows partition [0, I_n)
    counts = np.bincount(idx[:, n].astype(np.int64), minlength=dims[n])
    assert np.array_equal(v["row_id"], np.nonzero(counts)[0])
    assert np.array_equal(v["empty_rows"], np.nonzero(counts == 0)[0])
    assert v["nrows_nz"] + v["nempty"] == dims[n]
    # a start bit exactly where a new row begins
    if nnz:
        starts = np.ones(nnz, dtype=bool)
        starts[1:] = rows[1:] != rows[:-1]
        assert np.array_equal(bits.astype(bool), starts)
        # padding bits are zero
        last = v["winfo"].reshape(-1, 2)[-1, 0]
        tail = nnz % 32
        if tail:
            assert (int(last) >> tail) == 0


CASES = {
    "random3": ((30, 20, 10), 500, 0),
    "random4_dups": ((9, 7, 5, 4), 300, 40),
    "random5": ((6, 5, 4, 3, 2), 200, 0),
    "tiny": ((3, 3, 3), 5, 0),
    "single_nnz": ((4, 5, 6), 1, 0),
    "exactly32": ((40, 40, 40), 32, 0),
    "dim_one": ((1, 50, 7), 120, 0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_layout_invariants(case):
    dims, nnz, dup = CASES[case]
    rng = np.random.default_rng(hash(case) % 2 ** 32)
    idx, val = pins.rand_coo(rng, dims, nnz, dup=dup)
    val = val.astype(np.float32)
    h = host_layout(idx, val, dims)
    for n in range(len(dims)):
        check_view(idx, val, dims, capi.mttkrp_layout_view(h, n), n)
    h.free()


def test_layout_one_heavy_row_and_empty_edges():
    """All nonzeros in one output row; leading and trailing empty rows."""
    rng = np.random.default_rng(3)
    dims = (100, 60, 50)
    nnz = 2000
    idx = np.stack([np.full(nnz, 57), rng.integers(0, 60, nnz), rng.integers(0, 50, nnz)], axis=1).astype(np.uint32)
    val = rng.random(nnz).astype(np.float32)
    h = host_layout(idx, val, dims)
    v = capi.mttkrp_layout_view(h, 0)
    check_view(idx, val, dims, v, 0)
    assert v["nrows_nz"] == 1 and list(v["row_id"]) == [57]
    assert v["nempty"] == 99
    for n in (1, 2):
        check_view(idx, val, dims, capi.mttkrp_layout_view(h, n), n)


def test_layout_empty_tensor():
    dims = (5, 6, 7)
    h = host_layout(np.zeros((0, 3), np.uint32), np.zeros(0, np.float32), dims)
    for n in range(3):
        v = capi.mttkrp_layout_view(h, n)
        assert v["nnz"] == 0 and v["nnz_pad"] == 0 and v["nrows_nz"] == 0
        assert np.array_equal(v["empty_rows"], np.arange(dims[n]))


def test_layout_wide_keys():
    """Packed coordinate keys wider than 64 bits: the 128-bit key sort."""
    rng = np.random.default_rng(4)
    dims = (50, 100_000, 100_000, 100_000, 100_000)  # 4 x 17 bits > 64
    nnz = 400
    idx = np.stack([rng.integers(0, d, nnz) for d in dims], axis=1).astype(np.uint32)
    idx[::7, 1] = idx[0, 1]  # ties in the first comparison key
    val = rng.random(nnz).astype(np.float32)
    h = host_layout(idx, val, dims)
    for n in range(5):
        check_view(idx, val, dims, capi.mttkrp_layout_view(h, n), n)


def test_layout_keys_over_128_bits():
    """Keys wider than 128 bits (8 modes of 2^17): the comparison sort."""
    rng = np.random.default_rng(5)
    dims = (1 << 17,) * 8
    nnz = 300
    idx = np.stack([rng.integers(0, 3 if m == 1 else d, nnz) for m, d in enumerate(dims)], axis=1).astype(np.uint32)
    idx[::5, 2] = idx[0, 2]
    val = rng.random(nnz).astype(np.float32)
    h = host_layout(idx, val, dims)
    for n in range(8):
        check_view(idx, val, dims, capi.mttkrp_layout_view(h, n), n)


@pytest.mark.parametrize("hot_rows", [0, 64])
@pytest.mark.parametrize("dims", [(300, 200, 150), (9000, 70_000, 100_000, 120, 100_000)])
def test_layout_threaded_sort(dims, hot_rows):
    """Enough nonzeros for the multithreaded sort (64- and 128-bit keys):
    Zipf-skewed rows, one row holding a quarter of the nonzeros, duplicates;
    with and without hot-row slots in the decoded indices."""
    rng = np.random.default_rng(6)
    nnz = 150_000
    idx = np.stack([np.minimum(rng.zipf(1.3, nnz) - 1, d - 1) for d in dims], axis=1).astype(np.uint32)
    idx[: nnz // 4, 0] = 7
    idx[1::97] = idx[0::97][: idx[1::97].shape[0]]
    val = rng.random(nnz).astype(np.float32)
    h = host_layout(idx, val, dims, hot_rows)
    for n in range(len(dims)):
        v = capi.mttkrp_layout_view(h, n)
        assert (v["nhot"] > 0) == (hot_rows > 0)     # capped by LDS room at 5 modes
        check_view(idx, val, dims, v, n)


def test_errors():
    idx = np.array([[0, 1, 2]], dtype=np.uint32)
    val = np.ones(1, np.float32)
    with pytest.raises(capi.MttkrpError) as e:
        host_layout(idx, val, (1, 1, 3))
    assert e.value.status == capi.MTTKRP_ERANGE
    with pytest.raises(capi.MttkrpError) as e:
        host_layout(np.zeros((1, 2), np.uint32), val, (3, 3))
    assert e.value.status == capi.MTTKRP_EUNSUPPORTED
    with pytest.raises(capi.MttkrpError) as e:
        host_layout(np.zeros((1, 3), np.uint32), val, (0, 3, 3))
    assert e.value.status == capi.MTTKRP_EINVAL
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_footprint((3, 3, 3), 10, opts=dict(max_R=48))
    assert e.value.status == capi.MTTKRP_EUNSUPPORTED
    # runs are refused on host-only handles, before any device call
    h = host_layout(idx, val, (1, 2, 3))
    with pytest.raises(capi.MttkrpError) as e:
        capi._check(capi._lib.mttkrp_run(ctypes.c_void_p(h.ptr), 0, (ctypes.c_void_p * 3)(), ctypes.c_void_p(0), 16,
                                         ctypes.c_void_p(0)))
    assert e.value.status == capi.MTTKRP_EINVAL
    # over-budget footprint is refused before anything is allocated
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_layout_build(idx, val, (1, 2, 3), opts=dict(hbm_budget_bytes=1024))
    assert e.value.status == capi.MTTKRP_ENOMEM


def test_footprint_formula():
    dims = (1000, 800, 600)
    nnz = 100_000
    fp = capi.mttkrp_footprint(dims, nnz, opts=dict(max_R=16))
    pad = (nnz + 31) // 32 * 32
    copies = sum(pad * (4 * 2 + 4) + pad // 32 * 8 + 4 * d for d in dims)
    assert copies <= fp <= copies + 16 * 1024 * 1024
    # the paper's memory model: N copies of nnz elements of sum(log2 dims) + 32 bits
    bits = sum(math.ceil(math.log2(d)) for d in dims) + 32
    assert 3 * nnz * bits / 8 <= copies
    fp64 = capi.mttkrp_footprint(dims, nnz, opts=dict(max_R=64))
    fpbf = capi.mttkrp_footprint(dims, nnz, opts=dict(max_R=64, factor_dtype=capi.MTTKRP_BF16))
    assert fp < fp64 < fpbf


def test_header_symbols_exported():
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(mttkrp_\w+|cpd_als_\w+)\s*\(", text, re.M))
    assert declared == set(capi.EXPORTED), declared ^ set(capi.EXPORTED)
    lib = ctypes.CDLL(capi.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("N,R,dtype", [(3, 32, capi.MTTKRP_FP32), (3, 64, capi.MTTKRP_FP32), (4, 64, capi.MTTKRP_FP32),
                                       (5, 16, capi.MTTKRP_FP32), (4, 64, capi.MTTKRP_BF16), (8, 16, capi.MTTKRP_FP32)])
@pytest.mark.parametrize("nnz", [0, 1, 33, 20_000_000, 100_000_000, 2_200_000_000, 4_000_000_000, 2**32 - 1])
def test_launch_plan_bounds_every_chain(N, R, dtype, nnz):
    """For every nnz the header accepts, each lane group's FP32 register chain
    is at most 4096 nonzeros (sequential FP32 sums past a few thousand terms
    lose the 1e-5 bar), the partitions cover every nonzero once, and the carry
    buffer holds two rows per partition."""
    p = capi.mttkrp_launch_plan(nnz, N, R, dtype)
    assert p["nonzeros_per_group"] % 32 == 0 and 32 <= p["nonzeros_per_group"] <= 4096
    assert p["nonzeros_per_part"] == p["nonzeros_per_group"] * p["lane_groups"]
    assert p["lane_groups"] * p["lanes_per_group"] == p["wg_threads"]
    if nnz:
        assert (p["nparts"] - 1) * p["nonzeros_per_part"] < nnz <= p["nparts"] * p["nonzeros_per_part"]
    else:
        assert p["nparts"] == 0
    assert p["carry_bytes"] >= p["nparts"] * 2 * R * 4
    # the default target: about 8 partitions per CU of a 256-CU device (fewer by
    # the round-up of each run to whole 32-nonzero batches) while chains allow it
    if 20_000_000 <= nnz <= 100_000_000 and N == 3:
        assert 0.8 * 2048 <= p["nparts"] <= 2048 + 256


def test_launch_plan_errors():
    for args in [(10, 2, 32), (10, 9, 32), (10, 3, 48)]:
        with pytest.raises(capi.MttkrpError) as e:
            capi.mttkrp_launch_plan(*args)
        assert e.value.status == capi.MTTKRP_EUNSUPPORTED
    with pytest.raises(capi.MttkrpError) as e:
        capi.mttkrp_launch_plan(2**32, 3, 32)
    assert e.value.status == capi.MTTKRP_EINVAL


def test_16bit_coordinates_footprint_and_modes():
    """A copy whose input dimensions are all <= 65536 stores 16-bit
    coordinates (3- to 5-mode tensors, nonzero split, no hot rows): the
    footprint shrinks by 2 bytes per input coordinate of such copies, and
    wide_indices=1 keeps 32 bits everywhere."""
    dims = (70000, 500, 400)           # copy 0 reads modes 1, 2 (16-bit); copies 1, 2 read mode 0 (32-bit)
    nnz = 100_000
    pad = (nnz + 31) // 32 * 32
    f16 = capi.mttkrp_footprint(dims, nnz)
    f32 = capi.mttkrp_footprint(dims, nnz, opts=dict(wide_indices=1))
    assert f32 - f16 == pad * 2 * 2     # one copy, two input coordinates each
    t = np.zeros((10, 3), dtype=np.uint32)
    h = capi.mttkrp_layout_build(t, np.ones(10, np.float32), dims, opts=dict(host_only=1))
    assert capi.mttkrp_layout_info(h)["idx16_modes"] == 0b001
    h2 = capi.mttkrp_layout_build(t, np.ones(10, np.float32), dims, opts=dict(host_only=1, wide_indices=1))
    assert capi.mttkrp_layout_info(h2)["idx16_modes"] == 0
    h3 = capi.mttkrp_layout_build(t, np.ones(10, np.float32), dims, opts=dict(host_only=1, hot_rows=8))
    assert capi.mttkrp_layout_info(h3)["idx16_modes"] == 0   # hot-row coordinates need the top bit
    small = (300, 200, 100, 50, 20, 10)  # 6 modes: no 16-bit kernels
    t6 = np.zeros((5, 6), dtype=np.uint32)
    h6 = capi.mttkrp_layout_build(t6, np.ones(5, np.float32), small, opts=dict(host_only=1))
    assert capi.mttkrp_layout_info(h6)["idx16_modes"] == 0
    t5 = np.zeros((5, 5), dtype=np.uint32)
    h5 = capi.mttkrp_layout_build(t5, np.ones(5, np.float32), small[:5], opts=dict(host_only=1))
    assert capi.mttkrp_layout_info(h5)["idx16_modes"] == 0b11111


def test_tuned_shape_options():
    """part_threads / part_gathers: validated, reported by layout_info where
    they apply (3-mode tensors without hot rows or steps) and ignored
    elsewhere; the shape autotuner's default candidates."""
    dims = (300, 200, 100)
    t = np.zeros((10, 3), dtype=np.uint32)
    v = np.ones(10, np.float32)
    for bad in (dict(part_threads=300), dict(part_threads=128), dict(part_gathers=3), dict(part_gathers=-1)):
        with pytest.raises(capi.MttkrpError):
            capi.mttkrp_layout_build(t, v, dims, opts=dict(host_only=1, **bad))
    h = capi.mttkrp_layout_build(t, v, dims, opts=dict(host_only=1, part_threads=1024, part_gathers=2))
    i = capi.mttkrp_layout_info(h)
    assert (i["wg_threads"], i["gathers_in_flight"]) == (1024, 2)
    h = capi.mttkrp_layout_build(t, v, dims, opts=dict(host_only=1, max_R=16))
    i = capi.mttkrp_layout_info(h)
    assert (i["wg_threads"], i["gathers_in_flight"]) == (512, 2)
    h = capi.mttkrp_layout_build(t, v, dims, opts=dict(host_only=1, part_threads=256, hot_rows=8))
    assert capi.mttkrp_layout_info(h)["wg_threads"] == 512           # hot rows: the default kernels
    t4 = np.zeros((10, 4), dtype=np.uint32)
    h = capi.mttkrp_layout_build(t4, v, dims + (50,), opts=dict(host_only=1, part_threads=1024))
    assert capi.mttkrp_layout_info(h)["wg_threads"] == 256           # 4 modes: the default kernels
    d3 = capi.mttkrp_batch_autotune_default_shapes(3)
    assert len(d3) == 36 and len(set(d3)) == 36
    assert {s[1] for s in d3} == {256, 512, 1024} and {s[2] for s in d3} == {2, 4}
    assert capi.mttkrp_batch_autotune_default_shapes(5) == [(p, 0, 0) for p in (1, 2, 4, 8, 16, 32)]


def test_degree_relabelling_host():
    """relabel=1 renumbers each mode by decreasing nonzero count (ties: lower
    index first) and then builds exactly the copies of the renumbered tensor."""
    rng = np.random.default_rng(12)
    dims = (300, 200, 100)
    base = np.stack([rng.zipf(1.5, 20000) % d for d in dims], axis=1).astype(np.uint32)
    idx = np.concatenate([base, base[:500]])            # duplicates too
    val = rng.random(idx.shape[0]).astype(np.float32)
    h = capi.mttkrp_layout_build(idx, val, dims, opts=dict(host_only=1, relabel=1))
    perms = [capi.mttkrp_layout_perm(h, m) for m in range(3)]
    remapped = np.stack([perms[m][idx[:, m]] for m in range(3)], axis=1).astype(np.uint32)
    for m, d in enumerate(dims):
        p = perms[m]
        assert np.array_equal(np.sort(p), np.arange(d, dtype=np.uint32))
        deg = np.bincount(idx[:, m], minlength=d)
        order = np.argsort(p)                            # old index at each new position
        assert np.all(np.diff(deg[order]) <= 0)
        ties = np.diff(deg[order]) == 0
        assert np.all(np.diff(order)[ties] > 0)          # equal counts keep the original order
    ref = capi.mttkrp_layout_build(remapped, val, dims, opts=dict(host_only=1))
    for n in range(3):
        a, b = capi.mttkrp_layout_view(h, n), capi.mttkrp_layout_view(ref, n)
        for k in ("val", "winfo", "row_id", "empty_rows", "src_pos"):
            assert np.array_equal(a[k], b[k]), (n, k)
        for x, y in zip(a["idx"], b["idx"]):
            assert np.array_equal(x, y)
    plain = capi.mttkrp_layout_build(idx, val, dims, opts=dict(host_only=1))
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_layout_perm(plain, 0)
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_layout_build(idx, val, dims, opts=dict(host_only=1, relabel=2))
