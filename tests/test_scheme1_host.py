"""Load-balancing scheme 1 (Sec. III-B) on the host, no GPU: the LPT
partitioner against brute-force optima (the 4/3 bound the paper quotes is
Graham's bound for longest-processing-time-first, (4/3 - 1/(3 kappa)) OPT),
the cyclic dealing that the bound does not hold for, and the regrouped mode
copies of a MTTKRP_PART_ROWS_LPT host-only layout."""

import itertools

import numpy as np
import pytest

import workloads
from paper_2503_18198_amd import capi


def brute_force_opt(loads, kappa):
    best = None
    for assign in itertools.product(range(kappa), repeat=len(loads)):
        ms = np.zeros(kappa, dtype=np.int64)
        for r, p in enumerate(assign):
            ms[p] += loads[r]
        m = int(ms.max())
        best = m if best is None else min(best, m)
    return best


def cyclic_makespan(loads, kappa):
    """Rows sorted by decreasing load, dealt to partitions 0, 1, ..., kappa-1, 0, ..."""
    order = sorted(range(len(loads)), key=lambda r: (-loads[r], r))
    ms = np.zeros(kappa, dtype=np.int64)
    for i, r in enumerate(order):
        ms[i % kappa] += loads[r]
    return int(ms.max())


@pytest.mark.parametrize("kappa", [2, 3, 4])
def test_lpt_within_graham_bound_of_brute_force(kappa):
    rng = np.random.default_rng(kappa)
    worst = 0.0
    for trial in range(60):
        n = int(rng.integers(1, 9 if kappa <= 3 else 8))
        loads = rng.integers(1, 40, size=n).astype(np.uint64)
        part, pl = capi.mttkrp_lpt_partition(loads, kappa)
        assert part.shape == (n,) and np.all(part < kappa)
        # the reported loads are the sums of the assignment
        assert np.array_equal(pl, np.bincount(part, weights=loads, minlength=kappa).astype(np.uint64))
        opt = brute_force_opt([int(x) for x in loads], kappa)
        ratio = int(pl.max()) / opt
        worst = max(worst, ratio)
        assert ratio <= 4 / 3 - 1 / (3 * kappa) + 1e-12, (loads, part, pl, opt)
    print(f"kappa {kappa}: worst LPT / OPT {worst:.3f}")


def test_graham_tight_instance_and_cyclic_counterexample():
    # The classic tight instance for kappa = 2: loads {3, 3, 2, 2, 2}; OPT = 6 ({3,3}, {2,2,2}),
    # LPT = 7 = (4/3 - 1/6) * 6.
    part, pl = capi.mttkrp_lpt_partition([3, 3, 2, 2, 2], 2)
    assert int(pl.max()) == 7 and brute_force_opt([3, 3, 2, 2, 2], 2) == 6
    # Cyclic dealing of sorted rows breaks the bound: {2, 1, 1} on 2 partitions
    # gives {3, 1}, 1.5 x the optimum {2, 2}; LPT finds the optimum.
    assert cyclic_makespan([2, 1, 1], 2) == 3
    part, pl = capi.mttkrp_lpt_partition([2, 1, 1], 2)
    assert sorted(pl.tolist()) == [2, 2]


def test_lpt_tie_rules_and_degenerate_sizes():
    # equal loads: rows in index order, each to the lowest least-loaded partition
    part, pl = capi.mttkrp_lpt_partition([5, 5, 5, 5], 2)
    assert part.tolist() == [0, 1, 0, 1] and pl.tolist() == [10, 10]
    part, pl = capi.mttkrp_lpt_partition([], 3)
    assert part.size == 0 and pl.tolist() == [0, 0, 0]
    part, pl = capi.mttkrp_lpt_partition([7, 1], 5)     # more partitions than rows
    assert part.tolist() == [0, 1] and pl.tolist() == [7, 1, 0, 0, 0]
    with pytest.raises(capi.MttkrpError):
        capi.mttkrp_lpt_partition([1, 2], 0)


@pytest.mark.parametrize("dims,nnz,kappa,dist", [((300, 200, 100), 20_000, 16, "zipf"),
                                                  ((50, 40, 30, 20), 3_000, 7, "uniform"),
                                                  ((1, 60, 70), 500, 4, "uniform"),
                                                  ((400, 300, 200), 33, 256, "zipf")])
def test_lpt_layout_holds_whole_rows_in_lpt_order(dims, nnz, kappa, dist):
    """Every partition of every scheme-1 mode copy holds whole output rows in
    increasing row order, starts at a multiple of 32, has the LPT load of the
    row degrees, and each row carries exactly the nonzeros (same order,
    coordinates and values) of the default copy's row."""
    t = workloads.random_tensor(dims, nnz, dist=dist, s=1.2 if dist == "zipf" else None, seed=3)
    plain = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(host_only=1))
    lpt = capi.mttkrp_layout_build(t.idx, t.val, t.dims,
                                   opts=dict(host_only=1, partitioner=capi.MTTKRP_PART_ROWS_LPT, lpt_parts=kappa))
    N = len(dims)
    for n in range(N):
        a = capi.mttkrp_layout_view(plain, n)
        b = capi.mttkrp_layout_view(lpt, n)
        pr = b["part_range"]
        assert pr.shape == (kappa, 2)
        assert np.all(pr[:, 0] % 32 == 0) and np.all(np.diff(pr[:, 0].astype(np.int64)) >= 0)
        assert int(pr[:, 1].sum()) == t.nnz
        # the plain copy's rows, with their extents
        starts = [k for k in range(a["nnz"]) if (a["winfo"][2 * (k // 32)] >> (k % 32)) & 1]
        ext = dict(zip(a["row_id"].tolist(), zip(starts, starts[1:] + [a["nnz"]])))
        deg = np.array([ext[r][1] - ext[r][0] for r in a["row_id"].tolist()], dtype=np.uint64)
        want_part, want_load = capi.mttkrp_lpt_partition(deg, kappa)
        assert np.array_equal(pr[:, 1], want_load)
        owner = dict(zip(a["row_id"].tolist(), want_part.tolist()))
        # walk the scheme-1 copy partition by partition
        ords = iter(range(b["nrows_nz"]))
        bits = lambda k: (b["winfo"][2 * (k // 32)] >> (k % 32)) & 1
        for p in range(kappa):
            lo, cnt = int(pr[p, 0]), int(pr[p, 1])
            k, prev = lo, -1
            while k < lo + cnt:
                assert bits(k) == 1, f"mode {n} partition {p}: no row starts at {k}"
                r = int(b["row_id"][next(ords)])
                assert r > prev and owner[r] == p
                prev = r
                s0, s1 = ext[r]
                L = s1 - s0
                assert k + L <= lo + cnt
                for j in range(N - 1):
                    assert np.array_equal(b["idx"][j][k:k + L], a["idx"][j][s0:s1])
                assert np.array_equal(b["val"][k:k + L], a["val"][s0:s1])
                assert np.array_equal(b["src_pos"][k:k + L], a["src_pos"][s0:s1])
                assert not any(bits(q) for q in range(k + 1, k + L))
                k += L
        assert next(ords, None) is None
        assert np.array_equal(b["empty_rows"], a["empty_rows"])
    assert capi.mttkrp_layout_info(lpt)["lpt_parts"] == kappa
