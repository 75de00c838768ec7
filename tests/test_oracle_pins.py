"""The FP64 oracle against independent pins, and proof that the pins bite.

Every pin in ``pins.py`` must pass for the oracle; for each planted mistake
(a copy of the oracle's sum with one plausible error) at least one pin must
fail.  The planted copies live here, on the CPU; the oracle itself is never
modified.
"""

import numpy as np
import pytest

import oracle
from tests import pins


def oracle_f(idx, val, dims, factors, mode):
    return oracle.mttkrp(idx, val, dims, factors, mode)


def oracle_f_threads(idx, val, dims, factors, mode):
    return oracle.mttkrp(idx, val, dims, factors, mode, threads=3)


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_oracle_passes_pin(pin):
    pin(oracle_f)


@pytest.mark.parametrize("pin", [pins.pin_dense_khatri_rao, pins.pin_invariants, pins.pin_large_dense_and_slices],
                         ids=lambda p: p.__name__)
def test_threaded_oracle_passes_pin(pin):
    pin(oracle_f_threads)


def test_large_pin_reaches_threaded_branch():
    """The large pin's tensors are above the oracle's serial cut-off (4,096
    nonzeros), so with threads > 1 they run the thread-private branch; a
    planted mistake confined to that branch (one thread's slice dropped) is
    caught by it."""
    def drop_last_thread_slice(idx, val, dims, factors, mode):
        idx = np.asarray(idx)
        if idx.shape[0] >= 4096:
            keep = idx.shape[0] - idx.shape[0] // 3
            idx, val = idx[:keep], np.asarray(val)[:keep]
        return oracle.mttkrp(idx, val, dims, factors, mode, threads=3)
    with pytest.raises(AssertionError):
        pins.pin_large_dense_and_slices(drop_last_thread_slice)


def test_threaded_matches_serial_large():
    rng = np.random.default_rng(7)
    dims = (300, 200, 100)
    idx, val = pins.rand_coo(rng, dims, 20000)
    A = pins.rand_factors(rng, dims, 8)
    for n in range(3):
        a = oracle.mttkrp(idx, val, dims, A, n, threads=1)
        b = oracle.mttkrp(idx, val, dims, A, n, threads=4)
        assert pins.rel_fro(b, a) <= 1e-14


def test_rows_subset_matches_full():
    rng = np.random.default_rng(8)
    dims = (50, 40, 30)
    idx, val = pins.rand_coo(rng, dims, 3000)
    A = pins.rand_factors(rng, dims, 6)
    for n in range(3):
        full = oracle.mttkrp(idx, val, dims, A, n)
        rows = np.array([0, 5, 5, dims[n] - 1, 17], dtype=np.uint32)
        sub = oracle.mttkrp_rows(idx, val, dims, A, n, rows)
        assert np.array_equal(sub, full[rows.astype(np.int64)])


def test_oracle_rejects_out_of_range_index():
    idx = np.array([[0, 0, 5]], dtype=np.uint32)
    A = [np.ones((2, 2)), np.ones((2, 2)), np.ones((5, 2))]
    with pytest.raises(ValueError):
        oracle.mttkrp(idx, np.ones(1), (2, 2, 5), A, 0)


def test_empty_tensor_gives_zero():
    idx = np.zeros((0, 3), dtype=np.uint32)
    A = [np.ones((3, 2)), np.ones((4, 2)), np.ones((5, 2))]
    out = oracle.mttkrp(idx, np.zeros(0), (3, 4, 5), A, 1)
    assert out.shape == (4, 2) and not out.any()


# ------------------------------------------------------------ planted mistakes
def _planted(kind):
    def f(idx, val, dims, factors, mode):
        idx = np.asarray(idx, dtype=np.int64)
        val = np.asarray(val, dtype=np.float64)
        N = len(dims)
        R = next(np.asarray(a).shape[1] for m, a in enumerate(factors) if m != mode)
        out = np.zeros((dims[mode], R))
        inputs = [m for m in range(N) if m != mode]
        for k in range(idx.shape[0]):
            t = np.full(R, val[k])
            if kind == "val_squared":
                t = t * val[k]
            if kind == "ignore_val":
                t = np.ones(R)
            for j, m in enumerate(inputs):
                if kind == "drop_term" and j == len(inputs) - 1:
                    continue
                row = idx[k, m]
                fac = np.asarray(factors[m], dtype=np.float64)
                if kind == "wrong_index" and j == 0:
                    row = idx[k, mode] % dims[m]
                if kind == "wrong_operand" and j == 0:
                    other = inputs[-1]
                    fac = np.asarray(factors[other], dtype=np.float64)
                    row = idx[k, other]
                if kind == "reversed_columns" and j == 0:
                    t = t * fac[row, ::-1]
                    continue
                t = t * fac[row]
            if kind == "extra_term":
                t = t * np.asarray(factors[(mode + 1) % N], dtype=np.float64)[idx[k, (mode + 1) % N]]
            dst = idx[k, mode]
            if kind == "row_shift":
                dst = (dst + 1) % dims[mode]
            if kind == "first_wins" and out[dst].any():
                continue
            out[dst] += t
        return out
    return f


PLANTED = ["drop_term", "wrong_index", "wrong_operand", "ignore_val", "val_squared", "row_shift",
           "extra_term", "reversed_columns", "first_wins"]


def test_correct_planted_copy_passes():
    """The planted-mistake scaffold without a mistake passes every pin, so the
    failures below come from the mistakes and not from the scaffold."""
    f = _planted("none")
    for pin in pins.ALL_PINS:
        pin(f)


@pytest.mark.parametrize("kind", PLANTED)
def test_pins_catch_planted_mistake(kind):
    f = _planted(kind)
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(f)
        except (AssertionError, IndexError, ValueError):
            failed.append(pin.__name__)
    assert failed, f"no pin caught planted mistake {kind!r}"
