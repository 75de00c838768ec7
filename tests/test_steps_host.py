"""Hot-steps copies on the host, no GPU (host-only layouts with hot_steps=1):
every step lies in one output row; each row holds exactly its nonzeros,
ordered by hot/cold class (reflected Gray order of the cold-input bits) and,
inside a class, in the nonzero-ordered copy's order; padding entries (value
0, the zero row kHotBit | nhot) only fill each row's last step; the hot rows
are the most gathered rows of each input."""

import numpy as np
import pytest

import workloads
from paper_2503_18198_amd import capi

HOT = np.uint32(0x80000000)


def gray_rank(c):
    r = c
    sh = 1
    while sh < 32:
        r ^= r >> sh
        sh <<= 1
    return r


def step_rows(v):
    """Output row of every step, from the per-32-step row-start bits and ordinals."""
    ns = v["nsteps"]
    w = v["winfo"].reshape(-1, 2)
    rows = np.empty(ns, dtype=np.int64)
    for s in range(ns):
        if s % 32 == 0:
            o = int(w[s // 32, 1])
        elif (w[s // 32, 0] >> (s % 32)) & 1:
            o += 1
        rows[s] = v["row_id"][o]
    starts = np.array([(w[s // 32, 0] >> (s % 32)) & 1 for s in range(ns)], dtype=bool)
    return rows, starts


@pytest.mark.parametrize("dims,nnz,R,dist", [((400, 300, 200), 30_000, 32, "zipf"),
                                             ((300, 200, 100, 30), 20_000, 16, "zipf"),
                                             ((50, 40, 30), 3_000, 64, "uniform")])
def test_step_copy_rows_classes_and_padding(dims, nnz, R, dist):
    t = workloads.random_tensor(dims, nnz, dist=dist, s=1.2 if dist == "zipf" else None, seed=4)
    N = len(dims)
    plain = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(host_only=1))
    st = capi.mttkrp_layout_build(t.idx, t.val, t.dims, opts=dict(host_only=1, hot_steps=1, max_R=R))
    for n in range(N):
        a = capi.mttkrp_layout_view(plain, n)
        b = capi.mttkrp_layout_view(st, n)
        P = b["step_entries"]
        nhot = b["nhot"]
        assert P == 64 // (R // 4) and nhot >= 1
        ns = b["nsteps"]
        assert b["nnz_pad"] == (ns + 31) // 32 * 32 * P
        pos = lambda s, e: (s // 32) * 32 * P + e * 32 + s % 32
        rows, starts = step_rows(b)
        # hot rows: the highest-degree rows of each input mode
        for j, m in enumerate(b["in_modes"]):
            deg = np.bincount(t.idx[:, m].astype(np.int64), minlength=dims[m])
            hot_set = np.unique(b["idx"][j][(b["idx"][j] & HOT) != 0] & ~HOT)
            hot_set = hot_set[hot_set < nhot]
            hr = np.unique(b["hot_rows"][j][hot_set])
            if hr.size:
                cold = np.setdiff1d(np.arange(dims[m]), hr)
                assert deg[hr].min() >= (deg[cold].max() if cold.size else 0), "hot rows are the most gathered"
        # the plain copy's rows with their extents
        astarts = [k for k in range(a["nnz"]) if (a["winfo"][2 * (k // 32)] >> (k % 32)) & 1]
        ext = dict(zip(a["row_id"].tolist(), zip(astarts, astarts[1:] + [a["nnz"]])))

        def decode(raw, j):
            raw = raw.astype(np.int64)
            out = raw.copy()
            h = (raw & 0x80000000) != 0
            out[h] = b["hot_rows"][j][raw[h] & 0x7FFFFFFF] if nhot else raw[h]
            return out, h

        s = 0
        seen_rows = []
        while s < ns:
            assert starts[s]
            r = int(rows[s])
            s1 = s + 1
            while s1 < ns and not starts[s1]:
                s1 += 1
            assert np.all(rows[s:s1] == r)
            ent = [pos(q, e) for q in range(s, s1) for e in range(P)]
            vals = b["val"][ent]
            coords = [b["idx"][j][ent] for j in range(N - 1)]
            pad = coords[0] == (HOT | np.uint32(nhot))
            for j in range(1, N - 1):
                assert np.array_equal(pad, coords[j] == (HOT | np.uint32(nhot)))
            assert np.all(vals[pad] == 0)
            npad = int(pad.sum())
            assert npad < P and not pad[: len(ent) - npad].any(), "padding only at the row's end"
            real = len(ent) - npad
            s0, s1r = ext[r]
            assert real == s1r - s0
            # same nonzeros: a class-sorted stable permutation of the plain row
            # (the plain copy is built without hot sets: classify by the step copy's tables)
            cls_plain = np.zeros(real, dtype=np.int64)
            plain_coords = [a["idx"][j][s0:s1r].astype(np.int64) for j in range(N - 1)]
            for j in range(N - 1):
                hot_set = set(b["hot_rows"][j][:nhot].tolist())
                cold = np.array([c not in hot_set for c in plain_coords[j]], dtype=np.int64)
                cls_plain |= cold << j
            order = np.argsort(np.array([gray_rank(int(c)) for c in cls_plain]), kind="stable")
            for j in range(N - 1):
                got, _ = decode(coords[j][:real], j)
                assert np.array_equal(got, plain_coords[j][order]), f"mode {n} row {r} input {j}"
            assert np.array_equal(vals[:real], a["val"][s0:s1r][order])
            seen_rows.append(r)
            s = s1
        assert seen_rows == a["row_id"].tolist()
        assert np.array_equal(b["empty_rows"], a["empty_rows"])
    assert capi.mttkrp_layout_info(st)["step_entries"] == 64 // (R // 4)
