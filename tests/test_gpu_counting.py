"""Counting and top-k (Algorithm 2's last phase; Sec. 1 keeps only the
endpoints some walk reached) over crafted endpoint rows, through
fppr_aggregate, against the definition written out in counting_ref: rows
whose counts take many distinct values (the ranking hands out top-k
positions one count value at a time), rows of all-distinct endpoints, of a
single endpoint, of two, rows with FPPR_NO_NODE entries, ties across the
k-th position, node ids near 2^32; walk budgets on every side of the one-,
two- and four-register layouts of the per-source wave kernel (R <= 256) and
of the tile kernel above it."""
import sys

import numpy as np
import pytest

import counting_ref

pytestmark = pytest.mark.gpu

NO_NODE = counting_ref.NO_NODE


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fp():
    import torch

    from paper_1903_11749_amd import fppr

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fppr.lib()
    return fppr


def crafted_rows(R, n_rows, seed):
    """n_rows rows of R endpoints, each row one of the patterns above, its
    slots shuffled."""
    rng = np.random.default_rng(seed)
    rows = np.empty((n_rows, R), dtype=np.uint32)
    for r in range(n_rows):
        kind = r % 8
        base = int(rng.integers(0, 2**32 - 2**20))
        if kind == 0:  # counts 1, 2, ..., m (as many distinct values as fit), then singles
            vals = []
            c = 1
            while len(vals) + c <= R:
                vals += [base + c] * c
                c += 1
            vals += [base + 100000 + i for i in range(R - len(vals))]
        elif kind == 1:  # all distinct
            vals = list(base + rng.choice(1 << 20, R, replace=False))
        elif kind == 2:  # one endpoint
            vals = [base] * R
        elif kind == 3:  # two endpoints
            cut = int(rng.integers(1, R)) if R > 1 else 1
            vals = [base] * cut + [base + 7] * (R - cut)
        elif kind == 4:  # FPPR_NO_NODE entries among the endpoints
            vals = list(base + rng.integers(0, max(2, R // 3), R))
            holes = rng.random(R) < 0.3
            vals = [NO_NODE if h else v for v, h in zip(vals, holes)]
        elif kind == 5:  # many ties at count 2 (more pairs than k)
            vals = [base + i // 2 for i in range(R)]
        elif kind == 6:  # ids near 2^32 (FPPR_NO_NODE excluded)
            vals = list(np.uint64(2**32 - 2) - rng.integers(0, max(2, R // 2), R).astype(np.uint64))
        else:  # a few heavy endpoints over light ones, like walks from a node
            heavy = rng.integers(0, 6, R)
            vals = [base + int(h) if rng.random() < 0.5 else base + 1000 + int(rng.integers(0, 4 * R)) for h in heavy]
        row = np.array(vals, dtype=np.uint64).astype(np.uint32)
        rows[r] = row[rng.permutation(R)]
    return rows


@pytest.mark.parametrize("R", [1, 17, 63, 64, 65, 100, 128, 129, 200, 256, 300])
def test_crafted_counting(fp, R):
    import torch

    rows = crafted_rows(R, 96, 1000 + R)
    n = rows.shape[0]
    src = np.arange(5, 5 + 3 * n, 3, dtype=np.uint32)
    dev = torch.from_numpy(rows.reshape(-1).view(np.int32)).cuda()
    for k in sorted({1, min(16, R), min(32, R), R}):
        say(f"case: crafted rows R={R} k={k}")
        tk, dg, nd, cn = counting_ref.count_reference(rows, src, k)
        for counts in (True, False):
            o = fp.count(dev, R, k, sources=src, counts=counts)
            torch.cuda.synchronize()
            assert np.array_equal(o.topk.cpu().numpy().view(np.uint32).reshape(n, k, 2), tk)
            assert np.array_equal(o.digest.cpu().numpy().view(np.uint64), dg)
            if counts:
                assert np.array_equal(o.n_distinct.cpu().numpy().view(np.uint32), nd)
                assert np.array_equal(o.counts.cpu().numpy().view(np.uint32).reshape(n, R, 2), cn)
