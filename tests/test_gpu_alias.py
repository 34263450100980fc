"""Alias tables built on the GPU (Sec. 2.2, Algorithm 1) are bit-identical,
row by row, to the oracle's integer alias tables: every row of graphs with
hub rows of thousands of edges, weights up to 2^31 and unit weights, both
layouts; on the R-MAT scale-20 graph, the largest rows and a sample of the
rest. The build time is printed."""
import sys

import numpy as np
import pytest

import synth
from oracle import alias as A

pytestmark = pytest.mark.gpu


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


def fetch(fp, G):
    import torch

    P, al = G.alias_tables()
    torch.cuda.synchronize()
    return P.cpu().numpy().view(np.uint64), al.cpu().numpy().view(np.uint32)


def rows_equal(g, P, al, rows):
    bad = []
    for v in rows:
        a, b = int(g.row_offsets[v]), int(g.row_offsets[v + 1])
        if a == b:
            continue
        Po, alo, _ = A.alias_table(g.w[a:b])
        if P[a:b].tolist() != Po or al[a:b].tolist() != alo:
            bad.append(int(v))
    return bad


CASES = {
    "chung-lu hubs": lambda: synth.chung_lu(3000, 60000, 2.05, 200, seed=5),
    "weights to 2^31": lambda: synth.chung_lu(2000, 30000, 2.2, 2_000_000_000, seed=6),
    "r-mat scale 12": lambda: synth.rmat(12, 16, .57, .19, .19, 10000, seed=7, zipf_s=1.2),
    "unit weights": lambda: synth.chung_lu(500, 4000, 2.1, 1, seed=8),
}


@pytest.mark.parametrize("name", list(CASES))
def test_alias_tables_equal_oracle(fp, name):
    g = CASES[name]()
    say(f"case: alias tables, {name}, n={g.n}, m={g.m}, max out-degree {g.degrees().max()}")
    layouts = [fp.FPPR_LAYOUT_WIDE]
    if int(g.w.max()) * int(g.degrees().max()) < 2**32:
        layouts.append(fp.FPPR_LAYOUT_NARROW)
    for lay in layouts:
        G = fp.Graph(g, layout=lay)
        P, al = fetch(fp, G)
        assert rows_equal(g, P, al, range(g.n)) == []
        # a second call on the same graph gives the same tables
        P2, al2 = fetch(fp, G)
        assert np.array_equal(P, P2) and np.array_equal(al, al2)


def test_alias_tables_scale20_sampled(fp):
    import torch

    g = synth.medium_graph()
    deg = g.degrees()
    say(f"case: alias tables, R-MAT scale 20, m={g.m}, max out-degree {deg.max()}")
    G = fp.Graph(g)
    G.alias_tables()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    P, al = G.alias_tables()
    t1.record()
    torch.cuda.synchronize()
    say(f"  alias tables of every row: {t0.elapsed_time(t1):.2f} ms")
    P = P.cpu().numpy().view(np.uint64)
    al = al.cpu().numpy().view(np.uint32)
    top = np.argsort(deg)[-64:]
    rng = np.random.default_rng(9)
    sample = rng.choice(np.flatnonzero(deg > 0), 4000, replace=False)
    assert rows_equal(g, P, al, np.concatenate([top, sample])) == []
