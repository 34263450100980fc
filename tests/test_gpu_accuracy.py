"""Accuracy of the GPU's top-k lists against exact PPR (the paper's accuracy
axis, Sec. 5.2, on a synthetic graph instead of its datasets): NDCG@k and
MAP@k over every source, at walk budgets around the one Definition 1's
guarantee gives for the paper's default epsilon = delta = 0.5, p_f = 1/n.

* Plain walks estimate the exact PPR: accuracy grows with R towards 1.
* Stitched walks estimate the pool-conditioned chain (the pool is a fixed
  sample of short walks): against that chain accuracy grows towards 1 as
  well, while against the exact PPR it levels off at the pool's O(1/K) bias,
  which a larger pool shrinks.
The numbers are printed (and quoted with the design notes)."""
import sys

import numpy as np
import pytest

import synth
from exact_ppr import chain_exact, ppr_exact
from ranking import ap_at_k, ndcg_at_k

pytestmark = pytest.mark.gpu

K = 16


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


def mean_scores(pi, topk, n):
    nd, ap = [], []
    for s in range(pi.shape[0]):
        est = topk[s, :, 0]
        est = est[est < n]
        nd.append(ndcg_at_k(pi[s], est, K))
        ap.append(ap_at_k(pi[s], est, K))
    return float(np.mean(nd)), float(np.mean(ap))


def test_topk_accuracy_against_exact_ppr(fp):
    import torch

    g = synth.small_graph()
    alpha, S, L = 0.2, 8, 3
    src = np.arange(g.n)
    pi = ppr_exact(g.n, g.row_offsets, g.col, g.w, alpha, src)
    small = np.flatnonzero((g.degrees() >= 1) & (g.degrees() <= S))
    R_g = fp.fppr_walks_for_guarantee(0.5, 0.5, 1.0 / g.n)
    say(f"case: accuracy, n={g.n}, alpha={alpha}, guaranteed R={R_g}")
    budgets = (max(K, R_g // 4), R_g, 4 * R_g)

    def topk_of(G, R, stitch):
        out = fp.run(G, alpha, R, 41, topk=K, stitch=stitch, counts=False, stats=False)
        torch.cuda.synchronize()
        return out.topk.cpu().numpy().view(np.uint32).reshape(g.n, K, 2)

    G = fp.Graph(g)
    plain = []
    for R in budgets:
        nd, mp = mean_scores(pi, topk_of(G, R, False), g.n)
        plain.append((nd, mp))
        say(f"  plain     R={R:5d}  vs exact: NDCG@{K}={nd:.4f} MAP@{K}={mp:.4f}")
    assert plain[0][0] < plain[1][0] < plain[2][0] and plain[0][1] < plain[2][1]
    assert plain[2][0] > 0.95

    last_exact = {}
    for Kp in (16, 64):
        G.build_pool(S=S, L=L, K=Kp, alpha=alpha, seed=5)
        chain = chain_exact(g.n, g.row_offsets, g.col, g.w, alpha, src, small, G.export_pool(), Kp)
        vs_chain = []
        for R in budgets:
            tk = topk_of(G, R, True)
            nd_c, mp_c = mean_scores(chain, tk, g.n)
            nd_e, mp_e = mean_scores(pi, tk, g.n)
            vs_chain.append(nd_c)
            last_exact[Kp] = nd_e
            say(f"  stitched K={Kp:3d} R={R:5d}  vs chain: NDCG@{K}={nd_c:.4f} MAP@{K}={mp_c:.4f}"
                f"   vs exact: NDCG@{K}={nd_e:.4f} MAP@{K}={mp_e:.4f}")
        assert vs_chain[0] < vs_chain[1] < vs_chain[2] and vs_chain[2] > 0.95
    assert last_exact[64] > last_exact[16], "a larger pool must bring stitched walks closer to exact PPR"


def test_topk_accuracy_at_depth(fp):
    """The paper's accuracy axis at its depth (Sec. 5.2: NDCG and MAP of the
    top-1000) and defaults (epsilon = delta = alpha = 0.5, p_f = 1/n), on
    R-MAT scale 17 (131,072 nodes, 2.1M edges, the scale-24 workload's
    skew and weight law): 64 sampled sources with out-edges, exact PPR in
    FP64, GPU top-k lists at R_g, 4 R_g and 16 R_g walks (R_g from
    Definition 1's guarantee), plain walks against exact PPR and stitched
    walks (S = 32, L = 3, K = 64) against their pool's chain and against
    exact PPR, at k = 16, 64 and 1000."""
    import torch

    from exact_ppr import chain_exact

    alpha = 0.5
    g = synth.rmat(17, 16, 0.57, 0.19, 0.19, wmax=10000, seed=1017, weight_law="zipf", zipf_s=1.2)
    rng = np.random.default_rng(5)
    src = np.sort(rng.choice(np.flatnonzero(g.degrees() > 0), 64, replace=False)).astype(np.uint32)
    R_g = fp.fppr_walks_for_guarantee(0.5, 0.5, 1.0 / g.n)
    say(f"case: accuracy at depth, n={g.n}, m={g.m}, alpha={alpha}, guaranteed R={R_g}, 64 sources")
    pi = ppr_exact(g.n, g.row_offsets, g.col, g.w, alpha, src)
    say("  exact PPR done")
    G = fp.Graph(g)
    G.build_pool(S=32, L=3, K=64, alpha=alpha, seed=7)
    small = np.flatnonzero((g.degrees() >= 1) & (g.degrees() <= 32))
    chain = chain_exact(g.n, g.row_offsets, g.col, g.w, alpha, src, small, G.export_pool(), 64)
    say("  pool chain done")

    def scores(ref, topk, k):
        nd, ap = [], []
        for r in range(ref.shape[0]):
            est = topk[r, :, 0]
            est = est[est < g.n]
            nd.append(ndcg_at_k(ref[r], est, k))
            ap.append(ap_at_k(ref[r], est, k))
        return float(np.mean(nd)), float(np.mean(ap))

    table = {}
    for stitch in (False, True):
        for R in (R_g, 4 * R_g, 16 * R_g):
            kk = min(1000, R)
            out = fp.run(G, alpha, R, 41, sources=src, topk=kk, stitch=stitch, counts=False, stats=False)
            torch.cuda.synchronize()
            tk = out.topk.cpu().numpy().view(np.uint32).reshape(src.size, kk, 2)
            for k in (16, 64, 1000):
                table[(stitch, R, k, "exact")] = scores(pi, tk, k)
                if stitch:
                    table[(stitch, R, k, "chain")] = scores(chain, tk, k)
            line = "  ".join(f"@{k} NDCG {table[(stitch, R, k, 'exact')][0]:.4f} MAP {table[(stitch, R, k, 'exact')][1]:.4f}"
                             for k in (16, 64, 1000))
            say(f"  {'stitched' if stitch else 'plain   '} R={R:5d} vs exact: {line}")
            if stitch:
                line = "  ".join(f"@{k} NDCG {table[(stitch, R, k, 'chain')][0]:.4f} MAP {table[(stitch, R, k, 'chain')][1]:.4f}"
                                 for k in (16, 64, 1000))
                say(f"           R={R:5d} vs chain: {line}")
    for k in (16, 64, 1000):
        nd = [table[(False, R, k, "exact")][0] for R in (R_g, 4 * R_g, 16 * R_g)]
        assert nd[0] < nd[1] < nd[2], (k, nd)
        ndc = [table[(True, R, k, "chain")][0] for R in (R_g, 4 * R_g, 16 * R_g)]
        assert ndc[0] < ndc[1] < ndc[2], (k, ndc)
    assert table[(False, 16 * R_g, 16, "exact")][0] > 0.95
    assert table[(True, 16 * R_g, 16, "chain")][0] > 0.95
