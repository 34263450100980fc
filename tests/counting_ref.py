"""Algorithm 2's last phase written out for tests: per source the distinct
endpoints of its walks with their counts, the top-k by count descending then
node id ascending, and the digest as the oracle defines it. Entries equal to
FPPR_NO_NODE (0xFFFFFFFF) are not endpoints and are not counted."""
import numpy as np

NO_NODE = 0xFFFFFFFF


def count_reference(ep, sources, k, R=None):
    """ep: [n_src, R] uint32. Returns (topk [n_src, k, 2], digest [n_src],
    n_distinct [n_src], counts [n_src, R, 2]: (t, count) by t, zero-padded)."""
    from oracle import oracle as O

    ep = np.asarray(ep, dtype=np.uint32)
    R = ep.shape[1] if R is None else R
    topk = np.zeros((len(sources), k, 2), dtype=np.uint32)
    topk[:, :, 0] = NO_NODE
    digest = np.zeros(len(sources), dtype=np.uint64)
    nd = np.zeros(len(sources), dtype=np.uint32)
    counts = np.zeros((len(sources), R, 2), dtype=np.uint32)
    for r, s in enumerate(sources):
        t, c = np.unique(ep[r][ep[r] != NO_NODE], return_counts=True)
        nd[r] = t.size
        counts[r, :t.size, 0] = t
        counts[r, :t.size, 1] = c
        order = np.lexsort((t, -c))[:k]
        topk[r, :order.size, 0] = t[order]
        topk[r, :order.size, 1] = c[order]
        d = 0
        for tt, cc in zip(t, c):
            d = (d + O.digest_term(int(s), int(tt), int(cc))) % 2**64
        digest[r] = d
    return topk, digest, nd, counts
