"""Ranking accuracy of estimated top-k lists against exact PPR (the accuracy
axis of Sec. 5.2: NDCG and MAP of the top-k nodes of each source).

For one source with exact scores pi (dense, FP64) and an estimated ranking
est (node ids, best first, at most k of them):
* ideal ranking: the k nodes with the largest pi, ties by smaller id;
* NDCG@k = DCG(est) / DCG(ideal), DCG(r) = sum_i pi[r_i] / log2(i + 2) over
  positions i = 0, 1, ... (gain = the exact score);
* AP@k = (1 / k) sum_i [est_i in ideal] * (hits among est_0..est_i) / (i + 1),
  MAP@k its mean over sources.
"""
from __future__ import annotations

import numpy as np


def ideal_topk(pi: np.ndarray, k: int) -> np.ndarray:
    """The k nodes with the largest score, ties by smaller id."""
    order = np.lexsort((np.arange(pi.shape[0]), -pi))
    return order[:k]


def ndcg_at_k(pi: np.ndarray, est: np.ndarray, k: int) -> float:
    est = np.asarray(est[:k], dtype=np.int64)
    disc = 1.0 / np.log2(np.arange(2, k + 2))
    ideal = ideal_topk(pi, k)
    idcg = float(np.sum(pi[ideal] * disc[: ideal.shape[0]]))
    if idcg == 0.0:
        return 1.0
    return float(np.sum(pi[est] * disc[: est.shape[0]])) / idcg


def ap_at_k(pi: np.ndarray, est: np.ndarray, k: int) -> float:
    est = np.asarray(est[:k], dtype=np.int64)
    rel = np.isin(est, ideal_topk(pi, k))
    hits = np.cumsum(rel)
    prec = hits / np.arange(1, est.shape[0] + 1)
    return float(np.sum(prec * rel)) / k
