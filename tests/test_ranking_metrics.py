"""Pins of the ranking metrics used by the accuracy study (CPU)."""
import math

import numpy as np

from ranking import ap_at_k, ideal_topk, ndcg_at_k


def test_ideal_ranking_scores_one():
    pi = np.array([0.1, 0.4, 0.0, 0.3, 0.2])
    assert list(ideal_topk(pi, 3)) == [1, 3, 4]
    assert ndcg_at_k(pi, ideal_topk(pi, 3), 3) == 1.0
    assert ap_at_k(pi, ideal_topk(pi, 3), 3) == 1.0


def test_ties_break_by_smaller_id():
    pi = np.array([0.2, 0.5, 0.2, 0.1])
    assert list(ideal_topk(pi, 3)) == [1, 0, 2]


def test_hand_computed_values():
    pi = np.array([0.1, 0.4, 0.0, 0.3, 0.2])
    est = np.array([3, 1, 2])  # swapped top two, third is irrelevant
    dcg = 0.3 / math.log2(2) + 0.4 / math.log2(3) + 0.0 / math.log2(4)
    idcg = 0.4 / math.log2(2) + 0.3 / math.log2(3) + 0.2 / math.log2(4)
    assert abs(ndcg_at_k(pi, est, 3) - dcg / idcg) < 1e-15
    # relevant = {1, 3, 4}: hits at positions 0, 1 -> (1/1 + 2/2) / 3
    assert abs(ap_at_k(pi, est, 3) - 2.0 / 3.0) < 1e-15
    # nothing relevant
    assert ap_at_k(pi, np.array([0, 2]), 2) == 0.0
