"""Clustering quality against ground-truth labels: ACC, NMI and ARI as the
paper defines them for its quality tables (Appendix, evaluation metrics).

These are host-side evaluation measures (numpy, integer contingency counts,
FP64 logarithms), not part of the clustering path.

Reading of the printed NMI: the logarithm in its numerator lacks the factor
|U| (as printed the ratio |C*_i & C_j| / (|C*_i| |C_j|) is below one and the
measure is not normalised); the standard mutual information
sum n_ij log(|U| n_ij / (n_i n_j)) over the geometric mean of the two
entropies (the printed denominator) is used.
"""
from __future__ import annotations

import numpy as np


def contingency(truth, pred) -> np.ndarray:
    """table[i, j] = |C*_i & C_j| over the label values that occur (int64)."""
    truth = np.asarray(truth).ravel()
    pred = np.asarray(pred).ravel()
    if truth.shape != pred.shape:
        raise ValueError("label arrays differ in length")
    _, ti = np.unique(truth, return_inverse=True)
    _, pi = np.unique(pred, return_inverse=True)
    table = np.zeros((ti.max(initial=-1) + 1, pi.max(initial=-1) + 1), np.int64)
    np.add.at(table, (ti, pi), 1)
    return table


def acc(truth, pred) -> float:
    """Fraction of nodes whose predicted cluster, mapped one-to-one onto the
    ground-truth clusters by the Hungarian method (maximum total overlap),
    equals their ground-truth cluster."""
    from scipy.optimize import linear_sum_assignment

    t = contingency(truth, pred)
    if t.size == 0:
        return 1.0
    r, c = linear_sum_assignment(-t)
    return float(t[r, c].sum() / t.sum())


def nmi(truth, pred) -> float:
    """Mutual information of the two partitions over the geometric mean of
    their entropies; 1 when both are a single cluster (or identical)."""
    t = contingency(truth, pred).astype(np.float64)
    n = t.sum()
    if n == 0:
        return 1.0
    a = t.sum(axis=1)
    b = t.sum(axis=0)
    nz = t > 0
    mi = float(np.sum(t[nz] * np.log(n * t[nz] / np.outer(a, b)[nz])))
    ha = float(-np.sum(a * np.log(a / n)))
    hb = float(-np.sum(b * np.log(b / n)))
    if ha == 0.0 or hb == 0.0:
        return 1.0 if ha == hb else 0.0
    return float(mi / np.sqrt(ha * hb))


def _pairs(x) -> np.ndarray:
    x = np.asarray(x, np.float64)
    return x * (x - 1.0) / 2.0


def ari(truth, pred) -> float:
    """Hubert-Arabie adjusted Rand index from the pair counts of the
    contingency table; 1 for identical partitions."""
    t = contingency(truth, pred)
    n = int(t.sum())
    if n < 2:
        return 1.0
    s_ij = float(_pairs(t).sum())
    s_a = float(_pairs(t.sum(axis=1)).sum())
    s_b = float(_pairs(t.sum(axis=0)).sum())
    expected = s_a * s_b / (n * (n - 1) / 2.0)
    top = 0.5 * (s_a + s_b)
    if top == expected:
        return 1.0
    return (s_ij - expected) / (top - expected)


def report(truth, pred) -> dict:
    return {"acc": acc(truth, pred), "nmi": nmi(truth, pred), "ari": ari(truth, pred)}
