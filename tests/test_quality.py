"""ACC, NMI and ARI (Appendix, evaluation metrics) pinned against scikit-learn's
independent implementations, brute force over label maps, and their
invariances; the target-V view of a planted graph."""
import itertools

import numpy as np
import pytest
from sklearn import metrics as skm

import abg_synth as synth
from paper_2405_11922_amd import quality


def _pairs(seed, n, ka, kb):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, ka, n)
    b = np.where(rng.random(n) < 0.6, a % kb, rng.integers(0, kb, n))
    return a, b


@pytest.mark.parametrize("seed,n,ka,kb", [(0, 50, 3, 3), (1, 400, 5, 4), (2, 1000, 7, 9), (3, 30, 1, 4)])
def test_against_sklearn(seed, n, ka, kb):
    a, b = _pairs(seed, n, ka, kb)
    assert quality.nmi(a, b) == pytest.approx(
        skm.normalized_mutual_info_score(a, b, average_method="geometric"), abs=1e-12)
    assert quality.ari(a, b) == pytest.approx(skm.adjusted_rand_score(a, b), abs=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_acc_is_the_best_one_to_one_map(seed):
    """Brute force over every injective map of predicted onto true labels."""
    a, b = _pairs(seed, 60, 4, 4)
    best = 0
    for perm in itertools.permutations(range(4)):
        best = max(best, int(np.sum(np.asarray(perm)[b] == a)))
    assert quality.acc(a, b) == pytest.approx(best / a.size, abs=0)


def test_special_values_and_invariances():
    a, b = _pairs(7, 300, 5, 5)
    perm = np.array([3, 0, 4, 1, 2])
    r = quality.report(a, b)
    r2 = quality.report(a, perm[b])  # relabelling the prediction changes nothing
    for key in r:
        assert r[key] == pytest.approx(r2[key], abs=1e-12)
    assert quality.report(a, perm[a]) == pytest.approx({"acc": 1.0, "nmi": 1.0, "ari": 1.0})
    # symmetric measures
    assert quality.nmi(a, b) == pytest.approx(quality.nmi(b, a), abs=1e-12)
    assert quality.ari(a, b) == pytest.approx(quality.ari(b, a), abs=1e-12)
    # one predicted cluster against k equal true ones: ACC = 1/k, NMI = 0, ARI = 0
    t = np.repeat(np.arange(4), 25)
    assert quality.acc(t, np.zeros_like(t)) == pytest.approx(0.25)
    assert quality.nmi(t, np.zeros_like(t)) == 0.0
    assert quality.ari(t, np.zeros_like(t)) == pytest.approx(0.0, abs=1e-15)


def test_target_v_view():
    g = synth.planted_abg(300, 200, 2000, 4, 8, seed=3)
    xv = synth.planted_attributes(g.labels_v, 32, seed=3)
    assert xv.shape == (200, 32) and xv.dtype == np.float32
    h = synth.target_v(g, xv)
    assert (h.n_u, h.n_v, h.d_u) == (200, 300, 32)
    assert np.array_equal(h.edge_u, g.edge_v) and np.array_equal(h.edge_v, g.edge_u)
    assert np.array_equal(h.labels_u, g.labels_v)
    # the planted means separate V's clusters: nearest mean recovers them
    mu = np.stack([xv[g.labels_v == c].mean(0) for c in range(4)])
    near = np.argmin(((xv[:, None, :] - mu[None]) ** 2).sum(-1), axis=1)
    assert quality.acc(g.labels_v, near) > 0.9
