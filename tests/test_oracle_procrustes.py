"""Pins of the oracle's Procrustes form of the NCI Phi update (Section 3.4:
the orthogonal Phi minimising ||Ups Phi - Y||), independent of the SVD it is
computed with: brute force over the orthogonal 2 x 2 matrices, optimality
against random orthogonal matrices, the exact answer for a rotated indicator
matrix, and the partial isometry for an empty cluster."""
import numpy as np
import pytest

import oracle


def _indicator(labels, k):
    n = labels.size
    y = np.zeros((n, k))
    y[np.arange(n), labels] = 1.0
    cnt = y.sum(0)
    y[:, cnt > 0] /= np.sqrt(cnt[cnt > 0])
    return y


def _loss(ups, phi, y):
    return float(np.linalg.norm(ups @ phi - y))


def test_brute_force_k2():
    """k = 2: every orthogonal matrix is a rotation or a reflection by an
    angle; a fine scan of both finds the same minimiser."""
    rng = np.random.default_rng(0)
    ups = np.abs(rng.standard_normal((60, 2)))
    y = _indicator(rng.integers(0, 2, 60), 2)
    phi = oracle.polar_factor(ups.T @ y)
    th = np.linspace(0.0, 2 * np.pi, 200_001)
    c, s = np.cos(th), np.sin(th)
    best = np.inf
    for refl in (1.0, -1.0):
        # Phi = [[c, -refl s], [s, refl c]]
        p00, p01, p10, p11 = c, -refl * s, s, refl * c
        r0 = ups[:, :1] * p00 + ups[:, 1:] * p10 - y[:, :1]
        r1 = ups[:, :1] * p01 + ups[:, 1:] * p11 - y[:, 1:]
        loss = np.sqrt((r0 ** 2).sum(0) + (r1 ** 2).sum(0))
        i = int(np.argmin(loss))
        if loss[i] < best:
            best = loss[i]
            arg = np.array([[p00[i], p01[i]], [p10[i], p11[i]]])
    assert _loss(ups, phi, y) <= best + 1e-12
    assert np.max(np.abs(phi - arg)) < 1e-4


@pytest.mark.parametrize("k", [3, 6, 11])
def test_orthogonal_and_optimal(k):
    rng = np.random.default_rng(k)
    ups = np.abs(rng.standard_normal((200, k)))
    y = _indicator(rng.integers(0, k, 200), k)
    phi = oracle.polar_factor(ups.T @ y)
    assert np.allclose(phi.T @ phi, np.eye(k), atol=1e-12)
    f = _loss(ups, phi, y)
    for _ in range(200):
        q, _ = np.linalg.qr(rng.standard_normal((k, k)))
        assert f <= _loss(ups, q, y) + 1e-12
        # and near Phi (small orthogonal perturbations)
        a = rng.standard_normal((k, k)) * 1e-3
        near = phi @ np.linalg.qr(np.eye(k) + (a - a.T))[0]
        assert f <= _loss(ups, near, y) + 1e-12


def test_rotated_indicator_is_recovered():
    """Ups = Y Q with Q orthogonal: M = Ups^T Y = Q^T, so the update returns
    Q^T and Ups Phi = Y exactly (here M is orthogonal already, so the
    literal update would give the same Phi)."""
    rng = np.random.default_rng(5)
    k, n = 5, 100
    lab = rng.permutation(n) % k
    y = _indicator(lab, k)
    q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    ups = y @ q
    phi = oracle.polar_factor(ups.T @ y)
    assert np.allclose(phi, q.T, atol=1e-12)
    assert np.allclose(ups @ phi, y, atol=1e-12)


def test_empty_cluster_partial_isometry():
    rng = np.random.default_rng(9)
    k = 4
    ups = np.abs(rng.standard_normal((50, k)))
    lab = rng.integers(0, 3, 50)  # cluster 3 empty
    m = ups.T @ _indicator(lab, k)
    assert np.all(m[:, 3] == 0)
    phi = oracle.polar_factor(m)
    assert np.all(np.abs(phi[:, 3]) < 1e-15)
    assert np.allclose(phi @ phi.T @ phi, phi, atol=1e-12)
    assert np.linalg.matrix_rank(phi) == 3
    assert np.array_equal(oracle.polar_factor(np.zeros((3, 3))), np.zeros((3, 3)))
    assert oracle.polar_factor(np.array([[2.5]]))[0, 0] == pytest.approx(1.0)


def test_nci_variant_behaviour():
    rng = np.random.default_rng(3)
    ups = np.abs(rng.standard_normal((300, 6)))
    # T_g = 0 and T_g = 1 use Phi = I only: both variants agree
    for t in (0, 1):
        assert np.array_equal(oracle.nci(ups, t)[0], oracle.nci(ups, t, "procrustes")[0])
    lab, phi = oracle.nci(ups, 8, "procrustes")
    assert np.allclose(phi.T @ phi, np.eye(6), atol=1e-10) or np.linalg.matrix_rank(phi) < 6
    with pytest.raises(ValueError):
        oracle.nci(ups, 3, "other")
