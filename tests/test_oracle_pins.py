"""Pins of the FP64 oracle against values and facts the paper and the
mathematics fix independently of the oracle's own code.

Each test names the passage it pins.  Every oracle function is covered by at
least one check that a plausible slip (dropped term, wrong sign, index or
transpose) would fail.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as o

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rand_graph(rng, n_u, n_v, n_e, weighted=False, dup=False):
    eu = rng.integers(0, n_u, n_e)
    ev = rng.integers(0, n_v, n_e)
    if dup:
        eu = np.concatenate([eu, eu[:5]])
        ev = np.concatenate([ev, ev[:5]])
    w = rng.uniform(0.2, 2.0, eu.shape[0]) if weighted else None
    return eu, ev, w


# ---------------------------------------------------------------- Eq. s ----
def test_running_example_msa_values(golden_dir):
    """Appendix running example: Eq. s on the printed Z_hat gives the printed s.

    Tolerance derived from the printing: Z_hat entries are rounded to 0.005, so
    Z_hat_i . Z_hat_j moves by at most 0.005 (|z_i|_1 + |z_j|_1) < 0.0175 and s
    (about 0.145) by at most 0.0175 * 0.148 < 2.6e-3; s itself is rounded to
    5e-4.  A row-wise (asymmetric) softmax misses this bound (3.6e-3), as does
    a doubled exponent (6.5e-3)."""
    with open(os.path.join(golden_dir, "running_example.json")) as f:
        g = json.load(f)
    zhat = np.array(g["zhat"])
    s_print = np.array(g["s"])
    bound = 0.005 * 2 * np.max(np.abs(zhat).sum(1)) * s_print.max() + 5e-4
    s = o.msa_matrix(zhat)
    assert np.max(np.abs(s - s_print)) <= bound
    assert np.allclose(s, s.T)
    e = np.exp(zhat @ zhat.T)
    assert np.max(np.abs(e / e.sum(1, keepdims=True) - s_print)) > bound


def test_msa_closed_form_properties():
    """Eq. s: symmetric, positive, and S = D^-1/2 E D^-1/2 with E = exp(Zh Zh^T)."""
    rng = np.random.default_rng(1)
    zh = o.normalize_rows(rng.standard_normal((9, 4)))
    s = o.msa_matrix(zh)
    for i in range(9):
        for j in range(9):
            num = math.exp(float(zh[i] @ zh[j]))
            di = sum(math.exp(float(zh[i] @ zh[l])) for l in range(9))
            dj = sum(math.exp(float(zh[j] @ zh[l])) for l in range(9))
            assert abs(s[i, j] - num / math.sqrt(di * dj)) < 1e-14


# ---------------------------------------------------- Section 2.1 / 2.2 ----
def test_coneighbour_worked_value(golden_dir):
    """Section 2.2: w_hat(u3, u4) = 1/3 + 1/2 + 1/4 on the running example."""
    with open(os.path.join(golden_dir, "coneighbour_example.json")) as f:
        g = json.load(f)
    e = np.array(g["edges_u1_based"]) - 1
    b = o.bipartite_adjacency(g["n_u"], g["n_v"], e[:, 0], e[:, 1])
    w = o.coneighbour_weights(b).toarray()
    num, den = g["expected_w_hat_u3_u4"]
    assert abs(w[2, 3] - num / den) < 1e-15
    assert abs(w[3, 2] - num / den) < 1e-15


def test_adjacency_and_degrees_bruteforce():
    """Section 2.1: B_U[i,j] = w(u_i,v_j) (duplicates summed), D_U, D_V row and
    column weight sums, checked against explicit loops."""
    rng = np.random.default_rng(2)
    eu, ev, w = _rand_graph(rng, 6, 5, 14, weighted=True, dup=True)
    b = o.bipartite_adjacency(6, 5, eu, ev, w).toarray()
    ref = np.zeros((6, 5))
    for a, c, ww in zip(eu, ev, w):
        ref[a, c] += ww
    assert np.allclose(b, ref, rtol=0, atol=1e-15)
    du, dv = o.weighted_degrees(sp.csr_matrix(ref))
    for i in range(6):
        assert abs(du[i] - sum(ref[i, j] for j in range(5))) < 1e-14
    for j in range(5):
        assert abs(dv[j] - sum(ref[i, j] for i in range(6))) < 1e-14


def test_adjacency_rejects_bad_input():
    with pytest.raises(ValueError):
        o.bipartite_adjacency(3, 3, [0, 3], [0, 1])
    with pytest.raises(ValueError):
        o.bipartite_adjacency(3, 3, [0, 1], [0, -1])
    with pytest.raises(ValueError):
        o.bipartite_adjacency(3, 3, [0, 1], [0, 1], [1.0, -0.5])


def test_normalized_adjacency_entries_and_invariants():
    """Eq. L entry by entry, and the row-stochastic rewrite used in the proof of
    Lemma FF-ZZ: D_U^-1 B 1 = 1, D_V^-1 B^T 1 = 1 on non-isolated rows,
    L L^T (D_U^1/2 1) = D_U^1/2 1."""
    rng = np.random.default_rng(3)
    eu, ev, w = _rand_graph(rng, 8, 7, 20, weighted=True)
    bm = o.bipartite_adjacency(8, 7, eu, ev, w)
    b = bm.toarray()
    du, dv = b.sum(1), b.sum(0)
    lm = o.normalized_adjacency(bm).toarray()
    for i in range(8):
        for j in range(7):
            exp = b[i, j] / math.sqrt(du[i] * dv[j]) if b[i, j] else 0.0
            assert abs(lm[i, j] - exp) < 1e-15
    nz_u, nz_v = du > 0, dv > 0
    assert np.allclose((b / np.where(nz_u, du, 1)[:, None]).sum(1)[nz_u], 1.0)
    assert np.allclose((b.T / np.where(nz_v, dv, 1)[:, None]).sum(1)[nz_v], 1.0)
    x = np.sqrt(du)
    assert np.allclose(lm @ (lm.T @ x), x, atol=1e-13)
    # w_hat = (L L^T) scaled back by sqrt(D_i D_j)
    wh = o.coneighbour_weights(bm).toarray()
    mm = lm @ lm.T
    for i in range(8):
        for j in range(8):
            if du[i] > 0 and du[j] > 0:
                assert abs(wh[i, j] - mm[i, j] * math.sqrt(du[i] * du[j])) < 1e-13


def test_isolated_nodes_get_zero_scale():
    """Reading A3: D^-1/2 := 0 for an isolated node; isolated U rows keep X."""
    d = np.array([0.0, 4.0, 1.0])
    assert np.allclose(o.inv_sqrt_or_zero(d), [0.0, 0.5, 1.0])
    bm = o.bipartite_adjacency(3, 4, [1, 1, 2], [0, 2, 2])
    x = np.arange(12.0).reshape(3, 4) + 1
    z = o.propagate(bm, x, 0.5, 4)
    assert np.allclose(z[0], 0.5 * x[0])
    # adding isolated V nodes changes nothing
    bm2 = o.bipartite_adjacency(3, 9, [1, 1, 2], [0, 2, 2])
    assert np.allclose(o.propagate(bm2, x, 0.5, 4), z)


# ------------------------------------------------- Eq. PX / Lemma ZPX ----
@pytest.mark.parametrize("alpha,gamma", [(0.5, 0), (0.5, 1), (0.5, 5), (0.9, 7), (0.0, 3)])
def test_propagation_matches_dense_powers(alpha, gamma):
    """Eq. PX: Horner evaluation equals the term-by-term dense sum."""
    rng = np.random.default_rng(4)
    eu, ev, w = _rand_graph(rng, 10, 12, 30, weighted=True)
    bm = o.bipartite_adjacency(10, 12, eu, ev, w)
    x = rng.standard_normal((10, 3))
    z = o.propagate(bm, x, alpha, gamma)
    ref = o.propagate_dense_powers(bm, x, alpha, gamma)
    assert np.allclose(z, ref, rtol=1e-12, atol=1e-13)
    # independent second route: the row-stochastic similarity of the proof of
    # Lemma FF-ZZ, P = D_U^1/2 sum (alpha D_U^-1 B D_V^-1 B^T)^r D_U^-1/2
    b = bm.toarray()
    du, dv = b.sum(1), b.sum(0)
    iu = np.where(du > 0, 1 / np.where(du > 0, du, 1), 0)
    iv = np.where(dv > 0, 1 / np.where(dv > 0, dv, 1), 0)
    m = (iu[:, None] * b) @ (iv[:, None] * b.T)
    hs = np.where(du > 0, np.sqrt(du), 0)
    his = np.where(du > 0, 1 / np.sqrt(np.where(du > 0, du, 1)), 0)
    xt = his[:, None] * x
    wacc = np.zeros_like(x)
    p = np.eye(10)
    for r in range(gamma + 1):
        wacc += alpha ** r * (p @ xt)
        p = p @ m
    zz = hs[:, None] * wacc
    iso = du == 0
    zz[iso] = x[iso]
    assert np.allclose(z, (1 - alpha) * zz, rtol=1e-12, atol=1e-13)


def test_gamma_zero_and_alpha_zero():
    """gamma = 0 gives Z_hat = rownorm(X); alpha = 0 gives Z = X (Section 2.2)."""
    rng = np.random.default_rng(5)
    eu, ev, _ = _rand_graph(rng, 10, 10, 25)
    bm = o.bipartite_adjacency(10, 10, eu, ev)
    x = rng.standard_normal((10, 4))
    assert np.allclose(o.normalize_rows(o.propagate(bm, x, 0.7, 0)), o.normalize_rows(x))
    assert np.allclose(o.propagate(bm, x, 0.0, 6), x)


def test_propagation_neumann_limit():
    """Lemma ZPX: as gamma grows Z tends to (1-alpha)(I - alpha L L^T)^-1 X,
    the stationary point of the objective of Eq. Z-obj."""
    rng = np.random.default_rng(6)
    eu, ev, _ = _rand_graph(rng, 12, 9, 40)
    bm = o.bipartite_adjacency(12, 9, eu, ev)
    x = rng.standard_normal((12, 3))
    zc = o.propagate_closed_form(bm, x, 0.6)
    assert np.allclose(o.propagate(bm, x, 0.6, 200), zc, atol=1e-13)
    # gradient of Eq. Z-obj (trace form) vanishes at the closed form
    lm = o.normalized_adjacency(bm).toarray()
    grad = (1 - 0.6) * (zc - x) + 0.6 * (np.eye(12) - lm @ lm.T) @ zc
    assert np.max(np.abs(grad)) < 1e-13


def test_og_trace_identity_bruteforce():
    """Proof of Lemma ZPX: the pairwise form of Eq. Og equals
    Tr(Z^T (I - L L^T) Z) (diagonal i = j terms of w_hat included)."""
    rng = np.random.default_rng(7)
    eu, ev, w = _rand_graph(rng, 7, 6, 20, weighted=True)
    # drop isolated U nodes: Eq. Og divides by D_U
    bm = o.bipartite_adjacency(7, 6, eu, ev, w)
    du, _ = o.weighted_degrees(bm)
    keep = np.where(du > 0)[0]
    bm = bm[keep]
    n = bm.shape[0]
    du, _ = o.weighted_degrees(bm)
    wh = o.coneighbour_weights(bm).toarray()
    z = rng.standard_normal((n, 3))
    og = 0.0
    for i in range(n):
        for j in range(n):
            dvec = z[i] / math.sqrt(du[i]) - z[j] / math.sqrt(du[j])
            og += 0.5 * wh[i, j] * float(dvec @ dvec)
    zero_x = np.zeros_like(z)
    # z_objective with alpha = 1 is exactly the trace form of Og
    assert abs(o.z_objective(bm, zero_x, z, 1.0) - og) < 1e-12


def test_z_objective_non_increasing_over_hops():
    """Eq. Z-obj evaluated at the Horner iterates is non-increasing in gamma
    (error shrinks as (alpha lambda)^(t+1) per eigendirection of L L^T)."""
    rng = np.random.default_rng(8)
    eu, ev, _ = _rand_graph(rng, 40, 50, 200)
    bm = o.bipartite_adjacency(40, 50, eu, ev)
    x = rng.standard_normal((40, 5))
    vals = [o.z_objective(bm, x, o.propagate(bm, x, 0.8, t), 0.8) for t in range(12)]
    assert all(b <= a + 1e-12 for a, b in zip(vals, vals[1:]))
    assert vals[-1] < vals[0]


# ------------------------------------------------------ Eq. Z, Q, R', R ----
def test_normalize_rows():
    z = np.array([[3.0, 4.0], [0.0, 0.0], [-1.0, 0.0]])
    assert np.allclose(o.normalize_rows(z), [[0.6, 0.8], [0, 0], [-1, 0]])


def test_orthogonal_from_gaussian_is_positive_diagonal_qr():
    """Algorithm 1: Q orthogonal and Q^T G upper triangular with a
    positive diagonal (the unique such QR factor)."""
    rng = np.random.default_rng(9)
    g = rng.standard_normal((16, 16))
    q = o.orthogonal_from_gaussian(g)
    assert np.allclose(q.T @ q, np.eye(16), atol=1e-14)
    r = q.T @ g
    assert np.allclose(np.tril(r, -1), 0, atol=1e-13)
    assert np.all(np.diag(r) > 0)


def test_random_feature_identities():
    """Eq. R-prime: ||R'[i]||^2 = e and R'[i].R'[j] = (e/d) sum cos(Zo_i - Zo_j);
    Eq. Ri: R R^T x = x for x_i = sqrt(R'[i].r), so R has singular value 1
    with right vector r/||r||."""
    rng = np.random.default_rng(10)
    zh = o.normalize_rows(rng.standard_normal((30, 8)))
    q = o.orthogonal_from_gaussian(rng.standard_normal((8, 8)))
    r, rp, rsum = o.random_features(zh, q)
    assert np.allclose(np.sum(rp * rp, 1), math.e, rtol=1e-14)
    zo = math.sqrt(8) * zh @ q.T
    for i, j in [(0, 1), (3, 7), (5, 5)]:
        ref = math.e / 8 * float(np.sum(np.cos(zo[i] - zo[j])))
        assert abs(float(rp[i] @ rp[j]) - ref) < 1e-13
    assert np.allclose(rsum, rp.sum(0))
    x = np.sqrt(rp @ rsum)
    assert np.allclose(r @ (r.T @ x), x, rtol=1e-13)
    assert np.allclose(r.T @ x, rsum, rtol=1e-13)
    sv = np.linalg.svd(r, compute_uv=False)
    assert abs(sv[0] - 1.0) < 1e-12


def test_theorem_rr_statistical():
    """Theorem RR: E[R_i . R_j] is within the stated factor of s(u_i, u_j).
    Monte Carlo over Q seeds; band widened by 4 standard errors."""
    rng = np.random.default_rng(11)
    d, n, trials = 32, 6, 3000
    zh = o.normalize_rows(rng.standard_normal((n, d)) + 0.5)
    s = o.msa_matrix(zh)
    acc = np.zeros((n, n))
    acc2 = np.zeros((n, n))
    for _ in range(trials):
        q = o.orthogonal_from_gaussian(rng.standard_normal((d, d)))
        # E[R_i.R_j] through Eq. Ri needs r over all of U: use a population of
        # n nodes exactly as the algorithm does
        r, _, _ = o.random_features(zh, q)
        m = r @ r.T
        acc += m
        acc2 += m * m
    mean = acc / trials
    se = np.sqrt(np.maximum(acc2 / trials - mean ** 2, 0) / trials)
    c = 17 / (16 * d * d) + 1 / (4 * d)
    lo, hi = (1 - c) / (1 + c), (1 + c) / (1 - c)
    ratio_lo = (mean + 4 * se) / s
    ratio_hi = (mean - 4 * se) / s
    assert np.all(ratio_lo >= lo), ratio_lo.min()
    assert np.all(ratio_hi <= hi), ratio_hi.max()


def test_random_features_reject_nonpositive_normaliser():
    """Reading A8: a non-positive or non-finite R'[i] . r is an error."""
    q = np.eye(2)
    with pytest.raises(FloatingPointError):
        o.random_features(np.array([[np.nan, 0.0]]), q)


# ------------------------------------------------ RandomizedSVD / Eq. Xd ----
def _gapped(rng, n, m, k, gap=50.0):
    u = o.orthonormal_basis(rng.standard_normal((n, m)))
    v = o.orthonormal_basis(rng.standard_normal((m, m)))
    s = np.concatenate([np.linspace(gap, gap / 2, k), np.linspace(1.0, 0.1, m - k)])
    return (u * s) @ v.T


def test_randomized_svd_matches_exact_on_gapped_spectrum():
    """Algorithm 2 (Halko et al.): with q power iterations and a spectral
    gap the randomized top-k SVD equals the exact one."""
    rng = np.random.default_rng(12)
    a = _gapped(rng, 300, 24, 5)
    om = rng.standard_normal((24, 9))
    g1, s1, p1 = o.randomized_svd(a, 5, om, 6)
    g2, s2, p2 = o.exact_svd(a, 5)
    assert np.allclose(s1, s2, rtol=1e-12)
    assert np.allclose(g1, g2, atol=1e-10)
    assert np.allclose(p1, p2, atol=1e-10)
    # SVD relations and sign convention
    assert np.allclose(a @ p1, g1 * s1, atol=1e-10)
    assert np.allclose(a.T @ g1, p1 * s1, atol=1e-10)
    assert np.allclose(g1.T @ g1, np.eye(5), atol=1e-12)
    assert np.all(g1.sum(0) > 0)
    assert np.all(np.diff(s1) <= 0)


def test_randomized_svd_converges_with_q():
    """More power iterations never move the sketch further from the exact
    top-k subspace on a slowly decaying spectrum (observed, with slack)."""
    rng = np.random.default_rng(13)
    u = o.orthonormal_basis(rng.standard_normal((200, 30)))
    v = o.orthonormal_basis(rng.standard_normal((30, 30)))
    a = (u * (0.9 ** np.arange(30))) @ v.T
    om = rng.standard_normal((30, 8))
    ge, _, _ = o.exact_svd(a, 4)
    errs = [o.subspace_sin_theta(o.randomized_svd(a, 4, om, q)[0], ge) for q in (0, 2, 6, 20)]
    assert errs[-1] < 1e-6
    assert all(b <= a_ * 1.5 + 1e-15 for a_, b in zip(errs, errs[1:]))


def test_sign_convention_flip_invariance():
    rng = np.random.default_rng(14)
    a = _gapped(rng, 100, 12, 4)
    g, s, p = o.exact_svd(a, 4)
    flips = np.array([1, -1, -1, 1.0])
    g2, p2 = o.column_sign_convention(g * flips, p * flips)
    assert np.allclose(g2, g) and np.allclose(p2, p)
    # degenerate column sum falls back to the largest entry's sign
    col = np.array([[1.0], [-1.0], [0.5], [-0.5], [-2.0]])
    col = col - col.mean()
    (fixed,) = o.column_sign_convention(col)
    assert fixed[np.argmax(np.abs(fixed)), 0] > 0
    # with a right vector, its largest entry decides the degenerate case
    right = np.array([[0.1], [-0.9], [0.3]])
    g3, r3 = o.column_sign_convention(col, right)
    assert r3[1, 0] > 0 and np.allclose(g3, -col)
    # a clear column sum wins over the right vector
    g4, r4 = o.column_sign_convention(-col + 0.2, right)
    assert np.allclose(g4, -col + 0.2) and np.allclose(r4, right)


def test_attribute_reduction_matches_exact_with_gap():
    """Section 3.2.1: the randomized top-d route equals the exact top-d SVD when
    there is a gap, and X' = X Psi_d = Gamma Sigma (Eq. Xd)."""
    rng = np.random.default_rng(15)
    x = _gapped(rng, 400, 32, 6, gap=40.0)
    om = rng.standard_normal((32, 12))
    psi, sig = o.top_d_attribute_svd(x, 6, om, 8)
    psi_e, sig_e = o.exact_top_d_attribute_svd(x, 6)
    assert np.allclose(sig, sig_e, rtol=1e-12)
    assert np.allclose(psi, psi_e, atol=1e-10)
    u, s, vt = np.linalg.svd(x, full_matrices=False)
    xp = x @ psi
    # Gamma Sigma of Eq. Xd, up to the column sign convention
    assert np.allclose(np.abs(xp), np.abs(u[:, :6] * s[:6]), atol=1e-10)
    assert np.all(xp.sum(0) > 0)


def test_gram_basis_matches_exact_with_gap():
    """Section 3.2.1 from the Gram matrix alone: with a spectral gap the basis
    equals LAPACK's top-d right singular vectors of X, with the column sign
    convention read through X's column sums."""
    rng = np.random.default_rng(21)
    x = _gapped(rng, 400, 32, 6, gap=40.0)
    om = rng.standard_normal((32, 12))
    psi, sig = o.top_d_gram_basis(x.T @ x, x.sum(0), x.shape[0], 6, om, 8)
    psi_e, sig_e = o.exact_top_d_attribute_svd(x, 6)
    assert np.allclose(sig, sig_e, rtol=1e-12)
    assert np.allclose(psi, psi_e, atol=1e-10)
    assert np.all((x @ psi).sum(0) > 0)


def test_gram_basis_sign_fallback_on_centred_columns():
    """Zero column sums of X Psi (centred X) leave the sign to the entry of
    largest magnitude of each basis column, which comes out positive."""
    rng = np.random.default_rng(22)
    x = _gapped(rng, 300, 16, 4, gap=30.0)
    x = x - x.mean(0)
    om = rng.standard_normal((16, 8))
    psi, _ = o.top_d_gram_basis(x.T @ x, x.sum(0), x.shape[0], 4, om, 10)
    for j in range(4):
        assert psi[int(np.argmax(np.abs(psi[:, j]))), j] > 0
    u, s, vt = np.linalg.svd(x, full_matrices=False)
    assert np.allclose(np.abs(psi), np.abs(vt[:4].T), atol=1e-10)


def test_gram_basis_rayleigh_ritz_with_another_matrix():
    """With c_final the Rayleigh-Ritz step uses that matrix: when the iterated
    matrix and c_final share their leading invariant subspace but order its
    eigenvalues differently, the basis comes out as c_final's eigenvectors in
    c_final's order (LAPACK eigh of c_final)."""
    rng = np.random.default_rng(23)
    v, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    lam1 = np.concatenate([[50, 45, 40, 35, 30, 25], 0.1 * rng.uniform(size=14)])
    lam2 = np.concatenate([[30, 50, 25, 45, 35, 40], 0.1 * rng.uniform(size=14)])
    c1 = (v * lam1) @ v.T
    c2 = (v * lam2) @ v.T
    x_colsum = rng.standard_normal(20)
    om = rng.standard_normal((20, 6))
    psi, sig = o.top_d_gram_basis(c1, x_colsum, 100, 4, om, 30, c_final=c2)
    w, u = np.linalg.eigh(c2)
    top = u[:, np.argsort(-w)[:4]]
    assert np.allclose(sig ** 2, np.sort(w)[::-1][:4], rtol=1e-10)
    assert np.allclose(np.abs(psi.T @ top), np.eye(4), atol=1e-8)
    # without c_final: c1's own order
    psi1, _ = o.top_d_gram_basis(c1, x_colsum, 100, 4, om, 30)
    assert np.allclose(np.abs(psi1.T @ v[:, :4]), np.eye(4), atol=1e-8)


def test_lemma_ff_zz_bound():
    """Lemma FF-ZZ: |Z'_i . Z'_j - Z_i . Z_j| <= sigma_{d+1}^2 sqrt(D_i D_j)/(1-alpha)
    with the exact top-d SVD and the gamma -> infinity propagation."""
    rng = np.random.default_rng(16)
    n_u, n_v = 25, 20
    eu = np.concatenate([np.arange(n_u), rng.integers(0, n_u, 40)])
    ev = np.concatenate([rng.integers(0, n_v, n_u), rng.integers(0, n_v, 40)])
    bm = o.bipartite_adjacency(n_u, n_v, eu, ev)
    x = rng.standard_normal((n_u, 10))
    d, alpha = 4, 0.5
    psi, _ = o.exact_top_d_attribute_svd(x, d)
    s_all = np.linalg.svd(x, compute_uv=False)
    z = o.propagate_closed_form(bm, x, alpha)
    zp = o.propagate_closed_form(bm, x @ psi, alpha)
    du, _ = o.weighted_degrees(bm)
    bound = s_all[d] ** 2 * np.sqrt(np.outer(du, du)) / (1 - alpha)
    assert np.all(np.abs(zp @ zp.T - z @ z.T) <= bound + 1e-10)


# ----------------------------------------------------------- ONMF (Alg 2) ----
def test_onmf_exact_svd_is_fixed_point():
    """Eqs. init-HY, update-Q, update-Y: at an exact SVD init every ratio is 1
    (Eckart-Young optimum of the relaxed problem), so Ups stays Gamma."""
    rng = np.random.default_rng(17)
    zh = o.normalize_rows(rng.standard_normal((80, 6)))
    q = o.orthogonal_from_gaussian(rng.standard_normal((6, 6)))
    r, _, _ = o.random_features(zh, q)
    g, s, p = o.exact_svd(r, 3)
    ups, h, hits = o.onmf(r, g, s, p, 5)
    assert np.allclose(ups, g, atol=1e-10)
    assert np.allclose(h, p * s, atol=1e-10)
    assert hits == 0


def test_onmf_one_step_elementwise_bruteforce():
    """One round of Eqs. update-Q then update-Y written with explicit sums on a
    non-negative example (no guards involved)."""
    rng = np.random.default_rng(18)
    n, m, k = 7, 5, 3
    r = rng.uniform(0.1, 1.0, (n, m))
    g = rng.uniform(0.1, 1.0, (n, k))
    p = rng.uniform(0.1, 1.0, (m, k))
    s = np.ones(k)
    ups, h, _ = o.onmf(r, g, s, p, 1)
    h0 = p.copy()
    hn = np.zeros_like(h0)
    for j in range(m):
        for l in range(k):
            num = sum(r[i, j] * g[i, l] for i in range(n))
            den = sum(h0[j, t] * sum(g[i, t] * g[i, l] for i in range(n)) for t in range(k))
            hn[j, l] = h0[j, l] * num / den
    assert np.allclose(h, hn, rtol=1e-13)
    rh = np.array([[sum(r[i, j] * hn[j, l] for j in range(m)) for l in range(k)] for i in range(n)])
    yrh = np.array([[sum(g[i, t] * rh[i, l] for i in range(n)) for l in range(k)] for t in range(k)])
    un = np.zeros_like(g)
    for i in range(n):
        for l in range(k):
            den = sum(g[i, t] * yrh[t, l] for t in range(k))
            un[i, l] = g[i, l] * math.sqrt(rh[i, l] / den)
    assert np.allclose(ups, un, rtol=1e-13)


def test_onmf_guards():
    """Reading A11: zero denominators keep the entry, negative Eq. update-Y
    ratios zero it, and each is counted."""
    r = np.array([[1.0, -1.0], [0.0, 0.0]])
    g = np.array([[1.0], [0.0]])
    p = np.array([[1.0], [1.0]])
    ups, h, hits = o.onmf(r, g, np.array([1.0]), p, 1)
    assert np.all(np.isfinite(ups)) and hits > 0


# ------------------------------------------------------------ NCI (Alg 3) ----
def _nci_loops(ups, t_g):
    n, k = len(ups), len(ups[0])
    phi = [[1.0 if a == b else 0.0 for b in range(k)] for a in range(k)]
    labels = [max(range(k), key=lambda l: (ups[i][l], -l)) for i in range(n)]
    for _ in range(t_g):
        labels = []
        for i in range(n):
            best, arg = None, 0
            for l in range(k):
                v = sum(ups[i][t] * phi[t][l] for t in range(k))
                if best is None or v > best:
                    best, arg = v, l
            labels.append(arg)
        cnt = [labels.count(l) for l in range(k)]
        phi = [[sum(ups[i][t] for i in range(n) if labels[i] == l) / math.sqrt(cnt[l]) if cnt[l] else 0.0
                for l in range(k)] for t in range(k)]
    return labels


@pytest.mark.parametrize("t_g", [0, 1, 3, 20])
def test_nci_matches_loops(t_g):
    """Algorithm 3 restated with explicit loops (Eqs. ell-ast, Y-update, y-norm,
    Phi <- Ups^T Y); first maximum wins ties."""
    rng = np.random.default_rng(19 + t_g)
    ups = rng.standard_normal((40, 4))
    labels, _ = o.nci(ups, t_g)
    assert list(labels) == _nci_loops(ups.tolist(), t_g)


def test_nci_tie_break_and_empty_cluster():
    ups = np.array([[1.0, 1.0, 0.0], [0.5, 0.5, 0.0], [0.0, 2.0, 2.0]])
    labels, _ = o.nci(ups, 0)
    assert list(labels) == [0, 0, 1]
    labels, phi = o.nci(ups, 3)
    assert np.all(np.isfinite(phi))


def test_nci_recovers_exact_indicator():
    """An exact NCI matrix (Eq. Y) is a fixed point of Algorithm 3."""
    lab = np.array([0, 2, 1, 1, 0, 2, 2, 1])
    k = 3
    y = np.zeros((8, k))
    y[np.arange(8), lab] = 1
    y /= np.sqrt(y.sum(0))
    labels, phi = o.nci(y, 5)
    assert list(labels) == list(lab)
    assert np.allclose(phi, np.eye(k))


# ----------------------------------------------------------- Eq. obj1 ----
def test_objective_matches_bruteforce_and_lemma_obj2():
    """Eq. obj1 pair by pair over S = R R^T, and Lemma obj2:
    obj1 = Tr(Y^T (S_d - S) Y), trace form = Tr(Y^T S Y)."""
    rng = np.random.default_rng(20)
    zh = o.normalize_rows(rng.standard_normal((25, 5)))
    q = o.orthogonal_from_gaussian(rng.standard_normal((5, 5)))
    r, _, _ = o.random_features(zh, q)
    lab = rng.integers(0, 4, 25)
    lab[lab == 3] = 2  # leave cluster 3 empty
    s = r @ r.T
    obj, tr = o.objective(r, lab, 4)
    assert abs(obj - o.objective_bruteforce(s, lab, 4)) < 1e-13
    y = np.zeros((25, 4))
    y[np.arange(25), lab] = 1
    cnt = y.sum(0)
    y[:, cnt > 0] /= np.sqrt(cnt[cnt > 0])
    sd = np.diag(s.sum(1))
    assert abs(obj - np.trace(y.T @ (sd - s) @ y)) < 1e-13
    assert abs(tr - np.trace(y.T @ s @ y)) < 1e-13


# --------------------------------------------------- comparison helpers ----
def test_label_permutation_helper():
    a = np.array([0, 0, 1, 2, 2])
    assert o.labels_match_up_to_permutation(a, np.array([2, 2, 0, 1, 1]))
    assert not o.labels_match_up_to_permutation(a, np.array([2, 2, 0, 0, 1]))
    assert not o.labels_match_up_to_permutation(a, np.array([0, 0, 1, 1, 1]))


def test_subspace_sin_theta_helper():
    e = np.eye(4)
    assert o.subspace_sin_theta(e[:, :2], e[:, [1, 0]]) < 1e-15
    t = 1e-7
    b = np.stack([np.array([1, 0, t, 0]) / math.hypot(1, t), e[:, 1]], 1)
    assert abs(o.subspace_sin_theta(e[:, :2], b) - t) < 1e-12 + 1e-3 * t


# ---------------------------------------------------- whole pipeline ----
def test_pipeline_small_job_runs_and_is_deterministic():
    import abg_synth as synth
    g = synth.planted_abg(300, 400, 2500, 4, 16, seed=3)
    mm = synth.method_matrices(7, 16, 8, 4)
    kw = dict(k=4, alpha=0.5, gamma=3, g=mm.g, omega=mm.omega,
              omega_r=mm.omega_reduce, d=8, q=20, t_f=5, t_g=20)
    r1 = o.tpo(g.n_u, g.n_v, g.edge_u, g.edge_v, g.x_u, **kw)
    r2 = o.tpo(g.n_u, g.n_v, g.edge_u, g.edge_v, g.x_u, **kw)
    assert np.array_equal(r1.labels, r2.labels)
    assert r1.objective == r2.objective
    assert r1.labels.min() >= 0 and r1.labels.max() < 4
    assert np.isfinite(r1.objective)
