"""FP64 reference implementation of the TPO pipeline, step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring): imported by tests/,
__graft_entry__.smoke() and bench.py's cpu_baseline leg, never by the product.

Every function follows one passage of the paper and says which.  Readings of
points the paper leaves open are marked "Reading:".  Library primitives used
as single steps: scipy.sparse products, numpy matmul, numpy.linalg.qr / svd /
eigh, numpy argmax.

Pins (tests/test_oracle_*.py, all CPU): the running example's printed MSA
values, the co-neighbour weight worked value, dense matrix powers and the
Neumann closed form of Lemma ZPX, row-stochastic invariants, monotone
Z-objective, the sin/cos feature identities, Theorem RR statistically,
Eckart-Young fixed point of the ONMF updates, exact SVD vs the randomized
one on gapped spectra, Lemma FF-ZZ, brute-force NCI/objective on tiny inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "OracleResult",
    "bipartite_adjacency",
    "weighted_degrees",
    "inv_sqrt_or_zero",
    "normalized_adjacency",
    "coneighbour_weights",
    "propagate",
    "propagate_dense_powers",
    "propagate_closed_form",
    "z_objective",
    "normalize_rows",
    "msa_matrix",
    "orthogonal_from_gaussian",
    "random_features",
    "orthonormal_basis",
    "randomized_svd",
    "exact_svd",
    "column_sign_convention",
    "top_d_attribute_svd",
    "exact_top_d_attribute_svd",
    "top_d_gram_basis",
    "reduce_attributes",
    "onmf",
    "nci",
    "polar_factor",
    "objective",
    "objective_bruteforce",
    "tpo",
    "labels_match_up_to_permutation",
    "subspace_sin_theta",
]


# ---------------------------------------------------------------------------
# Section 2.1: the bipartite adjacency B_U and the degree matrices D_U, D_V
# ---------------------------------------------------------------------------
def bipartite_adjacency(n_u: int, n_v: int, edge_u, edge_v, edge_w=None) -> sp.csr_matrix:
    """B_U[i, j] = w(u_i, v_j) for (u_i, v_j) in E, else 0 (Section 2.1).

    Reading: a (u, v) pair listed more than once contributes the sum of its
    weights; edges without weights have w = 1.  Negative weights are rejected.
    """
    eu = np.asarray(edge_u, dtype=np.int64)
    ev = np.asarray(edge_v, dtype=np.int64)
    if eu.shape != ev.shape:
        raise ValueError("edge arrays differ in length")
    if eu.size and (eu.min() < 0 or eu.max() >= n_u or ev.min() < 0 or ev.max() >= n_v):
        raise ValueError("edge endpoint out of range")
    w = np.ones(eu.shape[0]) if edge_w is None else np.asarray(edge_w, dtype=np.float64)
    if w.size and w.min() < 0:
        raise ValueError("negative edge weight")
    b = sp.coo_matrix((w, (eu, ev)), shape=(n_u, n_v)).tocsr()
    b.sum_duplicates()
    b.sort_indices()
    return b


def weighted_degrees(b: sp.csr_matrix) -> tuple[np.ndarray, np.ndarray]:
    """Diagonals of D_U (row sums of B_U) and D_V (column sums), Section 2.1."""
    d_u = np.asarray(b.sum(axis=1)).ravel().astype(np.float64)
    d_v = np.asarray(b.sum(axis=0)).ravel().astype(np.float64)
    return d_u, d_v


def inv_sqrt_or_zero(d: np.ndarray) -> np.ndarray:
    """D^{-1/2} with the reading 0^{-1/2} := 0 for isolated nodes (the paper's
    datasets drop isolated nodes; the formula is undefined there)."""
    out = np.zeros_like(d, dtype=np.float64)
    pos = d > 0
    out[pos] = 1.0 / np.sqrt(d[pos])
    return out


def normalized_adjacency(b: sp.csr_matrix) -> sp.csr_matrix:
    """L_U = D_U^{-1/2} B_U D_V^{-1/2} (Eq. L, Lemma ZPX)."""
    d_u, d_v = weighted_degrees(b)
    return (sp.diags(inv_sqrt_or_zero(d_u)) @ b @ sp.diags(inv_sqrt_or_zero(d_v))).tocsr()


def coneighbour_weights(b: sp.csr_matrix) -> sp.csr_matrix:
    """w_hat(u_i, u_j) = sum over common neighbours v_l of
    w(u_i, v_l) w(v_l, u_j) / D_V[l, l] (the weight in Eq. Og)."""
    _, d_v = weighted_degrees(b)
    inv = np.zeros_like(d_v)
    inv[d_v > 0] = 1.0 / d_v[d_v > 0]
    return (b @ sp.diags(inv) @ b.T).tocsr()


# ---------------------------------------------------------------------------
# Section 2.2 / Algorithm 1: multi-hop propagation
# ---------------------------------------------------------------------------
def propagate(b: sp.csr_matrix, x: np.ndarray, alpha: float, gamma: int) -> np.ndarray:
    """Z_U = (1 - alpha) * sum_{r=0..gamma} alpha^r (L L^T)^r X (Eq. PX).

    Evaluated by gamma Horner steps Z <- X + alpha * L (L^T Z) from Z = X, the
    update of Eq. update-Z with the product grouped as the paper groups it.
    Reading: Algorithm 1 starts from alpha*X and multiplies the whole update
    by alpha, which yields Eq. PX times alpha/(1 - alpha); a positive row scale
    cancels in Eq. Z, so we return Eq. PX's own scaling (this also gives
    Z = X at alpha = 0, as the text states).
    """
    if not (0.0 <= alpha < 1.0):
        raise ValueError("alpha must lie in [0, 1)")
    if gamma < 0:
        raise ValueError("gamma must be >= 0")
    lmat = normalized_adjacency(b)
    lt = lmat.T.tocsr()
    x = np.asarray(x, dtype=np.float64)
    z = x.copy()
    for _ in range(gamma):
        z = x + alpha * (lmat @ (lt @ z))
    return (1.0 - alpha) * z


def propagate_dense_powers(b: sp.csr_matrix, x: np.ndarray, alpha: float, gamma: int) -> np.ndarray:
    """Eq. PX term by term with dense matrix powers (tiny graphs only)."""
    lmat = normalized_adjacency(b).toarray()
    m = lmat @ lmat.T
    acc = np.zeros_like(x, dtype=np.float64)
    p = np.eye(m.shape[0])
    for r in range(gamma + 1):
        acc += alpha ** r * (p @ x)
        p = p @ m
    return (1.0 - alpha) * acc


def propagate_closed_form(b: sp.csr_matrix, x: np.ndarray, alpha: float) -> np.ndarray:
    """The gamma -> infinity limit: (1 - alpha) (I - alpha L L^T)^{-1} X
    (proof of Lemma ZPX, Neumann series)."""
    lmat = normalized_adjacency(b).toarray()
    a = np.eye(lmat.shape[0]) - alpha * (lmat @ lmat.T)
    return (1.0 - alpha) * np.linalg.solve(a, np.asarray(x, dtype=np.float64))


def z_objective(b: sp.csr_matrix, x: np.ndarray, z: np.ndarray, alpha: float) -> float:
    """(1 - alpha) ||Z - X||_F^2 + alpha * Tr(Z^T (I - L L^T) Z) (Eqs. Z-obj,
    Oa, and the trace form of Og from the proof of Lemma ZPX)."""
    lmat = normalized_adjacency(b)
    lz = lmat.T @ z
    og = float(np.sum(z * z) - np.sum(lz * lz))
    oa = float(np.sum((z - x) ** 2))
    return (1.0 - alpha) * oa + alpha * og


# ---------------------------------------------------------------------------
# Eq. Z, Eq. s
# ---------------------------------------------------------------------------
def normalize_rows(z: np.ndarray) -> np.ndarray:
    """Z_hat[i] = Z[i] / ||Z[i]|| (Eq. Z).  Reading: an all-zero row stays 0."""
    z = np.asarray(z, dtype=np.float64)
    nrm = np.sqrt(np.sum(z * z, axis=1))
    out = np.zeros_like(z)
    pos = nrm > 0
    out[pos] = z[pos] / nrm[pos, None]
    return out


def msa_matrix(zhat: np.ndarray) -> np.ndarray:
    """Exact MSA s(u_i, u_j): the symmetric softmax of Eq. s, O(n^2)."""
    e = np.exp(zhat @ zhat.T)
    rs = np.sqrt(e.sum(axis=1))
    return e / rs[:, None] / rs[None, :]


# ---------------------------------------------------------------------------
# Algorithm 1: random features (Eqs. R-prime and Ri)
# ---------------------------------------------------------------------------
def orthogonal_from_gaussian(g: np.ndarray) -> np.ndarray:
    """Q from a QR decomposition of the Gaussian matrix G (Algorithm 1).

    Reading: Householder QR with the column signs chosen so that diag(R) > 0,
    which makes Q a deterministic function of G and Haar-distributed.
    """
    q, r = np.linalg.qr(np.asarray(g, dtype=np.float64))
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def random_features(zhat: np.ndarray, q: np.ndarray):
    """R' = sqrt(e/d) [sin(Zo) || cos(Zo)], Zo = sqrt(d) Z_hat Q^T (Eq. R-prime),
    then R[i] = R'[i] / sqrt(R'[i] . r) with r = sum_l R'[l] (Eq. Ri).

    d is the working attribute width (d_U, or the reduced d).  Raises
    FloatingPointError when some R'[i] . r <= 0 (not addressed by the paper).
    Returns (R, R', r).
    """
    zhat = np.asarray(zhat, dtype=np.float64)
    d = zhat.shape[1]
    zo = math.sqrt(d) * (zhat @ q.T)
    rp = math.sqrt(math.e / d) * np.hstack([np.sin(zo), np.cos(zo)])
    r = rp.sum(axis=0)
    den = rp @ r
    if not np.all(den > 0):
        raise FloatingPointError("R'[i] . r <= 0 or not finite")
    return rp / np.sqrt(den)[:, None], rp, r


# ---------------------------------------------------------------------------
# Algorithm 2: RandomizedSVD(R, k) (Halko, Martinsson and Tropp 2011)
# ---------------------------------------------------------------------------
def orthonormal_basis(a: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(a) by Householder QR (thin Q factor)."""
    return np.linalg.qr(a, mode="reduced")[0]


def column_sign_convention(gamma: np.ndarray, *others: np.ndarray):
    """Reading (the paper fixes no sign for singular vectors): flip column c
    of gamma (and of each matrix in `others`) so that sum_i gamma[i, c] > 0.
    When that sum is within 1e-9 * sqrt(rows) * ||gamma[:, c]||_2 of zero (a
    bound on 1e-9 * ||gamma[:, c]||_1), use instead the sign of the entry of
    largest magnitude of the first matrix in `others` (the right singular
    vector; gamma itself when none is given), lowest row index on ties."""
    gamma = np.array(gamma, dtype=np.float64, copy=True)
    others = [np.array(o, dtype=np.float64, copy=True) for o in others]
    key = others[0] if others else gamma
    rows = gamma.shape[0]
    for c in range(gamma.shape[1]):
        col = gamma[:, c]
        s = col.sum()
        if abs(s) <= 1e-9 * math.sqrt(rows) * np.linalg.norm(col):
            kc = key[:, c]
            s = kc[int(np.argmax(np.abs(kc)))]
        if s < 0:
            gamma[:, c] = -col
            for o in others:
                o[:, c] = -o[:, c]
            if not others:
                key = gamma
    return (gamma, *others)


def randomized_svd(a: np.ndarray, k: int, omega: np.ndarray, q: int):
    """Top-k SVD of `a` by randomized subspace iteration (Halko et al. 2011,
    Algorithm 4.4, then the direct SVD of Algorithm 5.1).

    Reading of the unstated details: the sketch is a -> a @ omega with the
    Gaussian omega given (width k' = k + oversampling), q power iterations,
    the basis re-orthonormalised after every product with a or a^T.
    Returns (Gamma n x k, Sigma k, Psi m x k) with the column sign convention.
    """
    a = np.asarray(a, dtype=np.float64)
    qm = orthonormal_basis(a @ omega)
    for _ in range(q):
        w = orthonormal_basis(a.T @ qm)
        qm = orthonormal_basis(a @ w)
    bsm = qm.T @ a
    ub, s, vt = np.linalg.svd(bsm, full_matrices=False)
    u = qm @ ub
    gam, psi = column_sign_convention(u[:, :k], vt[:k].T)
    return gam, s[:k].copy(), psi


def exact_svd(a: np.ndarray, k: int):
    """Exact top-k SVD (LAPACK) with the same sign convention; the value the
    randomized SVD approaches as q grows."""
    u, s, vt = np.linalg.svd(np.asarray(a, dtype=np.float64), full_matrices=False)
    gam, psi = column_sign_convention(u[:, :k], vt[:k].T)
    return gam, s[:k].copy(), psi


# ---------------------------------------------------------------------------
# Section 3.2.1: SVD-based attribute dimension reduction (Eq. Xd)
# ---------------------------------------------------------------------------
def top_d_attribute_svd(x: np.ndarray, d: int, omega_r: np.ndarray, q: int):
    """Top-d right singular vectors Psi_d and values of X for Eq. Xd.

    Reading: the paper does not name the algorithm for this top-d SVD.  We
    use the same randomized subspace iteration as Algorithm 2 (Halko et al.
    Algorithm 4.4 with re-orthonormalisation after every product), applied to
    the Gram matrix C = X^T X, whose eigenvectors are X's right singular
    vectors and whose eigenvalues are the squared singular values, followed by
    the Rayleigh-Ritz step (Halko et al. Algorithm 5.3): eigenpairs of
    Q^T C Q, the top d kept.  Returns (Psi_d d_U x d, sigma_d), where
    X' = X Psi_d equals Gamma Sigma of Eq. Xd.  Signs: column c of X Psi_d has
    a positive sum (the column sign convention).
    """
    x = np.asarray(x, dtype=np.float64)
    c = x.T @ x
    qm = orthonormal_basis(c @ omega_r)
    for _ in range(q):
        qm = orthonormal_basis(c @ qm)
    t = qm.T @ c @ qm
    t = 0.5 * (t + t.T)
    evals, evecs = np.linalg.eigh(t)
    order = np.argsort(-evals, kind="stable")[:d]
    psi = qm @ evecs[:, order]
    sig = np.sqrt(np.maximum(evals[order], 0.0))
    _, psi = column_sign_convention(x @ psi, psi)
    return psi, sig


def top_d_gram_basis(c: np.ndarray, colsum_x: np.ndarray, n_rows: int, d: int, omega_r: np.ndarray, q: int,
                     c_final: np.ndarray = None):
    """The reduction basis Psi_d of Section 3.2.1 from the Gram matrix alone:
    the same randomized subspace iteration and Rayleigh-Ritz step as
    top_d_attribute_svd, applied to a given C = X^T X, with the column sign
    convention evaluated through X's column sums (sum_i (X Psi)[i, c] =
    colsum_x . Psi[:, c], ||X Psi[:, c]||_2 = sqrt(Psi[:, c]^T C Psi[:, c])).
    For checking a device's Psi_d against the device's own Gram when X itself
    is too large to hold on the host.

    c_final: the matrix of the Rayleigh-Ritz step, when it differs from the
    one the iteration used (the sparse-attribute precision form iterates on a
    Gram formed from FP8 codes and refines with the exact Gram; not in the
    paper).  Returns (Psi_d, sigma_d)."""
    c = np.asarray(c, dtype=np.float64)
    c = 0.5 * (c + c.T)
    cf = c if c_final is None else 0.5 * (np.asarray(c_final, dtype=np.float64) + np.asarray(c_final).T)
    qm = orthonormal_basis(c @ omega_r)
    for _ in range(q):
        qm = orthonormal_basis(c @ qm)
    c = cf
    t = qm.T @ c @ qm
    t = 0.5 * (t + t.T)
    evals, evecs = np.linalg.eigh(t)
    order = np.argsort(-evals, kind="stable")[:d]
    psi = qm @ evecs[:, order]
    sig = np.sqrt(np.maximum(evals[order], 0.0))
    colsum_x = np.asarray(colsum_x, dtype=np.float64)
    for j in range(psi.shape[1]):
        s = float(colsum_x @ psi[:, j])
        norm2 = math.sqrt(max(float(psi[:, j] @ c @ psi[:, j]), 0.0))
        if abs(s) <= 1e-9 * math.sqrt(n_rows) * norm2:
            s = psi[int(np.argmax(np.abs(psi[:, j]))), j]
        if s < 0:
            psi[:, j] = -psi[:, j]
    return psi, sig


def exact_top_d_attribute_svd(x: np.ndarray, d: int):
    """Exact top-d right singular vectors of X (LAPACK), same sign convention."""
    x = np.asarray(x, dtype=np.float64)
    _, s, vt = np.linalg.svd(x, full_matrices=False)
    psi = vt[:d].T
    _, psi = column_sign_convention(x @ psi, psi)
    return psi, s[:d].copy()


def reduce_attributes(x: np.ndarray, d: int, omega_r: np.ndarray, q: int):
    """X' = Gamma Sigma = X Psi_d (Eq. Xd).  Returns (X', Psi_d, sigma_d)."""
    psi, sig = top_d_attribute_svd(x, d, omega_r, q)
    return np.asarray(x, dtype=np.float64) @ psi, psi, sig


# ---------------------------------------------------------------------------
# Algorithm 2: greedy orthogonal NMF (Eqs. init-HY, update-Q, update-Y)
# ---------------------------------------------------------------------------
def onmf(r: np.ndarray, gam: np.ndarray, sig: np.ndarray, psi: np.ndarray, t_f: int):
    """Upsilon = Gamma, H = Psi Sigma (Eq. init-HY), then t_f rounds of
    H <- H * (R^T Ups) / (H (Ups^T Ups))          (Eq. update-Q)
    Ups <- Ups * sqrt((R H) / (Ups (Ups^T (R H)))) (Eq. update-Y)
    with H updated first and Ups second in each round, all entries at once.

    Reading (guards the paper does not need for non-negative data): where a
    denominator is exactly 0 the entry is kept; where the ratio of Eq.
    update-Y is negative the entry is set to 0.  Returns (Ups, H, guard_hits).
    Parity with the paper's own implementation of this stage is unpinned; the
    formulas themselves are pinned (exact fixed point at an exact SVD).
    """
    r = np.asarray(r, dtype=np.float64)
    ups = np.array(gam, dtype=np.float64, copy=True)
    h = np.asarray(psi, dtype=np.float64) * np.asarray(sig, dtype=np.float64)[None, :]
    hits = 0
    for _ in range(t_f):
        num = r.T @ ups
        den = h @ (ups.T @ ups)
        nz = den != 0
        hits += int((~nz).sum())
        h = np.where(nz, h * np.divide(num, den, out=np.ones_like(num), where=nz), h)
        rh = r @ h
        den = ups @ (ups.T @ rh)
        nz = den != 0
        ratio = np.divide(rh, den, out=np.ones_like(rh), where=nz)
        neg = ratio < 0
        hits += int((~nz).sum()) + int(neg.sum())
        ups = np.where(neg, 0.0, ups * np.sqrt(np.where(neg, 0.0, ratio)))
    return ups, h, hits


def polar_factor(m: np.ndarray) -> np.ndarray:
    """The orthogonal factor of M's polar decomposition, U V^T for the SVD
    M = U S V^T: the orthogonal Phi that minimises ||A Phi - B||_F when
    M = A^T B (orthogonal Procrustes).

    Reading: an empty cluster leaves a zero column in M, and the factor is
    then not unique; the polar factor of the nonzero columns is taken, with
    the empty cluster's column zero (the partial isometry, which leaves that
    column zero as the literal update does); M = 0 gives Phi = 0.  M is taken
    to have full rank on its nonzero columns."""
    m = np.asarray(m, dtype=np.float64)
    phi = np.zeros_like(m)
    nz = np.any(m != 0.0, axis=0)
    if nz.any():
        u, _, vt = np.linalg.svd(m[:, nz], full_matrices=False)
        phi[:, nz] = u @ vt
    return phi


def nci(ups: np.ndarray, t_g: int, variant: str = "literal"):
    """Phi = I; t_g times: l* = argmax_l (Ups Phi)[i, l] per row, Y one-hot,
    columns of Y scaled to unit L2 norm, Phi <- Ups^T Y (Algorithm 3, Eqs.
    ell-ast, Y-update, y-norm).

    variant "procrustes": Phi <- the polar factor of Ups^T Y instead, the
    minimiser over orthogonal Phi of ||Ups Phi - Y|| that Section 3.4 says the
    update solves (Ups^T Y itself is not orthogonal).

    Readings: ties go to the lowest cluster index (numpy.argmax); an empty
    column of Y stays zero; the labels are those of the last argmax; with
    t_g = 0 they are argmax of Ups itself.  Returns (labels int64, Phi).
    """
    if variant not in ("literal", "procrustes"):
        raise ValueError("variant is 'literal' or 'procrustes'")
    ups = np.asarray(ups, dtype=np.float64)
    n, k = ups.shape
    phi = np.eye(k)
    labels = np.argmax(ups, axis=1)
    for _ in range(t_g):
        labels = np.argmax(ups @ phi, axis=1)
        y = np.zeros((n, k))
        y[np.arange(n), labels] = 1.0
        cnt = y.sum(axis=0)
        scale = np.zeros(k)
        scale[cnt > 0] = 1.0 / np.sqrt(cnt[cnt > 0])
        y *= scale[None, :]
        phi = ups.T @ y
        if variant == "procrustes":
            phi = polar_factor(phi)
    return labels.astype(np.int64), phi


# ---------------------------------------------------------------------------
# Eq. obj1 (the k-ABGC objective) with s(u_i, u_j) ~ R[i] . R[j]
# ---------------------------------------------------------------------------
def objective(r: np.ndarray, labels: np.ndarray, k: int) -> tuple[float, float]:
    """obj1 = sum_l (1/|C_l|) sum_{i in C_l, j not in C_l} R[i].R[j]
    = sum_l c_l . (tot - c_l) / |C_l| with c_l the sum of R over C_l and tot the
    sum over all rows (Eq. obj1 with s ~ R R^T).  Also returns the trace form
    Tr(Y^T R R^T Y) = sum_l ||c_l||^2 / |C_l| (Lemma obj2, Eq. J-YRRY).
    Empty clusters contribute 0."""
    r = np.asarray(r, dtype=np.float64)
    labels = np.asarray(labels)
    tot = r.sum(axis=0)
    obj = 0.0
    tr = 0.0
    for ell in range(k):
        mask = labels == ell
        sz = int(mask.sum())
        if sz == 0:
            continue
        c = r[mask].sum(axis=0)
        obj += float(c @ (tot - c)) / sz
        tr += float(c @ c) / sz
    return obj, tr


def objective_bruteforce(s: np.ndarray, labels: np.ndarray, k: int) -> float:
    """Eq. obj1 summed pair by pair over a dense affinity matrix (tiny n)."""
    labels = np.asarray(labels)
    total = 0.0
    for ell in range(k):
        inside = np.where(labels == ell)[0]
        if inside.size == 0:
            continue
        outside = np.where(labels != ell)[0]
        acc = 0.0
        for i in inside:
            for j in outside:
                acc += s[i, j]
        total += acc / inside.size
    return total


# ---------------------------------------------------------------------------
# The whole pipeline (Section 3.1: Algorithms 1, 2, 3 in order)
# ---------------------------------------------------------------------------
@dataclass
class OracleResult:
    labels: np.ndarray
    objective: float
    trace: float
    b: sp.csr_matrix = None
    x_prime: np.ndarray = None
    psi_d: np.ndarray = None
    z: np.ndarray = None
    zhat: np.ndarray = None
    q: np.ndarray = None
    r: np.ndarray = None
    gamma: np.ndarray = None
    sigma: np.ndarray = None
    psi: np.ndarray = None
    ups: np.ndarray = None
    h: np.ndarray = None
    phi: np.ndarray = None
    guard_hits: int = 0
    times: dict = field(default_factory=dict)


def tpo(n_u, n_v, edge_u, edge_v, x, *, k, alpha, gamma, g, omega,
        omega_r=None, d=0, q=20, t_f=5, t_g=20, edge_w=None, nci_variant="literal") -> OracleResult:
    """TPO(G, k): optional reduction (Section 3.2.1), Algorithm 1, Algorithm 2,
    Algorithm 3, and Eq. obj1 of the result."""
    import time

    times = {}
    t0 = time.perf_counter()
    b = bipartite_adjacency(n_u, n_v, edge_u, edge_v, edge_w)
    times["ingest"] = time.perf_counter() - t0
    x64 = np.asarray(x, dtype=np.float64)
    d_u = x64.shape[1]
    psi_d = None
    t0 = time.perf_counter()
    if 0 < d < d_u:
        if omega_r is None:
            raise ValueError("reduction needs omega_r")
        xp, psi_d, _ = reduce_attributes(x64, d, omega_r, q)
    else:
        xp = x64
    times["reduce"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    z = propagate(b, xp, alpha, gamma)
    times["propagate"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    zhat = normalize_rows(z)
    qmat = orthogonal_from_gaussian(g)
    r, _, _ = random_features(zhat, qmat)
    times["features"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    gam, sig, psi = randomized_svd(r, k, omega, q)
    times["embed"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    ups, h, hits = onmf(r, gam, sig, psi, t_f)
    times["onmf"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    labels, phi = nci(ups, t_g, nci_variant)
    times["nci"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    obj, tr = objective(r, labels, k)
    times["objective"] = time.perf_counter() - t0
    return OracleResult(labels=labels, objective=obj, trace=tr, b=b, x_prime=xp,
                        psi_d=psi_d, z=z, zhat=zhat, q=qmat, r=r, gamma=gam,
                        sigma=sig, psi=psi, ups=ups, h=h, phi=phi,
                        guard_hits=hits, times=times)


# ---------------------------------------------------------------------------
# Comparison helpers used by the parity tests
# ---------------------------------------------------------------------------
def labels_match_up_to_permutation(a: np.ndarray, b: np.ndarray) -> bool:
    """True iff the contingency table of the two labelings is a permutation
    matrix on the labels that occur (a bijection of label values)."""
    a = np.asarray(a).astype(np.int64)
    b = np.asarray(b).astype(np.int64)
    if a.shape != b.shape:
        return False
    pairs = np.unique(np.stack([a, b], axis=1), axis=0)
    return (np.unique(pairs[:, 0]).size == pairs.shape[0]
            and np.unique(pairs[:, 1]).size == pairs.shape[0])


def subspace_sin_theta(a: np.ndarray, b: np.ndarray) -> float:
    """Largest principal-angle sine between range(a) and range(b) of equal
    dimension, as the 2-norm of the part of b's basis outside range(a)."""
    qa = orthonormal_basis(np.asarray(a, dtype=np.float64))
    qb = orthonormal_basis(np.asarray(b, dtype=np.float64))
    return float(np.linalg.norm(qb - qa @ (qa.T @ qb), 2))
