"""The sparse-attribute precision form (TPO_X_CSR) against the FP64 oracle:
sparse TF-IDF rows (abg_synth.tfidf_csr: 4,096 columns, 2% of the words
drawn per row, log-normal weights, unit rows) of a planted-partition graph
with k = 50, reduced to d = 64 (Section 3.2.1, Eq. Xd).

The device stages the rows as FP8 E4M3 codes with per-column scales, forms
the Gram on FP8 MFMA, iterates on it, and refines: the Rayleigh-Ritz product
is taken with the exact FP32 values.  Checked here:
* the device Gram against the FP64 Gram of the E4M3-encoded values (the codes
  come from torch's encoder, which the CPU tests pin to the library's), entry
  by entry within 256 u of each entry's magnitude sum (FP32 sums of 256-row
  blocks of exact products, added in FP64);
* Psi_d against the oracle's basis iterated on the device Gram with the
  Rayleigh-Ritz step on the exact Gram (oracle.top_d_gram_basis with
  c_final), and X' = X Psi_d from the exact values;
* every later stage against the oracle run from that X', and the decisions
  on the device's own inputs;
* end to end against the FP64 oracle on the exact attributes, with 0 to 4
  refinement steps: label agreement, objective difference and the Psi_d and
  Upsilon subspace angles, reported.
"""
import numpy as np
import pytest

import abg_synth as synth
import oracle
from tests.gpu_harness import log, rel_fro, row_rel_max

pytestmark = pytest.mark.gpu

N_U, N_V, E, K, D_U = 12_000, 18_000, 180_000, 50, 4096
KW = dict(k=K, alpha=0.5, gamma=5, d=64, q=20, oversample=10, t_f=5, t_g=20)


@pytest.fixture(scope="module")
def job():
    import torch

    abg = synth.planted_abg(N_U, N_V, E, K, 1, zipf_a=2.0, seed=5)
    rowptr, col, val = synth.tfidf_csr(torch.from_numpy(abg.labels_u), D_U, device="cpu", seed=5)
    x = np.zeros((N_U, D_U), np.float64)
    rows = np.repeat(np.arange(N_U), np.diff(rowptr.numpy()))
    x[rows, col.numpy()] = val.numpy()
    log(f"[csr] n_u={N_U} n_v={N_V} E={abg.n_edges} d_u={D_U} nnz={int(rowptr[-1])}")
    return abg, (rowptr, col, val), x


def _run(abg, csr, x_refine=1):
    import torch

    import paper_2405_11922_amd as tpo

    dev = torch.device("cuda:0")
    rowptr, col, val = (t.to(dev) for t in csr)
    xs = tpo.CsrX(rowptr, col, val, D_U)
    eu = torch.from_numpy(abg.edge_u).to(dev)
    ev = torch.from_numpy(abg.edge_v).to(dev)
    plan = tpo.Plan.create(abg.n_u, abg.n_v, abg.n_edges, D_U, device=dev, x_dtype="csr", x_nnz=xs.nnz,
                           x_refine=x_refine, seed=0, **KW)
    try:
        labels = torch.empty(abg.n_u, dtype=torch.int32, device=dev)
        emb = torch.empty(abg.n_u, K, dtype=torch.float32, device=dev)
        obj = tpo.tpo_execute(plan.handle, eu, ev, xs, plan.workspace, labels, emb)
        torch.cuda.synchronize()
        out = {name: plan.buffer(name).cpu().numpy() for name in
               ("gram_c", "colsum_x", "psi_d", "xprime", "z", "r", "gamma", "upsilon")}
        out["labels"] = labels.cpu().numpy()
        out["objective"] = obj
    finally:
        plan.close()
    return out


def _oracle_from(abg, xprime, mm):
    """The oracle's pipeline from a given X' (reduction off on X' itself)."""
    return oracle.tpo(abg.n_u, abg.n_v, abg.edge_u, abg.edge_v, xprime, k=K, alpha=KW["alpha"], gamma=KW["gamma"],
                      g=mm.g, omega=mm.omega, d=0, q=KW["q"], t_f=KW["t_f"], t_g=KW["t_g"])


def test_csr_form_against_oracle(job):
    import torch

    abg, csr, x = job
    mm = synth.method_matrices(0, D_U, KW["d"], K, KW["oversample"])
    out = _run(abg, csr)
    d = KW["d"]
    # the Gram of the encoded values (scales as the device forms them)
    xf = x.astype(np.float32)
    amax = np.abs(xf).max(axis=0)
    scale = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    q = torch.from_numpy(xf / scale[None, :]).clamp(-448.0, 448.0).to(torch.float8_e4m3fn)
    xq = q.to(torch.float64).numpy() * scale.astype(np.float64)[None, :]
    c_q = xq.T @ xq
    bound = 256 * 2.0 ** -24 * (np.abs(xq).T @ np.abs(xq)) + 1e-300
    e_gram = float(np.max(np.abs(out["gram_c"] - c_q) / bound))
    c_exact = x.T @ x
    log(f"[csr] Gram of the E4M3 values: largest error {e_gram:.2f} of the 256u bound; the FP8 Gram differs from the "
        f"exact one by {np.linalg.norm(c_q - c_exact) / np.linalg.norm(c_exact):.2e} (Frobenius, relative)")
    assert e_gram <= 1.0
    assert np.allclose(out["colsum_x"], x.sum(0), rtol=1e-12, atol=1e-12)
    # Psi_d: iterations on the device Gram, Rayleigh-Ritz with the exact Gram
    psi_ref, _ = oracle.top_d_gram_basis(out["gram_c"], x.sum(0), N_U, d, mm.omega_reduce, KW["q"], c_final=c_exact)
    e_psi = float(np.max(np.abs(out["psi_d"] - psi_ref)))
    xp = out["xprime"][:, :d]
    e_xp = rel_fro(xp, x @ out["psi_d"])
    log(f"[csr] Psi_d vs the oracle's refined basis {e_psi:.2e}; X' = X Psi_d {e_xp:.2e}")
    assert e_psi < 1e-6
    assert e_xp < 1e-6
    # later stages from the device's X'
    ref = _oracle_from(abg, xp.astype(np.float64), mm)
    e_z = row_rel_max(out["z"][:, :d], ref.z)
    e_r = rel_fro(out["r"], ref.r)
    sin_u = oracle.subspace_sin_theta(out["upsilon"], ref.ups)
    log(f"[csr] from the device X': Z {e_z:.2e}  R {e_r:.2e}  sin(Ups) {sin_u:.2e}")
    assert e_z < 2e-5 and e_r < 2e-5 and sin_u < 1e-4
    lab, _ = oracle.nci(out["upsilon"], KW["t_g"])
    assert np.array_equal(out["labels"], lab)
    assert oracle.labels_match_up_to_permutation(out["labels"], ref.labels)


def test_csr_form_error_against_fp64_oracle(job):
    """End to end against the oracle on the exact attributes, with 0, 1, 2
    and 4 refinement steps (reported; with the default single step the labels
    must agree on nearly every row)."""
    abg, csr, x = job
    mm = synth.method_matrices(0, D_U, KW["d"], K, KW["oversample"])
    ref = oracle.tpo(abg.n_u, abg.n_v, abg.edge_u, abg.edge_v, x, k=K, alpha=KW["alpha"], gamma=KW["gamma"],
                     g=mm.g, omega=mm.omega, omega_r=mm.omega_reduce, d=KW["d"], q=KW["q"], t_f=KW["t_f"],
                     t_g=KW["t_g"])
    from scipy.optimize import linear_sum_assignment

    res = {}
    for refine in (1, 0, 2, 4):
        out = _run(abg, csr, refine)
        table = np.zeros((K, K), np.int64)
        np.add.at(table, (out["labels"].astype(np.int64), ref.labels.astype(np.int64)), 1)
        r, c = linear_sum_assignment(-table)
        agree = table[r, c].sum() / N_U
        rel = abs(out["objective"][0] - ref.objective) / abs(ref.objective)
        sin_psi = oracle.subspace_sin_theta(out["psi_d"], ref.psi_d)
        sin_u = oracle.subspace_sin_theta(out["upsilon"], ref.ups)
        res[refine] = (agree, rel, sin_psi, sin_u)
        log(f"[csr] vs the FP64 oracle on the exact attributes, x_refine={refine}: label agreement {agree:.6f}, "
            f"objective rel err {rel:.2e}, Psi_d sin theta {sin_psi:.2e}, Upsilon sin theta {sin_u:.2e}")
    assert res[1][0] >= 0.99
