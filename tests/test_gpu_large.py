"""The 150M-edge workload at its full size on the GPU: |U| = 5,000,000,
|V| = 10,000,000, 150M distinct edges from the degree-corrected SBM (k = 100,
Zipf(1.9) degree weights, largest expected degree 1e5), attributes
5,000,000 x 512 reduced to d = 64, 10 hops.

The FP64 oracle cannot run this job in test time, so the device result is
checked through what holds at any size:
* the CSR of B_U and of its transpose equal a sort of the edge list (exact);
* Psi_d is the oracle's reduction basis (the randomized subspace iteration
  and Rayleigh-Ritz step of Section 3.2.1) computed in FP64 from the device's
  own Gram C and column sums, and X' = X Psi_d on sampled rows; the distance
  of Psi_d from C's exact top-d eigenvectors and the gap sigma_d/sigma_{d+1}
  are logged (the randomized basis is the method's, reading A14);
* the last hop of the propagation (both SpMMs) on sampled rows, from the
  device's own W and T; the samples include the 100 rows of most neighbours
  on each side (hub rows, whose sums run through ~400 chunk partials);
* the random features on sampled rows and the column sums r over all rows;
* Gamma has orthonormal columns and R^T Gamma = Psi Sigma;
* the NCI labels are the oracle's NCI run on the device's Upsilon, and the
  objective is the oracle's objective of the device's labels on the device's R.
The input is drawn on the GPU (abg_synth.planted_abg_device).  The job runs
twice: with X in FP32, and in the precision form with X stored as bfloat16
(the BF16 MFMA Gram); the checks take X at the precision the job saw.
"""
import math

import numpy as np
import pytest

import abg_synth as synth
import oracle
from tests.gpu_harness import log

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SAMPLE = 2000


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("x_dtype", ["f32", "bf16"])
def test_large_workload_properties(x_dtype):
    import time

    import torch

    import paper_2405_11922_amd as tpo

    dev = torch.device("cuda:0")
    shape = synth.CONFIGS["large"]
    n, m, E, k = shape.n_u, shape.n_v, shape.n_edges, shape.k
    t0 = time.time()
    eu, ev, x, _, _ = synth.planted_abg_device(n, m, E, k, shape.d_u, device=dev, zipf_a=shape.zipf_a,
                                               sigma=shape.sigma, in_out_ratio=shape.in_out_ratio,
                                               max_degree=shape.max_degree, seed=0)
    torch.cuda.synchronize()
    log(f"[large {x_dtype}] generated n_u={n} n_v={m} E={E} d_u={shape.d_u} in {time.time() - t0:.1f}s")
    if x_dtype == "bf16":
        x = x.to(torch.bfloat16)
    plan = tpo.Plan.create(n, m, E, shape.d_u, device=dev, k=k, alpha=shape.alpha, gamma=shape.gamma, d=shape.d,
                           q=shape.q, oversample=shape.oversample, t_f=shape.t_f, t_g=shape.t_g, seed=0,
                           x_dtype=x_dtype)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    t0 = time.time()
    obj = tpo.tpo_execute(plan.handle, eu, ev, x, plan.workspace, labels)
    torch.cuda.synchronize()
    log(f"[large {x_dtype}] tpo_execute {1e3 * (time.time() - t0):.1f} ms, objective {obj[0]:.6g}")
    st = tpo.tpo_plan_stats(plan.handle)
    assert st["n_unique_edges"] == E

    def buf(name):
        return tpo.tpo_plan_buffer(plan.handle, plan.workspace, name)

    # CSR structure (exact)
    key = torch.sort(eu.long() * m + ev.long()).values
    cnt = torch.bincount(eu.long(), minlength=n)
    rp = buf("rowptr_u").long()
    assert int(rp[0]) == 0 and torch.equal(rp[1:], torch.cumsum(cnt, 0))
    assert torch.equal(buf("col_u")[:E].long(), key % m)
    key = torch.sort(ev.long() * n + eu.long()).values
    cnt = torch.bincount(ev.long(), minlength=m)
    rp = buf("rowptr_v").long()
    assert int(rp[0]) == 0 and torch.equal(rp[1:], torch.cumsum(cnt, 0))
    assert torch.equal(buf("col_v")[:E].long(), key % n)
    del key, cnt, rp
    log(f"[large {x_dtype}] CSR of B_U and B_U^T exact")

    rng = np.random.default_rng(1)
    deg_u = torch.diff(buf("rowptr_u").long())
    deg_v = torch.diff(buf("rowptr_v").long())
    top_u = torch.topk(deg_u, 100).indices.cpu().numpy()
    top_v = torch.topk(deg_v, 100).indices.cpu().numpy()
    log(f"[large {x_dtype}] sampled hub rows: neighbours {int(deg_u[top_u[0]])}..{int(deg_u[top_u[-1]])} (U), "
        f"{int(deg_v[top_v[0]])}..{int(deg_v[top_v[-1]])} (V)")
    su = np.unique(np.concatenate([rng.choice(n, SAMPLE, replace=False), top_u]))
    sv = np.unique(np.concatenate([rng.choice(m, SAMPLE, replace=False), top_v]))

    # attribute reduction: the oracle's basis from the device's own Gram
    psi = buf("psi_d").cpu().numpy()
    d = psi.shape[1]
    assert np.max(np.abs(psi.T @ psi - np.eye(d))) < 1e-10
    c_dev = buf("gram_c").cpu().numpy()
    mm = synth.method_matrices(0, shape.d_u, shape.d, k, shape.oversample)
    psi_ref, _ = oracle.top_d_gram_basis(c_dev, buf("colsum_x").cpu().numpy(), n, d, mm.omega_reduce, shape.q)
    e_psi = float(np.max(np.abs(psi - psi_ref)))
    lam, vec = np.linalg.eigh(0.5 * (c_dev + c_dev.T))
    lam, vec = lam[::-1], vec[:, ::-1]
    sin_exact = oracle.subspace_sin_theta(psi, vec[:, :d])
    log(f"[large {x_dtype}] Psi_d vs the oracle's basis from the device Gram: max abs err {e_psi:.2e}; "
        f"vs C's exact top-{d} eigenvectors sin theta {sin_exact:.2e}, sigma_d/sigma_(d+1) "
        f"{math.sqrt(lam[d - 1] / lam[d]):.5f}")
    assert e_psi < 1e-6
    xs = x[torch.from_numpy(su).to(dev)].double().cpu().numpy()
    xp = buf("xprime")[torch.from_numpy(su).to(dev)].cpu().numpy()[:, :d]
    e_xp = _rel(xp, xs @ psi)
    log(f"[large {x_dtype}] Psi_d orthonormal; X' on sampled rows rel err {e_xp:.2e}")
    assert e_xp < 2e-5

    # last hop of the propagation, from the device's own W and T
    alpha = shape.alpha
    rowptr_u = buf("rowptr_u").cpu().numpy().astype(np.int64)
    col_u = buf("col_u").cpu().numpy()
    rowptr_v = buf("rowptr_v").cpu().numpy().astype(np.int64)
    col_v = buf("col_v").cpu().numpy()
    scu = buf("scale_u").cpu().numpy().astype(np.float64)
    scv = buf("scale_v").cpu().numpy().astype(np.float64)
    w = buf("w_last")
    t = buf("t")
    z = buf("z")
    e_t = 0.0
    for v in sv:
        nb = torch.from_numpy(col_v[rowptr_v[v]:rowptr_v[v + 1]].astype(np.int64)).to(dev)
        ref = scv[v] * w[nb].double().sum(0).cpu().numpy()
        got = t[int(v)].double().cpu().numpy()
        e_t = max(e_t, float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30)))
    e_z = 0.0
    for u in su:
        nb = torch.from_numpy(col_u[rowptr_u[u]:rowptr_u[u + 1]].astype(np.int64)).to(dev)
        acc = t[nb].double().sum(0).cpu().numpy() if nb.numel() else 0.0
        ref = (1.0 - alpha) * (buf("xprime")[int(u)].double().cpu().numpy() + alpha * scu[u] * acc)
        got = z[int(u)].double().cpu().numpy()
        e_z = max(e_z, float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30)))
    log(f"[large {x_dtype}] last hop on sampled rows: T rel err {e_t:.2e}, Z rel err {e_z:.2e}")
    assert e_t < 1e-5 and e_z < 1e-5

    # random features: sampled rows, and r over all rows (FP64 on the GPU)
    q = torch.from_numpy(buf("q").cpu().numpy()).to(dev)
    rsum = buf("rsum").cpu().numpy()
    amp = math.sqrt(math.e / d)
    r_all = torch.zeros(2 * d, dtype=torch.float64, device=dev)
    for c0 in range(0, n, 500_000):
        zc = z[c0:c0 + 500_000, :d].double()
        zh = zc / zc.norm(dim=1, keepdim=True).clamp_min(1e-300)
        a = math.sqrt(d) * (zh @ q.T)
        r_all += amp * torch.cat([torch.sin(a), torch.cos(a)], dim=1).sum(0)
    e_r = _rel(rsum, r_all.cpu().numpy())
    zs = z[torch.from_numpy(su).to(dev), :d].double()
    zh = zs / zs.norm(dim=1, keepdim=True)
    a = math.sqrt(d) * (zh @ q.T)
    rp_ = amp * torch.cat([torch.sin(a), torch.cos(a)], dim=1)
    ref = (rp_ / torch.sqrt(rp_ @ torch.from_numpy(rsum).to(dev))[:, None]).cpu().numpy()
    R = buf("r")
    e_rr = _rel(R[torch.from_numpy(su).to(dev)].double().cpu().numpy(), ref)
    log(f"[large {x_dtype}] features: r rel err {e_r:.2e}, sampled R rel err {e_rr:.2e}")
    assert e_r < 1e-6 and e_rr < 2e-5

    # embedding: orthonormal Gamma and R^T Gamma = Psi Sigma (FP64 on the GPU)
    gam = buf("gamma")
    gtg = torch.zeros(k, k, dtype=torch.float64, device=dev)
    rtg = torch.zeros(2 * d, k, dtype=torch.float64, device=dev)
    for c0 in range(0, n, 500_000):
        g = gam[c0:c0 + 500_000].double()
        gtg += g.T @ g
        rtg += R[c0:c0 + 500_000].double().T @ g
    sig = buf("sigma").cpu().numpy()
    psi_e = buf("psi").cpu().numpy()
    e_o = float(np.max(np.abs(gtg.cpu().numpy() - np.eye(k))))
    e_b = _rel(rtg.cpu().numpy(), psi_e * sig[None, :])
    log(f"[large {x_dtype}] embedding: |Gamma^T Gamma - I| {e_o:.2e}, R^T Gamma vs Psi Sigma rel {e_b:.2e}")
    assert e_o < 1e-4 and e_b < 1e-4
    assert np.all(np.diff(sig) <= 1e-12 * sig[0])

    # decisions on the device's own inputs
    ups = buf("upsilon").cpu().numpy()
    assert np.all(np.isfinite(ups))
    t0 = time.time()
    lab_ref, _ = oracle.nci(ups, shape.t_g)
    lab = labels.cpu().numpy()
    log(f"[large {x_dtype}] oracle NCI on device Upsilon in {time.time() - t0:.1f}s")
    assert np.array_equal(lab, lab_ref)
    o, tr = oracle.objective(R.cpu().numpy(), lab, k)
    rel = abs(obj[0] - o) / abs(o)
    rel_t = abs(obj[1] - tr) / abs(tr)
    log(f"[large {x_dtype}] objective vs oracle objective of device labels: {rel:.2e} / {rel_t:.2e}")
    assert rel < 1e-9 and rel_t < 1e-9
    plan.close()
