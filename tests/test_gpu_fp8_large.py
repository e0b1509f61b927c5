"""The FP8 TF-IDF workload at its full size on the GPU: |U| = |V| =
2,000,000, 60M distinct edges from the degree-corrected SBM (k = 50), 4,096
sparse TF-IDF attribute columns (2% density) handed over as FP8 E4M3 codes
with one scale per column, reduced to d = 64, 10 hops.

The oracle cannot run this job in test time; the device result is checked
through what holds at any size:
* the attribute Gram C = X^T X of the FP8 MFMA kernel, entry by entry,
  against an FP64 Gram of the decoded attributes (computed on the GPU with
  torch): X >= 0, so each entry's FP32 sums over 256-row blocks are within
  256 u of the entry itself (u = 2^-24); the column sums of X to FP64
  rounding (the kernel sums the codes exactly in FP32 groups of 64 rows);
* Psi_d is orthonormal and X' = X Psi_d on sampled rows;
* the NCI labels are the oracle's NCI run on the device's Upsilon, and the
  objective is the oracle's objective of the device's labels on the device's R.
"""
import time

import numpy as np
import pytest

import abg_synth as synth
import oracle
from tests.gpu_harness import log

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SAMPLE = 2000


def test_fp8_workload_properties():
    import torch

    import paper_2405_11922_amd as tpo

    dev = torch.device("cuda:0")
    shape = synth.CONFIGS["fp8_tfidf"]
    n, m, E, k, du = shape.n_u, shape.n_v, shape.n_edges, shape.k, shape.d_u
    t0 = time.time()
    eu, ev, _, truth, _ = synth.planted_abg_device(n, m, E, k, 1, device=dev, zipf_a=shape.zipf_a,
                                                   sigma=shape.sigma, in_out_ratio=shape.in_out_ratio,
                                                   max_degree=shape.max_degree, seed=0)
    codes, scale = synth.tfidf_fp8_device(truth, du, device=dev, seed=0)
    x8 = codes.view(torch.float8_e4m3fn)
    torch.cuda.synchronize()
    log(f"[fp8 full] generated n_u={n} n_v={m} E={E} d_u={du} in {time.time() - t0:.1f}s")
    plan = tpo.Plan.create(n, m, E, du, device=dev, k=k, alpha=shape.alpha, gamma=shape.gamma, d=shape.d,
                           q=shape.q, oversample=shape.oversample, t_f=shape.t_f, t_g=shape.t_g, seed=0,
                           x_dtype="fp8")
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    t0 = time.time()
    obj = tpo.tpo_execute(plan.handle, eu, ev, x8, plan.workspace, labels, x_scale=scale)
    torch.cuda.synchronize()
    log(f"[fp8 full] tpo_execute {1e3 * (time.time() - t0):.1f} ms, objective {obj[0]:.6g}")

    def buf(name):
        return tpo.tpo_plan_buffer(plan.handle, plan.workspace, name)

    # the Gram of the decoded attributes in FP64 (X >= 0 for TF-IDF rows)
    sc = scale.double()
    c_ref = torch.zeros(du, du, dtype=torch.float64, device=dev)
    cs_ref = torch.zeros(du, dtype=torch.float64, device=dev)
    for r0 in range(0, n, 125_000):
        xd = x8[r0:r0 + 125_000].double() * sc[None, :]
        assert bool((xd >= 0).all())
        c_ref += xd.T @ xd
        cs_ref += xd.sum(0)
        del xd
    c_dev = buf("gram_c")
    diff = c_dev - c_ref
    nz = c_ref > 0
    log(f"[fp8 full] Gram entries below / above the FP64 value: {float((diff[nz] < 0).double().mean()):.3f} / "
        f"{float((diff[nz] > 0).double().mean()):.3f}; mean signed rel err "
        f"{float((diff[nz] / c_ref[nz]).mean()):.2e}")
    err = diff.abs()
    bound = 256.0 * 2.0 ** -24 * c_ref * 1.01 + 1e-300
    worst = float((err / bound).max())
    log(f"[fp8 full] Gram: max |C - C_fp64| / (256 u C) = {worst:.3f}, max rel {float((err / c_ref.clamp_min(1e-300)).max()):.2e}")
    assert worst <= 1.0
    e_cs = float(((buf("colsum_x") - cs_ref).abs() / cs_ref.abs().clamp_min(1e-300)).max())
    log(f"[fp8 full] column sums of X: max rel err {e_cs:.2e}")
    assert e_cs < 1e-12
    del c_ref, err, bound

    # reduction basis and projection on sampled rows
    psi = buf("psi_d").cpu().numpy()
    d = psi.shape[1]
    assert np.max(np.abs(psi.T @ psi - np.eye(d))) < 1e-10
    su = np.sort(np.random.default_rng(1).choice(n, SAMPLE, replace=False))
    idx = torch.from_numpy(su).to(dev)
    xs = (x8[idx].double() * sc[None, :]).cpu().numpy()
    xp = buf("xprime")[idx].cpu().numpy()[:, :d]
    ref = xs @ psi
    e_xp = float(np.linalg.norm(xp - ref) / np.linalg.norm(ref))
    log(f"[fp8 full] Psi_d orthonormal; X' on sampled rows rel err {e_xp:.2e}")
    assert e_xp < 2e-5

    # decisions on the device's own inputs
    ups = buf("upsilon").cpu().numpy()
    assert np.all(np.isfinite(ups))
    lab_ref, _ = oracle.nci(ups, shape.t_g)
    lab = labels.cpu().numpy()
    assert np.array_equal(lab, lab_ref)
    o, tr = oracle.objective(buf("r").cpu().numpy(), lab, k)
    rel = abs(obj[0] - o) / abs(o)
    rel_t = abs(obj[1] - tr) / abs(tr)
    log(f"[fp8 full] NCI labels identical to the oracle's on device Upsilon; objective rel err {rel:.2e} / {rel_t:.2e}")
    assert rel < 1e-9 and rel_t < 1e-9
    plan.close()
