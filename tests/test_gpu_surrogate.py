"""GPU: the learned surrogate end to end at the surrogate workload's aperture
(D = 10 mm, f/5, N = 16384, ROI 128^2) on a reduced data set: CZT targets,
training by the library's kernels, the calibrated ensemble gate, the CZT
fallback, and what the network gains over solving every case by CZT.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2609_01978_amd as P  # noqa: E402
from paper_2609_01978_amd import surrogate as SG  # noqa: E402
from oracle import fzp_oracle as O  # noqa: E402
from fzp_inputs import surrogate_draws, workload  # noqa: E402

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-surrogate] {msg}", flush=True)


def test_targets_match_fp64_path():
    """Split-path targets of two deformed instances against the FP64 path."""
    w = workload("surrogate")
    cr, lam = surrogate_draws(99, 2, w["D"], w["lambda0"])
    t_split, _ = SG.CZTSolver(w).solve(cr, lam)
    t_fp64, _ = SG.CZTSolver(w, path="fp64").solve(cr, lam)
    a = np.exp(t_split.cpu().numpy().astype(np.float64))
    b = np.exp(t_fp64.cpu().numpy().astype(np.float64))
    for k in range(2):
        e = float(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k]))
        announce(f"target {k} rel-L2 (intensity) {e:.2e}")
        assert e <= 1e-4


def test_surrogate_gate_and_gain():
    w = workload("surrogate")
    n_tr, n_val, n_te = 4096, 512, 512
    cr_tr, lam_tr = surrogate_draws(w["train_seed"], n_tr + n_val, w["D"], w["lambda0"])
    cr_te, lam_te = surrogate_draws(w["test_seed"], n_te, w["D"], w["lambda0"])
    solver = SG.CZTSolver(w)
    t_all, sec_all = solver.solve(cr_tr, lam_tr)
    t_te, sec_te = solver.solve(cr_te, lam_te)
    czt_per_case = (sec_all + sec_te) / (n_tr + n_val + n_te)
    announce(f"CZT data: {n_tr + n_val + n_te} solves, {czt_per_case * 1e3:.2f} ms per solve")
    f_all = SG.features(cr_tr, lam_tr, w["D"], w["lambda0"])
    f_te = SG.features(cr_te, lam_te, w["D"], w["lambda0"])
    assert SG.in_training_box(f_all).all() and SG.in_training_box(f_te).all()
    x_all = torch.from_numpy(f_all).cuda()
    x_te = torch.from_numpy(f_te).cuda()
    x_tr, t_tr = x_all[:n_tr], t_all[:n_tr]
    x_val, t_val = x_all[n_tr:], t_all[n_tr:]

    S = SG.Surrogate(w)
    S.init(t_sample=t_tr[:1024])
    t0 = time.perf_counter()
    losses = S.fit(x_tr, t_tr, epochs=30, log=None)
    torch.cuda.synchronize()
    announce(f"training 2 x 30 epochs: {time.perf_counter() - t0:.1f} s, loss {losses[0][0]:.4f} -> "
             f"{losses[0][-1]:.4f} / {losses[1][0]:.4f} -> {losses[1][-1]:.4f}")
    for ls in losses:
        assert ls[-1] < 0.95 * ls[0]

    fw_val = S.reader.fwhm(t_val)
    fw_te = S.reader.fwhm(t_te)
    cal = S.calibrate(x_val, fw_val, f_all[n_tr:])
    announce(f"gate calibration on validation: {cal}")
    acc, y, f_pred, dis = S.accept(x_te, f_te)
    err = np.abs(f_pred / fw_te - 1.0)
    announce(f"test: accepted {acc.mean() * 100:.1f} %, FWHM error accepted max "
             f"{(err[acc].max() if acc.any() else 0) * 100:.3f} %, all cases median {np.median(err) * 100:.3f} %")
    # accepted predictions meet the FWHM target; the rest go to the CZT
    assert (not acc.any()) or err[acc].max() <= 0.005

    # inference cost per case vs one CZT solve
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        S.predict(x_te)
    torch.cuda.synchronize()
    net_per_case = (time.perf_counter() - t0) / (3 * n_te)   # both members
    announce(f"network {net_per_case * 1e6:.1f} us per case vs CZT {czt_per_case * 1e3:.2f} ms: "
             f"{czt_per_case / net_per_case:.0f}x")
    assert czt_per_case / net_per_case > 20

    # an input outside the training box is never accepted: the CZT answers it
    cr_out, lam_out = cr_te[:4].copy(), np.full(4, 900e-9)
    f_out = SG.features(cr_out, lam_out, w["D"], w["lambda0"])
    acc_out, _, _, _ = S.accept(torch.from_numpy(f_out).cuda(), f_out)
    assert not acc_out.any()
    t_out, _ = solver.solve(cr_out, lam_out)
    assert torch.isfinite(t_out).all()
