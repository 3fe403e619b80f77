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


@pytest.fixture(scope="module")
def trained():
    """CZT data of the surrogate aperture (4096 training, 512 validation and 512
    test solves), a two-member ensemble trained by the library's kernels, and its
    gate calibrated on the validation solves."""
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
    x_all = torch.from_numpy(f_all).cuda()
    x_te = torch.from_numpy(f_te).cuda()
    S = SG.Surrogate(w)
    S.init(t_sample=t_all[:1024])
    t0 = time.perf_counter()
    losses = S.fit(x_all[:n_tr], t_all[:n_tr], epochs=30, log=None)
    torch.cuda.synchronize()
    announce(f"training 2 x 30 epochs: {time.perf_counter() - t0:.1f} s, loss {losses[0][0]:.4f} -> "
             f"{losses[0][-1]:.4f} / {losses[1][0]:.4f} -> {losses[1][-1]:.4f}")
    fw_val = S.reader.fwhm(t_all[n_tr:])
    cal = S.calibrate(x_all[n_tr:], fw_val, f_all[n_tr:])
    announce(f"gate calibration on validation: {cal}")
    fw_te = S.reader.fwhm(t_te)
    acc, y, f_pred, dis = S.accept(x_te, f_te)
    err = np.abs(f_pred / fw_te - 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        S.predict(x_te)
    torch.cuda.synchronize()
    net_per_case = (time.perf_counter() - t0) / (3 * n_te)   # both members
    frac = float(acc.mean())
    mixed = net_per_case + (1.0 - frac) * czt_per_case
    announce(f"test: accepted {frac * 100:.1f} %, FWHM error accepted max "
             f"{(err[acc].max() if acc.any() else 0) * 100:.3f} %, all cases median {np.median(err) * 100:.3f} %; "
             f"network {net_per_case * 1e6:.1f} us per case vs CZT {czt_per_case * 1e3:.2f} ms; "
             f"gain with fallback x{czt_per_case / mixed:.3f}")
    return dict(w=w, S=S, solver=solver, losses=losses, cal=cal, acc=acc, err=err, frac=frac,
                cr_te=cr_te, f_te=f_te, czt_per_case=czt_per_case, net_per_case=net_per_case,
                gain=czt_per_case / mixed)


def test_surrogate_trains_and_gate_is_calibrated(trained):
    """Training reduces both members' loss; the calibrated gate keeps every
    accepted validation case within the FWHM target; an input outside the
    training box is never accepted and the CZT answers it."""
    for ls in trained["losses"]:
        assert ls[-1] < 0.95 * ls[0]
    assert trained["cal"]["max_err_accepted"] <= 0.005
    assert 0.0 <= trained["cal"]["tau"] <= 0.0025
    S, w = trained["S"], trained["w"]
    cr_out, lam_out = trained["cr_te"][:4].copy(), np.full(4, 900e-9)
    f_out = SG.features(cr_out, lam_out, w["D"], w["lambda0"])
    acc_out, _, _, _ = S.accept(torch.from_numpy(f_out).cuda(), f_out)
    assert not acc_out.any()
    t_out, _ = trained["solver"].solve(cr_out, lam_out)
    assert torch.isfinite(t_out).all()
    # one network evaluation (both members) costs far less than one CZT solve:
    # the gain available to an accepted case
    assert trained["czt_per_case"] / trained["net_per_case"] > 20


@pytest.mark.xfail(strict=True, reason=(
    "measured: at the configured deformations (8 creases up to lambda0/2) the gate accepts no test "
    "case (the network's FWHM error, median ~9 %, does not beat a constant prediction), so every case "
    "falls back to the CZT and the gain with fallback is x1.0"))
def test_surrogate_gains_over_czt(trained):
    """What the trained network gains over solving every case by CZT: a share of
    the held-out cases accepted, each within 0.5 % of the CZT's FWHM, and an
    end-to-end speed-up that includes the fallback solves."""
    assert trained["frac"] >= 0.05
    assert trained["err"][trained["acc"]].max() <= 0.005
    assert trained["gain"] > 1.05
