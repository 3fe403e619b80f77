"""GPU: the learned surrogate end to end at the surrogate workload's aperture
(D = 10 mm, f/5, N = 16384, ROI 128^2) on a reduced data set: CZT targets,
the physics prior (fzp_pupil_prior), training of the residual network by the
library's kernels, the calibrated ensemble gate with its conditioning checks
(fzp_fwhm_batch), the CZT fallback, and what the trained surrogate gains over
solving every case by CZT.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2609_01978_amd import surrogate as SG  # noqa: E402
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
def report():
    """SG.run on 12000 training, 2000 validation and 1000 test CZT solves,
    150 epochs: the prior, the residual ensemble, the gate calibrated on the
    validation solves, and the test-set report."""
    w = workload("surrogate")
    t0 = time.perf_counter()
    r = SG.run(w, 12000, 2000, 1000, 150, log=lambda m: announce(m) if ("gate" in m or "CZT" in m) else None)
    announce(f"run: {time.perf_counter() - t0:.1f} s; " + ", ".join(f"{k} {v}" for k, v in r.items()))
    return r


def test_prior_and_gate(report):
    """The prior alone reads the FWHM within the target for most held-out
    cases, and the gate calibrates to a positive threshold."""
    assert report["prior_frac_within_target"] >= 0.95
    assert report["gate_tau"] > 0.0


def test_network_improves_on_the_prior(report):
    """What the trained network adds to the physics prior on the held-out
    cases: a smaller median FWHM error and a smaller median ROI intensity
    error than the prior alone."""
    assert report["fwhm_err_all_median"] < report["prior_fwhm_err_median"]
    assert report["roi_rel_l2_median"] < report["prior_roi_rel_l2_median"]


def test_surrogate_gains_over_czt(report):
    """What the trained surrogate gains over solving every case by CZT: a share
    of the held-out cases accepted, each within 0.5 % of the CZT's FWHM, and an
    end-to-end speed-up that counts the prior, both members, the gate's FWHM
    readings and the fallback solves."""
    assert report["accepted_fraction"] >= 0.2
    assert report["fwhm_err_accepted_max"] <= 0.005
    assert report["speedup_with_fallback"] > 1.2
    assert report["speedup_accepted"] > 20


def test_out_of_box_input_is_never_accepted():
    """A wavelength outside the training range is rejected before any network
    evaluation, and the CZT answers it."""
    w = workload("surrogate")
    cr, _ = surrogate_draws(5, 4, w["D"], w["lambda0"])
    f_out = SG.features(cr, np.full(4, 900e-9), w["D"], w["lambda0"])
    assert not SG.in_training_box(f_out).any()
    t_out, _ = SG.CZTSolver(w).solve(cr, np.full(4, 900e-9))
    assert torch.isfinite(t_out).all()
