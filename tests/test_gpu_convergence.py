"""Grid convergence of the accuracy study's plate (Sec. 4.1, Figs. 6-8) on the
GPU: the binary, negative-centred FZP D = 0.08 m, f = 1.5 m at 532 nm, ROI
512^2 at +-8 lambda f/#.  At the study's largest grid (N = 28672) both paths'
FWHM, main-lobe DE and MTF at half cutoff lie within 1e-4 of the continuous
plate's values from the oracle's radial integral (the MTF of that radial
intensity sampled on the same ROI grid), and the split ROI within 1e-4 of the
FP64 ROI at every grid.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2609_01978_amd as P  # noqa: E402
from oracle import fzp_oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu
D, F, LAM = 0.08, 1.5, 532e-9
M = 512


def announce(msg):
    print(f"[gpu-convergence] {msg}", flush=True)


def gpu_metrics(N, path):
    plan = P.Plan(dict(D=D, f0=F, lambda0=LAM, N=N), [dict(lam=LAM, M=M)], path=path, allow_undersampled=True)
    ws, roi = plan.alloc()
    plan.propagate(ws, roi)
    m = plan.metrics(ws, roi)[0]
    I = plan.roi_view(roi, 0).abs().square().cpu().numpy()
    return m, I


@pytest.fixture(scope="module")
def continuous():
    ap = O.Aperture(D=D, f0=F, lambda0=LAM, N=2)
    h = O.hankel_metrics(ap)
    r = O.resolve(ap, O.Instance(lam=LAM, M=M))
    dxo = r["dx_out"]
    # the radial intensity on a fine radius grid, interpolated onto the ROI grid
    pos = (np.arange(M) - 0.5 * M) * dxo
    rr = np.hypot(pos[:, None], pos[None, :])
    grid = np.linspace(0.0, rr.max() * 1.0001, 6001)
    Ir = O.hankel_intensity(grid, ap, LAM, F)
    I2 = np.interp(rr, grid, Ir)
    mtf = O.mtf_half_cut(I2, dxo, D / (LAM * F))
    return dict(fwhm=h["fwhm"], de=h["de"], mtf=mtf)


@pytest.mark.parametrize("N", [8192, 28672])
def test_grid_convergence(N, continuous):
    out = {}
    for path in ("fp64", "split"):
        m, I = gpu_metrics(N, path)
        out[path] = (m, I)
        fw = 0.5 * (m["fwhm_x"] + m["fwhm_y"]) / continuous["fwhm"] - 1
        de = m["de"] / continuous["de"] - 1
        mt = m["mtf_half_cut"] / continuous["mtf"] - 1
        announce(f"N={N} {path}: FWHM {fw:+.2e}, DE {de:+.2e}, MTF {mt:+.2e} vs the continuous plate")
        if N == 28672:
            assert abs(fw) < 1e-4 and abs(de) < 1e-4 and abs(mt) < 1e-4  # observed <= 3e-6
    e = float(np.linalg.norm(out["split"][1] - out["fp64"][1]) / np.linalg.norm(out["fp64"][1]))
    announce(f"  split vs fp64 intensity rel-L2 {e:.2e}")
    assert e <= 1e-4
