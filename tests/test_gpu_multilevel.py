"""GPU parity of L-level phase plates (the revised engine's element, Fig. 18
stage 3) through the C ABI, both paths against the FP64 oracle.

Bars as for the amplitude plate: complex rel-L2 <= 1e-9 for the FP64 path,
intensity (and complex) rel-L2 <= 1e-4 for the split-BF16 path, whose phase
plate runs through the complex-stripe kernels.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2609_01978_amd as P  # noqa: E402
from oracle import fzp_oracle as O  # noqa: E402
from fzp_inputs import crease_draws, workload  # noqa: E402

pytestmark = pytest.mark.gpu
LAM0 = 632.8e-9


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(msg):
    print(f"[gpu-multilevel] {msg}", flush=True)


def run(ap, insts, path, rows=None, **kw):
    plan = P.Plan(ap, insts, path=path, **kw)
    ws, roi = plan.alloc()
    if rows is None:
        plan.propagate(ws, roi)
    else:
        plan.propagate_range(ws, roi, rows[0], rows[1], accumulate=False)
    torch.cuda.synchronize()
    return plan, ws, roi, [plan.roi_view(roi, k).cpu().numpy() for k in range(len(insts))]


def oracle(ap, inst):
    a = O.Aperture(D=ap["D"], f0=ap["f0"], lambda0=ap["lambda0"], N=ap["N"], pitch=ap.get("pitch", 0.0),
                   levels=ap.get("levels", 0), centre_open=ap.get("centre_open", 0))
    i = O.Instance(lam=inst["lam"], M=inst["M"], x0=inst.get("x0", 0.0), y0=inst.get("y0", 0.0),
                   half_width=inst.get("half_width", 0.0), creases=inst.get("creases"))
    return a, i


@pytest.mark.parametrize("L,N,M", [(2, 2048, 128), (3, 1999, 64), (4, 3000, 144), (8, 4096, 256), (16, 4096, 96)])
def test_phase_plate_both_paths(L, N, M):
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=N, levels=L)
    inst = dict(lam=600e-9, M=M, x0=1e-6, y0=-0.5e-6)
    announce(f"L={L} N={N} M={M}")
    _, _, _, (U64,) = run(ap, [inst], "fp64", allow_undersampled=True)
    _, _, _, (Us,) = run(ap, [inst], "split", allow_undersampled=True)
    a, i = oracle(ap, inst)
    ref = O.propagate(a, i, stripe=512)
    e64, es = rel_l2(U64, ref), rel_l2(O.intensity(Us), O.intensity(ref))
    announce(f"  fp64 complex {e64:.2e}, split intensity {es:.2e}, split complex {rel_l2(Us, ref):.2e}")
    assert e64 < 1e-9
    assert es <= 1e-4 and rel_l2(Us, ref) <= 1e-4


def test_two_levels_is_open_minus_closed_amplitude_plate():
    """On the GPU as in the oracle: L = 2 equals the centre-open amplitude plate
    minus the centre-opaque one (FP64 path, each its own kernels)."""
    kw = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2500)
    inst = dict(lam=LAM0, M=128)
    _, _, _, (U2,) = run(dict(levels=2, **kw), [inst], "fp64")
    _, _, _, (Uo,) = run(dict(centre_open=1, **kw), [inst], "fp64")
    _, _, _, (Uc,) = run(dict(centre_open=0, **kw), [inst], "fp64")
    assert rel_l2(U2, Uo - Uc) < 1e-12


@pytest.mark.parametrize("path", ["fp64", "split"])
def test_phase_plate_with_creases_and_chunks(path):
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=3001, levels=4)
    cr = crease_draws(21, 2e-3, LAM0, 6) * np.array([1, 1, 0.3, 1])
    inst = dict(lam=700e-9, M=272, creases=cr)
    announce(f"{path} L=4 creases chunk 384")
    _, _, _, (U,) = run(ap, [inst], path, allow_undersampled=True, chunk_rows=384)
    a, i = oracle(ap, inst)
    ref = O.propagate(a, i, stripe=512)
    e = rel_l2(U, ref)
    announce(f"  complex rel-L2 {e:.2e}")
    assert e < (1e-9 if path == "fp64" else 1e-4)


@pytest.mark.parametrize("path", ["fp64", "split"])
def test_ml100mm_sampled_stripes(path):
    """The benchmarked phase plate: 64-row stripes through the centre and near
    the edge against the oracle's restricted row sum."""
    w = workload("ml100mm")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"], levels=w["levels"])
    inst = dict(lam=w["lambda0"], M=w["M"])
    plan = P.Plan(ap, [inst], path=path, stripe_rows=w["stripe"])
    ws, roi = plan.alloc()
    a, i = oracle(ap, inst)
    N = w["N"]
    for j0 in (N // 2 - 32, N // 2 + 90001, 7001):
        announce(f"ml100mm {path} rows {j0}..{j0 + 64}")
        plan.propagate_range(ws, roi, j0, j0 + 64, accumulate=False)
        torch.cuda.synchronize()
        U = plan.roi_view(roi, 0).cpu().numpy()
        ref = O.propagate(a, i, rows=(j0, j0 + 64), stripe=32)
        e = rel_l2(U, ref)
        announce(f"  complex rel-L2 {e:.2e}")
        assert e <= (1e-6 if path == "fp64" else 1e-4)


def test_ml100mm_whole_plate_efficiency():
    """Whole ml100mm plate: the split ROI within 1e-4 of the FP64 path's, and
    the main-lobe DE within 2e-4 of the 4-level ladder value
    sinc^2(1/4) * 0.837785 (observed 1.5e-6; the oracle's radial integral gives
    the continuous plate's value)."""
    w = workload("ml100mm")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"], levels=w["levels"])
    inst = dict(lam=w["lambda0"], M=w["M"])
    ps, wss, rois, (Us,) = run(ap, [inst], "split", stripe_rows=w["stripe"])
    p6, ws6, roi6, (U6,) = run(ap, [inst], "fp64")
    e = rel_l2(O.intensity(Us), O.intensity(U6))
    ms, m6 = ps.metrics(wss, rois)[0], p6.metrics(ws6, roi6)[0]
    x = math.pi / w["levels"]
    ladder = (math.sin(x) / x) ** 2 * O.AIRY_LOBE_FRACTION
    h = O.hankel_metrics(oracle(ap, inst)[0])
    announce(f"  split vs fp64 intensity {e:.2e}; DE split {ms['de']:.6f} fp64 {m6['de']:.6f} "
             f"radial {h['de']:.6f} ladder {ladder:.6f}; FWHM / radial - 1 {m6['fwhm_x'] / h['fwhm'] - 1:.2e}")
    assert e <= 1e-4
    assert abs(ms["de"] / m6["de"] - 1) < 1e-4
    assert abs(m6["de"] / ladder - 1) < 2e-4
    assert abs(m6["de"] / h["de"] - 1) < 2e-4
    assert abs(m6["fwhm_x"] / h["fwhm"] - 1) < 1e-2


def test_two_level_plate_on_the_binary_kernels():
    """A crease-free 2-level plate runs on the split path as disc - 2 mask: the
    binary-stripe GEMM for the odd-zone mask and float64 prefix sums of the row
    kernel for the disc.  The 0.1 m plate at L = 2: sampled stripes against the
    oracle, the whole plate against the FP64 path and the ladder value
    sinc^2(1/2) * 0.837785."""
    w = workload("ml100mm")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"], levels=2)
    inst = dict(lam=w["lambda0"], M=w["M"])
    plan = P.Plan(ap, [inst], path="split", stripe_rows=w["stripe"])
    ws, roi = plan.alloc()
    a, i = oracle(ap, inst)
    N = w["N"]
    for j0 in (N // 2 - 32, 7001):
        plan.propagate_range(ws, roi, j0, j0 + 64, accumulate=False)
        torch.cuda.synchronize()
        U = plan.roi_view(roi, 0).cpu().numpy()
        ref = O.propagate(a, i, rows=(j0, j0 + 64), stripe=32)
        e = rel_l2(U, ref)
        announce(f"  L=2 split rows {j0}..{j0 + 64}: complex rel-L2 {e:.2e}")
        assert e <= 1e-4
    plan.propagate(ws, roi)
    ms = plan.metrics(ws, roi)[0]
    Us = plan.roi_view(roi, 0).cpu().numpy()
    p6, ws6, roi6, (U6,) = run(ap, [inst], "fp64")
    m6 = p6.metrics(ws6, roi6)[0]
    e = rel_l2(O.intensity(Us), O.intensity(U6))
    ladder = (2.0 / math.pi) ** 2 * O.AIRY_LOBE_FRACTION
    announce(f"  L=2 whole plate: split vs fp64 intensity {e:.2e}; DE split {ms['de']:.6f} fp64 {m6['de']:.6f} "
             f"ladder {ladder:.6f}")
    assert e <= 1e-4
    assert abs(m6["de"] / ladder - 1) < 1e-3
