"""GPU parity of the int8 row pass (FZP_FLAG_SPLIT_INT8) through the C ABI
against the FP64 oracle.

The int8 form holds the kernel row (and a complex stripe) in fixed point of
step 1/16256 (at most 3.1e-5 per component) and sums the products exactly in
int32; the column pass is the split path's.  Bar: complex and intensity
rel-L2 <= 1e-4, as for the split-BF16 path (the quantisation is incoherent
over the aperture: measured errors are near 1e-6).  Cases: ragged row and
column tiles with several K stages and segments, 2- and 4-level phase plates
(prefix sums minus binary GEMMs), rows that miss the disc, sampled stripes of
the 1 m element at full size, and complex stripes: creases, 3- and 8-level
plates, creases on a 4-level plate over several chunks, a mixed graph batch.
"""
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
    print(f"[gpu-int8] {msg}", flush=True)


def run(ap, inst, rows=None, **kw):
    plan = P.Plan(ap, [inst], **kw)
    ws, roi = plan.alloc()
    if rows is None:
        plan.propagate(ws, roi)
    else:
        plan.propagate_range(ws, roi, rows[0], rows[1], accumulate=False)
    torch.cuda.synchronize()
    return plan, ws, roi, plan.roi_view(roi, 0).cpu().numpy()


def oracle(ap, inst):
    a = O.Aperture(D=ap["D"], f0=ap["f0"], lambda0=ap["lambda0"], N=ap["N"], levels=ap.get("levels", 0),
                   centre_open=ap.get("centre_open", 0))
    i = O.Instance(lam=inst["lam"], M=inst["M"], x0=inst.get("x0", 0.0), y0=inst.get("y0", 0.0),
                   half_width=inst.get("half_width", 0.0), creases=inst.get("creases"))
    return a, i


@pytest.mark.parametrize("L,N,M", [(0, 3000, 48), (0, 2500, 128), (0, 4096, 384), (0, 777, 16),
                                   (2, 2048, 128), (4, 3000, 144), (4, 2048, 64)])
def test_int8_full_roi(L, N, M):
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=N, levels=L, centre_open=1 if N == 777 else 0)
    inst = dict(lam=600e-9 if L else LAM0, M=M, x0=1e-6 if L else 0.0)
    announce(f"levels {L} N={N} M={M}")
    _, _, _, U8 = run(ap, inst, path="split", int8=True, allow_undersampled=True)
    _, _, _, Ub = run(ap, inst, path="split", allow_undersampled=True)
    ref = O.propagate(*oracle(ap, inst), stripe=512)
    e8, eb = rel_l2(U8, ref), rel_l2(Ub, ref)
    ei = rel_l2(O.intensity(U8), O.intensity(ref))
    announce(f"  int8 complex {e8:.2e} intensity {ei:.2e}; BF16 split complex {eb:.2e}")
    assert e8 <= 1e-4 and ei <= 1e-4


def test_int8_rows_outside_the_disc_and_ranges_add_up():
    """Rows wholly outside the disc add exactly nothing; two row ranges add up
    to the oracle's full sum."""
    ap = dict(D=1e-3, f0=4e-3, lambda0=LAM0, N=1001, pitch=1e-3 / 997)
    inst = dict(lam=LAM0, M=64, z=4.05e-3)
    plan = P.Plan(ap, [inst], path="split", int8=True, allow_undersampled=True, stripe_rows=256)
    ws, roi = plan.alloc()
    roi.fill_(1.0)
    # disc radius 997/2 samples about the centre of a 1001-sample grid: rows 0, 1 miss it
    plan.propagate_range(ws, roi, 0, 2, accumulate=False)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(roi)) == 0
    for a, b in ((0, 501), (501, 1001)):
        plan.propagate_range(ws, roi, a, b, accumulate=a > 0)
    torch.cuda.synchronize()
    U = plan.roi_view(roi, 0).cpu().numpy()
    a_ = O.Aperture(D=ap["D"], f0=ap["f0"], lambda0=LAM0, N=1001, pitch=ap["pitch"])
    i_ = O.Instance(lam=LAM0, M=64, z=4.05e-3)
    ref = O.propagate(a_, i_, stripe=512)
    e = rel_l2(U, ref)
    announce(f"two ranges vs oracle complex {e:.2e}")
    assert e <= 1e-4


def test_fzp1m_sampled_stripes_int8():
    w = workload("fzp1m")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    inst = dict(lam=w["lambda0"], M=w["M"])
    plan = P.Plan(ap, [inst], path="split", int8=True, stripe_rows=w["stripe"])
    ws, roi = plan.alloc()
    a, i = oracle(ap, inst)
    S = w["stripe"]
    for j0 in (w["N"] // 2 - 64, 777 * 128):
        announce(f"fzp1m int8 stripe rows {j0}..{j0 + S}")
        plan.propagate_range(ws, roi, j0, j0 + S, accumulate=False)
        torch.cuda.synchronize()
        U = plan.roi_view(roi, 0).cpu().numpy()
        ref = O.propagate(a, i, method="bluestein", rows=(j0, j0 + S), stripe=32)
        e = rel_l2(U, ref)
        announce(f"  complex rel-L2 {e:.3e}")
        assert e <= 1e-4


CPLX = {
    "creases": (dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=1536),
                dict(lam=700e-9, M=96, creases=crease_draws(5, 2e-3, LAM0, 8) * np.array([1, 1, 0.2, 1])), 0),
    "levels3_ragged": (dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=1999, levels=3), dict(lam=600e-9, M=64, x0=1e-6), 0),
    "levels8": (dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096, levels=8), dict(lam=600e-9, M=256), 0),
    "creased_4level_chunks": (dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=3001, levels=4),
                              dict(lam=700e-9, M=272,
                                   creases=crease_draws(21, 2e-3, LAM0, 6) * np.array([1, 1, 0.3, 1])), 700),
}


@pytest.mark.parametrize("case", list(CPLX))
def test_int8_complex_stripes_full_roi(case):
    ap, inst, chunk = CPLX[case]
    announce(f"complex stripes {case}: N={ap['N']} M={inst['M']} levels={ap.get('levels', 0)} chunk {chunk}")
    _, _, _, U8 = run(ap, inst, path="split", int8=True, allow_undersampled=True, chunk_rows=chunk)
    _, _, _, Ub = run(ap, inst, path="split", allow_undersampled=True, chunk_rows=chunk)
    ref = O.propagate(*oracle(ap, inst), stripe=512)
    e8, eb = rel_l2(U8, ref), rel_l2(Ub, ref)
    ei = rel_l2(O.intensity(U8), O.intensity(ref))
    announce(f"  int8 complex {e8:.2e} intensity {ei:.2e}; BF16 split complex {eb:.2e}")
    assert e8 <= 1e-4 and ei <= 1e-4


def test_int8_mixed_batch_graph_matches_eager_and_oracle():
    """Binary and creased instances of mixed ROI sizes in one plan on two
    lanes: the captured graph equals the eager propagation bit for bit (int8
    sums are exact and the column pass is deterministic), and each instance
    is within the bar of the oracle."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048)
    cr = crease_draws(9, 2e-3, LAM0, 8) * np.array([1, 1, 0.2, 1])
    insts = [dict(lam=LAM0, M=64), dict(lam=560e-9, M=128, creases=cr), dict(lam=700e-9, M=96, creases=cr[:3])]
    plan = P.Plan(ap, insts, path="split", int8=True, lanes=2, chunk_rows=512)
    ws, roi = plan.alloc()
    plan.propagate(ws, roi)
    torch.cuda.synchronize()
    eager = roi.clone()
    g = plan.graph(ws, roi)
    other = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(3):
        roi.fill_(float("nan"))
        other.add_(1.0)                      # eager work between replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(roi, eager), rep
    for k, inst in enumerate(insts):
        U = plan.roi_view(roi, k).cpu().numpy()
        ref = O.propagate(*oracle(ap, inst), stripe=512)
        e = rel_l2(U, ref)
        announce(f"  batch instance {k} M={inst['M']} creased={'creases' in inst} complex rel-L2 {e:.2e}")
        assert e <= 1e-4


def test_int8_binary_sums_do_not_depend_on_the_schedule(tmp_path):
    """The int8 binary row pass sums exactly (int32 per K segment, int64 over
    segments), so its partial sums, and with them the ROI, are the same bit
    for bit whatever the K segment length, the lane count and the operand
    overlap.  The segment length is set through the autotuner's cache: one
    tuning run writes the plan's entry, which is then rewritten to each
    candidate length and read back."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=16384)   # K segments of 4096 (the default), 8192, 16384
    insts = [dict(lam=LAM0, M=128), dict(lam=600e-9, M=64, x0=2e-6)]
    cache = tmp_path / "tune.txt"
    ref = None
    for kw in (dict(), dict(overlap_operand=True), dict(lanes=2)):
        plan = P.Plan(ap, insts, path="split", int8=True, chunk_rows=1024, allow_undersampled=True, **kw)
        ws, roi = plan.alloc()
        plan.propagate(ws, roi)
        torch.cuda.synchronize()
        if ref is None:
            ref = roi.clone()
            tune = plan.autotune(ws, roi, str(cache))
            announce(f"autotune {tune}")
            assert tune["variant"] % 8 == 4       # the int8 row pass has one form; the BF16 default stays
            key, _, ln, tl = cache.read_text().split("\n")[0].split()
            assert key.endswith("/128f/64f") and "/i8" in key
            for seg in (4096, 8192, 16384):
                cache.write_text(f"{key} {seg} {ln} {tl}\n")
                got = plan.autotune(ws, roi, str(cache))
                assert got["seg_len"] == seg
                plan.propagate(ws, roi)
                torch.cuda.synchronize()
                announce(f"K segments of {seg}: bit-identical {torch.equal(roi, ref)}")
                assert torch.equal(roi, ref), seg
        else:
            announce(f"schedule {kw}: bit-identical {torch.equal(roi, ref)}")
            assert torch.equal(roi, ref), kw
        del ws, roi, plan


LIMITS = {
    "roi_m16": (dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048), dict(lam=LAM0, M=16)),
    "roi_m2048": (dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048), dict(lam=LAM0, M=2048)),
    "n100": (dict(D=1e-3, f0=10e-3, lambda0=LAM0, N=100), dict(lam=LAM0, M=32)),
    "n100_creased": (dict(D=1e-3, f0=10e-3, lambda0=LAM0, N=100),
                     dict(lam=LAM0, M=32, creases=crease_draws(3, 1e-3, LAM0, 4) * np.array([1, 1, 0.3, 1]))),
    "creased_m1024": (dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048),
                      dict(lam=600e-9, M=1024, creases=crease_draws(4, 2e-3, LAM0, 8) * np.array([1, 1, 0.2, 1]))),
}


@pytest.mark.parametrize("case", list(LIMITS))
def test_int8_limits(case):
    """The smallest and largest ROIs, an aperture smaller than one row tile and
    one K stage (binary and creased), and a large creased ROI (16 column
    tiles), against the oracle."""
    ap, inst = LIMITS[case]
    announce(f"limits {case}: N={ap['N']} M={inst['M']}")
    _, _, _, U = run(ap, inst, path="split", int8=True, allow_undersampled=True)
    ref = O.propagate(*oracle(ap, inst), stripe=64 if ap["N"] < 512 else 512)
    e, ei = rel_l2(U, ref), rel_l2(O.intensity(U), O.intensity(ref))
    announce(f"  complex {e:.2e} intensity {ei:.2e}")
    assert e <= 1e-4 and ei <= 1e-4


def test_int8_largest_aperture_sampled_stripe():
    """N = 2^21 (the split path's largest grid in one segment schedule): a 2 m
    f/5 plate at 0.95 um pitch, 64 rows through the centre against the
    oracle's restricted row sum."""
    N = 1 << 21
    ap = dict(D=2.0, f0=10.0, lambda0=LAM0, N=N)
    inst = dict(lam=LAM0, M=512)
    plan = P.Plan(ap, [inst], path="split", int8=True, stripe_rows=64)
    ws, roi = plan.alloc()
    j0 = N // 2 - 32
    announce(f"N=2^21 int8 stripe rows {j0}..{j0 + 64}")
    plan.propagate_range(ws, roi, j0, j0 + 64, accumulate=False)
    torch.cuda.synchronize()
    U = plan.roi_view(roi, 0).cpu().numpy()
    ref = O.propagate(*oracle(ap, inst), method="bluestein", rows=(j0, j0 + 64), stripe=16)
    e = rel_l2(U, ref)
    announce(f"  complex rel-L2 {e:.3e}")
    assert e <= 1e-4


def test_int8_tall_ridge_phase_reduction():
    """A ridge far wider than the pupil and 300.37 wavelengths tall adds a
    near-uniform phase of about 300 turns, beyond the transcendental unit's
    +-256-turn input range unless the stripe generator reduces the turns
    first: the intensity must still be the oracle's (a uniform phase is
    invisible in it), on both split forms."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=1536)
    inst = dict(lam=LAM0, M=96, creases=np.array([[0.3, 0.0, 1e6, 300.37 * LAM0]]))
    ref = O.intensity(O.propagate(*oracle(ap, inst), stripe=512))
    for int8 in (True, False):
        _, _, _, U = run(ap, inst, path="split", int8=int8, allow_undersampled=True)
        e = rel_l2(O.intensity(U), ref)
        announce(f"tall ridge int8={int8}: intensity rel-L2 {e:.2e}")
        assert e <= 1e-4
