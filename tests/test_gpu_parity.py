"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Full-ROI comparisons at sizes the oracle finishes in seconds; at the full
workload sizes, sampled stripes of aperture rows (the library's row-range
call against the oracle's restricted row sum) plus properties that hold at any
size.  Bars: ROI intensity rel-L2 <= 1e-6 for the FP64 Bluestein path and
<= 1e-4 for the split-BF16 path; FWHM and DE within 0.1 % of the oracle.
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


def run_gpu(ap: dict, insts: list, path="fp64", rows=None, **kw):
    plan = P.Plan(ap, insts, path=path, **kw)
    ws, roi = plan.alloc()
    if rows is None:
        plan.propagate(ws, roi)
    else:
        plan.propagate_range(ws, roi, rows[0], rows[1], accumulate=False)
    torch.cuda.synchronize()
    out = [plan.roi_view(roi, k).cpu().numpy() for k in range(len(insts))]
    return plan, ws, roi, out


def oracle_case(ap: dict, inst: dict):
    a = O.Aperture(D=ap["D"], f0=ap["f0"], lambda0=ap["lambda0"], N=ap["N"], pitch=ap.get("pitch", 0.0),
                   centre_open=ap.get("centre_open", 0))
    i = O.Instance(lam=inst["lam"], M=inst["M"], z=inst.get("z", 0.0), x0=inst.get("x0", 0.0),
                   y0=inst.get("y0", 0.0), half_width=inst.get("half_width", 0.0), creases=inst.get("creases"))
    return a, i


def announce(msg):
    print(f"[gpu-parity] {msg}", flush=True)


# ---------------------------------------------------------------------------
# Full ROI against the oracle
# ---------------------------------------------------------------------------

SMALL = [
    # (name, aperture, instance, allow_undersampled)
    ("tiny_offcentre_open", dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=777, centre_open=1),
     dict(lam=560e-9, M=48, x0=1.5e-6, y0=-2.25e-6, half_width=40e-6), True),
    ("pitch_ragged", dict(D=1e-3, f0=4e-3, lambda0=LAM0, N=1001, pitch=1e-3 / 997),
     dict(lam=LAM0, M=64, z=4.05e-3), True),
    ("creases", dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=1536),
     dict(lam=700e-9, M=96, creases=crease_draws(5, 2e-3, LAM0, 8) * np.array([1, 1, 0.2, 1])), True),
    ("multi_block_m1024", dict(D=4e-3, f0=20e-3, lambda0=LAM0, N=8192),
     dict(lam=LAM0, M=1024), False),
]


@pytest.mark.parametrize("case", SMALL, ids=[c[0] for c in SMALL])
def test_fp64_full_roi_small(case):
    name, ap, inst, und = case
    announce(f"fp64 {name} N={ap['N']} M={inst['M']}")
    plan, ws, roi, (U,) = run_gpu(ap, [inst], allow_undersampled=und)
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=256)
    assert rel_l2(U, ref) < 1e-9
    assert rel_l2(O.intensity(U), O.intensity(ref)) < 1e-9


def test_fp64_fzp2mm_full_and_metrics():
    w = workload("fzp2mm")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    inst = dict(lam=w["lambda0"], M=w["M"])
    announce("fp64 fzp2mm full ROI + metrics")
    plan, ws, roi, (U,) = run_gpu(ap, [inst], stripe_rows=w["stripe"])
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=512)
    e_int = rel_l2(O.intensity(U), O.intensity(ref))
    announce(f"fzp2mm intensity rel-L2 {e_int:.3e}")
    assert e_int <= 1e-6
    assert rel_l2(U, ref) < 1e-9
    m = plan.metrics(ws, roi)[0]
    mo = O.metrics(ref, a, i)
    for key in ("fwhm_x", "fwhm_y", "de", "strehl", "i_peak", "p_lobe", "p_in"):
        assert abs(m[key] / mo[key] - 1) < 1e-8, (key, m[key], mo[key])
    assert abs(m["mtf_half_cut"] / mo["mtf_half_cut"] - 1) < 1e-8
    # and against the continuous radial reference (finite-zone closed form)
    h = O.hankel_metrics(a)
    assert abs(m["fwhm_x"] / h["fwhm"] - 1) < 1e-3 and abs(m["de"] / h["de"] - 1) < 1e-3


def test_fp64_bitwise_reproducible_and_ranges_add_up():
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096)
    inst = dict(lam=LAM0, M=256)
    plan = P.Plan(ap, [inst], chunk_rows=512)
    ws, roi = plan.alloc()
    plan.propagate(ws, roi)
    a = roi.clone()
    plan.propagate(ws, roi)
    torch.cuda.synchronize()
    assert torch.equal(a, roi)
    # two ranges split on a chunk boundary reproduce the full run bit for bit
    plan.propagate_range(ws, roi, 0, 1536, accumulate=False)
    plan.propagate_range(ws, roi, 1536, 4096, accumulate=True)
    torch.cuda.synchronize()
    assert torch.equal(a, roi)


def test_split_fzp2mm_vs_fp64_and_oracle():
    w = workload("fzp2mm")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    inst = dict(lam=w["lambda0"], M=w["M"])
    announce("split fzp2mm")
    _, _, _, (U64,) = run_gpu(ap, [inst])
    plan, ws, roi, (Us,) = run_gpu(ap, [inst], path="split", stripe_rows=128)
    e = rel_l2(O.intensity(Us), O.intensity(U64))
    announce(f"split vs fp64 intensity rel-L2 {e:.3e}")
    assert e <= 1e-4
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=512)
    assert rel_l2(O.intensity(Us), O.intensity(ref)) <= 1e-4
    m = plan.metrics(ws, roi)[0]
    mo = O.metrics(ref, a, i)
    assert abs(m["fwhm_x"] / mo["fwhm_x"] - 1) < 1e-3 and abs(m["de"] / mo["de"] - 1) < 1e-3


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("N,M", [(3000, 48), (2500, 128), (4096, 384)])
def test_split_shapes_ragged(N, M, variant):
    """Row tiles with a ragged tail, column tiles wider than 2M, several K stages,
    every binary-stripe GEMM variant."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=N)
    inst = dict(lam=LAM0, M=M)
    announce(f"split N={N} M={M} variant {variant}")
    _, _, _, (U64,) = run_gpu(ap, [inst], allow_undersampled=True)
    _, _, _, (Us,) = run_gpu(ap, [inst], path="split", allow_undersampled=True, variant=variant)
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=512)
    assert rel_l2(O.intensity(U64), O.intensity(ref)) < 1e-9
    e = rel_l2(O.intensity(Us), O.intensity(ref))
    announce(f"  split vs oracle intensity rel-L2 {e:.3e}")
    assert e <= 1e-4


def test_split_creases_small():
    """Deformed (complex) stripes: the three-product split against both references."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048)
    cr = crease_draws(7, 2e-3, LAM0, 8)
    inst = dict(lam=600e-9, M=128, creases=cr)
    announce("split creases N=2048 M=128")
    _, _, _, (U64,) = run_gpu(ap, [inst])
    _, _, _, (Us,) = run_gpu(ap, [inst], path="split")
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=512)
    assert rel_l2(U64, ref) < 1e-9
    e = rel_l2(O.intensity(Us), O.intensity(ref))
    announce(f"  split creases vs oracle intensity rel-L2 {e:.3e}")
    assert e <= 1e-4
    assert rel_l2(Us, ref) <= 1e-4
    # the creases matter at this size
    _, _, _, (Uflat,) = run_gpu(ap, [dict(lam=600e-9, M=128)], path="split")
    assert rel_l2(O.intensity(Uflat), O.intensity(ref)) > 1e-2


@pytest.mark.parametrize("N,M,chunk", [(3000, 48, 384), (2500, 272, 0), (1999, 16, 256)])
def test_split_creases_ragged(N, M, chunk):
    """Ragged row tiles and padded stripe rows, several chunks, column tiles past 2M."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=N)
    cr = crease_draws(11 + N, 2e-3, LAM0, 8) * np.array([1, 1, 0.3, 1])
    inst = dict(lam=700e-9, M=M, x0=1e-6, y0=-2e-6, creases=cr)
    announce(f"split creases N={N} M={M} chunk={chunk}")
    kw = dict(allow_undersampled=True)
    if chunk:
        kw["chunk_rows"] = chunk
    _, _, _, (Us,) = run_gpu(ap, [inst], path="split", **kw)
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=512)
    e = rel_l2(Us, ref)
    announce(f"  complex rel-L2 {e:.3e}")
    assert e <= 1e-4


@pytest.mark.parametrize("N,M", [(2500, 272), (1999, 48), (5000, 512)])
def test_split_binary_variants_agree_bit_for_bit(N, M):
    """Every binary-stripe GEMM variant sums each output over the same K
    sequence in the same order: the same ROI bit for bit as the default."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=N)
    inst = dict(lam=600e-9, M=M, y0=0.7e-6)
    announce(f"binary variants N={N} M={M}")
    _, _, _, (U4,) = run_gpu(ap, [inst], path="split", allow_undersampled=True, variant=4)
    for v in (0, 1, 2, 3):
        _, _, _, (Uv,) = run_gpu(ap, [inst], path="split", allow_undersampled=True, variant=v)
        assert np.array_equal(Uv, U4), v


@pytest.mark.parametrize("N,M,levels", [(2500, 272, 0), (1999, 48, 8), (3000, 128, 0)])
def test_split_complex_tiles_agree_bit_for_bit(N, M, levels):
    """The complex-stripe GEMM's 128-column tiles (cplx_tile = 1, and 2 with two
    work-groups per compute unit) give the 256-column tile's ROI bit for bit (every output sums the same K sequence in
    the same order) and both agree with the oracle; column tiles past 2M,
    ragged rows, a creased amplitude plate and a creased 8-level phase plate."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=N, levels=levels)
    cr = crease_draws(31 + N, 2e-3, LAM0, 6) * np.array([1, 1, 0.3, 1])
    inst = dict(lam=650e-9, M=M, x0=0.5e-6, creases=cr)
    announce(f"complex tiles N={N} M={M} levels={levels}")
    _, _, _, (U0,) = run_gpu(ap, [inst], path="split", allow_undersampled=True, chunk_rows=640)
    _, _, _, (U1,) = run_gpu(ap, [inst], path="split", allow_undersampled=True, chunk_rows=640, cplx_tile=1)
    _, _, _, (U2,) = run_gpu(ap, [inst], path="split", allow_undersampled=True, chunk_rows=640, cplx_tile=2)
    assert np.array_equal(U0, U1) and np.array_equal(U0, U2)
    a = O.Aperture(D=ap["D"], f0=ap["f0"], lambda0=ap["lambda0"], N=N, levels=levels)
    _, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=512)
    e = rel_l2(U1, ref)
    announce(f"  complex rel-L2 {e:.3e}")
    assert e <= 1e-4


@pytest.mark.parametrize("M,creased", [(272, False), (512, True)])
def test_split_ranges_at_odd_rows_add_up(M, creased):
    """Row ranges that start and end inside the 16- and 32-row blocks of the
    column GEMM's K operand (rows outside a range are masked to zero there)
    add up to the whole aperture; ROI row tiles past M are ragged."""
    N = 2048
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=N)
    inst = dict(lam=LAM0, M=M)
    if creased:
        inst["creases"] = crease_draws(5, 2e-3, LAM0, 8)
    announce(f"split ranges at odd rows M={M} creased={creased}")
    plan = P.Plan(ap, [inst], path="split")
    ws, roi = plan.alloc()
    cuts = [0, 37, 1000, 1001, 1013, 1531, N]
    for k in range(len(cuts) - 1):
        plan.propagate_range(ws, roi, cuts[k], cuts[k + 1], accumulate=k > 0)
    torch.cuda.synchronize()
    U = plan.roi_view(roi, 0).cpu().numpy()
    _, _, _, (Uw,) = run_gpu(ap, [inst], path="split")
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=512)
    e = rel_l2(O.intensity(U), O.intensity(ref))
    announce(f"  ranges vs oracle intensity rel-L2 {e:.3e}, vs one call {rel_l2(U, Uw):.3e}")
    assert e <= 1e-4
    assert rel_l2(U, Uw) <= 1e-4


def test_split_mixed_instances():
    """One plan, one workspace: a flat and a creased instance at two wavelengths,
    sharing the operand table (lambda z is fixed at the first-order focus)."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048)
    cr = crease_draws(3, 2e-3, LAM0, 8)
    insts = [dict(lam=520e-9, M=128), dict(lam=760e-9, M=128, creases=cr), dict(lam=LAM0, M=64)]
    announce("split mixed instances")
    plan, ws, roi, outs = run_gpu(ap, insts, path="split")
    for inst, U in zip(insts, outs):
        a, i = oracle_case(ap, inst)
        ref = O.propagate(a, i, method="bluestein", stripe=512)
        assert rel_l2(U, ref) <= 1e-4
    ms = plan.metrics(ws, roi)
    assert len(ms) == 3 and all(m["de"] > 0 for m in ms)


# ---------------------------------------------------------------------------
# Full workload sizes: sampled stripes and properties
# ---------------------------------------------------------------------------

def _sampled_stripes(name, path, stripes, **kw):
    w = workload(name)
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    inst = dict(lam=w["lambda0"], M=w["M"])
    plan = P.Plan(ap, [inst], path=path, stripe_rows=w["stripe"], **kw)
    ws, roi = plan.alloc()
    a, i = oracle_case(ap, inst)
    S = w["stripe"]
    for j0 in stripes:
        announce(f"{name} {path} stripe rows {j0}..{j0 + S}")
        plan.propagate_range(ws, roi, j0, j0 + S, accumulate=False)
        torch.cuda.synchronize()
        U = plan.roi_view(roi, 0).cpu().numpy()
        ref = O.propagate(a, i, method="bluestein", rows=(j0, j0 + S), stripe=32)
        e = rel_l2(U, ref)
        announce(f"  complex rel-L2 {e:.3e}")
        assert e <= (1e-6 if path == "fp64" else 1e-4)


def test_fzp20mm_sampled_stripes_fp64():
    N = workload("fzp20mm")["N"]
    _sampled_stripes("fzp20mm", "fp64", [N // 2 - 128, 1024, N - 3 * 256])


def test_fzp20mm_sampled_stripes_split():
    N = workload("fzp20mm")["N"]
    _sampled_stripes("fzp20mm", "split", [N // 2 - 128, 3072])


def test_fzp1m_sampled_stripes_fp64():
    N = workload("fzp1m")["N"]
    _sampled_stripes("fzp1m", "fp64", [N // 2 - 64, 100 * 128])


def test_fzp1m_sampled_stripes_split():
    N = workload("fzp1m")["N"]
    _sampled_stripes("fzp1m", "split", [N // 2 - 64])


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_fzp1m_sampled_stripes_split_variants(variant):
    N = workload("fzp1m")["N"]
    _sampled_stripes("fzp1m", "split", [N // 2 - 64, 777 * 128], variant=variant)


def test_fzp20mm_creased_stripes_split():
    """A creased instance of the 20 mm element (the batch workload's aperture):
    sampled stripes of the split path against the oracle's restricted row sum."""
    w = workload("fzp20mm")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    inst = dict(lam=550e-9, M=512, creases=crease_draws(1, w["D"], w["lambda0"], 8))
    plan = P.Plan(ap, [inst], path="split", stripe_rows=w["stripe"])
    ws, roi = plan.alloc()
    a, i = oracle_case(ap, inst)
    N, S = w["N"], w["stripe"]
    for j0 in (N // 2 - 128, 5000):
        announce(f"fzp20mm creased split stripe rows {j0}..{j0 + S}")
        plan.propagate_range(ws, roi, j0, j0 + S, accumulate=False)
        torch.cuda.synchronize()
        U = plan.roi_view(roi, 0).cpu().numpy()
        ref = O.propagate(a, i, method="bluestein", rows=(j0, j0 + S), stripe=64)
        e = rel_l2(U, ref)
        announce(f"  complex rel-L2 {e:.3e}")
        assert e <= 1e-4


# ---------------------------------------------------------------------------
# Whole apertures at the large workloads: both paths, metrics against the
# oracle's extractor, the radial (Hankel) integral and the Airy closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["fzp20mm", "fzp1m"])
def test_full_aperture_metrics(name):
    w = workload(name)
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    inst = dict(lam=w["lambda0"], M=w["M"])
    res = {}
    for path in ("split", "fp64"):
        announce(f"{name} full aperture, {path}")
        plan = P.Plan(ap, [inst], path=path, stripe_rows=w["stripe"])
        ws, roi = plan.alloc()
        plan.propagate(ws, roi)
        m = plan.metrics(ws, roi)[0]
        U = plan.roi_view(roi, 0).cpu().numpy()
        res[path] = (U, m)
        del ws, roi
        torch.cuda.empty_cache()
    a, i = oracle_case(ap, inst)
    I_split, I_fp64 = O.intensity(res["split"][0]), O.intensity(res["fp64"][0])
    e = rel_l2(I_split, I_fp64)
    announce(f"  split vs fp64 intensity rel-L2 {e:.3e}")
    assert e <= 1e-4
    h = O.hankel_metrics(a)
    lz = w["lambda0"] * w["f0"]
    airy_fwhm = O.AIRY_FWHM * lz / w["D"]
    airy_de = O.AIRY_LOBE_FRACTION / np.pi ** 2
    for path, (U, m) in res.items():
        # the GPU extractor against the oracle's on the same ROI
        mo = O.metrics(U, a, i)
        for key in ("fwhm_x", "fwhm_y", "de", "strehl", "mtf_half_cut"):
            assert abs(m[key] / mo[key] - 1) < 1e-8, (path, key, m[key], mo[key])
        # FWHM and DE within 0.1 % of the continuous aperture and of the Airy forms
        announce(f"  {path}: FWHM/Hankel-1 {m['fwhm_x'] / h['fwhm'] - 1:.2e}, DE/Hankel-1 {m['de'] / h['de'] - 1:.2e}, "
                 f"FWHM/Airy-1 {m['fwhm_x'] / airy_fwhm - 1:.2e}, DE/Airy-1 {m['de'] / airy_de - 1:.2e}")
        for key in ("fwhm_x", "fwhm_y"):
            assert abs(m[key] / h["fwhm"] - 1) < 1e-3 and abs(m[key] / airy_fwhm - 1) < 1e-3
        assert abs(m["de"] / h["de"] - 1) < 1e-3 and abs(m["de"] / airy_de - 1) < 1e-3


# ---------------------------------------------------------------------------
# Limits and degenerate cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("path,M", [("fp64", 2), ("fp64", 2048), ("split", 16), ("split", 2048)])
def test_roi_size_limits(path, M):
    """The smallest and largest ROI the plan accepts (M in 2 .. 2048; the split
    path takes multiples of 16) against the oracle."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048)
    inst = dict(lam=LAM0, M=M)
    announce(f"{path} ROI size limit M={M}")
    _, _, _, (U,) = run_gpu(ap, [inst], path=path)
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=512)
    if path == "fp64":
        assert rel_l2(U, ref) < 1e-9
    else:
        e = rel_l2(O.intensity(U), O.intensity(ref))
        announce(f"  intensity rel-L2 {e:.3e}")
        assert e <= 1e-4


@pytest.mark.parametrize("path", ["fp64", "split"])
def test_aperture_smaller_than_one_tile(path):
    """N = 100: fewer rows than one GEMM row tile, K shorter than one stage
    block of the table, one Bluestein block per line."""
    ap = dict(D=1e-3, f0=10e-3, lambda0=LAM0, N=100)
    inst = dict(lam=LAM0, M=32)
    announce(f"{path} N=100 M=32")
    _, _, _, (U,) = run_gpu(ap, [inst], path=path, allow_undersampled=True)
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=64)
    if path == "fp64":
        assert rel_l2(U, ref) < 1e-9
    else:
        assert rel_l2(O.intensity(U), O.intensity(ref)) <= 1e-4


@pytest.mark.parametrize("path", ["fp64", "split"])
def test_empty_and_outside_row_ranges(path):
    """An empty row range writes a zero ROI, or leaves it as it was when
    accumulating; rows wholly outside the disc add exactly nothing."""
    ap = dict(D=1e-3, f0=4e-3, lambda0=LAM0, N=1001, pitch=1e-3 / 997)
    inst = dict(lam=LAM0, M=64, z=4.05e-3)
    announce(f"{path} empty and outside-disc row ranges")
    plan = P.Plan(ap, [inst], path=path, allow_undersampled=True)
    ws, roi = plan.alloc()
    roi.fill_(1.0)
    plan.propagate_range(ws, roi, 0, 0, accumulate=False)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(roi)) == 0
    # disc radius 997/2 samples about the centre of a 1001-sample grid: rows 0, 1 miss it
    roi.fill_(1.0)
    plan.propagate_range(ws, roi, 0, 2, accumulate=False)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(roi)) == 0
    plan.propagate(ws, roi)
    full = roi.clone()
    plan.propagate_range(ws, roi, 500, 500, accumulate=True)
    plan.propagate_range(ws, roi, 1001, 1001, accumulate=True)
    plan.propagate_range(ws, roi, 999, 1001, accumulate=True)
    torch.cuda.synchronize()
    assert torch.equal(roi, full)


def test_zero_height_creases_match_binary():
    """Creases of zero height take the complex-stripe kernels but must give
    the undeformed plate: against the binary-stripe kernels of the same plan
    shape."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=3000)
    cr = crease_draws(11, 2e-3, LAM0, 8)
    cr[:, 3] = 0.0
    announce("split zero-height creases vs binary stripes")
    _, _, _, (Uc,) = run_gpu(ap, [dict(lam=LAM0, M=128, creases=cr)], path="split", allow_undersampled=True)
    _, _, _, (Ub,) = run_gpu(ap, [dict(lam=LAM0, M=128)], path="split", allow_undersampled=True)
    e = rel_l2(O.intensity(Uc), O.intensity(Ub))
    announce(f"  intensity rel-L2 {e:.3e}")
    assert e <= 1e-4


@pytest.mark.parametrize("path", ["fp64", "split"])
def test_largest_aperture_sampled_stripe(path):
    """N = 2^21 (the largest grid the plan accepts): a 2 m f/5 plate at
    0.95 um pitch, a stripe of 64 rows through the centre against the
    oracle's restricted row sum."""
    N = 1 << 21
    ap = dict(D=2.0, f0=10.0, lambda0=LAM0, N=N)
    inst = dict(lam=LAM0, M=512)
    plan = P.Plan(ap, [inst], path=path, stripe_rows=64)
    ws, roi = plan.alloc()
    a, i = oracle_case(ap, inst)
    j0 = N // 2 - 32
    announce(f"N=2^21 {path} stripe rows {j0}..{j0 + 64}")
    plan.propagate_range(ws, roi, j0, j0 + 64, accumulate=False)
    torch.cuda.synchronize()
    U = plan.roi_view(roi, 0).cpu().numpy()
    ref = O.propagate(a, i, method="bluestein", rows=(j0, j0 + 64), stripe=16)
    e = rel_l2(U, ref)
    announce(f"  complex rel-L2 {e:.3e}")
    assert e <= (1e-6 if path == "fp64" else 1e-4)


# ---------------------------------------------------------------------------
# Seeded random shapes: both paths, every binary GEMM variant, creased or not
# ---------------------------------------------------------------------------

def _random_cases(n=16, seed=2026):
    rng = np.random.Generator(np.random.PCG64(seed))
    cases = []
    for k in range(n):
        N = int(rng.integers(64, 3200))
        D = float(rng.uniform(0.5e-3, 3e-3))
        f0 = D * float(rng.uniform(3.0, 8.0))
        M = 16 * int(rng.integers(1, 17))                # 16 .. 256, the split path's multiples of 16
        ap = dict(D=D, f0=f0, lambda0=LAM0, N=N, centre_open=int(rng.integers(0, 2)))
        if rng.random() < 0.3:
            ap["pitch"] = D / (N - int(rng.integers(0, 8)))   # disc slightly smaller than the grid
        lam = float(rng.uniform(500e-9, 800e-9))
        hw = 8 * lam * (f0 * LAM0 / lam) / D
        inst = dict(lam=lam, M=M, x0=float(rng.uniform(-0.3, 0.3)) * hw, y0=float(rng.uniform(-0.3, 0.3)) * hw,
                    half_width=hw * float(rng.uniform(0.5, 1.5)))
        if rng.random() < 0.4:
            inst["creases"] = crease_draws(int(rng.integers(0, 1000)), D, LAM0, int(rng.integers(1, 9)))
        cases.append((k, ap, inst, int(rng.integers(0, 5))))
    return cases


@pytest.mark.parametrize("case", _random_cases(), ids=lambda c: f"r{c[0]}")
def test_random_shapes_both_paths(case):
    k, ap, inst, variant = case
    announce(f"random case {k}: N={ap['N']} M={inst['M']} creases={len(inst.get('creases', []))} variant {variant}")
    _, _, _, (U64,) = run_gpu(ap, [inst], allow_undersampled=True)
    _, _, _, (Us,) = run_gpu(ap, [inst], path="split", allow_undersampled=True, variant=variant)
    a, i = oracle_case(ap, inst)
    ref = O.propagate(a, i, method="bluestein", stripe=256)
    Iref = O.intensity(ref)
    if np.linalg.norm(Iref) == 0.0:
        assert np.abs(U64).max() == 0.0 and np.abs(Us).max() == 0.0
        return
    e64 = rel_l2(U64, ref)
    es = rel_l2(O.intensity(Us), Iref)
    announce(f"  fp64 complex rel-L2 {e64:.2e}, split intensity rel-L2 {es:.2e}")
    assert e64 < 1e-9
    assert es <= 1e-4


def test_auto_path_runs_the_chosen_path():
    """path="auto" resolves at plan time and then runs exactly that path."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048)
    inst = dict(lam=LAM0, M=128)
    pa, _, _, (Ua,) = run_gpu(ap, [inst], path="auto")
    _, _, _, (Us,) = run_gpu(ap, [inst], path="split")
    assert pa.info()["path"] == 1 and np.array_equal(Ua, Us)
    pf, _, _, (Uf,) = run_gpu(ap, [dict(lam=LAM0, M=2000)], path="auto")
    _, _, _, (U6,) = run_gpu(ap, [dict(lam=LAM0, M=2000)], path="fp64")
    assert pf.info()["path"] == 0 and np.array_equal(Uf, U6)
