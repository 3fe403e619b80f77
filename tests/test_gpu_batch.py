"""GPU: batched execution - lanes, graph replay, autotuner, and the 64-instance
batch of the 20 mm element (16 wavelengths x 4 crease maps, uneven ROI sizes).

Bars: split-BF16 intensity within rel-L2 1e-4 of the FP64 path per instance;
lanes, graph replays and tuned plans reproduce their eager single-lane results
(bit for bit where the arithmetic is the same).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2609_01978_amd as P  # noqa: E402
from oracle import fzp_oracle as O  # noqa: E402
from fzp_inputs import batch64_instances, crease_draws, workload  # noqa: E402

pytestmark = pytest.mark.gpu
LAM0 = 632.8e-9


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(msg):
    print(f"[gpu-batch] {msg}", flush=True)


def small_batch():
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048)
    insts = []
    for k, (lam, M) in enumerate([(500e-9, 128), (560e-9, 64), (620e-9, 256), (700e-9, 128), (780e-9, 64)]):
        inst = dict(lam=lam, M=M)
        if k % 2 == 0:
            inst["creases"] = crease_draws(20 + k, ap["D"], LAM0, 8)
        insts.append(inst)
    return ap, insts


def views(plan, roi):
    return [plan.roi_view(roi, k).cpu().numpy() for k in range(plan.n_instances)]


@pytest.mark.parametrize("path", ["split", "fp64"])
def test_lanes_reproduce_single_lane(path):
    ap, insts = small_batch()
    announce(f"lanes {path}")
    p1 = P.Plan(ap, insts, path=path)
    ws1, roi1 = p1.alloc()
    p1.propagate(ws1, roi1)
    p3 = P.Plan(ap, insts, path=path, lanes=3)
    ws3, roi3 = p3.alloc()
    assert p3.workspace_size > p1.workspace_size
    p3.propagate(ws3, roi3)
    torch.cuda.synchronize()
    assert torch.equal(roi1, roi3)


def test_graph_replays_match_eager():
    ap, insts = small_batch()
    plan = P.Plan(ap, insts, path="split", lanes=2)
    ws, roi = plan.alloc()
    plan.propagate(ws, roi)
    torch.cuda.synchronize()
    eager = roi.clone()
    g = plan.graph(ws, roi)
    other = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(3):
        announce(f"graph replay {rep}")
        roi.fill_(float("nan"))
        other.add_(1.0)                      # eager work between replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(roi, eager), rep
    # the plan still runs eagerly after capture
    plan.propagate(ws, roi)
    torch.cuda.synchronize()
    assert torch.equal(roi, eager)


def test_autotune_and_cache(tmp_path):
    ap, insts = small_batch()
    cache = str(tmp_path / "tune.txt")
    plan = P.Plan(ap, insts, path="split", lanes=2)
    ws, roi = plan.alloc()
    t = plan.autotune(ws, roi, cache)
    announce(f"autotune {t}")
    assert t["lanes"] in (1, 2) and t["seg_len"] >= 4096 and t["ms"] > 0
    plan.propagate(ws, roi)
    torch.cuda.synchronize()
    ref_plan = P.Plan(ap, insts, path="fp64")
    wsr, roir = ref_plan.alloc()
    ref_plan.propagate(wsr, roir)
    torch.cuda.synchronize()
    for a, b in zip(views(plan, roi), views(ref_plan, roir)):
        assert rel_l2(O.intensity(a), O.intensity(b)) <= 1e-4
    # a second plan of the same shape takes the cached choice without timing
    plan2 = P.Plan(ap, insts, path="split", lanes=2)
    ws2, roi2 = plan2.alloc()
    t2 = plan2.autotune(ws2, roi2, cache)
    assert t2["ms"] == 0.0 and t2["seg_len"] == t["seg_len"] and t2["lanes"] == t["lanes"]
    assert t2["variant"] == t["variant"] and t["variant"] % 8 in (0, 1, 2, 3, 4) and t["variant"] // 8 in (0, 1, 2)
    plan2.propagate(ws2, roi2)
    torch.cuda.synchronize()
    assert torch.equal(roi2, roi)


def test_batch64_split_vs_fp64():
    """The 64-instance batch, graph-launched on both paths; every instance of the
    split path within rel-L2 1e-4 of the FP64 path; two instances also against
    the oracle on a sampled stripe."""
    w = workload("batch64")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    insts = batch64_instances()
    outs = {}
    for path, lanes in (("split", 2), ("fp64", 2)):
        announce(f"batch64 {path}")
        plan = P.Plan(ap, insts, path=path, lanes=lanes)
        ws, roi = plan.alloc()
        g = plan.graph(ws, roi)
        g.launch()
        torch.cuda.synchronize()
        outs[path] = [O.intensity(u) for u in views(plan, roi)]
        del g, ws, roi
        torch.cuda.empty_cache()
    errs = [rel_l2(a, b) for a, b in zip(outs["split"], outs["fp64"])]
    announce(f"batch64 max rel-L2 {max(errs):.3e}")
    assert max(errs) <= 1e-4
    # sampled stripes of two instances against the oracle (split path, range call)
    for k in (5, 47):
        inst = insts[k]
        plan = P.Plan(ap, [inst], path="split", stripe_rows=w["stripe"])
        ws, roi = plan.alloc()
        j0 = w["N"] // 2 - 128 + 3000 * (k % 3)
        plan.propagate_range(ws, roi, j0, j0 + w["stripe"], accumulate=False)
        torch.cuda.synchronize()
        U = plan.roi_view(roi, 0).cpu().numpy()
        a = O.Aperture(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
        i = O.Instance(lam=inst["lam"], M=inst["M"], creases=inst["creases"])
        ref = O.propagate(a, i, method="bluestein", rows=(j0, j0 + w["stripe"]), stripe=64)
        e = rel_l2(U, ref)
        announce(f"  instance {k} M={inst['M']} stripe rel-L2 {e:.3e}")
        assert e <= 1e-4


def test_overlap_operand_reproduces():
    """Operands made on the auxiliary stream one chunk ahead: same result bit for bit."""
    ap, insts = small_batch()
    outs = []
    for ov in (False, True):
        announce(f"overlap_operand={ov}")
        plan = P.Plan(ap, insts, path="split", chunk_rows=512, overlap_operand=ov)
        ws, roi = plan.alloc()
        plan.propagate(ws, roi)
        plan.propagate(ws, roi)
        torch.cuda.synchronize()
        outs.append(roi.clone())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("path,tol", [("fp64", 1e-9), ("split", 1e-4)])
def test_graph_batch_against_oracle(path, tol):
    """A graph-launched two-lane batch of mixed ROI sizes (64, 128, 256), flat and
    creased, at N = 2048: every instance's whole ROI against the oracle's
    Bluestein evaluation of Eq. 2 (complex rel-L2 for the FP64 path, intensity
    rel-L2 for the split path)."""
    ap, insts = small_batch()
    plan = P.Plan(ap, insts, path=path, lanes=2)
    ws, roi = plan.alloc()
    g = plan.graph(ws, roi)
    roi.fill_(float("nan"))
    torch.cuda.synchronize()
    g.launch()
    torch.cuda.synchronize()
    oa = O.Aperture(D=ap["D"], f0=ap["f0"], lambda0=ap["lambda0"], N=ap["N"])
    for k, (U, inst) in enumerate(zip(views(plan, roi), insts)):
        ref = O.propagate(oa, O.Instance(lam=inst["lam"], M=inst["M"], creases=inst.get("creases")),
                          method="bluestein", stripe=512)
        e = rel_l2(U, ref) if path == "fp64" else rel_l2(O.intensity(U), O.intensity(ref))
        announce(f"graph batch {path} instance {k} M={inst['M']} creased={'creases' in inst} rel-L2 {e:.2e}")
        assert e <= tol, (k, e)


@pytest.mark.skip(reason="capturing a plan with FZP_FLAG_OVERLAP_OPERAND ended in a host segmentation "
                         "fault inside fzp_graph_create, also with the auxiliary streams made before the "
                         "capture; the cause is not found, so the library refuses the combination "
                         "(FZP_E_UNSUPPORTED, tested on the CPU) and this case stays off the GPU")
def test_graph_with_overlap_operand_matches_eager():
    """FZP_FLAG_OVERLAP_OPERAND under graph capture: the auxiliary streams are
    made before the capture; the replays equal the eager single-stream result."""
    ap, insts = small_batch()
    ref = P.Plan(ap, insts, path="split", chunk_rows=512)
    wsr, roir = ref.alloc()
    ref.propagate(wsr, roir)
    plan = P.Plan(ap, insts, path="split", chunk_rows=512, lanes=2, overlap_operand=True)
    ws, roi = plan.alloc()
    announce("graph capture with overlap_operand")
    g = plan.graph(ws, roi)
    for rep in range(2):
        roi.fill_(float("nan"))
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(roi, roir), rep
