#!/usr/bin/env python3
"""Throughput of the stripe-CZT Fresnel zone plate propagation on one MI355X.

Workload (default): the binary-amplitude FZP of D = 1.0 m, f/5 (f = 5 m),
lambda = 632.8 nm, sampled on 1048576^2 points (never materialised) and
propagated onto a 512^2 ROI spanning +-8 lambda f/# at focus.  One step is one
full propagation of that aperture (row pass, column pass, output factor) plus
the focal-spot metrics (FWHM, DE, MTF), i.e. every step of the hot path.

Metric: aperture Gsamples/s into the ROI (N^2 per step / step time) for the
split-BF16 MFMA path, next to the float64 Bluestein path on the same GPU; the
split result is valid only when its ROI intensity is within rel-L2 1e-4 of the
float64 path's.  Inputs are synthetic and analytic (the zone plate itself).

Besides the headline it reports, on the same GPU: the 64-instance creased
batch of the 20 mm element (graph-launched, autotuned, with the roofline of
its complex-stripe GEMM), the 0.1 m 4- and 2-level phase plates
(``ml100mm``, ``ml100mm_l2``), the 2 mm and 20 mm elements on both paths
(``configs``), the non-paraxial path on the accuracy study's plate at
N = 28672 (``sa_czt``), a reduced run of the learned surrogate (``surrogate``; the
full 20k-solve run with ``--surrogate``), the CPU oracle on a sample of the
workload (on every core this process may use), and on request the
grid-convergence sweep of the accuracy study (``--convergence``).

Prints exactly one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fzp1m", choices=["fzp2mm", "fzp20mm", "fzp1m"])
    ap.add_argument("--fp64-steps", type=int, default=5, help="timed steps of the float64 comparison path")
    ap.add_argument("--fp64-warmup", type=int, default=1, help="untimed steps of the float64 comparison path")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 comparison path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="aperture rows in the CPU oracle sample (0: sized for about 15 s of oracle work)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 2 mm and 20 mm elements (both paths, full aperture)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the reduced surrogate run (12000 + 2000 + 1000 CZT solves, 150 epochs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch of the 20 mm element")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file for the batch plan")
    ap.add_argument("--no-multilevel", action="store_true", help="skip the 0.1 m 4-level phase plate")
    ap.add_argument("--convergence", action="store_true",
                    help="also run the grid-convergence sweep of the accuracy study (D = 0.08 m, f = 1.5 m, "
                         "532 nm, N = 1024 .. 28672) on both paths")
    ap.add_argument("--multilevel-steps", type=int, default=2)
    ap.add_argument("--surrogate", action="store_true",
                    help="train and evaluate the learned surrogate at full size (20k + 1k CZT solves) instead "
                         "of the reduced run")
    ap.add_argument("--surrogate-epochs", type=int, default=300)
    ap.add_argument("--no-sa", action="store_true",
                    help="skip the non-paraxial path on the accuracy study's plate at N = 28672")
    ap.add_argument("--sa-steps", type=int, default=3)
    ap.add_argument("--no-int8", action="store_true",
                    help="skip the int8 row pass (FZP_FLAG_SPLIT_INT8) on the same workload")
    ap.add_argument("--only", choices=["batch", "ml100mm", "sa", "configs", "blas", "surrogate", "int8",
                                       "batch_split_one_lane", "batch_int8_one_lane"],
                    default=None,
                    help="run only this section (for profiling its kernels) and print its JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (the reference kernel for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# sources of the row GEMMs whose committed counters (profiles/) the bench
# reports: the binary BF16 kernel (the dominant one), the int8 kernels and the
# complex BF16 kernel; each figure is reported only while its sources are unchanged
GEMM_SOURCES = ["paper_2609_01978_amd/csrc/fzp_gemm.hip", "paper_2609_01978_amd/csrc/fzp_split.h"]
I8_SOURCES = ["paper_2609_01978_amd/csrc/fzp_i8.hip", "paper_2609_01978_amd/csrc/fzp_split.h"]
CPLX_SOURCES = ["paper_2609_01978_amd/csrc/fzp_cplx.hip", "paper_2609_01978_amd/csrc/fzp_split.h"]

# MI355X published peaks
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP64_TFLOPS = 78.6
PEAK_INT8_TOPS = 5000.0        # dense int8 MFMA
PEAK_HBM_GBS = 8000.0


def kernel_sources_sha256(kernel_srcs) -> str:
    """SHA-256 over the concatenated kernel source files (repository-relative)."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in kernel_srcs:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_value(kernel_srcs, summary: str, key: str):
    """A `key: value` figure from a committed rocprofv3 summary, or None when the
    kernel sources changed since its counters were taken."""
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(here, summary)).read()
        digest = kernel_sources_sha256(kernel_srcs)
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and not line.startswith(("|", "#")))
    if vals.get("kernel_source_sha256", "").strip() != digest or key not in vals:
        return None
    return float(vals[key])


def committed_traffic(kernel_srcs, summary: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources changed since the counters were taken."""
    return committed_value(kernel_srcs, summary, "traffic_bytes_per_launch")


def bluestein_blocks(N: int, B: int) -> int:
    """Blocks of B samples covering every aperture row's disc chord (row pass)."""
    import numpy as np
    c = 2 * np.arange(N, dtype=np.int64) - (N - 1)
    rem = N * N - c * c
    m = np.floor(np.sqrt(np.maximum(rem, 0).astype(np.float64))).astype(np.int64)
    m -= (m * m > rem)
    m += ((m + 1) * (m + 1) <= rem)
    lo = (N - 1 - m + 1) // 2
    hi = (N - 1 + m) // 2 + 1
    length = np.where(rem >= 0, hi - lo, 0)
    return int(np.sum((length + B - 1) // B))


def host_cpu():
    """(CPU model, threads this process may use): the affinity mask, capped by
    OMP_NUM_THREADS when the host sets it (the host's share of its cores)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return model, max(n, 1)


def cpu_baseline(w, rows_n: int):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload:
    `rows_n` aperture rows through the middle of the aperture, Bluestein form,
    with scipy.fft's workers (and the BLAS threads) on every core this process
    may use.  rows_n = 0 sizes the sample for about 15 s from a 64-row probe."""
    import numpy as np
    from scipy import fft as sfft
    from oracle import fzp_oracle as O
    model, cores = host_cpu()
    a = O.Aperture(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    i = O.Instance(lam=w["lambda0"], M=w["M"])
    N = a.N
    stripe = 64

    def timed(rows):
        j0 = N // 2 - rows // 2
        t = time.perf_counter()
        with sfft.set_workers(cores):
            O.propagate(a, i, method="bluestein", rows=(j0, j0 + rows), stripe=stripe)
        return time.perf_counter() - t

    if rows_n <= 0:
        probe = timed(stripe)
        rows_n = int(min(max(15.0 / max(probe, 1e-3) * stripe, stripe), N)) // stripe * stripe
    dt = timed(rows_n)
    return dict(value=rows_n * N / dt / 1e9, unit="Gsamples/s", cores=cores, cpu_model=model, kind="oracle",
                sample=f"{rows_n} aperture rows x {N} columns through the centre of the {w['D']} m aperture "
                       f"(float64 Bluestein form, scipy.fft with {cores} workers, NumPy's elementwise steps on one "
                       f"thread), {dt:.1f} s")


def run_batch(args, dev):
    """64 instances of the 20 mm element (16 wavelengths x 4 crease maps, ROI
    sizes from {256, 512, 1024}), each path captured as one HIP graph; the split
    plans (BF16, and the int8 row pass) are autotuned first.  Valid when every
    instance's split intensity is within rel-L2 1e-4 of the FP64 path's."""
    import numpy as np
    import torch
    import paper_2609_01978_amd as P
    from fzp_inputs import workload, batch64_instances
    w = workload("batch64")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    insts = batch64_instances()
    samples = len(insts) * float(w["N"]) ** 2
    res, I = {}, {}
    for path in ("split", "split_int8", "fp64"):
        i8 = path == "split_int8"
        plan = P.Plan(ap, insts, path="fp64" if path == "fp64" else "split", lanes=2, int8=i8)
        ws, roi = plan.alloc(dev)
        plan.prepare(ws)
        tune = plan.autotune(ws, roi, args.tune_cache if not i8 else None) if path != "fp64" else None
        g = plan.graph(ws, roi)
        g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            g.launch()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.batch_steps
        log(f"batch64 {path}: {dt * 1e3:.1f} ms per batch")
        I[path] = [plan.roi_view(roi, k).abs().square().cpu().numpy() for k in range(len(insts))]
        res[path] = {"gsamples_s": round(samples / dt / 1e9, 3), "ms_per_batch": round(dt * 1e3, 3),
                     "workspace_gib": round(plan.workspace_size / 2 ** 30, 2)}
        if tune is not None:
            res[path]["autotune"] = tune
        del g, ws, roi
        torch.cuda.empty_cache()
        if path == "fp64":
            continue
        # Roofline of the batch's dominant kernel, the complex-stripe row GEMM:
        # 24 M operations per disc sample of a creased instance (three split
        # products of a complex product; BF16 pairs, or int8 digits).  One more
        # propagation on a one-lane plan with HIP events around each launch, so
        # that no interval holds another lane's kernels.
        plan = P.Plan(ap, insts, path="split", lanes=1, int8=i8)
        ws, roi = plan.alloc(dev)
        plan.propagate(ws, roi)
        torch.cuda.synchronize()
        plan.profile(True)
        plan.profile_read(reset=True)
        plan.propagate(ws, roi)
        torch.cuda.synchronize()
        pr = plan.profile_read(reset=True)
        disc = float(plan.info()["disc_samples"])
        flops = sum(24.0 * inst["M"] * disc for inst in insts)
        ach = flops / (pr["row_ms"] * 1e-3) / 1e12
        peak = PEAK_INT8_TOPS if i8 else PEAK_BF16_TFLOPS
        # counters of this configuration's row GEMM, taken in runs of their own
        # (bench.py --only batch_split_one_lane / batch_int8_one_lane)
        summary = ("profiles/counters_k_row_pass_i8_cplx_batch64.md" if i8
                   else "profiles/counters_k_row_pass_split_cplx_batch64.md")
        srcs = I8_SOURCES if i8 else CPLX_SOURCES
        traffic = committed_traffic(srcs, summary)
        busy = committed_value(srcs, summary, "mfma_busy_fraction_of_cycles")
        res[path]["roofline"] = dict(bound="mfma", achieved=round(ach, 1), peak=peak,
                                     unit="TOP/s" if i8 else "TFLOP/s", frac=round(ach / peak, 4),
                                     traffic=traffic, mfma_busy=busy,
                                     committed_from=summary + " (traffic per launch, mfma_busy)"
                                     if traffic is not None or busy is not None else None,
                                     kernel="k_row_pass_i8_cplx" if i8 else "k_row_pass_split_cplx",
                                     launches=pr["row_launches"], row_gemm_ms=round(pr["row_ms"], 3),
                                     stripe_ms=round(pr["mask_ms"], 3), col_pass_ms=round(pr["col_ms"], 3),
                                     flops_per_batch=flops,
                                     work="24 M operations per disc sample of each creased instance (one lane, "
                                          "default K segments)")
        del ws, roi, plan
        torch.cuda.empty_cache()
    errs = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(I["split"], I["fp64"])]
    errs8 = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(I["split_int8"], I["fp64"])]
    res["split_int8"].update({"max_rel_l2_vs_fp64": max(errs8), "valid_rel_l2_le_1e-4": max(errs8) <= 1e-4,
                              "speedup_vs_fp64": round(res["fp64"]["ms_per_batch"] /
                                                       res["split_int8"]["ms_per_batch"], 3)})
    return {"workload": "64 instances: D=20 mm f/5 N=32768^2, lambda 500-800 nm x 4 crease maps (8 creases), "
                        "M in {256,512,1024}", "instances": len(insts), "steps": args.batch_steps,
            "split_bf16": res["split"], "fp64_bluestein": res["fp64"], "split_int8": res["split_int8"],
            "max_rel_l2_split_vs_fp64": max(errs), "valid_rel_l2_le_1e-4": max(errs) <= 1e-4,
            "speedup_split_vs_fp64": round(res["fp64"]["ms_per_batch"] / res["split"]["ms_per_batch"], 3)}


def run_batch_one_lane(dev, int8: bool):
    """One propagation of the creased batch on the split path (int8 or BF16
    row pass), one lane, default K segments and tile: the configuration of the
    batch roofline, alone, for counter runs of its kernels."""
    import torch
    import paper_2609_01978_amd as P
    from fzp_inputs import workload, batch64_instances
    w = workload("batch64")
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    insts = batch64_instances()
    plan = P.Plan(ap, insts, path="split", lanes=1, int8=int8)
    ws, roi = plan.alloc(dev)
    t0 = time.perf_counter()
    plan.propagate(ws, roi)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"instances": len(insts), "ms_first_propagation": round(dt * 1e3, 3)}


def run_multilevel(args, dev, levels=None):
    """The 0.1 m f/5 L-level phase plate (the revised engine's kind of element;
    L = 4 by default, 2 for the 2-level shortcut) on both paths: one
    propagation plus metrics per step.  Valid when the split
    intensity is within rel-L2 1e-4 of the FP64 path's; the main-lobe DE is
    reported next to the L-level ladder value sinc^2(1/L) times the Airy lobe
    share 1 - J0(j_{1,1})^2."""
    import math
    import numpy as np
    import torch
    from scipy import special
    import paper_2609_01978_amd as P
    from fzp_inputs import workload
    w = workload("ml100mm")
    L = w["levels"] if levels is None else levels
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"], levels=L)
    inst = dict(lam=w["lambda0"], M=w["M"])
    samples = float(w["N"]) ** 2
    res, I = {}, {}
    # the int8 row pass covers the 2- and 4-level plates (binary-mask products)
    for path in ("split", "fp64") + (("split_int8",) if L in (2, 4) else ()):
        i8 = path == "split_int8"
        plan = P.Plan(ap, [inst], path="fp64" if path == "fp64" else "split",
                      stripe_rows=0 if path == "fp64" else w["stripe"], int8=i8)
        ws, roi = plan.alloc(dev)
        plan.prepare(ws)
        plan.propagate(ws, roi)
        plan.metrics(ws, roi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.multilevel_steps):
            plan.propagate(ws, roi)
            m = plan.metrics(ws, roi)[0]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.multilevel_steps
        log(f"ml100mm L={L} {path}: {dt * 1e3:.1f} ms per propagation")
        I[path] = plan.roi_view(roi, 0).abs().square().cpu().numpy()
        res[path] = {"gsamples_s": round(samples / dt / 1e9, 3), "ms_per_step": round(dt * 1e3, 3),
                     "de": m["de"], "fwhm_x": m["fwhm_x"], "strehl": m["strehl"]}
        if path != "fp64":
            # the row GEMM's own time (HIP events around its launches, one more
            # propagation): 8 M flops per disc sample for a 2-level plate (the
            # binary GEMM of its odd zones), 16 M for a 4-level plate (two binary
            # GEMMs: the odd zones and the levels 1 and 2), 24 M otherwise
            plan.profile(True)
            plan.profile_read(reset=True)
            plan.propagate(ws, roi)
            torch.cuda.synchronize()
            pr = plan.profile_read(reset=True)
            plan.profile(False)
            per = (8.0 if L == 2 else 16.0 if L == 4 else 24.0) * w["M"]
            flops = per * float(plan.info()["disc_samples"])
            ach = flops / (pr["row_ms"] * 1e-3) / 1e12
            peak = PEAK_INT8_TOPS if i8 else PEAK_BF16_TFLOPS
            res[path]["roofline"] = dict(bound="mfma", achieved=round(ach, 1), peak=peak,
                                         unit="TOP/s" if i8 else "TFLOP/s", frac=round(ach / peak, 4),
                                         kernel="k_row_pass_i8" if i8 else
                                         "k_row_pass_split" if L in (2, 4) else "k_row_pass_split_cplx",
                                         launch_ms=round(
                                             pr["row_ms"] / max(pr["row_launches"], 1), 3),
                                         work=f"{per / w['M']:.0f} M flops per disc sample")
        del ws, roi, plan
        torch.cuda.empty_cache()
    e = float(np.linalg.norm(I["split"] - I["fp64"]) / np.linalg.norm(I["fp64"]))
    x = math.pi / L
    lobe = 1.0 - float(special.j0(special.jn_zeros(1, 1)[0])) ** 2
    out = {"workload": f"{L}-level phase FZP D={w['D']} m f/5 lambda0=632.8 nm, N={w['N']}^2, ROI {w['M']}^2",
           "steps": args.multilevel_steps, "split_bf16": res["split"], "fp64_bluestein": res["fp64"],
           "rel_l2_split_vs_fp64": e, "valid_rel_l2_le_1e-4": e <= 1e-4,
           "de_ladder_sinc2": round((math.sin(x) / x) ** 2 * lobe, 6),
           "speedup_split_vs_fp64": round(res["fp64"]["ms_per_step"] / res["split"]["ms_per_step"], 3)}
    if "split_int8" in res:
        e8 = float(np.linalg.norm(I["split_int8"] - I["fp64"]) / np.linalg.norm(I["fp64"]))
        out["split_int8"] = dict(res["split_int8"], **{
            "rel_l2_vs_fp64": e8, "valid_rel_l2_le_1e-4": e8 <= 1e-4,
            "speedup_vs_fp64": round(res["fp64"]["ms_per_step"] / res["split_int8"]["ms_per_step"], 3)})
    return out


def run_configs(dev, steps: int = 3):
    """The 2 mm (N = 4096, M = 256) and 20 mm (N = 32768, M = 1024) elements on
    both paths and the int8 row pass: whole-aperture propagation plus metrics
    per step, after one warm-up step; split intensities against the FP64
    path's."""
    import numpy as np
    import torch
    import paper_2609_01978_amd as P
    from fzp_inputs import workload
    out = {}
    for name in ("fzp2mm", "fzp20mm"):
        w = workload(name)
        ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
        inst = dict(lam=w["lambda0"], M=w["M"])
        samples = float(w["N"]) ** 2
        res, I = {}, {}
        for path in ("split", "split_int8", "fp64"):
            plan = P.Plan(ap, [inst], path="fp64" if path == "fp64" else "split",
                          stripe_rows=0 if path == "fp64" else w["stripe"], int8=path == "split_int8")
            ws, roi = plan.alloc(dev)
            plan.propagate(ws, roi)
            plan.metrics(ws, roi)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.propagate(ws, roi)
                m = plan.metrics(ws, roi)[0]
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            I[path] = plan.roi_view(roi, 0).abs().square().cpu().numpy()
            res[path] = {"gsamples_s": round(samples / dt / 1e9, 3), "ms_per_step": round(dt * 1e3, 3),
                         "fwhm_x": m["fwhm_x"], "de": m["de"]}
            del ws, roi, plan
            torch.cuda.empty_cache()
        e = float(np.linalg.norm(I["split"] - I["fp64"]) / np.linalg.norm(I["fp64"]))
        e8 = float(np.linalg.norm(I["split_int8"] - I["fp64"]) / np.linalg.norm(I["fp64"]))
        log(f"{name}: split {res['split']['ms_per_step']} ms, int8 {res['split_int8']['ms_per_step']} ms, "
            f"fp64 {res['fp64']['ms_per_step']} ms, rel-L2 {e:.2e} / {e8:.2e}")
        res["split_int8"].update({"rel_l2_vs_fp64": e8, "valid_rel_l2_le_1e-4": e8 <= 1e-4,
                                  "speedup_vs_fp64": round(res["fp64"]["ms_per_step"] /
                                                           res["split_int8"]["ms_per_step"], 3)})
        out[name] = {"workload": f"binary FZP D={w['D']} m f/5 lambda=632.8 nm, N={w['N']}^2, ROI {w['M']}^2",
                     "steps": steps, "split_bf16": res["split"], "fp64_bluestein": res["fp64"],
                     "split_int8": res["split_int8"],
                     "rel_l2_split_vs_fp64": e, "valid_rel_l2_le_1e-4": e <= 1e-4,
                     "speedup_split_vs_fp64": round(res["fp64"]["ms_per_step"] / res["split"]["ms_per_step"], 3)}
    return out


def run_sa(args, dev):
    """The non-paraxial path (FZP_PATH_SA_CZT) on the accuracy study's plate
    (Sec. 4.1: binary, D = 0.08 m, f = 1.5 m, 532 nm, Eq. 3 radii) at its
    largest grid N = 28672 (padded to 43200^2, 29.9 GB in HBM), ROI 512^2:
    one propagation plus metrics per step.  Roofline of the padded-field
    passes: HBM-bound, 13 sweeps of the padded field per propagation (the
    first pass writes it, six passes read and write it).  The oracle is timed
    on a 4096^2 sample of the same plate (padded to 6144^2) for context."""
    import numpy as np
    import torch
    import paper_2609_01978_amd as P
    from oracle import fzp_oracle as O
    from oracle import sa_czt_oracle as S
    from scipy import fft as sfft
    D, f, lam, N, M = 0.08, 1.5, 532e-9, 28672, 512
    plan = P.Plan(dict(D=D, f0=f, lambda0=lam, N=N), [dict(lam=lam, M=M)], path="sa")
    g = plan.geometry()
    ws, roi = plan.alloc(dev)
    plan.prepare(ws)
    plan.propagate(ws, roi)
    plan.metrics(ws, roi)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.sa_steps):
        plan.propagate(ws, roi)
        m = plan.metrics(ws, roi)[0]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.sa_steps
    pr = plan.profile_read(reset=True)
    plan.profile(False)
    log(f"sa_czt N={N}: {dt * 1e3:.1f} ms per propagation")
    del ws, roi, plan
    torch.cuda.empty_cache()
    Np = g["padded_n"]
    field_ms = pr["mask_ms"] / args.sa_steps
    bytes_field = 13.0 * Np * Np * 16.0
    ach = bytes_field / (field_ms * 1e-3) / 1e9
    model, cores = host_cpu()
    a = O.Aperture(D=D, f0=f, lambda0=lam, N=4096)
    t1 = time.perf_counter()
    with sfft.set_workers(cores):
        S.sa_czt(a, O.Instance(lam=lam, M=M))
    t_cpu = time.perf_counter() - t1
    return {"workload": f"binary FZP with Eq. 3 radii, D={D} m f={f} m lambda=532 nm, N={N}^2 padded to {Np}^2 "
                        f"({g['fft_n1']} x {g['fft_n2']} per axis), ROI {M}^2",
            "steps": args.sa_steps, "ms_per_step": round(dt * 1e3, 3),
            "gsamples_s": round(float(N) * N / dt / 1e9, 3),
            "padded_gsamples_s": round(float(Np) * Np / dt / 1e9, 3),
            "field_ms": round(field_ms, 3), "zoom_row_ms": round(pr["row_ms"] / args.sa_steps, 3),
            "zoom_col_ms": round(pr["col_ms"] / args.sa_steps, 3),
            "metrics": m, "zones_eq3": g["zones_exact"], "zoom_distance_m": g["zoom_distance"],
            "roofline": dict(bound="hbm", achieved=round(ach, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                             frac=round(ach / PEAK_HBM_GBS, 4), kernel="k_sa_pass (7 launches)",
                             bytes_per_step=bytes_field,
                             work="13 sweeps of the padded float64 complex field per propagation"),
            "cpu_oracle_sample": {"value": round(4096.0 * 4096 / t_cpu / 1e9, 5), "unit": "Gsamples/s",
                                  "cores": cores, "cpu_model": model, "kind": "oracle",
                                  "sample": f"the same plate on 4096^2 samples (padded 6144^2), {t_cpu:.1f} s"}}


# Closed forms of the ideal Airy pattern (aberration-free circular pupil):
# FWHM = 1.028994 lambda f / D (half maximum of (2 J1(v)/v)^2 at v = 1.61634),
# main-lobe share 1 - J0(j11)^2 of the first order, which carries 1/pi^2 of the
# incident power for a binary amplitude plate, and the incoherent MTF
# (2/pi)(acos(s) - s sqrt(1 - s^2)) at s = 1/2.
AIRY_FWHM_FACTOR = 1.028994


def run_convergence(dev):
    """Grid-convergence sweep of the accuracy study (Sec. 4.1, Figs. 6-8): the
    binary, negative-centred plate D = 0.08 m, f = 1.5 m at 532 nm on grids
    N = 1024 .. 28672, ROI 512^2 at +-8 lambda f/#; FWHM, main-lobe DE and MTF
    at half cutoff against the Airy closed forms, for both paths."""
    import math
    import numpy as np
    import torch
    from scipy import special
    import paper_2609_01978_amd as P
    D, f, lam = 0.08, 1.5, 532e-9
    j11 = float(special.jn_zeros(1, 1)[0])
    ref = {"fwhm": AIRY_FWHM_FACTOR * lam * f / D,
           "de": (1.0 - float(special.j0(j11)) ** 2) / math.pi ** 2,
           "mtf": 2.0 / math.pi * (math.acos(0.5) - 0.5 * math.sqrt(0.75))}
    rows = []
    for N in (1024, 2048, 4096, 8192, 12288, 16384, 20480, 24576, 28672):
        ap = dict(D=D, f0=f, lambda0=lam, N=N)
        inst = dict(lam=lam, M=512)
        I = {}
        for path in ("split", "fp64"):
            plan = P.Plan(ap, [inst], path=path, allow_undersampled=True)
            ws, roi = plan.alloc(dev)
            plan.prepare(ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.propagate(ws, roi)
            m = plan.metrics(ws, roi)[0]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            I[path] = plan.roi_view(roi, 0).abs().square().cpu().numpy()
            rows.append({"N": N, "path": path, "ms": round(dt * 1e3, 3),
                         "fwhm_err_pct": round(100.0 * (0.5 * (m["fwhm_x"] + m["fwhm_y"]) / ref["fwhm"] - 1), 5),
                         "de_err_pct": round(100.0 * (m["de"] / ref["de"] - 1), 5),
                         "mtf_err_pct": round(100.0 * (m["mtf_half_cut"] / ref["mtf"] - 1), 5)})
            del ws, roi, plan
            torch.cuda.empty_cache()
        e = float(np.linalg.norm(I["split"] - I["fp64"]) / np.linalg.norm(I["fp64"]))
        rows[-2]["rel_l2_vs_fp64"] = e
        log(f"convergence N={N}: {rows[-1]}; split rel-L2 vs fp64 {e:.2e}")
    return {"workload": "binary FZP D=0.08 m f=1.5 m lambda=532 nm, ROI 512^2 at +-8 lambda f/#",
            "reference": {k: round(v, 9) for k, v in ref.items()}, "rows": rows}


def run_surrogate(args):
    """The learned surrogate: CZT data, prior, training, gate, test report; the
    configured size (20k solves, 300 epochs) with --surrogate, else reduced."""
    from paper_2609_01978_amd import surrogate as SG
    from fzp_inputs import workload
    sw = workload("surrogate")
    if args.surrogate:
        return SG.run(sw, sw["n_train"] - 2000, 2000, sw["n_test"], args.surrogate_epochs, log=log)
    r = SG.run(sw, 12000, 2000, 1000, 150, log=log)
    r["reduced"] = "12000 training, 2000 validation, 1000 test solves, 150 epochs"
    return r


def run_blas(dev):
    """The vendor BF16 GEMM (torch.matmul, hipBLASLt on ROCm) on this GPU, for
    what a library GEMM attains against the same 2.5 PFLOP/s dense peak: a
    square 16384^3 product and one shaped like a binary-stripe row pass (16384
    aperture rows x one 65536-column K segment x 1024 real ROI columns)."""
    import torch
    out = {}
    for name, (m, k, n) in {"square_16384": (16384, 16384, 16384),
                            "row_pass_shape": (16384, 65536, 1024)}.items():
        a = torch.randn(m, k, device=dev, dtype=torch.bfloat16)
        b = torch.randn(k, n, device=dev, dtype=torch.bfloat16)
        for _ in range(3):
            c = a @ b
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 2.0 * m * k * n / ms / 1e9
        out[name] = {"m": m, "k": k, "n": n, "ms": round(ms, 4), "tflops": round(tf, 1),
                     "frac_of_bf16_peak": round(tf / PEAK_BF16_TFLOPS, 4)}
        log(f"torch.matmul bf16 {m}x{k}x{n}: {ms:.3f} ms, {tf:.0f} TFLOP/s")
        del a, b, c
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; a multi-GPU job gives each GPU a range of aperture rows "
              "(fzp_propagate_roi_range) and sums the ROIs.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2609_01978_amd as P
    from fzp_inputs import workload

    if args.copy_calibration:
        # 1 GiB read + 1 GiB written per copy; FETCH_SIZE / WRITE_SIZE of this
        # kernel scale the counters of the library's kernels to bytes
        n = 1 << 30
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}), flush=True)
        return

    if args.only is not None and args.only != "int8":
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        run = {"batch": lambda: run_batch(args, dev), "ml100mm": lambda: run_multilevel(args, dev),
               "sa": lambda: run_sa(args, dev), "configs": lambda: run_configs(dev),
               "blas": lambda: run_blas(dev), "surrogate": lambda: run_surrogate(args),
               "batch_split_one_lane": lambda: run_batch_one_lane(dev, int8=False),
               "batch_int8_one_lane": lambda: run_batch_one_lane(dev, int8=True)}[args.only]
        print(json.dumps({args.only: run()}), flush=True)
        return

    w = workload(args.workload)
    ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
    inst = dict(lam=w["lambda0"], M=w["M"])
    N, M, S = w["N"], w["M"], w["stripe"]
    samples = float(N) * float(N)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def run_path(path, steps, warmup, int8=False):
        plan = P.Plan(ap, [inst], path=path, stripe_rows=S, int8=int8)
        ws, roi = plan.alloc(dev)
        t0 = time.perf_counter()
        plan.prepare(ws)
        torch.cuda.synchronize()
        t_prep = time.perf_counter() - t0
        for k in range(warmup):
            plan.propagate(ws, roi)
            plan.metrics(ws, roi)
            log(f"{path} warmup {k + 1}/{warmup} done")
        torch.cuda.synchronize()
        plan.profile(True)
        plan.profile_read(reset=True)
        t0 = time.perf_counter()
        metrics = None
        for k in range(steps):
            plan.propagate(ws, roi)
            metrics = plan.metrics(ws, roi)[0]   # synchronises the stream
            log(f"{path} step {k + 1}/{steps} done")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = plan.profile_read(reset=True)
        plan.profile(False)
        I = plan.roi_view(roi, 0).abs().square().cpu().numpy()
        info = plan.info()
        del ws, roi
        torch.cuda.empty_cache()
        return dict(ms=dt / steps * 1e3, prep_s=t_prep, prof=prof, metrics=metrics, I=I, info=info)

    def int8_section(ref_I, split_I, split_ms):
        """The int8 row pass on the same workload: samples/s, the row GEMM
        against the int8 matrix-core peak (8 M int8 operations per disc sample:
        2 digits x 2 real columns x 2 per multiply-add), intensity against the
        FP64 path's and the BF16 split's."""
        r = run_path("split", args.steps, args.warmup, int8=True)
        pr8 = r["prof"]
        row8 = pr8["row_ms"] / max(args.steps, 1)
        ops = 8.0 * M * float(r["info"]["disc_samples"])
        ach8 = ops / (row8 * 1e-3) / 1e12
        res = {"dtype": "i8", "gsamples_s": round(samples / (r["ms"] * 1e-3) / 1e9, 3), "ms_per_step": round(r["ms"], 3),
               "row_pass_ms": round(row8, 3), "mask_bits_ms": round(pr8["mask_ms"] / max(args.steps, 1), 3),
               "col_pass_ms": round(pr8["col_ms"] / max(args.steps, 1), 3), "metrics": r["metrics"],
               "roofline": dict(bound="mfma", achieved=round(ach8, 1), peak=PEAK_INT8_TOPS, unit="TOP/s",
                                frac=round(ach8 / PEAK_INT8_TOPS, 4), kernel="k_row_pass_i8",
                                traffic=committed_traffic(I8_SOURCES, "profiles/hbm_traffic_k_row_pass_i8_fzp1m.md")
                                if args.workload == "fzp1m" else None,
                                mfma_busy=committed_value(I8_SOURCES, "profiles/sq_counters_k_row_pass_i8_fzp1m.md",
                                                          "mfma_busy_fraction_of_cycles")
                                if args.workload == "fzp1m" else None,
                                committed_from="profiles/hbm_traffic_k_row_pass_i8_fzp1m.md (traffic), "
                                               "profiles/sq_counters_k_row_pass_i8_fzp1m.md (mfma_busy)",
                                launch_ms=round(pr8["row_ms"] / max(pr8["row_launches"], 1), 3),
                                work="8 M int8 operations per aperture sample inside the disc (two digits)")}
        if ref_I is not None:
            e = float(np.linalg.norm(r["I"] - ref_I) / np.linalg.norm(ref_I))
            res["rel_l2_vs_fp64"] = e
            res["valid_rel_l2_le_1e-4"] = e <= 1e-4
        if split_I is not None:
            res["rel_l2_vs_split_bf16"] = float(np.linalg.norm(r["I"] - split_I) / np.linalg.norm(split_I))
            res["speedup_vs_split_bf16"] = round(split_ms / r["ms"], 3)
        return res

    if args.only == "int8":
        print(json.dumps({"int8": int8_section(None, None, None)}), flush=True)
        return

    log(f"workload {args.workload}: N={N} M={M} stripe={S}")
    split = run_path("split", args.steps, args.warmup)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_path("fp64", args.fp64_steps, args.fp64_warmup)

    value = samples / (split["ms"] * 1e-3) / 1e9
    rel = None
    if fp64 is not None:
        rel = float(np.linalg.norm(split["I"] - fp64["I"]) / np.linalg.norm(fp64["I"]))

    # Roofline of the dominant kernel, the split row-pass GEMM (k_row_pass_split).
    # Algorithmic work: the binary stripe times the hi/lo split kernel matrix is
    # 2 real products (hi, lo) x 2 real MACs (re, im) per complex ROI column per
    # aperture sample inside the disc = 8 M flops per disc sample.  The launch
    # time comes from HIP events around each launch on the library's stream.
    info = split["info"]
    disc = float(info["disc_samples"])
    pr = split["prof"]
    launches_per_step = pr["row_launches"] / max(args.steps, 1)
    row_ms_step = pr["row_ms"] / max(args.steps, 1)
    flops_step = 8.0 * M * disc
    achieved = flops_step / (row_ms_step * 1e-3) / 1e12
    traffic = committed_traffic(GEMM_SOURCES, "profiles/hbm_traffic_k_row_pass_split_fzp1m.md") \
        if args.workload == "fzp1m" else None
    # matrix-core busy share of the kernel's cycles (SQ counters): with the
    # clock under load it accounts for the gap between `frac` and 1
    mfma_busy = committed_value(GEMM_SOURCES, "profiles/sq_counters_k_row_pass_split_fzp1m.md",
                                "mfma_busy_fraction_of_cycles") if args.workload == "fzp1m" else None
    roofline = dict(bound="mfma", achieved=round(achieved, 1), peak=PEAK_BF16_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_BF16_TFLOPS, 4), traffic=traffic,
                    traffic_unit="bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    mfma_busy=mfma_busy,
                    committed_from=("profiles/hbm_traffic_k_row_pass_split_fzp1m.md (traffic), "
                                    "profiles/sq_counters_k_row_pass_split_fzp1m.md (mfma_busy): rocprofv3 "
                                    "counter runs of the same sources, not this run"),
                    kernel="k_row_pass_split",
                    launch_ms=round(pr["row_ms"] / max(pr["row_launches"], 1), 3),
                    launches_per_step=launches_per_step,
                    flops_per_launch=flops_step / max(launches_per_step, 1),
                    work="8 M flops per aperture sample inside the disc (binary stripe, hi+lo BF16 products)")

    out = {
        "metric": "aperture Gsamples/s into ROI: split-BF16 MFMA vs FP64 Bluestein, rel-L2<=1e-4",
        "value": round(value, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(split["ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"binary FZP D={w['D']} m f/5 lambda=632.8 nm, N={N}^2 samples, ROI {M}^2, "
                               f"stripe {S} rows", "N": N, "M": M, "stripe_rows": S,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "split_bf16": {"gsamples_s": round(value, 3), "ms_per_step": round(split["ms"], 3),
                       "row_pass_ms": round(row_ms_step, 3),
                       "mask_bits_ms": round(pr["mask_ms"] / max(args.steps, 1), 3),
                       "col_pass_ms": round(pr["col_ms"] / max(args.steps, 1), 3),
                       "prepare_s": round(split["prep_s"], 3), "metrics": split["metrics"]},
        "valid_rel_l2_le_1e-4": (rel is not None and rel <= 1e-4),
        "rel_l2_split_vs_fp64": rel,
    }
    if fp64 is not None:
        pf = fp64["prof"]
        row_ms64 = pf["row_ms"] / max(args.fp64_steps, 1)
        L, B = fp64["info"]["fft_len"], fp64["info"]["block"]
        nblk = bluestein_blocks(N, B)
        # algorithmic work per block: forward + inverse FFT of length L (5 L log2 L
        # flops each) and the complex product with the filter spectrum (6 L)
        flops64 = nblk * (2 * 5.0 * L * np.log2(L) + 6.0 * L)
        ach64 = flops64 / (row_ms64 * 1e-3) / 1e12
        out["fp64_bluestein"] = {"gsamples_s": round(samples / (fp64["ms"] * 1e-3) / 1e9, 3),
                                 "ms_per_step": round(fp64["ms"], 3),
                                 "row_pass_ms": round(row_ms64, 3),
                                 "col_pass_ms": round(pf["col_ms"] / max(args.fp64_steps, 1), 3),
                                 "prepare_s": round(fp64["prep_s"], 3), "metrics": fp64["metrics"],
                                 "fft_len": L, "block": B, "bluestein_blocks": int(nblk),
                                 "roofline": dict(bound="alu", achieved=round(ach64, 2), peak=PEAK_FP64_TFLOPS,
                                                  unit="TFLOP/s", frac=round(ach64 / PEAK_FP64_TFLOPS, 4),
                                                  kernel="k_row_pass_fp64")}
        out["speedup_split_vs_fp64"] = round(fp64["ms"] / split["ms"], 3)
    if not args.no_int8:
        out["split_int8"] = int8_section(fp64["I"] if fp64 is not None else None, split["I"], split["ms"])
    if not args.no_batch:
        out["batch64"] = run_batch(args, dev)
    if not args.no_multilevel:
        out["ml100mm"] = run_multilevel(args, dev)
        out["ml100mm_l2"] = run_multilevel(args, dev, levels=2)
    if not args.no_configs:
        out["configs"] = run_configs(dev)
    if not args.no_sa:
        out["sa_czt"] = run_sa(args, dev)
    if args.convergence:
        out["convergence"] = run_convergence(dev)
    if args.surrogate or not args.no_surrogate:
        out["surrogate"] = run_surrogate(args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
