"""Learned surrogate of the deformed zone plate's focal spot.

A 33 -> 512 -> 512 -> M^2 perceptron (the library's ``fzp_mlp_*`` kernels)
maps 8 straight creases (angle, offset, width, height) and the wavelength to
the log-intensity ``ln(I / I0 + FLOOR)`` of the M x M focal-plane ROI, with
``I0 = (R^2 / (lambda0 f0))^2`` the peak scale of the undeformed plate (its
on-axis intensity is close to the square of twice the number of open zones).
It is trained on the split-BF16 CZT propagation of the same plate; the CZT is
also its arbiter and its fallback: a 2-member ensemble is trained from two
seeds, and a prediction is accepted only when the input lies inside the
training box and the two members' FWHMs agree within a threshold calibrated
on held-out validation solves so that accepted validation cases keep the FWHM
error within the target.  Everything numeric runs in the library's kernels
(propagation, targets, network, FWHM); this module orchestrates them.
"""
from __future__ import annotations

import math
import time
from typing import Optional

import numpy as np

from . import _lib

N_IN = 33
HIDDEN = 512
# Log floor relative to I0: intensities far below the main lobe and the first
# rings (which set the FWHM) are flattened instead of resolving every null.
FLOOR = 1e-2


def i0_scale(D: float, f0: float, lambda0: float) -> float:
    """(R^2/(lambda0 f0))^2: the undeformed plate's peak intensity scale (N_F^2)."""
    R = 0.5 * D
    return (R * R / (lambda0 * f0)) ** 2


def features(creases: np.ndarray, lams: np.ndarray, D: float, lambda0: float,
             lam_lo: float = 500e-9, lam_hi: float = 800e-9) -> np.ndarray:
    """Network inputs in [-1, 1] over the training box: per crease the angle
    (U[0, pi)), offset (U[-R, R]), width (U[0.5, 2] mm) and height (U[0, lambda0/2]),
    then the wavelength (U[lam_lo, lam_hi]).  Returns float32 [n, 8*4 + 1].
    The creases of a map are an unordered set; they are listed by decreasing
    height (the strongest phase ridge first) so that one deformation has one
    input vector."""
    cr = np.array(creases, dtype=np.float64)
    order = np.argsort(-cr[..., 3], axis=1, kind="stable")
    cr = np.take_along_axis(cr, order[..., None], axis=1)
    lams = np.asarray(lams, dtype=np.float64)
    R = 0.5 * D
    f = np.empty(cr.shape[:2] + (4,), dtype=np.float64)
    f[..., 0] = cr[..., 0] / math.pi * 2.0 - 1.0
    f[..., 1] = cr[..., 1] / R
    f[..., 2] = (cr[..., 2] - 1.25e-3) / 0.75e-3
    f[..., 3] = cr[..., 3] / (0.25 * lambda0) - 1.0
    lam = (2.0 * lams - (lam_lo + lam_hi)) / (lam_hi - lam_lo)
    return np.concatenate([f.reshape(len(cr), -1), lam[:, None]], axis=1).astype(np.float32)


def in_training_box(feats: np.ndarray, slack: float = 1e-6) -> np.ndarray:
    return np.all(np.abs(np.asarray(feats)) <= 1.0 + slack, axis=1)


def init_params(seed: int, n_in: int, hidden: int, n_out: int, out_bias: Optional[np.ndarray] = None) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights (PCG64 seeded), zero
    hidden biases, and the output bias set to `out_bias` (the mean target) when
    given, so training starts from the mean log-intensity map."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, fan_out in ((n_in, hidden), (hidden, hidden), (hidden, n_out)):
        a = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-a, a, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    if out_bias is not None:
        parts[-1] = np.asarray(out_bias, dtype=np.float64).reshape(n_out)
    return np.concatenate(parts).astype(np.float32)


class CZTSolver:
    """Batches of deformed instances through the split-BF16 propagation; returns
    log-intensity targets on the GPU."""

    def __init__(self, w: dict, chunk: int = 128, lanes: int = 2, path: str = "split", device="cuda",
                 floor: float = FLOOR):
        self.w = w
        self.floor = floor
        self.ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
        self.M = w["M"]
        self.chunk = chunk
        self.lanes = lanes
        self.path = path
        self.device = device
        self.i0 = i0_scale(w["D"], w["f0"], w["lambda0"])

    def solve(self, creases: np.ndarray, lams: np.ndarray, out=None):
        """Targets [n, M*M] (float32, device) for n instances; also the seconds spent."""
        import torch
        n = len(lams)
        MM = self.M * self.M
        if out is None:
            out = torch.empty((n, MM), dtype=torch.float32, device=self.device)
        t0 = time.perf_counter()
        for s in range(0, n, self.chunk):
            e = min(s + self.chunk, n)
            insts = [dict(lam=float(lams[k]), M=self.M, creases=creases[k]) for k in range(s, e)]
            plan = _lib.Plan(self.ap, insts, path=self.path, lanes=self.lanes)
            ws, roi = plan.alloc(self.device)
            plan.propagate(ws, roi)
            _lib.log_intensity(roi, (e - s) * MM, self.i0, self.floor, out[s:e])
            del plan, ws, roi
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0


class FWHMReader:
    """FWHM (x) of predicted intensities through the library's metric kernels."""

    def __init__(self, w: dict, batch: int, device="cuda", floor: float = FLOOR):
        ap = dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"])
        self.floor = floor
        self.M = w["M"]
        self.batch = batch
        self.i0 = i0_scale(w["D"], w["f0"], w["lambda0"])
        self.plan = _lib.Plan(ap, [dict(lam=w["lambda0"], M=self.M)] * batch, path="fp64")
        self.ws, self.roi = self.plan.alloc(device)

    def fwhm(self, y) -> np.ndarray:
        """y: [n, M*M] log-intensity (device) -> FWHM_x [n] in metres."""
        n = int(y.shape[0])
        out = np.empty(n)
        MM = self.M * self.M
        for s in range(0, n, self.batch):
            e = min(s + self.batch, n)
            _lib.field_from_log_intensity(y[s:e], (e - s) * MM, self.i0, self.floor, self.roi)
            ms = self.plan.metrics(self.ws, self.roi)
            out[s:e] = [m["fwhm_x"] for m in ms[: e - s]]
        return out


def cosine_lr(step: int, total: int, lr0: float) -> float:
    return 0.5 * lr0 * (1.0 + math.cos(math.pi * min(step, total) / max(total, 1)))


def train(mlp, x, t, epochs: int, batch: int, lr0: float, seed: int, log=None) -> list:
    """Adam with cosine decay over contiguous minibatches of (x, t), visited in a
    seeded random order each epoch.  Returns the per-epoch mean loss."""
    n = int(x.shape[0])
    nb = n // batch
    total = epochs * nb
    rng = np.random.Generator(np.random.PCG64(seed))
    losses = []
    step = 0
    for ep in range(epochs):
        order = rng.permutation(nb)
        acc = 0.0
        for b in order:
            s = int(b) * batch
            loss = mlp.train_step(x[s:s + batch], t[s:s + batch], cosine_lr(step, total, lr0))
            acc += float(loss.item())
            step += 1
        losses.append(acc / nb)
        if log is not None:
            log(f"epoch {ep + 1}/{epochs} loss {losses[-1]:.5f}")
    return losses


class Surrogate:
    """Two-member ensemble with a calibrated acceptance gate; the CZT decides the rest."""

    def __init__(self, w: dict, batch_max: int = 256, device="cuda", floor: float = FLOOR):
        self.w = w
        self.M = w["M"]
        self.members = [_lib.MLP(N_IN, HIDDEN, self.M * self.M, batch_max, device) for _ in range(2)]
        self.reader = FWHMReader(w, 64, device, floor)
        self.tau = 0.0025
        self.batch_max = batch_max
        self.device = device

    def init(self, seeds=(100, 101), t_sample=None):
        """Seeded initial weights; `t_sample` (targets, device) gives the output bias."""
        import torch
        bias = None
        if t_sample is not None:
            bias = t_sample.cpu().numpy().astype(np.float64).mean(axis=0)
        for m, sd in zip(self.members, seeds):
            m.set_params(torch.from_numpy(init_params(sd, N_IN, HIDDEN, self.M * self.M, bias)).to(self.device))

    def fit(self, x, t, epochs: int, batch: int = 256, lr0: float = 1e-3, seeds=(200, 201), log=None):
        return [train(m, x, t, epochs, batch, lr0, sd, log) for m, sd in zip(self.members, seeds)]

    def predict(self, x):
        """Both members' log-intensity predictions [n, M*M] (device)."""
        import torch
        n = int(x.shape[0])
        ys = []
        for m in self.members:
            y = torch.empty((n, self.M * self.M), dtype=torch.float32, device=x.device)
            for s in range(0, n, self.batch_max):
                e = min(s + self.batch_max, n)
                m.forward(x[s:e], out=y[s:e])
            ys.append(y)
        return ys

    def disagreement(self, x):
        """(first member's prediction, its FWHM, relative FWHM disagreement of the members)."""
        y1, y2 = self.predict(x)
        f1, f2 = self.reader.fwhm(y1), self.reader.fwhm(y2)
        return y1, f1, np.abs(f1 - f2) / (0.5 * (f1 + f2))

    def calibrate(self, x_val, fwhm_true: np.ndarray, feats_val: np.ndarray, target: float = 0.005,
                  tau_max: float = 0.0025) -> dict:
        """Largest threshold <= tau_max whose accepted validation cases all have
        FWHM error <= target."""
        _, fm, dis = self.disagreement(x_val)
        err = np.abs(fm / fwhm_true - 1.0)
        box = in_training_box(feats_val)
        best = 0.0
        for tau in np.sort(np.unique(np.concatenate([dis[box], [tau_max]]))):
            if tau > tau_max:
                break
            acc = box & (dis <= tau)
            if acc.any() and err[acc].max() <= target:
                best = float(tau)
        self.tau = best
        acc = box & (dis <= best)
        return dict(tau=best, accepted=float(acc.mean()), max_err_accepted=float(err[acc].max()) if acc.any() else 0.0)

    def accept(self, x, feats) -> tuple:
        ym, fm, dis = self.disagreement(x)
        return in_training_box(feats) & (dis <= self.tau), ym, fm, dis


def run(w: dict, n_train: int, n_val: int, n_test: int, epochs: int, log=None, floor: float = FLOOR,
        height_scale: float = 1.0, lr0: float = 1e-3) -> dict:
    """Data generation by CZT, training of both members, gate calibration on
    validation, and the accepted-case FWHM error, fallback rate and speed gain
    on the test set (seeds of the workload).  Returns a report dict."""
    import torch
    from fzp_inputs import surrogate_draws
    log = log or (lambda m: None)
    cr_a, lam_a = surrogate_draws(w["train_seed"], n_train + n_val, w["D"], w["lambda0"])
    cr_t, lam_t = surrogate_draws(w["test_seed"], n_test, w["D"], w["lambda0"])
    cr_a[..., 3] *= height_scale
    cr_t[..., 3] *= height_scale
    solver = CZTSolver(w, floor=floor)
    t_a, sec_a = solver.solve(cr_a, lam_a)
    log(f"CZT training data: {n_train + n_val} solves in {sec_a:.1f} s")
    t_t, sec_t = solver.solve(cr_t, lam_t)
    czt_per_case = (sec_a + sec_t) / (n_train + n_val + n_test)
    f_a = features(cr_a, lam_a, w["D"], height_scale * w["lambda0"])
    f_t = features(cr_t, lam_t, w["D"], height_scale * w["lambda0"])
    x_a, x_t = torch.from_numpy(f_a).cuda(), torch.from_numpy(f_t).cuda()
    S = Surrogate(w, floor=floor)
    S.init(t_sample=t_a[: min(2048, n_train)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = S.fit(x_a[:n_train], t_a[:n_train], epochs, lr0=lr0, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    fw_val = S.reader.fwhm(t_a[n_train:])
    cal = S.calibrate(x_a[n_train:], fw_val, f_a[n_train:])
    log(f"gate: {cal}")
    fw_t = S.reader.fwhm(t_t)
    acc, y, f_pred, dis = S.accept(x_t, f_t)
    err = np.abs(f_pred / fw_t - 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.predict(x_t)
    torch.cuda.synchronize()
    net_per_case = (time.perf_counter() - t0) / n_test
    frac = float(acc.mean())
    # expected cost per case with the fallback: network always, CZT when rejected
    mixed = net_per_case + (1.0 - frac) * czt_per_case
    fw_spread = float(np.std(fw_t) / np.mean(fw_t))
    return dict(n_train=n_train, n_val=n_val, n_test=n_test, epochs=epochs, train_s=round(train_s, 2),
                floor=floor, height_scale=height_scale, true_fwhm_rel_std=fw_spread,
                final_loss=[round(l[-1], 5) for l in losses], gate_tau=cal["tau"],
                accepted_fraction=round(frac, 4), fallback_rate=round(1.0 - frac, 4),
                fwhm_err_accepted_max=float(err[acc].max()) if acc.any() else None,
                fwhm_err_all_median=float(np.median(err)), fwhm_err_all_p90=float(np.percentile(err, 90)),
                czt_ms_per_case=round(czt_per_case * 1e3, 3), net_us_per_case=round(net_per_case * 1e6, 2),
                speedup_accepted=round(czt_per_case / net_per_case, 1),
                speedup_with_fallback=round(czt_per_case / mixed, 3))
