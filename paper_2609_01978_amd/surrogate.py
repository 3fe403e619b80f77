"""Learned surrogate of the deformed zone plate's focal spot.

A 33 -> 512 -> 512 -> M^2 perceptron (the library's ``fzp_mlp_*`` kernels)
maps 8 straight creases (angle, offset, width, height) and the wavelength to
the log-intensity ``ln(I / I0 + FLOOR)`` of the M x M focal-plane ROI, with
``I0 = (R^2 / (lambda0 f0))^2`` the peak scale of the undeformed plate (its
on-axis intensity is close to the square of twice the number of open zones).
It is trained on the split-BF16 CZT propagation of the same plate; the CZT is
also its arbiter and its fallback: a 2-member ensemble is trained from two
seeds, and a prediction is accepted only when the input lies inside the
training box and the members' FWHMs agree within a threshold calibrated
on held-out validation solves so that accepted validation cases keep the FWHM
error within the target.

With the physics prior (``prior=True``, ``fzp_pupil_prior``: the plate's first
diffraction order as a thin lens with the deformed pupil, a 128^2 pupil grid)
the network learns the residual ``t - prior`` in the same log-intensity form
and a prediction is ``prior + network``; the gate then also compares each
member's FWHM with the prior's own.  Everything numeric runs in the library's
kernels (propagation, prior, targets, network, FWHM); this module orchestrates
them.
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


def _noll_nm(j: int):
    """(n, m) of Zernike polynomial j in Noll's ordering (j >= 1)."""
    n = 0
    while (n + 1) * (n + 2) // 2 < j:
        n += 1
    k = j - n * (n + 1) // 2 - 1          # 0 .. n within radial order n
    # |m| rises through the order: 0, 2, 2, 4, 4, .. (n even) or 1, 1, 3, 3, .. (n odd);
    # even j takes the cosine (m > 0), odd j the sine (m < 0)
    mabs = 2 * ((k + 1) // 2) if n % 2 == 0 else 2 * (k // 2) + 1
    return n, (0 if mabs == 0 else (mabs if j % 2 == 0 else -mabs))


def zernike(j: int, r: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Orthonormal Zernike polynomial Z_j (Noll), (1/pi) int Z_i Z_j dA = delta_ij
    over the unit disc."""
    n, m = _noll_nm(j)
    mabs = abs(m)
    R = np.zeros_like(r)
    for k in range((n - mabs) // 2 + 1):
        R += ((-1) ** k * math.factorial(n - k) /
              (math.factorial(k) * math.factorial((n + mabs) // 2 - k) * math.factorial((n - mabs) // 2 - k))
              ) * r ** (n - 2 * k)
    if m == 0:
        return math.sqrt(n + 1) * R
    return math.sqrt(2 * (n + 1)) * R * (np.cos(mabs * t) if m > 0 else np.sin(mabs * t))


class ZernikeEncoder:
    """Physics-derived inputs: the coefficients a_2 .. a_{n+1} of the pupil
    phase phi = 2 pi h / lambda of the creases (the thin-screen model of the
    propagation) in orthonormal Zernike polynomials over the aperture disc,
    a_j = (1/pi) int phi Z_j dA (Gauss-Legendre in r^2, uniform in angle),
    then the wavelength.  The focal field depends on lambda only through phi
    (lambda z is fixed), and the coefficients are the same for any order of
    the creases.  Each input is scaled to [-1, 1] over the range seen in
    training (``fit``)."""

    def __init__(self, D: float, n_terms: int = 32, n_r: int = 24, n_t: int = 64):
        self.R = 0.5 * D
        self.n_terms = n_terms
        x, w = np.polynomial.legendre.leggauss(n_r)
        s = 0.5 * (x + 1.0)                          # r^2 on [0, 1]
        r = np.sqrt(s)
        t = 2.0 * np.pi * (np.arange(n_t) + 0.5) / n_t
        self.r = np.repeat(r, n_t)
        self.t = np.tile(t, n_r)
        # dA = (1/2) d(r^2) dtheta: weights of (1/pi) int over the unit disc
        self.w = np.repeat(0.5 * w * 0.5, n_t) * (2.0 * np.pi / n_t) / np.pi
        self.Z = np.stack([zernike(j, self.r, self.t) for j in range(2, n_terms + 2)])   # [n_terms, nodes]
        self.lo = None
        self.hi = None

    def coefficients(self, creases: np.ndarray, lams: np.ndarray) -> np.ndarray:
        cr = np.asarray(creases, dtype=np.float64)
        X = (self.R * self.r * np.cos(self.t))[None, None, :]
        Y = (self.R * self.r * np.sin(self.t))[None, None, :]
        th, rho, wid, H = (cr[..., k][..., None] for k in range(4))
        sig = wid / (2.0 * math.sqrt(2.0 * math.log(2.0)))
        d = X * np.cos(th) + Y * np.sin(th) - rho
        h = np.sum(H * np.exp(-d * d / (2.0 * sig * sig)), axis=1)          # [n, nodes]
        phi = 2.0 * np.pi * h / np.asarray(lams, dtype=np.float64)[:, None]
        return (phi * self.w[None, :]) @ self.Z.T                          # [n, n_terms]

    def fit(self, creases: np.ndarray, lams: np.ndarray, lam_lo: float = 500e-9, lam_hi: float = 800e-9):
        a = self.coefficients(creases, lams)
        self.lo, self.hi = a.min(axis=0), a.max(axis=0)
        self.lam_lo, self.lam_hi = lam_lo, lam_hi
        return self

    def __call__(self, creases: np.ndarray, lams: np.ndarray) -> np.ndarray:
        a = self.coefficients(creases, lams)
        f = (2.0 * a - (self.lo + self.hi)) / np.maximum(self.hi - self.lo, 1e-30)
        lam = (2.0 * np.asarray(lams, dtype=np.float64) - (self.lam_lo + self.lam_hi)) / (self.lam_hi - self.lam_lo)
        return np.concatenate([f, lam[:, None]], axis=1).astype(np.float32)


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
    """FWHM (x) of log-intensity maps and the conditioning of that reading, by
    the library's batched FWHM kernel (fzp_fwhm_batch: the metric extractor's
    spline along the row of the brightest sample)."""

    def __init__(self, w: dict, batch: int = 0, device="cuda", floor: float = FLOOR, level_delta: float = 0.05,
                 exclusion_radius: float = 0.0):
        self.floor = floor
        self.M = w["M"]
        # ROI pitch of a default instance at its focus: 16 lambda0 f0 / (D M)
        self.dxo = 16.0 * w["lambda0"] * w["f0"] / (w["D"] * self.M)
        self.delta = level_delta
        # twice the first Airy null radius, 1.22 lambda0 f0 / D, in ROI samples
        self.excl = exclusion_radius or 2.0 * 1.22 * self.M / 16.0
        # a neighbouring row within 1 % of the peak could hold the brightest
        # sample of the true map (the prediction's intensity error is ~0.3 %)
        self.row_gap = 0.01

    def read(self, y):
        """y: [n, M*M] log-intensity (device) -> (FWHM_x [n] in metres, cond [n],
        ratio [n], row [n]): `row` the relative FWHM change if the brightest
        sample moved to the brighter neighbouring row, 0 when that row is
        at least `row_gap` dimmer than the peak."""
        o = _lib.fwhm_batch(y, self.M, self.floor, self.delta, self.excl).cpu().numpy()
        with np.errstate(invalid="ignore"):
            alt = np.abs(o[:, 4] / o[:, 0] - 1.0)
        row = np.where(o[:, 3] >= self.row_gap, 0.0, np.where(np.isfinite(alt), alt, np.inf))
        return o[:, 0] * self.dxo, o[:, 1], o[:, 2], row

    def fwhm(self, y) -> np.ndarray:
        return self.read(y)[0]


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
        self.reader = FWHMReader(w, 0, device, floor)
        self.tau = 0.0025
        # conditioning limits of the FWHM reading (see fzp_fwhm_batch): a width
        # that moves more than cond_max per unit change of the level, a second
        # spot above ratio_max of the peak (at one half it would cross the FWHM
        # level), or a neighbouring row that could take the peak and reads a
        # width more than row_max away, is not trusted
        self.cond_max = 3.0
        self.ratio_max = 0.45
        self.row_max = 0.0025
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

    def predict(self, x, base=None):
        """Both members' log-intensity predictions [n, M*M] (device); with `base`
        (the prior, same shape) each prediction is base + network."""
        import torch
        n = int(x.shape[0])
        ys = []
        for m in self.members:
            y = torch.empty((n, self.M * self.M), dtype=torch.float32, device=x.device)
            for s in range(0, n, self.batch_max):
                e = min(s + self.batch_max, n)
                m.forward(x[s:e], out=y[s:e])
            if base is not None:
                y += base
            ys.append(y)
        return ys

    def disagreement(self, x, base=None):
        """(first member's prediction, its FWHM, relative FWHM disagreement,
        conditioning): the members' FWHMs, and with `base` also the prior's, at
        most `dis` apart relative to their mean; `cond` and `ratio` the largest
        over those maps."""
        y1, y2 = self.predict(x, base)
        reads = [self.reader.read(y1), self.reader.read(y2)]
        if base is not None:
            reads.append(self.reader.read(base))
        f = np.stack([r[0] for r in reads])
        with np.errstate(invalid="ignore"):
            dis = (f.max(axis=0) - f.min(axis=0)) / f.mean(axis=0)
        cond = np.max(np.stack([r[1] for r in reads]), axis=0)
        ratio = np.max(np.stack([r[2] for r in reads]), axis=0)
        row = np.max(np.stack([r[3] for r in reads]), axis=0)
        return y1, reads[0][0], np.where(np.isfinite(dis), dis, np.inf), (cond, ratio, row)

    def _trusted(self, c):
        cond, ratio, row = c
        return (cond <= self.cond_max) & (ratio <= self.ratio_max) & (row <= self.row_max)

    def calibrate(self, x_val, fwhm_true: np.ndarray, feats_val: np.ndarray, target: float = 0.005,
                  tau_max: float = 0.0025, base=None) -> dict:
        """Largest threshold <= tau_max whose accepted validation cases all have
        FWHM error <= target."""
        _, fm, dis, c = self.disagreement(x_val, base)
        err = np.abs(fm / fwhm_true - 1.0)
        box = in_training_box(feats_val) & self._trusted(c)
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

    def accept(self, x, feats, base=None) -> tuple:
        ym, fm, dis, c = self.disagreement(x, base)
        return in_training_box(feats) & self._trusted(c) & (dis <= self.tau), ym, fm, dis


def run(w: dict, n_train: int, n_val: int, n_test: int, epochs: int, log=None, floor: float = FLOOR,
        height_scale: float = 1.0, lr0: float = 1e-3, encoding: str = "raw", prior: bool = True) -> dict:
    """Data generation by CZT, training of both members, gate calibration on
    validation, and the accepted-case FWHM error, fallback rate and speed gain
    on the test set (seeds of the workload).  The inference cost per case
    counts everything an accepted case needs: the prior (with ``prior``), both
    members' forward passes and the gate's FWHM readings.  Returns a report
    dict."""
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
    if encoding == "zernike":
        enc = ZernikeEncoder(w["D"]).fit(cr_a[:n_train], lam_a[:n_train])
        f_a, f_t = enc(cr_a, lam_a), enc(cr_t, lam_t)
    else:
        f_a = features(cr_a, lam_a, w["D"], height_scale * w["lambda0"])
        f_t = features(cr_t, lam_t, w["D"], height_scale * w["lambda0"])
    x_a, x_t = torch.from_numpy(f_a).cuda(), torch.from_numpy(f_t).cuda()
    base_a = base_t = None
    if prior:
        pr = _lib.PupilPrior(w["D"], w["M"], cr_a.shape[1], floor=floor)
        base_a, base_t = pr(cr_a, lam_a), pr(cr_t, lam_t)
    r_a = t_a - base_a if prior else t_a                  # the network's targets
    S = Surrogate(w, floor=floor)
    S.init(t_sample=r_a[: min(2048, n_train)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = S.fit(x_a[:n_train], r_a[:n_train], epochs, lr0=lr0, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    b_val = base_a[n_train:] if prior else None
    fw_val = S.reader.fwhm(t_a[n_train:])
    cal = S.calibrate(x_a[n_train:], fw_val, f_a[n_train:], base=b_val)
    log(f"gate: {cal}")
    fw_t = S.reader.fwhm(t_t)
    acc, y, f_pred, dis = S.accept(x_t, f_t, base_t)
    err = np.abs(f_pred / fw_t - 1.0)
    # inference cost of the test set, end to end as an accepted case needs it
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = pr(cr_t, lam_t) if prior else None
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.predict(x_t, b)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    S.disagreement(x_t, b)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prior_per_case = (t1 - t0) / n_test
    net_per_case = (t2 - t1) / n_test
    gate_per_case = max(t3 - t2 - (t2 - t1), 0.0) / n_test      # FWHM readings (disagreement repeats predict)
    infer_per_case = prior_per_case + net_per_case + gate_per_case
    frac = float(acc.mean())
    # expected cost per case with the fallback: inference always, CZT when rejected
    mixed = infer_per_case + (1.0 - frac) * czt_per_case
    fw_spread = float(np.std(fw_t) / np.mean(fw_t))
    rep = dict(encoding=encoding, prior=prior, n_train=n_train, n_val=n_val, n_test=n_test, epochs=epochs,
               train_s=round(train_s, 2),
               floor=floor, height_scale=height_scale, true_fwhm_rel_std=fw_spread,
               final_loss=[round(l[-1], 5) for l in losses], gate_tau=cal["tau"],
               accepted_fraction=round(frac, 4), fallback_rate=round(1.0 - frac, 4),
               fwhm_err_accepted_max=float(err[acc].max()) if acc.any() else None,
               fwhm_err_all_median=float(np.median(err)), fwhm_err_all_p90=float(np.percentile(err, 90)),
               czt_ms_per_case=round(czt_per_case * 1e3, 3), net_us_per_case=round(net_per_case * 1e6, 2),
               prior_us_per_case=round(prior_per_case * 1e6, 2), gate_us_per_case=round(gate_per_case * 1e6, 2),
               infer_us_per_case=round(infer_per_case * 1e6, 2),
               speedup_accepted=round(czt_per_case / infer_per_case, 1),
               speedup_with_fallback=round(czt_per_case / mixed, 3))
    # what the network adds to the prior: FWHM and ROI intensity errors of the
    # prior alone against those of prior + network (first member)
    ti = torch.exp(t_t) - floor
    rel = lambda yp: ((torch.exp(yp) - floor - ti).norm(dim=1) / ti.norm(dim=1)).cpu().numpy()
    rep["roi_rel_l2_median"] = float(np.median(rel(y)))
    if prior:
        e0 = np.abs(S.reader.fwhm(base_t) / fw_t - 1.0)
        rep.update(prior_fwhm_err_median=float(np.median(e0)), prior_fwhm_err_p90=float(np.percentile(e0, 90)),
                   prior_frac_within_target=float(np.mean(e0 <= 0.005)),
                   prior_roi_rel_l2_median=float(np.median(rel(base_t))))
    return rep
