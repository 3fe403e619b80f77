"""FP64 CPU oracle of the surrogate's physics prior: the focal-plane intensity
of a deformed binary zone plate's first diffraction order, modelled as a thin
lens with the plate's pupil.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this module; the GPU
library shares no code with it.

Physics (readings listed in the design notes).  The binary plate of Eq. 4
(open where floor(r^2 / (lambda0 f0)) is odd) is periodic in
s = r^2 / (lambda0 f0) with period 2; its Fourier series in s has
coefficients of modulus 1/(pi |m|) for odd m, so the order m = -1 is the
converging lens term exp(-i pi r^2 / (lambda0 f0)) with amplitude 1/pi (its
power is the first-order efficiency 1/pi^2).  At that order's focus
(lambda z = lambda0 f0) the Fresnel integral of Eq. 2 loses its input chirp
and becomes a Fourier transform of the pupil P times the membrane phase
screen exp(2 pi i h / lambda) (the thin-screen crease model of the
propagation oracle):

    I(x', y') = |(1/pi) / (lambda0 f0) int P e^{2 pi i h/lambda}
                 e^{-2 pi i (x x' + y y') / (lambda0 f0)} dx dy|^2,

reported relative to I0 = (R^2 / (lambda0 f0))^2, the undeformed peak.  The
zero order (amplitude 1/2) and the orders |m| >= 3 (defocused at this plane)
are left out: that is the prior's model error, which the network learns.

Discretisation (everything a plain formula):

* an Np x Np pupil grid over [-R, R]^2, pixel centres
  u_i = (2 i + 1 - Np) / (2 Np) D;
* the pupil value of a pixel is the fraction of its ss x ss sub-sample
  centres inside the disc, decided in exact integers: sub-sample centre
  c = 2 (i ss + s) + 1 - Np ss (units D / (2 Np ss)) is inside when
  c_x^2 + c_y^2 <= (Np ss)^2;
* the ROI of the propagation (M x M, spacing 16 lambda0 f0 / (D M), samples at
  (q - M/2) spacing) makes the transform kernel an exact rational number of
  turns, u_i x'_q / (lambda0 f0) = 4 (2 i + 1 - Np)(2 q - M) / (Np M);
* S = E g E^T with E[q][i] = exp(-2 pi i u_i x'_q / (lambda0 f0)) and
  g = P e^{2 pi i h / lambda}; then I / I0 = 16 |S|^2 / (pi^2 Np^4) (the pixel
  area (D/Np)^2 and the 1/pi amplitude), and the surrogate's target form
  ln(I / I0 + floor).
"""
from __future__ import annotations

import numpy as np

from . import fzp_oracle as F

__all__ = ["coverage", "pupil_coords", "dft_turns", "pupil_field", "prior_intensity", "prior_log_intensity"]


def coverage(Np: int, ss: int) -> np.ndarray:
    """Fraction of each pupil pixel's ss x ss sub-sample centres inside the disc
    (float64 [Np, Np]; exact multiples of 1/ss^2)."""
    n = Np * ss
    c = 2 * np.arange(n, dtype=np.int64) + 1 - n                  # sub-sample centres
    inside = (c[:, None] ** 2 + c[None, :] ** 2) <= n * n
    return inside.reshape(Np, ss, Np, ss).sum(axis=(1, 3)) / float(ss * ss)


def pupil_coords(D: float, Np: int) -> np.ndarray:
    """Pupil pixel centres u_i = (2 i + 1 - Np) / (2 Np) D [m]."""
    return (2.0 * np.arange(Np, dtype=np.float64) + 1.0 - Np) / (2.0 * Np) * D


def dft_turns(Np: int, M: int) -> np.ndarray:
    """u_i x'_q / (lambda0 f0) in turns, reduced exactly modulo 1: [M, Np]."""
    a = 2 * np.arange(Np, dtype=np.int64) + 1 - Np
    b = 2 * np.arange(M, dtype=np.int64) - M
    den = Np * M
    num = np.mod(4 * np.outer(b, a), den)                           # exact integers
    return num.astype(np.float64) / den


def pupil_field(D: float, Np: int, ss: int, creases, lam: float) -> np.ndarray:
    """g[j][i] = P(u_i, v_j) exp(2 pi i h(u_i, v_j) / lambda) (complex128 [Np, Np],
    rows j along y)."""
    u = pupil_coords(D, Np)
    h = F.crease_height(u[None, :], u[:, None], creases)
    return coverage(Np, ss) * np.exp(2j * np.pi * h / lam)


def prior_intensity(D: float, M: int, creases, lam: float, Np: int = 128, ss: int = 4) -> np.ndarray:
    """I / I0 on the M x M ROI [y = p][x = q] at the first-order focus."""
    E = np.exp(-2j * np.pi * dft_turns(Np, M))                     # [M, Np]
    S = E @ pupil_field(D, Np, ss, creases, lam) @ E.T
    return 16.0 * (S.real ** 2 + S.imag ** 2) / (np.pi ** 2 * float(Np) ** 4)


def prior_log_intensity(D: float, M: int, creases, lam: float, Np: int = 128, ss: int = 4,
                        floor: float = 1e-2) -> np.ndarray:
    """ln(I / I0 + floor), the surrogate's target form."""
    return np.log(prior_intensity(D, M, creases, lam, Np, ss) + floor)
