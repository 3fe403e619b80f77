"""Seeded synthetic inputs for the zone-plate propagation workloads.

This module is shared by the tests, the benchmark and the smoke check, and it
feeds both the GPU library and the CPU oracle. It holds parameters and seeded
random draws only: no grid, mask, chirp, transform or metric arithmetic lives
here.

Workloads (all synthetic, analytic binary-amplitude Fresnel zone plates under a
unit-amplitude, normally incident plane wave; the paper studies the same kind of
element in its accuracy study, Sec. 4.1, and its meter-class runs, Tables 1-5):

* ``fzp2mm``   D=2 mm,  f=10 mm (f/5), lambda0=632.8 nm, N=4096,  M=256,  stripe 64
* ``fzp20mm``  D=20 mm, f=100 mm,      lambda0=632.8 nm, N=32768, M=1024, stripe 256
* ``fzp1m``    D=1 m,   f=5 m,         lambda0=632.8 nm, N=2^20,  M=512,  stripe 128
* ``batch64``  64 instances of the D=20 mm element: 16 wavelengths (500-800 nm)
               x 4 crease maps, ROI sizes drawn from {256, 512, 1024}
* ``surrogate`` D=10 mm, f=50 mm, N=16384, M=128, 8 random creases + lambda
* ``ml100mm``  D=0.1 m, f=0.5 m (f/5), lambda0=632.8 nm, a 4-level phase plate,
               N=2^18 (0.38 um pitch, finer than the revised engine's grid rule
               Lambda_edge / (4 max(L, 2)) = 0.40 um), M=512, stripe 128

The crease model (a thin phase screen of straight Gaussian ridges) is a reading
of the membrane deformations that the introduction names as the motivation for
full 2-D simulation; the draws below are its only random inputs.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "WORKLOADS",
    "workload",
    "crease_draws",
    "batch_wavelengths",
    "batch_roi_sizes",
    "surrogate_draws",
    "batch64_instances",
]

LAMBDA0 = 632.8e-9

WORKLOADS = {
    "fzp2mm": dict(D=2e-3, f0=10e-3, lambda0=LAMBDA0, N=4096, M=256, stripe=64),
    "fzp20mm": dict(D=20e-3, f0=100e-3, lambda0=LAMBDA0, N=32768, M=1024, stripe=256),
    "fzp1m": dict(D=1.0, f0=5.0, lambda0=LAMBDA0, N=1 << 20, M=512, stripe=128),
    "batch64": dict(D=20e-3, f0=100e-3, lambda0=LAMBDA0, N=32768, M=None, stripe=256,
                    n_lambda=16, n_maps=4, map_seeds=(0, 1, 2, 3), m_seed=4,
                    m_choices=(256, 512, 1024), n_creases=8),
    "surrogate": dict(D=10e-3, f0=50e-3, lambda0=LAMBDA0, N=16384, M=128, stripe=128,
                      n_creases=8, lambda_lo=500e-9, lambda_hi=800e-9,
                      n_train=20000, n_test=1000, train_seed=10, test_seed=11),
    "ml100mm": dict(D=0.1, f0=0.5, lambda0=LAMBDA0, N=1 << 18, M=512, stripe=128, levels=4),
}


def workload(name: str) -> dict:
    """Return a copy of the named workload's parameters."""
    return dict(WORKLOADS[name])


def crease_draws(seed: int, D: float, lambda0: float, n: int = 8) -> np.ndarray:
    """Seeded crease parameters, one row per crease: (theta, offset, width, height).

    theta ~ U[0, pi) rad, offset ~ U[-R, R] m with R = D/2, width (ridge FWHM)
    ~ U[0.5, 2] mm, height (optical path difference) ~ U[0, lambda0/2] m.
    PCG64 stream seeded with ``seed``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    R = 0.5 * D
    theta = rng.uniform(0.0, np.pi, n)
    offset = rng.uniform(-R, R, n)
    width = rng.uniform(0.5e-3, 2.0e-3, n)
    height = rng.uniform(0.0, 0.5 * lambda0, n)
    return np.stack([theta, offset, width, height], axis=1)


def batch_wavelengths(n: int = 16, lo: float = 500e-9, hi: float = 800e-9) -> np.ndarray:
    """Evenly spaced wavelengths from ``lo`` to ``hi`` inclusive (metres)."""
    return np.linspace(lo, hi, n)


def batch_roi_sizes(seed: int, n: int, choices=(256, 512, 1024)) -> np.ndarray:
    """Seeded ROI side lengths, one per instance, drawn uniformly from ``choices``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asarray(choices, dtype=np.int64)[rng.integers(0, len(choices), n)]


def surrogate_draws(seed: int, n: int, D: float, lambda0: float, n_creases: int = 8,
                    lambda_lo: float = 500e-9, lambda_hi: float = 800e-9):
    """Seeded surrogate inputs: ``(creases[n, n_creases, 4], wavelengths[n])``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = 0.5 * D
    theta = rng.uniform(0.0, np.pi, (n, n_creases))
    offset = rng.uniform(-R, R, (n, n_creases))
    width = rng.uniform(0.5e-3, 2.0e-3, (n, n_creases))
    height = rng.uniform(0.0, 0.5 * lambda0, (n, n_creases))
    lam = rng.uniform(lambda_lo, lambda_hi, n)
    return np.stack([theta, offset, width, height], axis=2), lam


def batch64_instances(w: dict = None) -> list:
    """The 64 instances of the batch workload: instance k = 16 m + l takes crease
    map m (seeded ``map_seeds[m]``), wavelength l of ``batch_wavelengths`` and the
    k-th seeded ROI size; each sits at its first-order focus (z = 0)."""
    w = WORKLOADS["batch64"] if w is None else w
    lams = batch_wavelengths(w["n_lambda"])
    Ms = batch_roi_sizes(w["m_seed"], w["n_lambda"] * w["n_maps"], w["m_choices"])
    out = []
    for m in range(w["n_maps"]):
        cr = crease_draws(w["map_seeds"][m], w["D"], w["lambda0"], w["n_creases"])
        for li in range(w["n_lambda"]):
            k = m * w["n_lambda"] + li
            out.append(dict(lam=float(lams[li]), M=int(Ms[k]), creases=cr))
    return out
