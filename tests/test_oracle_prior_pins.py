"""Pins of the surrogate's physics-prior oracle (``oracle.prior_oracle``) to
what the mathematics and the propagation fix, on the CPU:

* the pupil coverage: exact multiples of 1/ss^2, total area -> pi R^2;
* undeformed pupil: the Airy pattern (2 J1(v)/v)^2 of a clear disc
  (scipy's Bessel function; the prior's own DFT never sees it);
* Parseval in the DFT window (M = Np = 16 makes the ROI exactly one period of
  the pupil grid's DFT): sum I / I0 = 16 sum P^2 / (pi^2 Np^2) for any phase;
* a uniform phase screen leaves the intensity unchanged;
* a pupil symmetric in x gives an intensity symmetric in x' (the pixel
  centres and ROI samples are placed symmetrically);
* the full zone-plate propagation (the CZT oracle of Eq. 2 on the Eq. 4
  plate with the same creases) agrees within 2 % of the peak on a 158-zone
  plate at two wavelengths: the first-order lens model leaves out only the
  zero order and the defocused orders.
"""
import numpy as np
import pytest
from scipy.special import j1

from oracle import fzp_oracle as F
from oracle import prior_oracle as PR

LAM0 = 632.8e-9


def _creases(seed, n, D, wmin, wmax):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.stack([rng.uniform(0, np.pi, n), rng.uniform(-D / 2, D / 2, n), rng.uniform(wmin, wmax, n),
                     rng.uniform(0, 0.5 * LAM0, n)], axis=1)


def test_coverage_exact_and_area():
    for Np, ss in ((16, 1), (64, 16), (100, 3)):
        a = PR.coverage(Np, ss)
        k = a * ss * ss
        assert np.array_equal(k, np.rint(k)) and a.min() >= 0.0 and a.max() <= 1.0
        assert np.array_equal(a, a[::-1, :]) and np.array_equal(a, a.T)
    a = PR.coverage(64, 16)                     # 1024 sub-samples per side
    area = a.sum() * (1.0 / 64) ** 2            # unit-diameter pupil
    assert abs(area / (np.pi / 4) - 1.0) < 1e-3


def test_airy_undeformed():
    M = 128
    I = PR.prior_intensity(10e-3, M, None, LAM0, Np=128, ss=4)
    k = np.arange(M) - M / 2
    rho = np.hypot(k[None, :], k[:, None])
    v = 16.0 * np.pi * rho / M                  # pi D r / (lambda0 f0), r = rho 16 lambda0 f0 / (D M)
    with np.errstate(invalid="ignore", divide="ignore"):
        A = np.where(v == 0, 1.0, (2.0 * j1(v) / v) ** 2)
    assert np.abs(I - A).max() < 2e-4
    assert abs(I[M // 2, M // 2] - 1.0) < 2e-4


def test_parseval_in_dft_window():
    Np = M = 16
    D = 10e-3
    for seed in (1, 2):
        cr = _creases(seed, 8, D, 0.5e-3, 2e-3)
        I = PR.prior_intensity(D, M, cr, 600e-9, Np=Np, ss=4)
        P = PR.coverage(Np, 4)
        assert abs(I.sum() / (16.0 * np.sum(P * P) / (np.pi ** 2 * Np ** 2)) - 1.0) < 1e-12


def test_uniform_phase_is_invisible():
    D = 10e-3
    flat = np.array([[0.3, 0.0, 1e6, 0.37 * LAM0]])      # a ridge far wider than the pupil
    I0 = PR.prior_intensity(D, 64, None, LAM0, Np=64, ss=2)
    I1 = PR.prior_intensity(D, 64, flat, LAM0, Np=64, ss=2)
    assert np.abs(I1 - I0).max() < 1e-9


def test_mirror_symmetry():
    D, M = 10e-3, 64
    cr = np.array([[0.0, 0.0, 1.2e-3, 0.4 * LAM0], [np.pi / 2, 1.5e-3, 0.8e-3, 0.3 * LAM0]])  # even in x
    I = PR.prior_intensity(D, M, cr, 650e-9, Np=96, ss=4)
    assert np.abs(I[:, 1:] - I[:, :0:-1]).max() < 1e-12 * I.max()
    assert np.abs(I[1:, :] - I[:0:-1, :]).max() > 1e-3 * I.max()     # the second ridge is not even in y


@pytest.mark.parametrize("lam", [LAM0, 560e-9])
def test_matches_zone_plate_czt(lam):
    D, f0, N, M = 2e-3, 10e-3, 2048, 32
    cr = _creases(7, 6, D, 0.1e-3, 0.4e-3)
    ap = F.Aperture(D=D, f0=f0, lambda0=LAM0, N=N)
    U = F.propagate(ap, F.Instance(lam=lam, M=M, creases=cr), method="bluestein")
    It = F.intensity(U) / (0.25 * D * D / (LAM0 * f0)) ** 2
    Ip = PR.prior_intensity(D, M, cr, lam, Np=128, ss=4)
    assert np.abs(Ip - It).max() < 0.02 * It.max()
