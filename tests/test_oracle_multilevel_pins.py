"""Pins of the oracle's L-level phase plates (the revised engine's element,
Fig. 18 stage 3; Tables 1-5 use L = 16, 8, 4, 4, 2).

Each test ties the multilevel part of the oracle to something other than
itself: exact rational arithmetic per sample, the binary amplitude plates
(L = 2 is their difference), the direct Eq. 1 sum, and the scalar-diffraction
efficiency of an L-step kinoform, sinc^2(1/L), in its first order.  CPU only.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import fzp_oracle as O

LAM0 = 632.8e-9


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sinc2(L):
    """First-order efficiency of an L-step quantised lens phase: (sin(pi/L)/(pi/L))^2."""
    x = math.pi / L
    return (math.sin(x) / x) ** 2


@pytest.mark.parametrize("L,N", [(2, 64), (4, 63), (8, 50), (16, 47), (3, 41)])
def test_phase_level_exact_rationals(L, N):
    """Per sample, in exact rationals: s = r^2/(lambda0 f0), level = floor(L frac(s/2))."""
    ap = O.Aperture(D=2e-3, f0=3e-3, lambda0=LAM0, N=N, levels=L)
    got = O.phase_level(ap)
    dx = Fraction(ap.dx)
    a = Fraction(ap.lambda0) * Fraction(ap.f0)
    for j in range(N):
        for i in range(N):
            K = (2 * i - N + 1) ** 2 + (2 * j - N + 1) ** 2
            half = Fraction(K) * dx * dx / 4 / a / 2
            want = math.floor(L * (half - math.floor(half)))
            assert got[j, i] == want, (j, i)


def test_transmission_is_unit_modulus_on_the_disc():
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=200, levels=8)
    t = O.aperture_field(ap, O.Instance(lam=LAM0, M=8))
    disc = O.disc_mask(ap)
    assert np.allclose(np.abs(t[disc]), 1.0, rtol=0, atol=1e-15)
    assert np.all(t[~disc] == 0)
    assert np.count_nonzero(disc) == O.incident_count(ap)
    # the centre sample sits in level 0 (phase 0); levels advance outwards
    assert O.phase_level(ap)[100, 100] == 0


def test_two_levels_is_open_minus_closed_amplitude_plate():
    """L = 2 transmits +1 on even zones and -1 on odd zones: the centre-open
    amplitude plate minus the centre-opaque one, field for field."""
    kw = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=300)
    inst = O.Instance(lam=700e-9, M=24)
    U2 = O.propagate(O.Aperture(levels=2, **kw), inst, stripe=64)
    Uo = O.propagate(O.Aperture(centre_open=1, **kw), inst, stripe=64)
    Uc = O.propagate(O.Aperture(centre_open=0, **kw), inst, stripe=64)
    assert rel_l2(U2, Uo - Uc) < 1e-12


@pytest.mark.parametrize("L", [3, 4])
def test_separable_matches_direct_eq1(L):
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=90, levels=L)
    inst = O.Instance(lam=600e-9, M=10, x0=2e-6)
    ref = O.fresnel_direct(ap, inst)
    assert rel_l2(O.propagate(ap, inst, stripe=37), ref) < 1e-12
    assert rel_l2(O.propagate(ap, inst, method="dft"), ref) < 1e-12


@pytest.mark.parametrize("L", [2, 4, 8, 16])
def test_efficiency_ladder_at_many_zones(L):
    """1580 zones: main-lobe DE -> sinc^2(1/L) * 0.837785 (the Airy lobe share of
    the first order), on-axis intensity -> sinc^2(1/L) (pi R^2/(lambda z))^2, FWHM
    -> the Airy value; the radial integral and its on-axis closed form."""
    ap = O.Aperture(D=0.02, f0=0.1, lambda0=LAM0, N=2, levels=L)
    h = O.hankel_metrics(ap)
    lz = LAM0 * ap.f0
    assert abs(h["de"] / (sinc2(L) * O.AIRY_LOBE_FRACTION) - 1) < 2e-4
    axis = O.on_axis_closed_form(ap) / (math.pi * (0.5 * ap.D) ** 2 / lz) ** 2
    assert abs(axis / sinc2(L) - 1) < 3e-4
    assert abs(h["i0"] / (O.on_axis_closed_form(ap)) - 1) < 1e-9
    assert abs(h["fwhm"] / (O.AIRY_FWHM * lz / ap.D) - 1) < 1e-4


@pytest.mark.parametrize("L", [2, 4, 8])
def test_strehl_tends_to_sinc2(L):
    """An L-step kinoform keeps sinc^2(1/L) of an ideal lens's focal peak
    (pi R^2/(lambda z))^2 at many zones: the Strehl of the radial integral."""
    ap = O.Aperture(D=0.02, f0=0.1, lambda0=LAM0, N=2, levels=L)
    assert abs(O.hankel_metrics(ap)["strehl"] / sinc2(L) - 1) < 2e-4


@pytest.mark.parametrize("L,N", [(4, 4096), (2, 2048)])
def test_grid_matches_hankel(L, N):
    """The 2-D sampled plate against the continuous radial integral."""
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=N, levels=L)
    inst = O.Instance(lam=LAM0, M=256)
    U = O.propagate(ap, inst, stripe=512)
    m = O.metrics(U, ap, inst)
    h = O.hankel_metrics(ap)
    assert abs(m["fwhm_x"] / h["fwhm"] - 1) < 1e-4
    assert abs(m["de"] / h["de"] - 1) < 2e-4
    assert abs(O.intensity(U)[128, 128] / h["i0"] - 1) < 2e-4


def test_small_grid_on_axis_matches_hankel():
    """Fast check of the sampled L = 4 plate: the focal-point intensity of a
    1024^2 grid against the radial integral (0.05 % apart at 1.6 samples per
    outer zone)."""
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=1024, levels=4)
    inst = O.Instance(lam=LAM0, M=32)
    I = O.intensity(O.propagate(ap, inst, stripe=256))
    h = O.hankel_metrics(ap)
    assert abs(I[16, 16] / h["i0"] - 1) < 2e-3
