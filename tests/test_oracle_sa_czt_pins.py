"""Pins of the non-paraxial (SA-CZT) oracle against what the paper and the
mathematics fix independently of it:

* the zone index of Eq. 3 in exact rational arithmetic;
* the on-axis Rayleigh-Sommerfeld field of clear annuli in closed form (itself
  checked by quadrature of the Rayleigh-Sommerfeld kernel), which a zone plate
  with Eq. 3 radii focuses in phase: the propagated field at its focus, at
  f/2 where the paraxial zone plate loses 90 % of its peak;
* the paraxial limit: at f/200 the exact propagation equals the Fresnel
  (paraxial) oracle's field;
* unitarity of the angular-spectrum step and Parseval's identity of the zoom
  in the DFT window;
* the split of k_z into the fitted quadratic and the remainder is immaterial:
  two fit points give the same field.

CPU only; the GPU path is not involved.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate

from oracle import fzp_oracle as F
from oracle import sa_czt_oracle as S

LAM0 = 632.8e-9


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def eq3_open_annuli(D, f, lam, centre_open=0):
    """Open annuli of the Eq. 3 plate (odd zones), radii r_n^2 = n lam f + (n lam/2)^2,
    clipped at D/2."""
    R = 0.5 * D
    nmax = int(math.floor(2.0 * (math.sqrt(f * f + R * R) - f) / lam)) + 1
    r = [min(math.sqrt(n * lam * f + (n * lam / 2.0) ** 2), R) for n in range(nmax + 1)]
    return [(r[n], r[n + 1]) for n in range(nmax) if (n % 2 == 1) != bool(centre_open) and r[n] < r[n + 1]]


@pytest.mark.parametrize("N,D,f", [(64, 1e-3, 2e-3), (65, 2e-3, 5e-3)])
def test_eq3_zone_index_in_exact_rationals(N, D, f):
    """floor(n_exact) is the largest n with n lam f + n^2 lam^2 / 4 <= r^2, r^2 =
    K dx^2 / 4, decided in exact rationals of the float64 inputs."""
    ap = F.Aperture(D=D, f0=f, lambda0=LAM0, N=N)
    got = S.zone_index_eq3(ap)
    lam, ff, dx = Fraction(ap.lambda0), Fraction(ap.f0), Fraction(ap.dx)
    ci = [2 * i - (N - 1) for i in range(N)]
    seen_sag = False
    for j in range(N):
        for i in range(N):
            r2 = Fraction(ci[i] * ci[i] + ci[j] * ci[j]) * dx * dx / 4
            n = int(r2 / (lam * ff))                      # paraxial index: an upper bound
            while n > 0 and n * lam * ff + n * n * lam * lam / 4 > r2:
                n -= 1
            assert got[j, i] == n, (j, i, got[j, i], n)
            seen_sag = seen_sag or n != int(r2 / (lam * ff))
    assert seen_sag                                      # the sag term moves some samples


def test_rs_closed_form_against_quadrature():
    """The on-axis Rayleigh-Sommerfeld field of an annulus [a, b],
    int_a^b (z/rho)(1/rho - i k)(e^{i k rho}/rho) r dr, by adaptive quadrature."""
    lam, z = 50e-6, 1e-3                                  # few oscillations for the quadrature
    k = 2 * math.pi / lam
    for a, b in ((0.0, 0.4e-3), (0.3e-3, 0.9e-3)):
        def f(r, part):
            rho = math.hypot(z, r)
            v = (z / rho) * complex(1.0 / rho, -k) * complex(math.cos(k * rho), math.sin(k * rho)) / rho * r
            return v.real if part == 0 else v.imag
        re = integrate.quad(f, a, b, args=(0,), epsabs=1e-12, epsrel=1e-10, limit=1000)[0]
        im = integrate.quad(f, a, b, args=(1,), epsabs=1e-12, epsrel=1e-10, limit=1000)[0]
        cf = S.rs_on_axis_annuli([(a, b)], lam, z)
        assert abs(complex(re, im) - cf) < 1e-9 * max(1.0, abs(cf))


def test_eq3_plate_focuses_in_phase_at_f2():
    """f/2 (NA 0.24, 198 zones): the propagated on-axis field equals the closed
    form sum over open annuli, amplitude and phase; with the same radii under
    this propagation every open zone adds in phase, while the paraxial radii
    of Eq. 4 keep about a tenth of the peak intensity."""
    D, f = 1e-3, 2e-3
    ap = F.Aperture(D=D, f0=f, lambda0=LAM0, N=2048)
    inst = F.Instance(lam=LAM0, M=16)
    U = S.sa_czt(ap, inst, radii="eq3")
    ref = S.rs_on_axis_annuli(eq3_open_annuli(D, f, LAM0), LAM0, f)
    assert abs(U[8, 8] - ref) / abs(ref) < 3e-4
    # in phase: |ref| = sum over open zones of the obliquity factors f/rho at both edges
    amp = sum(f / math.hypot(f, a) + f / math.hypot(f, b) for a, b in eq3_open_annuli(D, f, LAM0))
    assert abs(abs(ref) / amp - 1) < 2e-3
    Up = S.sa_czt(ap, inst, radii="paraxial")
    assert abs(Up[8, 8]) ** 2 < 0.2 * abs(ref) ** 2


def test_paraxial_limit_matches_fresnel_oracle():
    """f/200: the exact propagation of the paraxial plate equals the Fresnel
    oracle's complex field (Eq. 2) up to the non-paraxial and wrap-around
    residue (pad 3)."""
    ap = F.Aperture(D=1e-3, f0=0.2, lambda0=LAM0, N=512)
    inst = F.Instance(lam=LAM0, M=64)
    Uf = F.propagate(ap, inst, stripe=512)
    Us = S.sa_czt(ap, inst, radii="paraxial", pad=3.0)
    assert rel_l2(Us, Uf) < 1e-3
    assert rel_l2(F.intensity(Us), F.intensity(Uf)) < 5e-4


def test_angular_spectrum_step_is_unitary():
    """No evanescent frequency on the grid (dx > lambda/2): |H| = 1, so the step
    keeps the energy; with dx < lambda/2 the evanescent part is removed."""
    rng = np.random.Generator(np.random.PCG64(3))
    U0 = rng.standard_normal((96, 96)) + 1j * rng.standard_normal((96, 96))
    U1 = S.angular_spectrum_step(U0, 2e-6, LAM0, 5e-3)
    assert abs(np.sum(np.abs(U1) ** 2) / np.sum(np.abs(U0) ** 2) - 1) < 1e-12
    U1e = S.angular_spectrum_step(U0, 0.2e-6, LAM0, 5e-3)
    assert np.isfinite(U1e).all()
    assert np.sum(np.abs(U1e) ** 2) < 0.95 * np.sum(np.abs(U0) ** 2)


def test_zoom_parseval_in_dft_window():
    """With M = Np and dx_out = Z/(Np dx) the zoom is a DFT: sum |U|^2 dx_out^2 with
    |U| = |zoom| / Z equals sum |U1|^2 dx^2."""
    rng = np.random.Generator(np.random.PCG64(4))
    Np, dx, Z = 64, 1.3e-6, 2.7e-9
    U1 = rng.standard_normal((Np, Np)) + 1j * rng.standard_normal((Np, Np))
    dxo = Z / (Np * dx)
    xq = F.roi_coords(Np, 0.0, dxo)
    acc = S.zoom(U1, dx, Z, xq, xq)
    assert abs(np.sum(np.abs(acc / Z) ** 2) * dxo * dxo / (np.sum(np.abs(U1) ** 2) * dx * dx) - 1) < 1e-10


def test_fit_split_is_immaterial():
    """The remainder h and the analytic chirp Z come from the same fit, so the
    fit point does not change the field (pad 3)."""
    ap = F.Aperture(D=1e-3, f0=20e-3, lambda0=LAM0, N=512)
    inst = F.Instance(lam=LAM0, M=32)
    a = S.sa_czt(ap, inst, pad=3.0, k_fit=2.0 / 3.0)
    b = S.sa_czt(ap, inst, pad=3.0, k_fit=0.5)
    assert rel_l2(a, b) < 1e-3


def test_pad_size_rule():
    for N in (1, 2, 100, 511, 1024, 4096, 28672, 1 << 15):
        m = S.pad_size(N)
        assert m >= 1.5 * N and (m - N) % 2 == 0
        k = m
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        assert k == 1
        # smallest such size
        assert all(not (c >= 1.5 * N and (c - N) % 2 == 0 and S._smooth(c)) for c in range(int(math.ceil(1.5 * N)), m))
    assert S.pad_size(4096) == 6144 and S.pad_size(28672) == 43200


def test_zero_height_creases_and_constant_screen():
    """The crease screen: zero heights leave the field bit for bit; a crease
    whose profile is constant over the aperture (a very wide ridge through the
    centre) only multiplies the field by its constant phase."""
    ap = F.Aperture(D=1e-3, f0=5e-3, lambda0=LAM0, N=256)
    base = S.sa_czt(ap, F.Instance(lam=LAM0, M=16))
    z0 = S.sa_czt(ap, F.Instance(lam=LAM0, M=16, creases=np.array([[0.3, 1e-4, 2e-4, 0.0]])))
    assert np.array_equal(base, z0)
    H = 0.3 * LAM0
    wide = S.sa_czt(ap, F.Instance(lam=LAM0, M=16, creases=np.array([[0.3, 0.0, 1e3, H]])))
    assert rel_l2(wide, base * np.exp(2j * np.pi * H / LAM0)) < 1e-9
