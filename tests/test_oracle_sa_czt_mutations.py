"""Planted mistakes in the non-paraxial (SA-CZT) oracle must each break at least
one of its pins (``test_oracle_sa_czt_pins``).  Each case replaces one oracle
function by a copy with a plausible mistake (a dropped term, a wrong sign, a
wrong constant, a paraxial shortcut); CPU only."""
import numpy as np
import pytest

from oracle import fzp_oracle as F
from oracle import sa_czt_oracle as S
import test_oracle_sa_czt_pins as pins

ORIG = {name: getattr(S, name) for name in dir(S) if callable(getattr(S, name))}


def _pins():
    """Cheapest first; a mutant is caught at the first failing pin."""
    return [
        ("pad", pins.test_pad_size_rule),
        ("eq3_rational", lambda: pins.test_eq3_zone_index_in_exact_rationals(64, 1e-3, 2e-3)),
        ("rs_quad", pins.test_rs_closed_form_against_quadrature),
        ("unitary", pins.test_angular_spectrum_step_is_unitary),
        ("zoom_parseval", pins.test_zoom_parseval_in_dft_window),
        ("paraxial_limit", pins.test_paraxial_limit_matches_fresnel_oracle),
        ("fit_split", pins.test_fit_split_is_immaterial),
        ("f2_focus", pins.test_eq3_plate_focuses_in_phase_at_f2),
    ]


def m_eq3_paraxial(ap, j0=0, j1=None):
    j1 = ap.N if j1 is None else j1
    N = ap.N
    ci = 2 * np.arange(N, dtype=np.int64) - (N - 1)
    cj = 2 * np.arange(j0, j1, dtype=np.int64) - (N - 1)
    K = (cj[:, None] ** 2 + ci[None, :] ** 2).astype(np.float64)
    return np.floor(K * (ap.dx * ap.dx / (4.0 * ap.lambda0 * ap.f0))).astype(np.int64)


def m_eq3_sag_doubled(ap, j0=0, j1=None):
    j1 = ap.N if j1 is None else j1
    N = ap.N
    ci = 2 * np.arange(N, dtype=np.int64) - (N - 1)
    cj = 2 * np.arange(j0, j1, dtype=np.int64) - (N - 1)
    r2 = (cj[:, None] ** 2 + ci[None, :] ** 2).astype(np.float64) * ap.dx * ap.dx / 4.0
    lam, f = ap.lambda0, ap.f0                         # (lam^2/2) n^2 + lam f n = r^2
    return np.floor((-lam * f + np.sqrt(lam * lam * f * f + 2 * lam * lam * r2)) / (lam * lam)).astype(np.int64)


def m_sa_no_constant_phase(ap, inst, radii="eq3", pad=1.5, k_fit=2.0 / 3.0, method="bluestein"):
    U = ORIG["sa_czt"](ap, inst, radii, pad, k_fit, method)
    r = F.resolve(ap, inst)
    k0, kmax, c, d = S.fit_constants(r["lam"], k_fit)
    return U * np.exp(-1j * np.mod(c * kmax * r["z"], 2.0 * np.pi))   # e^{i c k_max z} dropped


def m_as_conj(U0, dx, lam, z, k_fit=2.0 / 3.0):
    return ORIG["angular_spectrum_step"](U0, dx, lam, -z, k_fit)


def m_as_paraxial_kz(U0, dx, lam, z, k_fit=2.0 / 3.0):
    k0, kmax, c, d = S.fit_constants(lam, k_fit)
    Np = U0.shape[0]
    nu = np.fft.fftfreq(Np, d=dx)
    K2 = (2.0 * np.pi) ** 2 * (nu[:, None] ** 2 + nu[None, :] ** 2)
    h = (k0 - K2 / (2.0 * k0)) - c * kmax - d * K2 / kmax
    return np.fft.ifft2(np.fft.fft2(U0) * np.exp(1j * h * z))


def m_as_no_evanescent_cut(U0, dx, lam, z, k_fit=2.0 / 3.0):
    k0, kmax, c, d = S.fit_constants(lam, k_fit)
    Np = U0.shape[0]
    nu = np.fft.fftfreq(Np, d=dx)
    K2 = (2.0 * np.pi) ** 2 * (nu[:, None] ** 2 + nu[None, :] ** 2)
    h = np.sqrt(k0 * k0 - K2) - c * kmax - d * K2 / kmax
    return np.fft.ifft2(np.fft.fft2(U0) * np.exp(1j * h * z))


def m_zoom_no_dx2(U1, dx, Z, xq, yp, method="bluestein"):
    return ORIG["zoom"](U1, dx, Z, xq, yp, method) / (dx * dx)


def m_zoom_chirp_sign(U1, dx, Z, xq, yp, method="bluestein"):
    Np = U1.shape[0]
    u = (np.arange(Np, dtype=np.float64) - 0.5 * (Np - 1)) * dx
    ch = np.exp(-2j * np.pi * u * u / Z)               # conj(chirp) applied on top of the chirp
    return ORIG["zoom"](U1 * ch[None, :] * ch[:, None], dx, Z, xq, yp, method)


def m_sa_z_with_k0(ap, inst, radii="eq3", pad=1.5, k_fit=2.0 / 3.0, method="bluestein"):
    r = F.resolve(ap, inst)
    lam, z = r["lam"], r["z"]
    k0, kmax, c, d = S.fit_constants(lam, k_fit)
    U1 = S.angular_spectrum_step(S.padded_aperture(ap, radii, pad, inst), ap.dx, lam, z, k_fit)
    Z = 4.0 * np.pi * abs(d) * z / k0
    xq = F.roi_coords(inst.M, inst.x0, r["dx_out"])
    yp = F.roi_coords(inst.M, inst.y0, r["dx_out"])
    acc = S.zoom(U1, ap.dx, Z, xq, yp, method)
    pre = np.exp(1j * np.mod(c * kmax * z, 2.0 * np.pi)) / (1j * Z)
    return pre * np.exp(1j * np.pi * (yp[:, None] ** 2 + xq[None, :] ** 2) / Z) * acc


def m_pad_parity(N, pad=1.5):
    m = ORIG["pad_size"](N, pad)
    return m + 1 if N > 1 else m


def m_rs_no_obliquity(edges, lam, z):
    k = 2.0 * np.pi / lam
    return complex(sum(np.exp(1j * k * np.hypot(z, a)) - np.exp(1j * k * np.hypot(z, b)) for a, b in edges))


MUTANTS = {
    "zone_index_eq3/paraxial": m_eq3_paraxial,
    "zone_index_eq3/sag": m_eq3_sag_doubled,
    "sa_czt/constant_phase": m_sa_no_constant_phase,
    "angular_spectrum_step/conj": m_as_conj,
    "angular_spectrum_step/paraxial_kz": m_as_paraxial_kz,
    "angular_spectrum_step/evanescent": m_as_no_evanescent_cut,
    "zoom/dx2": m_zoom_no_dx2,
    "zoom/chirp": m_zoom_chirp_sign,
    "sa_czt/Z": m_sa_z_with_k0,
    "pad_size/parity": m_pad_parity,
    "rs_on_axis_annuli/obliquity": m_rs_no_obliquity,
}


@pytest.mark.parametrize("key", list(MUTANTS))
def test_planted_mistake_is_caught(key, monkeypatch):
    monkeypatch.setattr(S, key.split("/")[0], MUTANTS[key])
    for pin_name, fn in _pins():
        try:
            with np.errstate(all="ignore"):
                fn()
        except (AssertionError, ValueError, IndexError, ZeroDivisionError, FloatingPointError):
            return
    pytest.fail(f"no pin catches the planted mistake {key}")
