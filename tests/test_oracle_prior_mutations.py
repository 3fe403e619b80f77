"""Planted mistakes in the physics-prior oracle must each break at least one of
its pins (``test_oracle_prior_pins``).  Each case replaces one oracle function
by a copy with a plausible mistake; CPU only."""
import numpy as np
import pytest

from oracle import fzp_oracle as F
from oracle import prior_oracle as PR
import test_oracle_prior_pins as pins

ORIG = {name: getattr(PR, name) for name in PR.__all__}


def _pins():
    return [
        ("coverage", pins.test_coverage_exact_and_area),
        ("airy", pins.test_airy_undeformed),
        ("parseval", pins.test_parseval_in_dft_window),
        ("uniform", pins.test_uniform_phase_is_invisible),
        ("mirror", pins.test_mirror_symmetry),
        ("czt_633", lambda: pins.test_matches_zone_plate_czt(pins.LAM0)),
        ("czt_560", lambda: pins.test_matches_zone_plate_czt(560e-9)),
    ]


def m_coverage_centre_only(Np, ss):
    return ORIG["coverage"](Np, 1)


def m_coverage_lt_half(Np, ss):
    n = Np * ss
    c = 2 * np.arange(n, dtype=np.int64) + 1 - n
    inside = (c[:, None] ** 2 + c[None, :] ** 2) <= (n * n) // 4           # radius halved
    return inside.reshape(Np, ss, Np, ss).sum(axis=(1, 3)) / float(ss * ss)


def m_coords_half_pixel(D, Np):
    return (np.arange(Np, dtype=np.float64) - 0.5 * Np) / Np * D


def m_turns_no_four(Np, M):
    a = 2 * np.arange(Np, dtype=np.int64) + 1 - Np
    b = 2 * np.arange(M, dtype=np.int64) - M
    return np.mod(np.outer(b, a), Np * M).astype(np.float64) / (Np * M)


def m_turns_sign(Np, M):
    return np.mod(-ORIG["dft_turns"](Np, M), 1.0)


def m_field_conj(D, Np, ss, creases, lam):
    return np.conj(ORIG["pupil_field"](D, Np, ss, creases, lam))


def m_field_lambda0(D, Np, ss, creases, lam):
    return ORIG["pupil_field"](D, Np, ss, creases, pins.LAM0)


def m_field_no_two_pi(D, Np, ss, creases, lam):
    u = PR.pupil_coords(D, Np)
    h = F.crease_height(u[None, :], u[:, None], creases)
    return PR.coverage(Np, ss) * np.exp(1j * h / lam)


def m_field_amplitude(D, Np, ss, creases, lam):
    u = PR.pupil_coords(D, Np)
    h = F.crease_height(u[None, :], u[:, None], creases)
    return PR.coverage(Np, ss) * (1.0 + 2.0 * np.pi * h / lam)             # linearised screen


def m_field_transposed(D, Np, ss, creases, lam):
    return ORIG["pupil_field"](D, Np, ss, creases, lam).T


def m_intensity_no_pi2(D, M, creases, lam, Np=128, ss=4):
    return ORIG["prior_intensity"](D, M, creases, lam, Np, ss) * np.pi ** 2


def m_intensity_np2(D, M, creases, lam, Np=128, ss=4):
    return ORIG["prior_intensity"](D, M, creases, lam, Np, ss) * float(Np) ** 2


def m_intensity_amplitude(D, M, creases, lam, Np=128, ss=4):
    return np.sqrt(ORIG["prior_intensity"](D, M, creases, lam, Np, ss))


MUTANTS = {
    "coverage_centre_only": ("coverage", m_coverage_centre_only),
    "coverage_half_radius": ("coverage", m_coverage_lt_half),
    "coords_half_pixel": ("pupil_coords", m_coords_half_pixel),
    "turns_no_four": ("dft_turns", m_turns_no_four),
    "turns_sign": ("dft_turns", m_turns_sign),
    "field_conj": ("pupil_field", m_field_conj),
    "field_lambda0": ("pupil_field", m_field_lambda0),
    "field_no_two_pi": ("pupil_field", m_field_no_two_pi),
    "field_amplitude": ("pupil_field", m_field_amplitude),
    "field_transposed": ("pupil_field", m_field_transposed),
    "intensity_no_pi2": ("prior_intensity", m_intensity_no_pi2),
    "intensity_np2": ("prior_intensity", m_intensity_np2),
    "intensity_amplitude": ("prior_intensity", m_intensity_amplitude),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    fn_name, fn = MUTANTS[name]
    monkeypatch.setattr(PR, fn_name, fn)
    caught = None
    for pin_name, pin in _pins():
        try:
            pin()
        except AssertionError:
            caught = pin_name
            break
    assert caught is not None, f"mutant {name} passes every pin"


def test_original_passes_every_pin():
    for _, pin in _pins():
        pin()
