"""Planted mistakes in the oracle must each break at least one pin.

Every case below replaces one oracle function by a copy with a plausible
mistake in it (a dropped term, a wrong sign, an off-by-one grid, a transposed
operand, a wrong constant) and runs a fast subset of the pins in
``test_oracle_pins``; the case passes when at least one pin fails.  This checks
the pins, not the library: everything runs on the CPU and nothing here touches
the GPU path.
"""
import math

import numpy as np
import pytest

from oracle import fzp_oracle as O
import test_oracle_pins as pins
import test_oracle_multilevel_pins as mpins

ORIG = {name: getattr(O, name) for name in dir(O) if callable(getattr(O, name))}


def _pins():
    """(name, callable) of the fast pins."""
    return [
        ("czt_dft", lambda: pins.test_czt_reduces_to_dft(64)),
        ("czt_def", lambda: pins.test_bluestein_matches_definition(100, 17, 0.0123, 0.31)),
        ("czt_sum", pins.test_czt_explicit_sum_small),
        ("mask_bf", lambda: pins.test_zone_mask_brute_force(64, 0.0, 0)),
        ("mask_bf_open", lambda: pins.test_zone_mask_brute_force(63, 0.0, 1)),
        ("count_bf", lambda: pins.test_incident_count_brute_force(65, 0.0)),
        ("direct0", lambda: pins.test_separable_matches_direct_eq1(0)),
        ("direct1", lambda: pins.test_separable_matches_direct_eq1(1)),
        ("direct_creases", pins.test_separable_matches_direct_with_creases),
        ("crease_profile", pins.test_crease_height_profile),
        ("parseval", pins.test_parseval_in_the_dft_window),
        ("symmetry", pins.test_symmetry_undeformed),
        ("lambda_inv", pins.test_wavelength_invariance_at_first_order_focus),
        ("tilt", pins.test_tilt_shifts_and_constant_phase_leaves_intensity),
        ("fwhm_gauss", pins.test_fwhm_extraction_on_gaussian),
        ("fwhm_airy", pins.test_fwhm_extraction_on_sampled_airy),
        ("mtf_delta", pins.test_mtf_delta_and_constant),
        ("mtf_airy", pins.test_mtf_of_ideal_airy),
        ("hankel_axis", pins.test_hankel_on_axis_closed_form),
        ("hankel_airy", pins.test_hankel_tends_to_airy_at_many_zones),
        ("airy_consts", pins.test_airy_constants_against_paper),
        ("eq3", pins.test_zone_count_eq3),
        ("ml_levels", lambda: mpins.test_phase_level_exact_rationals(4, 63)),
        ("ml_two", mpins.test_two_levels_is_open_minus_closed_amplitude_plate),
        ("ml_ladder", lambda: mpins.test_efficiency_ladder_at_many_zones(4)),
        ("ml_axis", mpins.test_small_grid_on_axis_matches_hankel),
        ("strehl", pins.test_strehl_is_the_share_of_an_ideal_lens_peak),
        ("ml_strehl", lambda: mpins.test_strehl_tends_to_sinc2(4)),
    ]


# --- the planted mistakes ----------------------------------------------------

def m_bluestein_post_chirp_sign(x, M, w, a):
    r = ORIG["czt_bluestein"](x, M, w, a)
    m = np.arange(M, dtype=np.float64)
    return r * np.exp(2j * np.pi * w * m * m)          # W^{-m^2/2} instead of W^{m^2/2}


def m_czt_direct_a_sign(x, M, w, a):
    return ORIG["czt_direct"](x, M, w, -a)


def m_coords_off_by_half(ap):
    return (np.arange(ap.N, dtype=np.float64) - 0.5 * ap.N) * ap.dx


def m_roi_symmetric(M, centre, dx_out):
    return centre + (np.arange(M, dtype=np.float64) - 0.5 * (M - 1)) * dx_out


def m_zone_even_open(ap, j0=0, j1=None):
    j1 = ap.N if j1 is None else j1
    inside = ORIG["zone_mask"](O.Aperture(D=ap.D, f0=ap.f0, lambda0=ap.lambda0, N=ap.N, pitch=ap.pitch,
                                          centre_open=1 - ap.centre_open), j0, j1)
    return inside


def m_zone_kappa_twice(ap, j0=0, j1=None):
    return ORIG["zone_mask"](O.Aperture(D=ap.D, f0=2 * ap.f0, lambda0=ap.lambda0, N=ap.N, pitch=ap.pitch,
                                        centre_open=ap.centre_open), j0, j1)


def m_output_no_dx2(ap, inst):
    return ORIG["output_factor"](ap, inst) / ap.dx ** 2


def m_output_conj_chirp(ap, inst):
    f = ORIG["output_factor"](ap, inst)
    r = O.resolve(ap, inst)
    xq = O.roi_coords(inst.M, inst.x0, r["dx_out"])
    yp = O.roi_coords(inst.M, inst.y0, r["dx_out"])
    ch = np.exp(1j * np.pi * (yp[:, None] ** 2 + xq[None, :] ** 2) / (r["lam"] * r["z"]))
    return f / ch / ch


def m_axis_no_origin_shift(g, xs, dx, xo, lz, method):
    return ORIG["_axis_czt"](g, xs, dx, xo, lz, method) * np.exp(2j * np.pi * xs * xo / lz)


def m_axis_transposed_roi(g, xs, dx, xo, lz, method):
    return ORIG["_axis_czt"](g, xs, dx, xo[::-1].copy(), lz, method)


def m_crease_sigma_is_width(x, y, creases):
    if creases is None:
        return ORIG["crease_height"](x, y, creases)
    c = np.array(creases, dtype=np.float64)
    c[:, 2] *= 2.0 * math.sqrt(2.0 * math.log(2.0))
    return ORIG["crease_height"](x, y, c)


def m_crease_angle(x, y, creases):
    if creases is None:
        return ORIG["crease_height"](x, y, creases)
    c = np.array(creases, dtype=np.float64)
    c[:, 0] += 0.5 * math.pi
    return ORIG["crease_height"](x, y, c)


def m_intensity_modulus(U):
    return np.abs(U)


def m_resolve_z_wrong(ap, inst):
    r = ORIG["resolve"](ap, inst)
    if inst.z <= 0.0:
        r["z"] = ap.f0 * inst.lam / ap.lambda0
        r["hw"] = inst.half_width if inst.half_width > 0.0 else 8.0 * inst.lam * r["z"] / ap.D
        r["dx_out"] = 2.0 * r["hw"] / inst.M
    return r


def m_fwhm_at_third(row):
    return ORIG["fwhm_1d"](np.asarray(row) ** 1.5)


def m_fwhm_no_spline(row):
    row = np.asarray(row, dtype=np.float64)
    k = int(np.argmax(row))
    half = 0.5 * row[k]
    left = k
    while left > 0 and row[left] >= half:
        left -= 1
    right = k
    while right < len(row) - 1 and row[right] >= half:
        right += 1
    return float(right - left - 1)


def m_mtf_no_normalise(I, dx_out, nu_cut):
    return ORIG["mtf_half_cut"](I, dx_out, nu_cut) * float(np.sum(I))


def m_mtf_bins_floor(I, dx_out, nu_cut):
    return ORIG["mtf_half_cut"](I, dx_out, 0.98 * nu_cut)


def m_hankel_no_quadratic_phase(rho, ap, lam, z, nodes=16):
    return ORIG["hankel_field"](rho, ap, lam, 1e3 * z, nodes) * 1e3


def m_closed_form_centre_open(ap, lam=None, z=None):
    a = O.Aperture(D=ap.D, f0=ap.f0, lambda0=ap.lambda0, N=ap.N, centre_open=1 - ap.centre_open)
    return ORIG["on_axis_closed_form"](a, lam, z)


def m_incident_off_by_one(ap):
    return ORIG["incident_count"](ap) + 1


def m_eq3_paraxial(D, lam, f):
    return (0.5 * D) ** 2 / (lam * f)


def m_level_kappa_full_l(ap, j0=0, j1=None):
    j1 = ap.N if j1 is None else j1
    a = O.Aperture(D=ap.D, f0=ap.f0, lambda0=ap.lambda0, N=ap.N, pitch=ap.pitch, levels=2 * ap.levels)
    return ORIG["phase_level"](a, j0, j1) % ap.levels      # kappa * L instead of kappa * L/2


def m_field_phase_sign(ap, inst, j0=0, j1=None):
    return np.conj(ORIG["aperture_field"](ap, inst, j0, j1)) if ap.levels >= 2 else \
        ORIG["aperture_field"](ap, inst, j0, j1)


def m_intervals_phase_sign(ap, s_max):
    lo, hi, t = ORIG["_open_zone_intervals"](ap, s_max)
    return lo, hi, np.conj(t)


def m_metrics_strehl_no_pi2(U_or_I, ap, inst, p_in_count=None):
    m = ORIG["metrics"](U_or_I, ap, inst, p_in_count)
    m["strehl"] *= math.pi ** 2                         # peak over (R^2/(lambda z))^2
    return m


def m_hankel_strehl_no_pi2(ap, lam=None, z=None, nodes=16, lobe_nodes=96):
    h = ORIG["hankel_metrics"](ap, lam, z, nodes, lobe_nodes)
    h["strehl"] *= math.pi ** 2
    return h


MUTANTS = {
    "czt_bluestein": m_bluestein_post_chirp_sign,
    "czt_direct": m_czt_direct_a_sign,
    "aperture_coords": m_coords_off_by_half,
    "roi_coords": m_roi_symmetric,
    "zone_mask/even": m_zone_even_open,
    "zone_mask/kappa": m_zone_kappa_twice,
    "output_factor/dx2": m_output_no_dx2,
    "output_factor/conj": m_output_conj_chirp,
    "_axis_czt/shift": m_axis_no_origin_shift,
    "_axis_czt/reversed": m_axis_transposed_roi,
    "crease_height/sigma": m_crease_sigma_is_width,
    "crease_height/angle": m_crease_angle,
    "intensity": m_intensity_modulus,
    "resolve": m_resolve_z_wrong,
    "fwhm_1d/level": m_fwhm_at_third,
    "fwhm_1d/nospline": m_fwhm_no_spline,
    "mtf_half_cut/norm": m_mtf_no_normalise,
    "mtf_half_cut/cut": m_mtf_bins_floor,
    "hankel_field": m_hankel_no_quadratic_phase,
    "on_axis_closed_form": m_closed_form_centre_open,
    "incident_count": m_incident_off_by_one,
    "zone_count_exact": m_eq3_paraxial,
    "phase_level/kappa": m_level_kappa_full_l,
    "aperture_field/phase_sign": m_field_phase_sign,
    "_open_zone_intervals/phase_sign": m_intervals_phase_sign,
    "metrics/strehl": m_metrics_strehl_no_pi2,
    "hankel_metrics/strehl": m_hankel_strehl_no_pi2,
}


@pytest.mark.parametrize("key", list(MUTANTS))
def test_planted_mistake_is_caught(key, monkeypatch):
    name = key.split("/")[0]
    monkeypatch.setattr(O, name, MUTANTS[key])
    failed = []
    for pin_name, fn in _pins():
        try:
            with np.errstate(all="ignore"):
                fn()
        except (AssertionError, ValueError, IndexError, ZeroDivisionError, FloatingPointError):
            failed.append(pin_name)
    assert failed, f"no pin catches the planted mistake {key}"


def test_unmutated_oracle_passes_every_pin():
    for pin_name, fn in _pins():
        fn()
