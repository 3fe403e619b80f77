"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself: a value
the paper prints, a closed form, a textbook routine, brute force on tiny
inputs, or an exact invariant.  All run on the CPU.
"""
import math
import os

import numpy as np
import pytest
from scipy import special

from oracle import fzp_oracle as O
from fzp_inputs import crease_draws

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LAM0 = 632.8e-9


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _golden_values():
    out = {}
    with open(os.path.join(GOLDEN, "worked_values.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                parts = line.split()
                out[parts[0]] = float(parts[1])
    return out


# --------------------------------------------------------------------------
# Chirp-z transform (Eq. 9, Sec. 2.6)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 7, 64, 250])
def test_czt_reduces_to_dft(n):
    """A = 1, W = exp(-2 pi i/N), M = N gives the DFT (Sec. 2.6)."""
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = np.fft.fft(x)
    scale = np.abs(ref).max()
    assert np.abs(O.czt_bluestein(x, n, 1.0 / n, 0.0) - ref).max() <= 1e-12 * scale * max(1, n / 16)
    assert np.abs(O.czt_direct(x, n, 1.0 / n, 0.0) - ref).max() <= 1e-12 * scale * max(1, n / 16)


@pytest.mark.parametrize("n,m,w,a", [(100, 17, 0.0123, 0.31), (13, 200, 1e-3, -0.2),
                                     (512, 512, 16.0 / (512 * 64), 0.0), (1, 5, 0.1, 0.4)])
def test_bluestein_matches_definition(n, m, w, a):
    rng = np.random.default_rng(7)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    assert rel_l2(O.czt_bluestein(x, m, w, a), O.czt_direct(x, m, w, a)) < 1e-12


def test_czt_explicit_sum_small():
    """Eq. 9 term by term with a pure-Python loop."""
    x = np.array([1.0, -2.0 + 0.5j, 0.25j, 3.0])
    M, w, a = 3, 0.07, 0.11
    A, W = np.exp(2j * np.pi * a), np.exp(-2j * np.pi * w)
    ref = [sum(x[n] * A ** (-n) * W ** (m * n) for n in range(4)) for m in range(M)]
    assert np.allclose(O.czt_bluestein(x, M, w, a), ref, rtol=0, atol=1e-13)


# --------------------------------------------------------------------------
# Zone mask and incident power (Sec. 2.2, Fig. 2 stage 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,pitch,centre_open", [(64, 0.0, 0), (63, 0.0, 1), (50, 2e-3 / 47, 0)])
def test_zone_mask_brute_force(N, pitch, centre_open):
    """Per-sample loop: r^2 = x^2 + y^2, zone n = floor(r^2/(lambda0 f0)), open if odd, r <= D/2."""
    ap = O.Aperture(D=2e-3, f0=3e-3, lambda0=LAM0, N=N, pitch=pitch, centre_open=centre_open)
    dx = ap.dx
    got = O.zone_mask(ap)
    for j in range(N):
        y = (j - (N - 1) / 2) * dx
        for i in range(N):
            x = (i - (N - 1) / 2) * dx
            r2 = x * x + y * y
            n = math.floor(r2 / (ap.lambda0 * ap.f0))
            want = (r2 <= (ap.D / 2) ** 2 * (1 + 1e-15)) and ((n % 2 == 1) != bool(centre_open))
            assert got[j, i] == want, (j, i)


def test_zone_mask_symmetry_and_rows():
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=256)
    m = O.zone_mask(ap)
    assert np.array_equal(m, m[::-1, :]) and np.array_equal(m, m[:, ::-1]) and np.array_equal(m, m.T)
    assert np.array_equal(O.zone_mask(ap, 40, 77), m[40:77])
    # the centre zone is opaque, the first ring open
    c = ap.N // 2
    assert not m[c, c]


@pytest.mark.parametrize("N,pitch", [(64, 0.0), (65, 0.0), (101, 1e-3 / 97), (2, 0.0), (1, 0.0)])
def test_incident_count_brute_force(N, pitch):
    ap = O.Aperture(D=1e-3, f0=1e-2, lambda0=LAM0, N=N, pitch=pitch)
    c = 2 * np.arange(N) - (N - 1)
    K = c[:, None] ** 2 + c[None, :] ** 2
    assert O.incident_count(ap) == int(np.count_nonzero(K <= ap.k_max))


def test_incident_power_tends_to_disc_area():
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096)
    p_in = O.incident_count(ap) * ap.dx ** 2
    assert abs(p_in / (math.pi * 1e-6) - 1.0) < 2.0 / ap.N


def test_zone_count_eq3():
    """Eq. 3 at r_n = D/2; tends to the paraxial N_F = R^2/(lambda f) (Eq. 4) when n lambda << f."""
    for D, f, lam in [(2e-3, 10e-3, LAM0), (1.0, 5.0, 532e-9)]:
        n = O.zone_count_exact(D, lam, f)
        assert abs(n * lam * f + n * n * lam * lam / 4 - (D / 2) ** 2) < 1e-12 * (D / 2) ** 2
        nf = (D / 2) ** 2 / (lam * f)
        assert n < nf and abs(n / nf - 1) < 0.01


# --------------------------------------------------------------------------
# Closed forms and printed numbers (Sec. 2.3, Sec. 4.2, Sec. 8.3)
# --------------------------------------------------------------------------

def test_airy_constants_against_paper():
    g = _golden_values()
    # Sec. 2.3 prints the coefficient truncated (1.028), Fig. 2 rounded (1.029)
    assert math.floor(O.AIRY_FWHM * 1000) / 1000 == g["airy_fwhm_coeff_sec23"]
    assert abs(O.AIRY_FWHM - g["airy_fwhm_coeff_fig2"]) < 1e-3
    assert round(1.0 / math.pi ** 2, 3) == g["binary_de_first_order"]
    assert round(O.J11 / math.pi, 2) == g["airy_null_coeff"]
    fw = O.AIRY_FWHM * 532e-9 * 1.5 / 0.08
    assert round(fw * 1e6, 2) == round(g["lit_fwhm_d008_f15_532"] * 1e6, 2)
    fw1 = O.AIRY_FWHM * 532e-9 * 5.0 / 1.0
    assert abs(fw1 / g["sim_fwhm_d1_f5_532"] - 1.0) < 1e-4
    # encircled energy inside the first null of the Airy pattern
    assert abs(O.AIRY_LOBE_FRACTION - 0.837785) < 1e-6


def test_fwhm_extraction_on_sampled_airy():
    """The FWHM extractor on an analytic Airy pattern returns 1.028994 lambda f / D."""
    for M in (128, 256, 512):
        dxo = 16.0 / M                       # lambda z / D = 1
        x = (np.arange(M) - M / 2) * dxo
        v = np.pi * np.hypot(x[:, None], x[None, :])
        with np.errstate(invalid="ignore", divide="ignore"):
            I = np.where(v == 0, 1.0, (2 * special.j1(v) / v) ** 2)
        assert abs(O.fwhm_1d(I[M // 2]) * dxo / O.AIRY_FWHM - 1) < 1e-5


def test_fwhm_extraction_on_gaussian():
    M = 101
    x = np.arange(M) - 50.3
    sig = 6.0
    g = np.exp(-x * x / (2 * sig * sig))
    assert abs(O.fwhm_1d(g) / (2 * math.sqrt(2 * math.log(2)) * sig) - 1) < 2e-4


def test_mtf_of_ideal_airy():
    """MTF of an aberration-free circular pupil at nu_cut/2:
    (2/pi)(acos(1/2) - (1/2) sqrt(3/4)) = 0.3910.  A wide window keeps truncation small."""
    M, half = 1024, 64.0                     # half-width 64 lambda z / D
    dxo = 2 * half / M
    x = (np.arange(M) - M / 2) * dxo
    v = np.pi * np.hypot(x[:, None], x[None, :])
    with np.errstate(invalid="ignore", divide="ignore"):
        I = np.where(v == 0, 1.0, (2 * special.j1(v) / v) ** 2)
    ideal = 2 / math.pi * (math.acos(0.5) - 0.5 * math.sqrt(0.75))
    assert abs(O.mtf_half_cut(I, dxo, 1.0) / ideal - 1) < 0.01


def test_mtf_delta_and_constant():
    I = np.zeros((64, 64)); I[32, 32] = 1.0
    assert abs(O.mtf_half_cut(I, 1.0, 0.25) - 1.0) < 1e-14
    assert abs(O.mtf_half_cut(np.ones((64, 64)), 1.0, 0.25)) < 1e-14


# --------------------------------------------------------------------------
# The propagated field (Eqs. 1-2, 9-10)
# --------------------------------------------------------------------------

CASES = [
    dict(ap=dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=96), inst=dict(lam=LAM0, M=12)),
    dict(ap=dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=81, centre_open=1),
         inst=dict(lam=560e-9, M=9, x0=2e-6, y0=-3e-6, half_width=30e-6)),
    dict(ap=dict(D=1e-3, f0=4e-3, lambda0=LAM0, N=70, pitch=1e-3 / 66),
         inst=dict(lam=LAM0, M=16, z=4.1e-3)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_separable_matches_direct_eq1(case):
    """Eq. 1 summed sample by sample equals the separable CZT and DFT forms."""
    ap = O.Aperture(**CASES[case]["ap"])
    inst = O.Instance(**CASES[case]["inst"])
    ref = O.fresnel_direct(ap, inst)
    for method in ("bluestein", "dft", "czt_direct"):
        assert rel_l2(O.propagate(ap, inst, method=method, stripe=23), ref) < 1e-12


def test_separable_matches_direct_with_creases():
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=90)
    cr = crease_draws(3, ap.D, LAM0, 8)
    cr[:, 2] *= 0.1                          # narrow ridges so they vary across this small aperture
    inst = O.Instance(lam=700e-9, M=10, creases=cr)
    ref = O.fresnel_direct(ap, inst)
    assert rel_l2(O.propagate(ap, inst, stripe=37), ref) < 1e-12
    flat = O.propagate(ap, O.Instance(lam=700e-9, M=10))
    assert rel_l2(flat, ref) > 1e-3          # the creases do change the field


def test_parseval_in_the_dft_window():
    """With dx_out = lambda z/(N dx) and M = N the kernel is a DFT, so
    sum |U|^2 dx_out^2 = sum |t|^2 dx^2 (discrete Parseval)."""
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=128)
    z = ap.f0
    hw = LAM0 * z / (2 * ap.dx)
    inst = O.Instance(lam=LAM0, M=128, half_width=hw, z=z)
    U = O.propagate(ap, inst)
    dxo = O.resolve(ap, inst)["dx_out"]
    p_out = float(np.sum(O.intensity(U))) * dxo * dxo
    p_open = float(np.count_nonzero(O.zone_mask(ap))) * ap.dx ** 2
    assert abs(p_out / p_open - 1) < 1e-12


def test_row_ranges_add_up():
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=256)
    inst = O.Instance(lam=LAM0, M=32)
    full = O.propagate(ap, inst, stripe=64)
    parts = O.propagate(ap, inst, rows=(0, 100), stripe=64) + O.propagate(ap, inst, rows=(100, 256), stripe=64)
    assert rel_l2(parts, full) < 1e-13


def test_symmetry_undeformed():
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=512)
    inst = O.Instance(lam=LAM0, M=64)
    I = O.intensity(O.propagate(ap, inst))
    s = I[1:, 1:]
    assert rel_l2(s[::-1, :], s) < 1e-12 and rel_l2(s[:, ::-1], s) < 1e-12 and rel_l2(s.T, s) < 1e-12


def test_babinet():
    """t(centre opaque) + t(centre open) = the clear disc, and the field is linear in t."""
    kw = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=200)
    a0, a1 = O.Aperture(**kw), O.Aperture(centre_open=1, **kw)
    inst = O.Instance(lam=LAM0, M=24)
    c = 2 * np.arange(200) - 199

    def disc(j0, j1):
        K = c[j0:j1, None] ** 2 + c[None, :] ** 2
        return (K <= a0.k_max).astype(np.complex128)

    u = O.propagate(a0, inst) + O.propagate(a1, inst)
    assert rel_l2(u, O.propagate(a0, inst, field_fn=disc)) < 1e-12


def test_wavelength_invariance_at_first_order_focus():
    """At z = f0 lambda0 / lambda the product lambda z is fixed, so the undeformed
    focal intensity does not depend on lambda."""
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=300)
    I0 = O.intensity(O.propagate(ap, O.Instance(lam=LAM0, M=32)))
    for lam in (500e-9, 800e-9):
        assert rel_l2(O.intensity(O.propagate(ap, O.Instance(lam=lam, M=32))), I0) < 1e-11


def test_tilt_shifts_and_constant_phase_leaves_intensity():
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=256)
    inst = O.Instance(lam=LAM0, M=32)
    r = O.resolve(ap, inst)
    x = O.aperture_coords(ap)
    k = 3
    a = k * r["dx_out"] / r["z"]             # tilt angle moving the spot by k ROI samples

    def tilted(j0, j1):
        return O.zone_mask(ap, j0, j1) * np.exp(2j * np.pi * a * x[None, :] / LAM0)

    def const(j0, j1):
        return O.zone_mask(ap, j0, j1) * np.exp(1j * 0.7)

    I = O.intensity(O.propagate(ap, inst))
    It = O.intensity(O.propagate(ap, inst, field_fn=tilted))
    assert rel_l2(It[:, k:], I[:, :-k]) < 1e-11
    assert rel_l2(O.intensity(O.propagate(ap, inst, field_fn=const)), I) < 1e-12


def test_zero_height_creases_are_bit_identical():
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=128)
    cr = crease_draws(0, ap.D, LAM0)
    cr[:, 3] = 0.0
    a = O.propagate(ap, O.Instance(lam=LAM0, M=16, creases=cr))
    b = O.propagate(ap, O.Instance(lam=LAM0, M=16))
    assert np.array_equal(a, b)


# --------------------------------------------------------------------------
# Continuous radial reference (Hankel form of Eq. 2) and the 2-D grid against it
# --------------------------------------------------------------------------

def test_hankel_on_axis_closed_form():
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096)
    assert abs(float(O.hankel_intensity(0.0, ap, LAM0, ap.f0)[0]) / O.on_axis_closed_form(ap) - 1) < 1e-12
    # 158 full zones at N_F = 158.03: each open zone adds 2 to the axial amplitude
    n_open = int(((ap.D / 2) ** 2 / (LAM0 * ap.f0)) // 2)
    assert abs(O.on_axis_closed_form(ap) / (2 * n_open) ** 2 - 1) < 2e-3


def test_hankel_tends_to_airy_at_many_zones():
    """Many zones: FWHM -> 1.028994 lambda f/D and main-lobe DE -> 0.837785/pi^2."""
    ap = O.Aperture(D=0.2, f0=1.0, lambda0=LAM0, N=2)
    h = O.hankel_metrics(ap)
    lz = LAM0 * ap.f0
    assert abs(h["fwhm"] / (O.AIRY_FWHM * lz / ap.D) - 1) < 2e-5
    assert abs(h["de"] / (O.AIRY_LOBE_FRACTION / math.pi ** 2) - 1) < 2e-4


def test_strehl_is_the_share_of_an_ideal_lens_peak():
    """Strehl = peak / (pi R^2/(lambda z))^2, where pi R^2/(lambda z) is the focal
    field of an ideal lens of radius R (the disc area over lambda z).  A binary
    plate whose last zone is opaque has n_open full open zones, each adding 2 to
    the axial amplitude, so pi^2 Strehl = (2 n_open / N_F)^2 -> 1 (the 1/pi^2 of
    a binary amplitude plate); the 2-D grid gives the same within its sampling
    error."""
    ap = O.Aperture(D=0.02, f0=0.1, lambda0=LAM0, N=2)
    nf = (0.5 * ap.D) ** 2 / (LAM0 * ap.f0)                    # 1580.28 zones
    n_open = int(nf) // 2                                       # zones 1, 3, .., 1579; zone 1580 is opaque
    assert int(nf) % 2 == 0
    want = (2 * n_open / nf) ** 2
    assert abs(O.hankel_metrics(ap)["strehl"] * math.pi ** 2 - want) < 1e-6
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=1024)      # 158.03 zones, 1.6 samples per outer zone
    nf = (0.5 * ap.D) ** 2 / (LAM0 * ap.f0)
    inst = O.Instance(lam=LAM0, M=32)
    m = O.metrics(O.propagate(ap, inst, stripe=512), ap, inst)
    assert abs(m["strehl"] * math.pi ** 2 - (2 * (int(nf) // 2) / nf) ** 2) < 2e-3


def test_grid_matches_hankel_fzp2mm():
    """4096^2 grid (6.5 samples per outer zone) vs the continuous radial integral."""
    ap = O.Aperture(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096)
    inst = O.Instance(lam=LAM0, M=256)
    U = O.propagate(ap, inst, stripe=512)
    m = O.metrics(U, ap, inst)
    h = O.hankel_metrics(ap)
    assert abs(m["fwhm_x"] / h["fwhm"] - 1) < 1e-4
    assert abs(m["fwhm_y"] / h["fwhm"] - 1) < 1e-4
    assert abs(m["de"] / h["de"] - 1) < 2e-4
    I = O.intensity(U)
    assert abs(I[128, 128] / h["i0"] - 1) < 1e-4
    # the finite zone count puts this element 0.32 % / 0.75 % below the Airy values
    lz = LAM0 * ap.f0
    assert -0.004 < m["fwhm_x"] / (O.AIRY_FWHM * lz / ap.D) - 1 < -0.002


# --------------------------------------------------------------------------
# Grid rule of the revised engine (Fig. 18 stage 1, Tables 1-5)
# --------------------------------------------------------------------------

def _tables():
    rows = []
    with open(os.path.join(GOLDEN, "v8_grid_tables.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t, D, f, L, dx, nx = line.split()
                rows.append((int(t), float(D), float(f), int(L), float(dx), int(nx)))
    return rows


@pytest.mark.parametrize("row", _tables(), ids=lambda r: f"table{r[0]}")
def test_v8_grid_rule(row):
    t, D, f, L, dx_um, nx = row
    if t == 5:
        dx, n = O.v8_grid(D, f, 532e-9, L)
        assert n != nx                       # the printed L = 2 does not reproduce Table 5
        dx, n = O.v8_grid(D, f, 532e-9, 4)   # its numbers are those of four levels
    else:
        dx, n = O.v8_grid(D, f, 532e-9, L)
    assert n == nx
    assert abs(dx * 1e6 - dx_um) <= 0.0006


# --------------------------------------------------------------------------
# Deformation model: straight Gaussian ridges, width given as the FWHM
# --------------------------------------------------------------------------

def test_crease_height_profile():
    """h = H at the ridge line, H/2 at a distance of half the width (FWHM),
    H/16 at a full width, and the ridge runs along theta + pi/2."""
    H, w, th, rho = 3e-7, 1.2e-3, 0.4, 2e-4
    cr = np.array([[th, rho, w, H]])
    n = np.array([math.cos(th), math.sin(th)])
    t = np.array([-math.sin(th), math.cos(th)])
    for s in (-2e-3, 0.0, 5e-4):              # any point along the ridge
        p0 = rho * n + s * t
        for d, want in ((0.0, H), (0.5 * w, 0.5 * H), (-0.5 * w, 0.5 * H), (w, H / 16)):
            p = p0 + d * n
            assert abs(float(O.crease_height(p[0], p[1], cr)) - want) <= 1e-12 * H
    # ridges add
    cr2 = np.array([[th, rho, w, H], [th + 1.0, -rho, 2 * w, 0.5 * H]])
    x, y = 1.3e-4, -7e-4
    assert abs(float(O.crease_height(x, y, cr2)) - float(O.crease_height(x, y, cr2[:1]))
               - float(O.crease_height(x, y, cr2[1:]))) < 1e-20
