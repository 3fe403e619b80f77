"""FP64 CPU oracle for the stripe-processed chirp-z Fresnel propagation of a
binary-amplitude (or L-level phase) Fresnel zone plate (FZP) onto a focal-plane
region of interest.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this module.  The GPU
library never calls it and shares no code with it; the two meet only through
the seeded parameters in ``fzp_inputs``.

Everything here is plain NumPy/SciPy in float64 / complex128 and is written to
be checked against the paper by eye:

* the grids, the zone mask and the incident power follow the CZT method's
  stages 1-2 (Sec. 3.3, Fig. 2) with the zone radii of Eq. 4 and the zone count
  of Eq. 3;
* the field is Eq. 2 discretised: ``fresnel_direct`` sums Eq. 1 literally (tiny
  grids only), ``propagate(method="dft")`` evaluates the separable row/column
  sums as matrix products, and ``propagate(method="bluestein")`` evaluates each
  1-D sum as the chirp-z transform of Eq. 9 with the Fresnel mapping of Eq. 10,
  computed through Bluestein's identity (Sec. 2.6);
* ``hankel_*`` is the 1-D radial (Hankel) form of Eq. 2 for the continuous,
  axisymmetric, undeformed aperture, integrated zone by zone;
* ``metrics`` extracts FWHM, main-lobe diffraction efficiency, MTF at half the
  cutoff and Strehl as in the shared metric extractor (Sec. 3.3 stage 4 and
  Fig. 18 stage 5).

Readings where the paper is silent or ambiguous (all of them are listed, with
reasons, in the design notes of the repository):

* sample positions ``x_i = (i - (N-1)/2) dx`` (cell centred, no axis sample for
  even N) and ROI positions ``x'_q = x0 + (q - M/2) dx_out``,
  ``dx_out = 2 hw / M``, default half width ``hw = 8 lambda z / D``;
* zone index ``n = floor(K * kappa)`` with the exact integer
  ``K = (2i-N+1)^2 + (2j-N+1)^2`` and ``kappa = dx*dx / (4*lambda0*f0)``
  (one float64 product, so ``4 r^2 = K dx^2``); a sample is open when it lies in
  the disc ``K <= K_max`` and ``n`` is odd (``centre_open`` flips the parity);
  ``K_max = N^2`` for the default pitch ``D/N`` and ``floor((D/pitch)^2)``
  otherwise;
* an L-level phase plate (the revised engine's element, Fig. 18 stage 3)
  transmits ``exp(-2 pi i l / L)`` on the whole disc with the level
  ``l = floor(K * kappa_L) mod L``, ``kappa_L = kappa * (L/2)``: the ideal lens
  phase ``-pi r^2/(lambda0 f0)`` quantised into L equal steps per period of two
  zones (``L = 2`` gives +1 / -1 on even / odd zones);
* each instance is evaluated at its first-order focus ``z = f0 lambda0 / lambda``
  unless ``z`` is given;
* a membrane deformation is a thin phase screen ``phi = 2 pi h / lambda`` of
  straight Gaussian ridges ``h = sum_k H_k exp(-d_k^2 / (2 sigma_k^2))`` with
  ``d_k = x cos(theta_k) + y sin(theta_k) - rho_k`` and
  ``sigma_k = w_k / (2 sqrt(2 ln 2))``;
* FWHM: not-a-knot cubic spline through the row (column) of samples that
  contains the brightest sample, spline peak, half-maximum crossings found by
  bisection on the bracketing sample intervals;
* DE: main-lobe power inside ``r_null = j_{1,1}/pi * lambda z / D`` around the
  ROI centre over the incident power ``P_in = (#samples in the disc) dx^2``;
* MTF: ``|FFT2(I)|`` normalised at DC over the full ROI, averaged over radial
  bins ``round(|nu| / dnu)``, ``dnu = 1/(M dx_out)``, read by linear
  interpolation at ``nu_cut / 2`` with ``nu_cut = D / (lambda z)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
from scipy import fft as sfft
from scipy import special
from scipy.interpolate import CubicSpline

__all__ = [
    "Aperture", "Instance", "resolve", "aperture_coords", "roi_coords",
    "zone_mask", "disc_mask", "phase_level", "incident_count", "crease_height", "aperture_field",
    "fresnel_direct", "czt_direct", "czt_bluestein", "propagate",
    "output_factor", "intensity", "metrics", "fwhm_1d", "mtf_half_cut",
    "hankel_field", "hankel_intensity", "hankel_metrics", "on_axis_closed_form",
    "zone_count_exact", "v8_grid", "J11", "AIRY_FWHM", "AIRY_LOBE_FRACTION",
]

# First zero of J1.  r_null = J11/pi * lambda z / D (the Airy null, 1.22 lambda f/D
# in the paper's rounding).
J11 = float(special.jn_zeros(1, 1)[0])


def _airy_half_max_v() -> float:
    from scipy.optimize import brentq
    return brentq(lambda v: (2.0 * special.j1(v) / v) ** 2 - 0.5, 1.0, 2.0, xtol=1e-15)


# FWHM of |2 J1(v)/v|^2 in units of lambda f / D (Sec. 2.3: 1.028).
AIRY_FWHM = 2.0 * _airy_half_max_v() / np.pi
# Encircled energy of the Airy pattern inside its first null.
AIRY_LOBE_FRACTION = 1.0 - special.j0(J11) ** 2 - special.j1(J11) ** 2


@dataclass
class Aperture:
    """An FZP sampled on an N x N grid (Sec. 2.2, Sec. 3.3): binary amplitude
    (levels = 0), or an L-level phase plate (levels = L >= 2, the revised
    engine's element, Fig. 18 stage 3 and Tables 1-5)."""
    D: float                 # aperture diameter [m]
    f0: float                # design focal length [m]
    lambda0: float           # design wavelength [m]
    N: int                   # samples per side
    pitch: float = 0.0       # sample pitch [m]; 0 means D / N
    centre_open: int = 0     # 0: zone 0 (the centre) opaque; 1: centre open (amplitude plates)
    levels: int = 0          # 0: binary amplitude; L >= 2: L-level phase

    @property
    def dx(self) -> float:
        return self.pitch if self.pitch > 0.0 else self.D / self.N

    @property
    def k_max(self) -> int:
        """Largest K = 4 r^2 / dx^2 inside the aperture disc r <= D/2."""
        if self.pitch > 0.0:
            return int(np.floor((self.D / self.pitch) ** 2))
        return int(self.N) * int(self.N)


@dataclass
class Instance:
    """One propagation: wavelength, distance and ROI (Eq. 10 free parameters)."""
    lam: float
    M: int
    z: float = 0.0           # 0 means the first-order focus f0 lambda0 / lam
    x0: float = 0.0          # ROI centre [m]
    y0: float = 0.0
    half_width: float = 0.0  # 0 means 8 lam z / D
    creases: Optional[np.ndarray] = None   # (n, 4): theta, offset, width(FWHM), height(OPD)


def resolve(ap: Aperture, inst: Instance) -> dict:
    """Resolved scalars of one instance."""
    z = inst.z if inst.z > 0.0 else ap.f0 * ap.lambda0 / inst.lam
    hw = inst.half_width if inst.half_width > 0.0 else 8.0 * inst.lam * z / ap.D
    return dict(dx=ap.dx, z=z, lam=inst.lam, hw=hw, dx_out=2.0 * hw / inst.M,
                M=inst.M, N=ap.N, x0=inst.x0, y0=inst.y0)


def aperture_coords(ap: Aperture) -> np.ndarray:
    """Sample centres x_i = (i - (N-1)/2) dx."""
    return (np.arange(ap.N, dtype=np.float64) - 0.5 * (ap.N - 1)) * ap.dx


def roi_coords(M: int, centre: float, dx_out: float) -> np.ndarray:
    """ROI sample positions centre + (q - M/2) dx_out."""
    return centre + (np.arange(M, dtype=np.float64) - 0.5 * M) * dx_out


def zone_mask(ap: Aperture, j0: int = 0, j1: Optional[int] = None) -> np.ndarray:
    """Binary zone mask for aperture rows j0..j1-1 (bool, rows x N).

    Paraxial zone radii r_n^2 = n lambda0 f0 (Eq. 4): the sample at radius r
    lies in zone n = floor(r^2 / (lambda0 f0)); it is open when n is odd (the
    centre zone n = 0 is opaque) and it lies inside the aperture disc.
    """
    j1 = ap.N if j1 is None else j1
    N = ap.N
    ci = 2 * np.arange(N, dtype=np.int64) - (N - 1)
    cj = 2 * np.arange(j0, j1, dtype=np.int64) - (N - 1)
    K = cj[:, None] ** 2 + ci[None, :] ** 2                     # exact 4 r^2 / dx^2
    kappa = ap.dx * ap.dx / (4.0 * ap.lambda0 * ap.f0)
    n = np.floor(K.astype(np.float64) * kappa).astype(np.int64)
    odd = (n % 2) == 1
    if ap.centre_open:
        odd = ~odd
    return (K <= ap.k_max) & odd


def disc_mask(ap: Aperture, j0: int = 0, j1: Optional[int] = None) -> np.ndarray:
    """Samples of rows j0..j1-1 inside the aperture disc K <= K_max (bool)."""
    j1 = ap.N if j1 is None else j1
    N = ap.N
    ci = 2 * np.arange(N, dtype=np.int64) - (N - 1)
    cj = 2 * np.arange(j0, j1, dtype=np.int64) - (N - 1)
    return cj[:, None] ** 2 + ci[None, :] ** 2 <= ap.k_max


def phase_level(ap: Aperture, j0: int = 0, j1: Optional[int] = None) -> np.ndarray:
    """Phase level l in 0..L-1 of an L-level phase plate on rows j0..j1-1.

    With s = r^2 / (lambda0 f0) (the zone coordinate of Eq. 4; zone n covers
    n <= s < n + 1), the ideal lens phase -pi s is quantised per period of two
    zones into L equal steps (Fig. 18 stage 3): l = floor(L frac(s / 2)), i.e.
    l = floor(K kappa_L) mod L with kappa_L = kappa * (L/2), one float64 product
    like the zone rule (for L = 2, l is the zone parity).  The transmission is
    exp(-2 pi i l / L) inside the disc.
    """
    j1 = ap.N if j1 is None else j1
    L = int(ap.levels)
    N = ap.N
    ci = 2 * np.arange(N, dtype=np.int64) - (N - 1)
    cj = 2 * np.arange(j0, j1, dtype=np.int64) - (N - 1)
    K = cj[:, None] ** 2 + ci[None, :] ** 2
    kappa = ap.dx * ap.dx / (4.0 * ap.lambda0 * ap.f0)
    kappa_l = kappa * (0.5 * L)
    return np.floor(K.astype(np.float64) * kappa_l).astype(np.int64) % L


def incident_count(ap: Aperture) -> int:
    """Number of samples inside the aperture disc K <= K_max (exact integers).

    For each row, the admissible c = 2i-N+1 (same parity as N-1) satisfy
    c^2 <= K_max - c_j^2.
    """
    N = ap.N
    cj = 2 * np.arange(N, dtype=np.int64) - (N - 1)
    rem = ap.k_max - cj * cj
    total = 0
    for r in rem[rem >= 0]:
        m = _isqrt(int(r))
        # count integers c with |c| <= m and c = N-1 (mod 2), |c| <= N-1
        m = min(m, N - 1)
        if (N - 1) % 2 == 0:          # c even
            total += 2 * (m // 2) + 1
        else:                          # c odd
            total += 2 * ((m + 1) // 2)
    return total


def _isqrt(v: int) -> int:
    import math
    return math.isqrt(v)


def crease_height(x: np.ndarray, y: np.ndarray, creases: Optional[np.ndarray]) -> np.ndarray:
    """Optical path difference h(x, y) of straight Gaussian ridges [m]."""
    h = np.zeros(np.broadcast(x, y).shape)
    if creases is None:
        return h
    for theta, rho, width, height in np.asarray(creases, dtype=np.float64):
        sigma = width / (2.0 * np.sqrt(2.0 * np.log(2.0)))
        d = x * np.cos(theta) + y * np.sin(theta) - rho
        h = h + height * np.exp(-d * d / (2.0 * sigma * sigma))
    return h


def aperture_field(ap: Aperture, inst: Instance, j0: int = 0, j1: Optional[int] = None) -> np.ndarray:
    """Aperture transmittance t * exp(i phi) on rows j0..j1-1 (complex, rows x N)."""
    j1 = ap.N if j1 is None else j1
    if ap.levels >= 2:
        L = int(ap.levels)
        t = np.where(disc_mask(ap, j0, j1), np.exp(-2j * np.pi * phase_level(ap, j0, j1) / L), 0.0)
    else:
        t = zone_mask(ap, j0, j1).astype(np.complex128)
    if inst.creases is not None and len(inst.creases):
        x = aperture_coords(ap)
        y = x[j0:j1]
        h = crease_height(x[None, :], y[:, None], inst.creases)
        t = t * np.exp(2j * np.pi * h / inst.lam)
    return t


def output_factor(ap: Aperture, inst: Instance) -> np.ndarray:
    """exp(ikz)/(i lambda z) exp(i pi (x'^2 + y'^2)/(lambda z)) dx^2 on the ROI (Eq. 2)."""
    r = resolve(ap, inst)
    lz = r["lam"] * r["z"]
    xq = roi_coords(inst.M, inst.x0, r["dx_out"])
    yp = roi_coords(inst.M, inst.y0, r["dx_out"])
    kz = 2.0 * np.pi * np.mod(r["z"] / r["lam"], 1.0)
    chirp = np.exp(1j * np.pi * (yp[:, None] ** 2 + xq[None, :] ** 2) / lz)
    return np.exp(1j * kz) / (1j * lz) * chirp * r["dx"] ** 2


def fresnel_direct(ap: Aperture, inst: Instance) -> np.ndarray:
    """Riemann sum of Eq. 1 on the sample grid, one output sample at a time.

    U(x', y') = e^{ikz}/(i lambda z) sum_{j,i} U0_ji exp{i k/(2z)[(x'-x_i)^2 + (y'-y_j)^2]} dx^2.
    Tiny grids only (the cost is N^2 M^2).
    """
    r = resolve(ap, inst)
    lz = r["lam"] * r["z"]
    x = aperture_coords(ap)
    U0 = aperture_field(ap, inst)
    xq = roi_coords(inst.M, inst.x0, r["dx_out"])
    yp = roi_coords(inst.M, inst.y0, r["dx_out"])
    kz = 2.0 * np.pi * np.mod(r["z"] / r["lam"], 1.0)
    pref = np.exp(1j * kz) / (1j * lz) * r["dx"] ** 2
    U = np.empty((inst.M, inst.M), dtype=np.complex128)
    for p in range(inst.M):
        ey = np.exp(1j * np.pi * (yp[p] - x) ** 2 / lz)           # over rows j
        for q in range(inst.M):
            ex = np.exp(1j * np.pi * (xq[q] - x) ** 2 / lz)       # over columns i
            U[p, q] = pref * np.sum(U0 * ey[:, None] * ex[None, :])
    return U


def czt_direct(x: np.ndarray, M: int, w: float, a: float) -> np.ndarray:
    """Chirp-z transform by its definition (Eq. 9), along the last axis.

    X[m] = sum_n x[n] A^{-n} W^{mn},  A = exp(2 pi i a),  W = exp(-2 pi i w).
    """
    n = np.arange(x.shape[-1], dtype=np.float64)
    m = np.arange(M, dtype=np.float64)
    kern = np.exp(-2j * np.pi * (a * n[:, None] + w * m[None, :] * n[:, None]))
    return x @ kern


def czt_bluestein(x: np.ndarray, M: int, w: float, a: float) -> np.ndarray:
    """Chirp-z transform (Eq. 9) through Bluestein's identity, along the last axis.

    With mn = (n^2 + m^2 - (m-n)^2)/2:
      y[n] = x[n] A^{-n} W^{n^2/2},   v[k] = W^{-k^2/2} for k = -(N-1) .. M-1,
      X[m] = W^{m^2/2} (y * v)[m],
    the linear convolution taken by FFT of length L >= N + M - 1.
    A = exp(2 pi i a), W = exp(-2 pi i w).
    """
    Nn = x.shape[-1]
    L = sfft.next_fast_len(Nn + M - 1)
    n = np.arange(Nn, dtype=np.float64)
    m = np.arange(M, dtype=np.float64)
    y = x * np.exp(-2j * np.pi * (a * n + 0.5 * w * n * n))     # A^{-n} W^{n^2/2}
    k = np.arange(-(Nn - 1), M, dtype=np.float64)
    v = np.exp(1j * np.pi * w * k * k)                            # W^{-k^2/2}
    # circular layout: index 0 holds k = 0, negative k wrap to the end
    vc = np.zeros(L, dtype=np.complex128)
    vc[:M] = v[Nn - 1:]
    vc[L - (Nn - 1):] = v[:Nn - 1]
    Y = sfft.fft(y, n=L, axis=-1)
    conv = sfft.ifft(Y * sfft.fft(vc), axis=-1)[..., :M]
    return np.exp(2j * np.pi * (-0.5 * w * m * m)) * conv        # W^{m^2/2}


def _axis_czt(g: np.ndarray, xs: float, dx: float, xo: np.ndarray, lz: float,
              method: str) -> np.ndarray:
    """sum_n g[n] exp(-2 pi i x_n x'_m / (lambda z)) along the last axis.

    x_n = xs + n dx, x'_m = xo[m] = xo[0] + m dx_out.  Eq. 10 identifies
    W = exp(-2 pi i dx_out dx / (lambda z)), A = exp(2 pi i x'_0 dx / (lambda z));
    the remaining factor exp(-2 pi i xs x'_m / (lambda z)) moves the origin.
    """
    M = xo.shape[0]
    dx_out = xo[1] - xo[0] if M > 1 else 1.0
    if method == "dft":
        xn = xs + dx * np.arange(g.shape[-1], dtype=np.float64)
        return g @ np.exp(-2j * np.pi * np.outer(xn, xo) / lz)
    w = dx_out * dx / lz
    a = xo[0] * dx / lz
    czt = czt_bluestein if method == "bluestein" else czt_direct
    return czt(g, M, w, a) * np.exp(-2j * np.pi * xs * xo / lz)


def propagate(ap: Aperture, inst: Instance, method: str = "bluestein",
              rows: Optional[tuple] = None, stripe: int = 1024,
              with_output_factor: bool = True, field_fn=None) -> np.ndarray:
    """Complex focal-plane field U on the M x M ROI, [y = p][x = q] (Eq. 2).

    Separable evaluation (Sec. 2.6): for each stripe of aperture rows the row
    pass transforms every row onto the M ROI columns, the column pass transforms
    the stripe's columns onto the M ROI rows, and the stripes are summed.
    ``rows=(j0, j1)`` restricts the aperture sum to rows j0..j1-1.
    ``method`` is "bluestein" (Eq. 9 by Bluestein), "dft" (matrix products) or
    "czt_direct" (Eq. 9 by definition).  ``field_fn(j0, j1)``, when given,
    replaces the zone-plate transmittance of rows j0..j1-1 (used by the
    invariance tests).
    """
    r = resolve(ap, inst)
    lz = r["lam"] * r["z"]
    x = aperture_coords(ap)
    xs = x[0]
    xq = roi_coords(inst.M, inst.x0, r["dx_out"])
    yp = roi_coords(inst.M, inst.y0, r["dx_out"])
    chirp = np.exp(1j * np.pi * x * x / lz)          # e^{i pi x^2/(lambda z)}, same for y
    j0, j1 = (0, ap.N) if rows is None else rows
    acc = np.zeros((inst.M, inst.M), dtype=np.complex128)
    for s0 in range(j0, j1, stripe):
        s1 = min(s0 + stripe, j1)
        t = aperture_field(ap, inst, s0, s1) if field_fn is None else field_fn(s0, s1)
        u = t * chirp[None, :] * chirp[s0:s1, None]
        T = _axis_czt(u, xs, ap.dx, xq, lz, method)                 # (rows, M): row pass
        # column pass over the stripe's rows y_j = xs + j dx
        acc += _axis_czt(T.T, x[s0], ap.dx, yp, lz, method).T       # (M_p, M_q)
    if with_output_factor:
        acc = acc * output_factor(ap, inst)
    return acc


def intensity(U: np.ndarray) -> np.ndarray:
    return (U.real ** 2 + U.imag ** 2)


def fwhm_1d(row: np.ndarray, frac: float = 0.5) -> float:
    """Full width at half maximum of a sampled profile, in samples (with
    ``frac``: the full width at that fraction of the maximum).

    Not-a-knot cubic spline through all samples; the spline peak is the largest
    spline value on the two sample intervals next to the brightest sample; the
    crossings of half that value are found by bisection on the sample intervals
    that bracket them.  NaN if a crossing falls outside the profile.
    """
    row = np.asarray(row, dtype=np.float64)
    M = row.shape[0]
    k = int(np.argmax(row))
    if k == 0 or k == M - 1:
        return float("nan")
    cs = CubicSpline(np.arange(M, dtype=np.float64), row, bc_type="not-a-knot")
    cand = [float(k)]
    for lo in (k - 1, k):
        c = cs.c[:, lo]                                 # c0 t^3 + c1 t^2 + c2 t + c3
        for t in np.roots([3.0 * c[0], 2.0 * c[1], c[2]]):
            if abs(t.imag) == 0.0 and 0.0 <= t.real <= 1.0:
                cand.append(lo + float(t.real))
    peak = max(float(cs(t)) for t in cand)
    half = frac * peak
    left = k
    while left >= 0 and row[left] >= half:
        left -= 1
    right = k
    while right < M and row[right] >= half:
        right += 1
    if left < 0 or right >= M:
        return float("nan")

    def bisect(lo: float, hi: float, rising: bool) -> float:
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid == lo or mid == hi:
                break
            above = float(cs(mid)) >= half
            if above == rising:
                hi = mid
            else:
                lo = mid
        return 0.5 * (lo + hi)

    xl = bisect(float(left), float(left + 1), True)
    xr = bisect(float(right - 1), float(right), False)
    return xr - xl


def mtf_half_cut(I: np.ndarray, dx_out: float, nu_cut: float) -> float:
    """MTF at nu_cut/2: radial mean of |FFT2(I)|/|FFT2(I)|(0), linear interpolation."""
    M = I.shape[0]
    F = np.abs(np.fft.fft2(I))
    F = F / F[0, 0]
    k = np.fft.fftfreq(M) * M
    rb = np.rint(np.hypot(k[:, None], k[None, :])).astype(np.int64)
    nb = int(rb.max()) + 1
    sums = np.bincount(rb.ravel(), weights=F.ravel(), minlength=nb)
    cnt = np.bincount(rb.ravel(), minlength=nb)
    radial = sums / np.maximum(cnt, 1)
    t = 0.5 * nu_cut * M * dx_out                      # (nu_cut/2) / dnu
    return float(np.interp(t, np.arange(nb, dtype=np.float64), radial))


def metrics(U_or_I: np.ndarray, ap: Aperture, inst: Instance, p_in_count: Optional[int] = None) -> dict:
    """FWHM (x, y) [m], main-lobe DE, MTF(nu_cut/2), Strehl, peak, P_in, P_lobe."""
    I = intensity(U_or_I) if np.iscomplexobj(U_or_I) else np.asarray(U_or_I, dtype=np.float64)
    r = resolve(ap, inst)
    lz = r["lam"] * r["z"]
    M = inst.M
    dxo = r["dx_out"]
    pk = int(np.argmax(I))
    p, q = divmod(pk, M)
    fwhm_x = fwhm_1d(I[p, :]) * dxo
    fwhm_y = fwhm_1d(I[:, q]) * dxo
    rel = (np.arange(M, dtype=np.float64) - 0.5 * M) * dxo      # positions about the ROI centre
    r2 = rel[:, None] ** 2 + rel[None, :] ** 2
    r_null = J11 / np.pi * lz / ap.D
    p_lobe = float(np.sum(I[r2 <= r_null * r_null])) * dxo * dxo
    cnt = incident_count(ap) if p_in_count is None else p_in_count
    p_in = cnt * ap.dx * ap.dx
    R = 0.5 * ap.D
    return dict(fwhm_x=fwhm_x, fwhm_y=fwhm_y, de=p_lobe / p_in,
                mtf_half_cut=mtf_half_cut(I, dxo, ap.D / lz),
                strehl=float(I.max()) / (np.pi * R * R / lz) ** 2,
                i_peak=float(I.max()), p_in=p_in, p_lobe=p_lobe)


# ----------------------------------------------------------------------------
# Continuous, axisymmetric reference (1-D radial / Hankel form of Eq. 2)
# ----------------------------------------------------------------------------

def _open_zone_intervals(ap: Aperture, s_max: float):
    """Intervals of s = r^2 with constant transmission, clipped at s_max, and
    that transmission.  Amplitude plate: the open zones
    [n lambda0 f0, (n+1) lambda0 f0] for odd n (even n when the centre is open),
    transmission 1.  L-level phase plate: the steps
    [m, m+1] * 2 lambda0 f0 / L, transmission exp(-2 pi i (m mod L) / L)."""
    a = ap.lambda0 * ap.f0
    if ap.levels >= 2:
        L = int(ap.levels)
        step = 2.0 * a / L
        nz = int(np.ceil(s_max / step)) + 1
        m = np.arange(nz)
        lo = m * step
        hi = np.minimum((m + 1) * step, s_max)
        ok = lo < hi
        return lo[ok], hi[ok], np.exp(-2j * np.pi * (m[ok] % L) / L)
    nz = int(np.ceil(s_max / a)) + 1
    n = np.arange(nz)
    keep = (n % 2 == 1) if not ap.centre_open else (n % 2 == 0)
    lo = n[keep] * a
    hi = np.minimum((n[keep] + 1) * a, s_max)
    ok = lo < hi
    return lo[ok], hi[ok], np.ones(int(ok.sum()), dtype=np.complex128)


def hankel_field(rho: np.ndarray, ap: Aperture, lam: float, z: float, nodes: int = 16) -> np.ndarray:
    """(pi/(lambda z)) int_0^{R^2} t(s) e^{i pi s/(lambda z)} J0(2 pi rho sqrt(s)/(lambda z)) ds.

    Its squared modulus is the focal intensity of the continuous aperture, in
    the same units as |U|^2 from ``propagate``.  Gauss-Legendre per open zone.
    """
    lz = lam * z
    lo, hi, tz = _open_zone_intervals(ap, (0.5 * ap.D) ** 2)
    t, wts = np.polynomial.legendre.leggauss(nodes)
    half = 0.5 * (hi - lo)
    s = (0.5 * (hi + lo))[:, None] + half[:, None] * t[None, :]
    wt = (tz[:, None] * half[:, None] * wts[None, :]).ravel()
    s = s.ravel()
    ph = np.exp(1j * np.pi * s / lz) * wt
    rho = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    out = np.empty(rho.shape, dtype=np.complex128)
    sq = np.sqrt(s)
    for idx, rv in np.ndenumerate(rho):
        out[idx] = np.sum(ph * special.j0(2.0 * np.pi * rv * sq / lz))
    return np.pi / lz * out


def hankel_intensity(rho, ap: Aperture, lam: float, z: float, nodes: int = 16) -> np.ndarray:
    return np.abs(hankel_field(rho, ap, lam, z, nodes)) ** 2


def hankel_metrics(ap: Aperture, lam: Optional[float] = None, z: Optional[float] = None,
                   nodes: int = 16, lobe_nodes: int = 96) -> dict:
    """FWHM [m] and main-lobe DE (power inside r_null over pi R^2) of the
    continuous aperture, from the radial integral."""
    from scipy.optimize import brentq
    lam = ap.lambda0 if lam is None else lam
    z = ap.f0 * ap.lambda0 / lam if z is None else z
    lz = lam * z
    i0 = float(hankel_intensity(0.0, ap, lam, z, nodes)[0])
    r_null = J11 / np.pi * lz / ap.D
    rho_half = brentq(lambda rr: float(hankel_intensity(rr, ap, lam, z, nodes)[0]) - 0.5 * i0,
                      1e-3 * r_null, r_null, xtol=1e-15 * r_null, rtol=1e-14)
    t, wts = np.polynomial.legendre.leggauss(lobe_nodes)
    rr = 0.5 * r_null * (t + 1.0)
    Ir = hankel_intensity(rr, ap, lam, z, nodes)
    p_lobe = float(np.sum(0.5 * r_null * wts * Ir * 2.0 * np.pi * rr))
    R = 0.5 * ap.D
    return dict(fwhm=2.0 * rho_half, de=p_lobe / (np.pi * R * R), i0=i0,
                strehl=i0 / (np.pi * R * R / lz) ** 2)


def on_axis_closed_form(ap: Aperture, lam: Optional[float] = None, z: Optional[float] = None) -> float:
    """On-axis intensity of the continuous aperture in closed form.

    With rho = 0 the radial integrand is t(s) e^{i pi s/(lambda z)}, whose
    integral over an open zone [s_lo, s_hi] is (lambda z/(i pi))(e^{i pi b_hi} - e^{i pi b_lo}),
    b = s/(lambda z); hence I(0) = |sum_zones (e^{i pi b_hi} - e^{i pi b_lo})|^2.
    """
    lam = ap.lambda0 if lam is None else lam
    z = ap.f0 * ap.lambda0 / lam if z is None else z
    lz = lam * z
    lo, hi, tz = _open_zone_intervals(ap, (0.5 * ap.D) ** 2)
    s = np.sum(tz * (np.exp(1j * np.pi * hi / lz) - np.exp(1j * np.pi * lo / lz)))
    return float(abs(s) ** 2)


def zone_count_exact(D: float, lam: float, f: float) -> float:
    """Real root n of (lambda^2/4) n^2 + lambda f n = R^2 (Eq. 3 at r_n = D/2)."""
    R = 0.5 * D
    a, b, c = 0.25 * lam * lam, lam * f, -R * R
    return (-b + np.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)


def v8_grid(D: float, f: float, lam0: float, L: int, s_samp: int = 4):
    """Grid rule of the revised engine (Fig. 18 stage 1): Lambda_edge = lambda0 f / R,
    dx_in = Lambda_edge / (S_samp max(L, 2)), Nx = ceil(D / dx_in) forced odd."""
    lam_edge = lam0 * f / (0.5 * D)
    dx = lam_edge / (s_samp * max(L, 2))
    nx = int(np.ceil(D / dx))
    if nx % 2 == 0:
        nx += 1
    return dx, nx
