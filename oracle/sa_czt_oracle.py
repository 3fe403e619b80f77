"""FP64 CPU oracle for the non-paraxial variant of the zone-plate propagation:
the semi-analytical chirp-z transform (SA-CZT, Sec. 3.6 and Fig. 5), i.e. the
exact angular-spectrum propagation of the semi-analytical Fourier transform
(Sec. 3.4, Fig. 3) with its final FFT replaced by a chirp-z zoom onto the
region of interest, applied to a binary-amplitude zone plate whose radii carry
the spherical sag term of Eq. 3.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this module.  The GPU
library never calls it and shares no code with it.

Steps, in the paper's order (plain NumPy in float64 / complex128):

1. grids: the aperture samples ``x_i = (i - (N-1)/2) dx`` (``dx = D/N``) are
   centred in a zero-padded square grid of ``Np`` samples per side at the same
   pitch (pad factor 1.5, see ``pad_size``);
2. the mask: zone index ``n = floor(n_exact)`` of the exact radii of Eq. 3,
   ``r_n^2 = n lambda0 f0 + (n lambda0 / 2)^2``, i.e. the real root
   ``n_exact = (2/lambda0)(sqrt(f0^2 + r^2) - f0)`` written without the
   cancellation as ``c2 q / (sqrt(1 + q) + 1)``, ``q = K c1``,
   ``c1 = dx^2 / (4 f0^2)``, ``c2 = 2 f0 / lambda0`` (``K`` the exact integer
   ``4 r^2 / dx^2``); open where ``n`` is odd inside the disc; no input chirp;
3. the exact transfer function ``exp(i k_z z)``, ``k_z(K) = sqrt(k0^2 - K^2)``,
   is split into a quadratic fit ``c k_max + d K^2 / k_max`` and the remainder
   ``h(K) = k_z - c k_max - d K^2 / k_max``; the remainder is applied to the
   2-D FFT of the padded mask and transformed back (evanescent ``K^2 > k0^2``
   set to zero), giving the field ``U1`` on the padded grid;
4. the quadratic part is a Fresnel-type transform with ``Z = 4 pi |d| z /
   k_max`` in place of ``lambda z`` (the output sample spacing of the zoom in
   frequency is ``dx_out k_max / (4 pi |d| z)``): the chirp
   ``exp(i pi u^2 / Z)``, the chirp-z transform along the rows and then the
   columns onto the ROI (times ``dx^2``), and the prefactor
   ``exp(i c k_max z) / (i Z) exp(i pi (x'^2 + y'^2) / Z)``.

Readings where the paper is silent or garbled (listed in the design notes):
``k_max = 2 k0 / 3`` with ``c, d`` from the two-point fit that matches
``k_z`` at ``K = 0`` and ``K = k_max`` (``c = k0 / k_max``,
``d = (sqrt(k0^2 - k_max^2) - k0) / k_max``); the padded size is the smallest
``2^a 3^b 5^c >= 1.5 N`` with the parity of N (so the aperture sits on the
padded grid's own sample positions); the ROI grid, wavelength and focus
conventions are those of the paraxial oracle (``fzp_oracle.resolve``).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import fzp_oracle as F

__all__ = ["pad_size", "fit_constants", "zone_index_eq3", "zone_mask_eq3", "padded_aperture",
           "angular_spectrum_step", "zoom", "sa_czt", "rs_on_axis_annuli"]


def _smooth(m: int) -> bool:
    for p in (2, 3, 5):
        while m % p == 0:
            m //= p
    return m == 1


def pad_size(N: int, pad: float = 1.5) -> int:
    """Smallest Np >= pad * N of the form 2^a 3^b 5^c with Np = N (mod 2)."""
    m = int(np.ceil(pad * N))
    while not (_smooth(m) and (m - N) % 2 == 0):
        m += 1
    return m


def fit_constants(lam: float, k_fit: float = 2.0 / 3.0):
    """(k0, k_max, c, d): k_max = k_fit k0 and the quadratic c k_max + d K^2 / k_max
    through k_z(0) = k0 and k_z(k_max) = sqrt(k0^2 - k_max^2)."""
    k0 = 2.0 * np.pi / lam
    kmax = k_fit * k0
    c = k0 / kmax
    d = (np.sqrt(k0 * k0 - kmax * kmax) - k0) / kmax
    return k0, kmax, c, d


def zone_index_eq3(ap: F.Aperture, j0: int = 0, j1: Optional[int] = None) -> np.ndarray:
    """floor(n_exact) of Eq. 3 for rows j0..j1-1 (int64, rows x N)."""
    j1 = ap.N if j1 is None else j1
    N = ap.N
    ci = 2 * np.arange(N, dtype=np.int64) - (N - 1)
    cj = 2 * np.arange(j0, j1, dtype=np.int64) - (N - 1)
    K = (cj[:, None] ** 2 + ci[None, :] ** 2).astype(np.float64)   # exact integers
    c1 = ap.dx * ap.dx / (4.0 * ap.f0 * ap.f0)
    c2 = 2.0 * ap.f0 / ap.lambda0
    q = K * c1                                                      # r^2 / f0^2
    n_exact = c2 * (q / (np.sqrt(1.0 + q) + 1.0))
    return np.floor(n_exact).astype(np.int64)


def zone_mask_eq3(ap: F.Aperture, j0: int = 0, j1: Optional[int] = None) -> np.ndarray:
    """Binary mask with the sag-corrected radii of Eq. 3: open where the zone
    index is odd (even with centre_open) inside the disc K <= K_max."""
    n = zone_index_eq3(ap, j0, j1)
    odd = (n % 2) == 1
    if ap.centre_open:
        odd = ~odd
    return F.disc_mask(ap, j0, j1) & odd


def padded_aperture(ap: F.Aperture, radii: str = "eq3", pad: float = 1.5,
                    inst: Optional[F.Instance] = None) -> np.ndarray:
    """The mask (radii 'eq3', 'paraxial' or 'disc' for a clear aperture) centred
    in the zero-padded Np x Np grid (complex128), times the membrane phase
    screen exp(2 pi i h / lambda) of the instance's creases when it has any (the
    thin-screen deformation model of the paraxial oracle)."""
    Np = pad_size(ap.N, pad)
    off = (Np - ap.N) // 2
    if radii == "eq3":
        m = zone_mask_eq3(ap)
    elif radii == "paraxial":
        m = F.zone_mask(ap)
    elif radii == "disc":
        m = F.disc_mask(ap)
    else:
        raise ValueError(radii)
    t = m.astype(np.complex128)
    if inst is not None and inst.creases is not None and len(inst.creases):
        x = F.aperture_coords(ap)
        t = t * np.exp(2j * np.pi * F.crease_height(x[None, :], x[:, None], inst.creases) / inst.lam)
    U0 = np.zeros((Np, Np), dtype=np.complex128)
    U0[off:off + ap.N, off:off + ap.N] = t
    return U0


def angular_spectrum_step(U0: np.ndarray, dx: float, lam: float, z: float, k_fit: float = 2.0 / 3.0):
    """U1 = IFFT2{ FFT2{U0} exp(i h(K) z) } with h(K) = k_z - c k_max - d K^2 / k_max,
    k_z = sqrt(k0^2 - K^2), evanescent frequencies set to zero."""
    k0, kmax, c, d = fit_constants(lam, k_fit)
    Np = U0.shape[0]
    nu = np.fft.fftfreq(Np, d=dx)
    K2 = (2.0 * np.pi) ** 2 * (nu[:, None] ** 2 + nu[None, :] ** 2)
    prop = K2 <= k0 * k0
    kz = np.sqrt(np.where(prop, k0 * k0 - K2, 0.0))
    h = kz - c * kmax - d * K2 / kmax
    H = np.where(prop, np.exp(1j * h * z), 0.0)
    return np.fft.ifft2(np.fft.fft2(U0) * H)


def zoom(U1: np.ndarray, dx: float, Z: float, xq: np.ndarray, yp: np.ndarray, method: str = "bluestein"):
    """sum_{j,i} U1[j,i] e^{i pi (u_i^2 + v_j^2)/Z} e^{-2 pi i (x'_q u_i + y'_p v_j)/Z} dx^2 on
    the ROI [p][q]: the chirp, then the chirp-z transform along the rows, then
    along the columns (Eq. 9 with the Eq. 10 parameters, Z in place of lambda z)."""
    Np = U1.shape[0]
    u = (np.arange(Np, dtype=np.float64) - 0.5 * (Np - 1)) * dx
    ch = np.exp(1j * np.pi * u * u / Z)
    g = U1 * ch[None, :] * ch[:, None]
    T = F._axis_czt(g, u[0], dx, xq, Z, method)                 # (Np rows, M_q)
    return F._axis_czt(T.T, u[0], dx, yp, Z, method).T * dx * dx


def sa_czt(ap: F.Aperture, inst: F.Instance, radii: str = "eq3", pad: float = 1.5, k_fit: float = 2.0 / 3.0,
           method: str = "bluestein") -> np.ndarray:
    """Complex focal-plane field U on the M x M ROI [y = p][x = q] by the SA-CZT."""
    r = F.resolve(ap, inst)
    lam, z = r["lam"], r["z"]
    k0, kmax, c, d = fit_constants(lam, k_fit)
    U0 = padded_aperture(ap, radii, pad, inst)
    U1 = angular_spectrum_step(U0, ap.dx, lam, z, k_fit)
    Z = 4.0 * np.pi * abs(d) * z / kmax
    xq = F.roi_coords(inst.M, inst.x0, r["dx_out"])
    yp = F.roi_coords(inst.M, inst.y0, r["dx_out"])
    acc = zoom(U1, ap.dx, Z, xq, yp, method)
    pre = np.exp(1j * np.mod(c * kmax * z, 2.0 * np.pi)) / (1j * Z)
    return pre * np.exp(1j * np.pi * (yp[:, None] ** 2 + xq[None, :] ** 2) / Z) * acc


def rs_on_axis_annuli(edges, lam: float, z: float) -> complex:
    """On-axis Rayleigh-Sommerfeld (first kind) field of a unit plane wave through
    clear annuli [a, b): each contributes (z/rho_a) e^{ik rho_a} - (z/rho_b) e^{ik rho_b},
    rho = sqrt(z^2 + r^2) (closed form; a = 0 gives e^{ikz} for its first term)."""
    k = 2.0 * np.pi / lam
    out = 0j
    for a, b in edges:
        ra, rb = np.hypot(z, a), np.hypot(z, b)
        out += z / ra * np.exp(1j * k * ra) - z / rb * np.exp(1j * k * rb)
    return complex(out)
