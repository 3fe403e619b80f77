"""GPU: fzp_fwhm_batch (the surrogate gate's FWHM reading and conditioning
numbers) against the oracle's metric extractor on the same float32
log-intensity maps: the FWHM along the brightest sample's row and along the
brighter neighbouring row (``fzp_oracle.fwhm_1d``, the same not-a-knot spline
and bisection), the level sensitivity from widths at 0.45 and 0.55 of the
peak, the second-spot ratio and the row gap.  Maps: the physics prior of
seeded creased pupils (aberrated spots), one with a planted second spot, and
one whose peak sits on the ROI edge row.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2609_01978_amd import _lib as L  # noqa: E402
from oracle import fzp_oracle as F  # noqa: E402
from oracle import prior_oracle as PR  # noqa: E402
from fzp_inputs import surrogate_draws  # noqa: E402

pytestmark = pytest.mark.gpu
FLOOR, DELTA = 1e-2, 0.05


def maps():
    M, D = 96, 10e-3
    cr, lam = surrogate_draws(5, 5, D, 632.8e-9)
    out = [PR.prior_intensity(D, M, cr[k], lam[k], Np=64, ss=2) for k in range(5)]
    I = out[0].copy()
    p, q = np.unravel_index(np.argmax(I), I.shape)
    I[(p + 30) % M, (q + 25) % M] = 0.6 * I.max()             # a planted second spot
    out.append(I)
    I = np.roll(out[1], M - 1 - int(np.unravel_index(np.argmax(out[1]), out[1].shape)[0]), axis=0)  # peak on the last row
    out.append(I)
    return M, np.stack([np.log(I + FLOOR) for I in out]).astype(np.float32)


def reference(y32, M, excl):
    I = (np.exp(y32.astype(np.float64)) - FLOOR).reshape(M, M)
    k = int(np.argmax(y32))                                   # first index on ties, as the kernel
    p, q = divmod(k, M)
    w = F.fwhm_1d(I[p])
    cond = (F.fwhm_1d(I[p], 0.5 - DELTA) - F.fwhm_1d(I[p], 0.5 + DELTA)) / (2 * DELTA * w)
    rr, cc = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    far = (rr - p) ** 2 + (cc - q) ** 2 > excl * excl
    ratio = (np.exp(float(y32.reshape(M, M)[far].max())) - FLOOR) / I[p, q] if far.any() else 0.0
    up = y32.reshape(M, M)[p - 1].max() if p > 0 else -np.inf
    dn = y32.reshape(M, M)[p + 1].max() if p < M - 1 else -np.inf
    pn = p - 1 if up >= dn else p + 1
    yn = max(up, dn)
    gap = 1.0 - (np.exp(float(yn)) - FLOOR) / I[p, q]
    return w, cond, ratio, gap, F.fwhm_1d(I[pn])


def test_fwhm_batch_matches_oracle():
    M, Y = maps()
    excl = 2.0 * 1.22 * M / 16.0
    out = L.fwhm_batch(torch.from_numpy(Y.reshape(len(Y), -1)).cuda(), M, FLOOR, DELTA, excl).cpu().numpy()
    for b in range(len(Y)):
        ref = reference(Y[b].ravel(), M, excl)
        print(f"[gpu-fwhm] map {b}: gpu {np.round(out[b], 6)} ref {np.round(ref, 6)}", flush=True)
        assert abs(out[b, 0] / ref[0] - 1) < 1e-9
        assert abs(out[b, 1] - ref[1]) < 1e-6 * max(1.0, abs(ref[1]))
        assert abs(out[b, 2] - ref[2]) < 1e-12 + 1e-9 * ref[2]
        assert abs(out[b, 3] - ref[3]) < 1e-9
        assert abs(out[b, 4] / ref[4] - 1) < 1e-9
    assert out[5, 2] > 0.55                                   # the planted spot is seen
    assert out[6, 3] >= 0.0                                   # edge row: the one neighbour is used
