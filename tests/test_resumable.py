"""Resumable propagation through a checkpoint file (fzp_propagate_resumable).

CPU: a malformed file and a checkpoint of another plan are refused before any
device work, and the file is left in place.  GPU: a run cut into time slices,
resumed by a fresh plan object, ends bit for bit on the ROI of one
fzp_propagate_roi call, and the finished run removes its file.
"""
import ctypes
import os
import struct

import numpy as np
import pytest

import paper_2609_01978_amd as P
from paper_2609_01978_amd import _lib as L

LAM0 = 632.8e-9
AP = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=3000)


def _plan(path="fp64", **kw):
    return P.Plan(AP, [dict(lam=LAM0, M=64), dict(lam=560e-9, M=48)], path=path, allow_undersampled=True,
                  chunk_rows=512, **kw)


def _call(plan, fname):
    lib = plan._lib
    nxt = ctypes.c_int64(-1)
    dummy = ctypes.c_void_p(256)   # never dereferenced: the file is refused first
    st = lib.fzp_propagate_resumable(plan._h, dummy, dummy, os.fsencode(str(fname)), 0, 0, 0, ctypes.byref(nxt),
                                     None)
    return st, lib.fzp_last_error().decode()


def test_malformed_checkpoint_is_refused(tmp_path):
    f = tmp_path / "ck.bin"
    f.write_bytes(b"not a checkpoint")
    st, msg = _call(_plan(), f)
    assert st == L.FZP_E_INVAL and "malformed" in msg
    assert f.read_bytes() == b"not a checkpoint"


def test_checkpoint_of_another_plan_is_refused(tmp_path):
    plan = _plan()
    n = plan.roi_elements
    f = tmp_path / "ck.bin"
    f.write_bytes(b"FZPCKPT1" + struct.pack("<Qqq", 12345, n, 512) + bytes(16 * n))
    st, msg = _call(plan, f)
    assert st == L.FZP_E_INVAL and "another plan" in msg
    assert f.exists()


@pytest.mark.gpu
@pytest.mark.parametrize("path,lanes", [("fp64", 2), ("split", 1)])
def test_time_sliced_run_matches_one_call(tmp_path, path, lanes):
    torch = pytest.importorskip("torch")
    ref_plan = _plan(path, lanes=lanes)
    ws, roi = ref_plan.alloc()
    ref_plan.propagate(ws, roi)
    torch.cuda.synchronize()
    ref = roi.cpu().numpy().copy()
    f = str(tmp_path / "run.ckpt")
    nxt = _plan(path, lanes=lanes).propagate_resumable(ws, roi, f, rows_per_checkpoint=600, max_rows=1000)
    assert nxt == 1024 and os.path.exists(f)
    roi.zero_()  # the next slice restores the ROI from the file
    nxt = _plan(path, lanes=lanes).propagate_resumable(ws, roi, f, rows_per_checkpoint=600, max_rows=1)
    assert nxt == 2048 and os.path.exists(f)
    nxt = _plan(path, lanes=lanes).propagate_resumable(ws, roi, f, rows_per_checkpoint=600)
    torch.cuda.synchronize()
    assert nxt == AP["N"] and not os.path.exists(f)
    assert np.array_equal(roi.cpu().numpy(), ref)


@pytest.mark.gpu
def test_finished_checkpoint_restores_the_roi(tmp_path):
    """keep=True leaves the finished checkpoint; a later call restores the ROI
    from it without propagating and then removes it."""
    torch = pytest.importorskip("torch")
    plan = _plan("fp64")
    ws, roi = plan.alloc()
    f = str(tmp_path / "done.ckpt")
    assert plan.propagate_resumable(ws, roi, f, keep=True) == AP["N"] and os.path.exists(f)
    torch.cuda.synchronize()
    ref = roi.cpu().numpy().copy()
    roi.fill_(7.0)
    assert _plan("fp64").propagate_resumable(ws, roi, f) == AP["N"]
    torch.cuda.synchronize()
    assert np.array_equal(roi.cpu().numpy(), ref) and not os.path.exists(f)
