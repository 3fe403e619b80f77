"""ctypes binding of ``libfzp.so`` (the C ABI declared in ``include/fzp.h``).

Argument marshalling only: every step of the propagation and of the metric
extraction runs in the library's HIP kernels.  PyTorch supplies device memory
and the current HIP stream.  The library must be built
(``python -m paper_2609_01978_amd.build``); the first call that needs it
raises ImportError when it is missing (there is no other implementation to
fall back to).  It is loaded on first use so that the build step itself can
import the package.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FZP_LIBRARY names another build of the same library (e.g. the host-sanitized
# one of build.py --host-sanitize); the default is the in-tree build
LIB_PATH = os.environ.get("FZP_LIBRARY") or os.path.join(_HERE, "libfzp.so")

FZP_OK = 0
FZP_E_INVAL = -1
FZP_E_SAMPLING = -2
FZP_E_NOMEM = -3
FZP_E_DEVICE = -4
FZP_E_UNSUPPORTED = -5
STATUS_NAMES = {0: "FZP_OK", -1: "FZP_E_INVAL", -2: "FZP_E_SAMPLING", -3: "FZP_E_NOMEM",
                -4: "FZP_E_DEVICE", -5: "FZP_E_UNSUPPORTED"}

PATH_FP64_BLUESTEIN = 0
PATH_SPLIT_BF16 = 1
PATH_AUTO = 2
PATH_SA_CZT = 3
FLAG_ALLOW_UNDERSAMPLED = 1
FLAG_BIN_TILE_256 = 2
FLAG_BIN_SHALLOW = 4
FLAG_BIN_PREFETCH = 8
FLAG_OVERLAP_OPERAND = 16
FLAG_BIN_DEEP = 32
FLAG_CPLX_TILE_128 = 128
FLAG_CPLX_TILE_DUAL = 256
FLAG_PARAXIAL_RADII = 64
FLAG_SPLIT_INT8 = 1024
STATIC_SCRATCH_BYTES = 64 << 20   # FZP_STATIC_SCRATCH_BYTES

EXPORTED = [
    "fzp_plan", "fzp_plan_workspace_size", "fzp_roi_elements", "fzp_roi_offset", "fzp_prepare",
    "fzp_propagate_roi", "fzp_propagate_roi_static", "fzp_propagate_roi_range", "fzp_propagate_resumable", "fzp_metrics", "fzp_plan_info", "fzp_plan_geometry", "fzp_grid_for_element", "fzp_destroy",
    "fzp_last_error", "fzp_profile_enable", "fzp_profile_read", "fzp_graph_create", "fzp_graph_launch",
    "fzp_graph_destroy", "fzp_autotune", "fzp_mlp_create", "fzp_mlp_info", "fzp_mlp_set_params",
    "fzp_mlp_get_params", "fzp_mlp_forward", "fzp_mlp_backward", "fzp_mlp_train_step", "fzp_mlp_adam_update",
    "fzp_mlp_destroy", "fzp_log_intensity", "fzp_field_from_log_intensity", "fzp_pupil_prior_workspace",
    "fzp_pupil_prior", "fzp_fwhm_batch",
]


class FZPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Aperture(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("f0", ctypes.c_double), ("lambda0", ctypes.c_double),
                ("pitch", ctypes.c_double), ("N", ctypes.c_int64), ("centre_open", ctypes.c_int32),
                ("levels", ctypes.c_int32)]


class Crease(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("offset", ctypes.c_double), ("width", ctypes.c_double),
                ("height", ctypes.c_double)]


class Instance(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("z", ctypes.c_double), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("half_width", ctypes.c_double), ("M", ctypes.c_int32),
                ("n_creases", ctypes.c_int32), ("creases", ctypes.POINTER(Crease))]


class Options(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("stripe_rows", ctypes.c_int32), ("chunk_rows", ctypes.c_int64),
                ("workspace_limit", ctypes.c_uint64), ("flags", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("pad", ctypes.c_double)]


class Geometry(ctypes.Structure):
    _fields_ = [("zones_exact", ctypes.c_double), ("total_zones", ctypes.c_int64), ("padded_n", ctypes.c_int64),
                ("fft_n1", ctypes.c_int32), ("fft_n2", ctypes.c_int32), ("zoom_distance", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class Metrics(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("fwhm_x", "fwhm_y", "de", "mtf_half_cut", "strehl", "i_peak", "p_in", "p_lobe")]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libfzp.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_01978_amd.build`")
    # torch's HIP runtime goes first: it and the library's runtime carry the same
    # soname, so the library then binds to the runtime that owns the device
    # buffers instead of loading a second copy (which sees no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int32
    P = ctypes.c_void_p
    lib.fzp_plan.argtypes = [ctypes.POINTER(Aperture), ctypes.POINTER(Instance), ctypes.c_int32,
                             ctypes.POINTER(Options), ctypes.POINTER(P)]
    lib.fzp_plan.restype = st
    lib.fzp_plan_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.fzp_plan_workspace_size.restype = st
    lib.fzp_roi_elements.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.fzp_roi_elements.restype = st
    lib.fzp_roi_offset.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    lib.fzp_roi_offset.restype = st
    lib.fzp_prepare.argtypes = [P, P, P]
    lib.fzp_prepare.restype = st
    lib.fzp_propagate_roi.argtypes = [P, P, P, P]
    lib.fzp_propagate_roi.restype = st
    lib.fzp_propagate_roi_static.argtypes = [P, P, P]
    lib.fzp_propagate_roi_static.restype = st
    lib.fzp_propagate_roi_range.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, P]
    lib.fzp_propagate_roi_range.restype = st
    lib.fzp_propagate_resumable.argtypes = [P, P, P, ctypes.c_char_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int64), P]
    lib.fzp_propagate_resumable.restype = st
    lib.fzp_metrics.argtypes = [P, P, P, ctypes.POINTER(Metrics), P]
    lib.fzp_metrics.restype = st
    lib.fzp_plan_info.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_double)]
    lib.fzp_plan_info.restype = st
    lib.fzp_grid_for_element.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]
    lib.fzp_grid_for_element.restype = st
    lib.fzp_plan_geometry.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Geometry)]
    lib.fzp_plan_geometry.restype = st
    lib.fzp_profile_enable.argtypes = [P, ctypes.c_int32]
    lib.fzp_profile_enable.restype = st
    lib.fzp_profile_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    lib.fzp_profile_read.restype = st
    lib.fzp_graph_create.argtypes = [P, P, P, ctypes.POINTER(P)]
    lib.fzp_graph_create.restype = st
    lib.fzp_graph_launch.argtypes = [P, P]
    lib.fzp_graph_launch.restype = st
    lib.fzp_graph_destroy.argtypes = [P]
    lib.fzp_graph_destroy.restype = None
    lib.fzp_autotune.argtypes = [P, P, P, P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_double)]
    lib.fzp_autotune.restype = st
    lib.fzp_destroy.argtypes = [P]
    lib.fzp_destroy.restype = None
    i32, i64, f32, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    lib.fzp_mlp_create.argtypes = [i32, i32, i32, i32, ctypes.POINTER(P)]
    lib.fzp_mlp_info.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(i64)]
    lib.fzp_mlp_set_params.argtypes = [P, P, P, P]
    lib.fzp_mlp_get_params.argtypes = [P, P, P, P]
    lib.fzp_mlp_forward.argtypes = [P, P, P, i32, P, P]
    lib.fzp_mlp_backward.argtypes = [P, P, P, P, i32, P, P, P, P, P]
    lib.fzp_mlp_train_step.argtypes = [P, P, P, P, i32, P, f32, P, P]
    lib.fzp_mlp_adam_update.argtypes = [P, P, P, f32, P]
    lib.fzp_log_intensity.argtypes = [P, i64, dbl, dbl, P, P]
    lib.fzp_field_from_log_intensity.argtypes = [P, i64, dbl, dbl, P, P]
    for name in ("fzp_mlp_create", "fzp_mlp_info", "fzp_mlp_set_params", "fzp_mlp_get_params", "fzp_mlp_forward",
                 "fzp_mlp_backward", "fzp_mlp_train_step", "fzp_mlp_adam_update", "fzp_log_intensity",
                 "fzp_field_from_log_intensity"):
        getattr(lib, name).restype = st
    lib.fzp_mlp_destroy.argtypes = [P]
    lib.fzp_mlp_destroy.restype = None
    lib.fzp_pupil_prior_workspace.argtypes = [ctypes.POINTER(PriorCfg), i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.fzp_pupil_prior.argtypes = [ctypes.POINTER(PriorCfg), P, P, i32, P, P, ctypes.c_size_t, P]
    lib.fzp_pupil_prior_workspace.restype = st
    lib.fzp_pupil_prior.restype = st
    lib.fzp_fwhm_batch.argtypes = [P, i32, i32, dbl, dbl, dbl, P, P]
    lib.fzp_fwhm_batch.restype = st
    lib.fzp_last_error.argtypes = []
    lib.fzp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(lib, status: int):
    if status != FZP_OK:
        raise FZPError(status, lib.fzp_last_error().decode(errors="replace"))


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t) -> int:
    return t.data_ptr() if hasattr(t, "data_ptr") else int(t)


class Plan:
    """A propagation plan: an aperture and one or more instances (lambda, z, ROI, creases).

    path: "fp64", "split", "auto" or "sa"; int8=True selects the split path's
    int8 row pass (FZP_FLAG_SPLIT_INT8); the other keywords map to
    fzp_options_t fields and FZP_FLAG_* bits as named."""

    def __init__(self, aperture: dict, instances: Sequence[dict], path: str = "fp64", stripe_rows: int = 0,
                 chunk_rows: int = 0, workspace_limit: int = 0, allow_undersampled: bool = False,
                 lanes: int = 0, variant: int = 4, overlap_operand: bool = False, pad: float = 0.0,
                 paraxial_radii: bool = False, cplx_tile: int = 0, int8: bool = False):
        lib = load_library()
        self._lib = lib
        ap = Aperture(D=aperture["D"], f0=aperture["f0"], lambda0=aperture["lambda0"],
                      pitch=aperture.get("pitch", 0.0), N=int(aperture["N"]),
                      centre_open=int(aperture.get("centre_open", 0)),
                      levels=int(aperture.get("levels", 0)))
        n = len(instances)
        arr = (Instance * n)()
        self._crease_bufs = []
        for k, inst in enumerate(instances):
            cr = inst.get("creases")
            ncr = 0 if cr is None else len(cr)
            cbuf = (Crease * max(ncr, 1))()
            for c in range(ncr):
                cbuf[c] = Crease(*[float(v) for v in cr[c]])
            self._crease_bufs.append(cbuf)
            arr[k] = Instance(lambda_=inst["lam"], z=inst.get("z", 0.0), x0=inst.get("x0", 0.0),
                              y0=inst.get("y0", 0.0), half_width=inst.get("half_width", 0.0), M=int(inst["M"]),
                              n_creases=ncr, creases=ctypes.cast(cbuf, ctypes.POINTER(Crease)))
        p = {"fp64": PATH_FP64_BLUESTEIN, "split": PATH_SPLIT_BF16, "auto": PATH_AUTO, "sa": PATH_SA_CZT}[path] \
            if isinstance(path, str) else int(path)
        opt = Options(path=p, stripe_rows=stripe_rows, chunk_rows=chunk_rows, workspace_limit=workspace_limit,
                      flags=(FLAG_ALLOW_UNDERSAMPLED if allow_undersampled else 0)
                      | {0: FLAG_BIN_SHALLOW, 1: FLAG_BIN_TILE_256, 2: FLAG_BIN_DEEP,
                         3: FLAG_BIN_PREFETCH, 4: 0}[variant]
                      | (FLAG_OVERLAP_OPERAND if overlap_operand else 0)
                      | (FLAG_PARAXIAL_RADII if paraxial_radii else 0)
                      | (FLAG_SPLIT_INT8 if int8 else 0)
                      | {0: 0, 1: FLAG_CPLX_TILE_128, 2: FLAG_CPLX_TILE_DUAL}[cplx_tile], lanes=int(lanes),
                      pad=float(pad))
        h = ctypes.c_void_p()
        _check(lib, lib.fzp_plan(ctypes.byref(ap), arr, n, ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self.n_instances = n
        self.Ms = [int(inst["M"]) for inst in instances]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.fzp_destroy(h)
            self._h = None

    # -- sizes ---------------------------------------------------------------
    @property
    def workspace_size(self) -> int:
        v = ctypes.c_size_t()
        _check(self._lib, self._lib.fzp_plan_workspace_size(self._h, ctypes.byref(v)))
        return int(v.value)

    @property
    def roi_elements(self) -> int:
        v = ctypes.c_int64()
        _check(self._lib, self._lib.fzp_roi_elements(self._h, ctypes.byref(v)))
        return int(v.value)

    def roi_offset(self, k: int) -> int:
        v = ctypes.c_int64()
        _check(self._lib, self._lib.fzp_roi_offset(self._h, k, ctypes.byref(v)))
        return int(v.value)

    def info(self) -> dict:
        a, b, s, pth = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        c, ds = ctypes.c_int64(), ctypes.c_int64()
        kap = ctypes.c_double()
        _check(self._lib, self._lib.fzp_plan_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                                  ctypes.byref(s), ctypes.byref(pth), ctypes.byref(ds),
                                                  ctypes.byref(kap)))
        return dict(fft_len=a.value, block=b.value, chunk_rows=c.value, stripe_rows=s.value, path=pth.value,
                    disc_samples=ds.value, kappa=kap.value)

    def geometry(self, k: int = 0) -> dict:
        """fzp_plan_geometry: the Eq. 3 zone count and, on the non-paraxial path,
        the padded grid, its FFT factors and the zoom distance of instance k."""
        g = Geometry()
        _check(self._lib, self._lib.fzp_plan_geometry(self._h, int(k), ctypes.byref(g)))
        return g.as_dict()

    # -- device buffers (torch) ---------------------------------------------
    def alloc(self, device="cuda"):
        """(workspace, roi): a uint8 workspace and a float64 ROI buffer of 2 * roi_elements."""
        import torch
        ws = torch.empty(self.workspace_size, dtype=torch.uint8, device=device)
        roi = torch.empty(2 * self.roi_elements, dtype=torch.float64, device=device)
        return ws, roi

    def roi_view(self, roi, k: int):
        """Complex [M, M] view of instance k inside the ROI buffer."""
        import torch
        M = self.Ms[k]
        off = self.roi_offset(k)
        return torch.view_as_complex(roi[2 * off: 2 * (off + M * M)].view(M * M, 2)).view(M, M)

    # -- calls ---------------------------------------------------------------
    def prepare(self, ws, stream=None):
        _check(self._lib, self._lib.fzp_prepare(self._h, _ptr(ws), _stream_handle(stream)))

    def propagate(self, ws, roi, stream=None):
        _check(self._lib, self._lib.fzp_propagate_roi(self._h, _ptr(ws), _ptr(roi), _stream_handle(stream)))

    def propagate_static(self, roi, stream=None):
        """fzp_propagate_roi_static: the whole aperture into roi with the library's
        own device array as the workspace (no device allocation)."""
        _check(self._lib, self._lib.fzp_propagate_roi_static(self._h, _ptr(roi), _stream_handle(stream)))

    def propagate_range(self, ws, roi, row_begin: int, row_end: int, accumulate: bool = False, stream=None):
        _check(self._lib, self._lib.fzp_propagate_roi_range(self._h, _ptr(ws), _ptr(roi), int(row_begin),
                                                            int(row_end), int(bool(accumulate)),
                                                            _stream_handle(stream)))

    def propagate_resumable(self, ws, roi, path: str, rows_per_checkpoint: int = 0, max_rows: int = 0,
                            keep: bool = False, stream=None) -> int:
        """fzp_propagate_resumable: whole aperture with a checkpoint file; returns
        the row where the next call starts (N when complete)."""
        nxt = ctypes.c_int64(0)
        _check(self._lib, self._lib.fzp_propagate_resumable(self._h, _ptr(ws), _ptr(roi), os.fsencode(path),
                                                            int(rows_per_checkpoint), int(max_rows),
                                                            int(bool(keep)), ctypes.byref(nxt),
                                                            _stream_handle(stream)))
        return int(nxt.value)

    def profile(self, on: bool = True):
        """Bracket every row-pass and column-pass launch with HIP events."""
        _check(self._lib, self._lib.fzp_profile_enable(self._h, int(bool(on))))

    def profile_read(self, reset: bool = True) -> dict:
        """Accumulated kernel milliseconds and launch counts (waits for the events)."""
        rm, cm, am = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rn, cn, an = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib, self._lib.fzp_profile_read(self._h, ctypes.byref(rm), ctypes.byref(rn), ctypes.byref(cm),
                                                     ctypes.byref(cn), ctypes.byref(am), ctypes.byref(an),
                                                     int(bool(reset))))
        return dict(row_ms=rm.value, row_launches=rn.value, col_ms=cm.value, col_launches=cn.value,
                    mask_ms=am.value, mask_launches=an.value)

    def metrics(self, ws, roi, stream=None) -> list:
        out = (Metrics * self.n_instances)()
        _check(self._lib, self._lib.fzp_metrics(self._h, _ptr(ws), _ptr(roi), out, _stream_handle(stream)))
        return [out[k].as_dict() for k in range(self.n_instances)]

    def autotune(self, ws, roi, cache_path: Optional[str] = None, stream=None) -> dict:
        """Pick the split GEMM's K-segment length, variant and lane count by timing (overwrites roi)."""
        sl, ln, tl, ms = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        cp = None if cache_path is None else os.fsencode(cache_path)
        _check(self._lib, self._lib.fzp_autotune(self._h, _ptr(ws), _ptr(roi), _stream_handle(stream), cp,
                                                 ctypes.byref(sl), ctypes.byref(ln), ctypes.byref(tl),
                                                 ctypes.byref(ms)))
        return dict(seg_len=sl.value, lanes=ln.value, variant=tl.value, ms=ms.value)

    def graph(self, ws, roi) -> "Graph":
        """One whole propagation of the plan captured as a HIP graph bound to ws and roi."""
        return Graph(self, ws, roi)


class Graph:
    """A captured propagation (fzp_graph_create); keeps its plan and buffers alive."""

    def __init__(self, plan: Plan, ws, roi):
        self._lib = plan._lib
        self._keep = (plan, ws, roi)
        g = ctypes.c_void_p()
        _check(self._lib, self._lib.fzp_graph_create(plan._h, _ptr(ws), _ptr(roi), ctypes.byref(g)))
        self._g = g

    def launch(self, stream=None):
        _check(self._lib, self._lib.fzp_graph_launch(self._g, _stream_handle(stream)))

    def __del__(self):
        g = getattr(self, "_g", None)
        if g is not None and g.value:
            self._lib.fzp_graph_destroy(g)
            self._g = None


class MLP:
    """The surrogate network (fzp_mlp_*): float32 tensors in, float32 out, on the GPU."""

    def __init__(self, n_in: int, n_hidden: int, n_out: int, batch_max: int, device="cuda"):
        import torch
        self._lib = load_library()
        h = ctypes.c_void_p()
        _check(self._lib, self._lib.fzp_mlp_create(n_in, n_hidden, n_out, batch_max, ctypes.byref(h)))
        self._h = h
        b, n = ctypes.c_size_t(), ctypes.c_int64()
        _check(self._lib, self._lib.fzp_mlp_info(h, ctypes.byref(b), ctypes.byref(n)))
        self.n_in, self.n_hidden, self.n_out, self.batch_max = n_in, n_hidden, n_out, batch_max
        self.n_params = int(n.value)
        self.ws = torch.empty(int(b.value), dtype=torch.uint8, device=device)
        self._loss = torch.zeros(1, dtype=torch.float32, device=device)
        self._y = torch.empty((batch_max, n_out), dtype=torch.float32, device=device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.fzp_mlp_destroy(h)
            self._h = None

    def set_params(self, theta, stream=None):
        assert theta.dtype.is_floating_point and theta.numel() == self.n_params and theta.is_contiguous()
        _check(self._lib, self._lib.fzp_mlp_set_params(self._h, _ptr(self.ws), _ptr(theta), _stream_handle(stream)))

    def get_params(self, stream=None):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.ws.device)
        _check(self._lib, self._lib.fzp_mlp_get_params(self._h, _ptr(self.ws), _ptr(out), _stream_handle(stream)))
        return out

    def _rows(self, x):
        assert x.dtype == self._y.dtype and x.is_contiguous() and x.shape[1] == self.n_in
        b = int(x.shape[0])
        assert 1 <= b <= self.batch_max
        return b

    def forward(self, x, out=None, stream=None):
        import torch
        b = self._rows(x)
        y = out if out is not None else torch.empty((b, self.n_out), dtype=torch.float32, device=x.device)
        _check(self._lib, self._lib.fzp_mlp_forward(self._h, _ptr(self.ws), _ptr(x), b, _ptr(y),
                                                    _stream_handle(stream)))
        return y

    def backward(self, x, t, stream=None):
        """(loss tensor[1], grads[n_params], dx[batch, n_in], y[batch, n_out]); no update."""
        import torch
        b = self._rows(x)
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        dx = torch.empty((b, self.n_in), dtype=torch.float32, device=x.device)
        y = torch.empty((b, self.n_out), dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(self._lib, self._lib.fzp_mlp_backward(self._h, _ptr(self.ws), _ptr(x), _ptr(t), b, _ptr(y), _ptr(g),
                                                     _ptr(dx), _ptr(loss), _stream_handle(stream)))
        return loss, g, dx, y

    def train_step(self, x, t, lr: float, stream=None):
        """One forward/backward/Adam step; returns the loss as a device tensor[1] (before the update)."""
        b = self._rows(x)
        _check(self._lib, self._lib.fzp_mlp_train_step(self._h, _ptr(self.ws), _ptr(x), _ptr(t), b, _ptr(self._y),
                                                       float(lr), _ptr(self._loss), _stream_handle(stream)))
        return self._loss

    def adam_update(self, grads, lr: float, stream=None):
        _check(self._lib, self._lib.fzp_mlp_adam_update(self._h, _ptr(self.ws), _ptr(grads), float(lr),
                                                        _stream_handle(stream)))


class PriorCfg(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("M", ctypes.c_int32), ("Np", ctypes.c_int32), ("ss", ctypes.c_int32),
                ("n_creases", ctypes.c_int32), ("floor_", ctypes.c_double)]


class PupilPrior:
    """fzp_pupil_prior: the surrogate's physics prior (first order as a thin lens
    with the deformed pupil) as log-intensity ln(I/I0 + floor) on the M x M ROI,
    for batches of up to n_max instances per library call."""

    def __init__(self, D: float, M: int, n_creases: int, Np: int = 128, ss: int = 4, floor: float = 1e-2,
                 n_max: int = 1024, device="cuda"):
        import torch
        self._lib = load_library()
        self.cfg = PriorCfg(D=float(D), M=int(M), Np=int(Np), ss=int(ss), n_creases=int(n_creases),
                            floor_=float(floor))
        self.M, self.n_creases, self.n_max, self.device = int(M), int(n_creases), int(n_max), device
        nb = ctypes.c_size_t()
        _check(self._lib, self._lib.fzp_pupil_prior_workspace(ctypes.byref(self.cfg), self.n_max, ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def __call__(self, creases, lams, out=None, stream=None):
        """creases [n, n_creases, 4] and lams [n] (host arrays) -> out [n, M*M] float32 (device)."""
        import torch
        cr = torch.as_tensor(np.asarray(creases, dtype=np.float64).reshape(len(lams), self.n_creases, 4),
                             device=self.device).contiguous()
        lm = torch.as_tensor(np.asarray(lams, dtype=np.float64), device=self.device).contiguous()
        n = int(lm.shape[0])
        if out is None:
            out = torch.empty((n, self.M * self.M), dtype=torch.float32, device=self.device)
        for s in range(0, n, self.n_max):
            e = min(s + self.n_max, n)
            _check(self._lib, self._lib.fzp_pupil_prior(ctypes.byref(self.cfg), _ptr(cr[s:e]) if self.n_creases else None,
                                                        _ptr(lm[s:e]), e - s, _ptr(out[s:e]), _ptr(self.ws),
                                                        self.ws_bytes, _stream_handle(stream)))
        return out


def fwhm_batch(y, M: int, floor: float, level_delta: float = 0.05, exclusion_radius: float = 10.0, stream=None):
    """fzp_fwhm_batch on y [n, M*M] (device float32 log-intensity maps): a device
    float64 tensor [n, 5] of (FWHM in samples, cond, ratio, gap, walt)."""
    import torch
    lib = load_library()
    n = int(y.shape[0])
    out = torch.empty((n, 5), dtype=torch.float64, device=y.device)
    _check(lib, lib.fzp_fwhm_batch(_ptr(y), n, int(M), float(floor), float(level_delta), float(exclusion_radius),
                                   _ptr(out), _stream_handle(stream)))
    return out


def grid_for_element(D: float, f0: float, lambda0: float, levels: int = 0, s_samp: int = 0):
    """fzp_grid_for_element: (pitch, N) of the revised engine's grid rule."""
    lib = load_library()
    dx, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib, lib.fzp_grid_for_element(float(D), float(f0), float(lambda0), int(levels), int(s_samp),
                                         ctypes.byref(dx), ctypes.byref(n)))
    return dx.value, n.value


def log_intensity(roi, n_complex: int, i0: float, floor: float, out, stream=None):
    """out[:n] = ln(|U|^2/i0 + floor) on the GPU (roi: float64 interleaved complex)."""
    lib = load_library()
    _check(lib, lib.fzp_log_intensity(_ptr(roi), int(n_complex), float(i0), float(floor), _ptr(out),
                                      _stream_handle(stream)))


def field_from_log_intensity(y, n_complex: int, i0: float, floor: float, roi, stream=None):
    """roi[:n] = sqrt(max(i0 (e^y - floor), 0)) + 0i on the GPU."""
    lib = load_library()
    _check(lib, lib.fzp_field_from_log_intensity(_ptr(y), int(n_complex), float(i0), float(floor), _ptr(roi),
                                                 _stream_handle(stream)))
