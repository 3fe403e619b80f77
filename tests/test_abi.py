"""Host-side tests of the C ABI (no GPU needed): the library loads, exports
every function that include/fzp.h declares, and validates its arguments."""
import ctypes
import math
import os
import re

import pytest

import paper_2609_01978_amd as P
from paper_2609_01978_amd import _lib as L
from oracle import fzp_oracle as O
from fzp_inputs import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LAM0 = 632.8e-9


def header_functions():
    text = open(os.path.join(ROOT, "include", "fzp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fzp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = P.load_library()
    declared = header_functions()
    assert "fzp_plan" in declared and "fzp_propagate_roi" in declared and "fzp_metrics" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(declared) == sorted(P.EXPORTED)


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(L.Aperture) == 48
    assert ctypes.sizeof(L.Crease) == 32
    assert ctypes.sizeof(L.Instance) == 56
    assert ctypes.sizeof(L.Options) == 40
    assert ctypes.sizeof(L.Geometry) == 40
    assert ctypes.sizeof(L.Metrics) == 64
    assert ctypes.sizeof(L.PriorCfg) == 32


def ap_of(name):
    w = workload(name)
    return dict(D=w["D"], f0=w["f0"], lambda0=w["lambda0"], N=w["N"]), w


def test_plan_facts_match_oracle():
    for name in ("fzp2mm", "fzp20mm"):
        ap, w = ap_of(name)
        plan = P.Plan(ap, [dict(lam=w["lambda0"], M=w["M"])])
        info = plan.info()
        oa = O.Aperture(D=ap["D"], f0=ap["f0"], lambda0=ap["lambda0"], N=ap["N"])
        assert info["disc_samples"] == O.incident_count(oa)
        assert info["kappa"] == oa.dx * oa.dx / (4.0 * oa.lambda0 * oa.f0)
        assert info["block"] == 4096 - w["M"] + 1
        assert plan.roi_elements == w["M"] ** 2


def test_sampling_limit_eq6():
    with pytest.raises(P.FZPError) as e:
        P.Plan(dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=1024), [dict(lam=LAM0, M=64)])
    assert e.value.status == P.FZP_E_SAMPLING
    # 2 samples per outermost zone is the limit: N = 2 D^2/(lambda f) passes
    N = int(2 * (2e-3) ** 2 / (LAM0 * 10e-3)) + 1
    P.Plan(dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=N), [dict(lam=LAM0, M=64)])
    P.Plan(dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=64), [dict(lam=LAM0, M=64)], allow_undersampled=True)


@pytest.mark.parametrize("bad", [
    dict(ap=dict(D=-1.0)), dict(ap=dict(N=0)), dict(ap=dict(N=(1 << 24) + 1)), dict(ap=dict(centre_open=2)),
    dict(inst=dict(M=1)), dict(inst=dict(M=4096)), dict(inst=dict(lam=float("nan"))), dict(inst=dict(z=-1.0)),
    dict(inst=dict(creases=[(0.0, 0.0, 0.0, 1e-7)])),
])
def test_invalid_arguments(bad):
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096)
    inst = dict(lam=LAM0, M=256)
    ap.update(bad.get("ap", {}))
    inst.update(bad.get("inst", {}))
    with pytest.raises(P.FZPError) as e:
        P.Plan(ap, [inst])
    assert e.value.status == P.FZP_E_INVAL


def test_workspace_limit_and_split_constraints():
    ap, w = ap_of("fzp1m")
    inst = dict(lam=w["lambda0"], M=w["M"])
    plan = P.Plan(ap, [inst], path="split")
    need = plan.workspace_size
    assert need > 4 * 2 ** 30                      # the BF16 hi/lo operand table of the 1 m element
    with pytest.raises(P.FZPError) as e:
        P.Plan(ap, [inst], path="split", workspace_limit=need - 1)
    assert e.value.status == P.FZP_E_NOMEM
    P.Plan(ap, [inst], path="split", workspace_limit=need)
    with pytest.raises(P.FZPError) as e:
        P.Plan(dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096), [dict(lam=LAM0, M=100)], path="split")
    assert e.value.status == P.FZP_E_UNSUPPORTED
    with pytest.raises(P.FZPError) as e:
        P.Plan(dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096), [dict(lam=LAM0, M=256)], path="split", stripe_rows=96)
    assert e.value.status == P.FZP_E_INVAL


def test_multi_instance_roi_offsets():
    ap = dict(D=20e-3, f0=100e-3, lambda0=LAM0, N=32768)
    Ms = [256, 1024, 512]
    plan = P.Plan(ap, [dict(lam=600e-9, M=m) for m in Ms])
    assert plan.roi_elements == sum(m * m for m in Ms)
    assert [plan.roi_offset(k) for k in range(3)] == [0, 256 ** 2, 256 ** 2 + 1024 ** 2]


def test_last_error_is_thread_local_message():
    lib = P.load_library()
    with pytest.raises(P.FZPError):
        P.Plan(dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=0), [dict(lam=LAM0, M=256)])
    assert b"N must be" in lib.fzp_last_error()


def test_split_creased_plan_layout():
    """Deformed stripes on the split path: the plan adds the complex stripe planes
    (8 bytes per sample of a chunk, chunks of whole 256-row tiles up to 8 GiB)."""
    from fzp_inputs import crease_draws
    ap, w = ap_of("fzp20mm")
    flat = P.Plan(ap, [dict(lam=w["lambda0"], M=512)], path="split")
    cr = crease_draws(0, w["D"], w["lambda0"], 8)
    bent = P.Plan(ap, [dict(lam=w["lambda0"], M=512, creases=cr)], path="split")
    c = bent.info()["chunk_rows"]
    assert c % 256 == 0 and c * w["N"] * 8 <= 2 ** 33
    table = 2 * (2 * 512) * w["N"] * 2               # hi/lo planes of the N x 2M BF16 operand table
    assert bent.workspace_size >= table + c * w["N"] * 8
    assert flat.workspace_size < table + c * w["N"] * 8


def test_mlp_create_and_layout():
    from oracle import mlp_oracle as Q
    lib = P.load_library()
    import ctypes
    h = ctypes.c_void_p()
    assert lib.fzp_mlp_create(33, 512, 16384, 256, ctypes.byref(h)) == P.FZP_OK
    b, n = ctypes.c_size_t(), ctypes.c_int64()
    assert lib.fzp_mlp_info(h, ctypes.byref(b), ctypes.byref(n)) == P.FZP_OK
    assert n.value == Q.param_count(33, 512, 16384) == 8685056
    # masters, BF16 copies, two moments, gradients, activations of 256 rows
    assert b.value >= n.value * (4 + 2 + 4 + 4 + 4) + 256 * 16384 * 6
    lib.fzp_mlp_destroy(h)
    for bad in ((0, 512, 16384, 256), (33, 512, 16384, 0), (33, 0, 10, 1), (33, 10, 10, 70000)):
        assert lib.fzp_mlp_create(*bad, ctypes.byref(h)) == P.FZP_E_INVAL
    assert b"sizes" in lib.fzp_last_error()


def test_missing_library_raises_import_error(monkeypatch):
    """No other implementation exists: without libfzp.so the first call that needs
    it raises ImportError."""
    from paper_2609_01978_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", L.LIB_PATH + ".absent")
    with pytest.raises(ImportError):
        L.load_library()
    with pytest.raises(ImportError):
        P.Plan(dict(D=2e-3, f0=10e-3, lambda0=632.8e-9, N=256), [dict(lam=632.8e-9, M=16)])


def test_phase_plate_plans():
    """levels: 0 or 2 .. 64, amplitude-only centre_open; a split phase plate
    takes the complex-stripe layout (stripe planes in the workspace)."""
    from paper_2609_01978_amd._lib import FZPError
    base = dict(D=2e-3, f0=10e-3, lambda0=632.8e-9, N=2048)
    for bad in (dict(levels=1), dict(levels=65), dict(levels=-2), dict(levels=4, centre_open=1)):
        with pytest.raises(FZPError) as ei:
            P.Plan(dict(base, **bad), [dict(lam=632.8e-9, M=32)])
        assert ei.value.status == L.FZP_E_INVAL
    flat = P.Plan(base, [dict(lam=632.8e-9, M=64)], path="split")
    for lv in (2, 4, 16, 64):
        ph = P.Plan(dict(base, levels=lv), [dict(lam=632.8e-9, M=64)], path="split")
        assert ph.workspace_size > flat.workspace_size
        assert P.Plan(dict(base, levels=lv), [dict(lam=632.8e-9, M=64)]).workspace_size > 0


@pytest.mark.parametrize("levels,creased,M,want", [
    (0, False, 512, L.PATH_SPLIT_BF16), (0, False, 1024, L.PATH_SPLIT_BF16), (0, False, 2048, L.PATH_FP64_BLUESTEIN),
    (0, True, 256, L.PATH_SPLIT_BF16), (0, True, 512, L.PATH_FP64_BLUESTEIN),
    (4, False, 256, L.PATH_SPLIT_BF16), (4, False, 512, L.PATH_FP64_BLUESTEIN), (4, True, 256, L.PATH_FP64_BLUESTEIN),
    (2, False, 1024, L.PATH_SPLIT_BF16), (2, False, 2048, L.PATH_FP64_BLUESTEIN), (2, True, 256, L.PATH_FP64_BLUESTEIN),
    (8, False, 128, L.PATH_SPLIT_BF16), (8, False, 256, L.PATH_FP64_BLUESTEIN),
    (0, False, 100, L.PATH_FP64_BLUESTEIN)])
def test_auto_path_follows_the_measured_crossover(levels, creased, M, want):
    ap = dict(D=2e-3, f0=10e-3, lambda0=632.8e-9, N=4096, levels=levels)
    inst = dict(lam=632.8e-9, M=M)
    if creased:
        inst["creases"] = [[0.3, 1e-4, 1e-4, 1e-7]]
    assert P.Plan(ap, [inst], path="auto").info()["path"] == want


@pytest.mark.parametrize("path", ["fp64", "split"])
def test_chunk_rows_above_n_are_taken_as_n(path):
    """A caller's chunk_rows beyond the aperture only enlarges the buffers; a
    huge value must not wrap the workspace byte counts: it is taken as N."""
    ap = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096)
    inst = [dict(lam=LAM0, M=256)]
    whole = P.Plan(ap, inst, path=path, chunk_rows=4096)
    for c in (4097, 1 << 40, (1 << 62) + 12345):
        p = P.Plan(ap, inst, path=path, chunk_rows=c)
        assert p.info()["chunk_rows"] == whole.info()["chunk_rows"] == 4096
        assert p.workspace_size == whole.workspace_size


def test_graph_of_overlap_operand_plan_is_refused():
    """fzp_graph_create refuses a split plan with FZP_FLAG_OVERLAP_OPERAND before
    any device call (its capture is not supported)."""
    lib = P.load_library()
    plan = P.Plan(dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048), [dict(lam=LAM0, M=64)], path="split",
                  overlap_operand=True)
    g = ctypes.c_void_p()
    st = lib.fzp_graph_create(plan._h, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21), ctypes.byref(g))
    assert st == L.FZP_E_UNSUPPORTED and not g.value
    assert b"OVERLAP_OPERAND" in lib.fzp_last_error()


def test_non_paraxial_plan_geometry_and_validation():
    """FZP_PATH_SA_CZT: the padded grid follows the pad rule of the oracle, factors
    into two LDS lengths, the Eq. 3 zone count matches the oracle's root, and the
    path refuses phase plates, bad pads and partial row ranges (before any device
    call)."""
    from oracle import sa_czt_oracle as S
    lib = P.load_library()
    for N, D, f, pad in ((4096, 2e-3, 10e-3, 0.0), (28672, 0.08, 1.5, 0.0), (1001, 1e-3, 5e-3, 2.0),
                         (2048, 1e-3, 2e-3, 3.0)):
        lam0 = 532e-9 if D == 0.08 else LAM0
        plan = P.Plan(dict(D=D, f0=f, lambda0=lam0, N=N), [dict(lam=lam0, M=64)], path="sa", pad=pad,
                      allow_undersampled=True)
        g = plan.geometry(0)
        assert g["padded_n"] == S.pad_size(N, pad or 1.5)
        assert g["fft_n1"] * g["fft_n2"] == g["padded_n"] and g["fft_n1"] <= g["fft_n2"] <= 1024
        assert abs(g["zones_exact"] / O.zone_count_exact(D, lam0, f) - 1) < 1e-12
        assert g["total_zones"] == int(O.zone_count_exact(D, lam0, f))
        # zoom distance Z / lambda = 4 pi |d| z / (k_max lambda) with the two-point fit at k_max = 2 k0 / 3
        k0, kmax, c, d = S.fit_constants(lam0)
        assert abs(g["zoom_distance"] / (4 * math.pi * abs(d) * f / (kmax * lam0)) - 1) < 1e-12
    assert P.Plan(dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=4096), [dict(lam=LAM0, M=64)]).geometry()["padded_n"] == 0
    base = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048)
    with pytest.raises(P.FZPError) as e:
        P.Plan(dict(base, levels=4), [dict(lam=LAM0, M=64)], path="sa")
    assert e.value.status == L.FZP_E_UNSUPPORTED
    for pad in (0.5, 9.0, float("nan")):
        with pytest.raises(P.FZPError) as e:
            P.Plan(base, [dict(lam=LAM0, M=64)], path="sa", pad=pad)
        assert e.value.status == L.FZP_E_INVAL
    plan = P.Plan(base, [dict(lam=LAM0, M=64)], path="sa")
    st = lib.fzp_propagate_roi_range(plan._h, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21), 0, 1024, 0, None)
    assert st == L.FZP_E_UNSUPPORTED


def _grid_tables():
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "v8_grid_tables.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t, D, f, L, dx, nx = line.split()
                rows.append((int(t), float(D), float(f), int(L), float(dx), int(nx)))
    return rows


@pytest.mark.parametrize("row", [r for r in _grid_tables() if r[0] <= 4], ids=lambda r: f"table{r[0]}")
def test_grid_for_element_reproduces_tables_1_to_4(row):
    """The library's grid rule gives the printed pitch and N_x of Tables 1-4
    (Sec. 7.1; 532 nm) and agrees with the oracle's rule."""
    t, D, f, L, dx_um, nx = row
    dx, n = P.grid_for_element(D, f, 532e-9, L)
    assert n == nx and abs(dx * 1e6 - dx_um) <= 0.0006
    assert (dx, n) == O.v8_grid(D, f, 532e-9, L)
    # the plan takes that grid (a pitch of its own and N up to 2^24)
    plan = P.Plan(dict(D=D, f0=f, lambda0=532e-9, N=n, pitch=dx, levels=L), [dict(lam=532e-9, M=64)])
    assert plan.info()["disc_samples"] > 0.78 * n * n


def test_grid_for_element_arguments():
    assert P.grid_for_element(1.0, 5.0, 532e-9, 0) == P.grid_for_element(1.0, 5.0, 532e-9, 2)
    with pytest.raises(P.FZPError):
        P.grid_for_element(-1.0, 5.0, 532e-9, 4)
    with pytest.raises(P.FZPError):
        P.Plan(dict(D=1.0, f0=5.0, lambda0=532e-9, N=(1 << 24) + 1), [dict(lam=532e-9, M=64)],
               allow_undersampled=True)


def test_pupil_prior_host_validation():
    """fzp_pupil_prior_workspace's size rule and the argument checks that both
    prior calls make on the host before any launch (the fake device addresses
    below are never touched: every call here returns before launching)."""
    lib = P.load_library()
    ok = dict(D=10e-3, M=128, Np=128, ss=4, n_creases=8, floor_=1e-2)
    nb = ctypes.c_size_t()
    assert lib.fzp_pupil_prior_workspace(ctypes.byref(L.PriorCfg(**ok)), 7, ctypes.byref(nb)) == L.FZP_OK
    a256 = lambda v: (v + 255) // 256 * 256
    assert nb.value == a256(128 * 128 * 8) + a256(7 * (128 * 128 + 128 * 128) * 8)
    for bad in (dict(Np=8), dict(Np=24), dict(Np=2048), dict(ss=0), dict(ss=17), dict(n_creases=65),
                dict(n_creases=-1), dict(M=0), dict(M=5000), dict(floor_=0.0), dict(D=0.0), dict(D=float("nan"))):
        cfg = L.PriorCfg(**{**ok, **bad})
        assert lib.fzp_pupil_prior_workspace(ctypes.byref(cfg), 1, ctypes.byref(nb)) == L.FZP_E_INVAL, bad
        assert lib.fzp_pupil_prior(ctypes.byref(cfg), 16, 16, 1, 16, 16, 1 << 30, None) == L.FZP_E_INVAL, bad
    cfg = L.PriorCfg(**ok)
    assert lib.fzp_pupil_prior_workspace(ctypes.byref(cfg), 0, ctypes.byref(nb)) == L.FZP_E_INVAL
    assert lib.fzp_pupil_prior(ctypes.byref(cfg), None, None, 0, None, None, 0, None) == L.FZP_OK      # nothing to do
    assert lib.fzp_pupil_prior(ctypes.byref(cfg), None, 16, 2, 16, 16, 1 << 30, None) == L.FZP_E_INVAL  # no creases
    assert lib.fzp_pupil_prior(ctypes.byref(cfg), 16, 16, 70000, 16, 16, 1 << 40, None) == L.FZP_E_INVAL
    lib.fzp_pupil_prior_workspace(ctypes.byref(cfg), 3, ctypes.byref(nb))
    assert lib.fzp_pupil_prior(ctypes.byref(cfg), 16, 16, 3, 16, 16, nb.value - 1, None) == L.FZP_E_NOMEM
    assert "workspace" in lib.fzp_last_error().decode()


def test_split_int8_plan_validation():
    """FZP_FLAG_SPLIT_INT8: any split plan (binary stripes, and complex ones:
    creases, other level counts); refused on the other paths, checked in
    fzp_plan before any device call."""
    base = dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048)
    for lv in (0, 2, 4, 8):
        P.Plan(dict(base, levels=lv), [dict(lam=LAM0, M=64)], path="split", int8=True)
    P.Plan(base, [dict(lam=LAM0, M=64, creases=[[0.3, 0.0, 2e-4, 1e-7]])], path="split", int8=True)
    for path in ("fp64", "sa"):
        with pytest.raises(P.FZPError) as e:
            P.Plan(base, [dict(lam=LAM0, M=64)], path=path, int8=True)
        assert e.value.status == P.FZP_E_UNSUPPORTED


@pytest.mark.parametrize("levels,creased,M,want", [
    (0, False, 2048, L.PATH_SPLIT_BF16), (0, True, 512, L.PATH_SPLIT_BF16), (0, True, 1024, L.PATH_FP64_BLUESTEIN),
    (4, False, 512, L.PATH_SPLIT_BF16), (8, False, 256, L.PATH_SPLIT_BF16), (8, False, 512, L.PATH_FP64_BLUESTEIN)])
def test_auto_path_with_int8_doubles_the_crossover(levels, creased, M, want):
    """With FZP_FLAG_SPLIT_INT8 the auto path takes the split path up to twice
    the BF16 crossovers (half the matrix-core time); when it picks the FP64
    path the flag is dropped instead of refused."""
    cr = [[0.3, 0.0, 2e-4, 1e-7]] if creased else None
    plan = P.Plan(dict(D=2e-3, f0=10e-3, lambda0=LAM0, N=2048, levels=levels),
                  [dict(lam=LAM0, M=M, creases=cr)], path="auto", int8=True)
    assert plan.info()["path"] == want
