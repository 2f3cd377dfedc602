"""The C-ABI library loads, exports every symbol the header declares, and rejects bad arguments
on the host before touching the device (runs without a GPU)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vettam_rad.h")


@pytest.fixture(scope="module")
def rad():
    from paper_2202_08778_amd import rad as r
    return r


def _declared():
    src = open(HEADER).read()
    decl = r"^(?:int|size_t|void|const char \*)\s*\*?\s*(rad_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, src, flags=re.M)))


def test_library_exports_every_declared_symbol(rad):
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(rad.lib, n), n
        assert n in rad.EXPORTED, n


def test_defaults(rad):
    p = rad.params()
    assert (p.c, p.a_R, p.c_v) == (1.0, 1.0, 1.0)
    assert p.gmres_m == 12 and p.prec == 0 and p.mode == 1 and p.eps_R == 1e-2 and p.anderson_m == 0
    assert p.vel_implicit == 0


def _step(rad, p, nx=4, ny=4, nz=4, ptr=0x1000, bc="periodic", dt=1.0, dx=1.0, ws=None, wsb=None):
    st = rad.Stats()
    need = rad.lib.rad_workspace_bytes(nx, ny, nz, ct.byref(p))
    ws = ws if ws is not None else 0x10000
    wsb = wsb if wsb is not None else need
    P = lambda: ptr
    return rad.lib.rad_step(nx, ny, nz, P(), P(), P(), P(), P(), P(), P(), dt, dx, rad.bc_array(bc),
                            ct.byref(p), ws, wsb, None, ct.byref(st))


@pytest.mark.parametrize("case,msg", [
    (dict(nx=0), "extents"),
    (dict(dt=-1.0), "dt"),
    (dict(dt=float("nan")), "dt"),
    (dict(dx=0.0), "dx"),
    (dict(bc=("periodic", "outflow", "periodic", "periodic", "periodic", "periodic")), "pairs"),
    (dict(bc="dirichlet"), "ghost data"),
    (dict(ptr=0), "NULL"),
    (dict(ws=0), "workspace"),
    (dict(ws=0x10001), "aligned"),
    (dict(wsb=16), "too small"),
])
def test_rad_step_rejects_bad_arguments_on_host(rad, case, msg):
    p = rad.params()
    rc = _step(rad, p, **case)
    assert rc in (rad.RAD_EINVAL, rad.RAD_ENOMEM)
    assert msg in rad.last_error()


def test_dirichlet_faces_need_ghost_data_on_host(rad):
    """A Dirichlet face of the single grid takes its data from params->ghost: without it the step,
    the residual and the autotuner refuse it; with it the boundary check passes (here the call then
    stops at the workspace check); the linear operator and the face speeds read no data; the
    two-level grid and faces of more than 2^26 cells are refused."""
    bc = ("dirichlet", "dirichlet", "periodic", "periodic", "periodic", "periodic")
    p = rad.params()
    assert _step(rad, p, bc=bc) == rad.RAD_EINVAL and "ghost[0]" in rad.last_error()
    p.ghost[0] = 0x1000
    assert _step(rad, p, bc=bc) == rad.RAD_EINVAL and "ghost[1]" in rad.last_error()
    p.ghost[1] = 0x2000
    assert _step(rad, p, bc=bc, ws=0) == rad.RAD_EINVAL and "workspace" in rad.last_error()
    q = rad.params()
    b = rad.bc_array(bc)
    assert rad.lib.rad_residual(4, 4, 4, *([8] * 10), 1.0, 1.0, b, ct.byref(q), 8, None) == rad.RAD_EINVAL
    assert "ghost" in rad.last_error()
    assert rad.lib.rad_autotune_step(4, 4, 4, *([8] * 7), 1.0, 1.0, b, ct.byref(q), 0x1000, 1 << 30, None, 1,
                                     None, None, None, None) == rad.RAD_EINVAL
    assert "ghost" in rad.last_error()
    # the linear operator and the face speeds pass the boundary check without data (then fail on dtype)
    assert rad.lib.rad_apply(4, 4, 4, 8, 8, 8, 8, 8, 8, 1.0, 1.0, b, ct.byref(q), 5, None) == rad.RAD_EINVAL
    assert "dtype" in rad.last_error()
    g = rad.amr_geometry((4, 4, 4), (1, 1, 1), (3, 3, 3))
    assert rad.lib.rad_step_amr2(ct.byref(g), *([8] * 7), 1.0, 1.0, b, ct.byref(p), 0x1000, 1 << 30, None,
                                 None) == rad.RAD_EINVAL
    assert "boundary" in rad.last_error()
    big = rad.params()
    big.ghost[0] = big.ghost[1] = 0x1000
    assert _step(rad, big, nx=1, ny=9000, nz=9000, bc=bc) == rad.RAD_EINVAL
    assert "2^26" in rad.last_error()


@pytest.mark.parametrize("field,val", [("gmres_m", 0), ("gmres_m", 65), ("c", 0.0), ("tol", 0.0), ("prec", 7),
                                       ("mode", 3), ("coef_dtype", 2), ("max_picard", 0), ("a_R", -1.0),
                                       ("anderson_m", -1), ("anderson_m", 6)])
def test_rad_step_rejects_bad_params(rad, field, val):
    p = rad.params()
    setattr(p, field, val)
    assert _step(rad, p) == rad.RAD_EINVAL
    assert rad.lib.rad_workspace_bytes(4, 4, 4, ct.byref(p)) == 0


def test_anderson_history_takes_workspace(rad):
    a = rad.lib.rad_workspace_bytes(32, 32, 32, ct.byref(rad.params()))
    b = rad.lib.rad_workspace_bytes(32, 32, 32, ct.byref(rad.params(anderson_m=3)))
    assert b - a >= 2 * 4 * 32 ** 3 * 8   # (m + 1) map values and residuals, FP64


def test_workspace_grows_with_restart_length_and_precision(rad):
    a = rad.lib.rad_workspace_bytes(32, 32, 32, ct.byref(rad.params(gmres_m=10)))
    b = rad.lib.rad_workspace_bytes(32, 32, 32, ct.byref(rad.params(gmres_m=20)))
    c = rad.lib.rad_workspace_bytes(32, 32, 32, ct.byref(rad.params(gmres_m=20, prec="mixed")))
    assert 0 < a < b and c < b
    # basis of (m+1) 4-component vectors dominates
    assert b - a >= 10 * 4 * 32 ** 3 * 8


def test_other_entry_points_validate(rad):
    p = rad.params()
    bc = rad.bc_array("periodic")
    assert rad.lib.rad_apply(4, 4, 4, None, None, None, None, None, None, 1.0, 1.0, bc, ct.byref(p), 0,
                             None) == rad.RAD_EINVAL
    assert rad.lib.rad_apply(4, 4, 4, 8, 8, 8, 8, 8, 8, 1.0, 1.0, bc, ct.byref(p), 5, None) == rad.RAD_EINVAL
    assert rad.lib.rad_exchange(0, 8, 8, 8, 8, 8, 1.0, ct.byref(p), None) == rad.RAD_EINVAL
    assert rad.lib.rad_face_speeds(4, 4, 4, None, 8, 8, 1.0, bc, ct.byref(p), 8, None) == rad.RAD_EINVAL
    assert rad.lib.rad_plan_launch_shape(None, None, None, None) == rad.RAD_EINVAL
    # closures: bad kind, c, dtype or pointers are rejected on the host; an empty grid is a no-op
    assert rad.lib.rad_closure(8, 8, 8, 2, 1.0, 8, 0, None) == rad.RAD_EINVAL
    assert rad.lib.rad_closure(8, 8, 8, 1, 0.0, 8, 0, None) == rad.RAD_EINVAL
    assert rad.lib.rad_closure(8, 8, 8, 1, 1.0, 8, 3, None) == rad.RAD_EINVAL
    assert rad.lib.rad_closure(8, None, 8, 1, 1.0, 8, 0, None) == rad.RAD_EINVAL
    assert rad.lib.rad_closure(-1, 8, 8, 1, 1.0, 8, 0, None) == rad.RAD_EINVAL
    assert rad.lib.rad_closure(0, None, None, 1, 1.0, None, 0, None) == rad.RAD_OK
    # autotune validates like rad_step before touching the device
    assert rad.lib.rad_autotune_step(4, 4, 4, None, 8, 8, 8, 8, 8, 8, 1.0, 1.0, bc, ct.byref(p), 0x1000, 1 << 30,
                                     None, 1, None, None, None, None) == rad.RAD_EINVAL
    assert rad.lib.rad_autotune_step(0, 4, 4, 8, 8, 8, 8, 8, 8, 8, 1.0, 1.0, bc, ct.byref(p), 0x1000, 1 << 30,
                                     None, 1, None, None, None, None) == rad.RAD_EINVAL


def test_amr2_geometry_is_validated_on_host(rad):
    p = rad.params()
    ws = lambda g: rad.lib.rad_workspace_bytes_amr2(ct.byref(g), ct.byref(p))
    ok = rad.amr_geometry((8, 8, 8), (2, 2, 2), (6, 7, 6))
    assert ws(ok) > rad.lib.rad_workspace_bytes(8, 8, 8, ct.byref(p))
    assert ws(rad.amr_geometry((8, 8, 8), (0, 0, 0), (8, 8, 8))) > 0   # box spanning every axis
    for lo, hi in [((0, 2, 2), (6, 6, 6)), ((2, 2, 2), (8, 6, 6)), ((3, 2, 2), (3, 6, 6)), ((2, 2, 2), (6, 6, 9)),
                   ((-1, 2, 2), (6, 6, 6))]:
        g = rad.amr_geometry((8, 8, 8), lo, hi)
        assert ws(g) == 0, (lo, hi)
        st = rad.Stats()
        P = 0x1000
        rc = rad.lib.rad_step_amr2(ct.byref(g), P, P, P, P, P, P, P, 1.0, 1.0, rad.bc_array("periodic"), ct.byref(p),
                                   0x10000, 1 << 30, None, ct.byref(st))
        assert rc == rad.RAD_EINVAL and "refined box" in rad.last_error(), (lo, hi, rad.last_error())
    # an invalid params struct is caught before the geometry is used
    bad = rad.params(gmres_m=0)
    assert rad.lib.rad_workspace_bytes_amr2(ct.byref(ok), ct.byref(bad)) == 0


def test_moving_step_is_validated_on_host(rad):
    p = rad.params()
    base = rad.lib.rad_workspace_bytes(8, 8, 8, ct.byref(p))
    assert rad.lib.rad_workspace_bytes_moving(8, 8, 8, ct.byref(p)) > base
    assert rad.lib.rad_workspace_bytes_moving(8, 8, 8, ct.byref(rad.params(vel_implicit=2))) == 0
    P, st = 0x1000, rad.Stats()
    call = lambda q, beta: rad.lib.rad_step_moving(8, 8, 8, P, P, P, P, P, P, P, beta, 1.0, 1.0,
                                                   rad.bc_array("periodic"), ct.byref(q), 0x10000, 1 << 30, None,
                                                   ct.byref(st))
    assert call(p, None) == rad.RAD_EINVAL and "beta" in rad.last_error()
    assert call(rad.params(vel_implicit=1, anderson_m=2), P) == rad.RAD_EINVAL and "anderson" in rad.last_error()
    assert call(rad.params(vel_implicit=3), P) == rad.RAD_EINVAL


def test_cubic_gas_is_validated(rad):
    assert rad.lib.rad_workspace_bytes(8, 8, 8, ct.byref(rad.params(cv_cubic=2))) == 0
    g = rad.amr_geometry((8, 8, 8), (2, 2, 2), (6, 6, 6))
    assert rad.lib.rad_workspace_bytes_amr2(ct.byref(g), ct.byref(rad.params(cv_cubic=1))) == 0
    assert rad.params().cv_cubic == 0


def test_plan_reorder_rejects_null(rad):
    assert rad.lib.rad_plan_reorder(None, None, None) == rad.RAD_EINVAL and "plan" in rad.last_error()


def test_krylov_polynomial_is_validated(rad):
    assert rad.params().krylov_poly == 1
    assert rad.lib.rad_workspace_bytes(8, 8, 8, ct.byref(rad.params(krylov_poly=3))) == 0
    assert "krylov_poly" in rad.last_error()
    assert rad.lib.rad_workspace_bytes(8, 8, 8, ct.byref(rad.params(krylov_poly=0))) > 0
    # multigrid: extents must halve at least once; its levels enlarge the workspace
    mg = rad.params(krylov_poly=2)
    assert rad.lib.rad_workspace_bytes(9, 8, 8, ct.byref(mg)) == 0 and "multigrid" in rad.last_error()
    assert rad.lib.rad_workspace_bytes(16, 16, 16, ct.byref(mg)) > rad.lib.rad_workspace_bytes(
        16, 16, 16, ct.byref(rad.params()))
    assert rad.lib.rad_workspace_bytes_moving(16, 16, 16, ct.byref(mg)) == 0
    g = rad.amr_geometry((8, 8, 8), (2, 2, 2), (6, 6, 6))
    assert rad.lib.rad_workspace_bytes_amr2(ct.byref(g), ct.byref(mg)) == 0
