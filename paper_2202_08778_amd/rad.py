"""ctypes binding of libvettam_rad.so (the C ABI in include/vettam_rad.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors, workspaces) and the current
stream; nothing here computes on the data.  If the library is missing the
import of this module fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvettam_rad.so")

RAD_OK, RAD_NOT_CONVERGED = 0, 1
RAD_EINVAL, RAD_ENOMEM, RAD_EHIP, RAD_ENOTIMPL, RAD_EDATA = -1, -2, -3, -4, -5
BC = {"periodic": 0, "outflow": 1, "dirichlet": 2, "open": 3, "marshak": 4, "reflect": 5}
PREC = {"fp64": 0, "mixed": 1}
MODE = {"lagged": 0, "linearised": 1}
DTYPE = {"f64": 0, "f32": 1}


class Params(ct.Structure):
    _fields_ = [("c", ct.c_double), ("a_R", ct.c_double), ("c_v", ct.c_double), ("tol", ct.c_double),
                ("eps_R", ct.c_double), ("eps_P", ct.c_double), ("max_picard", ct.c_int),
                ("max_krylov", ct.c_int), ("gmres_m", ct.c_int), ("prec", ct.c_int), ("mode", ct.c_int),
                ("coef_dtype", ct.c_int), ("anderson_m", ct.c_int), ("vel_implicit", ct.c_int),
                ("cv_cubic", ct.c_int), ("krylov_poly", ct.c_int), ("F_inc", ct.c_double * 6), ("eps_N", ct.c_double),
                ("energy_fix", ct.c_int), ("max_refine", ct.c_int), ("ghost", ct.c_void_p * 6)]


class Stats(ct.Structure):
    _fields_ = [("status", ct.c_int), ("picard_iters", ct.c_int), ("krylov_iters", ct.c_int),
                ("refine_sweeps", ct.c_int), ("neg_cells", ct.c_int), ("bad_cells", ct.c_int),
                ("scaled_residual", ct.c_double), ("res_E", ct.c_double), ("res_F", ct.c_double),
                ("res_T", ct.c_double), ("rel_change", ct.c_double), ("t_total_ms", ct.c_double),
                ("energy_defect", ct.c_double), ("dE_max", ct.c_double), ("bytes_moved", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BlockDesc(ct.Structure):
    _fields_ = [("n", ct.c_int), ("ng", ct.c_int), ("dx", ct.c_double), ("dt", ct.c_double),
                ("off", ct.c_longlong)]


class Amr2(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int), ("lo", ct.c_int * 3), ("hi", ct.c_int * 3)]


class RadError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rad error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2202_08778_amd.build.build()")
    L = ct.CDLL(LIB_PATH)
    P, I, D, LL, SZ = ct.c_void_p, ct.c_int, ct.c_double, ct.c_longlong, ct.c_size_t
    IA6 = ct.POINTER(ct.c_int)
    PP = ct.POINTER(Params)
    L.rad_default_params.argtypes = [PP]
    L.rad_default_params.restype = None
    L.rad_workspace_bytes.argtypes = [I, I, I, PP]
    L.rad_workspace_bytes.restype = SZ
    L.rad_step.argtypes = [I, I, I, P, P, P, P, P, P, P, D, D, IA6, PP, P, SZ, P, ct.POINTER(Stats)]
    L.rad_step.restype = I
    L.rad_workspace_bytes_moving.argtypes = [I, I, I, PP]
    L.rad_workspace_bytes_moving.restype = SZ
    L.rad_noalloc_max_bytes.argtypes = []
    L.rad_noalloc_max_bytes.restype = SZ
    L.rad_step_noalloc.argtypes = [I, I, I, P, P, P, P, P, P, P, D, D, IA6, PP, P, ct.POINTER(Stats)]
    L.rad_step_noalloc.restype = I
    L.rad_step_moving.argtypes = [I, I, I, P, P, P, P, P, P, P, P, D, D, IA6, PP, P, SZ, P, ct.POINTER(Stats)]
    L.rad_step_moving.restype = I
    L.rad_workspace_bytes_amr2.argtypes = [ct.POINTER(Amr2), PP]
    L.rad_workspace_bytes_amr2.restype = SZ
    L.rad_step_amr2.argtypes = [ct.POINTER(Amr2), P, P, P, P, P, P, P, D, D, IA6, PP, P, SZ, P, ct.POINTER(Stats)]
    L.rad_step_amr2.restype = I
    L.rad_residual.argtypes = [I, I, I, P, P, P, P, P, P, P, P, P, P, D, D, IA6, PP, P, P]
    L.rad_residual.restype = I
    L.rad_face_speeds.argtypes = [I, I, I, P, P, P, D, IA6, PP, P, P]
    L.rad_face_speeds.restype = I
    L.rad_apply.argtypes = [I, I, I, P, P, P, P, P, P, D, D, IA6, PP, I, P]
    L.rad_apply.restype = I
    L.rad_exchange.argtypes = [LL, P, P, P, P, P, D, PP, P]
    L.rad_exchange.restype = I
    L.rad_batched_workspace_bytes.argtypes = [I, ct.POINTER(BlockDesc), PP]
    L.rad_batched_workspace_bytes.restype = SZ
    L.rad_plan_batched.argtypes = [I, ct.POINTER(BlockDesc), PP, P, SZ, P, ct.POINTER(P)]
    L.rad_plan_batched.restype = I
    L.rad_autotune_scratch_bytes.argtypes = [P]
    L.rad_autotune_scratch_bytes.restype = SZ
    L.rad_autotune_batched.argtypes = [P, P, P, P, P, P, P, P, P, SZ, P]
    L.rad_autotune_batched.restype = I
    L.rad_step_batched.argtypes = [P, P, P, P, P, P, P, P, P, P]
    L.rad_step_batched.restype = I
    L.rad_autotune_step.argtypes = [I, I, I, P, P, P, P, P, P, P, D, D, IA6, PP, P, SZ, P, I,
                                    ct.POINTER(I), ct.POINTER(I), ct.POINTER(I), ct.POINTER(I)]
    L.rad_autotune_step.restype = I
    L.rad_closure.argtypes = [ct.c_longlong, P, P, I, ct.c_double, P, I, P]
    L.rad_closure.restype = I
    L.rad_plan_launch_shape.argtypes = [P, ct.POINTER(I), ct.POINTER(I), ct.POINTER(I)]
    L.rad_plan_launch_shape.restype = I
    L.rad_plan_reorder.argtypes = [P, P, P]
    L.rad_plan_reorder.restype = I
    L.rad_plan_destroy.argtypes = [P]
    L.rad_plan_destroy.restype = None
    L.rad_profile_enable.argtypes = [I]
    L.rad_profile_enable.restype = None
    L.rad_profile_reset.argtypes = []
    L.rad_profile_reset.restype = None
    L.rad_profile_count.argtypes = []
    L.rad_profile_count.restype = I
    L.rad_profile_get.argtypes = [I, ct.POINTER(ct.c_char_p), ct.POINTER(D), ct.POINTER(D), ct.POINTER(LL)]
    L.rad_profile_get.restype = I
    L.rad_last_error.argtypes = []
    L.rad_last_error.restype = ct.c_char_p
    L.rad_build_id.argtypes = []
    L.rad_build_id.restype = ct.c_char_p
    from .build import source_id
    built, here = L.rad_build_id().decode(), source_id()
    if built != here:
        raise ImportError(f"{LIB_PATH} was built from other sources (build id {built}, sources {here}): "
                          "rebuild it with paper_2202_08778_amd.build.build()")
    return L


lib = _load()

EXPORTED = ("rad_default_params", "rad_workspace_bytes", "rad_step", "rad_noalloc_max_bytes", "rad_step_noalloc",
            "rad_workspace_bytes_moving", "rad_step_moving",
            "rad_workspace_bytes_amr2", "rad_step_amr2",
            "rad_autotune_step", "rad_residual",
            "rad_face_speeds",
            "rad_apply", "rad_exchange", "rad_closure", "rad_batched_workspace_bytes", "rad_plan_batched",
            "rad_autotune_scratch_bytes", "rad_autotune_batched", "rad_step_batched", "rad_plan_launch_shape",
            "rad_plan_reorder", "rad_plan_destroy",
            "rad_profile_enable", "rad_profile_reset", "rad_profile_count", "rad_profile_get", "rad_last_error",
            "rad_build_id")


def last_error() -> str:
    return lib.rad_last_error().decode()


def params(**kw) -> Params:
    """rad_params_t with library defaults, overridden by keyword (strings accepted for enums)."""
    p = Params()
    lib.rad_default_params(ct.byref(p))
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PREC[v]
        elif k == "mode" and isinstance(v, str):
            v = MODE[v]
        elif k == "coef_dtype" and isinstance(v, str):
            v = DTYPE[v]
        elif k == "F_inc":
            v = (ct.c_double * 6)(*([float(v)] * 6 if isinstance(v, (int, float)) else [float(x) for x in v]))
        setattr(p, k, v)
    return p


def bc_array(bc):
    if isinstance(bc, str):
        bc = (bc,) * 6
    if len(bc) == 3:
        bc = (bc[0], bc[0], bc[1], bc[1], bc[2], bc[2])
    return (ct.c_int * 6)(*[BC[b] if isinstance(b, str) else int(b) for b in bc])


def _check(rc, allow=(RAD_OK,)):
    if rc not in allow:
        raise RadError(rc, last_error())
    return rc


# ------------------------------------------------------------ torch marshalling

def _torch():
    import torch
    return torch


def _ptr(t, dtype=None, numel=None, name="tensor"):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _coef_dtype(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return 0
    if t.dtype == torch.float32:
        return 1
    raise TypeError("coefficients must be float64 or float32")


def _set_ghost(p, ghost, shape):
    """Point p.ghost at the Dirichlet faces' ghost data: a sequence of six entries (faces -x,+x,-y,+y,-z,+z),
    each None or a contiguous float64 device tensor of (E, F_x, F_y, F_z) over the face's cells -- shape
    (4, nz, ny) for x faces, (4, nz, nx) for y faces, (4, ny, nx) for z faces.  The tensors must outlive the
    call."""
    if ghost is None:
        return
    torch = _torch()
    nz, ny, nx = shape
    if len(ghost) != 6:
        raise ValueError("ghost: one entry per face (-x,+x,-y,+y,-z,+z)")
    area = (ny * nz, nx * nz, nx * ny)
    for fi, t in enumerate(ghost):
        p.ghost[fi] = None if t is None else _ptr(t, torch.float64, 4 * area[fi // 2], f"ghost[{fi}]")


def workspace_bytes(shape, p: Params) -> int:
    nz, ny, nx = shape
    return int(lib.rad_workspace_bytes(nx, ny, nz, ct.byref(p)))


def alloc_workspace(nbytes, device=None):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def rad_step(E, F, T, rho, kappa_P, kappa_R, f, dt, dx, bc, p: Params, workspace=None, stream=None,
             check=True, ghost=None):
    """One implicit step in place on device tensors E (nz,ny,nx), F (3,...), T (...) (float64);
    rho, kappa_P, kappa_R, f (6,...) of one float dtype; ghost: the Dirichlet faces' data (see _set_ghost).
    Returns the stats dict."""
    torch = _torch()
    nz, ny, nx = E.shape
    N = nx * ny * nz
    p = Params.from_buffer_copy(p)
    _set_ghost(p, ghost, E.shape)
    p.coef_dtype = _coef_dtype(rho)
    cd = rho.dtype
    args = [_ptr(E, torch.float64, N, "E"), _ptr(F, torch.float64, 3 * N, "F"), _ptr(T, torch.float64, N, "T"),
            _ptr(rho, cd, N, "rho"), _ptr(kappa_P, cd, N, "kappa_P"), _ptr(kappa_R, cd, N, "kappa_R"),
            _ptr(f, cd, 6 * N, "f")]
    need = int(lib.rad_workspace_bytes(nx, ny, nz, ct.byref(p)))
    if workspace is None:
        workspace = alloc_workspace(need, E.device)
    st = Stats()
    rc = lib.rad_step(nx, ny, nz, *args, float(dt), float(dx), bc_array(bc), ct.byref(p),
                      _ptr(workspace, name="workspace"), workspace.numel() * workspace.element_size(),
                      _stream(stream), ct.byref(st))
    if check:
        _check(rc)
    d = st.as_dict()
    d["rc"] = rc
    return d


def rad_step_noalloc(E, F, T, rho, kappa_P, kappa_R, f, dt, dx, bc, p: Params, stream=None, check=True, ghost=None):
    """rad_step with the library's static device scratch as the workspace (no allocation in the call;
    grids whose workspace exceeds rad_noalloc_max_bytes() are refused with RAD_ENOMEM)."""
    torch = _torch()
    nz, ny, nx = E.shape
    N = nx * ny * nz
    p = Params.from_buffer_copy(p)
    _set_ghost(p, ghost, E.shape)
    p.coef_dtype = _coef_dtype(rho)
    cd = rho.dtype
    args = [_ptr(E, torch.float64, N, "E"), _ptr(F, torch.float64, 3 * N, "F"), _ptr(T, torch.float64, N, "T"),
            _ptr(rho, cd, N, "rho"), _ptr(kappa_P, cd, N, "kappa_P"), _ptr(kappa_R, cd, N, "kappa_R"),
            _ptr(f, cd, 6 * N, "f")]
    st = Stats()
    rc = lib.rad_step_noalloc(nx, ny, nz, *args, float(dt), float(dx), bc_array(bc), ct.byref(p), _stream(stream),
                              ct.byref(st))
    if check:
        _check(rc)
    d = st.as_dict()
    d["rc"] = rc
    return d


def rad_step_moving(E, F, T, rho, kappa_P, kappa_R, f, beta, dt, dx, bc, p: Params, workspace=None, stream=None,
                    check=True, ghost=None):
    """rad_step in a moving medium: beta = v/c as a (3, nz, ny, nx) tensor of the coefficients' dtype
    (held fixed over the step); p.vel_implicit selects the implicit O(v/c) gas-energy term."""
    torch = _torch()
    nz, ny, nx = E.shape
    N = nx * ny * nz
    p = Params.from_buffer_copy(p)
    _set_ghost(p, ghost, E.shape)
    p.coef_dtype = _coef_dtype(rho)
    cd = rho.dtype
    args = [_ptr(E, torch.float64, N, "E"), _ptr(F, torch.float64, 3 * N, "F"), _ptr(T, torch.float64, N, "T"),
            _ptr(rho, cd, N, "rho"), _ptr(kappa_P, cd, N, "kappa_P"), _ptr(kappa_R, cd, N, "kappa_R"),
            _ptr(f, cd, 6 * N, "f"), _ptr(beta, cd, 3 * N, "beta")]
    if workspace is None:
        workspace = alloc_workspace(int(lib.rad_workspace_bytes_moving(nx, ny, nz, ct.byref(p))), E.device)
    st = Stats()
    rc = lib.rad_step_moving(nx, ny, nz, *args, float(dt), float(dx), bc_array(bc), ct.byref(p),
                             _ptr(workspace, name="workspace"), workspace.numel() * workspace.element_size(),
                             _stream(stream), ct.byref(st))
    if check:
        _check(rc)
    d = st.as_dict()
    d["rc"] = rc
    return d


def amr_geometry(coarse_shape, lo, hi) -> Amr2:
    """rad_amr2_t of a coarse grid (nx, ny, nz) with the box [lo, hi) (coarse cells, x, y, z) refined by 2."""
    g = Amr2()
    g.nx, g.ny, g.nz = (int(v) for v in coarse_shape)
    for d in range(3):
        g.lo[d], g.hi[d] = int(lo[d]), int(hi[d])
    return g


def amr_pack(coarse, fine, comps=1):
    """Two-level layout of one field: the coarse level's planes, then the fine level's (flat, contiguous)."""
    torch = _torch()
    assert coarse.numel() % comps == 0 and fine.numel() % comps == 0
    return torch.cat([coarse.reshape(-1), fine.reshape(-1)]).contiguous()


def amr_unpack(flat, geom: Amr2, comps=1):
    """(coarse, fine) views of a two-level array: shapes (comps,) + (nz, ny, nx) and (comps,) + fine extents."""
    nc = (geom.nz, geom.ny, geom.nx)
    nf = tuple(2 * (geom.hi[d] - geom.lo[d]) for d in (2, 1, 0))
    Nc = nc[0] * nc[1] * nc[2]
    lead = (comps,) if comps > 1 else ()
    return flat[:comps * Nc].reshape(lead + nc), flat[comps * Nc:].reshape(lead + nf)


def workspace_bytes_amr2(geom: Amr2, p: Params) -> int:
    return int(lib.rad_workspace_bytes_amr2(ct.byref(geom), ct.byref(p)))


def rad_step_amr2(geom: Amr2, E, F, T, rho, kappa_P, kappa_R, f, dt, dx, bc, p: Params, workspace=None,
                  stream=None, check=True):
    """One implicit step on a two-level grid, in place on flat device tensors in the two-level
    layout (amr_pack): E, T (N), F (3N) float64; rho, kappa_P, kappa_R (N), f (6N) of one float dtype,
    N = coarse cells + fine cells.  dx: the coarse cell width.  Returns the stats dict."""
    torch = _torch()
    N = geom.nx * geom.ny * geom.nz + 8 * (geom.hi[0] - geom.lo[0]) * (geom.hi[1] - geom.lo[1]) * \
        (geom.hi[2] - geom.lo[2])
    p = Params.from_buffer_copy(p)
    p.coef_dtype = _coef_dtype(rho)
    cd = rho.dtype
    args = [_ptr(E, torch.float64, N, "E"), _ptr(F, torch.float64, 3 * N, "F"), _ptr(T, torch.float64, N, "T"),
            _ptr(rho, cd, N, "rho"), _ptr(kappa_P, cd, N, "kappa_P"), _ptr(kappa_R, cd, N, "kappa_R"),
            _ptr(f, cd, 6 * N, "f")]
    if workspace is None:
        need = workspace_bytes_amr2(geom, p)
        if need == 0:   # invalid geometry or params: let the library name the reason
            _check(lib.rad_step_amr2(ct.byref(geom), *args, float(dt), float(dx), bc_array(bc), ct.byref(p), None, 0,
                                     None, None))
        workspace = alloc_workspace(need, E.device)
    st = Stats()
    rc = lib.rad_step_amr2(ct.byref(geom), *args, float(dt), float(dx), bc_array(bc), ct.byref(p),
                           _ptr(workspace, name="workspace"), workspace.numel() * workspace.element_size(),
                           _stream(stream), ct.byref(st))
    if check:
        _check(rc)
    d = st.as_dict()
    d["rc"] = rc
    return d


def autotune_step(E, F, T, rho, kappa_P, kappa_R, f, dt, dx, bc, p: Params, tune_restart=True, workspace=None,
                  stream=None, ghost=None):
    """Autotune rad_step on this data (state left unchanged): returns {"kz_apply", "kz_residual", "gmres_m",
    "krylov_poly"}.  The z-ranges are cached and used by later rad_step calls; gmres_m and krylov_poly are
    recommendations."""
    torch = _torch()
    nz, ny, nx = E.shape
    N = nx * ny * nz
    p = Params.from_buffer_copy(p)
    _set_ghost(p, ghost, E.shape)
    p.coef_dtype = _coef_dtype(rho)
    cd = rho.dtype
    args = [_ptr(E, torch.float64, N, "E"), _ptr(F, torch.float64, 3 * N, "F"), _ptr(T, torch.float64, N, "T"),
            _ptr(rho, cd, N, "rho"), _ptr(kappa_P, cd, N, "kappa_P"), _ptr(kappa_R, cd, N, "kappa_R"),
            _ptr(f, cd, 6 * N, "f")]
    if workspace is None:
        workspace = alloc_workspace(int(lib.rad_workspace_bytes(nx, ny, nz, ct.byref(p))), E.device)
    ka, kr, m, kp = ct.c_int(), ct.c_int(), ct.c_int(), ct.c_int()
    _check(lib.rad_autotune_step(nx, ny, nz, *args, float(dt), float(dx), bc_array(bc), ct.byref(p),
                                 _ptr(workspace, name="workspace"), workspace.numel() * workspace.element_size(),
                                 _stream(stream), 1 if tune_restart else 0, ct.byref(ka), ct.byref(kr), ct.byref(m),
                                 ct.byref(kp)))
    return {"kz_apply": ka.value, "kz_residual": kr.value, "gmres_m": m.value, "krylov_poly": kp.value}


def rad_residual(En, Fn, Tn, E, F, T, rho, kappa_P, kappa_R, f, dt, dx, bc, p: Params, R=None, stream=None,
                 ghost=None):
    """Nonlinear residual (5, nz, ny, nx) float64 of a state; asynchronous on the stream."""
    torch = _torch()
    nz, ny, nx = E.shape
    N = nx * ny * nz
    p = Params.from_buffer_copy(p)
    _set_ghost(p, ghost, E.shape)
    p.coef_dtype = _coef_dtype(rho)
    cd = rho.dtype
    if R is None:
        R = torch.empty((5, nz, ny, nx), dtype=torch.float64, device=E.device)
    f64 = torch.float64
    _check(lib.rad_residual(nx, ny, nz, _ptr(En, f64, N, "En"), _ptr(Fn, f64, 3 * N, "Fn"),
                            _ptr(Tn, f64, N, "Tn"), _ptr(E, f64, N, "E"), _ptr(F, f64, 3 * N, "F"),
                            _ptr(T, f64, N, "T"), _ptr(rho, cd, N, "rho"), _ptr(kappa_P, cd, N, "kappa_P"),
                            _ptr(kappa_R, cd, N, "kappa_R"), _ptr(f, cd, 6 * N, "f"), float(dt), float(dx),
                            bc_array(bc), ct.byref(p), _ptr(R, f64, 5 * N, "R"), _stream(stream)))
    return R


def rad_face_speeds(rho, kappa_R, f, dx, bc, p: Params, C=None, stream=None):
    torch = _torch()
    nz, ny, nx = rho.shape
    N = nx * ny * nz
    p = Params.from_buffer_copy(p)
    p.coef_dtype = _coef_dtype(rho)
    cd = rho.dtype
    if C is None:
        C = torch.empty((3, nz, ny, nx), dtype=torch.float64, device=rho.device)
    _check(lib.rad_face_speeds(nx, ny, nz, _ptr(rho, cd, N, "rho"), _ptr(kappa_R, cd, N, "kappa_R"),
                               _ptr(f, cd, 6 * N, "f"), float(dx), bc_array(bc), ct.byref(p),
                               _ptr(C, torch.float64, 3 * N, "C"), _stream(stream)))
    return C


def rad_apply(x, dE, rho, kappa_R, f, dt, dx, bc, p: Params, y=None, stream=None):
    """y = A x for x (4, nz, ny, nx) of float64 or float32 (physical units)."""
    torch = _torch()
    _, nz, ny, nx = x.shape
    N = nx * ny * nz
    p = Params.from_buffer_copy(p)
    p.coef_dtype = _coef_dtype(rho)
    cd = rho.dtype
    dt_code = 0 if x.dtype == torch.float64 else 1
    if y is None:
        y = torch.empty_like(x)
    _check(lib.rad_apply(nx, ny, nz, _ptr(x, x.dtype, 4 * N, "x"), _ptr(y, x.dtype, 4 * N, "y"),
                         _ptr(dE, x.dtype, N, "dE"), _ptr(rho, cd, N, "rho"), _ptr(kappa_R, cd, N, "kappa_R"),
                         _ptr(f, cd, 6 * N, "f"), float(dt), float(dx), bc_array(bc), ct.byref(p), dt_code,
                         _stream(stream)))
    return y


def rad_exchange(E, Tn, rho, kappa_P, dt, p: Params, T=None, stream=None):
    torch = _torch()
    n = E.numel()
    p = Params.from_buffer_copy(p)
    p.coef_dtype = _coef_dtype(rho)
    cd = rho.dtype
    if T is None:
        T = torch.empty_like(E)
    f64 = torch.float64
    _check(lib.rad_exchange(n, _ptr(E, f64, n, "E"), _ptr(Tn, f64, n, "Tn"), _ptr(T, f64, n, "T"),
                            _ptr(rho, cd, n, "rho"), _ptr(kappa_P, cd, n, "kappa_P"), float(dt), ct.byref(p),
                            _stream(stream)))
    return T


CLOSURE = {"eddington": 0, "m1": 1}


def rad_closure(E, F, kind="m1", c=1.0, out_dtype=None, f=None, stream=None):
    """Eddington tensor of a local closure (Sec. 4.1) from the lagged (E, F): returns f_ij with shape
    (6,) + E.shape (planes xx, yy, zz, xy, xz, yz) in out_dtype (float64 default, or float32)."""
    torch = _torch()
    n = E.numel()
    f64 = torch.float64
    if f is None:
        f = torch.empty((6,) + tuple(E.shape), dtype=out_dtype or f64, device=E.device)
    od = 0 if f.dtype == f64 else 1
    _check(lib.rad_closure(n, _ptr(E, f64, n, "E"), _ptr(F, f64, 3 * n, "F"), CLOSURE[kind], float(c),
                           _ptr(f, f.dtype, 6 * n, "f"), od, _stream(stream)))
    return f


def profile(on=True):
    """on: False/0 off, True/1 every kernel class timed, 2 only the operator applies timed."""
    lib.rad_profile_enable(2 if on == 2 else (1 if on else 0))


def profile_reset():
    lib.rad_profile_reset()


def profile_read():
    """{kernel class: {"ms", "bytes", "launches"}} accumulated since the last reset."""
    out = {}
    for i in range(lib.rad_profile_count()):
        name, ms, b, n = ct.c_char_p(), ct.c_double(), ct.c_double(), ct.c_longlong()
        _check(lib.rad_profile_get(i, ct.byref(name), ct.byref(ms), ct.byref(b), ct.byref(n)))
        out[name.value.decode()] = {"ms": ms.value, "bytes": b.value, "launches": n.value}
    return out


# ------------------------------------------------------------------ batched

STATS_DTYPE = None


def _stats_dtype():
    import numpy as np
    global STATS_DTYPE
    if STATS_DTYPE is None:
        STATS_DTYPE = np.dtype([(k, np.int32 if t is ct.c_int else np.float64) for k, t in Stats._fields_])
        assert STATS_DTYPE.itemsize == ct.sizeof(Stats)
    return STATS_DTYPE


def pack_blocks(blocks):
    """Pack per-block padded arrays ((n+2ng)^3 each, from workloads.batched_blocks) into arenas.

    Returns (descs: BlockDesc array, arenas: dict of numpy arrays E (A), F (3, A), T, rho, kP, kR (A),
    f (6, A)) with block b's region at element offset descs[b].off of every arena."""
    import numpy as np
    nb = len(blocks)
    descs = (BlockDesc * nb)()
    off = 0
    for b, blk in enumerate(blocks):
        m = blk["n"] + 2 * blk["ng"]
        descs[b].n, descs[b].ng, descs[b].dx, descs[b].dt, descs[b].off = blk["n"], blk["ng"], blk["dx"], blk["dt"], off
        off += m ** 3
    A = off
    ar = {"E": np.empty(A), "F": np.empty((3, A)), "T": np.empty(A), "rho": np.empty(A), "kP": np.empty(A),
          "kR": np.empty(A), "f": np.empty((6, A))}
    for b, blk in enumerate(blocks):
        o, sz = descs[b].off, (blk["n"] + 2 * blk["ng"]) ** 3
        for k in ("E", "T", "rho", "kP", "kR"):
            ar[k][o:o + sz] = blk[k].ravel()
        for q in range(3):
            ar["F"][q, o:o + sz] = blk["F"][q].ravel()
        for q in range(6):
            ar["f"][q, o:o + sz] = blk["f"][q].ravel()
    return descs, ar


class Plan:
    """A batched plan: owns its device workspace (a torch tensor) and the library plan handle."""

    def __init__(self, descs, p: Params, device="cuda", stream=None):
        self.descs = descs
        self.nblocks = len(descs)
        self.p = Params.from_buffer_copy(p)
        need = int(lib.rad_batched_workspace_bytes(self.nblocks, descs, ct.byref(self.p)))
        if need == 0:
            _check(RAD_EINVAL if not last_error() else -1)
        self.workspace = alloc_workspace(need, device)
        h = ct.c_void_p()
        _check(lib.rad_plan_batched(self.nblocks, descs, ct.byref(self.p), _ptr(self.workspace, name="workspace"),
                                    self.workspace.numel(), _stream(stream), ct.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:
            try:
                lib.rad_plan_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None

    def _args(self, E, F, T, rho, kP, kR, f):
        torch = _torch()
        A = E.numel()
        cd = rho.dtype
        f64 = torch.float64
        return [_ptr(E, f64, A, "E"), _ptr(F, f64, 3 * A, "F"), _ptr(T, f64, A, "T"), _ptr(rho, cd, A, "rho"),
                _ptr(kP, cd, A, "kappa_P"), _ptr(kR, cd, A, "kappa_R"), _ptr(f, cd, 6 * A, "f")]

    def autotune(self, E, F, T, rho, kP, kR, f, stream=None):
        n = int(lib.rad_autotune_scratch_bytes(self.handle))
        scratch = alloc_workspace(n, E.device)
        _check(lib.rad_autotune_batched(self.handle, *self._args(E, F, T, rho, kP, kR, f),
                                        _ptr(scratch, name="scratch"), scratch.numel(), _stream(stream)))
        _torch().cuda.synchronize()

    def step(self, E, F, T, rho, kP, kR, f, stats=None, stream=None):
        """One step of every block (asynchronous).  Returns the device stats buffer (uint8 tensor)."""
        torch = _torch()
        if stats is None:
            stats = torch.empty(self.nblocks * ct.sizeof(Stats), dtype=torch.uint8, device=E.device)
        _check(lib.rad_step_batched(self.handle, *self._args(E, F, T, rho, kP, kR, f),
                                    _ptr(stats, name="stats"), _stream(stream)))
        return stats

    def reorder(self, stats, stream=None):
        """Queue the blocks longest measured solve first, from the stats buffer of an earlier step."""
        _check(lib.rad_plan_reorder(self.handle, _ptr(stats, name="stats"), _stream(stream)))

    def launch_shape(self):
        """(threads per workgroup, workgroups per CU, largest-first queue) of the plan's launch."""
        t, c, l = ct.c_int(), ct.c_int(), ct.c_int()
        _check(lib.rad_plan_launch_shape(self.handle, ct.byref(t), ct.byref(c), ct.byref(l)))
        return t.value, c.value, bool(l.value)

    @staticmethod
    def read_stats(stats):
        import numpy as np
        return np.frombuffer(stats.cpu().numpy().tobytes(), dtype=_stats_dtype())
