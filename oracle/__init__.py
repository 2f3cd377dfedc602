"""Plain FP64 CPU oracle for the implicit VET radiation step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library.  The arithmetic lives in ``oracle.c``; this module only
pads arrays, fills in the structs and calls it.

Array conventions: a scalar field is a float64 array of shape (nz, ny, nx)
(x fastest); F has shape (3, nz, ny, nx); the Eddington tensor f has shape
(6, nz, ny, nx) in the order xx, yy, zz, xy, xz, yz.  With ``padded=True``
every spatial extent carries one ghost layer on each side and the ghosts of
Dirichlet faces hold the boundary data.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.environ.get("VETTAM_ORACLE_SO") or os.path.join(_HERE, "liboracle.so")
_lib = None

BC = {"periodic": 0, "outflow": 1, "dirichlet": 2, "open": 3, "marshak": 4, "reflect": 5}
MODE = {"lagged": 0, "linearised": 1}


def build() -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _SO, src, "-lm"]
    subprocess.run(cmd, check=True)
    return _SO


class _Grid(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
                ("h", ct.c_double), ("dt", ct.c_double), ("c", ct.c_double),
                ("aR", ct.c_double), ("cv", ct.c_double), ("bc", ct.c_int * 6), ("cv_cubic", ct.c_int),
                ("finc", ct.c_double * 6)]


class _Coef(ct.Structure):
    _fields_ = [("rho", ct.c_void_p), ("kP", ct.c_void_p), ("kR", ct.c_void_p),
                ("f", ct.c_void_p * 6), ("beta", ct.c_void_p * 3), ("vel_implicit", ct.c_int)]


class _Params(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("lin_rtol", ct.c_double), ("max_picard", ct.c_int),
                ("gmres_m", ct.c_int), ("max_krylov", ct.c_int), ("mode", ct.c_int),
                ("eps_P", ct.c_double), ("eps_N", ct.c_double), ("energy_fix", ct.c_int)]


class _Stats(ct.Structure):
    _fields_ = [("picard_iters", ct.c_int), ("krylov_iters", ct.c_int), ("converged", ct.c_int),
                ("neg_cells", ct.c_int), ("scaled_residual", ct.c_double), ("res_E", ct.c_double),
                ("res_F", ct.c_double), ("res_T", ct.c_double), ("rel_change", ct.c_double),
                ("energy_defect", ct.c_double), ("dE_max", ct.c_double)]


def lib():
    global _lib
    if _lib is None:
        stale = not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(os.path.join(_HERE, "oracle.c"))
        if stale and not os.environ.get("VETTAM_ORACLE_SO"):
            build()
        L = ct.CDLL(_SO)
        P = ct.c_void_p
        L.or_fill_ghosts.argtypes = [ct.POINTER(_Grid), P]
        L.or_fill_tensor_ghosts.argtypes = [ct.POINTER(_Grid), ct.POINTER(P)]
        L.or_fill_state_ghosts.argtypes = [ct.POINTER(_Grid), ct.POINTER(_Coef), ct.POINTER(P), ct.c_void_p,
                                           ct.c_int]
        L.or_face_speeds.argtypes = [ct.POINTER(_Grid), ct.POINTER(_Coef), P, P, P]
        L.or_apply.argtypes = [ct.POINTER(_Grid), ct.POINTER(_Coef), P, ct.POINTER(P), ct.POINTER(P)]
        L.or_residual.argtypes = [ct.POINTER(_Grid), ct.POINTER(_Coef), P, ct.POINTER(P), P, P,
                                  ct.POINTER(P), P, ct.POINTER(P)]
        L.or_scaled_residual.argtypes = [ct.POINTER(_Grid), ct.POINTER(_Coef), P, ct.POINTER(P), P, P,
                                         ct.POINTER(P), P, ct.POINTER(ct.c_double)]
        L.or_exchange_T.argtypes = [ct.c_double] * 5 + [ct.POINTER(ct.c_int)]
        L.or_exchange_T.restype = ct.c_double
        L.or_rad_step.argtypes = [ct.POINTER(_Grid), ct.POINTER(_Coef), ct.POINTER(_Params), P,
                                  ct.POINTER(P), P, ct.POINTER(_Stats)]
        L.or_rad_step.restype = ct.c_int
        L.or_num_threads.restype = ct.c_int
        L.or_closure.argtypes = [ct.c_long, ct.c_int, ct.c_double] + [ct.c_void_p] * 5
        L.or_closure.restype = None
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


# ----------------------------------------------------------------- helpers

def _bc_codes(bc):
    if isinstance(bc, str):
        bc = (bc,) * 6
    if len(bc) == 3:
        bc = (bc[0], bc[0], bc[1], bc[1], bc[2], bc[2])
    codes = [BC[b] if isinstance(b, str) else int(b) for b in bc]
    for a in range(3):
        if (codes[2 * a] == 0) != (codes[2 * a + 1] == 0):
            raise ValueError("periodic faces must come in pairs")
    return codes


def _pad(a):
    """Interior (..., nz, ny, nx) -> padded float64 copy with zero ghosts."""
    a = np.asarray(a, dtype=np.float64)
    pw = [(0, 0)] * (a.ndim - 3) + [(1, 1)] * 3
    return np.ascontiguousarray(np.pad(a, pw))


def _interior(a):
    return np.ascontiguousarray(a[..., 1:-1, 1:-1, 1:-1])


class Problem:
    """Grid, constants and coefficient fields of one implicit step (padded internally)."""

    def __init__(self, rho, kP, kR, f, dt, dx, bc="periodic", c=1.0, aR=1.0, cv=1.0, padded=False, beta=None,
                 vel_implicit=False, cv_cubic=False, finc=None):
        """beta: gas velocity over c, shape (3,) + field shape (None: v = 0); vel_implicit: the O(v/c)
        gas-energy term implicit (else left to the explicit hydro update, the paper's default);
        cv_cubic: heat capacity rho cv T^3 (E_int = rho cv T^4 / 4) instead of rho cv.
        bc: one kind for all faces, three (per axis) or six (-x,+x,-y,+y,-z,+z) of periodic,
        outflow, dirichlet, open, marshak, reflect; finc: the incident flux of each Marshak face
        (six values, or one for all)."""
        self.padded = padded
        P = (lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64))) if padded else _pad
        self.rho, self.kP, self.kR = P(rho), P(kP), P(kR)
        self.f = P(f)
        self.beta = None if beta is None else P(beta)
        nzp, nyp, nxp = self.rho.shape
        self.shape = (nzp - 2, nyp - 2, nxp - 2)
        g = _Grid()
        g.nz, g.ny, g.nx = self.shape
        g.h, g.dt, g.c, g.aR, g.cv = float(dx), float(dt), float(c), float(aR), float(cv)
        for i, code in enumerate(_bc_codes(bc)):
            g.bc[i] = code
        g.cv_cubic = 1 if cv_cubic else 0
        fi = [0.0] * 6 if finc is None else ([float(finc)] * 6 if np.isscalar(finc) else [float(v) for v in finc])
        for i in range(6):
            g.finc[i] = fi[i]
        self.g = g
        self.c, self.aR, self.cv, self.dt, self.dx = float(c), float(aR), float(cv), float(dt), float(dx)
        L = lib()
        for a in (self.rho, self.kP, self.kR, *(self.beta if self.beta is not None else ())):
            L.or_fill_ghosts(ct.byref(g), a.ctypes.data)
        L.or_fill_tensor_ghosts(ct.byref(g), (ct.c_void_p * 6)(*(self.f[q].ctypes.data for q in range(6))))
        cf = _Coef()
        cf.rho, cf.kP, cf.kR = self.rho.ctypes.data, self.kP.ctypes.data, self.kR.ctypes.data
        for q in range(6):
            cf.f[q] = self.f[q].ctypes.data
        for q in range(3):
            cf.beta[q] = None if self.beta is None else self.beta[q].ctypes.data
        cf.vel_implicit = 1 if vel_implicit else 0
        self.cf = cf

    # padded state helpers -------------------------------------------------
    def state(self, E, F, T):
        if self.padded:
            c = lambda a: np.array(a, dtype=np.float64, order="C", copy=True)
            return c(E), c(F), c(T)
        return _pad(E), _pad(F), _pad(T)

    def out(self, a):
        return a.copy() if self.padded else _interior(a)

    def face_speeds(self):
        """(Cx, Cy, Cz) padded; Cd[k,j,i] is the speed of the low d-face of cell (i,j,k)."""
        C = [np.zeros_like(self.rho) for _ in range(3)]
        lib().or_face_speeds(ct.byref(self.g), ct.byref(self.cf), *(a.ctypes.data for a in C))
        return C

    def apply(self, x, dE):
        """y = dE*E + (dt/h) div Phi (E rows), (1+sR) F + (dt/h) div Phi (F rows).

        x: (4, nz, ny, nx) interior (ghosts filled as for the linear operator: the face
        conditions with their data dropped) unless the problem is padded, in which case x is
        padded and its ghosts are used as given."""
        if self.padded:
            xp = np.array(x, dtype=np.float64, copy=True)
            dEp = np.ascontiguousarray(dE, dtype=np.float64)
        else:
            xp = _pad(x)
            dEp = _pad(dE)
            XG = (ct.c_void_p * 4)(*(xp[q].ctypes.data for q in range(4)))
            lib().or_fill_state_ghosts(ct.byref(self.g), ct.byref(self.cf), XG, None, 1)
        yp = np.zeros_like(xp)
        XP = (ct.c_void_p * 4)(*(xp[q].ctypes.data for q in range(4)))
        YP = (ct.c_void_p * 4)(*(yp[q].ctypes.data for q in range(4)))
        lib().or_apply(ct.byref(self.g), ct.byref(self.cf), dEp.ctypes.data, XP, YP)
        return self.out(yp)

    def residual(self, En, Fn, Tn, E, F, T):
        """Nonlinear residual (R_E, R_Fx, R_Fy, R_Fz, R_T) of the backward-Euler system."""
        En, Fn, Tn = self.state(En, Fn, Tn)
        E, F, T = self.state(E, F, T)
        R = np.zeros((5,) + E.shape)
        A = lambda arr: (ct.c_void_p * len(arr))(*(a.ctypes.data for a in arr))
        lib().or_residual(ct.byref(self.g), ct.byref(self.cf), En.ctypes.data, A(list(Fn)), Tn.ctypes.data,
                          E.ctypes.data, A(list(F)), T.ctypes.data, A(list(R)))
        return self.out(R)

    def scaled_residual(self, En, Fn, Tn, E, F, T):
        """(res_E, res_F, res_T, max) scaled residual norms of a state."""
        En, Fn, Tn = self.state(En, Fn, Tn)
        E, F, T = self.state(E, F, T)
        out = (ct.c_double * 4)()
        A = lambda arr: (ct.c_void_p * len(arr))(*(a.ctypes.data for a in arr))
        lib().or_scaled_residual(ct.byref(self.g), ct.byref(self.cf), En.ctypes.data, A(list(Fn)),
                                 Tn.ctypes.data, E.ctypes.data, A(list(F)), T.ctypes.data, out)
        return tuple(out)

    def step(self, E, F, T, tol=1e-13, mode="linearised", max_picard=200, gmres_m=100,
             max_krylov=200000, lin_rtol=1e-12, eps_P=0.0, eps_N=0.0, energy_fix=False,
             allow_unconverged=False):
        """One implicit radiation step; returns (E, F, T, stats).  Raises if the nonlinear
        residual neither met tol nor settled at the FP64 floor, unless allow_unconverged.
        eps_P > 0 also stops on the relative change of [E, F, T]; eps_N > 0 stops each
        per-cell Newton solve at that relative change of T; energy_fix commits the gas
        temperature with the energy correction of Sec. 2.3.4."""
        E, F, T = self.state(E, F, T)
        p = _Params()
        p.tol, p.lin_rtol, p.max_picard = tol, lin_rtol, max_picard
        p.gmres_m, p.max_krylov, p.mode, p.eps_P = gmres_m, max_krylov, MODE[mode], eps_P
        p.eps_N, p.energy_fix = eps_N, 1 if energy_fix else 0
        st = _Stats()
        FP = (ct.c_void_p * 3)(*(F[q].ctypes.data for q in range(3)))
        lib().or_rad_step(ct.byref(self.g), ct.byref(self.cf), ct.byref(p), E.ctypes.data, FP,
                          T.ctypes.data, ct.byref(st))
        stats = {k: getattr(st, k) for k, _ in _Stats._fields_}
        if stats["converged"] == 0 and not allow_unconverged:
            raise RuntimeError(f"oracle step did not converge: {stats}")
        return self.out(E), self.out(F), self.out(T), stats


def exchange_T(alpha, Tn, sP, aR, E):
    """Per-cell gas temperature from eq. PicardTemp (scalar)."""
    neg = ct.c_int(0)
    T = lib().or_exchange_T(float(alpha), float(Tn), float(sP), float(aR), float(E), ct.byref(neg))
    return T, bool(neg.value)


CLOSURE = {"eddington": 0, "m1": 1}


def closure(E, F, kind="m1", c=1.0):
    """Local closure of Sec. 4.1 from the time-lagged (E, F): f of shape (6,) + E.shape (xx, yy, zz, xy, xz, yz)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    assert F.shape == (3,) + E.shape
    f = np.empty((6,) + E.shape, dtype=np.float64)
    fp = (ct.c_void_p * 6)(*(f[q].ctypes.data for q in range(6)))
    lib().or_closure(E.size, CLOSURE[kind], float(c), E.ctypes.data, F[0].ctypes.data, F[1].ctypes.data,
                     F[2].ctypes.data, fp)
    return f
