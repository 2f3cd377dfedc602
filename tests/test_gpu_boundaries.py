"""Open (characteristic), Marshak and reflecting walls on the GPU: face speeds, operator apply and
nonlinear residual element by element, and steps per field (<= 1e-10 FP64, <= 1e-8 mixed), against the
oracle on the same seeded inputs; ragged tiles along every axis and mixed wall kinds.  Also the open wall
on the Sec. 3.1 streaming pulse (implicit upwinding on an open line, a closed form)."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2202_08778_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-8


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def rad(torch):
    from paper_2202_08778_amd import rad as r
    return r


def _dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _relerr(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


FINC = [0.7, 0.2, 0.0, 0.4, 0.3, 0.0]

# (name, shape (nz, ny, nx), seed, bc per face -x,+x,-y,+y,-z,+z, crossings per step)
CASES = [
    ("open", (11, 13, 70), 2, ["open"] * 6, 50.0),
    ("open-1d", (1, 1, 90), 3, ["open", "open", "periodic", "periodic", "periodic", "periodic"], 20.0),
    ("marshak-reflect", (3, 4, 67), 4, ["marshak", "reflect", "periodic", "periodic", "periodic", "periodic"], 20.0),
    ("reflect", (9, 10, 12), 5, ["reflect"] * 6, 50.0),
    ("mixed-walls", (10, 9, 66), 6, ["open", "marshak", "outflow", "reflect", "marshak", "open"], 10.0),
]


def _case(name, shape, seed, bc, dt_cross):
    d = W.mixed_depth(shape=shape, seed=seed, steps=1, dt_cross=dt_cross)
    rng = np.random.default_rng(seed + 11)
    d["F"] = 0.05 * rng.standard_normal((3,) + shape) * d["E"]
    d["bc"] = bc
    return d


def _oracle_problem(d):
    return oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"], c=d["c"], aR=d["aR"],
                          cv=d["cv"], finc=FINC)


def _params(rad, d, **kw):
    return rad.params(c=d["c"], a_R=d["aR"], c_v=d["cv"], F_inc=FINC, **kw)


@pytest.mark.parametrize("name,shape,seed,bc,dtc", CASES)
def test_wall_face_speeds(torch, rad, name, shape, seed, bc, dtc):
    _say("wall face speeds", name, shape)
    d = _case(name, shape, seed, bc, dtc)
    Cx, Cy, Cz = _oracle_problem(d).face_speeds()
    want = np.stack([Cx[1:-1, 1:-1, 1:-1], Cy[1:-1, 1:-1, 1:-1], Cz[1:-1, 1:-1, 1:-1]])
    got = rad.rad_face_speeds(_dev(torch, d["rho"]), _dev(torch, d["kR"]), _dev(torch, d["f"]), d["dx"], d["bc"],
                              _params(rad, d)).cpu().numpy()
    assert np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300)) <= 1e-13


@pytest.mark.parametrize("name,shape,seed,bc,dtc", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_wall_operator_apply(torch, rad, name, shape, seed, bc, dtc, prec):
    """The linear operator of a Picard iteration: the walls' ghosts without their data."""
    _say("wall apply", name, shape, prec)
    d = _case(name, shape, seed, bc, dtc)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((4,) + shape)
    x[1:] *= d["c"]
    dE = rng.uniform(1.0, 3.0, shape)
    if prec == "f32":
        for k in ("rho", "kR", "f"):
            d[k] = W._f32(d[k])
        x, dE = W._f32(x), W._f32(dE)
    want = _oracle_problem(d).apply(x, dE)
    dt = torch.float64 if prec == "f64" else torch.float32
    got = rad.rad_apply(_dev(torch, x, dt), _dev(torch, dE, dt), _dev(torch, d["rho"], dt), _dev(torch, d["kR"], dt),
                        _dev(torch, d["f"], dt), d["dt"], d["dx"], d["bc"], _params(rad, d)).double().cpu().numpy()
    tol = 1e-13 if prec == "f64" else 2e-6
    scale = np.max(np.abs(want))
    for q in range(4):
        assert np.max(np.abs(got[q] - want[q])) <= tol * scale, (q, np.max(np.abs(got[q] - want[q])) / scale)


@pytest.mark.parametrize("name,shape,seed,bc,dtc", CASES)
def test_wall_nonlinear_residual(torch, rad, name, shape, seed, bc, dtc):
    """The nonlinear residual: the walls' ghosts with their data (old state, F_inc)."""
    _say("wall residual", name, shape)
    d = _case(name, shape, seed, bc, dtc)
    rng = np.random.default_rng(seed + 1)
    E = d["E"] * (1 + 0.1 * rng.standard_normal(shape))
    F = d["F"] + 0.1 * rng.standard_normal((3,) + shape) * d["E"]
    T = d["T"] * (1 + 0.1 * rng.standard_normal(shape))
    want = _oracle_problem(d).residual(d["E"], d["F"], d["T"], E, F, T)
    g = lambda a: _dev(torch, a)
    got = rad.rad_residual(g(d["E"]), g(d["F"]), g(d["T"]), g(E), g(F), g(T), g(d["rho"]), g(d["kP"]), g(d["kR"]),
                           g(d["f"]), d["dt"], d["dx"], d["bc"], _params(rad, d)).cpu().numpy()
    for q in range(5):
        scale = max(np.max(np.abs(want[q])), 1e-300)
        assert np.max(np.abs(got[q] - want[q])) <= 1e-12 * scale + 1e-13 * np.max(np.abs(want)), q


@pytest.mark.parametrize("name,shape,seed,bc,dtc", CASES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("poly", [1, 0], ids=["poly", "jacobi"])
def test_wall_step_matches_oracle(torch, rad, name, shape, seed, bc, dtc, prec, poly):
    _say("wall step", name, shape, prec, poly)
    d = _case(name, shape, seed, bc, dtc)
    if prec == "mixed":
        for k in ("E", "F", "T", "rho", "kP", "kR", "f"):
            d[k] = W._f32(d[k])
    ref = _oracle_problem(d).step(d["E"], d["F"], d["T"], tol=1e-14)
    cd = torch.float32 if prec == "mixed" else torch.float64
    g = lambda a, dt=None: _dev(torch, a, dt)
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    st = rad.rad_step(E, F, T, g(d["rho"], cd), g(d["kP"], cd), g(d["kR"], cd), g(d["f"], cd), d["dt"], d["dx"],
                      d["bc"], _params(rad, d, prec=prec, tol=1e-13, krylov_poly=poly, gmres_m=30))
    _say("  stats", st)
    errs = [_relerr(E.cpu().numpy(), ref[0]), _relerr(F.cpu().numpy(), ref[1]), _relerr(T.cpu().numpy(), ref[2])]
    _say("  relerr E F T", ["%.2e" % e for e in errs])
    assert max(errs) <= (FP64_TOL if prec == "fp64" else MIXED_TOL), errs


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_open_walls_multigrid_operator(torch, rad, prec):
    """krylov_poly = 2 on a grid with open walls (the coarse levels carry the same walls); the clumpy
    medium at 100 crossings (no cell at the T >= 0 bound, where T is ill-conditioned in E)."""
    _say("open multigrid", prec)
    d = W.periodic_clumpy(shape=(16, 8, 32), seed=6)
    d["bc"] = "open"
    if prec == "mixed":
        for k in ("E", "F", "T", "rho", "kP", "kR", "f"):
            d[k] = W._f32(d[k])
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"])
    ref = P.step(d["E"], d["F"], d["T"], tol=1e-14)
    cd = torch.float32 if prec == "mixed" else torch.float64
    g = lambda a, dt=None: _dev(torch, a, dt)
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    st = rad.rad_step(E, F, T, g(d["rho"], cd), g(d["kP"], cd), g(d["kR"], cd), g(d["f"], cd), d["dt"], d["dx"],
                      d["bc"], rad.params(prec=prec, tol=1e-13, krylov_poly=2, gmres_m=12))
    _say("  stats", st)
    errs = [_relerr(E.cpu().numpy(), ref[0]), _relerr(F.cpu().numpy(), ref[1]), _relerr(T.cpu().numpy(), ref[2])]
    _say("  relerr E F T", ["%.2e" % e for e in errs])
    assert max(errs) <= (FP64_TOL if prec == "fp64" else MIXED_TOL), errs


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_open_line_streaming_pulse(torch, rad, axis, prec):
    """Sec. 3.1 streaming limit through open walls: sigma = 0, f = e_d e_d, F = c E; every step is
    implicit upwinding on an open line, E_i <- (E_i + nu E_{i-1}^new) / (1 + nu), until the pulse has
    left.  The GPU follows that closed form and keeps F = c E."""
    _say("open streaming pulse", axis, prec)
    n, c, nu = 96, 1.0, 1.5
    h = 1.0 / n
    shape = [1, 1, 1]
    shape[2 - axis] = n
    shape = tuple(shape)
    x = np.arange(n)
    E0 = np.where((x >= 20) & (x < 60), np.sin(np.pi * (x - 19) / 41.0) ** 2, 0.0)
    F0 = np.zeros((3,) + shape)
    F0[axis] = (c * E0).reshape(shape)
    f = np.zeros((6,) + shape)
    f[axis] = 1.0
    zero = np.zeros(shape)
    bc = ["periodic"] * 6
    bc[2 * axis] = bc[2 * axis + 1] = "open"
    g = lambda a: _dev(torch, a)
    E, F, T = g(E0.reshape(shape)), g(F0), g(np.ones(shape))
    rho, kz, fd = g(np.ones(shape)), g(zero), g(f)
    p = rad.params(c=c, prec=prec, tol=1e-13)
    ref = E0.copy()
    for step in range(60):
        rad.rad_step(E, F, T, rho, kz, kz, fd, nu * h / c, h, bc, p)
        new = np.empty(n)
        prev = 0.0
        for i in range(n):
            new[i] = (ref[i] + nu * prev) / (1.0 + nu)
            prev = new[i]
        ref = new
    got = E.cpu().numpy().reshape(n)
    tol = 1e-10 if prec == "fp64" else 1e-8
    assert np.max(np.abs(got - ref)) <= tol * np.max(E0)
    assert np.max(np.abs(F.cpu().numpy()[axis].reshape(n) - c * got)) <= tol * np.max(E0)
    assert ref.sum() < 0.2 * E0.sum()
