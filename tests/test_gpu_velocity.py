"""Moving medium: parity of rad_step_moving (through the C ABI) with the oracle's O(v/c) terms on the
same seeded inputs -- normwise relative error per field <= 1e-10 (FP64 path) or <= 1e-8 (mixed
path), with the O(v/c) gas energy explicit (default) or implicit -- and the dynamic diffusion pulse
(Sec. 3.2) carried with the gas on the GPU as in the oracle."""
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


def _case(kind, shape, seed, bmax):
    if kind == "clumpy":
        d = W.periodic_clumpy(shape=shape, seed=seed)
    else:
        d = W.mixed_depth(shape=shape, seed=seed, steps=1, bc=kind, dt_cross=2.0 if kind == "outflow" else 20.0)
    rng = np.random.default_rng(seed + 100)
    d["F"] = 0.1 * rng.standard_normal((3,) + shape) * d["E"]
    # a smooth flow: a random drift plus a periodic shear, |beta| <= bmax
    nz, ny, nx = shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx,
                          indexing="ij")
    u = rng.standard_normal(3)
    u /= np.linalg.norm(u)
    d["beta"] = np.stack([0.5 * bmax * (u[q] + np.sin(2 * np.pi * (x + y + z) + q)) for q in range(3)])
    return d


# (kind, shape (nz, ny, nx), seed, max |beta|): the 70-wide case spans two x tiles with a ragged tail;
# in the mixed-depth media (cell optical depth up to 1e3) beta tau per cell reaches 1 (dynamic diffusion)
CASES = [("clumpy", (6, 9, 12), 1, 0.05), ("outflow", (5, 11, 70), 2, 1e-3), ("periodic", (8, 8, 8), 3, 1e-3)]


def _relerr(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def _gpu(torch, rad, d, prec, implicit, beta=True):
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    p = rad.params(c=d["c"], a_R=d["aR"], c_v=d["cv"], prec=prec, tol=1e-13, vel_implicit=int(implicit))
    args = (g(d["rho"]), g(d["kP"]), g(d["kR"]), g(d["f"]))
    if beta:
        st = rad.rad_step_moving(E, F, T, *args, g(d["beta"]), d["dt"], d["dx"], d["bc"], p)
    else:
        st = rad.rad_step(E, F, T, *args, d["dt"], d["dx"], d["bc"], p)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (E, F, T)], st


@pytest.mark.parametrize("implicit", [False, True], ids=["explicit", "implicit"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,shape,seed,bmax", CASES)
def test_moving_step_matches_oracle(torch, rad, kind, shape, seed, bmax, prec, implicit):
    _say("moving", kind, shape, seed, prec, "implicit" if implicit else "explicit")
    d = _case(kind, shape, seed, bmax)
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"], c=d["c"], aR=d["aR"],
                       cv=d["cv"], beta=d["beta"], vel_implicit=implicit)
    ref = P.step(d["E"], d["F"], d["T"], tol=1e-14)
    out, st = _gpu(torch, rad, d, prec, implicit)
    errs = {k: _relerr(a, b) for k, a, b in zip("EFT", out, ref[:3])}
    _say("  ", {k: f"{v:.2e}" for k, v in errs.items()}, "picard", st["picard_iters"], "krylov", st["krylov_iters"])
    assert max(errs.values()) <= (FP64_TOL if prec == "fp64" else MIXED_TOL), errs


def test_zero_velocity_matches_rad_step(torch, rad):
    d = _case("clumpy", (6, 9, 12), 4, 0.0)
    a, _ = _gpu(torch, rad, d, "fp64", True, beta=True)
    b, _ = _gpu(torch, rad, d, "fp64", False, beta=False)
    for x, y in zip(a, b):
        assert _relerr(x, y) <= 1e-13


def test_dynamic_diffusion_pulse_on_gpu(torch, rad):
    """Sec. 3.2 in code units (kappa_E = 0, sigma_F h ~ 16, beta = 0.02): 20 GPU steps follow the oracle's,
    and the pulse's centroid moves at v."""
    n, c, sig, b, mu, x0, steps, dt = 128, 1.0, 2000.0, 0.02, 25.0, 0.3, 20, 0.117
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    E0 = np.exp(-mu ** 2 * (x - x0) ** 2) + 1e-3
    F0 = (4.0 / 3.0) * b * c * E0 + c / (3 * sig) * 2 * mu ** 2 * (x - x0) * (E0 - 1e-3)
    one = np.ones((1, 1, n))
    f = np.zeros((6, 1, 1, n))
    f[:3] = 1.0 / 3.0
    beta = np.zeros((3, 1, 1, n))
    beta[0] = b
    d = dict(rho=one, kP=0 * one, kR=sig * one, f=f, beta=beta, dt=dt, dx=h, bc="periodic", c=c, aR=1.0, cv=1.0)
    P = oracle.Problem(one, 0 * one, sig * one, f, dt=dt, dx=h, c=c, beta=beta)
    Eo, Fo, To = E0.reshape(1, 1, n).copy(), np.zeros((3, 1, 1, n)), one.copy()
    Fo[0, 0, 0] = F0
    d.update(E=Eo.copy(), F=Fo.copy(), T=To.copy())
    for _ in range(steps):
        Eo, Fo, To, _ = P.step(Eo, Fo, To, tol=1e-13)
        out, st = _gpu(torch, rad, d, "mixed", False)
        d.update(E=out[0], F=out[1], T=out[2])
    assert _relerr(d["E"], Eo) <= 1e-7 and _relerr(d["F"], Fo) <= 1e-7
    e = d["E"][0, 0] - 1e-3
    shift = np.sum(x * e) / np.sum(e) - np.sum(x * (E0 - 1e-3)) / np.sum(E0 - 1e-3)
    _say("dynamic diffusion: centroid shift", shift, "v t", b * c * steps * dt)
    assert abs(shift - b * c * steps * dt) <= 0.05 * b * c * steps * dt
