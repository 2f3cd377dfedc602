"""Local closures (Sec. 4.1) on the GPU against the FP64 oracle: the tensor itself on random and
edge-case states, and steps closed by the tensor recomputed from the lagged state."""
import numpy as np
import pytest

import oracle
from paper_2202_08778_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def _say(*a):
    print(*a, flush=True)


def _states(rng, m, c):
    E = rng.uniform(0.05, 3.0, m)
    n = rng.standard_normal((3, m))
    n /= np.linalg.norm(n, axis=0)
    g = rng.uniform(0.0, 1.0, m)
    F = g * c * E * n
    # edge cases: no flux, exact beam, |F| > cE, E <= 0 with and without flux, tiny flux
    F[:, 0] = 0.0
    F[:, 1] = c * E[1] * n[:, 1]
    F[:, 2] = 3.0 * c * E[2] * n[:, 2]
    E[3], E[4], E[5] = 0.0, -1.0, -0.5
    F[:, 5] = 0.0
    F[:, 6] = 1e-300 * n[:, 6]
    return E, F


@pytest.mark.parametrize("kind", ["eddington", "m1"])
def test_closure_matches_oracle(torch, rad, kind):
    _say("closure", kind)
    c = 1.7
    rng = np.random.default_rng(31)
    E, F = _states(rng, 70001, c)   # ragged against the launch's 256-thread blocks
    fo = oracle.closure(E, F, kind, c)
    Ed, Fd = torch.from_numpy(E).cuda(), torch.from_numpy(F).cuda()
    f64 = rad.rad_closure(Ed, Fd, kind, c).cpu().numpy()
    f32 = rad.rad_closure(Ed, Fd, kind, c, out_dtype=torch.float32).cpu().numpy()
    err = np.max(np.abs(f64 - fo))
    _say("  max |f_gpu - f_oracle| (FP64)", err)
    assert err <= 1e-14
    # FP32 output: the FP64 tensor rounded once (within one FP32 ulp of the oracle's value)
    assert np.max(np.abs(f32.astype(np.float64) - fo) / np.maximum(np.abs(fo), 1e-30)
                  * (np.abs(fo) > 1e-30)) <= 2.0 ** -23
    if kind == "eddington":
        assert np.all(f64[:3] == 1.0 / 3.0) and np.all(f64[3:] == 0.0)


def test_closure_empty_is_noop(torch, rad):
    E = torch.empty(0, dtype=torch.float64, device="cuda")
    F = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    f = rad.rad_closure(E, F, "m1")
    assert f.shape == (6, 0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_m1_closed_steps_match_oracle(torch, rad, prec, tol):
    """Three steps, each closed by M1 recomputed from the state at its start (time-lagged), on a 16^3
    periodic mixed-depth medium with a source: GPU (rad_closure + rad_step) against the oracle doing the
    same with its own closure (rounded to FP32 by the oracle side for the mixed path).  Parity-run
    tolerances as for single steps: 1e-13 on the GPU, 1e-14 in the oracle."""
    _say("M1-closed steps", prec)
    d = W.mixed_depth(n=16, seed=7, steps=3, fp32_exact=(prec == "mixed"))
    c32 = prec == "mixed"
    cd = torch.float32 if c32 else torch.float64
    g = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dt).cuda()
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    rho, kP, kR = g(d["rho"], cd), g(d["kP"], cd), g(d["kR"], cd)
    p = rad.params(c=d["c"], a_R=d["aR"], c_v=d["cv"], prec=prec, tol=1e-13, coef_dtype=1 if c32 else 0)
    Eo, Fo, To = d["E"].copy(), d["F"].copy(), d["T"].copy()
    for s in range(3):
        f = rad.rad_closure(E, F, "m1", d["c"], out_dtype=cd)
        st = rad.rad_step(E, F, T, rho, kP, kR, f, d["dt"], d["dx"], "periodic", p)
        _say(f"  step {s}: rc {st['rc']}, krylov {st['krylov_iters']}, res {st['scaled_residual']:.2e}")
        assert st["rc"] == 0
        fo = oracle.closure(Eo, Fo, "m1", d["c"])
        if c32:
            fo = fo.astype(np.float32).astype(np.float64)
        P = oracle.Problem(d["rho"], d["kP"], d["kR"], fo, d["dt"], d["dx"], "periodic", c=d["c"], aR=d["aR"],
                           cv=d["cv"])
        Eo, Fo, To, _ = P.step(Eo, Fo, To, tol=1e-14)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    errs = (rel(E.cpu().numpy(), Eo), rel(F.cpu().numpy(), Fo), rel(T.cpu().numpy(), To))
    _say("  rel errors E F T", ["%.1e" % e for e in errs])
    assert max(errs) <= tol
