"""Anderson-accelerated Picard iteration (the acceleration Sec. 4.3 names for the linearly
convergent Picard scheme): same fixed point as the oracle's solution, far fewer iterations than the
paper's lagged iteration."""
import time

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


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _gpu(torch, rad, d, prec="fp64", **kw):
    c32 = prec == "mixed"
    cd = torch.float32 if c32 else torch.float64
    g = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dt).cuda()
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    p = rad.params(c=d["c"], a_R=d["aR"], c_v=d["cv"], prec=prec, coef_dtype=1 if c32 else 0, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = rad.rad_step(E, F, T, g(d["rho"], cd), g(d["kP"], cd), g(d["kR"], cd), g(d["f"], cd), d["dt"], d["dx"],
                      d["bc"], p, check=False)
    torch.cuda.synchronize()
    st["seconds"] = time.perf_counter() - t0
    return (E.cpu().numpy(), F.cpu().numpy(), T.cpu().numpy()), st


def _oracle(d, **kw):
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"], c=d["c"], aR=d["aR"],
                       cv=d["cv"])
    E, F, T, _ = P.step(d["E"], d["F"], d["T"], tol=1e-14, **kw)
    return E, F, T


def test_anderson_lagged_reaches_oracle_solution_in_far_fewer_iterations(torch, rad):
    """32^3 periodic clumpy medium at dt = 100 crossings (lagged Picard contracts at up to 0.99 per
    iteration there): lagged + Anderson(5) matches the oracle to 1e-10 in a small fraction of the
    plain lagged iteration's Picard count."""
    _say("anderson lagged 32^3")
    d = W.periodic_clumpy(n=32)
    ref = _oracle(d)
    (Ea, Fa, Ta), sa = _gpu(torch, rad, d, mode="lagged", tol=1e-13, max_picard=5000, anderson_m=5)
    (El, Fl, Tl), sl = _gpu(torch, rad, d, mode="lagged", tol=1e-13, max_picard=5000)
    _say(f"  lagged: {sl['picard_iters']} Picard, {sl['krylov_iters']} Krylov, {sl['seconds']:.2f} s, rc {sl['rc']}")
    _say(f"  lagged+Anderson(5): {sa['picard_iters']} Picard, {sa['krylov_iters']} Krylov, {sa['seconds']:.2f} s, "
         f"rc {sa['rc']}")
    assert sa["rc"] == 0
    errs = [_relerr(a, b) for a, b in zip((Ea, Fa, Ta), ref)]
    _say("  relerr E F T vs oracle", ["%.1e" % e for e in errs])
    assert max(errs) <= 1e-10
    assert sa["picard_iters"] * 5 <= sl["picard_iters"]


@pytest.mark.parametrize("prec,tol,mode,m", [("mixed", 1e-8, "lagged", 3), ("fp64", 1e-10, "linearised", 5),
                                             ("fp64", 1e-10, "lagged", 1), ("fp64", 1e-10, "lagged", 2)])
def test_anderson_matches_oracle(torch, rad, prec, tol, mode, m):
    _say("anderson", prec, mode, m)
    d = W.periodic_clumpy(shape=(10, 12, 14), seed=9)
    d["dt"] *= 0.2
    if prec == "mixed":
        for k in ("rho", "kP", "kR", "f"):
            d[k] = d[k].astype(np.float32).astype(np.float64)
    ref = _oracle(d)
    out, st = _gpu(torch, rad, d, prec=prec, mode=mode, tol=1e-13, max_picard=3000, anderson_m=m)
    _say(f"  {st['picard_iters']} Picard, {st['krylov_iters']} Krylov, rc {st['rc']}")
    assert st["rc"] == 0
    errs = [_relerr(a, b) for a, b in zip(out, ref)]
    _say("  relerr E F T", ["%.1e" % e for e in errs])
    assert max(errs) <= tol


def test_batched_plan_rejects_anderson(torch, rad):
    batch = W.batched_blocks(nblocks=4, seed=3, sizes=(4,))
    descs, _ = rad.pack_blocks(batch["blocks"])
    with pytest.raises(Exception):
        rad.Plan(descs, rad.params(anderson_m=2))
