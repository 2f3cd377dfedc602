"""Energy correction of the Picard iteration (Sec. 2.3.4) on the GPU, against the oracle on the same
seeded inputs: the per-step mismatch diagnostics (energy_defect, dE_max), the energy-fixed commit
(energy_fix = 1) in both Picard modes and both precisions, and the paper's own tolerances
(eps_N = eps_R = 1e-6, eps_P = 1e-3, lagged Picard)."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2202_08778_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def _gpu(torch, rad, d, prec="fp64", check=True, **kw):
    cd = torch.float32 if prec == "mixed" else torch.float64
    g = lambda a, dt=None: _dev(torch, a, dt)
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    p = rad.params(c=d["c"], a_R=d["aR"], c_v=d["cv"], prec=prec, **kw)
    st = rad.rad_step(E, F, T, g(d["rho"], cd), g(d["kP"], cd), g(d["kR"], cd), g(d["f"], cd), d["dt"], d["dx"],
                      d["bc"], p, check=check)
    return E.cpu().numpy(), F.cpu().numpy(), T.cpu().numpy(), st


def _clumpy(shape, seed, fp32):
    d = W.periodic_clumpy(shape=shape, seed=seed)
    if fp32:
        for k in ("E", "F", "T", "rho", "kP", "kR", "f"):
            d[k] = W._f32(d[k])
    return d


@pytest.mark.parametrize("mode", ["lagged", "linearised"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("fix", [False, True])
def test_three_picard_iterations_match_oracle(torch, rad, mode, prec, fix):
    """Exactly three Picard iterations with tight linear solves: the iterates, the energy mismatch of
    the last exchange and (with the fix) the corrected temperature follow the oracle's."""
    _say("three iterations", mode, prec, fix)
    d = _clumpy((8, 7, 9), 31, prec == "mixed")
    d["dt"] *= 0.1
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"])
    ref = P.step(d["E"], d["F"], d["T"], mode=mode, max_picard=3, lin_rtol=1e-14, energy_fix=fix,
                 allow_unconverged=True)
    out = _gpu(torch, rad, d, prec, check=False, mode=mode, max_picard=3, eps_R=1e-13, tol=1e-30, energy_fix=int(fix),
               gmres_m=30)
    st = out[3]
    _say("  gpu", st, "oracle", ref[3])
    assert st["picard_iters"] == 3 and ref[3]["picard_iters"] == 3
    tol = 1e-10 if prec == "fp64" else 1e-8
    errs = [_relerr(out[q], ref[q]) for q in range(3)]
    _say("  relerr E F T", ["%.2e" % e for e in errs])
    assert max(errs) <= tol
    assert abs(st["energy_defect"] - ref[3]["energy_defect"]) <= 1e-6 * abs(ref[3]["energy_defect"]) + 1e-14
    assert abs(st["dE_max"] - ref[3]["dE_max"]) <= 1e-6 * ref[3]["dE_max"] + 1e-14
    if mode == "lagged":   # three lagged iterations leave a visible mismatch (linearised: ~1e-11, Newton)
        assert abs(ref[3]["energy_defect"]) > 1e-8


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_mismatch_vanishes_at_convergence(torch, rad, prec):
    d = _clumpy((8, 8, 8), 32, prec == "mixed")
    out = _gpu(torch, rad, d, prec, tol=1e-12)
    _say("converged", out[3])
    assert out[3]["dE_max"] <= 1e-9
    assert abs(out[3]["energy_defect"]) <= 1e-10


def _total(E, T, alpha):
    return math.fsum((E + alpha * T).ravel())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_paper_preset_energy_accounting(torch, rad, prec):
    """The paper's tolerances (eps_N = eps_R = 1e-6, eps_P = 1e-3, lagged Picard) on a clumpy periodic
    grid at 100 crossings: the step stops on the relative change.  Without the fix the total energy
    moves by the reported mismatch; with it the total is conserved to the linear tolerance.  Both GPU
    states agree with the oracle's under the same settings far closer than either is to the converged
    solution (the same iteration, stopped at the same place)."""
    _say("paper preset", prec)
    d = _clumpy((8, 8, 8), 5, prec == "mixed")
    alpha = d["rho"] * d["cv"]
    e0 = _total(d["E"], d["T"], alpha)
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"])
    xs = P.step(d["E"], d["F"], d["T"], tol=1e-14)
    kw = dict(mode="lagged", eps_P=1e-3, eps_N=1e-6, eps_R=1e-6, tol=1e-30, max_picard=5000, gmres_m=30)
    for fix in (False, True):
        ref = P.step(d["E"], d["F"], d["T"], tol=0.0, mode="lagged", eps_P=1e-3, eps_N=1e-6, lin_rtol=1e-6,
                     max_picard=5000, gmres_m=30, energy_fix=fix)
        out = _gpu(torch, rad, d, prec, energy_fix=int(fix), **kw)
        st = out[3]
        drift = (_total(out[0], out[2], alpha) - e0) / e0
        _say(f"  fix={fix}: gpu {st['picard_iters']} it, drift {drift:.3e}, defect {st['energy_defect']:.3e}; "
             f"oracle {ref[3]['picard_iters']} it, defect {ref[3]['energy_defect']:.3e}")
        assert abs(st["picard_iters"] - ref[3]["picard_iters"]) <= 1
        if not fix:
            assert abs(drift + st["energy_defect"]) <= 1e-3 * abs(st["energy_defect"])
            assert abs(st["energy_defect"]) > 1e-4
        else:
            assert abs(drift) <= 1e-7
        for q in (0, 2):
            to_ref, to_x = _relerr(out[q], ref[q]), _relerr(ref[q], xs[q])
            _say(f"    field {q}: gpu vs oracle (same settings) {to_ref:.2e}, oracle vs solution {to_x:.2e}")
            assert to_ref <= 0.05 * to_x
