"""rad_step_noalloc (the allocation-free entry point, workspace in the library's static device
scratch) against rad_step (caller workspace) through the C ABI on the same inputs: two calls in a
row, the second on a smaller grid, FP64 and mixed; the results must be identical (same kernels,
same launch shapes, fixed-order reductions).  A step needing more workspace than the scratch holds
is refused with RAD_ENOMEM before any device work.  Collected last (name), so a failure here hides
no other test."""
import ctypes as ct
import sys

import numpy as np
import pytest

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


def _run(torch, rad, d, prec, noalloc):
    cd = torch.float32 if prec == "mixed" else torch.float64
    g = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a)).to(dt or torch.float64).cuda()
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    coef = (g(d["rho"], cd), g(d["kP"], cd), g(d["kR"], cd), g(d["f"], cd))
    p = rad.params(prec=prec, tol=1e-12)
    if noalloc:
        st = rad.rad_step_noalloc(E, F, T, *coef, d["dt"], d["dx"], d["bc"], p)
    else:
        st = rad.rad_step(E, F, T, *coef, d["dt"], d["dx"], d["bc"], p)
    torch.cuda.synchronize()
    return E.cpu().numpy(), F.cpu().numpy(), T.cpu().numpy(), st


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_rad_step_twice(torch, rad, prec):
    cases = [W.mixed_depth(shape=(20, 24, 70), seed=41, steps=1, dt_cross=20.0, fp32_exact=prec == "mixed"),
             W.mixed_depth(shape=(9, 11, 13), seed=42, steps=1, dt_cross=20.0, fp32_exact=prec == "mixed")]
    for i, d in enumerate(cases):
        _say("noalloc", prec, "call", i, d["E"].shape)
        a = _run(torch, rad, d, prec, noalloc=True)
        b = _run(torch, rad, d, prec, noalloc=False)
        _say("  noalloc", a[3]["picard_iters"], a[3]["krylov_iters"], "rad_step", b[3]["picard_iters"],
             b[3]["krylov_iters"])
        for q in range(3):
            assert np.array_equal(a[q], b[q]), (q, np.max(np.abs(a[q] - b[q])))
        assert a[3]["picard_iters"] == b[3]["picard_iters"] and a[3]["krylov_iters"] == b[3]["krylov_iters"]


def test_noalloc_refuses_oversize(torch, rad):
    p = rad.params()
    cap = rad.lib.rad_noalloc_max_bytes()
    n = 128
    assert rad.lib.rad_workspace_bytes(n, n, n, ct.byref(p)) > cap
    st = rad.Stats()
    rc = rad.lib.rad_step_noalloc(n, n, n, None, None, None, None, None, None, None, 1.0, 1.0 / n,
                                  rad.bc_array("periodic"), ct.byref(p), None, ct.byref(st))
    assert rc == rad.RAD_ENOMEM, rc
    assert "scratch" in rad.last_error()
