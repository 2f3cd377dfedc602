"""Single-grid autotuner: tile z-range per kernel and GMRES restart length timed on the caller's data,
cached per configuration, state left unchanged; later steps with the tuned tiles match the oracle."""
import os

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


def test_autotune_step_caches_tiles_and_keeps_state(torch, rad, tmp_path, monkeypatch):
    monkeypatch.setenv("VETTAM_RAD_CACHE_DIR", str(tmp_path))
    d = W.mixed_depth(shape=(40, 20, 24), seed=17, steps=1)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    coef = [g(d[k]) for k in ("rho", "kP", "kR", "f")]
    p = rad.params(c=d["c"], a_R=d["aR"], c_v=d["cv"], gmres_m=16, tol=1e-12)
    out = rad.autotune_step(E, F, T, *coef, d["dt"], d["dx"], d["bc"], p, tune_restart=True)
    print("autotune", out, flush=True)
    assert out["kz_apply"] in (8, 16, 32, 40) and out["kz_residual"] in (8, 16, 32, 40)
    assert out["gmres_m"] in (6, 8, 10, 12, 16) and out["krylov_poly"] in (0, 1)
    for t, a in zip((E, F, T), (d["E"], d["F"], d["T"])):
        assert np.array_equal(t.cpu().numpy(), a)
    lines = open(os.path.join(str(tmp_path), "autotune.txt")).read().splitlines()
    assert any(l.startswith("single|") and "|24x20x40|" in l for l in lines)
    # a step with the tuned tiles (read back from the cache) and restart length matches the oracle
    p.gmres_m = out["gmres_m"]
    p.krylov_poly = out["krylov_poly"]
    p.tol = 1e-13
    st = rad.rad_step(E, F, T, *coef, d["dt"], d["dx"], d["bc"], p)
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"], c=d["c"], aR=d["aR"],
                       cv=d["cv"])
    Eo, Fo, To, _ = P.step(d["E"], d["F"], d["T"], tol=1e-14)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    errs = (rel(E.cpu().numpy(), Eo), rel(F.cpu().numpy(), Fo), rel(T.cpu().numpy(), To))
    print("  step after autotune:", st["krylov_iters"], "Krylov; rel errors", errs, flush=True)
    assert max(errs) <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_apply_forming_face_speeds_matches_oracle(torch, rad, tmp_path, monkeypatch, prec):
    """The autotuner's other apply variant (face speeds formed per face from f and sR instead of read), chosen
    through a cache entry for a grid no other test uses, gives the oracle's step."""
    monkeypatch.setenv("VETTAM_RAD_CACHE_DIR", str(tmp_path))
    d = W.mixed_depth(shape=(9, 13, 70), seed=19, steps=1, dt_cross=20.0)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    coef = [g(d[k]) for k in ("rho", "kP", "kR", "f")]
    p = rad.params(c=d["c"], a_R=d["aR"], c_v=d["cv"], prec=prec, tol=1e-13)
    # learn the key format from a tuning run on another shape, then write this shape's entry by hand
    dt = W.mixed_depth(shape=(8, 8, 8), seed=20, steps=1)
    gt = [g(dt[k]) for k in ("E", "F", "T", "rho", "kP", "kR", "f")]
    rad.autotune_step(*gt, dt["dt"], dt["dx"], dt["bc"], rad.params(prec=prec), tune_restart=False)
    line = [l for l in open(os.path.join(str(tmp_path), "autotune.txt")).read().splitlines() if "|8x8x8|" in l][-1]
    key = line.split("\t")[0].replace("|8x8x8|", "|70x13x9|")
    with open(os.path.join(str(tmp_path), "autotune.txt"), "a") as fh:
        fh.write(f"{key}\t8 8 12 0\n")
    st = rad.rad_step(E, F, T, *coef, d["dt"], d["dx"], d["bc"], p)
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"], c=d["c"], aR=d["aR"],
                       cv=d["cv"])
    Eo, Fo, To, _ = P.step(d["E"], d["F"], d["T"], tol=1e-14)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    errs = (rel(E.cpu().numpy(), Eo), rel(F.cpu().numpy(), Fo), rel(T.cpu().numpy(), To))
    print("  formed face speeds:", prec, st["krylov_iters"], "Krylov; rel errors", errs, flush=True)
    assert max(errs) <= (1e-10 if prec == "fp64" else 1e-8)


def test_autotune_with_multigrid_workspace_tries_the_cycle(torch, rad, tmp_path, monkeypatch):
    """With krylov_poly = 2 (the workspace holds the multigrid levels) the restart trials include the V-cycle; the
    recommended operator and restart length give the oracle's step."""
    monkeypatch.setenv("VETTAM_RAD_CACHE_DIR", str(tmp_path))
    d = W.mixed_depth(shape=(16, 16, 32), seed=21, steps=1)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    E, F, T = g(d["E"]), g(d["F"]), g(d["T"])
    coef = [g(d[k]) for k in ("rho", "kP", "kR", "f")]
    p = rad.params(c=d["c"], a_R=d["aR"], c_v=d["cv"], gmres_m=8, tol=1e-12, krylov_poly=2)
    out = rad.autotune_step(E, F, T, *coef, d["dt"], d["dx"], d["bc"], p, tune_restart=True)
    print("autotune (multigrid workspace)", out, flush=True)
    assert out["krylov_poly"] in (0, 1, 2) and out["gmres_m"] in (6, 8)
    for t, a in zip((E, F, T), (d["E"], d["F"], d["T"])):
        assert np.array_equal(t.cpu().numpy(), a)
    p.gmres_m, p.krylov_poly, p.tol = out["gmres_m"], out["krylov_poly"], 1e-13
    rad.rad_step(E, F, T, *coef, d["dt"], d["dx"], d["bc"], p)
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], d["bc"], c=d["c"], aR=d["aR"],
                       cv=d["cv"])
    Eo, Fo, To, _ = P.step(d["E"], d["F"], d["T"], tol=1e-14)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)
    errs = (rel(E.cpu().numpy(), Eo), rel(F.cpu().numpy(), Fo), rel(T.cpu().numpy(), To))
    print("  step with the recommendation:", errs, flush=True)
    assert max(errs) <= 1e-10
