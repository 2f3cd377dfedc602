"""Pins of the oracle's convergence measure, the scaled nonlinear residual.

The scaled residual is the stopping rule of every step and the checker of every
full-size parity test, so it is pinned on its own here:
  res_E = || R_E / W_E || / ||E||,  res_F = || R_F / W_F || / (||F|| + c ||E||),
  res_T = || R_T / W_T || / ||T||,
with W_E = 1 + sP + (dt/2h) sum_faces C, W_F = 1 + sR + (dt/2h) sum_faces C and
W_T = alpha + 4 sP aR T^3 (norms are 2-norms over the cells, F over all three
components; a cell at the T >= 0 bound whose exchange row cannot be satisfied
counts as satisfied).

Two independent routes: a uniform periodic state, where every transport term
vanishes and each part has a closed form, and a brute-force evaluation on 2x1x1
and 3x2x1 grids that forms every face flux, residual row and weight by hand in
plain Python loops (its own face-speed formula, its own neighbour bookkeeping).
"""
import math

import numpy as np
import pytest

import oracle

TENS = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4, (1, 2): 5, (2, 1): 5}


def _speed(c, h, fL, fR, sigL, sigR):
    """Corrected HLLE speed of one face (Sec. 2.3.3): c sqrt(max f) sqrt((1 - e^-tau)/tau),
    tau the mean of the two cells' (10 h sigma_R)^2 / (2 f_dd); tau = 0 without opacity and
    infinite (speed 0) for f_dd = 0 with opacity."""
    def tau(sig, f):
        if sig == 0.0:
            return 0.0
        if f == 0.0:
            return math.inf
        return (10.0 * h * sig) ** 2 / (2.0 * f)
    t = 0.5 * (tau(sigL, fL) + tau(sigR, fR))
    if t == 0.0:
        corr = 1.0
    elif math.isinf(t):
        corr = 0.0
    else:
        corr = math.sqrt(-math.expm1(-t) / t)
    return c * math.sqrt(max(fL, fR)) * corr


def _by_hand(rho, kP, kR, f, E_n, F_n, T_n, E, F, T, dt, h, c, aR, cv):
    """Scaled residual of a periodic grid evaluated cell by cell with explicit neighbours."""
    nz, ny, nx = E.shape
    lam = dt / h
    cells = [(k, j, i) for k in range(nz) for j in range(ny) for i in range(nx)]

    def nb(cell, d, s):
        k, j, i = cell
        q = [i, j, k]
        n = [nx, ny, nz]
        q[d] = (q[d] + s) % n[d]
        return (q[2], q[1], q[0])

    def sig(cell):
        return rho[cell] * kR[cell]

    def flux(L, R, d):
        """HLL flux (E, Fx, Fy, Fz) through the face from cell L to cell R = L + e_d."""
        C = _speed(c, h, f[d][L], f[d][R], sig(L), sig(R))
        out = [0.5 * (F[d][L] + F[d][R]) - 0.5 * C * (E[R] - E[L])]
        for j in range(3):
            fdj = f[TENS[(d, j)]]
            out.append(0.5 * c * c * (fdj[L] * E[L] + fdj[R] * E[R]) - 0.5 * C * (F[j][R] - F[j][L]))
        return out, C

    sE = sF = sT = 0.0
    nE = nF = nT = 0.0
    for cell in cells:
        sP = c * dt * rho[cell] * kP[cell]
        sR = c * dt * rho[cell] * kR[cell]
        alpha = rho[cell] * cv
        div = [0.0] * 4
        sumC = 0.0
        for d in range(3):
            hi, Chi = flux(cell, nb(cell, d, +1), d)
            lo, Clo = flux(nb(cell, d, -1), cell, d)
            for q in range(4):
                div[q] += hi[q] - lo[q]
            sumC += Chi + Clo
        T4 = T[cell] ** 4
        RE = (1 + sP) * E[cell] - E_n[cell] - sP * aR * T4 + lam * div[0]
        RF = [(1 + sR) * F[j][cell] - F_n[j][cell] + lam * div[1 + j] for j in range(3)]
        RT = alpha * (T[cell] - T_n[cell]) + sP * (aR * T4 - E[cell])
        if T[cell] == 0.0 and RT > 0.0:
            RT = 0.0
        WE = 1 + sP + 0.5 * lam * sumC
        WF = 1 + sR + 0.5 * lam * sumC
        WT = alpha + 4 * sP * aR * T[cell] ** 3
        sE += (RE / WE) ** 2
        sF += sum((r / WF) ** 2 for r in RF)
        sT += (RT / WT) ** 2
        nE += E[cell] ** 2
        nF += sum(F[j][cell] ** 2 for j in range(3))
        nT += T[cell] ** 2
    rE = math.sqrt(sE) / math.sqrt(nE)
    rF = math.sqrt(sF) / (math.sqrt(nF) + c * math.sqrt(nE))
    rT = math.sqrt(sT) / math.sqrt(nT)
    return rE, rF, rT, max(rE, rF, rT)


def _random_fields(shape, seed, tiny_F=False, T_zero_cell=None):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, shape)
    kP = rng.uniform(0.2, 3.0, shape)
    kR = rng.uniform(0.2, 3.0, shape)
    A = rng.standard_normal((3, 3) + shape) * 0.05
    f = np.empty((6,) + shape)
    for n, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        f[n] = (1 / 3 if a == b else 0.0) + 0.5 * (A[a, b] + A[b, a])
    E_n = rng.uniform(0.5, 2.0, shape)
    F_n = rng.uniform(-0.3, 0.3, (3,) + shape)
    T_n = rng.uniform(0.5, 1.5, shape)
    E = E_n + 0.2 * rng.standard_normal(shape)
    F = F_n + 0.1 * rng.standard_normal((3,) + shape)
    if tiny_F:
        F_n *= 1e-6
        F *= 1e-6
    T = T_n + 0.1 * rng.standard_normal(shape)
    if T_zero_cell is not None:
        # a cell at the T >= 0 bound: E negative enough that the exchange row has no root,
        # so R_T(T = 0) = -alpha T_n - sP E > 0 and the row counts as satisfied
        E[T_zero_cell] = -5.0 * (rho[T_zero_cell] * T_n[T_zero_cell]) / (kP[T_zero_cell] * rho[T_zero_cell]) - 1.0
        T[T_zero_cell] = 0.0
    return rho, kP, kR, f, E_n, F_n, T_n, E, F, T


@pytest.mark.parametrize("shape,seed,tiny_F,tzero", [
    ((1, 1, 2), 1, False, None),
    ((1, 2, 3), 2, False, None),
    ((1, 2, 3), 3, True, None),            # ||F|| << c ||E||: the flux part's normaliser is c ||E||
    ((1, 2, 3), 4, False, (0, 1, 2)),      # one cell at the T >= 0 bound
])
def test_scaled_residual_matches_hand_evaluation(shape, seed, tiny_F, tzero):
    dt, h, c, aR, cv = 0.37, 0.25, 1.7, 0.8, 1.3
    rho, kP, kR, f, E_n, F_n, T_n, E, F, T = _random_fields(shape, seed, tiny_F, tzero)
    P = oracle.Problem(rho, kP, kR, f, dt, h, "periodic", c=c, aR=aR, cv=cv)
    got = P.scaled_residual(E_n, F_n, T_n, E, F, T)
    want = _by_hand(rho, kP, kR, f, E_n, F_n, T_n, E, F, T, dt, h, c, aR, cv)
    for g, w in zip(got, want):
        assert abs(g - w) <= 1e-13 * abs(w), (got, want)
    if tzero is not None:
        # the bound cell's exchange row would dominate if it were counted
        sP = c * dt * rho[tzero] * kP[tzero]
        RT = rho[tzero] * cv * (0.0 - T_n[tzero]) + sP * (0.0 - E[tzero])
        assert RT > 0.0
        assert got[2] < abs(RT) / (rho[tzero] * cv) / np.linalg.norm(T)


@pytest.mark.parametrize("tiny_F,part", [(False, None), (True, None), (False, 1)])
def test_scaled_residual_uniform_closed_form(tiny_F, part):
    """Uniform periodic state and medium: every flux difference vanishes, so R_E = (1 + sP) E - E_n -
    sP aR T^4, R_F = (1 + sR) F - F_n, R_T = alpha (T - T_n) + sP (aR T^4 - E), and the cell count
    cancels from every ratio: res_E = |R_E| / (W_E |E|), res_F = |R_F| / (W_F (|F| + c |E|)),
    res_T = |R_T| / (W_T |T|), with the six faces of a cell all at the speed C = c sqrt(f_dd)
    sqrt((1 - e^-tau)/tau), tau = (10 h rho kR)^2 / (2 f_dd) (isotropic f, so one C)."""
    shape = (3, 2, 4)
    dt, h, c, aR, cv = 0.9, 0.5, 1.3, 1.1, 0.7
    rho, kP, kR = 1.4, 0.9, 0.35
    E_n, T_n, E, T = 1.2, 0.8, 1.05, 0.93
    F_n = np.array([0.2, -0.1, 0.05])
    F = np.array([0.18, -0.07, 0.02])
    if tiny_F:
        F_n, F = F_n * 1e-7, F * 1e-7
    if part == 1:   # a state whose flux rows are furthest from solved
        F = F * 40.0
    f = np.zeros((6,) + shape)
    f[:3] = 1 / 3
    full = lambda v: np.full(shape, v)
    P = oracle.Problem(full(rho), full(kP), full(kR), f, dt, h, "periodic", c=c, aR=aR, cv=cv)
    Fn_a = np.stack([full(v) for v in F_n])
    F_a = np.stack([full(v) for v in F])
    got = P.scaled_residual(full(E_n), Fn_a, full(T_n), full(E), F_a, full(T))
    sP, sR, alpha = c * dt * rho * kP, c * dt * rho * kR, rho * cv
    tau = (10 * h * rho * kR) ** 2 / (2 / 3)
    C = c * math.sqrt(1 / 3) * math.sqrt((1 - math.exp(-tau)) / tau)
    W_E = 1 + sP + 0.5 * (dt / h) * 6 * C
    W_F = 1 + sR + 0.5 * (dt / h) * 6 * C
    W_T = alpha + 4 * sP * aR * T ** 3
    R_E = (1 + sP) * E - E_n - sP * aR * T ** 4
    R_F = np.linalg.norm((1 + sR) * F - F_n)
    R_T = alpha * (T - T_n) + sP * (aR * T ** 4 - E)
    want = (abs(R_E) / (W_E * abs(E)), R_F / (W_F * (np.linalg.norm(F) + c * abs(E))), abs(R_T) / (W_T * abs(T)))
    for g, w in zip(got[:3], want):
        assert abs(g - w) <= 1e-13 * w, (got, want)
    assert got[3] == max(got[:3])
    if part is not None:
        assert got[3] == got[part] > max(got[q] for q in range(3) if q != part)
