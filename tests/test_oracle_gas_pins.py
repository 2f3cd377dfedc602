"""Pins of the oracle's cubic-heat-capacity gas (C_v = alpha T^3, E_int = alpha T^4 / 4: the gas of the
Marshak-wave test, Sec. 3.4) against closed forms: with this gas the exchange row is linear in T^4, so a
uniform medium has a one-step closed form in T^4 (no root finding at all), total energy E + alpha T^4 / 4
is conserved on a periodic grid (with the Newton rate of the linearised iteration), and the equilibrium
reached after many steps solves aR T^4 = E with E + alpha T^4 / 4 unchanged."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("mode", ["linearised", "lagged"])
def test_uniform_medium_one_step_closed_form(mode):
    rho, kP, kR, cv, aR, c, dt = 1.3, 2.0, 3.0, 0.6, 1.2, 1.0, 0.5
    En, Tn, Fn = 0.7, 1.4, np.array([0.1, -0.2, 0.05])
    shape = (3, 4, 5)
    f = np.zeros((6,) + shape)
    f[:3] = 1.0 / 3.0
    P = oracle.Problem(np.full(shape, rho), np.full(shape, kP), np.full(shape, kR), f, dt=dt, dx=0.2, c=c, aR=aR,
                       cv=cv, cv_cubic=True)
    E1, F1, T1, _ = P.step(np.full(shape, En), np.broadcast_to(Fn[:, None, None, None], (3,) + shape).copy(),
                           np.full(shape, Tn), tol=1e-15, mode=mode, max_picard=2000)
    sP, sR, a = c * dt * rho * kP, c * dt * rho * kR, rho * cv
    # E = (En + sP aR T^4) / (1 + sP) in the gas row: (a/4)(T^4 - Tn^4) + sP (aR T^4 - E) = 0
    T4 = (0.25 * a * Tn ** 4 + sP * En / (1 + sP)) / (0.25 * a + sP * aR / (1 + sP))
    Ex = (En + sP * aR * T4) / (1 + sP)
    assert np.max(np.abs(T1 ** 4 - T4)) <= 1e-12 * T4
    assert np.max(np.abs(E1 - Ex)) <= 1e-12 * Ex
    assert np.max(np.abs(F1 - (Fn / (1 + sR))[:, None, None, None])) <= 1e-13


def test_periodic_grid_conserves_E_plus_gas_energy():
    rng = np.random.default_rng(5)
    shape = (4, 5, 6)
    rho = np.exp(0.3 * rng.standard_normal(shape))
    f = np.zeros((6,) + shape)
    f[:3] = 1.0 / 3.0
    f += 0.03 * rng.standard_normal((6,) + shape) * np.array([1, 1, 1, 0.5, 0.5, 0.5])[:, None, None, None]
    E = 1 + 0.3 * rng.random(shape)
    T = 1 + 0.2 * rng.random(shape)
    F = 0.1 * rng.standard_normal((3,) + shape)
    P = oracle.Problem(rho, 4.0 * np.ones(shape), 4.0 * np.ones(shape), f, dt=0.5, dx=0.25, cv=0.8, cv_cubic=True)
    E1, F1, T1, st = P.step(E, F, T, tol=1e-14)
    # the linearised iteration is Newton on the T-eliminated system (heat capacity alpha T^3 at T*):
    # quadratic convergence from this start (a constant-capacity linearisation needs about 10)
    assert st["picard_iters"] <= 4
    a = rho * 0.8
    before, after = np.sum(E + 0.25 * a * T ** 4), np.sum(E1 + 0.25 * a * T1 ** 4)
    assert abs(after - before) <= 1e-12 * before
    # the linear gas would give a different state (the pin has teeth)
    E2, _, T2, _ = oracle.Problem(rho, 4.0 * np.ones(shape), 4.0 * np.ones(shape), f, dt=0.5, dx=0.25,
                                  cv=0.8).step(E, F, T, tol=1e-14)
    assert np.max(np.abs(T2 - T1)) > 1e-3


def test_equilibrium_after_many_steps():
    shape = (2, 2, 3)
    rho, kap, cv, aR = 1.0, 50.0, 2.0, 1.0
    f = np.zeros((6,) + shape)
    f[:3] = 1.0 / 3.0
    P = oracle.Problem(np.full(shape, rho), np.full(shape, kap), np.full(shape, kap), f, dt=1.0, dx=0.5, aR=aR,
                       cv=cv, cv_cubic=True)
    E, F, T = np.full(shape, 3.0), np.zeros((3,) + shape), np.full(shape, 0.5)
    total = 3.0 + 0.25 * rho * cv * 0.5 ** 4
    for _ in range(40):
        E, F, T, _ = P.step(E, F, T, tol=1e-14)
    T4 = total / (aR + 0.25 * rho * cv)
    assert np.max(np.abs(T ** 4 - T4)) <= 1e-10 * T4
    assert np.max(np.abs(E - aR * T4)) <= 1e-10 * T4
