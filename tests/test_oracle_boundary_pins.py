"""Pins of the oracle's boundary kinds beyond periodic and Dirichlet.

- outflow (zero gradient, Sec. 3.3): the ghost is the boundary cell.  Uniform states stay
  uniform (the other pin file), but at tens of light-crossing times the boundary block of an
  optically thick cell is indefinite (test_boundary_stability.py).
- open (characteristic outflow): the ghost is the boundary cell with the amplitude of the
  incoming characteristic of the d-flux held at its start-of-step value.  Pinned by a streaming
  pulse that leaves the domain through implicit upwinding on an open line (closed form, no
  reflection) and by stationary uniform states.
- Marshak (Sec. 3.4): c E + 2 F_in = 4 F_inc at the wall.  Pinned by the exact steady state
  between two Marshak walls with no absorption, uniform sigma_R and f = I/3: a linear E and a
  constant F = -(c / (3 sigma_R)) dE/dx, which this first-order scheme reproduces exactly.
- reflect: a mirror.  Pinned against the mirror-symmetric periodic problem of twice the size,
  and by total energy conservation inside reflecting walls.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2202_08778_amd import workloads as W


def _axis_shape(n, axis):
    shape = [1, 1, 1]
    shape[2 - axis] = n
    return tuple(shape)


def _bc(axis, kind, other="periodic"):
    bc = [other] * 6
    bc[2 * axis] = bc[2 * axis + 1] = kind
    return bc


# --------------------------------------------------------------------- open

@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("nu", [0.6, 2.5])
def test_open_streaming_pulse_leaves_without_reflection(axis, nu):
    """sigma = 0, f = e_d e_d, F = c E: the scheme is implicit upwinding of w = E + F/c, and with
    open faces the line is open: E_i <- (E_i + nu E_{i-1}^new) / (1 + nu), the first cell fed by
    its own old value (zero here), nothing coming back from the far wall.  36 cells of travel carry
    most of the pulse out; F = c E holds throughout (the left-going characteristic stays zero)."""
    n, c = 40, 1.7
    h = 1.0 / n
    shape = _axis_shape(n, axis)
    x = np.arange(n)
    E0 = np.where((x >= 12) & (x < 28), np.sin(np.pi * (x - 11) / 17.0) ** 2, 0.0) + 0.0
    E0[20] += 0.3
    F0 = np.zeros((3,) + shape)
    F0[axis] = (c * E0).reshape(shape)
    f = np.zeros((6,) + shape)
    f[axis] = 1.0
    zero = np.zeros(shape)
    P = oracle.Problem(np.ones(shape), zero, zero, f, nu * h / c, h, _bc(axis, "open"), c=c)
    E, F, T = E0.reshape(shape), F0, np.ones(shape)
    ref = E0.copy()
    for step in range(int(36 / nu) + 1):
        E, F, T, st = P.step(E, F, T, tol=1e-15)
        new = np.empty(n)
        prev = 0.0
        for i in range(n):
            new[i] = (ref[i] + nu * prev) / (1.0 + nu)
            prev = new[i]
        ref = new
        got = E.reshape(n)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(E0), step
        assert np.max(np.abs(F[axis].reshape(n) - c * got)) <= 1e-12 * c * np.max(E0)
    assert ref.sum() < 0.5 * E0.sum()   # most of the pulse has left


@pytest.mark.parametrize("oblique", [False, True])
def test_open_wall_feeds_the_incoming_beam_its_old_amplitude(oblique):
    """A beam moving in -x (f = n n, F = c E n, n = -e_x or (-e_x + e_y)/sqrt 2, no opacity) is an
    eigenvector of the x-flux with speed a = c sqrt(f_xx), so the scheme upwinds it at
    nu_a = a dt / h.  The pulse starts against the right wall, where the beam is the incoming
    characteristic: the open ghost holds its amplitude at the old value of the boundary cell, so
    that cell keeps its value and the rest follows (1 + nu_a) E_i = E_i^old + nu_a E_{i+1}^new.
    The beam stays a beam (F = c E n); the left wall lets it out."""
    n_, c, nu = 30, 1.7, 1.4
    h = 1.0 / n_
    shape = (1, 1, n_)
    nvec = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0) if oblique else np.array([-1.0, 0.0, 0.0])
    f = np.zeros((6,) + shape)
    for q, (a_, b_) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        f[q] = nvec[a_] * nvec[b_]
    x = np.arange(n_)
    E0 = np.exp(-((x - (n_ - 3)) / 4.0) ** 2)
    F0 = np.stack([c * nvec[q] * E0 for q in range(3)]).reshape((3,) + shape)
    zero = np.zeros(shape)
    nu_a = nu * math.sqrt(f[0].ravel()[0])
    P = oracle.Problem(np.ones(shape), zero, zero, f, nu * h / c, h, _bc(0, "open"), c=c)
    E, F, T = E0.reshape(shape), F0, np.ones(shape)
    ref = E0.copy()
    for step in range(12):
        E, F, T, st = P.step(E, F, T, tol=1e-15)
        new = np.empty(n_)
        new[n_ - 1] = ref[n_ - 1]
        for i in range(n_ - 2, -1, -1):
            new[i] = (ref[i] + nu_a * new[i + 1]) / (1.0 + nu_a)
        ref = new
        got = E.ravel()
        assert np.max(np.abs(got - ref)) <= 1e-12, step
        for q in range(3):
            assert np.max(np.abs(F[q].ravel() - c * nvec[q] * got)) <= 1e-12 * c, (step, q)


def test_open_wall_removes_the_incoming_characteristic_flux():
    """Linear operator, no opacity (so the corrected speed of a wall face is a = c sqrt(f_dd)): the
    HLL flux through a wall is then (F(U_c) + F(U_g))/2 -+ a (U_g - U_c)/2, and the open ghost
    U_g = U_c - alpha_in r_in (alpha_in = (E +- F_d / a)/2 the incoming amplitude, r_in =
    (1, +-c^2 f_d. / a) its eigenvector of the d-flux) leaves exactly the outgoing part.  Against
    the zero-gradient wall (whose flux is F(U_c)) the boundary cell's rows change by
    (dt/h) a alpha_in r_in."""
    rng = np.random.default_rng(3)
    shape = (3, 4, 5)
    c, h, dt = 1.7, 0.2, 0.9
    A = rng.standard_normal((3, 3) + shape) * 0.1
    f = np.empty((6,) + shape)
    for q, (a_, b_) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        f[q] = (1 / 3 if a_ == b_ else 0.0) + 0.5 * (A[a_, b_] + A[b_, a_])
    zero = np.zeros(shape)
    rho = np.ones(shape)
    x = rng.standard_normal((4,) + shape)
    dE = rng.uniform(1, 2, shape)
    y_open = oracle.Problem(rho, zero, zero, f, dt, h, _bc(0, "open"), c=c).apply(x, dE)
    y_zg = oracle.Problem(rho, zero, zero, f, dt, h, _bc(0, "outflow"), c=c).apply(x, dE)
    want = np.zeros_like(y_open)
    TX = (0, 3, 4)   # f_xx, f_xy, f_xz
    for side, i in ((0, 0), (1, shape[2] - 1)):
        s_in = 1.0 if side == 0 else -1.0
        a = c * np.sqrt(f[0][..., i])
        alpha = 0.5 * (x[0][..., i] + s_in * x[1][..., i] / a)
        want[0][..., i] += (dt / h) * a * alpha
        for j in range(3):
            want[1 + j][..., i] += (dt / h) * a * alpha * s_in * c * c * f[TX[j]][..., i] / a
    assert np.max(np.abs((y_open - y_zg) - want)) <= 1e-13 * np.max(np.abs(y_zg))
    assert np.max(np.abs(want)) > 0.1


@pytest.mark.parametrize("dt_cross", [0.5, 50.0, 1e4])
def test_open_keeps_a_stationary_uniform_state(dt_cross):
    """A uniform medium in radiative equilibrium (E = aR T^4, F = 0) is a solution for any dt with
    open faces: every ghost equals its cell."""
    shape = (4, 5, 6)
    f = np.zeros((6,) + shape)
    f[0], f[1], f[2], f[3] = 0.5, 0.3, 0.2, 0.05
    h = 1.0 / 6
    T0 = 0.8
    P = oracle.Problem(np.full(shape, 1.3), np.full(shape, 7.0), np.full(shape, 7.0), f, dt_cross * h, h, "open",
                       aR=1.1)
    E0 = np.full(shape, 1.1 * T0 ** 4)
    E, F, T, st = P.step(E0, np.zeros((3,) + shape), np.full(shape, T0), tol=1e-15)
    assert np.max(np.abs(E - E0)) <= 1e-14 * E0.max()
    assert np.max(np.abs(F)) <= 1e-14 * E0.max()
    assert np.max(np.abs(T - T0)) <= 1e-14


@pytest.mark.parametrize("axis", [0, 2])
def test_open_keeps_a_uniform_beam(axis):
    """A uniform beam (sigma = 0, f = e_d e_d, F = c E) enters through one wall and leaves through
    the other: the open wall holds the incoming amplitude at its old value, so the beam is a
    stationary solution for any dt."""
    n, c = 10, 1.3
    shape = _axis_shape(n, axis)
    f = np.zeros((6,) + shape)
    f[axis] = 1.0
    zero = np.zeros(shape)
    F0 = np.zeros((3,) + shape)
    F0[axis] = c * 0.7
    for dt in (0.05, 30.0):
        P = oracle.Problem(np.ones(shape), zero, zero, f, dt, 0.1, _bc(axis, "open"), c=c)
        E, F, T, st = P.step(np.full(shape, 0.7), F0, np.ones(shape), tol=1e-15)
        assert np.max(np.abs(E - 0.7)) <= 1e-14
        assert np.max(np.abs(F - F0)) <= 1e-14


# ------------------------------------------------------------------ Marshak

def _marshak_profile(n, c, sig, FL, FR):
    """Cell-centre E and the constant F of the steady state between Marshak walls at x = 0, 1."""
    L = 1.0
    g = 4.0 * (FR - FL) / (c * (L + 4.0 / (3.0 * sig)))
    F = -c * g / (3.0 * sig)
    E0 = (4.0 * FL - 2.0 * F) / c
    x = (np.arange(n) + 0.5) / n
    return E0 + g * x, F


@pytest.mark.parametrize("dt_cross", [0.3, 50.0, 1e4])
def test_marshak_walls_keep_the_steady_diffusion_state(dt_cross):
    """No absorption, uniform sigma_R, f = I/3, Marshak walls with incident fluxes F_L (at x = 0) and
    F_R (at x = 1): E = E0 + g x and F = -(c / 3 sigma_R) g with c E(0) + 2F = 4 F_L and
    c E(1) - 2F = 4 F_R.  Central differences of a linear field are exact, the wall ghost is its
    linear continuation, so the state is returned unchanged for any dt."""
    n, c, sig = 24, 1.3, 5.0
    h = 1.0 / n
    FL, FR = 2.0, 0.5
    shape = (3, 2, n)
    Ex, Fx = _marshak_profile(n, c, sig, FL, FR)
    E = np.broadcast_to(Ex, shape).copy()
    F = np.zeros((3,) + shape)
    F[0] = Fx
    f = np.zeros((6,) + shape)
    f[:3] = 1 / 3
    bc = ["marshak", "marshak", "periodic", "periodic", "periodic", "periodic"]
    P = oracle.Problem(np.ones(shape), np.zeros(shape), np.full(shape, sig), f, dt_cross * h / c, h, bc, c=c,
                       finc=[FL, FR, 0, 0, 0, 0])
    E1, F1, T1, st = P.step(E, F, np.ones(shape), tol=1e-15, lin_rtol=1e-15)
    assert np.max(np.abs(E1 - E)) <= 1e-12 * np.max(np.abs(E))
    assert np.max(np.abs(F1[0] - Fx)) <= 1e-12 * abs(Fx)
    assert np.max(np.abs(F1[1:])) <= 1e-12 * abs(Fx)


def test_marshak_relaxes_onto_the_steady_state():
    """From a cold start (E = F = 0) a very long step reaches the closed-form steady state (the
    slowest diffusion mode decays by about dt c / (9 L^2 sigma), so 1e12 crossings leave ~1e-10)."""
    n, c, sig = 16, 1.0, 3.0
    h = 1.0 / n
    shape = (1, 1, n)
    Ex, Fx = _marshak_profile(n, c, sig, 1.0, 0.0)
    f = np.zeros((6,) + shape)
    f[:3] = 1 / 3
    bc = ["marshak", "marshak", "periodic", "periodic", "periodic", "periodic"]
    P = oracle.Problem(np.ones(shape), np.zeros(shape), np.full(shape, sig), f, 1e12 * h / c, h, bc, c=c,
                       finc=[1.0, 0.0, 0, 0, 0, 0])
    E1, F1, T1, st = P.step(np.zeros(shape), np.zeros((3,) + shape), np.ones(shape), tol=1e-15, lin_rtol=1e-15)
    assert np.max(np.abs(E1.ravel() - Ex)) <= 1e-7 * np.max(Ex)
    assert np.max(np.abs(F1[0].ravel() - Fx)) <= 1e-7 * abs(Fx)


def test_marshak_wall_feeds_a_cold_medium():
    """Sec. 3.4 setting in code units (cubic heat capacity, a reflecting far wall): a cold absorbing
    medium heated through a Marshak wall.  The energy that entered equals the time integral of
    the wall's HLL flux, Phi = (F_g + F_0)/2 - C (E_0 - E_g)/2 with the ghost of the new state
    (F_g = F_0, E_g = 8 F_inc / c - 4 F_0 / c - E_0) and C the cell's own corrected speed; the
    reflecting wall passes nothing.  The front moves away from the wall."""
    n, c, sig, cv = 64, 1.0, 40.0, 40.0
    h = 0.5 / n
    shape = (1, 1, n)
    f = np.zeros((6,) + shape)
    f[:3] = 1 / 3
    bc = ["marshak", "reflect", "periodic", "periodic", "periodic", "periodic"]
    Finc = 1.0
    dt = h / c
    P = oracle.Problem(np.ones(shape), np.full(shape, sig), np.full(shape, sig), f, dt, h, bc, c=c, cv=cv,
                       finc=[Finc, 0, 0, 0, 0, 0], cv_cubic=True)
    tau = (10 * h * sig) ** 2 / (2 / 3)
    C = c * math.sqrt(1 / 3) * math.sqrt(-math.expm1(-tau) / tau)
    E, F, T = np.zeros(shape), np.zeros((3,) + shape), np.zeros(shape)
    inflow = 0.0
    for _ in range(40):
        E, F, T, st = P.step(E, F, T, tol=1e-13)
        E0, F0 = E.ravel()[0], F[0].ravel()[0]
        Eg = 8 * Finc / c - 4 * F0 / c - E0
        inflow += (dt / h) * (F0 - 0.5 * C * (E0 - Eg))
    total = math.fsum(E.ravel()) + math.fsum((0.25 * cv * T ** 4).ravel())
    assert abs(total - inflow) <= 1e-10 * total
    prof = E.ravel()
    assert prof[0] > prof[n // 4] > prof[n // 2]


# ------------------------------------------------------------------ reflect

def _mirror_pair(n, seed):
    """A random medium on [0, L) and its mirror image on [-L, 0): fields even in x, F_x and the
    tensor components f_xy, f_xz odd."""
    rng = np.random.default_rng(seed)
    shape = (3, 2, n)
    d = W.mixed_depth(shape=shape, seed=seed, steps=1, dt_cross=8.0)
    for k in ("rho", "kP", "kR", "E", "T"):
        d[k] = d[k].copy()
    d["F"] = 0.2 * rng.standard_normal((3,) + shape)

    def double(a, odd=False):
        m = a[..., ::-1]
        return np.concatenate([-m if odd else m, a], axis=-1)

    full = {k: double(d[k]) for k in ("rho", "kP", "kR", "E", "T")}
    full["F"] = np.stack([double(d["F"][0], True), double(d["F"][1]), double(d["F"][2])])
    full["f"] = np.stack([double(d["f"][q], odd=q in (3, 4)) for q in range(6)])
    return d, full


def test_reflecting_walls_match_the_mirrored_periodic_problem():
    n = 7
    d, full = _mirror_pair(n, 21)
    h = d["dx"]
    bc = ["reflect", "reflect", "periodic", "periodic", "periodic", "periodic"]
    Ph = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], h, bc)
    Pf = oracle.Problem(full["rho"], full["kP"], full["kR"], full["f"], d["dt"], h, "periodic")
    a = Ph.step(d["E"], d["F"], d["T"], tol=1e-14)
    b = Pf.step(full["E"], full["F"], full["T"], tol=1e-14)
    half = (Ellipsis, slice(n, 2 * n))
    assert np.linalg.norm(a[0] - b[0][half]) <= 1e-11 * np.linalg.norm(a[0])
    assert np.linalg.norm(a[1] - b[1][half]) <= 1e-11 * np.linalg.norm(a[1])
    assert np.linalg.norm(a[2] - b[2][half]) <= 1e-11 * np.linalg.norm(a[2])


def test_reflecting_box_conserves_total_energy():
    d = W.periodic_clumpy(shape=(5, 6, 7), seed=4)
    P = oracle.Problem(d["rho"], d["kP"], d["kR"], d["f"], d["dt"], d["dx"], "reflect")
    E, F, T, st = P.step(d["E"], d["F"], d["T"], tol=1e-14)
    alpha = d["rho"] * d["cv"]
    e0 = math.fsum((d["E"] + alpha * d["T"]).ravel())
    e1 = math.fsum((E + alpha * T).ravel())
    assert abs(e1 - e0) <= 1e-11 * e0
