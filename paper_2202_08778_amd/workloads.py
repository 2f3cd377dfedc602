"""Seeded synthetic workloads for the implicit radiation step.

This module only draws inputs; it holds none of the method's arithmetic.  The
paper has no public dataset: its 3D problems are clumpy media whose cell
optical depth spans many decades (shadow tests, Sec. 3.6) and its 1D tests
are analytic (Sec. 3.1, 3.3).  The generators below stand in for those with
the same structure: lognormal density, a spatially correlated optical-depth
field that is log-uniform over a stated range, a random symmetric
positive-definite unit-trace Eddington tensor per cell and a central Gaussian
radiation source.

Conventions: a scalar field has shape (nz, ny, nx), x fastest; F has shape
(3, nz, ny, nx); the Eddington tensor f has shape (6, nz, ny, nx) ordered
xx, yy, zz, xy, xz, yz.  All arrays are float64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr

TENSOR_ORDER = ("xx", "yy", "zz", "xy", "xz", "yz")

# cgs constants used by the physical test problems
C_LIGHT = 2.99792458e10
A_RAD = 7.5657e-15
R_GAS = 8.314462618e7


def _smooth_periodic(G, sigma):
    """Periodic Gaussian filter (sigma in cells) through the FFT, then restandardised."""
    shape = G.shape
    k = [np.fft.fftfreq(n) for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    Gh = np.fft.rfftn(G)
    for ax, kk in enumerate(k):
        s = [1] * len(shape)
        s[ax] = kk.size
        Gh *= np.exp(-2.0 * (math.pi * sigma * kk) ** 2).reshape(s)
    out = np.fft.irfftn(Gh, s=shape, axes=tuple(range(len(shape))))
    out -= out.mean()
    out /= out.std()
    return out


def _random_rotations(rng, shape):
    """Haar-distributed rotations (det +1) from normalised Gaussian quaternions; (3, 3, *shape)."""
    q = rng.standard_normal((4,) + shape)
    q /= np.sqrt((q * q).sum(axis=0))
    w, x, y, z = q
    R = np.empty((3, 3) + shape)
    R[0, 0] = 1 - 2 * (y * y + z * z); R[0, 1] = 2 * (x * y - z * w); R[0, 2] = 2 * (x * z + y * w)
    R[1, 0] = 2 * (x * y + z * w); R[1, 1] = 1 - 2 * (x * x + z * z); R[1, 2] = 2 * (y * z - x * w)
    R[2, 0] = 2 * (x * z - y * w); R[2, 1] = 2 * (y * z + x * w); R[2, 2] = 1 - 2 * (x * x + y * y)
    return R


def random_spd_unit_trace(rng, shape):
    """f = Q diag(l) Q^T with l ~ Dirichlet(2,2,2) and Q Haar on SO(3); returns (6, *shape)."""
    l = rng.gamma(2.0, size=(3,) + shape)
    l /= l.sum(axis=0)
    Q = _random_rotations(rng, shape)
    f = np.empty((6,) + shape)
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for n, (a, b) in enumerate(pairs):
        f[n] = (Q[a, 0] * Q[b, 0] * l[0] + Q[a, 1] * Q[b, 1] * l[1] + Q[a, 2] * Q[b, 2] * l[2])
    return f


def isotropic_plus_traceless(rng, shape, amp):
    """f = I/3 + amp * P, P symmetric traceless with unit Frobenius norm from iid N(0,1) entries."""
    M = rng.standard_normal((3, 3) + shape)
    S = 0.5 * (M + M.transpose(1, 0, *range(2, M.ndim)))
    tr = (S[0, 0] + S[1, 1] + S[2, 2]) / 3.0
    for a in range(3):
        S[a, a] -= tr
    S /= np.sqrt((S * S).sum(axis=(0, 1)))
    f = np.empty((6,) + shape)
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for n, (a, b) in enumerate(pairs):
        f[n] = amp * S[a, b] + (1.0 / 3.0 if a == b else 0.0)
    return f


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def periodic_clumpy(n=32, seed=1, shape=None):
    """Plain FP64 case: periodic cube, lognormal(0.5) density, kappa = 10, f = I/3 + 0.05 P,
    E and T = 1 + 0.1 N(0,1), F = 0, dt = 100 cell light-crossing times, c = aR = cv = 1."""
    rng = np.random.default_rng(seed)
    shape = shape or (n, n, n)
    nz, ny, nx = shape
    h = 1.0 / nx
    rho = np.exp(0.5 * rng.standard_normal(shape))
    kP = np.full(shape, 10.0)
    kR = np.full(shape, 10.0)
    f = isotropic_plus_traceless(rng, shape, 0.05)
    E = 1.0 + 0.1 * rng.standard_normal(shape)
    T = 1.0 + 0.1 * rng.standard_normal(shape)
    F = np.zeros((3,) + shape)
    return dict(E=E, F=F, T=T, rho=rho, kP=kP, kR=kR, f=f, dt=100.0 * h, dx=h, bc="periodic",
                c=1.0, aR=1.0, cv=1.0, steps=1, name=f"periodic_clumpy_{nx}x{ny}x{nz}")


def _mixed_depth(rng, shape, sigma_rho, lg_lo, lg_hi, h):
    rho = np.exp(sigma_rho * rng.standard_normal(shape))
    G = _smooth_periodic(rng.standard_normal(shape), 4.0)
    tau = 10.0 ** (lg_lo + (lg_hi - lg_lo) * ndtr(G))
    kap = tau / (rho * h)
    return rho, kap


def _gaussian_source(shape, h, peak, width_cells, aR, T):
    nz, ny, nx = shape
    z = (np.arange(nz) + 0.5) / nz - 0.5
    y = (np.arange(ny) + 0.5) / ny - 0.5
    x = (np.arange(nx) + 0.5) / nx - 0.5
    r2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
    w = width_cells * h
    return aR * T ** 4 + peak * np.exp(-r2 / (2.0 * w * w))


def mixed_depth(n=128, seed=2, sigma_rho=1.5, lg_tau=(-3.0, 3.0), dt_cross=50.0, steps=10,
                fp32_exact=False, shape=None, bc="open"):
    """Cube with lognormal density, cell optical depth log-uniform over lg_tau and spatially
    correlated (Gaussian filter, 4 cells), random SPD unit-trace f, Gaussian source in E
    (peak 1e3, sigma 4 cells) on an equilibrium background, T = 0.1, F = 0, dt = dt_cross h / c.

    The outflow faces of this medium are open (characteristic) faces by default: with the
    zero-gradient ghost (the current boundary cell) and dt of tens of light-crossing times the
    discrete operator has eigenvalues with negative real part in optically thick boundary cells,
    so that reading is not well posed here; it remains available as bc="outflow"."""
    rng = np.random.default_rng(seed)
    shape = shape or (n, n, n)
    h = 1.0 / shape[2]
    rho, kap = _mixed_depth(rng, shape, sigma_rho, lg_tau[0], lg_tau[1], h)
    f = random_spd_unit_trace(rng, shape)
    T = np.full(shape, 0.1)
    E = _gaussian_source(shape, h, 1e3, 4.0, 1.0, T)
    F = np.zeros((3,) + shape)
    d = dict(E=E, F=F, T=T, rho=rho, kP=kap.copy(), kR=kap, f=f, dt=dt_cross * h, dx=h, bc=bc,
             c=1.0, aR=1.0, cv=1.0, steps=steps, name=f"mixed_depth_{bc}_{shape[2]}x{shape[1]}x{shape[0]}")
    if fp32_exact:
        for k in ("E", "F", "T", "rho", "kP", "kR", "f"):
            d[k] = _f32(d[k])
    return d


def mixed_depth_256(n=256, seed=3, steps=5):
    """Precision-comparison case: the mixed-depth recipe at 256^3, FP32-exact inputs."""
    d = mixed_depth(n=n, seed=seed, steps=steps, fp32_exact=True)
    d["name"] = f"mixed_depth_fp32exact_{n}^3"
    return d


def mixed_depth_512(n=512, seed=5, steps=3):
    """Scale case: lognormal sigma 2, optical depth 1e-4..1e4, dt = 200 crossings, FP32-exact."""
    d = mixed_depth(n=n, seed=seed, sigma_rho=2.0, lg_tau=(-4.0, 4.0), dt_cross=200.0, steps=steps,
                    fp32_exact=True)
    d["name"] = f"mixed_depth_sigma2_{n}^3"
    return d


SIZES = (8, 12, 16, 24, 32)


def batched_blocks(nblocks=1024, seed=4, ng=2, sizes=SIZES, fp32_exact=True):
    """Independent AMR-like blocks: edge n_b uniform on sizes, h_b = 1/n_b, ng ghost layers of fixed
    Dirichlet (E, F) data, dt_b = 10^U(0,3) h_b / c, scalar kappa_b = 10^U(-2,3); rho, f, E, T as
    in the mixed-depth recipe, drawn over the whole (n_b + 2 ng)^3 region."""
    rng = np.random.default_rng(seed)
    blocks = []
    for _ in range(nblocks):
        n = int(rng.choice(sizes))
        m = n + 2 * ng
        shape = (m, m, m)
        h = 1.0 / n
        dt = 10.0 ** rng.uniform(0.0, 3.0) * h
        kap = 10.0 ** rng.uniform(-2.0, 3.0)
        rho = np.exp(1.5 * rng.standard_normal(shape))
        f = random_spd_unit_trace(rng, shape)
        T = np.full(shape, 0.1)
        z = (np.arange(m) - ng + 0.5) / n - 0.5
        r2 = z[:, None, None] ** 2 + z[None, :, None] ** 2 + z[None, None, :] ** 2
        E = 1.0 * T ** 4 + 1e3 * np.exp(-r2 / (2.0 * (4.0 * h) ** 2))
        F = np.zeros((3,) + shape)
        b = dict(n=n, ng=ng, dx=h, dt=dt, E=E, F=F, T=T, rho=rho, kP=np.full(shape, kap),
                 kR=np.full(shape, kap), f=f)
        if fp32_exact:
            for k in ("E", "F", "T", "rho", "kP", "kR", "f"):
                b[k] = _f32(b[k])
        blocks.append(b)
    return dict(blocks=blocks, c=1.0, aR=1.0, cv=1.0, name=f"batched_{nblocks}_blocks")


def pulse_1d(regime="streaming", n=1024):
    """Radiating Gaussian pulse of Sec. 3.1 in cgs units along x (ny = nz = 1)."""
    rho0 = 1e-20
    if regime == "streaming":
        x0, kap, fxx, bc = 0.5, 1.0, 1.0, ("periodic", "periodic", "periodic")
    elif regime == "static":
        x0, kap, fxx, bc = 5.0, 4e21, 1.0 / 3.0, ("outflow", "periodic", "periodic")
    elif regime == "equilibrium":
        x0, kap, fxx, bc = 5.0, 4e24, 1.0 / 3.0, ("outflow", "periodic", "periodic")
    else:
        raise ValueError(regime)
    h = 2.0 * x0 / n
    x = -x0 + (np.arange(n) + 0.5) * h
    mu = 20.0
    shape = (1, 1, n)
    E = np.exp(-(mu * x) ** 2).reshape(shape)
    F = np.zeros((3,) + shape)
    if regime == "streaming":
        F[0] = C_LIGHT * E
    else:
        D = C_LIGHT / (3.0 * rho0 * kap)
        F[0] = (2.0 * D * mu * mu * x).reshape(shape) * E
    kR = np.full(shape, kap)
    f = np.zeros((6,) + shape)
    f[0] = fxx
    if regime != "streaming":
        f[1] = f[2] = fxx
    return dict(E=E, F=F, T=np.zeros(shape), rho=np.full(shape, rho0), kP=np.zeros(shape), kR=kR, f=f,
                dt=h / C_LIGHT, dx=h, bc=bc, c=C_LIGHT, aR=A_RAD, cv=1.0, x=x, mu=mu, kappa=kap,
                rho0=rho0, name=f"pulse_{regime}_{n}")


def thermal_coupling(rho, n=16, T0=100.0, Er0=7.567e-13, sigma_P=1.0, gamma=5.0 / 3.0, mu=0.6):
    """Uniform non-equilibrium gas/radiation box of Sec. 3.3 (cgs), rho * kappa_P = sigma_P."""
    shape = (1, 1, n)
    cv = R_GAS / (mu * (gamma - 1.0))  # internal energy per unit mass per kelvin
    h = 1.0 / n
    f = np.zeros((6,) + shape)
    f[0] = f[1] = f[2] = 1.0 / 3.0
    return dict(E=np.full(shape, Er0), F=np.zeros((3,) + shape), T=np.full(shape, T0),
                rho=np.full(shape, rho), kP=np.full(shape, sigma_P / rho), kR=np.full(shape, sigma_P / rho),
                f=f, dx=h, bc=("outflow", "periodic", "periodic"), c=C_LIGHT, aR=A_RAD, cv=cv,
                t_therm=1.0 / (sigma_P * C_LIGHT), name=f"thermal_rho{rho:g}")


def two_level(nc=(32, 32, 32), lo=(8, 8, 8), hi=(24, 24, 24), seed=6, sigma_rho=1.0, lg_tau=(-2.0, 2.0),
              dt_cross=20.0, bc="periodic", fp32_exact=False):
    """Two-level composite grid: the mixed-depth medium on a coarse grid (width h = 1/nx) with the
    box [lo, hi) (coarse cells, x, y, z) refined by 2.  Fine cells inherit their parent's opacity
    and tensor with sub-cell variation (density times a lognormal factor of sigma 0.3, tensor the
    mean of the parent's and a fresh random SPD unit-trace one); E is the Gaussian source (peak
    1e3, sigma 4 coarse cells) on an equilibrium background sampled at every cell centre, T = 0.1,
    F = 0, dt = dt_cross h / c.  Arrays are returned per level as (coarse, fine) pairs."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = nc
    sc = (nz, ny, nx)
    nf = tuple(2 * (b - a) for a, b in zip(lo, hi))
    sf = (nf[2], nf[1], nf[0])
    h = 1.0 / nx
    rho_c, kap_c = _mixed_depth(rng, sc, sigma_rho, lg_tau[0], lg_tau[1], h)
    f_c = random_spd_unit_trace(rng, sc)
    box = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    inj = lambda a: a.repeat(2, axis=-1).repeat(2, axis=-2).repeat(2, axis=-3)
    rho_f = inj(rho_c[box]) * np.exp(0.3 * rng.standard_normal(sf))
    kap_f = inj(kap_c[box])
    f_f = 0.5 * (inj(f_c[(slice(None),) + box]) + random_spd_unit_trace(rng, sf))

    def centres(n, a, w):
        return (a + (np.arange(n) + 0.5) * w) - 0.5

    def source(shape_xyz, org, w, T):
        x, y, z = (centres(shape_xyz[d], org[d], w) for d in range(3))
        r2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
        s = 4.0 * h
        return T ** 4 + 1e3 * np.exp(-r2 / (2.0 * s * s))

    T_c, T_f = np.full(sc, 0.1), np.full(sf, 0.1)
    E_c = source(nc, (0.0, 0.0, 0.0), h, T_c)
    E_f = source(nf, tuple(lo[d] * h for d in range(3)), 0.5 * h, T_f)
    d = dict(nc=tuple(nc), lo=tuple(lo), hi=tuple(hi), E=(E_c, E_f), F=(np.zeros((3,) + sc), np.zeros((3,) + sf)),
             T=(T_c, T_f), rho=(rho_c, rho_f), kP=(kap_c.copy(), kap_f.copy()), kR=(kap_c, kap_f), f=(f_c, f_f),
             dt=dt_cross * h, dx=h, bc=bc, c=1.0, aR=1.0, cv=1.0,
             name=f"two_level_{bc}_{nx}x{ny}x{nz}_box{'-'.join(map(str, lo))}_{'-'.join(map(str, hi))}")
    if fp32_exact:
        for k in ("E", "F", "T", "rho", "kP", "kR", "f"):
            d[k] = tuple(_f32(a) for a in d[k])
    return d
