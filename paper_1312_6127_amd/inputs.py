"""Seeded synthetic inputs and workload definitions.

This module holds no step of the GRRMHD method: it only describes grids and
draws initial primitive states (and opacities) from a counter-based
generator.  Both the GPU path's tests/benchmarks and the CPU oracle's tests
read their inputs from here, so the two always see identical bytes.

Counter-based generator: SplitMix64 (Steele, Lea & Flood 2014), value of draw
``d`` of cell ``c`` under seed ``s`` is ``splitmix64(s ^ (0x9E3779B97F4A7C15 *
(16 c + d)))`` mapped to a double in [0, 1) from its top 53 bits.
"""
from __future__ import annotations

import math

import numpy as np

NPRIM = 12
# primitive slots: rho0, u_g, u~^1..3 (gas), B^1..3, Ebar, u~^1..3 (radiation)
RHO, UU, U1, U2, U3, B1, B2, B3, ER, F1, F2, F3 = range(12)

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, cells: np.ndarray, draw: int) -> np.ndarray:
    """U[0,1) for each cell index in ``cells`` (int64 array), draw number ``draw``."""
    c = np.asarray(cells, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = (c * np.uint64(16) + np.uint64(draw)) * np.uint64(0x9E3779B97F4A7C15)
    z = splitmix64(np.uint64(seed) ^ ctr)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ---------------------------------------------------------------------------
# parameter sets
# ---------------------------------------------------------------------------

def default_params(**kw) -> dict:
    """Numerical parameters with the paper's defaults (Sec. 5 intro, Sec. 4.10-4.11)."""
    p = dict(
        n=(1, 1, 1), ng=2, metric="minkowski", a=0.0, R0=0.0,
        xlo=(0.0, 0.0, 0.0), xhi=(1.0, 1.0, 1.0),
        bc_lo=("periodic",) * 3, bc_hi=("periodic",) * 3,
        gam=5.0 / 3.0, arad=1.0, gamma_max=100.0, courant=0.5, flux="llf",
        precision="fp64", r_fp64=2.0,
        tol_pmhd=1e-12, tol_urad=1e-9, tol_accept=1e-9, tol_fail=1e-7,
        max_iter=20, roundoff=1,
        rho_floor=1e-20, u_floor=1e-22, bsq_rho_max=200.0, bsq_u_max=1e5,
        u_rho_max=1e10, erad_floor=1e-150, scheme="rk3", recon="mc", cold=1, cascade=0,
        ct="flux",
    )
    p.update(kw)
    return p


def nalloc(p: dict) -> tuple[int, int, int]:
    return tuple(n + 2 * (p["ng"] if n > 1 else 0) for n in p["n"])


def ncell(p: dict) -> int:
    a = nalloc(p)
    return a[0] * a[1] * a[2]


def interior(p: dict):
    """Slices selecting interior cells of an array shaped [..., N3, N2, N1]."""
    sl = []
    for d in (2, 1, 0):
        g = p["ng"] if p["n"][d] > 1 else 0
        sl.append(slice(g, g + p["n"][d]))
    return tuple(sl)


def cell_coords(p: dict):
    """Internal coordinates (x1, x2, x3) of every allocated cell centre, [N3, N2, N1]."""
    out = []
    na = nalloc(p)
    for d in range(3):
        g = p["ng"] if p["n"][d] > 1 else 0
        dx = (p["xhi"][d] - p["xlo"][d]) / p["n"][d]
        out.append(p["xlo"][d] + (np.arange(na[d]) - g + 0.5) * dx)
    x3, x2, x1 = np.meshgrid(out[2], out[1], out[0], indexing="ij")
    return x1, x2, x3


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def shock_tube_1d(n: int = 256, **kw):
    """1-D Minkowski radiative shock tube: x in [-1, 1], outflow, gamma = 5/3,
    no field, left (rho, p) = (1, 1e-2), right (0.125, 1e-3), at rest,
    Ebar = a_rad T^4 with T = p/rho, zero flux (radiation frame = gas frame),
    a_rad = 1e-2, per-mass opacities chi_abs = 1, chi_es = 0.5, HLL, C = 0.5.
    kw: further parameters (e.g. ng=4, recon="ppm")."""
    p = default_params(n=(n, 1, 1), xlo=(-1.0, 0.0, 0.0), xhi=(1.0, 1.0, 1.0),
                       bc_lo=("outflow",) * 3, bc_hi=("outflow",) * 3,
                       arad=1e-2, flux="hll")
    p.update(kw)
    N = ncell(p)
    x1, _, _ = cell_coords(p)
    x1 = x1.reshape(-1)
    P = np.zeros((NPRIM, N))
    left = x1 < 0.0
    rho = np.where(left, 1.0, 0.125)
    pg = np.where(left, 1e-2, 1e-3)
    P[RHO] = rho
    P[UU] = pg / (p["gam"] - 1.0)
    T = pg / rho
    P[ER] = p["arad"] * T ** 4
    chi_abs = np.full(N, 1.0)
    chi_es = np.full(N, 0.5)
    return p, P, chi_abs, chi_es


def disk_params(n=(128, 64, 1), a=0.9375, rin=1.2, rout=40.0, flux="llf", **kw):
    threed = n[2] > 1
    p = default_params(
        n=tuple(n), metric="ks", a=a, R0=0.0,
        xlo=(math.log(rin), 0.0, 0.0), xhi=(math.log(rout), 1.0, 1.0),
        bc_lo=("outflow", "polar" if threed else "reflect", "periodic"),
        bc_hi=("outflow", "polar" if threed else "reflect", "periodic"),
        gam=5.0 / 3.0, arad=1.247e5, flux=flux,
        rho_floor=1e-12, u_floor=1e-14,
    )
    p.update(kw)
    return p


def _ks_sqrtg(a, r, th):
    """sqrt(-g) of the Kerr-Schild metric in (r, theta, phi): Sigma |sin theta|.
    Used only to express the initial poloidal field as a discrete curl."""
    return (r * r + a * a * np.cos(th) ** 2) * np.abs(np.sin(th))


def accretion_disk(n=(128, 64, 1), seed=2, a=0.9375, rin=1.2, rout=40.0, flux="llf",
                   perturb3d=None, faces=False, **kw):
    """Synthetic accretion-shaped state on a log-r Kerr-Schild grid.

    rho0 = (r/r_in)^-1.5, p = 0.1 rho0/r, radial inflow u~^1 = -sqrt(2/r)/r
    (coordinate component in x1 = ln r, i.e. u~^r = -sqrt(2/r)), poloidal
    field from A_phi = max(rho0/rho_max - 0.2, 0) (r sin theta)^2 by a
    corner-centred discrete curl scaled to max p_gas / max p_mag = 100,
    pressure x (1 + 0.02 (U - 1/2)), Ebar = a_rad T^4 with T = p/rho0 and
    radiation frame = gas frame, chi_abs from a per-cell optical depth
    log-uniform in x1 from 1e4 (inner edge) to 1e-3 (outer edge), chi_es = 0.
    With perturb3d: rho0 x (1 + 0.04 (U - 1/2)) and each u~^i += 0.02
    sqrt(2/r) (2U - 1) in orthonormal-magnitude units.  kw: further
    parameters (e.g. ng=4, recon="ppm").  faces: also return the face field
    Bf [3][N] of the same potential (face_field_from_potential with A_3 at
    the corners, scaled alike) for a staggered-field grid."""
    if perturb3d is None:
        perturb3d = n[2] > 1
    p = disk_params(n=n, a=a, rin=rin, rout=rout, flux=flux, **kw)
    na = nalloc(p)
    N = ncell(p)
    x1, x2, x3 = cell_coords(p)
    r = np.exp(x1)
    th = math.pi * x2
    cells = np.arange(N, dtype=np.int64).reshape(x1.shape)
    rho = (r / rin) ** -1.5
    pg = 0.1 * rho / r
    if perturb3d:
        rho = rho * (1.0 + 0.04 * (uniform(seed, cells, 3) - 0.5))
    pg = pg * (1.0 + 0.02 * (uniform(seed, cells, 0) - 0.5))
    P = np.zeros((NPRIM,) + x1.shape)
    P[RHO] = rho
    P[UU] = pg / (p["gam"] - 1.0)
    vr = math.sqrt(2.0) * r ** -0.5
    P[U1] = -vr / r
    if perturb3d:
        P[U1] += 0.02 * vr * (2.0 * uniform(seed, cells, 4) - 1.0) / r
        P[U2] += 0.02 * vr * (2.0 * uniform(seed, cells, 5) - 1.0) / (math.pi * r)
        P[U3] += 0.02 * vr * (2.0 * uniform(seed, cells, 6) - 1.0) / (
            2.0 * math.pi * r * np.maximum(np.abs(np.sin(th)), 1e-3))
    # vector potential at cell corners (x1 face, x2 face), then B = curl A / sqrt(-g)
    g1 = p["ng"]
    g2 = p["ng"]
    dx1 = (p["xhi"][0] - p["xlo"][0]) / p["n"][0]
    dx2 = (p["xhi"][1] - p["xlo"][1]) / p["n"][1]
    xc1 = p["xlo"][0] + (np.arange(na[0] + 1) - g1) * dx1
    xc2 = p["xlo"][1] + (np.arange(na[1] + 1) - g2) * dx2
    X2c, X1c = np.meshgrid(xc2, xc1, indexing="ij")
    rc = np.exp(X1c)
    thc = math.pi * X2c
    rhoc = (rc / rin) ** -1.5
    Aphi = np.maximum(rhoc - 0.2, 0.0) * (rc * np.sin(thc)) ** 2
    # cell-centred curl from the four surrounding corners
    dA_dx2 = 0.5 * ((Aphi[1:, 1:] + Aphi[1:, :-1]) - (Aphi[:-1, 1:] + Aphi[:-1, :-1])) / dx2
    dA_dx1 = 0.5 * ((Aphi[1:, 1:] + Aphi[:-1, 1:]) - (Aphi[1:, :-1] + Aphi[:-1, :-1])) / dx1
    r2 = r[0]
    th2 = th[0]
    jac = r2 * math.pi * 2.0 * math.pi  # dr/dx1 * dth/dx2 * dph/dx3
    sg = _ks_sqrtg(a, r2, th2) * jac
    sg = np.maximum(sg, 1e-300)
    Bx1 = dA_dx2 / sg
    Bx2 = -dA_dx1 / sg
    # normalise: max gas pressure / max magnetic pressure ~ 100 (b^2/2 ~ rough B^2 g/2)
    bsq_est = (Bx1 * r2) ** 2 + (Bx2 * math.pi * np.sqrt(r2 ** 2 + a * a * np.cos(th2) ** 2)) ** 2
    pmax = float(np.max(pg))
    pbmax = float(np.max(0.5 * bsq_est))
    norm = math.sqrt(pmax / (100.0 * pbmax)) if pbmax > 0 else 0.0
    P[B1] = norm * Bx1[None, :, :]
    P[B2] = norm * Bx2[None, :, :]
    T = pg / rho
    P[ER] = p["arad"] * T ** 4
    P[F1] = P[U1]
    P[F2] = P[U2]
    P[F3] = P[U3]
    # opacity: per-cell optical depth tau = chi_abs rho0 * (r * dx1) (radial proper size ~ r dx1)
    frac = (x1 - p["xlo"][0]) / (p["xhi"][0] - p["xlo"][0])
    tau = 10.0 ** (4.0 - 7.0 * frac)
    chi_abs = tau / (rho * r * dx1)
    chi_es = np.zeros_like(chi_abs)
    out = (p, P.reshape(NPRIM, N), chi_abs.reshape(N), chi_es.reshape(N))
    if not faces:
        return out
    A = np.zeros((3,) + x1.shape)
    A[2] = norm * Aphi[None, :-1, :-1]
    return out + (face_field_from_potential(p, A),)


def face_field_from_potential(p: dict, A: np.ndarray) -> np.ndarray:
    """Face field Bf [3][N] (sqrt(-g) B^(d+1) on the lower d-face of each
    cell) as the discrete curl of an edge potential A [3][N] (A_e on the
    cell's edge along e, at its lower corner in the other two directions):
    Bf^p = d_q A_e - d_e A_q for cyclic (p, q, e), differences along
    inactive dimensions taken as zero.  Its discrete divergence vanishes up
    to rounding; the last layer along each axis (no upper neighbour) is left
    zero for the ghost fill."""
    na = nalloc(p)
    shape = (na[2], na[1], na[0])
    A = np.asarray(A, dtype=np.float64).reshape((3,) + shape)
    dx = [(p["xhi"][d] - p["xlo"][d]) / p["n"][d] for d in range(3)]
    ax = {0: 2, 1: 1, 2: 0}   # dimension -> numpy axis of [N3, N2, N1]

    def diff(f, d):
        out = np.zeros_like(f)
        if p["n"][d] == 1:
            return out
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[ax[d]] = slice(1, None)
        sl_lo[ax[d]] = slice(None, -1)
        out[tuple(sl_lo)] = (f[tuple(sl_hi)] - f[tuple(sl_lo)]) / dx[d]
        return out

    Bf = np.zeros((3,) + shape)
    for pp in range(3):
        q, e = (pp + 1) % 3, (pp + 2) % 3
        Bf[pp] = diff(A[e], q) - diff(A[q], e)
        # the outermost layer along any active axis lacks a neighbour
        for d in range(3):
            if p["n"][d] > 1:
                sl = [slice(None)] * 3
                sl[ax[d]] = slice(-1, None)
                Bf[pp][tuple(sl)] = 0.0
    return Bf.reshape(3, -1)


def implicit_batch(n: int, seed: int = 4, arad: float = 1.0, ugas_scale: float = 1.0):
    """Independent-cell batch for the implicit 4-force solve (Minkowski, B = 0).

    Per cell: rho0 log-uniform in [1e-6, 1]; T = p/rho0 log-uniform in
    [1e-4, 1e-1]; Ebar/(a_rad T^4) log-uniform in [1e-3, 1e3]; gas Lorentz
    factor uniform in [1, 5] with isotropic direction; the radiation frame
    moves relative to the gas with a 4-velocity of magnitude uniform in
    [0, 1.5] (Lorentz factor up to ~1.8, i.e. |F|/cE below ~0.9) in an
    isotropic direction, composed with the gas velocity by a Lorentz boost;
    dt kappa_tot log-uniform in [1e-3, 1e6] with kappa_abs = kappa_es; dt = 1.
    ugas_scale multiplies the gas 4-velocity u~ (before the radiation frame is
    composed with it): 0.14 keeps every gas flow below u~ = 0.7."""
    p = default_params(n=(n, 1, 1), arad=arad, tol_pmhd=1e-10)
    c = np.arange(n, dtype=np.int64)
    u = [uniform(seed, c, d) for d in range(12)]
    rho = 10.0 ** (-6.0 + 6.0 * u[0])
    T = 10.0 ** (-4.0 + 3.0 * u[1])
    ug = rho * T / (p["gam"] - 1.0)
    Ebar = arad * T ** 4 * 10.0 ** (-3.0 + 6.0 * u[2])
    gam = 1.0 + 4.0 * u[3]
    mu = 2.0 * u[4] - 1.0
    ph = 2.0 * math.pi * u[5]
    s = np.sqrt(1.0 - mu * mu)
    nhat = np.stack([s * np.cos(ph), s * np.sin(ph), mu])
    ugas = np.sqrt(gam * gam - 1.0) * nhat
    if ugas_scale != 1.0:
        ugas = ugas_scale * ugas
        gam = np.sqrt(1.0 + (ugas * ugas).sum(0))
    # radiation frame: relative 4-velocity w (in the gas frame), boosted to the lab
    wmag = 1.5 * u[6]
    mu2 = 2.0 * u[7] - 1.0
    ph2 = 2.0 * math.pi * u[8]
    s2 = np.sqrt(1.0 - mu2 * mu2)
    w = wmag * np.stack([s2 * np.cos(ph2), s2 * np.sin(ph2), mu2])
    w0 = np.sqrt(1.0 + (w * w).sum(0))
    # Lorentz boost of (w0, w) by gas 4-velocity (gam, ugas)
    udotw = (ugas * w).sum(0)
    urad = w + ugas * (w0 + udotw / (gam + 1.0))
    P = np.zeros((NPRIM, n))
    P[RHO] = rho
    P[UU] = ug
    P[U1:U3 + 1] = ugas
    P[ER] = Ebar
    P[F1:F3 + 1] = urad
    ktot = 10.0 ** (-3.0 + 9.0 * u[9])
    chi_abs = 0.5 * ktot / rho
    chi_es = 0.5 * ktot / rho
    dt = np.ones(n)
    return p, P, dt, chi_abs, chi_es


def random_states(n: int, seed: int, gmax: float = 50.0, bsq_rho_max: float = 1e3,
                  with_field: bool = True):
    """Random primitive states for pointwise round-trip checks (Minkowski or
    any metric): rho0 log-uniform [1e-4, 1], u/rho log-uniform [1e-8, 1e4],
    gas Lorentz factor log-uniform [1, gmax], B components with |B|^2/rho
    log-uniform [1e-6, bsq_rho_max], Ebar/u log-uniform [1e-12, 1e6],
    radiation Lorentz factor log-uniform [1, 20]."""
    c = np.arange(n, dtype=np.int64)
    u = [uniform(seed, c, d) for d in range(14)]
    rho = 10.0 ** (-4.0 + 4.0 * u[0])
    ug = rho * 10.0 ** (-8.0 + 12.0 * u[1])
    gam = 10.0 ** (math.log10(gmax) * u[2])
    def direction(a, b):
        mu = 2.0 * a - 1.0
        ph = 2.0 * math.pi * b
        s = np.sqrt(1.0 - mu * mu)
        return np.stack([s * np.cos(ph), s * np.sin(ph), mu])
    ugas = np.sqrt(gam * gam - 1.0) * direction(u[3], u[4])
    P = np.zeros((NPRIM, n))
    P[RHO] = rho
    P[UU] = ug
    P[U1:U3 + 1] = ugas
    if with_field:
        bmag = np.sqrt(rho * 10.0 ** (-6.0 + (6.0 + math.log10(bsq_rho_max)) * u[5]))
        P[B1:B3 + 1] = bmag * direction(u[6], u[7])
    P[ER] = ug * 10.0 ** (-12.0 + 18.0 * u[8])
    grad = 10.0 ** (math.log10(20.0) * u[9])
    P[F1:F3 + 1] = np.sqrt(grad * grad - 1.0) * direction(u[10], u[11])
    return P


def jitter(P, seed: int, rel: float = 1e-3):
    """A copy of P with seeded relative noise on every primitive, absolute
    noise of rel x max|B| on the field and rel on the radiation velocity:
    removes the exact ties (equal neighbours, zero field or flux) at which
    the limiters and wave-speed extrema are not differentiable, for
    finite-difference checks of derivatives."""
    c = np.arange(P.shape[1], dtype=np.int64)
    z = np.stack([np.sqrt(-2.0 * np.log(uniform(seed, c, 2 * q) + 1e-300)) *
                  np.cos(2.0 * math.pi * uniform(seed, c, 2 * q + 1)) for q in range(12)])
    out = P * (1.0 + rel * z)
    sc = np.abs(P[B1:B3 + 1]).max() + rel
    zb = np.stack([np.sqrt(-2.0 * np.log(uniform(seed + 1, c, 2 * q) + 1e-300)) *
                   np.cos(2.0 * math.pi * uniform(seed + 1, c, 2 * q + 1)) for q in range(6)])
    out[B1:B3 + 1] += rel * sc * zb[:3]
    out[F1:F3 + 1] += rel * zb[3:]
    return out
