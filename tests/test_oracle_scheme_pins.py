"""Pins of the oracle's discretisation: wave speeds, Courant step, ghost
fills, MC reconstruction, the Riemann fluxes' dissipation, and whole runs of
the scheme against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
- closed-form characteristic speeds (relativistic velocity addition, the
  oblique-flow sound speeds of relativistic hydrodynamics, the exact
  eigenvalues of the linearised gas and M1 systems);
- exact solutions of linear Riemann problems (an isolated acoustic wave, the
  M1 system at rest), which an upwind flux reproduces exactly;
- symmetry (a reflecting boundary against the mirrored domain; uniform
  Cartesian vectors across the polar axis);
- the variational characterisation of the MC slope and the monotonicity of
  a shock-tube profile;
- the paper's linear-wave table (Sec. 5.1: damping after one period, L1
  error converging at second order when thin and first order when thick and
  radiation-dominated) and the diffusion solution of Sec. 5.4 (eq. diffsol,
  D = 1/(3 kappa_tot)).
"""
import math
import os

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
SQ3 = math.sqrt(3.0)


def _prim(rho, u, v=(0.0, 0.0, 0.0), B=(0.0, 0.0, 0.0), E=0.0, vr=None):
    """Minkowski primitives from a 3-velocity v (gas) and vr (radiation frame;
    default comoving): u~^i = gamma v^i in flat space."""
    P = np.zeros(12)
    P[0], P[1], P[8] = rho, u, E
    v = np.asarray(v, float)
    P[2:5] = v / math.sqrt(1.0 - v @ v)
    P[5:8] = B
    vr = v if vr is None else np.asarray(vr, float)
    P[9:12] = vr / math.sqrt(1.0 - vr @ vr)
    return P


def _sound_speeds(v, c2, d=0):
    """Characteristic speeds along axis d of a wave moving at sqrt(c2) in a
    frame with 3-velocity v (relativistic hydrodynamics, oblique flow)."""
    v = np.asarray(v, float)
    v2, vx = v @ v, v[d]
    c = math.sqrt(c2)
    root = c * math.sqrt((1.0 - v2) * (1.0 - vx * vx - (v2 - vx * vx) * c2))
    den = 1.0 - v2 * c2
    return (vx * (1.0 - c2) - root) / den, (vx * (1.0 - c2) + root) / den


def _cs2(gam, rho, u):
    p = (gam - 1.0) * u
    return gam * p / (rho + u + p)


# ---------------------------------------------------------------------------
# characteristic speeds (Sec. 4.4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("v", [(0.0, 0.0, 0.0), (0.6, 0.0, 0.0), (-0.3, 0.5, 0.2), (0.1, -0.7, 0.6)])
def test_gas_sound_speeds_are_relativistic_addition(orc, v):
    """B = 0: the gas speeds are those of a sound wave c_s^2 = Gamma p / (rho0 +
    u + p) carried by the flow, in every direction."""
    pd = I.default_params(arad=1.0)
    g = orc.geom(pd, 0.0, 0.0)
    rho, u = 1.3, 0.7
    P = _prim(rho, u, v=v, E=0.2)
    c2 = _cs2(pd["gam"], rho, u)
    for d in range(3):
        vg, vr = orc.wavespeeds(pd, g, P, d + 1, 0.0)
        lm, lp = _sound_speeds(v, c2, d)
        assert abs(vg[0] - lm) < 1e-14 and abs(vg[1] - lp) < 1e-14, (d, vg, lm, lp)
        # comoving radiation: the same addition with c^2 = 1/3
        rm, rp = _sound_speeds(v, 1.0 / 3.0, d)
        assert abs(vr[0] - rm) < 1e-14 and abs(vr[1] - rp) < 1e-14, (d, vr, rm, rp)


def test_radiation_speeds_at_rest_and_in_the_beam_limit(orc):
    """Radiation frame at rest: +-1/sqrt(3) (the M1 speeds at zero flux);
    a radiation frame boosted to Lorentz factor G along x: both speeds tend to
    c = 1 as G grows, and transverse speeds to 0."""
    pd = I.default_params(gamma_max=1e4)
    g = orc.geom(pd, 0.0, 0.0)
    P = _prim(1.0, 0.1, E=1.0)
    vg, vr = orc.wavespeeds(pd, g, P, 1, 0.0)
    assert abs(vr[0] + 1 / SQ3) < 1e-15 and abs(vr[1] - 1 / SQ3) < 1e-15
    prev = 0.0
    for G in (2.0, 10.0, 100.0, 1000.0):
        vb = math.sqrt(1 - 1 / G ** 2)
        P = _prim(1.0, 0.1, E=1.0, vr=(vb, 0.0, 0.0))
        _, vr = orc.wavespeeds(pd, g, P, 1, 0.0)
        lm, lp = _sound_speeds((vb, 0.0, 0.0), 1.0 / 3.0)
        assert abs(vr[0] - lm) < 1e-13 and abs(vr[1] - lp) < 1e-13
        assert prev < vr[0] < vr[1] <= 1.0
        prev = vr[0]
        _, vt = orc.wavespeeds(pd, g, P, 2, 0.0)
        tm, tp = _sound_speeds((vb, 0.0, 0.0), 1.0 / 3.0, 1)
        assert abs(vt[0] - tm) < 1e-13 and abs(vt[1] - tp) < 1e-13
        assert abs(vt[0] + vt[1]) < 1e-13 and vt[1] < 1.0 / G
    assert 1.0 - prev < 1e-5


@pytest.mark.parametrize("vx", [0.0, 0.4, -0.25])
def test_thick_radiation_speed_limiter(orc, vx):
    """eq. wavespeedlimit: with optical depth tau = kappa_tot sqrt(g_dd) dx above
    4/3 the radiation speeds are those of a wave at 4/(3 tau) in the gas frame
    (relativistic addition with the gas velocity), unless the M1 speeds are
    already slower; tau <= 4/3 leaves them unlimited."""
    pd = I.default_params()
    g = orc.geom(pd, 0.0, 0.0)
    P = _prim(1.0, 0.1, v=(vx, 0.1, 0.0), E=0.5)
    _, free = orc.wavespeeds(pd, g, P, 1, 0.0)
    _, same = orc.wavespeeds(pd, g, P, 1, 1.2)
    assert np.array_equal(free, same)
    for tau in (2.0, 10.0, 1e3, 1e6):
        _, vr = orc.wavespeeds(pd, g, P, 1, tau)
        lm, lp = _sound_speeds((vx, 0.1, 0.0), (4.0 / (3.0 * tau)) ** 2)
        assert abs(vr[0] - max(lm, free[0])) < 1e-14 * max(1.0, abs(lm))
        assert abs(vr[1] - min(lp, free[1])) < 1e-14 * max(1.0, abs(lp))
    # deep in the thick limit the radiation moves with the gas
    _, vr = orc.wavespeeds(pd, g, P, 1, 1e12)
    vgas = P[2] / math.sqrt(1 + P[2:5] @ P[2:5])
    assert abs(vr[0] - vgas) < 1e-11 and abs(vr[1] - vgas) < 1e-11


def _block_eigs(orc, pd, g, P0, rows):
    """Eigenvalues of A^-1 B restricted to `rows` (A = dU/dP, B = dF^x/dP by
    fourth-order differences)."""

    def jac(f):
        J = np.zeros((12, 12))
        for j in range(12):
            h = 1e-4 * max(abs(P0[j]), 1e-2)
            e = np.eye(12)[j] * h
            fs = [f(P0 + m * e) for m in (-2, -1, 1, 2)]
            J[:, j] = (fs[0] - 8 * fs[1] + 8 * fs[2] - fs[3]) / (12 * h)
        return J

    A = jac(lambda P: orc.p2u(pd, g, P))[np.ix_(rows, rows)]
    B = jac(lambda P: orc.flux(pd, g, P, 1))[np.ix_(rows, rows)]
    return np.linalg.eigvals(np.linalg.solve(A, B))


@pytest.mark.parametrize("angle", [90.0, 60.0, 30.0, 0.0])
def test_fast_speed_bounds_linearised_eigenvalues(orc, angle):
    """At rest with field at `angle` to x, the exact characteristic speeds of
    the linearised equations (eigenvalues of A^-1 B) stay within the gas speed
    v_A^2 + c_s^2 (1 - v_A^2) that the fluxes use (equal for a field normal to
    x, where it is the exact fast speed), and the M1 block's eigenvalues are
    the radiation speeds +-1/sqrt(3)."""
    pd = I.default_params()
    g = orc.geom(pd, 0.0, 0.0)
    th = math.radians(angle)
    P0 = _prim(1.0, 0.4, B=(0.8 * math.cos(th), 0.8 * math.sin(th), 0.0), E=0.3)
    gas = _block_eigs(orc, pd, g, P0, [0, 1, 2, 3, 4, 5, 6, 7])
    rad = _block_eigs(orc, pd, g, P0, [8, 9, 10, 11])
    assert np.abs(gas.imag).max() < 1e-8 and np.abs(rad.imag).max() < 1e-8
    vg, vr = orc.wavespeeds(pd, g, P0, 1, 0.0)
    assert abs(vg[0] + vg[1]) < 1e-15
    lam = np.abs(gas.real).max()
    assert lam <= vg[1] * (1 + 1e-9), (lam, vg)
    if angle == 90.0:
        assert abs(lam - vg[1]) < 1e-9, (lam, vg)
    r = np.sort(rad.real)
    assert np.abs(r[[0, -1]] - np.array([-1, 1]) / SQ3).max() < 1e-9, r
    assert abs(vr[1] - 1 / SQ3) < 1e-15


# ---------------------------------------------------------------------------
# Courant step (Sec. 4.4, last paragraph)
# ---------------------------------------------------------------------------

def test_courant_step_of_a_uniform_flow(orc):
    """Uniform hot flow on a periodic 2-D box: dt = C / sum_d(v_d / dx^d), v_d
    the largest closed-form characteristic speed magnitude along d (the gas
    here, faster than the comoving radiation)."""
    n = (8, 6, 1)
    pd = I.default_params(n=n, courant=0.4, xhi=(1.0, 2.0, 1.0))
    N = I.ncell(pd)
    v = (0.3, -0.2, 0.1)
    Pc = _prim(1.0, 2.0, v=v, E=0.5)
    P = np.tile(Pc[:, None], (1, N))
    F, emf, vch = orc.fluxes(pd, P, np.zeros(N), np.zeros(N))
    dt = orc.timestep(pd, vch)
    c2 = _cs2(pd["gam"], 1.0, 2.0)
    assert c2 > 1.0 / 3.0
    inv = 0.0
    for d in range(2):
        lm, lp = _sound_speeds(v, c2, d)
        inv += max(abs(lm), abs(lp)) / ((pd["xhi"][d] - pd["xlo"][d]) / n[d])
    assert abs(dt - pd["courant"] / inv) < 1e-14 * dt, (dt, pd["courant"] / inv)
    # hand-computed cells: one fast x face and one fast y face elsewhere; each
    # cell takes the larger speed of its two faces per direction, so the
    # binding cells are the two sharing a fast face
    na = I.nalloc(pd)
    vch = np.full((3, na[1], na[0]), 1e-3)
    g = pd["ng"]
    dx1, dx2 = 1.0 / n[0], 2.0 / n[1]
    vch[0, g + 2, g + 4] = 0.9      # x face between cells (3, 2) and (4, 2)
    vch[1, g + 3, g + 6] = 0.8      # y face between cells (6, 2) and (6, 3)
    dt = orc.timestep(pd, vch.reshape(3, -1))
    want = pd["courant"] / max(0.9 / dx1 + 1e-3 / dx2, 1e-3 / dx1 + 0.8 / dx2)
    assert abs(dt - want) < 1e-15 * want, (dt, want)


# ---------------------------------------------------------------------------
# ghost fill (Sec. 4.2 step 1)
# ---------------------------------------------------------------------------

def _mirror_state(x, d, seed):
    """Smooth primitives along one axis (coordinate x) with a flow and field."""
    P = np.zeros((12, x.size))
    P[0] = 1.0 + 0.4 * np.exp(-((x - 0.3) / 0.2) ** 2) + 0.02 * I.uniform(seed, np.arange(x.size), 0)
    P[1] = 0.3 + 0.1 * np.cos(3 * x)
    P[2 + d] = -0.4 * np.sin(2.5 * x)                 # normal velocity towards the wall
    P[2 + (d + 1) % 3] = 0.2 * np.cos(x)
    P[5 + d] = 0.15 + 0.05 * x                        # normal field (odd under the mirror)
    P[5 + (d + 1) % 3] = 0.1 * np.sin(4 * x)
    P[8] = 0.5 + 0.3 * np.exp(-((x - 0.6) / 0.15) ** 2)
    P[9 + d] = P[2 + d] + 0.05 * np.sin(x)
    P[9 + (d + 1) % 3] = P[2 + (d + 1) % 3]
    return P


@pytest.mark.parametrize("d", [0, 1])
def test_reflecting_wall_equals_mirrored_domain(orc, d):
    """A reflecting boundary at x = 0 gives the same solution on (0, 1) as the
    domain (-1, 1) started from the mirror image (normal vector components
    negated), stepped alike; the mirrored domain stays mirror-symmetric."""
    n = 24
    nn = [1, 1, 1]
    nn[d] = n
    kw = dict(flux="hll", courant=0.4, arad=0.7)
    bl, bh = ["periodic"] * 3, ["periodic"] * 3
    bl[d], bh[d] = "reflect", "outflow"
    pa = I.default_params(n=tuple(nn), bc_lo=tuple(bl), bc_hi=tuple(bh), **kw)
    nn2 = list(nn)
    nn2[d] = 2 * n
    lo, hi = [0.0] * 3, [1.0] * 3
    lo[d] = -1.0
    bl[d] = "outflow"
    pb = I.default_params(n=tuple(nn2), xlo=tuple(lo), xhi=tuple(hi), bc_lo=tuple(bl),
                          bc_hi=tuple(bh), **kw)
    xa = I.cell_coords(pa)[d].reshape(-1)
    xb = I.cell_coords(pb)[d].reshape(-1)
    Pa = _mirror_state(np.abs(xa), d, 5)
    Pb = _mirror_state(np.abs(xb), d, 5)
    odd = [2 + d, 5 + d, 9 + d]
    Pb[odd] *= np.where(xb < 0, -1.0, 1.0)
    # the same cells' noise on both grids
    ia = np.round(np.abs(xa) * n - 0.5).astype(int)
    ib = np.round(np.abs(xb) * n - 0.5).astype(int)
    Pa[0] = 1.0 + 0.4 * np.exp(-((np.abs(xa) - 0.3) / 0.2) ** 2) + 0.02 * I.uniform(5, ia, 0)
    Pb[0] = 1.0 + 0.4 * np.exp(-((np.abs(xb) - 0.3) / 0.2) ** 2) + 0.02 * I.uniform(5, ib, 0)
    Na, Nb = I.ncell(pa), I.ncell(pb)
    ca, cb = np.full(Na, 0.8), np.full(Nb, 0.8)
    ea, eb = np.full(Na, 0.3), np.full(Nb, 0.3)
    Ua, Ub = orc.prim_to_cons(pa, Pa), orc.prim_to_cons(pb, Pb)
    dt = 0.004
    for _ in range(6):
        Pa, Ua, _, sa, _, na_ = orc.step(pa, Pa, Ua, ca, ea, dt=dt, dt_fixed=True)
        Pb, Ub, _, sb, _, nb_ = orc.step(pb, Pb, Ub, cb, eb, dt=dt, dt_fixed=True)
        assert na_ == 0 and nb_ == 0
    g = pa["ng"]
    A = Pa[:, g:g + n]
    Bpos = Pb[:, g + n:g + 2 * n]
    Bneg = Pb[:, g:g + n][:, ::-1].copy()
    Bneg[odd] *= -1.0
    scale = np.abs(A).max(axis=1, keepdims=True) + 1e-300
    assert (np.abs(A - Bpos) / scale).max() < 1e-13
    assert (np.abs(Bneg - Bpos) / scale).max() < 1e-13


def _ks_cart_components(pd, x1, x2, x3, V):
    """Internal-coordinate components (x1, x2, x3) of a uniform vector V given
    in the Kerr-Schild Cartesian frame x + i y = (r + i a) sin(th) e^{i phi},
    z = r cos(th), at internal coordinates with r = R0 + e^{x1},
    th = pi x2, phi = 2 pi x3."""
    a = pd["a"]
    r = pd["R0"] + math.exp(x1)
    th, ph = math.pi * x2, 2 * math.pi * x3
    st, ct, sp, cp = math.sin(th), math.cos(th), math.sin(ph), math.cos(ph)
    J = np.array([
        [st * cp, (r * cp - a * sp) * ct, -(r * sp + a * cp) * st],
        [st * sp, (r * sp + a * cp) * ct, (r * cp - a * sp) * st],
        [ct, -r * st, 0.0]])
    w = np.linalg.solve(J, V)          # (r, theta, phi) components
    return w / np.array([r - pd["R0"], math.pi, 2 * math.pi])


def test_polar_axis_continues_uniform_cartesian_vectors(orc):
    """POLAR boundary (3-D Kerr-Schild): the ghost cells beyond the axis (at
    -theta or 2 pi - theta, same phi) hold exactly what a uniform Cartesian
    velocity and field would have there, when the interior holds it: the
    ghost takes the cell at the same distance from the axis and phi + pi with
    the theta components negated, which is the coordinate continuation of a
    smooth vector field through the axis."""
    pd = I.disk_params(n=(4, 6, 8))
    N = I.ncell(pd)
    x1, x2, x3 = (c.reshape(-1) for c in I.cell_coords(pd))
    Vu = np.array([0.1, -0.2, 0.3])   # gas velocity
    Vb = np.array([0.0, 0.05, 0.4])   # field
    Vr = np.array([-0.3, 0.1, 0.05])  # radiation frame velocity
    P = np.zeros((12, N))
    P[0], P[1], P[8] = 1.0, 0.1, 0.2
    for c in range(N):
        P[2:5, c] = _ks_cart_components(pd, x1[c], x2[c], x3[c], Vu)
        P[5:8, c] = _ks_cart_components(pd, x1[c], x2[c], x3[c], Vb)
        P[9:12, c] = _ks_cart_components(pd, x1[c], x2[c], x3[c], Vr)
    na = I.nalloc(pd)
    g = pd["ng"]
    j = np.arange(N) // na[0] % na[1]
    i = np.arange(N) % na[0]
    k = np.arange(N) // (na[0] * na[1])
    inner = (j >= g) & (j < g + pd["n"][1]) & (i >= g) & (i < g + pd["n"][0]) & \
        (k >= g) & (k < g + pd["n"][2])
    Pin = np.where(inner, P, 0.0)
    out = orc.bc(pd, Pin)
    axis_ghost = ((j < g) | (j >= g + pd["n"][1])) & (i >= g) & (i < g + pd["n"][0])
    assert axis_ghost.sum() == 2 * g * pd["n"][0] * na[2]
    for q in list(range(2, 8)) + [9, 10, 11]:
        grp = slice(2, 5) if q < 5 else (slice(5, 8) if q < 8 else slice(9, 12))
        sc = np.abs(P[grp][:, axis_ghost]).max()
        err = np.abs(out[q, axis_ghost] - P[q, axis_ghost]).max() / sc
        assert err < 1e-12, (q, err)


# ---------------------------------------------------------------------------
# MC reconstruction (Sec. 4.3)
# ---------------------------------------------------------------------------

def test_mc_reconstruction_properties(orc):
    """The MC slope: exact on linear data, zero at an extremum, and on
    monotone data the steepest slope that is no steeper than the central
    difference and keeps both of the cell's face values between its
    neighbours' values (so it is either the central difference or puts a face
    value exactly on a neighbour's); the face values of every cell then stay
    within the range of the cell and its neighbours (no new extrema)."""
    for a, b in ((0.0, 1.0), (3.5, -0.25)):
        l, r = orc.mc_face([a + b * m for m in range(4)])
        assert abs(l - (a + 1.5 * b)) < 1e-15 and abs(r - (a + 1.5 * b)) < 1e-15
    assert orc.mc_face([0.0, 1.0, 0.5, 0.7])[0] == 1.0       # maximum: flat
    assert orc.mc_face([2.0, 1.0, 3.0, 3.5])[0] == 1.0       # minimum: flat
    rng = np.random.default_rng(3)
    n_touch = n_central = 0
    for _ in range(4000):
        a = np.cumsum(rng.exponential(1.0, 4) ** 3) * rng.choice([-1.0, 1.0])
        l, r = orc.mc_face(a)
        s = 2.0 * (l - a[1])                   # slope of cell 1
        lo_face = a[1] - 0.5 * s
        lo, hi = sorted((a[0], a[2]))
        assert lo - 1e-12 <= lo_face <= hi + 1e-12 and lo - 1e-12 <= l <= hi + 1e-12
        assert abs(s) <= 0.5 * abs(a[2] - a[0]) + 1e-14 * abs(a).max()
        # s is recovered from a face value, so it carries the rounding of |a|
        tol = 1e-14 * abs(a).max() + 1e-12 * abs(a[2] - a[0])
        central = abs(abs(s) - 0.5 * abs(a[2] - a[0])) < tol
        touch = min(abs(lo_face - a[0]), abs(l - a[2])) < tol
        assert central or touch
        n_touch += touch and not central
        n_central += central
        # right state: cell 2's left value, inside the range of cells 1..3
        assert min(a[1], a[3]) - 1e-12 <= r <= max(a[1], a[3]) + 1e-12
    assert n_touch > 500 and n_central > 500


def test_shock_tube_profile_stays_monotone(orc):
    """The radiative shock tube's density falls monotonically from left to
    right through rarefaction, contact and shock; the MC-limited scheme keeps
    it so (no new extrema, no overshoot of either state), up to the 1e-11
    compression the thin radiation's precursor makes ahead of the waves."""
    pd, P, ca, ce = I.shock_tube_1d(200)
    U = orc.prim_to_cons(pd, P)
    t = 0.0
    while t < 0.4:
        P, U, dt, st, it, nbad = orc.step(pd, P, U, ca, ce)
        assert nbad == 0
        t += dt
    rho = P[0, 2:-2]
    assert rho.max() <= 1.0 + 1e-10 and rho.min() >= 0.125 - 1e-10
    assert np.all(np.diff(rho) <= 1e-10), np.diff(rho).max()
    # the waves have moved: a rarefaction fan, a contact and a shock
    assert (rho < 0.99).sum() > 103 and (rho > 0.13).sum() > 104


# ---------------------------------------------------------------------------
# Riemann fluxes (eq. hll, eq. lax) against exact linear Riemann solutions
# ---------------------------------------------------------------------------

def _jump_fluxes(orc, pd, PL, PR, n=12):
    """Face fluxes of a 1-D grid whose left half holds PL and right half PR;
    returns the flux at the face between the halves."""
    N = I.ncell(pd)
    g = pd["ng"]
    P = np.where(np.arange(N) < g + n // 2, PL[:, None], PR[:, None])
    F, emf, vch = orc.fluxes(pd, P, np.zeros(N), np.zeros(N))
    return F[0][:, g + n // 2]


@pytest.mark.parametrize("flux", ["hll", "llf"])
@pytest.mark.parametrize("direction", [1, -1])
def test_riemann_flux_upwinds_an_acoustic_wave(orc, flux, direction):
    """Gas at rest (no field, uniform radiation) on the left and the state
    across an isolated sound wave moving right (left) of amplitude 1e-7: the
    exact Riemann solution at the face is the left (right) state, and both
    HLL and LAXF with the sound speeds give its flux to second order in the
    amplitude (their dissipation is exactly the upwinding of a wave at the
    sound speed)."""
    pd = I.default_params(n=(12, 1, 1), bc_lo=("outflow",) * 3, bc_hi=("outflow",) * 3, flux=flux)
    gam = pd["gam"]
    rho, u = 1.0, 0.05
    p = (gam - 1) * u
    c = math.sqrt(_cs2(gam, rho, u))
    dv = 1e-7
    # a wave f(x - s t), s = direction c: rho dv = s drho, (e + p) dv = s de, dp = s (e + p) dv
    s = direction * c
    drho = rho * dv / s
    du = (u + p) * dv / s
    PL = _prim(rho, u, E=1e-3)
    PR = _prim(rho + drho, u + du, v=(dv, 0.0, 0.0), E=1e-3)
    PR[9:12] = 0.0
    Fnum = _jump_fluxes(orc, pd, PL, PR)
    g = orc.geom(pd, 0.0, 0.0)
    FL, FR = orc.flux(pd, g, PL, 1), orc.flux(pd, g, PR, 1)
    Fex = FL if direction > 0 else FR
    jump = np.abs(FR - FL)[:5]
    assert np.all(jump[[0, 1, 2]] > 1e-9)
    assert np.all(np.abs(Fnum[:5] - Fex[:5]) <= 1e-5 * jump + 1e-15 * np.abs(FL[:5])), \
        (Fnum[:5] - Fex[:5]) / (jump + 1e-300)
    # the radiation is uniform: its flux is the common flux
    assert np.abs(Fnum[8:] - FL[8:]).max() < 1e-16


@pytest.mark.parametrize("flux", ["hll", "llf"])
def test_riemann_flux_of_radiation_at_rest_is_exact(orc, flux):
    """M1 radiation at rest with zero flux on both sides and energies E_L, E_R:
    the system is linear with speeds +-1/sqrt(3) (P = E/3), so the exact
    Godunov flux at the face is (-(E_L - E_R)/(2 sqrt 3), (E_L + E_R)/6) in the
    energy and x-momentum rows, which both solvers must give exactly."""
    pd = I.default_params(n=(12, 1, 1), bc_lo=("outflow",) * 3, bc_hi=("outflow",) * 3, flux=flux)
    EL, ER = 0.7, 0.2
    PL = _prim(1.0, 0.1, E=EL)
    PR = _prim(1.0, 0.1, E=ER)
    F = _jump_fluxes(orc, pd, PL, PR)
    assert abs(F[8] - (-(EL - ER) / (2 * SQ3))) < 1e-15
    assert abs(F[9] - (EL + ER) / 6.0) < 1e-15
    assert F[10] == 0.0 and F[11] == 0.0


def test_hll_is_upwind_for_supersonic_flow(orc):
    """All waves moving right (gas and radiation frames at 0.95 c, cold gas):
    HLL returns the left state's flux; all moving left: the right state's."""
    pd = I.default_params(n=(12, 1, 1), bc_lo=("outflow",) * 3, bc_hi=("outflow",) * 3, flux="hll")
    g = orc.geom(pd, 0.0, 0.0)
    for sgn in (1.0, -1.0):
        PL = _prim(1.0, 0.01, v=(sgn * 0.95, 0.1, 0.0), B=(0.05, 0.02, 0.0), E=0.01)
        PR = _prim(0.6, 0.004, v=(sgn * 0.93, -0.05, 0.02), B=(0.05, -0.01, 0.01), E=0.02)
        for P in (PL, PR):
            vg, vr = orc.wavespeeds(pd, g, P, 1, 0.0)
            assert sgn * vg[0 if sgn > 0 else 1] > 0 and sgn * vr[0 if sgn > 0 else 1] > 0
        F = _jump_fluxes(orc, pd, PL, PR)
        Fup = orc.flux(pd, g, PL if sgn > 0 else PR, 1)
        Fup[5] = 0.0
        assert np.all(np.abs(F - Fup) <= 1e-14 * (np.abs(Fup) + 1e-300)), F - Fup


# ---------------------------------------------------------------------------
# linear waves of Sec. 5.1 run through the scheme
# ---------------------------------------------------------------------------

def _load_waves():
    rows = {}
    with open(os.path.join(HERE, "golden", "linear_waves.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            panel, tau, Pr, mode, q, re_, im = line.split()
            r = rows.setdefault((panel, mode), {"tau": float(tau), "Pr": float(Pr)})
            r[q] = complex(float(re_), float(im))
    return rows


WAVES = _load_waves()


def _wave_run(orc, panel, mode, n):
    """One period of the tabulated eigenmode on a periodic box of n cells
    (LAXF, MC, RK3, Courant 0.5, dt fixed so the run ends at the period).
    Opacity reading as in the eigenmode pin: kappa_abs = tau, kappa_es = 0,
    a_rad = Ebar/T^4.  Returns (L1 of rho0 against the analytic solution,
    amplitude ratio of the k-mode, e^{-Im omega P}, phase error)."""
    ref = WAVES[(panel, mode)]
    gam, eg, B0 = 5.0 / 3.0, 0.009137055837563452, 0.10075854437197568
    T = (gam - 1.0) * eg
    E = 3.0 * ref["Pr"] * (gam - 1.0) * eg
    pd = I.default_params(n=(n, 1, 1), gam=gam, arad=E / T ** 4, flux="llf", courant=0.5)
    N = I.ncell(pd)
    x = I.cell_coords(pd)[0].reshape(-1)
    k = 2 * math.pi
    ph = np.exp(-1j * k * x)

    def q(name):
        return (ref[name] * ph).real

    P = np.zeros((12, N))
    P[0], P[1], P[2], P[3] = 1 + q("drho"), eg + q("du"), q("dux"), q("duy")
    if mode != "sound":
        P[5], P[6] = B0, B0 + q("dBy")
    P[8] = E + q("dE")
    # fluid-frame flux to first order: F^ = (4/3) Ebar (u~_rad - u~_gas)
    P[9] = P[2] + 0.75 / E * q("dFx")
    P[10] = P[3] + 0.75 / E * q("dFy")
    ca, ce = np.full(N, ref["tau"]), np.zeros(N)
    U = orc.prim_to_cons(pd, P)
    w = ref["omega"]
    per = 2 * math.pi / w.real
    dt0 = orc.step(pd, P, U, ca, ce)[2]
    ns = int(math.ceil(per / dt0))
    for _ in range(ns):
        P, U, _, st, it, nbad = orc.step(pd, P, U, ca, ce, dt=per / ns, dt_fixed=True)
        assert nbad == 0
    sl = slice(2, 2 + n)
    exact = 1 + (ref["drho"] * np.exp(1j * (w * per - k * x))).real
    L1 = np.abs(P[0, sl] - exact[sl]).mean()
    amp = (P[0, sl] - 1) @ np.exp(1j * k * x[sl]) * 2 / n
    return L1, abs(amp) / abs(ref["drho"]), math.exp(-w.imag * per), abs(np.angle(amp / ref["drho"]))


THIN = [("a", "sound"), ("a", "fast"), ("a", "slow"), ("c", "sound")]
THICK = [("d", "sound"), ("d", "fast")]


@pytest.mark.parametrize("case", THIN, ids=lambda c: "-".join(c))
def test_linear_wave_converges_at_second_order_when_thin(orc, case):
    """Optically thin (tau = 0.1): the L1 error of eq. 1 falls at second order,
    and the wave's amplitude after one period tends to e^{-Im omega P} with the
    phase error falling too (Sec. 5.1)."""
    res = {n: _wave_run(orc, *case, n) for n in (16, 32, 64)}
    order = math.log2(res[32][0] / res[64][0])
    assert order > 1.7, (case, order)
    ex = res[64][2]
    e32, e64 = abs(res[32][1] - ex), abs(res[64][1] - ex)
    assert e64 < 3e-3 * ex and e64 < 0.4 * e32, (res[32][1], res[64][1], ex)
    assert res[64][3] < 0.5 * res[32][3] and res[64][3] < 5e-3


@pytest.mark.parametrize("case", THICK, ids=lambda c: "-".join(c))
def test_linear_wave_converges_at_first_order_when_thick(orc, case):
    """Optically thick and radiation-dominated (tau = 10, P = 10): the implicit
    coupling, first order in dt, sets the L1 error's order to one (Sec. 5.1,
    panel (d)); the damping still tends to e^{-Im omega P}."""
    res = {n: _wave_run(orc, *case, n) for n in (32, 64, 128)}
    o1 = math.log2(res[32][0] / res[64][0])
    o2 = math.log2(res[64][0] / res[128][0])
    assert 0.9 < o2 < 1.5 and o2 < o1, (case, o1, o2)
    ex = res[128][2]
    assert abs(res[128][1] - ex) < 3e-3 * ex and abs(res[128][1] - ex) < abs(res[32][1] - ex)


# ---------------------------------------------------------------------------
# optically thick diffusion (Sec. 5.4, eq. diffsol)
# ---------------------------------------------------------------------------

def _pulse(orc, n, width=8.0, kes=1e3):
    """Planar radiation pulse in a cold, gas-dominated, purely scattering
    medium (rho0 = 1, kappa_es = kes per unit length, kappa_abs = 0) on
    x in [-50, 50] with n cells: -R^t_t = E0 (1e-3 + exp(-x^2 / (4 D t0))),
    t0 = width^2 / (4 D), D = 1/(3 kappa_tot), run to t = t0.  Returns the
    largest deviation from eq. diffsol (n = 1) over the profile, in units of
    the initial peak, and the peak ratio."""
    pd = I.default_params(n=(n, 1, 1), xlo=(-50.0, 0.0, 0.0), xhi=(50.0, 1.0, 1.0), arad=1.0,
                          flux="llf", courant=0.5)
    N = I.ncell(pd)
    x = I.cell_coords(pd)[0].reshape(-1)
    D = 1.0 / (3.0 * kes)
    t0 = width ** 2 / (4 * D)
    E0, bg = 1e-10, 1e-3
    P = np.zeros((12, N))
    P[0], P[1] = 1.0, 1e-8
    P[8] = E0 * (bg + np.exp(-x ** 2 / (4 * D * t0)))
    ca, ce = np.zeros(N), np.full(N, kes)
    U = orc.prim_to_cons(pd, P)
    t = 0.0
    while t < t0 * (1 - 1e-12):
        dt = min(orc.step(pd, P, U, ca, ce)[2], t0 - t)
        P, U, _, st, it, nbad = orc.step(pd, P, U, ca, ce, dt=dt, dt_fixed=True)
        assert nbad == 0
        t += dt
    sl = slice(2, 2 + n)
    ana = E0 * (bg + np.exp(-x[sl] ** 2 / (4 * D * (t + t0))) * ((t + t0) / t0) ** -0.5)
    prof = -U[8, sl]
    return np.abs(prof - ana).max() / E0, (prof.max() / E0 - bg) / ((t + t0) / t0) ** -0.5


def test_thick_pulse_follows_the_diffusion_solution(orc):
    """Sec. 5.4's thick pulse (tau = 1e3 per cell): the radiation energy follows
    eq. diffsol with D = 1/(3 kappa_tot) through a doubling of the pulse's
    variance, within 1% of the initial peak, and the deviation falls at second
    order with the cells per pulse width."""
    e_fine, pk = _pulse(orc, 100)
    e_coarse, _ = _pulse(orc, 50)
    assert e_fine < 1e-2 and abs(pk - 1) < 1.5e-2, (e_fine, pk)
    assert e_coarse / e_fine > 2.5, (e_coarse, e_fine)
