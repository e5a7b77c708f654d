"""Pins of the oracle's staggered face-centred field with four-state corner
EMFs (Sec. 4: the magnetic P_q, U_q at faces and their fluxes at corners;
Sec. 4.2 steps 8-11; Sec. 4.4 on the EMF speeds; Del Zanna et al. 2007).

Each test checks the oracle against something other than itself:
- Stokes' theorem: the face update is a circulation of the EMFs, so the
  discrete divergence of the face field keeps its initial value (zero for a
  field made as the curl of an edge potential) through whole steps, on flat
  boxes and on Kerr-Schild disks with the polar axis, and the total face
  flux of a periodic box is conserved;
- reduction: on a grid with one active dimension the four-state EMF is the
  two-state HLL/LAXF flux of the transverse field, so the staggered step
  equals the flux-CT step (which then uses the face fluxes themselves), along
  each of the three axes;
- symmetry: a cyclic relabelling of the axes of a 3-D periodic box commutes
  with the step; a reflecting wall equals the mirrored domain;
- the ghost fill continues a uniform Cartesian field through the polar axis;
- accuracy: an oblique Alfven wave (closed-form speed B/sqrt(w) in the
  fluid frame, w = rho0 + u_g + p + b^2) returns after one period with an L1
  error falling at second order.
"""
import math

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I
from test_oracle_scheme_pins import _ks_cart_components


def _stag(pd):
    return dict(pd, ct="staggered")


def _ijk(pd):
    na = I.nalloc(pd)
    N = I.ncell(pd)
    c = np.arange(N)
    return c % na[0], c // na[0] % na[1], c // (na[0] * na[1])


def _interior(pd):
    m = np.zeros(I.nalloc(pd)[::-1], dtype=bool)
    m[I.interior(pd)] = True
    return m.reshape(-1)


def _strides(pd):
    na = I.nalloc(pd)
    return [1, na[0], na[0] * na[1]]


def _div(pd, Bf):
    """Discrete divergence sum_p (Bf^p(c + e_p) - Bf^p(c)) / dx_p at the
    interior cells."""
    st = _strides(pd)
    m = np.nonzero(_interior(pd))[0]
    out = np.zeros(m.size)
    for p in range(3):
        if pd["n"][p] > 1:
            dx = (pd["xhi"][p] - pd["xlo"][p]) / pd["n"][p]
            out += (Bf[p][m + st[p]] - Bf[p][m]) / dx
    return out


def _random_box(n, seed, vmax=0.4, bscale=0.6, **kw):
    """Periodic flat box of cubic cells with random flow, gas, radiation and a
    random edge potential (its curl the face field; ghost faces unfilled)."""
    L = tuple(0.1 * v for v in n)
    pd = _stag(I.default_params(n=n, xhi=L, flux="hll", courant=0.4, arad=0.5, **kw))
    N = I.ncell(pd)
    cells = np.arange(N)
    u = lambda d: I.uniform(seed, cells, d)
    P = np.zeros((12, N))
    P[0] = 0.5 + u(0)
    P[1] = 0.2 + 0.3 * u(1)
    for d in range(3):
        P[2 + d] = vmax * (2 * u(2 + d) - 1)
        P[9 + d] = P[2 + d] + 0.1 * (2 * u(5 + d) - 1)
    P[8] = 0.1 + 0.2 * u(8)
    # the potential periodic too: draws of the wrapped interior position
    g, na = pd["ng"], I.nalloc(pd)
    i, j, k = _ijk(pd)
    wrap = ((i - g) % n[0] + g) + na[0] * (((j - g) % n[1] + g) + na[1] * ((k - g) % n[2] + g))
    A = np.stack([bscale * 0.1 * (2 * I.uniform(seed, wrap, 9 + d) - 1) for d in range(3)])
    Bf = I.face_field_from_potential(pd, A)
    ca, ce = 0.5 + u(12), 0.2 * u(13)
    return pd, P, Bf, ca, ce


def _consistent(orc, pd, P, Bf):
    """Primitives with the cell-centred field of the faces, ghost cells
    filled, and their conserved state."""
    P, _ = orc.face_to_center(pd, Bf, P, np.zeros_like(P))
    P = orc.bc(pd, P)
    return P, orc.prim_to_cons(pd, P)


# ---------------------------------------------------------------------------
# Stokes' theorem
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", ["rk3", "imex2", "imex2b", "imex3"])
def test_divergence_stays_at_roundoff_on_a_periodic_box(orc, scheme):
    """Every stage's faces change by the circulation of its EMFs, also in
    the IMEX tables (Sec. 4.1), whose stages without explicit fluxes combine
    earlier faces linearly."""
    pd, P, Bf, ca, ce = _random_box((10, 8, 6), seed=11)
    pd = dict(pd, scheme=scheme)
    Bf = orc.bc_face(pd, Bf)
    P, U = _consistent(orc, pd, P, Bf)
    scale = np.abs(Bf).max() / 0.1
    d0 = np.abs(_div(pd, Bf)).max() / scale
    tot0 = [Bf[p][_interior(pd)].sum() for p in range(3)]
    for _ in range(3):
        P, U, Bf, dt, st, it, nbad = orc.step_stag(pd, P, U, Bf, ca, ce)
        assert nbad == 0
    d1 = np.abs(_div(pd, Bf)).max() / scale
    assert d0 < 1e-14 and d1 < 1e-13, (d0, d1)
    # total flux through the faces of each direction: a telescoping sum
    for p in range(3):
        tot = Bf[p][_interior(pd)].sum()
        assert abs(tot - tot0[p]) <= 1e-13 * np.abs(Bf[p]).sum(), p
    # the field moved: the check is not vacuous
    assert np.abs(Bf - _random_box((10, 8, 6), seed=11)[2]).max() > 1e-3 * np.abs(Bf).max()


@pytest.mark.parametrize("n", [(40, 24, 1), (16, 12, 8)])
def test_divergence_stays_at_roundoff_on_a_kerr_schild_disk(orc, n):
    """The disk's poloidal field made as the curl of A_phi, with the polar
    axis (2-D reflecting, 3-D POLAR) and outflow in r."""
    pd, P, ca, ce, Bf = I.accretion_disk(n=n, seed=3, faces=True)
    pd = _stag(pd)
    Bf = orc.bc_face(pd, Bf)
    P, U = _consistent(orc, pd, P, Bf)
    dx = min((pd["xhi"][d] - pd["xlo"][d]) / pd["n"][d] for d in range(3) if pd["n"][d] > 1)
    scale = np.abs(Bf).max() / dx
    d0 = np.abs(_div(pd, Bf)).max() / scale
    B0 = Bf.copy()
    for _ in range(2):
        P, U, Bf, dt, st, it, nbad = orc.step_stag(pd, P, U, Bf, ca, ce)
    d1 = np.abs(_div(pd, Bf)).max() / scale
    assert d0 < 1e-14 and d1 < 1e-13, (d0, d1)
    assert np.abs(Bf - B0)[:, _interior(pd)].max() > 1e-6 * np.abs(B0).max()


# ---------------------------------------------------------------------------
# reduction to the two-state flux on one active dimension
# ---------------------------------------------------------------------------

def _tube(d, n=64, flux="hll"):
    """Relativistic Brio-Wu tube along axis d (Gamma = 2, normal field 0.5,
    transverse field +-1) with radiation coupled to the gas."""
    nn = [1, 1, 1]
    nn[d] = n
    lo, hi = [0.0] * 3, [1.0] * 3
    lo[d], hi[d] = -0.5, 0.5
    pd = I.default_params(n=tuple(nn), xlo=tuple(lo), xhi=tuple(hi), bc_lo=("outflow",) * 3,
                          bc_hi=("outflow",) * 3, gam=2.0, arad=1e-2, flux=flux, courant=0.4)
    N = I.ncell(pd)
    x = I.cell_coords(pd)[d].reshape(-1)
    left = x < 0
    P = np.zeros((12, N))
    P[0] = np.where(left, 1.0, 0.125)
    pg = np.where(left, 1.0, 0.1)
    P[1] = pg / (pd["gam"] - 1.0)
    P[5 + d] = 0.5
    P[5 + (d + 1) % 3] = np.where(left, 1.0, -1.0)
    P[5 + (d + 2) % 3] = np.where(left, 0.3, 0.2)
    P[2 + (d + 1) % 3] = np.where(left, 0.1, -0.05)
    P[8] = pd["arad"] * (pg / P[0]) ** 4
    P[9:12] = P[2:5]
    ca = np.full(N, 0.3)
    ce = np.full(N, 0.1)
    return pd, P, ca, ce


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("flux", ["hll", "llf"])
def test_one_active_dimension_equals_flux_ct(orc, d, flux):
    pd, P, ca, ce = _tube(d, flux=flux)
    U = orc.prim_to_cons(pd, P)
    ps = _stag(pd)
    Bf = np.zeros((3, P.shape[1]))
    Bf[:] = U[5:8]          # flat space: the faces of a one-dimensional field
    Bf = orc.bc_face(ps, Bf)
    Pa, Ua, Pb, Ub = P, U, P, U
    for _ in range(8):
        Pa, Ua, dta, sa, _, na_ = orc.step(pd, Pa, Ua, ca, ce)
        Pb, Ub, Bf, dtb, sb, _, nb_ = orc.step_stag(ps, Pb, Ub, Bf, ca, ce)
        assert na_ == 0 and nb_ == 0 and abs(dta / dtb - 1) < 1e-14
    m = _interior(pd)
    # per field over the field's (vector's) scale
    for grp in ((0,), (1,), (2, 3, 4), (5, 6, 7), (8,), (9, 10, 11)):
        for A, B in ((Pa, Pb), (Ua, Ub)):
            sc = np.abs(A[list(grp)][:, m]).max() + 1e-300
            assert np.abs(A[list(grp)][:, m] - B[list(grp)][:, m]).max() / sc < 1e-12, grp
    for t in range(3):
        if t != d:
            assert np.abs(Bf[t, m] - Ua[5 + t, m]).max() < 1e-12 * np.abs(Ua[5 + t, m]).max()
    # the normal field is constant
    assert np.abs(Bf[d, m] - 0.5).max() < 1e-15
    # the field's shock moved
    assert np.abs(Ua[5 + (d + 1) % 3, m] - U[5 + (d + 1) % 3, m]).max() > 0.1


@pytest.mark.parametrize("d", [0, 2])
@pytest.mark.parametrize("scheme", ["imex2", "imex2b", "imex3"])
def test_one_active_dimension_equals_flux_ct_imex(orc, d, scheme):
    """The IMEX tables: the faces of a stage without explicit fluxes are
    a Bf^n + b Bf^(j), as flux-CT combines the cell-centred field."""
    pd, P, ca, ce = _tube(d)
    pd = dict(pd, scheme=scheme)
    U = orc.prim_to_cons(pd, P)
    ps = _stag(pd)
    Bf = np.zeros((3, P.shape[1]))
    Bf[:] = U[5:8]
    Bf = orc.bc_face(ps, Bf)
    Pa, Ua, Pb, Ub = P, U, P, U
    for _ in range(4):
        Pa, Ua, dta, sa, _, na_ = orc.step(pd, Pa, Ua, ca, ce)
        Pb, Ub, Bf, dtb, sb, _, nb_ = orc.step_stag(ps, Pb, Ub, Bf, ca, ce)
        assert na_ == 0 and nb_ == 0 and abs(dta / dtb - 1) < 1e-14
    m = _interior(pd)
    for grp in ((0,), (1,), (2, 3, 4), (5, 6, 7), (8,), (9, 10, 11)):
        for A, B in ((Pa, Pb), (Ua, Ub)):
            sc = np.abs(A[list(grp)][:, m]).max() + 1e-300
            assert np.abs(A[list(grp)][:, m] - B[list(grp)][:, m]).max() / sc < 1e-12, grp
    for t in range(3):
        if t != d:
            assert np.abs(Bf[t, m] - Ua[5 + t, m]).max() < 1e-12 * np.abs(Ua[5 + t, m]).max()
    assert np.abs(Ua[5 + (d + 1) % 3, m] - U[5 + (d + 1) % 3, m]).max() > 0.05


def test_face_update_without_fluxes_combines_faces(orc):
    """c = 0: a Bn + b Bprev exactly on every evolved face, with no EMF
    read, and nothing written elsewhere."""
    pd, P, Bf, ca, ce = _random_box((6, 5, 4), seed=3)
    pd = _stag(pd)
    B1 = np.random.default_rng(1).standard_normal(Bf.shape)
    out = orc.face_update(pd, 2.0, -1.0, 0.0, 0.3, Bf, B1, None)
    want = 2.0 * Bf - 1.0 * B1
    na = I.nalloc(pd)
    g = pd["ng"]
    for p in range(3):
        ev = np.zeros(tuple(na[::-1]), bool)   # [x3][x2][x1]
        sl = [slice(g, g + pd["n"][d] + (1 if d == p else 0)) for d in range(3)]
        ev[sl[2], sl[1], sl[0]] = True
        ev = ev.reshape(-1)
        assert np.array_equal(out[p, ev], want[p, ev])
        assert np.all(out[p, ~ev] == 0.0)


def test_failed_inversion_returns_the_conserved_field(orc):
    """B^i = U_B^i / sqrt(-g) needs no inversion: a cell whose MHD inversion
    fails (negative rest-mass density rho u^t) keeps the guess's gas
    primitives but takes its field from U."""
    pd, P, Bf, ca, ce = _random_box((6, 5, 4), seed=5)
    U = orc.prim_to_cons(pd, P)
    c = _interior_index(pd)
    Ub = U.copy()
    Ub[0, c] = -abs(U[0, c])                 # no admissible density
    Pg = P.copy()
    Pg[5:8, c] += 0.3                        # a guess with another field
    Pout, st = orc.con2prim(pd, Ub, Pg)
    assert st[c] & orc.ST_C2P_FAIL
    assert np.array_equal(Pout[0:5, c], Pg[0:5, c])
    assert np.allclose(Pout[5:8, c], U[5:8, c], rtol=1e-15, atol=0)   # flat space: sqrt(-g) = 1


def _interior_index(pd):
    """One interior cell's flat index (the middle of the box)."""
    na = I.nalloc(pd)
    g = pd["ng"]
    i, j, k = (g + pd["n"][d] // 2 for d in range(3))
    return i + na[0] * (j + na[1] * k)


def test_failed_cell_takes_its_own_staggered_field(orc):
    """Staggered grid: a failed cell's neighbour average leaves B alone and
    sets it from the cell's conserved field, not from its (stale) guess; on
    a flux-CT grid B is averaged like the other primitives."""
    pd, P, Bf, ca, ce = _random_box((6, 5, 4), seed=7)
    U = orc.prim_to_cons(pd, P)
    c = _interior_index(pd)
    st = np.zeros(P.shape[1], np.int32)
    st[c] = orc.ST_FAIL
    Pstale = P.copy()
    Pstale[5:8, c] += 0.25
    Ps, Us, sts = orc.fixup(_stag(pd), Pstale, U, st)
    assert np.allclose(Ps[5:8, c], U[5:8, c], rtol=1e-15, atol=0)
    na = I.nalloc(pd)
    nbs = [c + s * st_ for st_ in (1, na[0], na[0] * na[1]) for s in (-1, 1)]
    assert np.allclose(Ps[0, c], np.mean([P[0, n] for n in nbs]), rtol=1e-14)
    Pf, Uf, stf = orc.fixup(dict(pd, ct="flux"), Pstale, U, st)
    assert np.allclose(Pf[5:8, c], np.mean([Pstale[5:8, n] for n in nbs], axis=0), rtol=1e-14)


# ---------------------------------------------------------------------------
# symmetry
# ---------------------------------------------------------------------------

def _cycle(pd, X, vec_rows):
    """Relabel axes x1 -> x2 -> x3 -> x1 of arrays [rows][N] (vector rows in
    groups of three are rotated alike)."""
    na = I.nalloc(pd)
    Y = X.reshape((X.shape[0], na[2], na[1], na[0])).transpose(0, 2, 3, 1).copy()
    for r0 in vec_rows:
        Y[r0:r0 + 3] = Y[[r0 + 2, r0, r0 + 1]]
    return Y.reshape(X.shape[0], -1)


def test_cyclic_relabelling_of_axes_commutes_with_the_step(orc):
    pd, P, Bf, ca, ce = _random_box((8, 6, 4), seed=17)
    Bf = orc.bc_face(pd, Bf)
    P, U = _consistent(orc, pd, P, Bf)
    n = pd["n"]
    pc = dict(pd, n=(n[2], n[0], n[1]), xhi=(pd["xhi"][2], pd["xhi"][0], pd["xhi"][1]))
    Pc, Uc, Bc = _cycle(pd, P, [2, 5, 9]), _cycle(pd, U, [2, 5, 9]), _cycle(pd, Bf, [0])
    cac, cec = _cycle(pd, ca[None], [])[0], _cycle(pd, ce[None], [])[0]
    P1, U1, B1, dt, *_ = orc.step_stag(pd, P, U, Bf, ca, ce)
    P2, U2, B2, dt2, *_ = orc.step_stag(pc, Pc, Uc, Bc, cac, cec)
    assert abs(dt2 / dt - 1) < 1e-14
    m = _interior(pc)
    for A, B in ((_cycle(pd, P1, [2, 5, 9]), P2), (_cycle(pd, U1, [2, 5, 9]), U2)):
        sc = np.abs(B[:, m]).max(axis=1) + 1e-300
        assert (np.abs(A[:, m] - B[:, m]).max(axis=1) / sc).max() < 1e-13
    A = _cycle(pd, B1, [0])
    assert np.abs(A[:, m] - B2[:, m]).max() < 1e-13 * np.abs(B2).max()


def _mirror2d(x, y):
    """A smooth 2-D state even in x with odd normal velocities, and the edge
    potential A_3 odd in x (so the normal field is odd and zero on x = 0)."""
    P = np.zeros((12, x.size))
    P[0] = 1.0 + 0.4 * np.exp(-((np.abs(x) - 0.3) / 0.2) ** 2) * (1 + 0.3 * np.sin(2 * np.pi * y))
    P[1] = 0.3 + 0.1 * np.cos(3 * x) * (1 + 0.2 * np.cos(2 * np.pi * y))
    P[2] = -0.4 * np.sin(2.5 * x)
    P[3] = 0.2 * np.cos(x) * np.sin(2 * np.pi * y)
    P[8] = 0.5 + 0.3 * np.exp(-((np.abs(x) - 0.6) / 0.15) ** 2)
    P[9] = P[2] + 0.05 * np.sin(x)
    P[10] = P[3]
    return P


@pytest.mark.parametrize("flux", ["hll", "llf"])
def test_reflecting_wall_equals_mirrored_domain(orc, flux):
    n, ny = 16, 8
    kw = dict(flux=flux, courant=0.4, arad=0.7)
    pa = _stag(I.default_params(n=(n, ny, 1), bc_lo=("reflect", "periodic", "periodic"),
                                bc_hi=("outflow", "periodic", "periodic"), **kw))
    pb = _stag(I.default_params(n=(2 * n, ny, 1), xlo=(-1.0, 0.0, 0.0),
                                bc_lo=("outflow", "periodic", "periodic"),
                                bc_hi=("outflow", "periodic", "periodic"), **kw))
    out = []
    for pd in (pa, pb):
        x, y, _ = (c.reshape(-1) for c in I.cell_coords(pd))
        P = _mirror2d(x, y)
        # A_3 at the cell's lower-left corner
        dx, dy = 1.0 / n, 1.0 / ny
        xc, yc = x - 0.5 * dx, y - 0.5 * dy
        A = np.zeros((3, x.size))
        A[2] = 0.05 * xc * (1 + 0.5 * np.cos(2 * np.pi * yc)) * np.exp(-xc ** 2)
        Bf = I.face_field_from_potential(pd, A)
        Bf[2] = 0.1 * np.cos(2 * x)          # B^3, even in x
        Bf = orc.bc_face(pd, Bf)
        P, U = _consistent(orc, pd, P, Bf)
        N = x.size
        ca, ce = np.full(N, 0.8), np.full(N, 0.3)
        for _ in range(4):
            P, U, Bf, dt, st, it, nbad = orc.step_stag(pd, P, U, Bf, ca, ce, dt=0.004,
                                                         dt_fixed=True)
            assert nbad == 0
        out.append((pd, P, Bf))
    (pa, Pa, Ba), (pb, Pb, Bb) = out
    g = pa["ng"]
    na_a, na_b = I.nalloc(pa), I.nalloc(pb)
    Pa = Pa.reshape(12, na_a[1], na_a[0])[:, g:g + ny, g:g + n]
    Pb = Pb.reshape(12, na_b[1], na_b[0])[:, g:g + ny]
    pos, neg = Pb[:, :, g + n:g + 2 * n], Pb[:, :, g:g + n][:, :, ::-1].copy()
    odd = [2, 5, 9]
    neg[odd] *= -1.0
    row = np.abs(Pa).reshape(12, -1).max(axis=1)
    for grp in ((2, 3, 4), (5, 6, 7), (9, 10, 11)):
        row[list(grp)] = row[list(grp)].max()
    sc = row[:, None, None] + 1e-300
    assert (np.abs(Pa - pos) / sc).max() < 1e-13
    assert (np.abs(neg - pos) / sc).max() < 1e-13
    # faces: x1 faces from the wall outwards, the others cell-aligned
    Ba = Ba.reshape(3, na_a[1], na_a[0])[:, g:g + ny]
    Bb = Bb.reshape(3, na_b[1], na_b[0])[:, g:g + ny]
    sc = np.abs(Ba).max()
    assert np.abs(Ba[0, :, g:g + n + 1] - Bb[0, :, g + n:g + 2 * n + 1]).max() < 1e-13 * sc
    assert np.abs(Ba[1:, :, g:g + n] - Bb[1:, :, g + n:g + 2 * n]).max() < 1e-13 * sc
    # the wall's normal field (zero at the start) stays zero up to rounding
    assert np.abs(Ba[0, :, g]).max() < 1e-16 * sc


def test_polar_axis_continues_uniform_cartesian_field(orc):
    """POLAR (3-D Kerr-Schild): ghost faces beyond the axis take sqrt(-g) B^p
    of the uniform Cartesian field at their own coordinates, when the evolved
    faces hold it."""
    pd = _stag(I.disk_params(n=(4, 6, 8)))
    N = I.ncell(pd)
    i, j, k = _ijk(pd)
    g = pd["ng"]
    dx = [(pd["xhi"][d] - pd["xlo"][d]) / pd["n"][d] for d in range(3)]
    Vb = np.array([0.1, 0.05, 0.4])
    Bf = np.zeros((3, N))
    for p in range(3):
        for c in range(N):
            x = [pd["xlo"][d] + (idx - g + (0.0 if d == p else 0.5)) * dx[d]
                 for d, idx in enumerate((i[c], j[c], k[c]))]
            if abs(math.sin(math.pi * x[1])) < 1e-12:
                continue                      # a face on the axis: sqrt(-g) = 0
            G = orc.geom(pd, x[0], x[1])
            Bf[p, c] = G.gdet * _ks_cart_components(pd, *x, Vb)[p]
    n = pd["n"]
    evolved = np.zeros((3, N), dtype=bool)
    for p in range(3):
        hi = [n[d] + (1 if d == p else 0) for d in range(3)]
        evolved[p] = ((i >= g) & (i < g + hi[0]) & (j >= g) & (j < g + hi[1]) &
                      (k >= g) & (k < g + hi[2]))
    out = orc.bc_face(pd, np.where(evolved, Bf, 0.0))
    axis_ghost = ((j < g) | (j > g + n[1])) & (i >= g) & (i < g + n[0])
    for p in range(3):
        sel = axis_ghost & ~evolved[p]
        sc = np.abs(Bf[p, sel]).max()
        assert sc > 0 and np.abs(out[p, sel] - Bf[p, sel]).max() < 1e-12 * sc, p


# ---------------------------------------------------------------------------
# an oblique Alfven wave
# ---------------------------------------------------------------------------

def _alfven_run(orc, n, eps=1e-6):
    """Periodic unit box, n x n cells, uniform field B0 along k = 2 pi (1, 1)
    on gas at rest (rho0 = 1, p = 1, Gamma = 5/3, no radiation coupling),
    both Alfven polarisations (in the plane and along x3) moving along +k at
    v_A = B0 / sqrt(w); L1 error of (u~, B) after one period, over eps."""
    pd = _stag(I.default_params(n=(n, n, 1), flux="hll", courant=0.4, arad=1e-8))
    N = I.ncell(pd)
    x, y, _ = (c.reshape(-1) for c in I.cell_coords(pd))
    h = 1.0 / n
    kv = 2 * math.pi * np.array([1.0, 1.0])
    kh = kv / np.linalg.norm(kv)
    nperp = np.array([-kh[1], kh[0]])
    B0, rho, pg, gam = 1.0, 1.0, 1.0, pd["gam"]
    ug = pg / (gam - 1)
    w = rho + ug + pg + B0 ** 2
    vA = B0 / math.sqrt(w)
    T = (2 * math.pi / np.linalg.norm(kv)) / vA

    def exact(t):
        ph = kv[0] * (x - vA * kh[0] * t) + kv[1] * (y - vA * kh[1] * t)
        Q = np.zeros((12, N))
        Q[0], Q[1] = rho, ug
        dv = eps * np.sin(ph)
        Q[2], Q[3] = dv * nperp[0], dv * nperp[1]
        Q[4] = 0.7 * dv
        Q[5], Q[6] = B0 * kh[0] - math.sqrt(w) * dv * nperp[0], B0 * kh[1] - math.sqrt(w) * dv * nperp[1]
        Q[7] = -math.sqrt(w) * 0.7 * dv
        Q[8] = 1e-10
        Q[9:12] = Q[2:5]
        return Q

    P = exact(0.0)
    # faces: the uniform part directly, the in-plane wave as the curl of
    # A_3 = -sqrt(w) eps cos(k.x) / |k| at the lower-left corners
    A = np.zeros((3, N))
    xc, yc = x - 0.5 * h, y - 0.5 * h
    A[2] = -math.sqrt(w) * eps * np.cos(kv[0] * xc + kv[1] * yc) / np.linalg.norm(kv)
    Bf = I.face_field_from_potential(pd, A)
    Bf[0] += B0 * kh[0]
    Bf[1] += B0 * kh[1]
    Bf[2] = P[7]
    Bf = orc.bc_face(pd, Bf)
    P, U = _consistent(orc, pd, P, Bf)
    ca, ce = np.zeros(N), np.zeros(N)
    # fixed steps: dt within the Courant limit of the fast speed (< 1)
    nsteps = int(math.ceil(T / (0.4 * h / 2.0)))
    dt = T / nsteps
    for _ in range(nsteps):
        P, U, Bf, _, st, it, nbad = orc.step_stag(pd, P, U, Bf, ca, ce, dt=dt, dt_fixed=True)
    m = _interior(pd)
    Q = exact(T)
    err = np.abs(P[2:8, m] - Q[2:8, m]).mean(axis=1)
    return err.sum() / eps


def test_oblique_alfven_wave_converges_at_second_order(orc):
    e = [_alfven_run(orc, n) for n in (8, 16, 32)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) > 1.7, (e, orders)
    assert e[-1] < 0.2, e
