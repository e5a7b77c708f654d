"""Adjoint of the PPM step (Sec. 4.3 reconstruction with the shock
flattener) through the C ABI, against central differences of the GPU step
and of the FP64 oracle's step, as tests/test_gpu_adjoint.py does for MC.

Beyond MC the PPM adjoint carries the six-cell stencil, the sqrt(-g)
weighting of vector primitives along r on Kerr-Schild, and the flattener:
its value enters each face state, it is the largest over the step's
sub-steps, and inside its ramp (0 < f < 1) it depends on the pressures,
densities and opacities of seven cells.  The shock box puts flattener cells
on that ramp (checked on the oracle's flattener before the GPU runs) and
the checks sample components around them.
"""
import math
import sys

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_gpu_adjoint import (_chi_check, _step_check, dev, fd_rows, host,  # noqa: E402
                              interior_idx, norm_err)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    from paper_1312_6127_amd import grrmhd

    grrmhd.lib()
    assert torch.cuda.is_available()
    return grrmhd


def shock_box(n=(32, 1, 1), w=1.0, seed=5):
    """Periodic Minkowski box with two smoothed jumps (width w cells) of
    pressure, density and radiation energy at a quarter and three quarters
    of x1, and a converging x1 flow at both: the flattener's compression
    test passes there and its ramp reads |dp1|/|dp2| = tanh(1/w)/tanh(2/w)
    (0.79 at w = 1, f = 0.4).  LAXF, a_rad = 0.5, per-mass opacities 1 and
    0.3 (tau = 0.04 per cell, flattener weight w = 0.08)."""
    pd = I.default_params(n=n, arad=0.5, flux="llf", ng=4, recon="ppm")
    N = I.ncell(pd)
    x1, x2, _ = I.cell_coords(pd)
    L1 = pd["xhi"][0] - pd["xlo"][0]
    i = (x1 - pd["xlo"][0]) / (L1 / n[0]) - 0.5
    jump = np.tanh((i - n[0] / 4) / w) - np.tanh((i - 3 * n[0] / 4) / w)
    kx = 2 * math.pi
    P = np.zeros((12,) + x1.shape)
    P[0] = 1.0 + 0.4 * jump + 0.05 * np.sin(kx * x2)
    P[1] = 0.6 + 0.35 * jump + 0.05 * np.cos(kx * x2)
    P[2] = -0.3 * np.sin(2 * kx * (x1 - pd["xlo"][0] - 0.25 * L1))
    P[3] = 0.1 * np.cos(kx * x1)
    P[4] = 0.05 + 0.03 * np.sin(kx * x1)
    P[5] = 0.2
    P[6] = 0.1 * np.sin(kx * x1)
    P[7] = 0.05 + 0.02 * np.cos(kx * x1)
    P[8] = 0.8 + 0.5 * jump
    P[9] = P[2] + 0.02
    P[10] = P[3]
    P[11] = P[4] - 0.01
    P = P.reshape(12, N)
    # jittered (relative noise 1e-3) so no limiter or speed extremum sits on
    # a tie, and no field is zero (a zero field's difference step would be
    # left to rounding)
    return pd, I.jitter(P, 11), np.full(N, 1.0), np.full(N, 0.3)


def disk_small_ppm():
    pd, P, ca, ce = I.accretion_disk(n=(12, 8, 4), seed=3, ng=4, recon="ppm")
    return pd, I.jitter(P, 11), ca, ce


def _ramp_cells(orc, pd, P, ca, ce):
    """Interior cells within three cells (along x1) of a flattener value on
    the ramp; asserts there are some."""
    fl = orc.flattener(pd, orc.bc(pd, P), ca, ce)
    ramp = np.flatnonzero(((fl[0] > 1e-3) & (fl[0] < 1 - 1e-3)).any(axis=0))
    assert ramp.size >= 4
    idx = interior_idx(pd)
    near = np.unique((ramp[:, None] + np.arange(-3, 4)[None, :]).reshape(-1))
    return np.intersect1d(near, idx)


def test_explicit_vjp_ppm_against_fd(G, orc):
    """Fluxes (with the flattener of P) + EMFs + update, with respect to the
    ghost-filled primitives, on the 2-D shock box around the ramp cells."""
    say("case explicit vjp, PPM shock box 2-D")
    pd, P, ca, ce = shock_box(n=(32, 6, 1))
    g = G.Grid(pd)
    cat, cet = dev(ca), dev(ce)
    Pb = host(g.apply_bc(dev(P)))
    cells = _ramp_cells(orc, pd, Pb, ca, ce)
    dt = dev(np.array([0.004]))
    Ut = g.prim_to_cons(dev(Pb))
    idx = interior_idx(pd)
    r = np.random.default_rng(3)
    lue = np.zeros_like(P)
    lue[:, idx] = r.standard_normal((12, idx.size))
    gP = host(g.explicit_vjp(0.25, dt, dev(Pb), cat, cet, dev(lue)))

    def Ue_of(Pp):
        Pt = dev(Pp)
        F, emf, vch = g.fluxes(Pt, cat, cet)
        return host(g.explicit_update(0.75, 0.25, 0.25, dt, Pt, Ut, Ut, F, emf))

    scale = np.abs(Pb).max(axis=1)
    comps = [(int(r.integers(12)), int(cells[r.integers(cells.size)])) for _ in range(48)]
    comps += [(int(r.integers(12)), int(r.integers(P.shape[1]))) for _ in range(16)]
    fd = fd_rows(comps, Pb, scale, Ue_of, lue)
    fd3 = fd_rows(comps, Pb, scale, Ue_of, lue, f=1 / 3)
    smooth = np.abs(fd - fd3) <= 1e-4 * np.abs(fd) + 1e-12
    say(f"  {int((~smooth).sum())} of {len(comps)} components straddle a kink")
    assert (~smooth).sum() <= 6
    adj = np.array([gP[q, c] for q, c in comps])[smooth]
    e = norm_err(adj, fd[smooth])
    say("  explicit vjp norm error", e)
    assert e < 1e-7
    g.close()


def test_step_adjoint_ppm_shock_box(G, orc):
    """RK3 step of the 1-D shock box: components around the flattener's
    ramp cells (and through them the sub-step rule) against GPU and oracle
    differences."""
    say("case step adjoint, PPM shock box")
    pd, P, ca, ce = shock_box()
    cells = _ramp_cells(orc, pd, P, ca, ce)
    _step_check(G, orc, pd, P, ca, ce, ncomp=64, n_oracle=32, tol=1e-6, kinks=8, cells=cells)


def test_step_adjoint_ppm_shock_box_2d(G, orc):
    say("case step adjoint, PPM shock box 2-D")
    pd, P, ca, ce = shock_box(n=(32, 6, 1))
    cells = _ramp_cells(orc, pd, P, ca, ce)
    _step_check(G, orc, pd, P, ca, ce, ncomp=48, n_oracle=16, tol=1e-6, kinks=8, cells=cells)


def test_step_adjoint_ppm_kerr_schild(G, orc):
    """The 12x8x4 Kerr-Schild disk: the sqrt(-g) weighting along r, the
    polar axis and six-cell stencils in three directions."""
    say("case step adjoint, PPM Kerr-Schild 12x8x4")
    _step_check(G, orc, *disk_small_ppm(), ncomp=64, n_oracle=32, tol=1e-6, kinks=6, f=10.0)


def test_step_adjoint_ppm_kerr_schild_ramp(G, orc):
    """The 32x8x4 Kerr-Schild disk, whose steep radial profiles put
    flattener values on the ramp near the inner edge and further out (the
    compression test reads the mass fluxes sqrt(-g) u^r): components around
    them against GPU and oracle differences."""
    say("case step adjoint, PPM Kerr-Schild 32x8x4, flattener ramp")
    pd, P, ca, ce = I.accretion_disk(n=(32, 8, 4), seed=3, ng=4, recon="ppm")
    P = I.jitter(P, 11)
    cells = _ramp_cells(orc, pd, P, ca, ce)
    _step_check(G, orc, pd, P, ca, ce, ncomp=48, n_oracle=16, tol=1e-6, kinks=8, f=10.0,
                cells=cells)


@pytest.mark.parametrize("scheme", ["imex2", "imex3"])
def test_step_adjoint_ppm_imex(G, orc, scheme):
    """IMEX stage tables with PPM: the flattener is the largest over the
    stages that evaluate fluxes."""
    say("case step adjoint, PPM shock box", scheme)
    pd, P, ca, ce = shock_box()
    cells = _ramp_cells(orc, pd, P, ca, ce)
    _step_check(G, orc, dict(pd, scheme=scheme), P, ca, ce, ncomp=48, n_oracle=16, tol=1e-6,
                kinks=8, cells=cells)


def test_opacity_gradient_ppm_shock_box(G, orc):
    """dL/dchi through the flattener's weights (ramp cells) as well as the
    radiation speed limiter and the implicit solve."""
    say("case opacity gradient, PPM shock box")
    pd, P, ca, ce = shock_box()
    r = np.random.default_rng(4)
    ca = ca * (1 + 0.3 * r.random(ca.size))
    ce = ce * (1 + 0.3 * r.random(ce.size))
    cells = _ramp_cells(orc, pd, P, ca, ce)
    _chi_check(G, orc, pd, P, ca, ce, ncomp=48, n_oracle=16, tol=1e-6, cells=cells)


def test_checkpointed_halves_ppm(G):
    """The two halves on a PPM grid give the whole adjoint bit for bit."""
    say("case checkpointed halves, PPM")
    pd, P, ca, ce = shock_box(n=(32, 6, 1))
    g = G.Grid(pd)
    cat, cet = dev(ca), dev(ce)
    dt = dev(np.array([0.004]))
    w = dev(np.random.default_rng(11).standard_normal(P.shape))
    Pn, Un, ws = g.step_checkpointed(dev(P), cat, cet, dt)
    gP, gc = g.step_adjoint(dev(P), cat, cet, dt, w, want_chi=True)
    gPs, gcs = g.step_adjoint_saved(ws, cat, cet, dt, w, want_chi=True)
    assert torch.equal(gP, gPs) and torch.equal(gc, gcs)
    g.close()
