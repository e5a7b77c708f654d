"""The staggered face-centred field with four-state corner EMFs on the GPU
against the oracle (Sec. 4, Sec. 4.2 steps 8-11, Sec. 4.4): ghost faces,
face-to-centre field, fluxes with the faces' normal field and the corner
EMFs, and whole RK3 and IMEX steps, per field to the one-step tolerance
(1e-12 of the field's scale; 1e-5 on the FP32-mixed path), plus the discrete
divergence of the GPU's faces at round-off at the benchmark's full size."""
import sys

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_gpu_parity import dev, field_err, host, interior_mask  # noqa: E402
from test_oracle_stag import _consistent, _div, _random_box, _stag, _tube  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    from paper_1312_6127_amd import grrmhd

    grrmhd.lib()
    assert torch.cuda.is_available()
    return grrmhd


def _disk(n, **kw):
    pd, P, ca, ce, Bf = I.accretion_disk(n=n, seed=3, faces=True, **kw)
    return _stag(pd), P, ca, ce, Bf


def _tube_case(d, flux="hll"):
    pd, P, ca, ce = _tube(d, flux=flux)
    Bf = np.zeros((3, P.shape[1]))
    Bf[:] = P[5:8]          # flat space, one active dimension
    return _stag(pd), P, ca, ce, Bf


def _box(seed=11, **kw):
    pd, P, Bf, ca, ce = _random_box((10, 8, 6), seed=seed, **kw)
    return pd, P, ca, ce, Bf


CASES = {
    "box3d": lambda: _box(),
    "tube_x1": lambda: _tube_case(0),
    "tube_x2_llf": lambda: _tube_case(1, "llf"),
    "tube_x3": lambda: _tube_case(2),
    "disk2d": lambda: _disk((40, 24, 1)),
    "disk3d": lambda: _disk((24, 12, 8)),
    "disk3d_hll": lambda: _disk((20, 10, 6), flux="hll"),
}


def _prepared(orc, case):
    pd, P, ca, ce, Bf = CASES[case]()
    Bf = orc.bc_face(pd, Bf)
    P, U = _consistent(orc, pd, P, Bf)
    return pd, P, U, ca, ce, Bf


def _evolved(pd):
    """Mask [3][N] of the evolved faces: [ng, ng+n] along the face's axis
    ([ng, ng+n) when periodic), the interior across."""
    na = I.nalloc(pd)
    N = I.ncell(pd)
    c = np.arange(N)
    idx = (c % na[0], c // na[0] % na[1], c // (na[0] * na[1]))
    m = np.zeros((3, N), dtype=bool)
    for p in range(3):
        ok = np.ones(N, dtype=bool)
        for d in range(3):
            g = pd["ng"] if pd["n"][d] > 1 else 0
            top = pd["n"][d] + (1 if (d == p and pd["n"][d] > 1 and pd["bc_hi"][d] != "periodic") else 0)
            ok &= (idx[d] >= g) & (idx[d] < g + top)
        m[p] = ok
    return m


def _face_err(a, b, mask):
    sc = np.abs(b[mask]).max()
    return np.abs(a[mask] - b[mask]).max() / sc if sc > 0 else np.abs(a[mask]).max()


@pytest.mark.parametrize("case", ["box3d", "tube_x2_llf", "disk2d", "disk3d"])
def test_ghost_faces_and_centre_field(G, orc, case):
    say("case", case, "face ghosts / centre field")
    pd, P, ca, ce, Bf = CASES[case]()
    gr = G.Grid(pd)
    Bt = dev(Bf)
    gr.apply_bc_faces(Bt)
    ref = orc.bc_face(pd, Bf)
    got = host(Bt)
    sc = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-15 * sc
    Pt, Ut = dev(P), dev(np.zeros_like(P))
    gr.face_to_center(dev(ref), Pt, Ut)
    Pr, Ur = orc.face_to_center(pd, ref, P, np.zeros_like(P))
    m = interior_mask(pd)
    assert np.array_equal(host(Ut)[5:8, m], Ur[5:8, m])
    assert field_err(host(Pt), Pr, m).max() < 1e-15
    gr.close()


@pytest.mark.parametrize("case", ["box3d", "tube_x1", "disk2d", "disk3d", "disk3d_hll"])
def test_fluxes_and_corner_emfs(G, orc, case):
    say("case", case, "staggered fluxes")
    pd, P, U, ca, ce, Bf = _prepared(orc, case)
    gr = G.Grid(pd)
    F, emf, vch = (host(x) for x in gr.fluxes_staggered(dev(P), dev(Bf), dev(ca), dev(ce)))
    Fr, emfr, vchr = orc.fluxes_stag(pd, P, Bf, ca, ce)
    gr.close()
    eF = field_err(F.reshape(36, -1), Fr.reshape(36, -1))
    eE = field_err(emf, emfr)
    eV = field_err(vch, vchr)
    say("  F", eF.max(), "emf", eE, "vchar", eV.max())
    assert eF.max() < 1e-12 and eE.max() < 1e-12 and eV.max() < 1e-13
    assert np.abs(emfr).max() > 0


def _gpu_steps(G, pd, P, U, Bf, ca, ce, nsteps, status=False):
    gr = G.Grid(pd)
    Pt, Ut, Bt = dev(P), dev(U), dev(Bf)
    dtt = torch.zeros(1, dtype=torch.float64, device="cuda")
    stt = torch.zeros(gr.N, dtype=torch.int32, device="cuda") if status else None
    dts = []
    for _ in range(nsteps):
        gr.step_staggered(Pt, Ut, Bt, dev(ca), dev(ce), dtt, status=stt)
        dts.append(float(host(dtt)[0]))
    out = host(Pt), host(Ut), host(Bt), dts, (host(stt) if status else None)
    gr.close()
    return out


@pytest.mark.parametrize("case,nsteps", [("box3d", 2), ("tube_x1", 3), ("tube_x2_llf", 2),
                                          ("tube_x3", 2), ("disk2d", 2), ("disk3d", 2),
                                          ("disk3d_hll", 1)])
def test_staggered_steps(G, orc, case, nsteps):
    say("case", case, "staggered steps", nsteps)
    pd, P, U, ca, ce, Bf = _prepared(orc, case)
    Pr, Ur, Br = P, U, Bf
    dtr = []
    for _ in range(nsteps):
        Pr, Ur, Br, dt, st, it, nbad = orc.step_stag(pd, Pr, Ur, Br, ca, ce)
        dtr.append(dt)
    Pg, Ug, Bg, dtg, _ = _gpu_steps(G, pd, P, U, Bf, ca, ce, nsteps)
    m = interior_mask(pd)
    ev = _evolved(pd)
    eP, eU = field_err(Pg, Pr, m), field_err(Ug, Ur, m)
    eB = [_face_err(Bg[p], Br[p], ev[p]) for p in range(3)]
    say("  dt", max(abs(a / b - 1) for a, b in zip(dtg, dtr)), "P", eP.max(), "U", eU.max(),
        "faces", eB)
    assert max(abs(a / b - 1) for a, b in zip(dtg, dtr)) < 1e-13
    tol = 1e-12 * nsteps
    assert eP.max() < tol and eU.max() < tol and max(eB) < tol
    # the field moved
    assert max(np.abs(Br[p][ev[p]] - Bf[p][ev[p]]).max() for p in range(3)) > 0


@pytest.mark.parametrize("scheme", ["imex2", "imex2b", "imex3"])
@pytest.mark.parametrize("case", ["box3d", "tube_x1", "disk3d"])
def test_staggered_imex_steps(G, orc, case, scheme):
    """The IMEX stage tables (Sec. 4.1) with the staggered field: each
    stage's faces with the stage's coefficients (no EMF term where the stage
    has no explicit flux), two steps against the oracle's; on the box the
    GPU's face divergence stays at round-off."""
    say("case", case, scheme, "staggered steps")
    pd, P, U, ca, ce, Bf = _prepared(orc, case)
    pd = dict(pd, scheme=scheme)
    Pr, Ur, Br = P, U, Bf
    dtr = []
    for _ in range(2):
        Pr, Ur, Br, dt, st, it, nbad = orc.step_stag(pd, Pr, Ur, Br, ca, ce)
        dtr.append(dt)
    Pg, Ug, Bg, dtg, _ = _gpu_steps(G, pd, P, U, Bf, ca, ce, 2)
    m = interior_mask(pd)
    ev = _evolved(pd)
    eP, eU = field_err(Pg, Pr, m), field_err(Ug, Ur, m)
    eB = [_face_err(Bg[p], Br[p], ev[p]) for p in range(3)]
    say("  dt", max(abs(a / b - 1) for a, b in zip(dtg, dtr)), "P", eP.max(), "U", eU.max(),
        "faces", eB)
    assert max(abs(a / b - 1) for a, b in zip(dtg, dtr)) < 1e-13
    assert eP.max() < 2e-12 and eU.max() < 2e-12 and max(eB) < 2e-12
    assert max(np.abs(Br[p][ev[p]] - Bf[p][ev[p]]).max() for p in range(3)) > 0
    if case == "box3d":
        scale = np.abs(Bf).max() / 0.1
        d0 = np.abs(_div(pd, Bf)).max() / scale
        d2 = np.abs(_div(pd, Bg)).max() / scale
        say("  divergence / (max|Bf|/dx): initial", d0, "after 2 GPU steps", d2)
        assert d0 < 1e-14 and d2 < 1e-13


def test_staggered_imex3_fixed_dt(G, orc):
    """IMEX3 with dt given: its first two stages evaluate no flux at all, so
    their faces come from Bf^n alone (the EMF buffer is not read before the
    third stage writes it)."""
    say("case box3d imex3 staggered, dt fixed")
    pd, P, U, ca, ce, Bf = _prepared(orc, "box3d")
    pd = dict(pd, scheme="imex3")
    dtv = 0.7 * orc.step_stag(pd, P, U, Bf, ca, ce)[3]
    Pr, Ur, Br, dt, st, it, nbad = orc.step_stag(pd, P, U, Bf, ca, ce, dt=dtv, dt_fixed=True)
    gr = G.Grid(pd)
    Pt, Ut, Bt = dev(P), dev(U), dev(Bf)
    dtt = torch.full((1,), dtv, dtype=torch.float64, device="cuda")
    gr.step_staggered(Pt, Ut, Bt, dev(ca), dev(ce), dtt, dt_fixed=True)
    Pg, Ug, Bg = host(Pt), host(Ut), host(Bt)
    gr.close()
    m = interior_mask(pd)
    ev = _evolved(pd)
    eP, eU = field_err(Pg, Pr, m), field_err(Ug, Ur, m)
    eB = [_face_err(Bg[p], Br[p], ev[p]) for p in range(3)]
    say("  P", eP.max(), "U", eU.max(), "faces", eB)
    assert np.all(np.isfinite(Bg)) and eP.max() < 1e-12 and eU.max() < 1e-12 and max(eB) < 1e-12


def test_staggered_ppm_and_cascade(G, orc):
    """PPM reconstruction (the flattener two cells out is zero on both sides)
    and the full implicit cascade with its entropy tracer, on the 3-D disk."""
    say("case disk3d ppm + cascade, staggered")
    pd, P, ca, ce, Bf = _disk((20, 12, 8), ng=4, recon="ppm", cascade=1)
    Bf = orc.bc_face(pd, Bf)
    P, U = _consistent(orc, pd, P, Bf)
    Pr, Ur, Br, dt, st, it, nbad = orc.step_stag(pd, P, U, Bf, ca, ce)
    Pg, Ug, Bg, dtg, _ = _gpu_steps(G, pd, P, U, Bf, ca, ce, 1)
    m = interior_mask(pd)
    ev = _evolved(pd)
    eP, eU = field_err(Pg, Pr, m), field_err(Ug, Ur, m)
    eB = [_face_err(Bg[p], Br[p], ev[p]) for p in range(3)]
    say("  P", eP.max(), "U", eU.max(), "faces", eB)
    assert abs(dtg[0] / dt - 1) < 1e-13
    assert eP.max() < 1e-12 and eU.max() < 1e-12 and max(eB) < 1e-12


def test_staggered_ppm_cascade_imex3(G, orc):
    """Every option of the step at once on the 3-D disk: the staggered
    field, PPM with the flattener, the full cascade with its entropy tracer
    and the IMEX3 table (stored sources, the tracer's stored sources, the
    stage faces, the final explicit inversion): one step against the
    oracle's."""
    say("case disk3d ppm + cascade + imex3, staggered")
    pd, P, ca, ce, Bf = _disk((20, 12, 8), ng=4, recon="ppm", cascade=1, scheme="imex3")
    Bf = orc.bc_face(pd, Bf)
    P, U = _consistent(orc, pd, P, Bf)
    Pr, Ur, Br, dt, st, it, nbad = orc.step_stag(pd, P, U, Bf, ca, ce)
    Pg, Ug, Bg, dtg, stg = _gpu_steps(G, pd, P, U, Bf, ca, ce, 1, status=True)
    m = interior_mask(pd)
    ev = _evolved(pd)
    eP, eU = field_err(Pg, Pr, m), field_err(Ug, Ur, m)
    eB = [_face_err(Bg[p], Br[p], ev[p]) for p in range(3)]
    say("  P", eP.max(), "U", eU.max(), "faces", eB, "failed", nbad)
    assert np.array_equal(stg[m], st[m])
    assert abs(dtg[0] / dt - 1) < 1e-13
    assert eP.max() < 1e-12 and eU.max() < 1e-12 and max(eB) < 1e-12


def test_staggered_mixed_precision(G, orc):
    say("case disk3d mixed, staggered")
    pd, P, ca, ce, Bf = _disk((24, 12, 8), precision="mixed", r_fp64=2.0)
    Bf = orc.bc_face(pd, Bf)
    P, U = _consistent(orc, pd, P, Bf)
    Pr, Ur, Br = P, U, Bf
    for _ in range(3):
        Pr, Ur, Br, dt, st, it, nbad = orc.step_stag(dict(pd, precision="fp64"), Pr, Ur, Br, ca, ce)
    Pg, Ug, Bg, dtg, _ = _gpu_steps(G, pd, P, U, Bf, ca, ce, 3)
    m = interior_mask(pd)
    ev = _evolved(pd)
    eP = field_err(Pg, Pr, m)
    eB = [_face_err(Bg[p], Br[p], ev[p]) for p in range(3)]
    say("  P", eP.max(), "faces", eB)
    assert eP.max() < 1e-5 and max(eB) < 1e-5


def test_full_size_disk_keeps_the_divergence(G, orc):
    """The 128x64x32 Kerr-Schild disk with the staggered field: one GPU step
    against the oracle's at every interior cell and evolved face, and the
    discrete divergence of the GPU's faces after three steps still at its
    initial round-off level."""
    say("case disk3d full size, staggered")
    pd, P, ca, ce, Bf = _disk((128, 64, 32))
    Bf = orc.bc_face(pd, Bf)
    P, U = _consistent(orc, pd, P, Bf)
    Pr, Ur, Br, dt, st, it, nbad = orc.step_stag(pd, P, U, Bf, ca, ce)
    Pg, Ug, Bg, dtg, _ = _gpu_steps(G, pd, P, U, Bf, ca, ce, 1)
    m = interior_mask(pd)
    ev = _evolved(pd)
    eP, eU = field_err(Pg, Pr, m), field_err(Ug, Ur, m)
    eB = [_face_err(Bg[p], Br[p], ev[p]) for p in range(3)]
    say("  P", eP.max(), "U", eU.max(), "faces", eB)
    assert eP.max() < 1e-12 and eU.max() < 1e-12 and max(eB) < 1e-12
    dx = min((pd["xhi"][d] - pd["xlo"][d]) / pd["n"][d] for d in range(3))
    scale = np.abs(Bf).max() / dx
    d0 = np.abs(_div(pd, Bf)).max() / scale
    Pg, Ug, Bg, dtg, _ = _gpu_steps(G, pd, P, U, Bf, ca, ce, 3)
    d3 = np.abs(_div(pd, Bg)).max() / scale
    say("  divergence / (max|Bf|/dx): initial", d0, "after 3 GPU steps", d3)
    assert d0 < 1e-14 and d3 < 1e-13


def test_staggered_entry_points_check_the_grid(G):
    pd, P, ca, ce, Bf = _disk((24, 12, 8))
    flux_pd = dict(pd, ct="flux")
    gf = G.Grid(flux_pd)
    gs = G.Grid(pd)
    dtt = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    Pt, Ut, Bt = dev(P), dev(np.zeros_like(P)), dev(Bf)
    with pytest.raises(RuntimeError, match="flux-CT"):
        gf.step_staggered(Pt, Ut, Bt, dev(ca), dev(ce), dtt)
    with pytest.raises(RuntimeError, match="staggered"):
        gs.step(Pt, Ut, dev(ca), dev(ce), dtt)
    with pytest.raises(RuntimeError, match="ct"):
        gs.step_adjoint(Pt, dev(ca), dev(ce), dtt, dev(np.ones_like(P)))
    with pytest.raises(RuntimeError, match="flux-CT"):
        gs.fixup_vjp(Pt, torch.zeros(gs.N, dtype=torch.int32, device="cuda"), Pt.clone(), Pt.clone())
    gi = G.Grid(dict(pd, scheme="imex3"))
    with pytest.raises(RuntimeError, match="ct"):
        gi.step_adjoint(Pt, dev(ca), dev(ce), dtt, dev(np.ones_like(P)))
    gi.close()
    gf.close()
    gs.close()
