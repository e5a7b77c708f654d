"""GPU (HIP, through the C ABI) vs FP64 CPU oracle, element by element.

Tolerance: 1e-12 relative per field (max over cells of |gpu - oracle| over
max over cells of |oracle|), or tighter where the arithmetic allows; bit-exact
for the ghost fill.  Floating-point decisions that set integer results
(status bits) are compared where both sides converged.
"""
import math
import sys

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    from paper_1312_6127_amd import grrmhd

    grrmhd.lib()
    assert torch.cuda.is_available()
    return grrmhd


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


GROUPS = [(0,), (1,), (2, 3, 4), (5, 6, 7), (8,), (9, 10, 11)]


def field_err(a, b, mask=None):
    """Per-field relative error max|a - b| / scale, the scale being the max of
    |b| over the cells and, for the three components of a vector (velocity,
    field, momentum), over the vector's components; absolute when the scale
    is zero.  Arrays with 12 rows use the state's vector groups."""
    out = np.zeros(a.shape[0])
    groups = GROUPS if a.shape[0] == 12 else [(q,) for q in range(a.shape[0])]
    for grp in groups:
        ys = [b[q][mask] if mask is not None else b[q] for q in grp]
        s = max((np.abs(y).max() if y.size else 0.0) for y in ys)
        for q in grp:
            x = a[q][mask] if mask is not None else a[q]
            y = b[q][mask] if mask is not None else b[q]
            d = np.abs(x - y).max() if y.size else 0.0
            out[q] = d / s if s > 0 else d
    return out


def interior_mask(pd):
    m = np.zeros(I.nalloc(pd)[::-1], dtype=bool)
    m[I.interior(pd)] = True
    return m.reshape(-1)


CASES = {
    "tube1d": lambda: I.shock_tube_1d(200),
    "disk2d": lambda: I.accretion_disk(n=(40, 24, 1), seed=2),
    "disk3d": lambda: I.accretion_disk(n=(24, 12, 8), seed=3),
    "disk3d_hll": lambda: I.accretion_disk(n=(20, 10, 6), seed=5, flux="hll"),
}


def _periodic3d():
    from test_oracle_pins import _periodic_box

    return _periodic_box((12, 10, 6), seed=7)


CASES["box3d"] = _periodic3d


@pytest.mark.parametrize("case", sorted(CASES))
def test_prim_to_cons_and_bc(G, orc, case):
    say("case", case, "prim_to_cons/bc")
    pd, P, ca, ce = CASES[case]()
    g = G.Grid(pd)
    Pt = dev(P)
    U = host(g.prim_to_cons(Pt))
    Ur = orc.prim_to_cons(pd, P)
    assert field_err(U, Ur).max() < 1e-13
    Pb = host(g.apply_bc(Pt.clone()))
    Pbr = orc.bc(pd, P)
    assert np.array_equal(Pb, Pbr)
    g.close()


@pytest.mark.parametrize("case", sorted(CASES))
def test_fluxes_timestep_update(G, orc, case):
    say("case", case, "fluxes/timestep/update")
    pd, P, ca, ce = CASES[case]()
    P = orc.bc(pd, P)
    g = G.Grid(pd)
    Pt, cat, cet = dev(P), dev(ca), dev(ce)
    F, emf, vch = g.fluxes(Pt, cat, cet)
    Fr, emfr, vchr = orc.fluxes(pd, P, ca, ce)
    F, emf, vch = host(F), host(emf), host(vch)
    for d in range(3):
        assert field_err(F[d], Fr[d]).max() < 1e-12, d
    assert field_err(emf, emfr).max() < 1e-12
    assert field_err(vch, vchr).max() < 1e-13
    dt = g.timestep(dev(vchr))
    dtr = orc.timestep(pd, vchr)
    assert abs(host(dt)[0] / dtr - 1) < 1e-14
    U = orc.prim_to_cons(pd, P)
    Uprev = U * (1 + 1e-3 * np.sin(np.arange(U.size)).reshape(U.shape))
    for (a, b, c) in [(1.0, 0.0, 1.0), (0.75, 0.25, 0.25), (1 / 3, 2 / 3, 2 / 3)]:
        Ue = host(g.explicit_update(a, b, c, dt, Pt, dev(U), dev(Uprev), dev(Fr), dev(emfr)))
        Uer = orc.explicit_update(pd, a, b, c, dtr, P, U, Uprev, Fr, emfr)
        m = interior_mask(pd)
        assert field_err(Ue, Uer, m).max() < 1e-12, (a, b, c, field_err(Ue, Uer, m))
    g.close()


@pytest.mark.parametrize("case", sorted(CASES))
def test_con2prim(G, orc, case):
    say("case", case, "con2prim")
    pd, P, ca, ce = CASES[case]()
    g = G.Grid(pd)
    U = orc.prim_to_cons(pd, P)
    Pg = P * (1 + 1e-2 * np.cos(np.arange(P.size)).reshape(P.shape))
    Pgpu, st = g.con2prim(dev(U), dev(Pg))
    Pr, str_ = orc.con2prim(pd, U, Pg)
    m = interior_mask(pd)
    assert np.array_equal(host(st)[m] & G.ST_C2P_FAIL, str_[m] & orc.ST_C2P_FAIL)
    assert field_err(host(Pgpu), Pr, m).max() < 1e-11
    g.close()


def _explicit_state(orc, pd, P, ca, ce):
    """U_(i) of stage 1 from the oracle (inputs identical on both sides)."""
    Pb = orc.bc(pd, P)
    F, emf, vch = orc.fluxes(pd, Pb, ca, ce)
    dt = orc.timestep(pd, vch)
    U = orc.prim_to_cons(pd, Pb)
    Ue = orc.explicit_update(pd, 1.0, 0.0, 1.0, dt, Pb, U, U, F, emf)
    return Pb, Ue, dt


@pytest.mark.parametrize("case", sorted(CASES))
def test_implicit_grid(G, orc, case):
    say("case", case, "implicit")
    pd, P, ca, ce = CASES[case]()
    Pb, Ue, dt = _explicit_state(orc, pd, P, ca, ce)
    g = G.Grid(pd)
    dtt = dev(np.array([dt]))
    Pg, Ug, itg, stg, errg = g.implicit(dev(Ue), dev(Pb), 1.0, dtt, dev(ca), dev(ce))
    Pr, Ur, itr, str_ = orc.implicit_grid(pd, Ue, Pb, dt, ca, ce)
    Pg, Ug, stg, errg = host(Pg), host(Ug), host(stg), host(errg)
    m = interior_mask(pd)
    # unique: whether a cell has a solution; not unique: which method found
    # it when both PMHD and URAD reach round-off (each is then checked valid)
    assert np.array_equal(stg[m] & orc.ST_FAIL, str_[m] & orc.ST_FAIL)
    ok = (str_[m] & orc.ST_FAIL) == 0
    assert np.all(((stg[m] & (orc.ST_PMHD | orc.ST_URAD)) != 0) | ~ok)
    good = m.copy()
    good[m] = ok & (errg[m] < 1e-12)
    assert good.sum() > 0.95 * m.sum()
    assert field_err(Pg, Pr, good).max() < 1e-12, field_err(Pg, Pr, good)
    assert field_err(Ug, Ur, good).max() < 1e-12, field_err(Ug, Ur, good)
    g.close()


@pytest.mark.parametrize("case", sorted(CASES))
def test_full_step(G, orc, case):
    say("case", case, "step")
    pd, P, ca, ce = CASES[case]()
    U = orc.prim_to_cons(pd, P)
    P1, U1, dt, st, it, nbad = orc.step(pd, P, U, ca, ce)
    g = G.Grid(pd)
    Pt, Ut = dev(P), dev(U)
    dtt = torch.zeros(1, dtype=torch.float64, device="cuda")
    stt = torch.zeros(g.N, dtype=torch.int32, device="cuda")
    itt = torch.zeros(g.N, dtype=torch.int32, device="cuda")
    g.step(Pt, Ut, dev(ca), dev(ce), dtt, status=stt, iters=itt)
    m = interior_mask(pd)
    assert abs(host(dtt)[0] / dt - 1) < 1e-14
    eP = field_err(host(Pt), P1, m)
    eU = field_err(host(Ut), U1, m)
    say("  step field errors P", eP.max(), "U", eU.max())
    assert eP.max() < 1e-12 and eU.max() < 1e-12, (eP, eU)
    assert np.array_equal(host(stt)[m] & orc.ST_FAIL, st[m] & orc.ST_FAIL)
    g.close()


def check_disagreeing(orc, pd, cells, Pg, stg, errg, Ui, dt, ca, ce, str_):
    """Cells where GPU and oracle disagree on the kind of solution (energy,
    cold, none): every GPU solution among them must satisfy its implicit
    equations, written out independently for flat space, to tol_fail (the
    energy-momentum exchange for an energy solution, the gas momentum
    equations for a cold one); cells whose radiation a limiter altered
    (TYPE2, BASIC) are counted apart.  Returns the counts."""
    from test_oracle_pins import _mink_momentum_residual, _mink_residual

    n = dict(gpu_energy=0, gpu_cold=0, gpu_none=0, limited=0, worst=0.0)
    for c in cells:
        s = int(stg[c])
        if s & orc.ST_FAIL:
            n["gpu_none"] += 1
            continue
        if s & (orc.ST_TYPE2_NEG | orc.ST_BASIC):
            n["limited"] += 1
            continue
        ka, ke = ca[c] * Pg[0, c], ce[c] * Pg[0, c]
        if s & orc.ST_COLD:
            r = _mink_momentum_residual(pd, Pg[:, c], Ui[:, c], dt[c], ka, ke)
            n["gpu_cold"] += 1
        else:
            r = max(_mink_residual(pd, Pg[:, c], Ui[:, c], dt[c], ka, ke))
            n["gpu_energy"] += 1
        n["worst"] = max(n["worst"], r)
        assert r <= pd["tol_fail"], (c, r, s, int(str_[c]), errg[c])
    return n


def test_implicit_batch(G, orc):
    say("case batch implicit")
    n = 3001
    pd, P, dt, ca, ce = I.implicit_batch(n, seed=4)
    g0 = orc.geom(pd, 0.0, 0.0)
    U = np.stack([orc.p2u(pd, g0, P[:, c]) for c in range(n)], axis=1)
    Ui = U.copy()
    Ui[8] *= 1.3
    Ui[1] -= 0.3 * U[8]
    Pr, Ur, itr, str_ = orc.implicit_batch(pd, Ui, P, dt, ca, ce)
    Pg, Ug, itg, stg, errg = G.implicit_source(pd, dev(Ui), dev(P), dev(dt), dev(ca), dev(ce))
    Pg, Ug, stg, errg = host(Pg), host(Ug), host(stg), host(errg)
    # whether a cell has an energy solution, a cold one or none: decided the
    # same way on both sides except near the edge of a root's existence,
    # where the two Newton iterations (exact and difference Jacobians) can
    # end on either side of it
    kind = orc.ST_FAIL | orc.ST_COLD
    fail_agree = (stg & kind) == (str_ & kind)
    assert fail_agree.mean() > 0.98
    cnt = check_disagreeing(orc, pd, np.nonzero(~fail_agree)[0], Pg, stg, errg, Ui, dt, ca, ce, str_)
    say(f"  kinds disagree on {(~fail_agree).sum()} of {n} cells: {cnt}")
    # both sides accept a method within 10 tol_pmhd (1e-11) when iterating to round-off
    good = fail_agree & ((str_ & orc.ST_FAIL) == 0) & (errg < 1e-11)
    assert good.sum() > 0.6 * n
    # per cell, conserved quantities against the cell's own energy scale
    scale = np.abs(Ur[1]) + np.abs(Ur[8]) + np.abs(Ur[2:5]).sum(0) + np.abs(Ur[9:12]).sum(0)
    d = np.abs(Ug - Ur)[1:12, good].max(axis=0) / scale[good]
    assert d.max() < 1e-12, d.max()
    # primitives per cell.  Where the two sides accept different methods
    # (both within tolerance) the fluid-frame energies agree against the
    # cell's total fluid-frame energy u_g + Ebar (the exchange conserves it),
    # not against Ebar alone, which is ill-conditioned in radiation-sub-
    # dominant cells; the radiation frame velocity is covered by R^t_i above.
    eng = np.abs(Pr[1, good]) + np.abs(Pr[8, good])
    # cold cells: the gas velocity (and rho0 = D/u^t) comes from a momentum
    # balance in which the gas is a small part of a radiation-dominated cell
    tv = np.where((str_[good] & orc.ST_COLD) != 0, 1e-10, 1e-12)
    assert np.all(np.abs(Pg[0, good] - Pr[0, good]) / Pr[0, good] < tv)
    for q in (1, 8):
        assert (np.abs(Pg[q, good] - Pr[q, good]) / eng).max() < 1e-10, q
    gsc = 1.0 + np.abs(Pr[2:5, good]).sum(0)
    assert np.all(np.abs(Pg[2:5, good] - Pr[2:5, good]).max(0) / gsc < tv)


def test_full_size_disk_step(G, orc):
    """The 128x64x32 Kerr-Schild step in the benchmark's launch configuration,
    compared at every interior cell."""
    say("case disk3d full size")
    pd, P, ca, ce = I.accretion_disk(n=(128, 64, 32), seed=3)
    U = orc.prim_to_cons(pd, P)
    P1, U1, dt, st, it, nbad = orc.step(pd, P, U, ca, ce)
    g = G.Grid(pd)
    Pt, Ut = dev(P), dev(U)
    dtt = torch.zeros(1, dtype=torch.float64, device="cuda")
    g.step(Pt, Ut, dev(ca), dev(ce), dtt)
    m = interior_mask(pd)
    eP = field_err(host(Pt), P1, m)
    eU = field_err(host(Ut), U1, m)
    say("  full-size field errors P", eP, "U", eU)
    assert eP.max() < 1e-12 and eU.max() < 1e-12
    g.close()


def _batch_cons(orc, pd, P):
    """Explicit state of a batch: the primitives' conserved form with the
    radiation energy raised 30% and the gas energy lowered to match."""
    g0 = orc.geom(pd, 0.0, 0.0)
    U = np.stack([orc.p2u(pd, g0, P[:, c]) for c in range(P.shape[1])], axis=1)
    Ui = U.copy()
    Ui[8] *= 1.3
    Ui[1] -= 0.3 * U[8]
    return Ui


FORMS = {"per_iteration": (1, 64, 0), "persistent64": (2, 64, 8), "persistent256": (2, 256, 16)}


@pytest.mark.parametrize("form", sorted(FORMS))
def test_implicit_batch_forms_identical(G, orc, form):
    """The per-iteration and persistent forms take the same decisions per
    cell as the per-cell form: identical bits in every output."""
    say("case batch forms", form)
    n = 5003
    pd, P, dt, ca, ce = I.implicit_batch(n, seed=6)
    args = [dev(_batch_cons(orc, pd, P)), dev(P), dev(dt), dev(ca), dev(ce)]
    ws0 = G.batch_workspace(n, G.PER_CELL)
    ref = [host(x) for x in G.implicit_source_ex(pd, *args, G.PER_CELL, 64, 1, ws=ws0)]
    s0 = G.batch_stats(ws0)
    mode, block, wpc = FORMS[form]
    ws = G.batch_workspace(n, mode)
    got = [host(x) for x in G.implicit_source_ex(pd, *args, mode, block, wpc, ws=ws)]
    for a, b in zip(got, ref):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    # same Newton trips and cascade cells; lane slots cover the trips
    s1 = G.batch_stats(ws)
    say("  stats per-cell", s0, form, s1)
    assert s1[0] == s0[0] and s1[2] == s0[2]
    # the compacted cascade: the same residual evaluations whatever the
    # order lanes took the cells in
    c0, c1 = G.batch_cascade_stats(ws0), G.batch_cascade_stats(ws)
    say("  cascade evaluations, lane slots", c0, c1)
    assert c0[0] == c1[0] and 0 < c0[0] <= c0[1] and c1[0] <= c1[1]
    assert s0[0] <= s0[1] and s1[0] <= s1[1]
    # every non-extreme cell takes between 1 and max_iter + 1 trips
    st = ref[3]
    nonext = int(((st & G.ST_EXTREME) == 0).sum())
    assert nonext <= s0[0] <= (pd["max_iter"] + 1) * nonext


def test_implicit_batch_autotune_and_reuse(G, orc):
    """The autotuner returns one of its candidates with outputs equal to the
    per-cell form's; the chosen form then reproduces the per-cell results on
    a smaller batch with the same workspace."""
    say("case batch autotune")
    n = 20000
    pd, P, dt, ca, ce = I.implicit_batch(n, seed=8)
    Ui = _batch_cons(orc, pd, P)
    args = [dev(Ui), dev(P), dev(dt), dev(ca), dev(ce)]
    t, allt, outs = G.autotune_implicit_source(pd, *args)
    say("  tuned", t.mode, t.block, t.waves_per_cu, t.ms)
    assert t.ms > 0 and min(a.ms for a in allt) == t.ms
    assert (t.mode, t.block, t.waves_per_cu) in [(a.mode, a.block, a.waves_per_cu) for a in allt]
    ref = [host(x) for x in G.implicit_source(pd, *args)]
    for a, b in zip([host(x) for x in outs], ref):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    ws = G.batch_workspace(n, t.mode)
    m = n // 3
    args = [dev(Ui[:, :m]), dev(P[:, :m]), dev(dt[:m]), dev(ca[:m]), dev(ce[:m])]
    got = [host(x) for x in G.implicit_source_ex(pd, *args, t.mode, t.block, max(t.waves_per_cu, 1),
                                                  ws=ws)]
    ref2 = [host(x) for x in G.implicit_source(pd, *args)]
    for a, b in zip(got, ref2):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def _gpu_steps(G, pd, P, ca, ce, nsteps):
    g = G.Grid(pd)
    Pt = dev(P)
    Ut = g.prim_to_cons(Pt)
    dtt = torch.zeros(1, dtype=torch.float64, device="cuda")
    stt = torch.zeros(g.N, dtype=torch.int32, device="cuda")
    cat, cet = dev(ca), dev(ce)
    for _ in range(nsteps):
        g.step(Pt, Ut, cat, cet, dtt, status=stt)
    out = host(Pt), host(Ut), host(dtt)[0], host(stt)
    g.close()
    return out


@pytest.mark.parametrize("case", ["tube1d", "disk3d", "disk3d_hll"])
def test_mixed_precision_step(G, orc, case):
    """FP32 reconstruction / face states / Riemann fluxes / EMFs with FP64
    state, update, inversions and implicit solve: per-field error against
    the FP64 oracle after 3 steps stays below the stated mixed bound 1e-5."""
    say("case", case, "mixed precision")
    pd, P, ca, ce = CASES[case]()
    U = orc.prim_to_cons(pd, P)
    Pr, Ur = P, U
    for _ in range(3):
        Pr, Ur, dtr, str_, itr, nb = orc.step(pd, Pr, Ur, ca, ce)
    m = interior_mask(pd)
    P64, U64, dt64, _ = _gpu_steps(G, pd, P, ca, ce, 3)
    Pmx, Umx, dtmx, _ = _gpu_steps(G, dict(pd, precision="mixed"), P, ca, ce, 3)
    e64 = max(field_err(P64, Pr, m).max(), field_err(U64, Ur, m).max())
    eP, eU = field_err(Pmx, Pr, m), field_err(Umx, Ur, m)
    say("  fp64", e64, "mixed P", eP.max(), "U", eU.max(), "dt", abs(dtmx / dtr - 1))
    assert e64 < 1e-12
    assert abs(dtmx / dtr - 1) < 1e-5
    assert eP.max() < 1e-5 and eU.max() < 1e-5, (eP, eU)
    # FP32 really ran: the mixed result differs from the FP64 one
    assert field_err(Umx, U64, m).max() > 1e-12


def test_mixed_precision_fp64_region(G):
    """With r_fp64 beyond the outer radius every face and edge keeps the FP64
    path: bit-identical to precision = fp64."""
    say("case mixed with all-FP64 region")
    pd, P, ca, ce = CASES["disk3d"]()
    a = _gpu_steps(G, pd, P, ca, ce, 1)
    b = _gpu_steps(G, dict(pd, precision="mixed", r_fp64=1e6), P, ca, ce, 1)
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("case", ["tube1d", "disk3d"])
def test_mixed_precision_radiation_at_the_floor(G, orc, case):
    """Cells whose radiation sits at the 1e-150 floor (below FP32's range, so
    their face radiation energy flushes to zero in the FP32 path): the mixed
    step stays finite, keeps Ebar at or above the floor, and meets the mixed
    bound against the FP64 oracle."""
    say("case", case, "mixed precision, radiation at the floor")
    pd, P, ca, ce = CASES[case]()
    x1 = I.cell_coords(pd)[0].reshape(-1)
    low = x1 > np.median(x1)
    P = P.copy()
    P[8, low] = pd["erad_floor"]
    P[9:12, low] = P[2:5, low]
    U = orc.prim_to_cons(pd, P)
    Pr, Ur = P, U
    for _ in range(3):
        Pr, Ur, dtr, str_, itr, nb = orc.step(pd, Pr, Ur, ca, ce)
    m = interior_mask(pd)
    Pmx, Umx, dtmx, stmx = _gpu_steps(G, dict(pd, precision="mixed"), P, ca, ce, 3)
    assert np.all(np.isfinite(Pmx[:, m])) and np.all(np.isfinite(Umx[:, m]))
    assert Pmx[8, m].min() >= pd["erad_floor"]
    eP, eU = field_err(Pmx, Pr, m), field_err(Umx, Ur, m)
    say("  mixed P", eP.max(), "U", eU.max(), "floor cells", int((low & m).sum()))
    assert eP.max() < 1e-5 and eU.max() < 1e-5, (eP, eU)
    assert np.array_equal(stmx[m] & orc.ST_FAIL, str_[m] & orc.ST_FAIL)


def test_radiation_front_into_floor_cells(G, orc):
    """The shock tube with its right half at the radiation floor (1e-150):
    the gas there emits radiation twenty orders of magnitude above the floor
    within one step, and the left state's radiation streams in, in cells
    whose radiation is extremely sub-dominant (URAD first).  Both sides solve
    every cell; the conserved state agrees to 1e-12 of each cell's energy
    scale, and every GPU solution satisfies the implicit equations, written
    out independently for flat space, to 1e-12."""
    say("case radiation front into floor cells")
    pd, P, ca, ce = CASES["tube1d"]()
    x1 = I.cell_coords(pd)[0].reshape(-1)
    P = P.copy()
    P[8, x1 > 0.0] = pd["erad_floor"]
    Pb, Ue, dt = _explicit_state(orc, pd, P, ca, ce)
    g = G.Grid(pd)
    Pg, Ug, itg, stg, errg = g.implicit(dev(Ue), dev(Pb), 1.0, dev(np.array([dt])), dev(ca), dev(ce))
    Pr, Ur, itr, str_ = orc.implicit_grid(pd, Ue, Pb, dt, ca, ce)
    Pg, Ug, stg, errg = host(Pg), host(Ug), host(stg), host(errg)
    g.close()
    m = interior_mask(pd)
    ext = m & ((stg & orc.ST_EXTREME) != 0)
    assert ext.sum() == (m & (x1 > 0)).sum()
    assert np.all((stg[m] & orc.ST_FAIL) == 0) and np.all((str_[m] & orc.ST_FAIL) == 0)
    from test_oracle_pins import _mink_residual

    worst = 0.0
    for c in np.nonzero(m)[0]:
        if stg[c] & (orc.ST_TYPE2_NEG | orc.ST_BASIC):
            continue
        rg, rr = _mink_residual(pd, Pg[:, c], Ue[:, c], dt, ca[c] * Pg[0, c], ce[c] * Pg[0, c])
        worst = max(worst, rg, rr)
    scale = np.abs(Ur[1]) + np.abs(Ur[8]) + np.abs(Ur[2:5]).sum(0) + np.abs(Ur[9:12]).sum(0)
    d = (np.abs(Ug - Ur)[1:12].max(axis=0) / scale)[m]
    say(f"  extreme cells {int(ext.sum())}, worst residual {worst:.2e}, max |dU|/cell scale {d.max():.2e}")
    assert worst < 1e-12 and d.max() < 1e-12
