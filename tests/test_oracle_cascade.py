"""Pins of the oracle's full implicit cascade (Sec. 4.7-4.11): PRAD, the
staged Newton approach and the entropy-based methods, against what the
equations fix rather than against the oracle itself:

- PRAD reaches the same root as PMHD where both converge (the method changes
  the iterated quantities, not the equations);
- cells where every undamped attempt stalls are solved by the staged
  approach, and its solutions satisfy the implicit equations written out
  independently for flat space;
- entropy-method solutions satisfy the entropy equation eq. source6 with
  G_S = -G^mu u_mu / T_gas (eq. GS), written out independently, together
  with the gas momentum equations and total energy-momentum conservation;
- for a small exchange the entropy and energy roots agree to second order in
  the exchange (T dS = du at fixed density), so a wrong sign or factor in
  G_S fails;
- the full cascade leaves far fewer batch cells without a solution than
  PMHD and URAD alone, and changes nothing where PMHD is accepted;
- in the IMEX tables (Sec. 4.1) the entropy tracer's bracket carries the
  stored entropy sources: nothing changes where PMHD is accepted, and on a
  box of far-from-equilibrium cells the entropy methods take cells the
  energy methods leave.
"""
import math

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I

from test_oracle_pins import _mink_momentum_residual, _mink_residual  # noqa: E402


def _batch(orc, n, seed):
    pd, P, dt, ca, ce = I.implicit_batch(n, seed=seed)
    g = orc.geom(pd, 0.0, 0.0)
    U = np.stack([orc.p2u(pd, g, P[:, c]) for c in range(n)], axis=1)
    Ui = U.copy()
    Ui[8] *= 1.3
    Ui[1] -= 0.3 * U[8]
    return pd, g, P, dt, ca, ce, Ui


def _si(orc, pd, P):
    """sqrt(-g) S u^t of a flat-space cell's primitives."""
    return orc.entropy(pd, P) * math.sqrt(1.0 + P[2:5] @ P[2:5])


def _limited(orc, st):
    return st & (orc.ST_TYPE2_NEG | orc.ST_BASIC | orc.ST_FAIL)


def test_prad_reaches_the_pmhd_root(orc):
    pd, g, P, dt, ca, ce, Ui = _batch(orc, 600, 21)
    both, worst = 0, 0.0
    for c in range(P.shape[1]):
        Si = _si(orc, pd, P[:, c])
        a = orc.implicit_attempt(pd, g, Ui[:, c], Si, P[:, c], dt[c], ca[c], ce[c], "pmhd")
        b = orc.implicit_attempt(pd, g, Ui[:, c], Si, P[:, c], dt[c], ca[c], ce[c], "prad")
        if a[4] < 1e-11 and b[4] < 1e-11 and not _limited(orc, a[2]) and not _limited(orc, b[2]):
            both += 1
            assert b[2] & orc.ST_PRAD
            scale = np.abs(a[1][1:5]).sum() + np.abs(a[1][8:12]).sum()
            worst = max(worst, np.abs(a[1] - b[1])[1:12].max() / scale)
    assert both > 50 and worst < 1e-13, (both, worst)


def test_staged_newton_solves_cells_where_undamped_attempts_stall(orc):
    pd, g, P, dt, ca, ce, Ui = _batch(orc, 600, 21)
    rescued, worst = 0, 0.0
    for c in range(P.shape[1]):
        Si = _si(orc, pd, P[:, c])
        normal = [orc.implicit_attempt(pd, g, Ui[:, c], Si, P[:, c], dt[c], ca[c], ce[c], m)
                  for m in ("pmhd", "urad", "prad")]
        if min(x[4] for x in normal) <= pd["tol_fail"]:
            continue
        staged = [orc.implicit_attempt(pd, g, Ui[:, c], Si, P[:, c], dt[c], ca[c], ce[c], m,
                                       staged=True) for m in ("pmhd", "urad", "prad")]
        best = min(staged, key=lambda x: x[4])
        if best[4] < pd["tol_accept"] and not _limited(orc, best[2]):
            rescued += 1
            Po = best[0]
            r = max(_mink_residual(pd, Po, Ui[:, c], dt[c], ca[c] * Po[0], ce[c] * Po[0]))
            worst = max(worst, r / (1e-13 + 10.0 * best[4]))
    assert rescued >= 10 and worst <= 1.0, (rescued, worst)


def _entropy_residual(pd, P, Ui, Si, dt, ka, ke):
    """T_gas (S u^t - S_i) + dt G^mu u_mu for flat-space primitives P, written
    out here: S = rho0 ln(p^n / rho0^(n+1)), G^mu from its gas-frame
    components as in _mink_residual; normalised by its own terms plus the
    gas energy scale."""
    gam = pd["gam"]
    eta = np.diag([-1.0, 1, 1, 1])
    rho, ug = P[0], P[1]
    pg = (gam - 1) * ug
    n = 1.0 / (gam - 1)
    S = rho * math.log(pg ** n / rho ** (n + 1))
    u = np.concatenate([[math.sqrt(1 + P[2:5] @ P[2:5])], P[2:5]])
    ur = np.concatenate([[math.sqrt(1 + P[9:12] @ P[9:12])], P[9:12]])
    Rup = P[8] * (4.0 / 3.0 * np.outer(ur, ur) + eta / 3.0)
    ucov = eta @ u
    Ehat = ucov @ Rup @ ucov
    Fvec = -(Rup @ ucov) - Ehat * u
    T = pg / rho
    lam = ka * pd["arad"] * T ** 4
    Gup = (ka * Ehat - lam) * u + (ka + ke) * Fvec
    Gu = Gup @ ucov
    res = T * (S * u[0] - Si) + dt * Gu
    Tup = (rho + ug + pg) * np.outer(u, u) + pg * eta
    Etot = abs(Tup[0] @ eta)[0] + abs(Ui[1])
    return abs(res) / (abs(T * S * u[0]) + abs(T * Si) + dt * abs(Gu) + Etot)


def test_entropy_solutions_satisfy_the_entropy_equation(orc):
    """The entropy-based PMHD and URAD attempts: the independently written
    entropy residual and gas momentum residual within 10 e_T, and gas plus
    radiation energy-momentum equal to the explicit state's (the energy
    equation is dropped, not total conservation)."""
    pd, g, P, dt, ca, ce, Ui = _batch(orc, 300, 23)
    checked, worst, cons = 0, 0.0, 0.0
    for c in range(P.shape[1]):
        Si = _si(orc, pd, P[:, c]) * 1.001     # an explicit entropy a little off the guess's
        for m in ("pmhd", "urad"):
            Po, Uo, st, it, err = orc.implicit_attempt(pd, g, Ui[:, c], Si, P[:, c], dt[c], ca[c],
                                                       ce[c], m, entropy=True)
            if err > 1e-11 or _limited(orc, st):
                continue
            assert st & orc.ST_ENTROPY
            checked += 1
            ka, ke = ca[c] * Po[0], ce[c] * Po[0]
            rs = _entropy_residual(pd, Po, Ui[:, c], Si, dt[c], ka, ke)
            rm = _mink_momentum_residual(pd, Po, Ui[:, c], dt[c], ka, ke)
            worst = max(worst, max(rs, rm) / (1e-13 + 10.0 * err))
            # total conservation holds unless the radiation inversion capped the
            # radiation frame's Lorentz factor (the radiation is then recomputed
            # from the capped primitives, as for the energy methods)
            if math.sqrt(1.0 + Po[9:12] @ Po[9:12]) < 0.9 * pd["gamma_max"]:
                tot = np.abs((Uo[1:5] + Uo[8:12]) - (Ui[1:5, c] + Ui[8:12, c]))
                sc = np.abs(Ui[1:5, c]).sum() + np.abs(Ui[8:12, c]).sum()
                cons = max(cons, tot.max() / sc)
    assert checked > 200 and worst <= 1.0 and cons < 1e-14, (checked, worst, cons)


@pytest.mark.parametrize("ka", [0.3, 3.0])
def test_entropy_and_energy_roots_agree_to_second_order(orc, ka):
    """Gas and radiation at rest out of equilibrium, exchanging energy over
    dt: the energy equation gives du = dt Q, the entropy equation T dS = dt Q;
    at fixed density T dS = du, so the two roots differ at second order in
    the exchange: halving dt divides their difference by about 4."""
    pd = I.default_params(arad=1.0)
    g = orc.geom(pd, 0.0, 0.0)
    P = np.zeros(12)
    P[0], P[1], P[8] = 1.0, 0.02, 0.005
    Ui = orc.p2u(pd, g, P)
    Si = _si(orc, pd, P)
    diffs = []
    for dt in (0.01, 0.005, 0.0025):
        e = orc.implicit_attempt(pd, g, Ui, Si, P, dt, ka, 0.0, "pmhd")
        s = orc.implicit_attempt(pd, g, Ui, Si, P, dt, ka, 0.0, "pmhd", entropy=True)
        assert e[4] < 1e-12 and s[4] < 1e-12
        du = e[0][1] - P[1]
        diffs.append(abs(s[0][1] - e[0][1]) / abs(du))
    # relative difference linear in the exchange: absolute difference quadratic
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 1.85 < r1 < 2.15 and 1.85 < r2 < 2.15, diffs


def test_full_cascade_rescues_batch_cells(orc):
    """On the batched workload the full cascade (PRAD, staged attempts,
    entropy methods) leaves at most a tenth of the cells without a solution
    that PMHD, URAD and the cold limit leave, and gives bit for bit the same
    result on every cell that the shorter cascade accepts with PMHD first."""
    pd, g, P, dt, ca, ce, Ui = _batch(orc, 3000, 25)
    P0, U0, it0, st0 = orc.implicit_batch(pd, Ui, P, dt, ca, ce)
    P1, U1, it1, st1 = orc.implicit_batch(dict(pd, cascade=1), Ui, P, dt, ca, ce)
    f0 = ((st0 & orc.ST_FAIL) != 0).sum()
    f1 = ((st1 & orc.ST_FAIL) != 0).sum()
    assert f0 > 100 and f1 <= 0.1 * f0, (f0, f1)
    first = ((st0 & orc.ST_PMHD) != 0) & ((st0 & (orc.ST_FAIL | orc.ST_NOT_ACCEPT | orc.ST_EXTREME)) == 0)
    assert np.array_equal(U0[:, first], U1[:, first]) and np.array_equal(P0[:, first], P1[:, first])
    for b in (orc.ST_PRAD, orc.ST_ENTROPY, orc.ST_STAGED):
        assert ((st1 & b) != 0).sum() > 0


def test_entropy_tracer_flux(orc):
    """The entropy tracer's face flux (the 13th flux, sqrt(-g) S u^d): for a
    uniform flow the physical flux S u^x with S = rho0 ln(p^n / rho0^(n+1))
    written out here; across a jump moving supersonically to the right HLL
    returns the left state's flux (the flux uses the gas speeds)."""
    n = 12
    for flux in ("llf", "hll"):
        pd = I.default_params(n=(n, 1, 1), bc_lo=("outflow",) * 3, bc_hi=("outflow",) * 3, flux=flux)
        N = I.ncell(pd)
        Pc = np.zeros(12)
        Pc[0], Pc[1], Pc[8] = 1.3, 0.4, 0.2
        Pc[2:5] = [0.3, -0.2, 0.1]
        Pc[9:12] = Pc[2:5]
        P = np.tile(Pc[:, None], (1, N))
        F, emf, vch, Fs = orc.fluxes_s(pd, P, np.zeros(N), np.zeros(N))
        gam = pd["gam"]
        nn = 1.0 / (gam - 1)
        S = Pc[0] * math.log(((gam - 1) * Pc[1]) ** nn / Pc[0] ** (nn + 1))
        assert abs(Fs[0][pd["ng"] + 3] - S * Pc[2]) < 1e-14 * abs(S * Pc[2])
    pd = I.default_params(n=(n, 1, 1), bc_lo=("outflow",) * 3, bc_hi=("outflow",) * 3, flux="hll")
    PL = np.zeros(12)
    PL[0], PL[1], PL[8], PL[2] = 1.0, 0.01, 1e-6, 0.95 / math.sqrt(1 - 0.95 ** 2)
    PL[9] = PL[2]
    PR = PL.copy()
    PR[0], PR[1] = 0.5, 0.003
    g = pd["ng"]
    P = np.where(np.arange(I.ncell(pd)) < g + n // 2, PL[:, None], PR[:, None])
    F, emf, vch, Fs = orc.fluxes_s(pd, P, np.zeros(P.shape[1]), np.zeros(P.shape[1]))
    SL = PL[0] * math.log(((pd["gam"] - 1) * PL[1]) ** 1.5 / PL[0] ** 2.5)
    assert abs(Fs[0][g + n // 2] - SL * PL[2]) < 1e-14 * abs(SL * PL[2])


def _batch_box(orc, n=256, seed=31, **kw):
    """A periodic 1-D box of batch-recipe cells (flows slowed tenfold,
    opacities raised a thousandfold): far-from-equilibrium neighbours whose
    step needs the entropy, staged and PRAD attempts."""
    pdb, Pb, dtb, cab, ceb = I.implicit_batch(n, seed=seed)
    pd = I.default_params(n=(n, 1, 1), arad=1.0, tol_pmhd=1e-10, courant=0.4, cascade=1, **kw)
    N = I.ncell(pd)
    g = pd["ng"]
    P = np.zeros((12, N))
    P[:, g:g + n] = Pb
    P[2:5] *= 0.1
    P[9:12] = P[2:5]
    ca, ce = np.zeros(N), np.zeros(N)
    ca[g:g + n], ce[g:g + n] = cab * 1e3, ceb * 1e3
    P = orc.bc(pd, P)
    for a in (ca, ce):
        a[:g], a[-g:] = a[n:n + g], a[g:2 * g]
    return pd, P, ca, ce


@pytest.mark.parametrize("scheme", ["imex2", "imex3"])
def test_imex_full_cascade_changes_nothing_where_pmhd_is_accepted(orc, scheme):
    from test_oracle_pins import _periodic_box

    pd, P, ca, ce = _periodic_box((8, 6, 4), seed=7)
    pd = dict(pd, scheme=scheme)
    U = orc.prim_to_cons(pd, P)
    P0, U0, dt0, st0, _, _ = orc.step(pd, P, U, ca, ce)
    P1, U1, dt1, st1, _, _ = orc.step(dict(pd, cascade=1), P, U, ca, ce)
    other = orc.ST_FAIL | orc.ST_ENTROPY | orc.ST_PRAD | orc.ST_STAGED | orc.ST_NOT_ACCEPT
    assert not np.any(st0 & other) and not np.any(st1 & other)
    assert dt0 == dt1 and np.array_equal(P0, P1) and np.array_equal(U0, U1)


@pytest.mark.parametrize("scheme", ["imex2", "imex3"])
def test_imex_entropy_methods_take_cells_the_energy_methods_leave(orc, scheme):
    pd, P, ca, ce = _batch_box(orc, scheme=scheme)
    U = orc.prim_to_cons(pd, P)
    m = np.zeros(P.shape[1], bool)
    m[pd["ng"]:pd["ng"] + pd["n"][0]] = True
    P0, U0, dt0, st0, _, _ = orc.step(dict(pd, cascade=0), P, U, ca, ce)
    P1, U1, dt1, st1, _, _ = orc.step(pd, P, U, ca, ce)
    f0 = int(((st0[m] & orc.ST_FAIL) != 0).sum())
    f1 = int(((st1[m] & orc.ST_FAIL) != 0).sum())
    ne = int(((st1[m] & orc.ST_ENTROPY) != 0).sum())
    assert ne > 0 and f1 < f0, (ne, f0, f1)
    assert np.all(np.isfinite(P1[:, m])) and np.all(P1[0, m] > 0) and np.all(P1[1, m] > 0)
