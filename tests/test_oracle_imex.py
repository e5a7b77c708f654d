"""Pins of the oracle's IMEX2, IMEX2B and IMEX3 steps (Sec. 4.1, eq. IMEX2,
IMEX2B, IMEX3), and of RK3 run through the same stage machinery.

- A uniform box at rest has no flux divergence, so every implicit stage is a
  gas-radiation energy exchange with a closed-form (quartic) solution, and
  the stored sources M^k follow from it: the whole step is a closed-form
  sequence of the printed coefficients.
- Temporal order: self-convergence of the oracle's step in dt, of the
  explicit part alone (one Kerr-Schild cell, geometric source, no coupling)
  and of the implicit part alone (the relaxing box).  A mistyped coefficient
  breaks the order the schemes are built for (2, 2, 3; RK3 with the same
  coefficients for both parts: 3 explicit, 1 implicit).
- Conservation of mass, total energy and momentum on periodic boxes.
"""
import math

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I

from test_oracle_pins import _periodic_box, _quartic_root

SCHEMES = ["rk3", "imex2", "imex2b", "imex3"]


def _stages(name):
    """(a, b, j, c, [m_k], g) per stage, written from the printed schemes."""
    if name == "imex2":
        g = 1 - 1 / math.sqrt(2)
        return [(1, 0, -1, 0, [], g),
                ((3 * g - 1) / g, (1 - 2 * g) / g, 0, 1, [], g),
                (0.5, 0.5, 1, 0.5, [g, (1 - g) / 2], 0)]
    if name == "imex2b":
        return [(1, 0, -1, 0, [], 0.25), (1, 0, -1, 0.5, [], 0.25),
                (0, 1, 1, 0.5, [1 / 3, 1 / 12], 1 / 3),
                (1 / 3, 2 / 3, 2, 1 / 3, [1 / 9, 1 / 9, 1 / 9], 0)]
    if name == "imex3":
        a, b, e = 0.24169426078821, 0.06042356519705, 0.12915286960590
        return [(1, 0, -1, 0, [], a), (2, -1, 0, 0, [], a), (1, 0, -1, 1, [0, 1 - a], a),
                (0.75, 0.25, 2, 0.25, [b, (-1 + a + 4 * e) / 4, (2 - 5 * a - 4 * (b + e)) / 4], a),
                (1 / 3, 2 / 3, 3, 2 / 3, [-2 * b / 3, (1 - 4 * e) / 6,
                                          (-1 + 4 * a + 4 * (b + e)) / 6, 4 * (1 - a) / 6], 0)]
    return [(1, 0, -1, 1, [], 1), (0.75, 0.25, 0, 0.25, [], 0.25),
            (1 / 3, 2 / 3, 1, 2 / 3, [], 2 / 3)]


def _relax_box(scheme, rho=0.7, u0=0.05, E0=0.4, ka=3.0, arad=0.8):
    pd = I.default_params(n=(4, 1, 1), arad=arad, scheme=scheme)
    N = I.ncell(pd)
    P = np.zeros((12, N))
    P[0], P[1], P[8] = rho, u0, E0
    return pd, P, np.full(N, ka / rho), np.full(N, 0.4)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_uniform_box_follows_the_stage_sequence(orc, scheme):
    """At rest, U1 = -u, U8 = -E; an implicit stage with dt_i = g dt solves the
    quartic exchange from its bracket (u_e, E_e); the source of stage k is
    du/dt = kappa (E - a T^4) (= -dE/dt), T = (gam - 1) u / rho; the final
    explicit combination is inverted exactly."""
    rho, u0, E0, ka, arad = 0.7, 0.05, 0.4, 3.0, 0.8
    pd, P, ca, ce = _relax_box(scheme, rho, u0, E0, ka, arad)
    dt = 0.37
    U = orc.prim_to_cons(pd, P)
    P1, U1, _, st, it, nbad = orc.step(pd, P, U, ca, ce, dt=dt, dt_fixed=True)
    assert nbad == 0
    g = pd["gam"]
    us, Es, Mu = [], [], []
    for (a, b, j, c, m, gi) in _stages(scheme):
        ue = a * u0 + (b * us[j] if j >= 0 else 0.0) + dt * sum(mk * Mu[k] for k, mk in enumerate(m))
        Ee = a * E0 + (b * Es[j] if j >= 0 else 0.0) - dt * sum(mk * Mu[k] for k, mk in enumerate(m))
        if gi > 0:
            u = _quartic_root(ue, Ee, rho, ka, gi * dt, arad, g)
            E = Ee + ue - u
        else:
            u, E = ue, Ee
        us.append(u)
        Es.append(E)
        T = (g - 1) * u / rho
        Mu.append(ka * (E - arad * T ** 4))
    assert np.all(P1[1, 2:-2] == P1[1, 2])
    assert abs(P1[1, 2] / us[-1] - 1) < 1e-12, (P1[1, 2], us[-1])
    assert abs(P1[8, 2] / Es[-1] - 1) < 1e-12, (P1[8, 2], Es[-1])


def _self_order(run, Ns):
    r = [run(N) for N in Ns]
    d = [np.abs(r[q] - r[q + 1]).max() for q in range(len(r) - 1)]
    return [math.log2(d[q] / d[q + 1]) for q in range(len(d) - 1)]


EXPLICIT_ORDER = {"rk3": 3, "imex2": 2, "imex2b": 2, "imex3": 3}
IMPLICIT_ORDER = {"rk3": 1, "imex2": 2, "imex2b": 2, "imex3": 3}


@pytest.mark.parametrize("scheme", SCHEMES)
def test_temporal_order_of_the_explicit_part(orc, scheme):
    """One Kerr-Schild cell (a = 0.9375, r ~ 6.5, orbiting gas and
    radiation), no coupling: only the geometric source drives the state."""
    pd0, P0, _, _ = I.accretion_disk(n=(12, 8, 4), seed=3)
    na = I.nalloc(pd0)
    c = (2 + 6) + na[0] * ((2 + 4) + na[1] * (2 + 2))
    dx = [(pd0["xhi"][d] - pd0["xlo"][d]) / pd0["n"][d] for d in range(2)]
    x = [pd0["xlo"][0] + 6.5 * dx[0], pd0["xlo"][1] + 4.5 * dx[1]]
    pd = dict(pd0, n=(1, 1, 1), scheme=scheme,
              xlo=(x[0] - dx[0] / 2, x[1] - dx[1] / 2, 0.0), xhi=(x[0] + dx[0] / 2, x[1] + dx[1] / 2, 1.0))
    zero = np.zeros(1)

    def run(N):
        P = P0[:, c:c + 1].copy()
        U = orc.prim_to_cons(pd, P)
        for _ in range(N):
            P, U, _, st, it, nbad = orc.step(pd, P, U, zero, zero, dt=2.0 / N, dt_fixed=True)
            assert nbad == 0
        return U[:, 0]

    p = _self_order(run, (8, 16, 32, 64))
    assert abs(p[-1] - EXPLICIT_ORDER[scheme]) < 0.1, p


@pytest.mark.parametrize("scheme", SCHEMES)
def test_temporal_order_of_the_implicit_part(orc, scheme):
    """The relaxing uniform box (dt kappa up to 0.4 per step)."""
    pd, P0, ca, ce = _relax_box(scheme)

    def run(N):
        P = P0.copy()
        U = orc.prim_to_cons(pd, P)
        for _ in range(N):
            P, U, _, st, it, nbad = orc.step(pd, P, U, ca, ce, dt=1.0 / N, dt_fixed=True)
            assert nbad == 0
        return np.array([P[1, 2], P[8, 2]])

    p = _self_order(run, (16, 32, 64, 128))
    assert abs(p[-1] - IMPLICIT_ORDER[scheme]) < 0.1, p


@pytest.mark.parametrize("scheme", ["imex2", "imex2b", "imex3"])
def test_imex_step_conserves_on_periodic_box(orc, scheme):
    pd, P, ca, ce = _periodic_box((24, 16, 1), seed=1)
    pd = dict(pd, scheme=scheme)
    U = orc.prim_to_cons(pd, P)
    sl = I.interior(pd)
    na = I.nalloc(pd)

    def totals(U):
        V = U.reshape((12,) + na[::-1])[(slice(None),) + sl].reshape(12, -1)
        s = V.sum(axis=1)
        return np.array([s[0], s[1] + s[8], s[2] + s[9], s[3] + s[10], s[4] + s[11], s[5], s[6], s[7]]), V

    t0, V = totals(U)
    P1, U1, dt, st, it, nbad = orc.step(pd, P, U, ca, ce)
    assert nbad == 0 and dt > 0
    t1, _ = totals(U1)
    scale = np.array([np.abs(V[0]).sum(), np.abs(V[1]).sum() + np.abs(V[8]).sum()] +
                     [np.abs(V[2 + i]).sum() + np.abs(V[9 + i]).sum() for i in range(3)] +
                     [np.abs(V[5 + i]).sum() + 1e-30 for i in range(3)])
    assert np.all(np.abs(t1 - t0) <= 5e-14 * scale), (t1 - t0) / scale
