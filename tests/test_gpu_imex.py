"""IMEX2, IMEX2B and IMEX3 steps (Sec. 4.1, eq. IMEX2, IMEX2B, IMEX3) on the
GPU (through the C ABI) against the oracle's, element by element, to the
tolerance of the RK3 step (1e-11 per field), with the FAIL bits equal."""
import sys

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_gpu_parity import dev, field_err, host, interior_mask  # noqa: E402
from test_oracle_imex import _relax_box  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    from paper_1312_6127_amd import grrmhd

    grrmhd.lib()
    assert torch.cuda.is_available()
    return grrmhd


def _box():
    from test_oracle_pins import _periodic_box

    return _periodic_box((12, 10, 6), seed=7)


CASES = {
    "tube1d": lambda: I.shock_tube_1d(200),
    "disk3d": lambda: I.accretion_disk(n=(24, 12, 8), seed=3),
    "box3d": _box,
    "relax": lambda: _relax_box("rk3"),
}


def _steps(G, orc, pd, P, ca, ce, nsteps):
    U = orc.prim_to_cons(pd, P)
    g = G.Grid(pd)
    Pt, Ut = dev(P), dev(U)
    cat, cet = dev(ca), dev(ce)
    dtt = torch.zeros(1, dtype=torch.float64, device="cuda")
    stt = torch.zeros(g.N, dtype=torch.int32, device="cuda")
    Pr, Ur = P.copy(), U.copy()
    m = interior_mask(pd)
    worst = 0.0
    for s in range(nsteps):
        Pr, Ur, dtr, st, it, nbad = orc.step(pd, Pr, Ur, ca, ce)
        g.step(Pt, Ut, cat, cet, dtt, status=stt)
        assert abs(host(dtt)[0] / dtr - 1) < 1e-13
        Pg, Ug = host(Pt), host(Ut)
        eP = field_err(Pg, Pr, m)
        eU = field_err(Ug, Ur, m)
        worst = max(worst, eP.max(), eU.max())
        if max(eP.max(), eU.max()) > 1e-11:
            q = int(np.argmax(eU))
            c = int(np.argmax(np.where(m, np.abs(Ug[q] - Ur[q]), 0.0)))
            say(f"  step {s}: P errors {np.array2string(eP, precision=2)}")
            say(f"  U errors {np.array2string(eU, precision=2)}; worst U[{q}] at cell {c}: "
                f"gpu {Ug[q, c]!r} oracle {Ur[q, c]!r} status {st[c]} chi {ca[c]:.3e}")
        assert np.array_equal(host(stt)[m] & orc.ST_FAIL, st[m] & orc.ST_FAIL)
    g.close()
    return worst


@pytest.mark.parametrize("scheme", ["imex2", "imex2b", "imex3"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_imex_step(G, orc, case, scheme):
    say("case", case, scheme)
    pd, P, ca, ce = CASES[case]()
    pd = dict(pd, scheme=scheme)
    e = _steps(G, orc, pd, P, ca, ce, 1)
    say("  field error", e)
    assert e < 1e-11


def test_imex3_three_steps_on_the_disk(G, orc):
    say("case disk3d imex3, 3 steps")
    pd, P, ca, ce = I.accretion_disk(n=(24, 12, 8), seed=3)
    e = _steps(G, orc, dict(pd, scheme="imex3"), P, ca, ce, 3)
    say("  field error", e)
    assert e < 1e-11


def test_imex_workspace_sizes(G):
    """Step and adjoint workspaces grow with the scheme's stages; a zero
    cotangent gives a zero adjoint on every scheme (whose gradients are
    checked against differences in the adjoint tests)."""
    say("case imex workspace sizes")
    pd, P, ca, ce = I.accretion_disk(n=(12, 8, 4), seed=3)
    sizes, asizes = {}, {}
    for s in ("rk3", "imex2", "imex2b", "imex3"):
        g = G.Grid(dict(pd, scheme=s))
        sizes[s] = g.ws_bytes
        asizes[s] = G.lib().grrmhd_adjoint_workspace_bytes(g.h)
        gP = g.step_adjoint(dev(P), dev(ca), dev(ce), dev(np.array([0.01])), dev(np.zeros_like(P)))
        assert not torch.any(gP != 0)
        g.close()
    # per stage: input, explicit state, output P and U, output P before the
    # fix-ups; plus the sources, their cotangents, the stage cotangents and
    # the final inversion's guess cotangent
    ns = {"imex2": 3, "imex2b": 4, "imex3": 5}
    for s, k in ns.items():
        assert asizes[s] >= asizes["rk3"] + ((k - 3) * 60 + 2 * 32 + k * 12 + 12) * 8 * I.ncell(pd) - 4096
    # stage U's (all but the last) and four stored sources on top of RK3's
    N = I.ncell(pd)
    assert sizes["imex2"] >= sizes["rk3"] + (2 * 12 + 4 * 8) * 8 * N
    assert sizes["imex2b"] >= sizes["rk3"] + (3 * 12 + 4 * 8) * 8 * N
    assert sizes["imex3"] >= sizes["rk3"] + (4 * 12 + 4 * 8) * 8 * N
