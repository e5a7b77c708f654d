"""PPM reconstruction with the shock flattener (Sec. 4.3) on the GPU
(through the C ABI) against the oracle: the fluxes of one state, whole
steps (the flattener kept as the largest over the step's sub-steps), with
IMEX3 and with FP32-mixed faces; the adjoint refuses PPM grids."""
import sys

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_gpu_parity import dev, field_err, host, interior_mask  # noqa: E402


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

    pd, P, ca, ce = _periodic_box((12, 10, 6), seed=7)
    pd4 = dict(pd, ng=4, recon="ppm")
    na2, na4 = I.nalloc(pd), I.nalloc(pd4)
    P4 = np.zeros((12,) + tuple(na4[::-1]))
    P4[(slice(None),) + I.interior(pd4)] = P.reshape((12,) + tuple(na2[::-1]))[
        (slice(None),) + I.interior(pd)]
    n4 = int(np.prod(na4))
    return pd4, P4.reshape(12, -1), np.full(n4, ca[0]), np.full(n4, ce[0])


CASES = {
    "tube1d": lambda: I.shock_tube_1d(200, ng=4, recon="ppm"),
    "disk2d": lambda: I.accretion_disk(n=(40, 24, 1), seed=2, ng=4, recon="ppm"),
    "disk3d": lambda: I.accretion_disk(n=(24, 12, 8), seed=3, ng=4, recon="ppm"),
    "box3d": _box,
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_ppm_fluxes(G, orc, case):
    say("case", case, "PPM fluxes")
    pd, P, ca, ce = CASES[case]()
    P = orc.bc(pd, P)
    g = G.Grid(pd)
    F, emf, vch = (host(x) for x in g.fluxes(dev(P), dev(ca), dev(ce)))
    Fr, emfr, vchr = orc.fluxes(pd, P, ca, ce)
    e = max(field_err(F[d], Fr[d]).max() for d in range(3))
    say("  flux error", e, "emf", field_err(emf, emfr).max(), "speeds", field_err(vch, vchr).max())
    assert e < 1e-12
    assert field_err(emf, emfr).max() < 1e-12
    assert field_err(vch, vchr).max() < 1e-13
    g.close()


def _steps(G, orc, pd, P, ca, ce, nsteps, ref_pd=None):
    U = orc.prim_to_cons(pd, P)
    g = G.Grid(pd)
    Pt, Ut = dev(P), dev(U)
    cat, cet = dev(ca), dev(ce)
    dtt = torch.zeros(1, dtype=torch.float64, device="cuda")
    stt = torch.zeros(g.N, dtype=torch.int32, device="cuda")
    Pr, Ur = P.copy(), U.copy()
    for _ in range(nsteps):
        Pr, Ur, dtr, st, it, nbad = orc.step(ref_pd or pd, Pr, Ur, ca, ce)
        g.step(Pt, Ut, cat, cet, dtt, status=stt)
    m = interior_mask(pd)
    eP = field_err(host(Pt), Pr, m)
    eU = field_err(host(Ut), Ur, m)
    fails = np.array_equal(host(stt)[m] & orc.ST_FAIL, st[m] & orc.ST_FAIL)
    g.close()
    return max(eP.max(), eU.max()), fails


def _oracle_sensitivity(orc, pd, P, ca, ce, nsteps):
    """Field error of the oracle's own run against the same run from inputs
    perturbed by seeded 1e-14 relative noise: the conditioning of the steps."""
    m = interior_mask(pd)
    r = np.random.default_rng(1)
    P2 = P * (1 + 1e-14 * r.standard_normal(P.shape))
    a = (P, orc.prim_to_cons(pd, P))
    b = (P2, orc.prim_to_cons(pd, P2))
    for _ in range(nsteps):
        a = orc.step(pd, a[0], a[1], ca, ce)[:2]
        b = orc.step(pd, b[0], b[1], ca, ce)[:2]
    return max(field_err(b[0], a[0], m).max(), field_err(b[1], a[1], m).max())


@pytest.mark.parametrize("case", sorted(CASES))
def test_ppm_steps(G, orc, case):
    """Three steps: the flattener of sub-steps 2 and 3 is the larger of its
    own and the earlier ones'.  Tolerance: 1e-12 per step, or 20 times the
    oracle's response to 1e-14 relative input noise where the steps amplify
    rounding more (the radiation frame velocity of the shock tube under PPM:
    1e-14 noise gives 6e-11 after three steps on the oracle alone)."""
    say("case", case, "PPM 3 steps")
    pd, P, ca, ce = CASES[case]()
    e, fails = _steps(G, orc, pd, P, ca, ce, 3)
    tol = 3e-12
    if e >= tol:
        sens = _oracle_sensitivity(orc, pd, P, ca, ce, 3)
        say("  oracle sensitivity to 1e-14 input noise", sens)
        tol = max(tol, 20 * sens)
    say("  field error", e, "tolerance", tol)
    assert e < tol and fails


def test_ppm_imex3_step(G, orc):
    say("case disk3d PPM + IMEX3")
    pd, P, ca, ce = CASES["disk3d"]()
    e, fails = _steps(G, orc, dict(pd, scheme="imex3"), P, ca, ce, 1)
    say("  field error", e)
    assert e < 1e-11 and fails


def test_ppm_mixed_precision(G, orc):
    say("case disk3d PPM, FP32-mixed faces, 3 steps")
    pd, P, ca, ce = CASES["disk3d"]()
    e, _ = _steps(G, orc, dict(pd, precision="mixed"), P, ca, ce, 3, ref_pd=pd)
    say("  field error vs the FP64 oracle", e)
    assert e < 1e-5


def test_ppm_guards(G):
    say("case PPM guards")
    pd, P, ca, ce = CASES["disk3d"]()
    with pytest.raises(RuntimeError):
        G.Grid(dict(pd, ng=2))
    with pytest.raises(RuntimeError):
        G.Grid(dict(pd, ng=3))
