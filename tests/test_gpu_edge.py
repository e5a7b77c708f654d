"""Edge cases on the GPU, through the C ABI, against the FP64 oracle: tiny and
ragged grids (a single cell, one or two cells per dimension, sizes that are
not multiples of the 16x4 wavefront tiles) stepped once, and batched
implicit solves of 0, 1 and around-a-wavefront counts of cells."""
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


def interior_mask(pd):
    m = np.zeros(I.nalloc(pd)[::-1], dtype=bool)
    m[I.interior(pd)] = True
    return m.reshape(-1)


def field_err(a, b, m):
    return np.array([np.abs(a[q, m] - b[q, m]).max() / max(np.abs(b[q, m]).max(), 1e-300)
                     for q in range(12)])


@pytest.mark.parametrize("n", [(1, 1, 1), (3, 1, 1), (2, 2, 2), (17, 5, 1), (5, 3, 2)])
def test_step_small_grids(G, orc, n):
    """One RK3 step of a periodic box.  Without an active dimension there is
    no Courant limit: the step then takes the dt it is given (dt_fixed)."""
    from test_oracle_pins import _periodic_box

    say("case small grid", n)
    pd, P, ca, ce = _periodic_box(n, seed=7)
    U = orc.prim_to_cons(pd, P)
    fixed = n == (1, 1, 1)
    P1, U1, dt, st, it, nbad = orc.step(pd, P, U, ca, ce, dt=0.05 if fixed else 0.0, dt_fixed=fixed)
    g = G.Grid(pd)
    Pt, Ut = dev(P), dev(U)
    dtt = dev(np.array([0.05 if fixed else 0.0]))
    stt = torch.zeros(g.N, dtype=torch.int32, device="cuda")
    g.step(Pt, Ut, dev(ca), dev(ce), dtt, status=stt, dt_fixed=fixed)
    m = interior_mask(pd)
    assert abs(host(dtt)[0] / dt - 1) < 1e-14
    eP, eU = field_err(host(Pt), P1, m), field_err(host(Ut), U1, m)
    say("  field errors P", eP.max(), "U", eU.max())
    assert eP.max() < 1e-11 and eU.max() < 1e-11
    assert np.array_equal(host(stt)[m] & orc.ST_FAIL, st[m] & orc.ST_FAIL)
    g.close()


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 257])
def test_batch_sizes(G, orc, n):
    """Batched solves of n independent cells (empty, one, around one
    wavefront): the same per-cell results as the oracle."""
    say("case batch size", n)
    pd, P, dt, ca, ce = I.implicit_batch(max(n, 1), seed=9)
    P, dt, ca, ce = P[:, :n], dt[:n], ca[:n], ce[:n]
    g0 = orc.geom(pd, 0.0, 0.0)
    U = np.stack([orc.p2u(pd, g0, P[:, c]) for c in range(n)], axis=1) if n else np.zeros((12, 0))
    Ui = U.copy()
    Ui[8] *= 1.3
    Ui[1] -= 0.3 * U[8]
    Pg, Ug, itg, stg, errg = [host(t) for t in G.implicit_source(pd, *[dev(a) for a in (Ui, P, dt, ca, ce)])]
    assert Pg.shape == (12, n) and stg.shape == (n,)
    if n == 0:
        return
    Pr, Ur, itr, str_ = orc.implicit_batch(pd, Ui, P, dt, ca, ce)
    kind = orc.ST_FAIL | orc.ST_COLD
    agree = (stg & kind) == (str_ & kind)
    assert agree.mean() >= 0.95
    good = agree & ((str_ & orc.ST_FAIL) == 0) & (errg < 1e-11)
    scale = np.abs(Ur[1:5]).sum(0) + np.abs(Ur[8:12]).sum(0)
    if good.any():
        d = np.abs(Ug - Ur)[1:12, good].max(axis=0) / scale[good]
        assert d.max() < 1e-12, d.max()
    # a failed cell returns its best attempt (not unique) or its inputs: finite
    assert np.isfinite(Pg).all() and np.isfinite(Ug).all()
