"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``; never by the product package.  The
oracle shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["geom.c", "phys.c", "invert.c", "implicit.c", "step.c", "stag.c"]

ST_PMHD, ST_URAD, ST_TYPE2_NEG, ST_BASIC, ST_C2P_FAIL, ST_FLOOR, ST_NOT_ACCEPT, ST_FAIL, \
    ST_NO_GOOD_NB, ST_EXTREME, ST_COLD, ST_PRAD, ST_ENTROPY, ST_STAGED = (1 << i for i in range(14))

_BC = {"outflow": 0, "periodic": 1, "reflect": 2, "polar": 3}
_SCHEME = {"rk3": 0, "imex2": 1, "imex2b": 2, "imex3": 3}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, FP64, no FMA contraction, no
    reassociation; -O3 for x86-64-v3 so the same build runs on the AVX2 hosts
    it is shipped to)."""
    if force or not os.path.exists(LIB) or any(
            os.path.getmtime(os.path.join(HERE, s)) > os.path.getmtime(LIB)
            for s in SOURCES + ["oracle.h", "oracle_internal.h"]):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off",
               "-o", LIB] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
        subprocess.run(cmd, check=True)
    return LIB


class Params(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3), ("ng", C.c_int), ("metric", C.c_int),
        ("a", C.c_double), ("R0", C.c_double),
        ("xlo", C.c_double * 3), ("xhi", C.c_double * 3),
        ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3),
        ("gam", C.c_double), ("arad", C.c_double), ("gamma_max", C.c_double),
        ("courant", C.c_double), ("flux", C.c_int),
        ("tol_pmhd", C.c_double), ("tol_urad", C.c_double),
        ("tol_accept", C.c_double), ("tol_fail", C.c_double),
        ("max_iter", C.c_int), ("roundoff", C.c_int),
        ("rho_floor", C.c_double), ("u_floor", C.c_double), ("bsq_rho_max", C.c_double),
        ("bsq_u_max", C.c_double), ("u_rho_max", C.c_double), ("erad_floor", C.c_double),
        ("scheme", C.c_int), ("recon", C.c_int), ("cold", C.c_int), ("cascade", C.c_int),
        ("ct", C.c_int),
    ]


class Geom(C.Structure):
    _fields_ = [("gcov", C.c_double * 16), ("gcon", C.c_double * 16),
                ("gdet", C.c_double), ("alpha", C.c_double)]


class ImplicitInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("err", C.c_double)]


def params(d: dict) -> Params:
    p = Params()
    p.n[:] = list(d["n"])
    p.ng = d["ng"]
    p.metric = 1 if d["metric"] in ("ks", "kerr-schild") else 0
    p.a = d["a"]
    p.R0 = d["R0"]
    p.xlo[:] = list(d["xlo"])
    p.xhi[:] = list(d["xhi"])
    p.bc_lo[:] = [_BC[b] for b in d["bc_lo"]]
    p.bc_hi[:] = [_BC[b] for b in d["bc_hi"]]
    for k in ("gam", "arad", "gamma_max", "courant", "tol_pmhd", "tol_urad", "tol_accept",
              "tol_fail", "rho_floor", "u_floor", "bsq_rho_max", "bsq_u_max", "u_rho_max",
              "erad_floor"):
        setattr(p, k, float(d[k]))
    p.flux = 1 if d["flux"] == "hll" else 0
    p.max_iter = int(d["max_iter"])
    p.roundoff = int(d["roundoff"])
    p.scheme = _SCHEME[d.get("scheme", "rk3")]
    p.recon = 1 if d.get("recon", "mc") == "ppm" else 0
    p.cold = int(d.get("cold", 1))
    p.cascade = int(d.get("cascade", 0))
    p.ct = 1 if d.get("ct", "flux") == "staggered" else 0
    return p


_lib = None

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        PP, GP = C.POINTER(Params), C.POINTER(Geom)
        sigs = {
            "orc_geom_point": (None, [PP, C.c_double, C.c_double, GP]),
            "orc_connection": (None, [PP, C.c_double, C.c_double, _D]),
            "orc_p2u": (None, [PP, GP, _D, _D]),
            "orc_flux": (None, [PP, GP, _D, C.c_int, _D]),
            "orc_source_geom": (None, [PP, GP, _D, _D, _D]),
            "orc_four_force": (None, [PP, GP, _D, C.c_double, C.c_double, _D]),
            "orc_fluid_frame_rad": (None, [GP, _D, _D, _D, _D]),
            "orc_wavespeeds": (None, [PP, GP, _D, C.c_int, C.c_double, _D, _D]),
            "orc_mhd_invert": (C.c_int, [PP, GP, _D, _D, _D]),
            "orc_rad_invert": (C.c_int, [PP, GP, _D, C.c_int, _D]),
            "orc_implicit_cell": (None, [PP, GP, _D, _D, C.c_double, C.c_double, C.c_double,
                                         _D, _D, C.POINTER(ImplicitInfo)]),
            "orc_implicit_cold": (None, [PP, GP, _D, _D, C.c_double, C.c_double, C.c_double,
                                         C.c_double, _D, _D, C.POINTER(ImplicitInfo)]),
            "orc_implicit_batch": (None, [PP, C.c_long, _D, _D, _D, _D, _D, _D, _D, _I, _I]),
            "orc_implicit_cell_s": (None, [PP, GP, _D, C.c_double, _D, C.c_double, C.c_double,
                                           C.c_double, _D, _D, C.POINTER(ImplicitInfo)]),
            "orc_implicit_attempt": (None, [PP, GP, _D, C.c_double, _D, C.c_double, C.c_double,
                                            C.c_double, C.c_int, C.c_int, C.c_int, _D, _D,
                                            C.POINTER(ImplicitInfo)]),
            "orc_entropy": (C.c_double, [PP, _D]),
            "orc_fluxes_s": (None, [PP, _D, _D, _D, _D, _D, _D, _D, _D]),
            "orc_implicit_grid_s": (None, [PP, _D, _D, _D, C.c_double, _D, _D, _D, _D, _I, _I]),
            "orc_ncell_alloc": (C.c_long, [PP]),
            "orc_bc": (None, [PP, _D]),
            "orc_prim_to_cons": (None, [PP, _D, _D]),
            "orc_fluxes": (None, [PP, _D, _D, _D, _D, _D, _D]),
            "orc_flattener": (None, [PP, _D, _D, _D, _D, C.c_int]),
            "orc_ppm_cell": (None, [_D, C.c_double, _D, _D]),
            "orc_mc_face": (None, [_D, _D, _D]),
            "orc_timestep": (C.c_double, [PP, _D]),
            "orc_explicit_update": (None, [PP, C.c_double, C.c_double, C.c_double, C.c_double,
                                           _D, _D, _D, _D, _D, _D]),
            "orc_con2prim": (None, [PP, _D, _D, _D, _I]),
            "orc_implicit_grid": (None, [PP, _D, _D, C.c_double, _D, _D, _D, _D, _I, _I]),
            "orc_fixup": (None, [PP, _D, _D, _I]),
            "orc_step": (C.c_int, [PP, _D, _D, _D, _D, _D, C.c_int, _I, _I]),
            "orc_bc_face": (None, [PP, _D]),
            "orc_face_to_center": (None, [PP, _D, _D, _D]),
            "orc_fluxes_stag": (None, [PP, _D, _D, _D, _D, _D, _D, _D, _D, _D]),
            "orc_face_update": (None, [PP, C.c_double, C.c_double, C.c_double, C.c_double,
                                       _D, _D, _D, _D]),
            "orc_step_stag": (C.c_int, [PP, _D, _D, _D, _D, _D, _D, C.c_int, _I, _I]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _ip(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# pointwise
# ---------------------------------------------------------------------------

def geom(pd: dict, x1: float, x2: float) -> Geom:
    g = Geom()
    lib().orc_geom_point(C.byref(params(pd)), x1, x2, C.byref(g))
    return g


def geom_arrays(g: Geom):
    return (np.array(g.gcov[:]).reshape(4, 4), np.array(g.gcon[:]).reshape(4, 4), g.gdet, g.alpha)


def connection(pd: dict, x1: float, x2: float) -> np.ndarray:
    out = np.zeros(64)
    lib().orc_connection(C.byref(params(pd)), x1, x2, _dp(out))
    return out.reshape(4, 4, 4)


def p2u(pd, g, P):
    P = _f64(P)
    U = np.zeros(12)
    lib().orc_p2u(C.byref(params(pd)), C.byref(g), _dp(P), _dp(U))
    return U


def flux(pd, g, P, d):
    P = _f64(P)
    F = np.zeros(12)
    lib().orc_flux(C.byref(params(pd)), C.byref(g), _dp(P), d, _dp(F))
    return F


def source_geom(pd, g, conn, P):
    P = _f64(P)
    S = np.zeros(12)
    cn = _f64(conn).reshape(-1).copy()
    lib().orc_source_geom(C.byref(params(pd)), C.byref(g), _dp(cn), _dp(P), _dp(S))
    return S


def four_force(pd, g, P, kabs, kes):
    P = _f64(P)
    G = np.zeros(4)
    lib().orc_four_force(C.byref(params(pd)), C.byref(g), _dp(P), kabs, kes, _dp(G))
    return G


def fluid_frame_rad(g, P):
    P = _f64(P)
    E = np.zeros(1)
    F = np.zeros(3)
    Ph = np.zeros(9)
    lib().orc_fluid_frame_rad(C.byref(g), _dp(P), _dp(E), _dp(F), _dp(Ph))
    return E[0], F, Ph.reshape(3, 3)


def wavespeeds(pd, g, P, d, kdx=0.0):
    P = _f64(P)
    vg = np.zeros(2)
    vr = np.zeros(2)
    lib().orc_wavespeeds(C.byref(params(pd)), C.byref(g), _dp(P), d, kdx, _dp(vg), _dp(vr))
    return vg, vr


def mhd_invert(pd, g, U, Pguess=None):
    U = _f64(U)
    P = np.zeros(12) if Pguess is None else _f64(Pguess).copy()
    rc = lib().orc_mhd_invert(C.byref(params(pd)), C.byref(g), _dp(U), _dp(P.copy()), _dp(P))
    return rc, P


def rad_invert(pd, g, U, limiter=0, P=None):
    U = _f64(U)
    P = np.zeros(12) if P is None else _f64(P).copy()
    fl = lib().orc_rad_invert(C.byref(params(pd)), C.byref(g), _dp(U), limiter, _dp(P))
    return fl, P


def implicit_cell(pd, g, Ui, Pguess, dt, chi_abs, chi_es):
    Ui = _f64(Ui)
    Pg = _f64(Pguess)
    Po = np.zeros(12)
    Uo = np.zeros(12)
    info = ImplicitInfo()
    lib().orc_implicit_cell(C.byref(params(pd)), C.byref(g), _dp(Ui), _dp(Pg), dt, chi_abs,
                            chi_es, _dp(Po), _dp(Uo), C.byref(info))
    return Po, Uo, info.status, info.iters, info.err


def implicit_cold(pd, g, Ui, Pguess, dt, chi_abs, chi_es, u_c):
    """The cold MHD solve alone: u_g held at u_c, the gas momentum equations
    solved for u~^i."""
    Ui = _f64(Ui)
    Pg = _f64(Pguess)
    Po = np.zeros(12)
    Uo = np.zeros(12)
    info = ImplicitInfo()
    lib().orc_implicit_cold(C.byref(params(pd)), C.byref(g), _dp(Ui), _dp(Pg), dt, chi_abs,
                            chi_es, u_c, _dp(Po), _dp(Uo), C.byref(info))
    return Po, Uo, info.status, info.iters, info.err


def implicit_cell_s(pd, g, Ui, Si, Pguess, dt, chi_abs, chi_es):
    """implicit_cell with the explicit entropy Si = sqrt(-g) [S u^t]_(i)."""
    Ui = _f64(Ui)
    Pg = _f64(Pguess)
    Po = np.zeros(12)
    Uo = np.zeros(12)
    info = ImplicitInfo()
    lib().orc_implicit_cell_s(C.byref(params(pd)), C.byref(g), _dp(Ui), float(Si), _dp(Pg), dt,
                              chi_abs, chi_es, _dp(Po), _dp(Uo), C.byref(info))
    return Po, Uo, info.status, info.iters, info.err


METHODS = {"pmhd": 0, "urad": 1, "prad": 2}


def implicit_attempt(pd, g, Ui, Si, Pguess, dt, chi_abs, chi_es, method, staged=False,
                     entropy=False):
    """One attempt of one method (pmhd, urad, prad), normal or staged, with
    the energy or the entropy equation."""
    Ui = _f64(Ui)
    Pg = _f64(Pguess)
    Po = np.zeros(12)
    Uo = np.zeros(12)
    info = ImplicitInfo()
    lib().orc_implicit_attempt(C.byref(params(pd)), C.byref(g), _dp(Ui), float(Si), _dp(Pg), dt,
                               chi_abs, chi_es, METHODS[method], int(staged), int(entropy),
                               _dp(Po), _dp(Uo), C.byref(info))
    return Po, Uo, info.status, info.iters, info.err


def entropy(pd, P):
    """S = rho0 ln(p^n / rho0^(n+1)) of one cell's primitives."""
    return lib().orc_entropy(C.byref(params(pd)), _dp(_f64(P)))


def implicit_batch(pd, Ui, Pg, dt, chi_abs, chi_es):
    Ui, Pg, dt, ca, ce = (_f64(a) for a in (Ui, Pg, dt, chi_abs, chi_es))
    n = Ui.shape[1]
    Po = np.zeros((12, n))
    Uo = np.zeros((12, n))
    it = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    lib().orc_implicit_batch(C.byref(params(pd)), n, _dp(Ui), _dp(Pg), _dp(dt), _dp(ca),
                             _dp(ce), _dp(Po), _dp(Uo), _ip(it), _ip(st))
    return Po, Uo, it, st


# ---------------------------------------------------------------------------
# grid level: arrays are [12][N] (P, U) or [N] (chi) in the allocated layout
# ---------------------------------------------------------------------------

def ncell(pd) -> int:
    return lib().orc_ncell_alloc(C.byref(params(pd)))


def bc(pd, P):
    P = _f64(P).copy()
    lib().orc_bc(C.byref(params(pd)), _dp(P))
    return P


def prim_to_cons(pd, P):
    P = _f64(P)
    U = np.zeros_like(P)
    lib().orc_prim_to_cons(C.byref(params(pd)), _dp(P), _dp(U))
    return U


def fluxes(pd, P, chi_abs, chi_es):
    P, ca, ce = _f64(P), _f64(chi_abs), _f64(chi_es)
    N = P.shape[1]
    F = np.zeros((3, 12, N))
    emf = np.zeros((3, N))
    vch = np.zeros((3, N))
    lib().orc_fluxes(C.byref(params(pd)), _dp(P), _dp(ca), _dp(ce), _dp(F), _dp(emf), _dp(vch))
    return F, emf, vch


def fluxes_s(pd, P, chi_abs, chi_es):
    """fluxes() plus the entropy tracer's face fluxes Fs [3][N]."""
    P, ca, ce = _f64(P), _f64(chi_abs), _f64(chi_es)
    N = P.shape[1]
    F = np.zeros((3, 12, N))
    emf = np.zeros((3, N))
    vch = np.zeros((3, N))
    Fs = np.zeros((3, N))
    lib().orc_fluxes_s(C.byref(params(pd)), _dp(P), _dp(ca), _dp(ce), None, _dp(F), _dp(emf),
                       _dp(vch), _dp(Fs))
    return F, emf, vch, Fs


# ---------------------------------------------------------------------------
# staggered face field: Bf [3][N], sqrt(-g) B^(p+1) on the lower p-face of each
# cell (pd["ct"] = "staggered")
# ---------------------------------------------------------------------------

def bc_face(pd, Bf):
    Bf = _f64(Bf).copy()
    lib().orc_bc_face(C.byref(params(pd)), _dp(Bf))
    return Bf


def face_to_center(pd, Bf, P, U):
    """P, U with the interior cells' field slots set from the faces."""
    P, U = _f64(P).copy(), _f64(U).copy()
    lib().orc_face_to_center(C.byref(params(pd)), _dp(_f64(Bf)), _dp(P), _dp(U))
    return P, U


def fluxes_stag(pd, P, Bf, chi_abs, chi_es):
    """Face fluxes, the four-state corner EMFs and the face speeds of P with
    the face field Bf (the PPM flattener of P alone, as at a step's start)."""
    P, Bf, ca, ce = _f64(P), _f64(Bf), _f64(chi_abs), _f64(chi_es)
    N = P.shape[1]
    F = np.zeros((3, 12, N))
    emf = np.zeros((3, N))
    vch = np.zeros((3, N))
    fl = None
    if pd.get("recon", "mc") == "ppm":
        fl = np.zeros((6, N))
        lib().orc_flattener(C.byref(params(pd)), _dp(P), _dp(ca), _dp(ce), _dp(fl), 0)
    lib().orc_fluxes_stag(C.byref(params(pd)), _dp(P), _dp(Bf), _dp(ca), _dp(ce),
                          _dp(fl) if fl is not None else None, _dp(F), _dp(emf), _dp(vch), None)
    return F, emf, vch


def face_update(pd, a, b, c, dt, Bn, Bprev, emf, Bout=None):
    """Faces a Bn + b Bprev + c dt (-curl emf); emf may be None when c = 0."""
    Bout = np.zeros_like(_f64(Bn)) if Bout is None else _f64(Bout).copy()
    if emf is None and c != 0.0:
        raise ValueError("face_update needs the EMFs when c != 0")
    lib().orc_face_update(C.byref(params(pd)), a, b, c, dt, _dp(_f64(Bn)), _dp(_f64(Bprev)),
                          _dp(_f64(emf)) if emf is not None else None, _dp(Bout))
    return Bout


def step_stag(pd, P, U, Bf, chi_abs, chi_es, dt=0.0, dt_fixed=False):
    """One step with the staggered field: (P, U, Bf, dt, status, iters, nbad)."""
    P, U, Bf = _f64(P).copy(), _f64(U).copy(), _f64(Bf).copy()
    ca, ce = _f64(chi_abs), _f64(chi_es)
    n = P.shape[1]
    dtv = np.array([dt], dtype=np.float64)
    st = np.zeros(n, np.int32)
    it = np.zeros(n, np.int32)
    nbad = lib().orc_step_stag(C.byref(params(pd)), _dp(P), _dp(U), _dp(Bf), _dp(ca), _dp(ce),
                               _dp(dtv), 1 if dt_fixed else 0, _ip(st), _ip(it))
    if nbad < 0:
        raise ValueError("staggered step needs ct='staggered'")
    return P, U, Bf, float(dtv[0]), st, it, nbad


def flattener(pd, P, chi_abs, chi_es, prev=None):
    """PPM flattener [3 directions][gas, radiation][N]; with prev, the larger
    of the new value and prev (earlier sub-steps of the same step)."""
    P, ca, ce = _f64(P), _f64(chi_abs), _f64(chi_es)
    fl = np.zeros((3, 2, P.shape[1])) if prev is None else _f64(prev).copy()
    lib().orc_flattener(C.byref(params(pd)), _dp(P), _dp(ca), _dp(ce), _dp(fl),
                        0 if prev is None else 1)
    return fl


def ppm_cell(a5, f):
    """PPM left and right values of the middle of five cell values."""
    a = _f64(a5)
    l, r = np.zeros(1), np.zeros(1)
    lib().orc_ppm_cell(_dp(a), float(f), _dp(l), _dp(r))
    return float(l[0]), float(r[0])


def mc_face(a4):
    """MC-limited values (left state, right state) at the face between the
    2nd and 3rd of four cell values."""
    a = _f64(a4)
    l, r = np.zeros(1), np.zeros(1)
    lib().orc_mc_face(_dp(a), _dp(l), _dp(r))
    return float(l[0]), float(r[0])


def timestep(pd, vch):
    return lib().orc_timestep(C.byref(params(pd)), _dp(_f64(vch)))


def explicit_update(pd, a, b, c, dt, P, Un, Uprev, F, emf):
    P, Un, Uprev, F, emf = (_f64(x) for x in (P, Un, Uprev, F, emf))
    Ue = Un.copy()
    lib().orc_explicit_update(C.byref(params(pd)), a, b, c, dt, _dp(P), _dp(Un), _dp(Uprev),
                              _dp(F), _dp(emf), _dp(Ue))
    return Ue


def con2prim(pd, U, Pguess):
    U, Pg = _f64(U), _f64(Pguess)
    P = Pg.copy()
    st = np.zeros(U.shape[1], np.int32)
    lib().orc_con2prim(C.byref(params(pd)), _dp(U), _dp(Pg), _dp(P), _ip(st))
    return P, st


def implicit_grid(pd, Uexp, Pguess, dt, chi_abs, chi_es):
    Ue, Pg, ca, ce = (_f64(x) for x in (Uexp, Pguess, chi_abs, chi_es))
    Po = Pg.copy()
    Uo = Ue.copy()
    n = Ue.shape[1]
    it = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    lib().orc_implicit_grid(C.byref(params(pd)), _dp(Ue), _dp(Pg), dt, _dp(ca), _dp(ce),
                            _dp(Po), _dp(Uo), _ip(it), _ip(st))
    return Po, Uo, it, st


def fixup(pd, P, U, status):
    P, U = _f64(P).copy(), _f64(U).copy()
    st = np.ascontiguousarray(status, dtype=np.int32).copy()
    lib().orc_fixup(C.byref(params(pd)), _dp(P), _dp(U), _ip(st))
    return P, U, st


def step(pd, P, U, chi_abs, chi_es, dt=0.0, dt_fixed=False):
    P, U, ca, ce = _f64(P).copy(), _f64(U).copy(), _f64(chi_abs), _f64(chi_es)
    n = P.shape[1]
    dtv = np.array([dt], dtype=np.float64)
    st = np.zeros(n, np.int32)
    it = np.zeros(n, np.int32)
    nbad = lib().orc_step(C.byref(params(pd)), _dp(P), _dp(U), _dp(ca), _dp(ce), _dp(dtv),
                          1 if dt_fixed else 0, _ip(st), _ip(it))
    return P, U, float(dtv[0]), st, it, nbad
