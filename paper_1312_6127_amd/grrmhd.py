"""Thin ctypes binding of ``libgrrmhd.so`` (include/grrmhd.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and the current HIP stream.  The
binding raises if the library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libgrrmhd.so")

ST_PMHD, ST_URAD, ST_TYPE2_NEG, ST_BASIC, ST_C2P_FAIL, ST_FLOOR, ST_NOT_ACCEPT, ST_FAIL, \
    ST_NO_GOOD_NB, ST_EXTREME, ST_COLD, ST_PRAD, ST_ENTROPY, ST_STAGED = (1 << i for i in range(14))

_BC = {"outflow": 0, "periodic": 1, "reflect": 2, "polar": 3}


class Params(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3), ("ng", C.c_int), ("metric", C.c_int),
        ("a", C.c_double), ("R0", C.c_double),
        ("xlo", C.c_double * 3), ("xhi", C.c_double * 3),
        ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3),
        ("gam", C.c_double), ("arad", C.c_double), ("gamma_max", C.c_double),
        ("courant", C.c_double), ("flux", C.c_int), ("precision", C.c_int), ("r_fp64", C.c_double),
        ("tol_pmhd", C.c_double), ("tol_urad", C.c_double),
        ("tol_accept", C.c_double), ("tol_fail", C.c_double),
        ("max_iter", C.c_int), ("roundoff", C.c_int),
        ("rho_floor", C.c_double), ("u_floor", C.c_double), ("bsq_rho_max", C.c_double),
        ("bsq_u_max", C.c_double), ("u_rho_max", C.c_double), ("erad_floor", C.c_double),
        ("scheme", C.c_int), ("recon", C.c_int), ("cold", C.c_int), ("cascade", C.c_int),
        ("ct", C.c_int),
    ]


class Tuning(C.Structure):
    _fields_ = [("mode", C.c_int), ("block", C.c_int), ("waves_per_cu", C.c_int), ("ms", C.c_float)]


SCHEMES = {"rk3": 0, "imex2": 1, "imex2b": 2, "imex3": 3}
PER_CELL, PER_ITERATION, PERSISTENT = 0, 1, 2
TUNE_CANDIDATES = 9
NOALLOC_MAX_CELLS = 262144  # GRRMHD_NOALLOC_MAX_CELLS
FORM_NAMES = {PER_CELL: "per_cell", PER_ITERATION: "per_iteration", PERSISTENT: "persistent"}


def params(d: dict) -> Params:
    p = Params()
    p.n[:] = list(d["n"])
    p.ng = d["ng"]
    p.metric = 1 if d["metric"] in ("ks", "kerr-schild") else 0
    p.a, p.R0 = d["a"], d["R0"]
    p.xlo[:] = list(d["xlo"])
    p.xhi[:] = list(d["xhi"])
    p.bc_lo[:] = [_BC[b] for b in d["bc_lo"]]
    p.bc_hi[:] = [_BC[b] for b in d["bc_hi"]]
    for k in ("gam", "arad", "gamma_max", "courant", "tol_pmhd", "tol_urad", "tol_accept",
              "tol_fail", "rho_floor", "u_floor", "bsq_rho_max", "bsq_u_max", "u_rho_max",
              "erad_floor"):
        setattr(p, k, float(d[k]))
    p.flux = 1 if d["flux"] == "hll" else 0
    p.precision = 1 if d.get("precision", "fp64") == "mixed" else 0
    p.r_fp64 = float(d.get("r_fp64", 2.0))
    p.max_iter = int(d["max_iter"])
    p.roundoff = int(d["roundoff"])
    p.scheme = SCHEMES[d.get("scheme", "rk3")]
    p.recon = 1 if d.get("recon", "mc") == "ppm" else 0
    p.cold = int(d.get("cold", 1))
    p.cascade = int(d.get("cascade", 0))
    p.ct = 1 if d.get("ct", "flux") == "staggered" else 0
    return p


_lib = None
_VP = C.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIBPATH)
        PP = C.POINTER(Params)
        sigs = {
            "grrmhd_default_params": (None, [PP]),
            "grrmhd_last_error": (C.c_char_p, []),
            "grrmhd_init_grid": (C.c_int, [PP, C.c_int, _VP, C.POINTER(_VP)]),
            "grrmhd_free_grid": (C.c_int, [_VP]),
            "grrmhd_set_stream": (C.c_int, [_VP, _VP]),
            "grrmhd_ncell_alloc": (C.c_long, [_VP]),
            "grrmhd_workspace_bytes": (C.c_size_t, [_VP]),
            "grrmhd_prim_to_cons": (C.c_int, [_VP, _VP, _VP]),
            "grrmhd_apply_bc": (C.c_int, [_VP, _VP]),
            "grrmhd_fluxes": (C.c_int, [_VP] + [_VP] * 6),
            "grrmhd_timestep": (C.c_int, [_VP, _VP, _VP]),
            "grrmhd_explicit_update": (C.c_int, [_VP, C.c_double, C.c_double, C.c_double] + [_VP] * 7),
            "grrmhd_con2prim": (C.c_int, [_VP] + [_VP] * 4),
            "grrmhd_implicit_grid": (C.c_int, [_VP, _VP, _VP, C.c_double] + [_VP] * 8),
            "grrmhd_fixup": (C.c_int, [_VP] * 5),
            "grrmhd_fixup_vjp": (C.c_int, [_VP] * 8),
            "grrmhd_step": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, C.c_int, _VP, _VP, _VP,
                                      C.c_size_t]),
            "grrmhd_adjoint_workspace_bytes": (C.c_size_t, [_VP]),
            "grrmhd_step_adjoint": (C.c_int, [_VP] * 11 + [C.c_size_t]),
            "grrmhd_step_checkpointed": (C.c_int, [_VP] * 8 + [C.c_size_t]),
            "grrmhd_step_adjoint_saved": (C.c_int, [_VP] * 8 + [C.c_size_t]),
            "grrmhd_implicit_vjp": (C.c_int, [_VP, _VP, _VP, _VP, C.c_double] + [_VP] * 6),
            "grrmhd_explicit_vjp_workspace_bytes": (C.c_size_t, [_VP]),
            "grrmhd_explicit_vjp": (C.c_int, [_VP, C.c_double] + [_VP] * 7 + [C.c_size_t]),
            "grrmhd_bc_vjp": (C.c_int, [_VP, _VP]),
            "grrmhd_con2prim_vjp": (C.c_int, [_VP] * 7),
            "grrmhd_implicit_source_workspace_bytes": (C.c_size_t, [C.c_long]),
            "grrmhd_implicit_source": (C.c_int, [PP, C.c_long] + [_VP] * 11 + [C.c_size_t, _VP]),
            "grrmhd_implicit_source_noalloc": (C.c_int, [PP, C.c_long] + [_VP] * 11),
            "grrmhd_implicit_source_workspace_bytes_ex": (C.c_size_t, [C.c_long, C.c_int]),
            "grrmhd_implicit_source_ex": (C.c_int, [PP, C.c_long] + [_VP] * 10 +
                                          [C.c_int, C.c_int, C.c_int, _VP, C.c_size_t, _VP]),
            "grrmhd_autotune_implicit_source": (C.c_int, [PP, C.c_long] + [_VP] * 11 +
                                                [C.c_size_t, _VP, C.POINTER(Tuning),
                                                 C.POINTER(Tuning), C.c_int]),
            "grrmhd_implicit_stats": (C.c_int, [_VP, C.POINTER(C.c_ulonglong)]),
            "grrmhd_time_implicit": (C.c_int, [_VP, C.c_int]),
            "grrmhd_implicit_time": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
            "grrmhd_implicit_source_stats": (C.c_int, [_VP, C.POINTER(C.c_ulonglong), _VP]),
            "grrmhd_implicit_source_cascade_stats": (C.c_int, [_VP, C.POINTER(C.c_ulonglong), _VP]),
            "grrmhd_apply_bc_faces": (C.c_int, [_VP, _VP]),
            "grrmhd_face_to_center": (C.c_int, [_VP] * 4),
            "grrmhd_fluxes_staggered": (C.c_int, [_VP] * 9 + [C.c_size_t]),
            "grrmhd_step_staggered": (C.c_int, [_VP] * 7 + [C.c_int, _VP, _VP, _VP, C.c_size_t]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise RuntimeError(f"grrmhd error {rc}: {lib().grrmhd_last_error().decode()}")


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors, contiguous"
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Grid:
    """A grid with its device geometry; arrays are [12, N] float64 tensors."""

    def __init__(self, pd: dict, device: int = 0):
        self.pd = dict(pd)
        self._p = params(pd)
        h = C.c_void_p()
        _check(lib().grrmhd_init_grid(C.byref(self._p), device, _stream(), C.byref(h)))
        self.h = h
        self.N = lib().grrmhd_ncell_alloc(h)
        self.ws_bytes = lib().grrmhd_workspace_bytes(h)
        self._ws = None

    def close(self):
        if self.h:
            _check(lib().grrmhd_free_grid(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(lib().grrmhd_set_stream(self.h, _stream()))

    def workspace(self):
        if self._ws is None:
            self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device="cuda")
        off = (-self._ws.data_ptr()) % 256
        return self._ws[off:off + self.ws_bytes]

    def prim_to_cons(self, P, U=None):
        self._sync_stream()
        U = torch.empty_like(P) if U is None else U
        _check(lib().grrmhd_prim_to_cons(self.h, _ptr(P), _ptr(U)))
        return U

    def apply_bc(self, P):
        self._sync_stream()
        _check(lib().grrmhd_apply_bc(self.h, _ptr(P)))
        return P

    def fluxes(self, P, chi_abs, chi_es):
        self._sync_stream()
        F = torch.empty((3, 12, self.N), dtype=torch.float64, device=P.device)
        emf = torch.empty((3, self.N), dtype=torch.float64, device=P.device)
        vch = torch.empty((3, self.N), dtype=torch.float64, device=P.device)
        _check(lib().grrmhd_fluxes(self.h, _ptr(P), _ptr(chi_abs), _ptr(chi_es), _ptr(F),
                                   _ptr(emf), _ptr(vch)))
        return F, emf, vch

    def timestep(self, vchar, dt=None):
        self._sync_stream()
        dt = torch.zeros(1, dtype=torch.float64, device=vchar.device) if dt is None else dt
        _check(lib().grrmhd_timestep(self.h, _ptr(vchar), _ptr(dt)))
        return dt

    def explicit_update(self, a, b, c, dt, P, Un, Uprev, F, emf, Uexp=None):
        self._sync_stream()
        Uexp = Un.clone() if Uexp is None else Uexp
        _check(lib().grrmhd_explicit_update(self.h, a, b, c, _ptr(dt), _ptr(P), _ptr(Un),
                                            _ptr(Uprev), _ptr(F), _ptr(emf), _ptr(Uexp)))
        return Uexp

    def con2prim(self, U, Pguess):
        self._sync_stream()
        P = Pguess.clone()
        st = torch.zeros(self.N, dtype=torch.int32, device=U.device)
        _check(lib().grrmhd_con2prim(self.h, _ptr(U), _ptr(Pguess), _ptr(P), _ptr(st)))
        return P, st

    def implicit(self, Uexp, Pguess, dt_scale, dt, chi_abs, chi_es):
        self._sync_stream()
        P = Pguess.clone()
        U = Uexp.clone()
        it = torch.zeros(self.N, dtype=torch.int32, device=U.device)
        st = torch.zeros(self.N, dtype=torch.int32, device=U.device)
        err = torch.zeros(self.N, dtype=torch.float64, device=U.device)
        _check(lib().grrmhd_implicit_grid(self.h, _ptr(Uexp), _ptr(Pguess), dt_scale, _ptr(dt),
                                          _ptr(chi_abs), _ptr(chi_es), _ptr(P), _ptr(U), _ptr(it),
                                          _ptr(st), _ptr(err)))
        return P, U, it, st, err

    def implicit_stats(self):
        """(Newton trips of first attempts, lane slots, cascade cells) of the
        last implicit launch on this grid."""
        out = (C.c_ulonglong * 3)()
        _check(lib().grrmhd_implicit_stats(self.h, out))
        return tuple(int(v) for v in out)

    def new_adjoint_workspace(self):
        """A fresh 256-byte aligned adjoint workspace: (tensor, bytes)."""
        nb = lib().grrmhd_adjoint_workspace_bytes(self.h)
        raw = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        off = (-raw.data_ptr()) % 256
        return raw[off:off + nb], nb

    def adjoint_workspace(self):
        if getattr(self, "_aws", None) is None:
            self._aws = self.new_adjoint_workspace()
        return self._aws

    def step_checkpointed(self, P, chi_abs, chi_es, dt, ws=None):
        """The forward half of step_adjoint (dt held fixed): returns P^{n+1},
        U^{n+1} and the workspace holding the stage checkpoints (a fresh one
        unless given), for step_adjoint_saved."""
        self._sync_stream()
        ws = self.new_adjoint_workspace() if ws is None else ws
        Pn = torch.empty_like(P)
        Un = torch.empty_like(P)
        _check(lib().grrmhd_step_checkpointed(self.h, _ptr(P), _ptr(chi_abs), _ptr(chi_es), _ptr(dt),
                                              _ptr(Pn), _ptr(Un), _ptr(ws[0]), ws[1]))
        return Pn, Un, ws

    def step_adjoint_saved(self, ws, chi_abs, chi_es, dt, gU, want_chi=False):
        """The reverse half of step_adjoint over the checkpoints in ws (from
        step_checkpointed with the same opacities and dt)."""
        self._sync_stream()
        gP = torch.empty((12, self.N), dtype=torch.float64, device=gU.device)
        gc = torch.empty((2, self.N), dtype=torch.float64, device=gU.device) if want_chi else None
        _check(lib().grrmhd_step_adjoint_saved(self.h, _ptr(chi_abs), _ptr(chi_es), _ptr(dt),
                                               _ptr(gU), _ptr(gP), _ptr(gc), _ptr(ws[0]), ws[1]))
        return (gP, gc) if want_chi else gP

    def step_adjoint(self, P, chi_abs, chi_es, dt, gU, want_next=False, want_chi=False):
        """dL/dP^n for L = sum(gU * U^{n+1}(P^n)), dt (1-element device
        tensor) held fixed and U^n = U(P^n).  Returns gP, then with want_chi
        the [2][N] opacity gradient (d/dchi_abs, d/dchi_es), then with
        want_next P^{n+1} and U^{n+1}."""
        self._sync_stream()
        ws, nb = self.adjoint_workspace()
        gP = torch.empty_like(P)
        gc = torch.empty((2, self.N), dtype=P.dtype, device=P.device) if want_chi else None
        Pn = torch.empty_like(P) if want_next else None
        Un = torch.empty_like(P) if want_next else None
        _check(lib().grrmhd_step_adjoint(self.h, _ptr(P), _ptr(chi_abs), _ptr(chi_es), _ptr(dt),
                                         _ptr(gU), _ptr(gP), _ptr(gc), _ptr(Pn), _ptr(Un),
                                         _ptr(ws), nb))
        out = (gP,) + ((gc,) if want_chi else ()) + ((Pn, Un) if want_next else ())
        return out if len(out) > 1 else gP

    def implicit_vjp(self, Uexp, P_out, status, dt_scale, dt, chi_abs, chi_es, gP, gU):
        self._sync_stream()
        gUe = torch.empty_like(Uexp)
        _check(lib().grrmhd_implicit_vjp(self.h, _ptr(Uexp), _ptr(P_out), _ptr(status), dt_scale,
                                         _ptr(dt), _ptr(chi_abs), _ptr(chi_es), _ptr(gP), _ptr(gU),
                                         _ptr(gUe)))
        return gUe

    def explicit_vjp(self, c, dt, P, chi_abs, chi_es, gUe):
        self._sync_stream()
        nb = lib().grrmhd_explicit_vjp_workspace_bytes(self.h)
        raw = torch.empty(nb + 256, dtype=torch.uint8, device=P.device)
        off = (-raw.data_ptr()) % 256
        ws = raw[off:off + nb]
        gP = torch.empty_like(P)
        _check(lib().grrmhd_explicit_vjp(self.h, c, _ptr(dt), _ptr(P), _ptr(chi_abs), _ptr(chi_es),
                                         _ptr(gUe), _ptr(gP), _ptr(ws), nb))
        return gP

    def bc_vjp(self, gP):
        self._sync_stream()
        _check(lib().grrmhd_bc_vjp(self.h, _ptr(gP)))
        return gP

    def con2prim_vjp(self, U, P, status, gP):
        """Cotangents of grrmhd_con2prim's U and guess for the cotangent gP
        of its result (P, status: con2prim's outputs)."""
        self._sync_stream()
        gU = torch.empty_like(U)
        gPg = torch.empty_like(U)
        _check(lib().grrmhd_con2prim_vjp(self.h, _ptr(U), _ptr(P), _ptr(status), _ptr(gP), _ptr(gU),
                                         _ptr(gPg)))
        return gU, gPg

    def time_implicit(self, on: bool):
        """Start (clearing the record) or stop HIP-event timing of the
        implicit kernel's launches on this grid's stream."""
        self._sync_stream()
        _check(lib().grrmhd_time_implicit(self.h, 1 if on else 0))

    def implicit_time(self):
        """(summed milliseconds, launches) of the timed implicit kernels."""
        ms, cnt = C.c_double(), C.c_int()
        _check(lib().grrmhd_implicit_time(self.h, C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def fixup(self, P, U, status):
        self._sync_stream()
        scratch = torch.zeros((13, self.N), dtype=torch.float64, device=P.device)
        _check(lib().grrmhd_fixup(self.h, _ptr(P), _ptr(U), _ptr(status), _ptr(scratch)))
        return P, U, status

    def fixup_vjp(self, P, status, gP, gU):
        """Cotangents of grrmhd_fixup's input P, U for output cotangents gP, gU
        (P, status: the fix-up's result)."""
        self._sync_stream()
        gPp = torch.empty_like(gP)
        gUp = torch.empty_like(gU)
        scratch = torch.empty((12, self.N), dtype=torch.float64, device=P.device)
        _check(lib().grrmhd_fixup_vjp(self.h, _ptr(P), _ptr(status), _ptr(gP), _ptr(gU), _ptr(gPp),
                                      _ptr(gUp), _ptr(scratch)))
        return gPp, gUp

    # staggered face field Bf [3][N] (pd["ct"] = "staggered")
    def apply_bc_faces(self, Bf):
        self._sync_stream()
        _check(lib().grrmhd_apply_bc_faces(self.h, _ptr(Bf)))
        return Bf

    def face_to_center(self, Bf, P=None, U=None):
        """Interior cells' field slots of P and/or U from the faces."""
        self._sync_stream()
        _check(lib().grrmhd_face_to_center(self.h, _ptr(Bf), _ptr(P), _ptr(U)))
        return P, U

    def fluxes_staggered(self, P, Bf, chi_abs, chi_es):
        self._sync_stream()
        F = torch.empty((3, 12, self.N), dtype=torch.float64, device=P.device)
        emf = torch.empty((3, self.N), dtype=torch.float64, device=P.device)
        vch = torch.empty((3, self.N), dtype=torch.float64, device=P.device)
        ws = self.workspace()
        _check(lib().grrmhd_fluxes_staggered(self.h, _ptr(P), _ptr(Bf), _ptr(chi_abs),
                                             _ptr(chi_es), _ptr(F), _ptr(emf), _ptr(vch),
                                             _ptr(ws), self.ws_bytes))
        return F, emf, vch

    def step_staggered(self, P, U, Bf, chi_abs, chi_es, dt, dt_fixed=False, status=None,
                       iters=None):
        """One step of the grid's scheme with the staggered field, in place on
        P, U, Bf."""
        self._sync_stream()
        ws = self.workspace()
        _check(lib().grrmhd_step_staggered(self.h, _ptr(P), _ptr(U), _ptr(Bf), _ptr(chi_abs),
                                           _ptr(chi_es), _ptr(dt), 1 if dt_fixed else 0,
                                           _ptr(status), _ptr(iters), _ptr(ws), self.ws_bytes))
        return P, U, Bf

    def step(self, P, U, chi_abs, chi_es, dt, dt_fixed=False, status=None, iters=None):
        """One step of the grid's scheme in place on P, U; dt is a 1-element device
        tensor."""
        self._sync_stream()
        ws = self.workspace()
        _check(lib().grrmhd_step(self.h, _ptr(P), _ptr(U), _ptr(chi_abs), _ptr(chi_es), _ptr(dt),
                                 1 if dt_fixed else 0, _ptr(status), _ptr(iters), _ptr(ws),
                                 self.ws_bytes))
        return P, U


def _batch_out(U_expl, P_guess):
    n = U_expl.shape[1]
    P = P_guess.clone()
    U = U_expl.clone()
    it = torch.zeros(n, dtype=torch.int32, device=U.device)
    st = torch.zeros(n, dtype=torch.int32, device=U.device)
    err = torch.zeros(n, dtype=torch.float64, device=U.device)
    return n, P, U, it, st, err


def batch_workspace(n: int, mode: int = PER_CELL):
    """Device workspace of the batched solve, 256-byte aligned."""
    wsb = lib().grrmhd_implicit_source_workspace_bytes_ex(n, mode)
    raw = torch.empty(wsb + 256, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % 256
    return raw[off:off + wsb], wsb


def implicit_source(pd: dict, U_expl, P_guess, dt_cell, chi_abs, chi_es):
    """Batched implicit 4-force solve of independent flat-space cells."""
    n, P, U, it, st, err = _batch_out(U_expl, P_guess)
    p = params(pd)
    ws, wsb = batch_workspace(n)
    _check(lib().grrmhd_implicit_source(C.byref(p), n, _ptr(U_expl), _ptr(P_guess), _ptr(dt_cell),
                                        _ptr(chi_abs), _ptr(chi_es), _ptr(P), _ptr(U), _ptr(it),
                                        _ptr(st), _ptr(err), _ptr(ws), wsb, _stream()))
    return P, U, it, st, err


def implicit_source_noalloc(pd: dict, U_expl, P_guess, dt_cell, chi_abs, chi_es, out=None):
    """The batched solve through the allocation-free entry point (scratch in
    the library's static device array; at most NOALLOC_MAX_CELLS cells)."""
    n, P, U, it, st, err = _batch_out(U_expl, P_guess) if out is None else out
    p = params(pd)
    _check(lib().grrmhd_implicit_source_noalloc(C.byref(p), n, _ptr(U_expl), _ptr(P_guess),
                                                _ptr(dt_cell), _ptr(chi_abs), _ptr(chi_es),
                                                _ptr(P), _ptr(U), _ptr(it), _ptr(st), _ptr(err),
                                                _stream()))
    return P, U, it, st, err


def implicit_source_ex(pd: dict, U_expl, P_guess, dt_cell, chi_abs, chi_es, mode=PERSISTENT,
                       block=256, waves_per_cu=8, out=None, ws=None):
    """Batched solve in an explicit execution form (per cell, one launch per
    Newton trip, or persistent with the given block and waves per CU)."""
    n, P, U, it, st, err = _batch_out(U_expl, P_guess) if out is None else out
    p = params(pd)
    ws, wsb = batch_workspace(n, mode) if ws is None else ws
    _check(lib().grrmhd_implicit_source_ex(C.byref(p), n, _ptr(U_expl), _ptr(P_guess),
                                           _ptr(dt_cell), _ptr(chi_abs), _ptr(chi_es), _ptr(P),
                                           _ptr(U), _ptr(it), _ptr(st), _ptr(err), mode, block,
                                           waves_per_cu, _ptr(ws), wsb, _stream()))
    return P, U, it, st, err


def autotune_implicit_source(pd: dict, U_expl, P_guess, dt_cell, chi_abs, chi_es):
    """Times the execution forms on these inputs; returns (best Tuning, list
    of every candidate's Tuning, outputs)."""
    n, P, U, it, st, err = _batch_out(U_expl, P_guess)
    p = params(pd)
    ws, wsb = batch_workspace(n, PER_ITERATION)
    t = Tuning()
    allt = (Tuning * TUNE_CANDIDATES)()
    _check(lib().grrmhd_autotune_implicit_source(C.byref(p), n, _ptr(U_expl), _ptr(P_guess),
                                                 _ptr(dt_cell), _ptr(chi_abs), _ptr(chi_es),
                                                 _ptr(P), _ptr(U), _ptr(it), _ptr(st), _ptr(err),
                                                 _ptr(ws), wsb, _stream(), C.byref(t), allt,
                                                 TUNE_CANDIDATES))
    return t, list(allt), (P, U, it, st, err)


def batch_stats(ws):
    """(Newton trips of first attempts, lane slots, cascade cells) of the
    last batched solve that used workspace ws (a (tensor, bytes) pair)."""
    out = (C.c_ulonglong * 3)()
    _check(lib().grrmhd_implicit_source_stats(_ptr(ws[0]), out, _stream()))
    return tuple(int(v) for v in out)


def batch_cascade_stats(ws):
    """(residual evaluations, lane slots) of the compacted cascade of the last
    batched solve that used workspace ws."""
    out = (C.c_ulonglong * 2)()
    _check(lib().grrmhd_implicit_source_cascade_stats(_ptr(ws[0]), out, _stream()))
    return tuple(int(v) for v in out)


class GRRMHDStep(torch.autograd.Function):
    """U^{n+1} = step(P^n) with dt fixed, differentiable in P^n through the
    library's hand-written adjoint.

    GRRMHDStep.apply(grid, P, chi_abs, chi_es, dt[, keep_checkpoints]) ->
    U_next; the backward returns dL/dP at interior cells (ghost entries zero)
    and, where they require it, dL/dchi_abs and dL/dchi_es at every allocated
    cell.  keep_checkpoints (default True): the forward keeps the stage
    checkpoints (one adjoint workspace per call, held until the backward),
    and the backward runs the reverse sweep alone; False: the forward keeps
    P only and the backward recomputes the step."""

    @staticmethod
    def forward(ctx, grid, P, chi_abs, chi_es, dt, keep_checkpoints=True):
        Pc = P.detach().contiguous()
        ctx.grid = grid
        ctx.ws = None
        if keep_checkpoints:
            _, Uw, ctx.ws = grid.step_checkpointed(Pc, chi_abs, chi_es, dt)
        else:
            Pw = Pc.clone()
            Uw = grid.prim_to_cons(Pw)
            grid.step(Pw, Uw, chi_abs, chi_es, dt, dt_fixed=True)
        ctx.save_for_backward(Pc, chi_abs, chi_es, dt)
        return Uw

    @staticmethod
    def backward(ctx, gU):
        Pc, chi_abs, chi_es, dt = ctx.saved_tensors
        want = ctx.needs_input_grad[2] or ctx.needs_input_grad[3]
        gU = gU.contiguous()
        if ctx.ws is not None:
            out = ctx.grid.step_adjoint_saved(ctx.ws, chi_abs, chi_es, dt, gU, want_chi=want)
            ctx.ws = None
        else:
            out = ctx.grid.step_adjoint(Pc, chi_abs, chi_es, dt, gU, want_chi=want)
        if not want:
            return None, out, None, None, None, None
        gP, gc = out
        return (None, gP, gc[0] if ctx.needs_input_grad[2] else None,
                gc[1] if ctx.needs_input_grad[3] else None, None, None)
