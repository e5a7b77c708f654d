// Host side of the GRRMHD library: grid set-up, launch shapes, the RK3-IMEX
// step orchestration and the extern "C" entry points declared in
// include/grrmhd.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "adjoint.h"
#include "stag.h"

struct grrmhd_grid {
  grrmhd_params p;
  Ctx C;
  int device;
  hipStream_t stream;
  double* geo;          // one allocation: centre table, x1-face table, x2-face table,
                        // then the dt slot, the implicit bookkeeping and work list
  unsigned long long* dtslot;    // Courant reduction of the stand-alone timestep call
  unsigned long long* dtstep[2]; // the step's reductions, alternating (each resets the other)
  int dtp = 0;
  int* cnt[2];          // cascade list lengths, alternating (each launch zeroes the other)
  double* flat = nullptr;  // PPM flattener of the step [3][gas, radiation][Ntot]
  // the implicit kernel's tiles: count, shape, cost keys of the last launch
  // and the dispatch order of the next one (int [ntiles] each)
  long ntiles = 0;
  int tile_i = 0;
  int* tkeys = nullptr;
  int* torder = nullptr;
  int cp = 0;
  Work W;               // implicit cascade list (interior indices), records, stats;
                        // W.counter is the list length of the last launch
  // optional HIP-event timing of the implicit kernel's launches
  static const int TCAP = 256;
  int timing = 0, nt = 0;
  hipEvent_t* ev = nullptr;   // 2 * TCAP events, created on first use
};

#ifndef GRRMHD_IMPLICIT_TILE_I
#define GRRMHD_IMPLICIT_TILE_I 16  // x1 extent of a wavefront's tile in the implicit kernel
#endif

static constexpr size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Cascade list of up to cap cells with the first attempts' records, laid out
// from `base` (256-byte aligned); returns the bytes used.
static constexpr size_t cascade_bytes(size_t cap) {
  return round256(sizeof(int) * cap) + round256(sizeof(double) * 13 * cap) +
         round256(sizeof(int) * 3 * cap);
}

static void cascade_layout(char* base, size_t cap, Work& W) {
  W.list = (int*)base;
  W.rec.d = (double*)(base + round256(sizeof(int) * cap));
  W.rec.i = (int*)(base + round256(sizeof(int) * cap) + round256(sizeof(double) * 13 * cap));
  W.rec.cap = (long)cap;
}

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(GRRMHD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)

#define LAUNCHCHK()                                                                     \
  do {                                                                                  \
    hipError_t e_ = hipGetLastError();                                                  \
    if (e_ != hipSuccess) return fail(GRRMHD_EHIP, std::string("launch: ") + hipGetErrorString(e_)); \
  } while (0)

static inline unsigned nblocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

extern "C" const char* grrmhd_last_error(void) { return g_err.c_str(); }

extern "C" void grrmhd_default_params(grrmhd_params* p) {
  memset(p, 0, sizeof(*p));
  p->n[0] = p->n[1] = p->n[2] = 1;
  p->ng = 2;
  p->metric = GRRMHD_MINKOWSKI;
  for (int d = 0; d < 3; d++) {
    p->xlo[d] = 0.0;
    p->xhi[d] = 1.0;
    p->bc_lo[d] = p->bc_hi[d] = GRRMHD_BC_PERIODIC;
  }
  p->gam = 5.0 / 3.0;
  p->arad = 1.0;
  p->gamma_max = 100.0;
  p->courant = 0.5;
  p->flux = GRRMHD_FLUX_LLF;
  p->precision = GRRMHD_FP64;
  p->scheme = GRRMHD_RK3;
  p->recon = GRRMHD_RECON_MC;
  p->cold = 1;
  p->cascade = 0;
  p->ct = GRRMHD_CT_FLUX;
  p->r_fp64 = 2.0;
  p->tol_pmhd = 1e-12;
  p->tol_urad = 1e-9;
  p->tol_accept = 1e-9;
  p->tol_fail = 1e-7;
  p->max_iter = 20;
  p->roundoff = 1;
  p->rho_floor = 1e-20;
  p->u_floor = 1e-22;
  p->bsq_rho_max = 200.0;
  p->bsq_u_max = 1e5;
  p->u_rho_max = 1e10;
  p->erad_floor = 1e-150;
}

static int validate(const grrmhd_params* p, bool need_grid) {
  if (!p) return fail(GRRMHD_EINVAL, "params is NULL");
  if (!(p->gam > 1.0) || !(p->arad >= 0.0) || !(p->gamma_max > 1.0) || !(p->courant > 0.0))
    return fail(GRRMHD_EINVAL, "gam > 1, arad >= 0, gamma_max > 1, courant > 0 required");
  if (p->max_iter < 1 || p->max_iter > 200) return fail(GRRMHD_EINVAL, "max_iter out of [1, 200]");
  if (p->flux != GRRMHD_FLUX_LLF && p->flux != GRRMHD_FLUX_HLL) return fail(GRRMHD_EINVAL, "bad flux");
  if (p->precision != GRRMHD_FP64 && p->precision != GRRMHD_MIXED)
    return fail(GRRMHD_EINVAL, "bad precision");
  if (p->metric != GRRMHD_MINKOWSKI && p->metric != GRRMHD_KERR_SCHILD)
    return fail(GRRMHD_EINVAL, "bad metric");
  if (p->scheme < GRRMHD_RK3 || p->scheme > GRRMHD_IMEX3) return fail(GRRMHD_EINVAL, "bad scheme");
  if (p->cold != 0 && p->cold != 1) return fail(GRRMHD_EINVAL, "cold must be 0 or 1");
  if (p->cascade != 0 && p->cascade != 1) return fail(GRRMHD_EINVAL, "cascade must be 0 or 1");
  if (p->ct != GRRMHD_CT_FLUX && p->ct != GRRMHD_CT_STAGGERED)
    return fail(GRRMHD_EINVAL, "ct must be GRRMHD_CT_FLUX or GRRMHD_CT_STAGGERED");
  if (p->recon != GRRMHD_RECON_MC && p->recon != GRRMHD_RECON_PPM)
    return fail(GRRMHD_EINVAL, "bad reconstruction");
  if (!need_grid) return 0;
  if (p->recon == GRRMHD_RECON_MC && p->ng != 2)
    return fail(GRRMHD_EINVAL, "ghost width must be 2 for MC reconstruction");
  if (p->recon == GRRMHD_RECON_PPM && p->ng != 4)
    return fail(GRRMHD_EINVAL, "ghost width must be 4 for PPM reconstruction");
  for (int d = 0; d < 3; d++) {
    if (p->n[d] < 1 || p->n[d] > (1 << 20)) return fail(GRRMHD_EINVAL, "n out of range");
    if (p->n[d] > 1 && p->n[d] < p->ng) return fail(GRRMHD_EINVAL, "active dimension shorter than ng");
    if (!(p->xhi[d] > p->xlo[d])) return fail(GRRMHD_EINVAL, "xhi must exceed xlo");
    for (int s = 0; s < 2; s++) {
      const int bc = s ? p->bc_hi[d] : p->bc_lo[d];
      if (bc < GRRMHD_BC_OUTFLOW || bc > GRRMHD_BC_POLAR) return fail(GRRMHD_EINVAL, "bad boundary");
      if (bc == GRRMHD_BC_POLAR && d != 1) return fail(GRRMHD_EINVAL, "polar boundary only on x2");
    }
  }
  if (p->n[1] > 1 && p->n[2] > 1 && (p->bc_lo[1] == GRRMHD_BC_POLAR || p->bc_hi[1] == GRRMHD_BC_POLAR) &&
      (p->n[2] % 2 != 0 || p->bc_lo[2] != GRRMHD_BC_PERIODIC))
    return fail(GRRMHD_EINVAL, "polar boundary needs an even, periodic x3");
  if (p->metric == GRRMHD_KERR_SCHILD && !(p->a >= 0.0 && p->a < 1.0))
    return fail(GRRMHD_EINVAL, "spin must be in [0, 1)");
  return 0;
}

static void fill_ctx(const grrmhd_params* p, Ctx& C) {
  memset(&C, 0, sizeof(C));
  for (int d = 0; d < 3; d++) {
    C.n[d] = p->n[d];
    C.ng[d] = p->n[d] > 1 ? p->ng : 0;
    C.N[d] = C.n[d] + 2 * C.ng[d];
    C.dx[d] = (p->xhi[d] - p->xlo[d]) / p->n[d];
    C.xlo[d] = p->xlo[d];
    C.bc_lo[d] = p->bc_lo[d];
    C.bc_hi[d] = p->bc_hi[d];
  }
  C.st[0] = 1;
  C.st[1] = C.N[0];
  C.st[2] = (long)C.N[0] * C.N[1];
  C.Ntot = C.st[2] * C.N[2];
  C.npos = C.N[0] * C.N[1];
  C.metric = p->metric;
  C.gam = p->gam;
  C.arad = p->arad;
  C.gamma_max = p->gamma_max;
  const double G = p->gamma_max * p->gamma_max;
  C.ymax = 16.0 * G * (G - 1.0) / ((4.0 * G - 1.0) * (4.0 * G - 1.0));
  C.courant = p->courant;
  C.flux = p->flux;
  C.recon = p->recon;
  C.cold = p->cold;
  C.cascade = p->cascade;
  C.ct = p->ct;
  // FP32 face path from the first x1 index i whose cell i-1 has r >= r_fp64
  C.mixed_i = 1 << 30;
  if (p->precision == GRRMHD_MIXED) {
    C.mixed_i = 0;
    if (p->metric == GRRMHD_KERR_SCHILD)
      while (C.mixed_i < C.N[0] &&
             p->R0 + exp(C.xlo[0] + (C.mixed_i - 1 - C.ng[0] + 0.5) * C.dx[0]) < p->r_fp64)
        C.mixed_i++;
  }
  C.tol_pmhd = p->tol_pmhd;
  C.tol_urad = p->tol_urad;
  C.tol_accept = p->tol_accept;
  C.tol_fail = p->tol_fail;
  C.max_iter = p->max_iter;
  C.roundoff = p->roundoff;
  C.rho_floor = p->rho_floor;
  C.u_floor = p->u_floor;
  C.bsq_rho_max = p->bsq_rho_max;
  C.bsq_u_max = p->bsq_u_max;
  C.u_rho_max = p->u_rho_max;
  C.erad_floor = p->erad_floor;
}

// Bookkeeping after the geometry tables: the stand-alone timestep's dt slot
// at 0, the cascade list lengths at 128 and 160, the lane statistics at 192,
// the step's two sets of Courant slots, then the cascade list and records.
static const size_t TAIL_DT0 = 256;
static const size_t TAIL_DT1 = TAIL_DT0 + 8 * GRRMHD_DT_SLOTS * GRRMHD_DT_STRIDE;
static const size_t TAIL_CASCADE = TAIL_DT1 + 8 * GRRMHD_DT_SLOTS * GRRMHD_DT_STRIDE;

extern "C" int grrmhd_init_grid(const grrmhd_params* p, int device, void* hip_stream,
                                grrmhd_grid** out) {
  if (!out) return fail(GRRMHD_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p, true);
  if (rc) return rc;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(GRRMHD_EINVAL, "device ordinal out of range");
  HIPCHK(hipSetDevice(device));
  grrmhd_grid* g = new grrmhd_grid;
  g->p = *p;
  g->device = device;
  g->stream = (hipStream_t)hip_stream;
  fill_ctx(p, g->C);
  const size_t tab = (size_t)g->C.npos;
  const size_t nd = tab * (GE_NCENTER + 2 * GE_NFACE);
  const size_t nint = (size_t)g->C.n[0] * g->C.n[1] * g->C.n[2];
  // [nd doubles][256 B: dt slot @0, list length @128, stats @192][cascade]
  // PPM: the flattener [3][gas, radiation][Ntot], and on Kerr-Schild the
  // per-cell mass fluxes it reads [6][Ntot]
  const size_t flat_n = (p->metric == GRRMHD_KERR_SCHILD) ? 12 : 6;
  const size_t flat_bytes =
      (p->recon == GRRMHD_RECON_PPM) ? round256(sizeof(double) * flat_n * (size_t)g->C.Ntot) : 0;
  // wavefront tiles of 16 x 4 cells in (x1, x2); 64 x 1 on one-dimensional grids
  g->tile_i = (g->C.n[1] > 1) ? GRRMHD_IMPLICIT_TILE_I : 64;
  {
    const int tj = 64 / g->tile_i;
    g->ntiles = (long)((g->C.n[0] + g->tile_i - 1) / g->tile_i) * ((g->C.n[1] + tj - 1) / tj) *
                g->C.n[2];
  }
  const size_t tile_bytes = 2 * round256(sizeof(int) * (size_t)g->ntiles);
  hipError_t e = hipMalloc(&g->geo, nd * sizeof(double) + TAIL_CASCADE + cascade_bytes(nint) +
                                        flat_bytes + tile_bytes);
  if (e != hipSuccess) {
    delete g;
    return fail(GRRMHD_ENOMEM, std::string("geometry allocation: ") + hipGetErrorString(e));
  }
  char* tail = (char*)(g->geo + nd);
  g->dtslot = (unsigned long long*)tail;
  g->dtstep[0] = (unsigned long long*)(tail + TAIL_DT0);
  g->dtstep[1] = (unsigned long long*)(tail + TAIL_DT1);
  g->cnt[0] = (int*)(tail + 128);
  g->cnt[1] = (int*)(tail + 160);
  g->W.counter = g->cnt[0];
  g->W.counter_next = nullptr;
  g->W.stats = (unsigned long long*)(tail + 192);
  cascade_layout(tail + TAIL_CASCADE, nint, g->W);
  {
    char* tb = tail + TAIL_CASCADE + cascade_bytes(nint) + flat_bytes;
    g->tkeys = (int*)tb;
    g->torder = (int*)(tb + round256(sizeof(int) * (size_t)g->ntiles));
  }
  if (flat_bytes) {
    // zero outside the flattener's range (cells within one of the interior):
    // the staggered field's face states two cells out read it there
    g->flat = (double*)(tail + TAIL_CASCADE + cascade_bytes(nint));
    e = hipMemsetAsync(g->flat, 0, flat_bytes, g->stream);
    if (e != hipSuccess) {
      (void)hipFree(g->geo);
      delete g;
      return fail(GRRMHD_EHIP, std::string("flattener set-up: ") + hipGetErrorString(e));
    }
  }
  g->C.geo_c = g->geo;
  g->C.geo_f1 = g->geo + tab * GE_NCENTER;
  g->C.geo_f2 = g->geo + tab * (GE_NCENTER + GE_NFACE);
  hipLaunchKernelGGL(k_geometry, dim3(nblocks(g->C.npos, 256)), dim3(256), 0, g->stream, g->C,
                     p->a, p->R0, g->geo, (double*)g->C.geo_f1, (double*)g->C.geo_f2);
  // both list lengths and the lane statistics (bytes 128..223 of the tail)
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, g->stream, (int*)(tail + 128), 24);
  // no costs known yet: the first launch takes the tiles in any order
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, g->stream, g->tkeys, (int)g->ntiles);
  hipLaunchKernelGGL(k_dt_init, dim3(1), dim3(64), 0, g->stream, g->dtslot, 1, 1);
  hipLaunchKernelGGL(k_dt_init, dim3(1), dim3(64), 0, g->stream, g->dtstep[0],
                     2 * GRRMHD_DT_SLOTS, GRRMHD_DT_STRIDE);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) {
    (void)hipFree(g->geo);
    delete g;
    return fail(GRRMHD_EHIP, std::string("geometry kernel: ") + hipGetErrorString(e));
  }
  *out = g;
  return 0;
}

extern "C" int grrmhd_free_grid(grrmhd_grid* g) {
  if (!g) return 0;
  HIPCHK(hipSetDevice(g->device));
  HIPCHK(hipStreamSynchronize(g->stream));
  if (g->ev) {
    for (int i = 0; i < 2 * grrmhd_grid::TCAP; i++) (void)hipEventDestroy(g->ev[i]);
    delete[] g->ev;
  }
  HIPCHK(hipFree(g->geo));
  delete g;
  return 0;
}

extern "C" int grrmhd_set_stream(grrmhd_grid* g, void* s) {
  if (!g) return fail(GRRMHD_EINVAL, "grid is NULL");
  g->stream = (hipStream_t)s;
  return 0;
}

extern "C" long grrmhd_ncell_alloc(const grrmhd_grid* g) { return g ? g->C.Ntot : -1; }

// workspace layout (doubles unless noted), each part 256-byte aligned
// ---------------------------------------------------------------------------
// Time integrators (Sec. 4.1) as stage tables.  Stage i:
//   U^i = a U^n + b U^j + c dt F^{i-1} + dt sum_k m_k M^k + g dt M(U^i),
// F^{i-1} the flux divergence and geometric source of the previous stage's
// primitives (of P^n at stage 0), M^k the 4-force source of stage k as its
// implicit solve found it.  g = 0 marks the final explicit combination (then
// inversions).
// ---------------------------------------------------------------------------
struct Stage {
  double a, b;
  int j;            // stage of the U^j term (-1: none)
  double c;
  double m[4];
  double g;
};

struct Scheme {
  int ns;
  Stage s[5];
  bool keep_m[4];   // M^k read by a later stage
};

static Scheme make_scheme(int which) {
  Scheme S;
  memset(&S, 0, sizeof(S));
  auto st = [&](double a, double b, int j, double c, double g, double m0 = 0.0, double m1 = 0.0,
                double m2 = 0.0, double m3 = 0.0) {
    Stage& x = S.s[S.ns++];
    x.a = a; x.b = b; x.j = j; x.c = c; x.g = g;
    x.m[0] = m0; x.m[1] = m1; x.m[2] = m2; x.m[3] = m3;
  };
  switch (which) {
    case GRRMHD_IMEX2: {            // eq. IMEX2
      const double gm = 1.0 - 1.0 / sqrt(2.0);
      st(1.0, 0.0, -1, 0.0, gm);
      st((3.0 * gm - 1.0) / gm, (1.0 - 2.0 * gm) / gm, 0, 1.0, gm);
      st(0.5, 0.5, 1, 0.5, 0.0, gm, 0.5 * (1.0 - gm));
      break;
    }
    case GRRMHD_IMEX2B:             // eq. IMEX2B
      st(1.0, 0.0, -1, 0.0, 0.25);
      st(1.0, 0.0, -1, 0.5, 0.25);
      st(0.0, 1.0, 1, 0.5, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 12.0);
      st(1.0 / 3.0, 2.0 / 3.0, 2, 1.0 / 3.0, 0.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0);
      break;
    case GRRMHD_IMEX3: {            // eq. IMEX3 with the printed alpha, beta, eta
      const double al = 0.24169426078821, be = 0.06042356519705, et = 0.12915286960590;
      st(1.0, 0.0, -1, 0.0, al);
      st(2.0, -1.0, 0, 0.0, al);
      st(1.0, 0.0, -1, 1.0, al, 0.0, 1.0 - al);
      st(0.75, 0.25, 2, 0.25, al, be, (-1.0 + al + 4.0 * et) / 4.0,
         (2.0 - 5.0 * al - 4.0 * (be + et)) / 4.0);
      st(1.0 / 3.0, 2.0 / 3.0, 3, 2.0 / 3.0, 0.0, -2.0 * be / 3.0, (1.0 - 4.0 * et) / 6.0,
         (-1.0 + 4.0 * al + 4.0 * (be + et)) / 6.0, 4.0 * (1.0 - al) / 6.0);
      break;
    }
    default:                        // RK3, implicit part with the same coefficients
      st(1.0, 0.0, -1, 1.0, 1.0);
      st(0.75, 0.25, 0, 0.25, 0.25);
      st(1.0 / 3.0, 2.0 / 3.0, 1, 2.0 / 3.0, 2.0 / 3.0);
      break;
  }
  for (int i = 0; i < S.ns; i++)
    for (int k = 0; k < 4; k++)
      if (S.s[i].m[k] != 0.0) S.keep_m[k] = true;
  return S;
}

struct WsLayout {
  size_t F, emf, vch, Uexp, Pa, Ua, err, st, it, Us, M, Fs, Sn, MS, VF, SP, Bs, total;
};

// IMEX schemes add the stage U's (all but the last) and the kept M^k
static WsLayout ws_layout(const Ctx& C, int scheme = GRRMHD_RK3) {
  WsLayout w;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t N = (size_t)C.Ntot;
  w.F = take(sizeof(double) * 36 * N);
  w.emf = take(sizeof(double) * 3 * N);
  w.vch = take(sizeof(double) * 3 * N);
  w.Uexp = take(sizeof(double) * 13 * N);
  w.Pa = take(sizeof(double) * 12 * N);
  w.Ua = take(sizeof(double) * 12 * N);
  w.err = take(sizeof(double) * N);
  w.st = take(sizeof(int) * N);
  w.it = take(sizeof(int) * N);
  w.Us = w.M = off;
  if (scheme != GRRMHD_RK3) {
    const Scheme S = make_scheme(scheme);
    w.Us = take(round256(sizeof(double) * 12 * N) * (S.ns - 1));
    w.M = take(round256(sizeof(double) * 8 * N) * 4);
  }
  // the full cascade's entropy tracer: face fluxes and U_S(P^n); in the IMEX
  // tables also the stored entropy sources M_S^k
  w.Fs = w.Sn = w.MS = off;
  if (C.cascade) {
    w.Fs = take(sizeof(double) * 3 * N);
    w.Sn = take(sizeof(double) * N);
    if (scheme != GRRMHD_RK3) w.MS = take(round256(sizeof(double) * N) * 4);
  }
  // the staggered field: face velocities and speeds, and the faces of every
  // stage but the last (which writes the caller's faces in place)
  w.VF = w.SP = w.Bs = off;
  if (C.ct) {
    const int ns = (scheme == GRRMHD_RK3) ? 3 : make_scheme(scheme).ns;
    w.VF = take(sizeof(double) * 18 * N);
    w.SP = take(sizeof(double) * 6 * N);
    w.Bs = take(round256(sizeof(double) * 3 * N) * (ns - 1));
  }
  w.total = off;
  return w;
}

extern "C" size_t grrmhd_workspace_bytes(const grrmhd_grid* g) {
  return g ? ws_layout(g->C, g->p.scheme).total : 0;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
static int launch_bc(grrmhd_grid* g, double* P) {
  const Ctx& C = g->C;
  hipLaunchKernelGGL(k_bc_all, dim3(nblocks(C.Ntot, 256)), dim3(256), 0, g->stream, C, P);
  LAUNCHCHK();
  return 0;
}

// faces normal to d: n + 1 along d; across it one cell beyond the interior
// (ext = 1), or two for the staggered field's corner interpolation (ext = 2)
static FaceRange face_range(const Ctx& C, int d, int ext = 1) {
  FaceRange R;
  R.total = 1;
  for (int e = 0; e < 3; e++) {
    if (e == d) { R.lo[e] = C.ng[e]; R.cnt[e] = C.n[e] + 1; }
    else if (C.n[e] > 1) { R.lo[e] = C.ng[e] - ext; R.cnt[e] = C.n[e] + 2 * ext; }
    else { R.lo[e] = 0; R.cnt[e] = 1; }
    R.total *= R.cnt[e];
  }
  return R;
}

static FaceRange edge_range(const Ctx& C, int a) {
  FaceRange R;
  R.total = 1;
  for (int e = 0; e < 3; e++) {
    if (e == a) { R.lo[e] = C.ng[e]; R.cnt[e] = C.n[e]; }
    else { R.lo[e] = C.ng[e]; R.cnt[e] = C.n[e] + 1; }
    R.total *= R.cnt[e];
  }
  return R;
}

// Split a range at x1 index i0: [lo, i0) and [i0, hi) (either may be empty).
static void split_x1(const FaceRange& R, int i0, FaceRange& a, FaceRange& b) {
  a = b = R;
  const int cut = std::min(std::max(i0, R.lo[0]), R.lo[0] + R.cnt[0]);
  a.cnt[0] = cut - R.lo[0];
  b.lo[0] = cut;
  b.cnt[0] = R.lo[0] + R.cnt[0] - cut;
  a.total = (long)a.cnt[0] * a.cnt[1] * a.cnt[2];
  b.total = (long)b.cnt[0] * b.cnt[1] * b.cnt[2];
}

// dtmin set: the Courant reduction over interior cells runs in the EMF launch.
// PPM: the flattener of P first; keep_flat: the larger of it and the step's
// earlier sub-steps' (0 at a step's first flux evaluation).
// Bf (staggered field): the face states take the faces' normal field, write
// their velocities and speeds to VF, SP, and the corner EMFs are the
// four-state ones.
// PPM flattener of P into the grid's buffer (keep_flat as launch_fluxes)
static int launch_flattener(grrmhd_grid* g, const double* P, const double* ca, const double* ce,
                            int keep_flat) {
  const Ctx& C = g->C;
  double* mf = nullptr;
  if (C.metric == GRRMHD_KERR_SCHILD) {
    mf = g->flat + 6 * (size_t)C.Ntot;
    hipLaunchKernelGGL(k_mass_flux, dim3(nblocks(C.Ntot, 256)), dim3(256), 0, g->stream, C, P, mf);
    LAUNCHCHK();
  }
  long nb = 1;   // (cell, active direction) pairs
  int nd = 0;
  for (int e = 0; e < 3; e++) {
    nb *= C.n[e] > 1 ? C.n[e] + 2 : 1;
    nd += C.n[e] > 1;
  }
  nb *= nd;
  if (nb == 0) return 0;
  hipLaunchKernelGGL(k_flatten, dim3(nblocks(nb, 256)), dim3(256), 0, g->stream, C, P, ca, ce,
                     g->flat, keep_flat, (const double*)mf);
  LAUNCHCHK();
  return 0;
}

static int launch_fluxes(grrmhd_grid* g, const double* P, const double* ca, const double* ce,
                         double* F, double* emf, double* vch,
                         unsigned long long* dtmin = nullptr, int keep_flat = 0,
                         double* Fs = nullptr, const double* Bf = nullptr, double* VF = nullptr,
                         double* SP = nullptr) {
  const Ctx& C = g->C;
  if (C.recon == GRRMHD_RECON_PPM) {
    const int rc = launch_flattener(g, P, ca, ce, keep_flat);
    if (rc) return rc;
  }
  // faces of every direction, FP64 part and FP32 part (split at mixed_i)
  FluxSegs S64, S32;
  S64.n = S32.n = 0;
  S64.total = S32.total = 0;
  for (int d = 0; d < 3; d++) {
    if (C.n[d] == 1) continue;
    FaceRange r64, r32;
    split_x1(face_range(C, d, Bf ? 2 : 1), C.mixed_i, r64, r32);
    if (r64.total > 0) {
      S64.R[S64.n] = r64; S64.D[S64.n] = d + 1; S64.start[S64.n] = S64.total;
      S64.total += r64.total; S64.n++;
    }
    if (r32.total > 0) {
      S32.R[S32.n] = r32; S32.D[S32.n] = d + 1; S32.start[S32.n] = S32.total;
      S32.total += r32.total; S32.n++;
    }
  }
  if (Bf) {
    const double* flp = (const double*)g->flat;
    if (S64.total > 0) {
      if (Fs)
        hipLaunchKernelGGL((k_flux_all_stag<double, true>), dim3(nblocks(S64.total, 128)), dim3(128),
                           0, g->stream, C, S64, P, ca, ce, F, vch, flp, Fs, Bf, VF, SP);
      else
        hipLaunchKernelGGL((k_flux_all_stag<double, false>), dim3(nblocks(S64.total, 128)),
                           dim3(128), 0, g->stream, C, S64, P, ca, ce, F, vch, flp, Fs, Bf, VF, SP);
      LAUNCHCHK();
    }
    if (S32.total > 0) {
      if (Fs)
        hipLaunchKernelGGL((k_flux_all_stag<float, true>), dim3(nblocks(S32.total, 128)), dim3(128),
                           0, g->stream, C, S32, P, ca, ce, F, vch, flp, Fs, Bf, VF, SP);
      else
        hipLaunchKernelGGL((k_flux_all_stag<float, false>), dim3(nblocks(S32.total, 128)),
                           dim3(128), 0, g->stream, C, S32, P, ca, ce, F, vch, flp, Fs, Bf, VF, SP);
      LAUNCHCHK();
    }
    // four-state corner EMFs at [ng, ng+n] on each active axis
    FaceRange R;
    R.total = 1;
    for (int e = 0; e < 3; e++) {
      R.lo[e] = C.ng[e];
      R.cnt[e] = C.n[e] > 1 ? C.n[e] + 1 : 1;
      R.total *= R.cnt[e];
    }
    if (dtmin) {
      const long n = std::max<long>(R.total, (long)C.n[0] * C.n[1] * C.n[2]);
      hipLaunchKernelGGL(k_emf_stag_dt, dim3(nblocks(n, 256)), dim3(256), 0, g->stream, C, R, Bf,
                         (const double*)VF, (const double*)SP, emf, (const double*)vch, dtmin);
    } else {
      hipLaunchKernelGGL(k_emf_stag, dim3(nblocks(R.total, 256)), dim3(256), 0, g->stream, C, R,
                         Bf, (const double*)VF, (const double*)SP, emf);
    }
    LAUNCHCHK();
    return 0;
  }
  if (S64.total > 0) {
    if (Fs)
      hipLaunchKernelGGL(k_flux_all_s<double>, dim3(nblocks(S64.total, 128)), dim3(128), 0,
                         g->stream, C, S64, P, ca, ce, F, vch, (const double*)g->flat, Fs);
    else
      hipLaunchKernelGGL(k_flux_all<double>, dim3(nblocks(S64.total, 128)), dim3(128), 0,
                         g->stream, C, S64, P, ca, ce, F, vch, (const double*)g->flat);
    LAUNCHCHK();
  }
  if (S32.total > 0) {
    if (Fs)
      hipLaunchKernelGGL(k_flux_all_s<float>, dim3(nblocks(S32.total, 128)), dim3(128), 0,
                         g->stream, C, S32, P, ca, ce, F, vch, (const double*)g->flat, Fs);
    else
      hipLaunchKernelGGL(k_flux_all<float>, dim3(nblocks(S32.total, 128)), dim3(128), 0,
                         g->stream, C, S32, P, ca, ce, F, vch, (const double*)g->flat);
    LAUNCHCHK();
  }
  // corner EMFs: union of the edge ranges (n + 1 positions along active axes)
  bool any = false;
  for (int a = 0; a < 3; a++) any = any || (C.n[(a + 1) % 3] > 1 && C.n[(a + 2) % 3] > 1);
  FaceRange R;
  R.total = 1;
  for (int e = 0; e < 3; e++) {
    R.lo[e] = C.ng[e];
    R.cnt[e] = C.n[e] > 1 ? C.n[e] + 1 : 1;
    R.total *= R.cnt[e];
  }
  if (!any) R.total = 0;
  if (dtmin) {
    const long n = std::max<long>(R.total, (long)C.n[0] * C.n[1] * C.n[2]);
    hipLaunchKernelGGL(k_emf_dt, dim3(nblocks(n, 256)), dim3(256), 0, g->stream, C, R, F, emf, vch,
                       dtmin);
    LAUNCHCHK();
  } else if (any) {
    hipLaunchKernelGGL(k_emf_all, dim3(nblocks(R.total, 256)), dim3(256), 0, g->stream, C, R, F,
                       emf);
    LAUNCHCHK();
  }
  return 0;
}

static long n_interior(const Ctx& C) { return (long)C.n[0] * C.n[1] * C.n[2]; }

static int launch_timestep(grrmhd_grid* g, const double* vch, double* dt_dev) {
  const Ctx& C = g->C;
  hipLaunchKernelGGL(k_dt_init, dim3(1), dim3(64), 0, g->stream, g->dtslot, 1, 1);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_dt_min, dim3(nblocks(n_interior(C), 256)), dim3(256), 0, g->stream, C, vch,
                     g->dtslot);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(1), 0, g->stream, g->dtslot, C.courant, dt_dev);
  LAUNCHCHK();
  return 0;
}

// dtmin set: dt = courant x *dtmin, stored in *dt_dev; *dtnext reset to +inf
static int launch_update(grrmhd_grid* g, double a, double b, double c, const double* dt_dev,
                         const double* P, const double* Un, const double* Up, const double* F,
                         const double* emf, double* Ue, const unsigned long long* dtmin = nullptr,
                         unsigned long long* dtnext = nullptr, const MTerms* mt = nullptr,
                         const double* Bface = nullptr) {
  MTerms MT;
  memset(&MT, 0, sizeof(MT));
  if (mt) MT = *mt;
  hipLaunchKernelGGL(k_update, dim3(nblocks(n_interior(g->C), 256)), dim3(256), 0, g->stream,
                     g->C, a, b, c, const_cast<double*>(dt_dev), dtmin, dtnext, P, Un, Up, F, emf,
                     MT, Ue, Bface);
  LAUNCHCHK();
  return 0;
}

// fallback grid: enough waves to spread a long list, grid-stride beyond
static unsigned list_blocks(long n) { return (unsigned)std::min<long>(nblocks(n, 64), 8192); }

static int launch_implicit(grrmhd_grid* g, const double* Ue, const double* Pg, double scale,
                           const double* dt_dev, const double* ca, const double* ce, double* P,
                           double* U, int* it, int* st, double* err,
                           const double* Sexp = nullptr) {
  const long n = n_interior(g->C);
  // this launch appends to cnt[cp] (zero: set at creation or by the previous
  // launch's cascade kernel) and its cascade kernel zeroes cnt[cp ^ 1]
  Work W = g->W;
  W.counter = g->cnt[g->cp];
  W.counter_next = g->cnt[g->cp ^ 1];
  const bool timed = g->timing && g->nt < grrmhd_grid::TCAP;
  // tiles costliest first by the previous launch's trip counts
  hipLaunchKernelGGL(k_tile_order, dim3(9), dim3(1024), 0, g->stream, g->ntiles,
                     (const int*)g->tkeys, g->torder);
  LAUNCHCHK();
  if (timed) HIPCHK(hipEventRecord(g->ev[2 * g->nt], g->stream));
  hipLaunchKernelGGL(k_implicit, dim3((unsigned)g->ntiles), dim3(64), 0, g->stream, g->C,
                     g->tile_i, Ue, Pg, scale, dt_dev, ca, ce, P, U, it, st, err, W,
                     (const int*)g->torder, g->tkeys);
  LAUNCHCHK();
  if (timed) {
    HIPCHK(hipEventRecord(g->ev[2 * g->nt + 1], g->stream));
    g->nt++;
  }
  if (g->C.cascade)
    hipLaunchKernelGGL(k_implicit_list<true>, dim3(list_blocks(n)), dim3(64), 0, g->stream, g->C,
                       Ue, Pg, scale, dt_dev, ca, ce, P, U, it, st, err, W, Sexp);
  else
    hipLaunchKernelGGL(k_implicit_list<false>, dim3(list_blocks(n)), dim3(64), 0, g->stream, g->C,
                       Ue, Pg, scale, dt_dev, ca, ce, P, U, it, st, err, W, Sexp);
  LAUNCHCHK();
  g->W.counter = W.counter;
  g->cp ^= 1;
  return 0;
}

static int launch_fixup(grrmhd_grid* g, double* P, double* U, int* st, double* scr, int* st_acc,
                        const int* it_stage, int* it_acc, int accumulate) {
  const long n = n_interior(g->C);
  hipLaunchKernelGGL(k_fixup_avg, dim3(nblocks(n, 256)), dim3(256), 0, g->stream, g->C, P, st, scr);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_fixup_apply, dim3(nblocks(n, 256)), dim3(256), 0, g->stream, g->C, P, U, st,
                     scr, st_acc, it_stage, it_acc, accumulate);
  LAUNCHCHK();
  return 0;
}

#define NEEDG()                                               \
  do {                                                        \
    if (!g) return fail(GRRMHD_EINVAL, "grid is NULL");       \
    HIPCHK(hipSetDevice(g->device));                          \
  } while (0)

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
extern "C" int grrmhd_prim_to_cons(grrmhd_grid* g, const double* P, double* U) {
  NEEDG();
  if (!P || !U) return fail(GRRMHD_EINVAL, "NULL array");
  hipLaunchKernelGGL(k_p2u, dim3(nblocks(g->C.Ntot, 256)), dim3(256), 0, g->stream, g->C, P, U);
  LAUNCHCHK();
  return 0;
}

extern "C" int grrmhd_apply_bc(grrmhd_grid* g, double* P) {
  NEEDG();
  if (!P) return fail(GRRMHD_EINVAL, "NULL array");
  return launch_bc(g, P);
}

extern "C" int grrmhd_fluxes(grrmhd_grid* g, const double* P, const double* chi_abs,
                             const double* chi_es, double* F, double* emf, double* vchar) {
  NEEDG();
  if (!P || !chi_abs || !chi_es || !F || !emf || !vchar) return fail(GRRMHD_EINVAL, "NULL array");
  const size_t N = (size_t)g->C.Ntot;
  HIPCHK(hipMemsetAsync(F, 0, sizeof(double) * 36 * N, g->stream));
  HIPCHK(hipMemsetAsync(emf, 0, sizeof(double) * 3 * N, g->stream));
  HIPCHK(hipMemsetAsync(vchar, 0, sizeof(double) * 3 * N, g->stream));
  return launch_fluxes(g, P, chi_abs, chi_es, F, emf, vchar);
}

extern "C" int grrmhd_timestep(grrmhd_grid* g, const double* vchar, double* dt_dev) {
  NEEDG();
  if (!vchar || !dt_dev) return fail(GRRMHD_EINVAL, "NULL array");
  return launch_timestep(g, vchar, dt_dev);
}

extern "C" int grrmhd_explicit_update(grrmhd_grid* g, double a, double b, double c,
                                      const double* dt_dev, const double* P, const double* Un,
                                      const double* Uprev, const double* F, const double* emf,
                                      double* Uexp) {
  NEEDG();
  if (!dt_dev || !P || !Un || !F || !emf || !Uexp || (b != 0.0 && !Uprev))
    return fail(GRRMHD_EINVAL, "NULL array");
  return launch_update(g, a, b, c, dt_dev, P, Un, Uprev, F, emf, Uexp);
}

extern "C" int grrmhd_con2prim(grrmhd_grid* g, const double* U, const double* Pguess, double* P,
                               int* status) {
  NEEDG();
  if (!U || !Pguess || !P) return fail(GRRMHD_EINVAL, "NULL array");
  hipLaunchKernelGGL(k_con2prim, dim3(nblocks(n_interior(g->C), 128)), dim3(128), 0, g->stream,
                     g->C, U, Pguess, P, status, 0);
  LAUNCHCHK();
  return 0;
}

extern "C" int grrmhd_implicit_grid(grrmhd_grid* g, const double* Uexp, const double* Pguess,
                                    double dt_scale, const double* dt_dev, const double* chi_abs,
                                    const double* chi_es, double* P, double* U, int* iters,
                                    int* status, double* err) {
  NEEDG();
  if (!Uexp || !Pguess || !dt_dev || !chi_abs || !chi_es || !P || !U)
    return fail(GRRMHD_EINVAL, "NULL array");
  if (U == Uexp) return fail(GRRMHD_EINVAL, "U may not alias Uexp");
  return launch_implicit(g, Uexp, Pguess, dt_scale, dt_dev, chi_abs, chi_es, P, U, iters, status, err);
}

extern "C" int grrmhd_fixup(grrmhd_grid* g, double* P, double* U, int* status, double* scratch) {
  NEEDG();
  if (!P || !U || !status || !scratch) return fail(GRRMHD_EINVAL, "NULL array");
  return launch_fixup(g, P, U, status, scratch, nullptr, nullptr, nullptr, 0);
}

// One step of an IMEX scheme (stage table above).  The latest primitives
// live in P (stage input of stage 0) or Pa; stage U's in the workspace; the
// last stage writes P and U.
// One step of an IMEX stage table; Bf: the staggered field (the faces of
// each stage a Bf^n + b Bf^(j) + c dt (-curl EMF), no EMF term where c = 0;
// stage faces in the workspace, the last stage's written to Bf in place),
// else null.
static int imex_step(grrmhd_grid* g, double* P, double* U, double* Bf, const double* chi_abs,
                     const double* chi_es, double* dt_dev, int dt_fixed, int* status, int* iters,
                     char* base, const WsLayout& w) {
  const Ctx& C = g->C;
  const Scheme S = make_scheme(g->p.scheme);
  const size_t N = (size_t)C.Ntot;
  double* F = (double*)(base + w.F);
  double* emf = (double*)(base + w.emf);
  double* vch = (double*)(base + w.vch);
  double* Ue = (double*)(base + w.Uexp);
  double* Pa = (double*)(base + w.Pa);
  double* err = (double*)(base + w.err);
  int* st = (int*)(base + w.st);
  int* it = (int*)(base + w.it);
  double* Us[4];
  double* Mk[4];
  for (int k = 0; k < 4; k++) {
    Us[k] = (double*)(base + w.Us + k * round256(sizeof(double) * 12 * N));
    Mk[k] = (double*)(base + w.M + k * round256(sizeof(double) * 8 * N));
  }
  const long nint = n_interior(C);
  double* VF = Bf ? (double*)(base + w.VF) : nullptr;
  double* SP = Bf ? (double*)(base + w.SP) : nullptr;
  const size_t b3 = round256(sizeof(double) * 3 * N);
  auto Bst = [&](int i) { return (i == S.ns - 1) ? Bf : (double*)(base + w.Bs + i * b3); };
  FaceRange RF;
  RF.total = 1;
  for (int e = 0; e < 3; e++) {
    RF.lo[e] = C.ng[e];
    RF.cnt[e] = C.n[e] > 1 ? C.n[e] + 1 : 1;
    RF.total *= RF.cnt[e];
  }
  // the full cascade's entropy tracer: U_S(P^n), the stage's face fluxes and
  // explicit value (row 12 of the explicit state, free until the fix-ups),
  // and the stored entropy sources
  double* Fs = C.cascade ? (double*)(base + w.Fs) : nullptr;
  double* Sn = C.cascade ? (double*)(base + w.Sn) : nullptr;
  double* Sexp = C.cascade ? Ue + 12 * N : nullptr;
  // the tracer's b term is taken from the stage input's primitives, so it
  // must be the previous stage's (it is in every table)
  for (int i = 0; C.cascade && i < S.ns; i++)
    if (S.s[i].g > 0.0 && S.s[i].b != 0.0 && S.s[i].j != i - 1)
      return fail(GRRMHD_EINVAL, "entropy tracer: a stage's b term must take the previous stage");
  const size_t b1 = round256(sizeof(double) * N);
  auto MSk = [&](int k) { return (double*)(base + w.MS + k * b1); };
  if (C.cascade) {
    hipLaunchKernelGGL(k_entropy_field, dim3(nblocks(nint, 256)), dim3(256), 0, g->stream, C, P, Sn);
    LAUNCHCHK();
  }
  double* Pcur = P;
  double* Bcur = Bf;   // the faces of Pcur
  int rc, nflux = 0;
  for (int i = 0; i < S.ns; i++) {
    const Stage& x = S.s[i];
    const bool last = (i == S.ns - 1);
    // dt from the wave speeds of P^n: the Courant reduction rides on the
    // first flux launch (made for it even when stage 0 has no explicit flux)
    const bool red = (i == 0 && !dt_fixed);
    unsigned long long* dmin = red ? g->dtstep[g->dtp] : nullptr;
    unsigned long long* dnext = red ? g->dtstep[g->dtp ^ 1] : nullptr;
    if (x.c != 0.0 || red) {
      if ((rc = launch_bc(g, Pcur))) return rc;
      if (Bf) {
        hipLaunchKernelGGL(k_bc_faces, dim3(nblocks(3 * C.Ntot, 256)), dim3(256), 0, g->stream, C,
                           Bcur);
        LAUNCHCHK();
      }
      if ((rc = launch_fluxes(g, Pcur, chi_abs, chi_es, F, emf, vch, dmin, nflux > 0, Fs, Bcur,
                              VF, SP)))
        return rc;
      nflux++;
    }
    if (Bf) {
      // the stage's faces (before the cell update, which averages them); Bf
      // is still Bf^n here (only the last stage writes it, face by face)
      hipLaunchKernelGGL(k_face_update, dim3(nblocks(RF.total, 256)), dim3(256), 0, g->stream, C,
                         RF, x.a, x.b, x.c, (const double*)dt_dev, (const unsigned long long*)dmin,
                         (const double*)Bf, (const double*)(x.j >= 0 ? Bst(x.j) : Bf),
                         (const double*)emf, Bst(i));
      LAUNCHCHK();
    }
    MTerms MT;
    memset(&MT, 0, sizeof(MT));
    for (int k = 0; k < i && k < 4; k++) {
      if (x.m[k] == 0.0) continue;
      MT.M[MT.n] = Mk[k];
      MT.m[MT.n] = x.m[k];
      MT.n++;
    }
    const double* Uj = (x.j >= 0) ? Us[x.j] : U;
    if ((rc = launch_update(g, x.a, x.b, x.c, dt_dev, Pcur, U, Uj, F, emf, Ue, dmin, dnext, &MT,
                            Bf ? Bst(i) : nullptr)))
      return rc;
    if (red) g->dtp ^= 1;
    if (C.cascade && x.g > 0.0) {
      // the b term's stage is the previous one (checked above): Pcur
      hipLaunchKernelGGL(k_entropy_update, dim3(nblocks(nint, 256)), dim3(256), 0, g->stream, C,
                         x.a, x.b, x.c, (const double*)dt_dev, (const double*)Sn,
                         (const double*)Pcur, (const double*)Fs, Sexp);
      LAUNCHCHK();
      if (MT.n > 0) {
        MTerms MS = MT;
        for (int q = 0, k = 0; k < i && k < 4; k++)
          if (x.m[k] != 0.0) MS.M[q++] = MSk(k);
        hipLaunchKernelGGL(k_entropy_mterms, dim3(nblocks(nint, 256)), dim3(256), 0, g->stream, C,
                           MS, (const double*)dt_dev, Sexp);
        LAUNCHCHK();
      }
    }
    double* Pout = last ? P : Pa;
    double* Uout = last ? U : Us[i];
    if (x.g > 0.0) {
      if ((rc = launch_implicit(g, Ue, Pcur, x.g, dt_dev, chi_abs, chi_es, Pout, Uout, it, st, err,
                                Sexp)))
        return rc;
      if (i < 4 && S.keep_m[i]) {   // the stage's source, before the fix-ups
        hipLaunchKernelGGL(k_stage_m, dim3(nblocks(nint, 256)), dim3(256), 0, g->stream, C, Ue,
                           Uout, st, x.g, dt_dev, Mk[i]);
        LAUNCHCHK();
        if (C.cascade) {
          hipLaunchKernelGGL(k_stage_ms, dim3(nblocks(nint, 256)), dim3(256), 0, g->stream, C,
                             (const double*)Pout, (const double*)Sexp, (const int*)st, x.g,
                             (const double*)dt_dev, MSk(i));
          LAUNCHCHK();
        }
      }
      if ((rc = launch_fixup(g, Pout, Uout, st, Ue, status, it, iters, i > 0))) return rc;
    } else {
      // final explicit combination: MHD and radiation inversions; a failed
      // MHD inversion makes a failed cell (neighbour average in the fix-up)
      hipLaunchKernelGGL(k_con2prim, dim3(nblocks(nint, 128)), dim3(128), 0, g->stream, C, Ue,
                         Pcur, Pout, st, (int)GRRMHD_ST_FAIL);
      LAUNCHCHK();
      hipLaunchKernelGGL(k_copy_interior12, dim3(nblocks(nint, 256)), dim3(256), 0, g->stream, C,
                         Ue, Uout);
      LAUNCHCHK();
      if ((rc = launch_fixup(g, Pout, Uout, st, Ue, status, nullptr, iters, i > 0))) return rc;
    }
    Pcur = Pout;
    Bcur = Bf ? Bst(i) : nullptr;
  }
  return 0;
}

// One RK3 step; Bf: the staggered field (stage faces in the workspace, the
// last stage written to Bf in place), else null.
static int rk3_step(grrmhd_grid* g, double* P, double* U, double* Bf, const double* chi_abs,
                    const double* chi_es, double* dt_dev, int dt_fixed, int* status, int* iters,
                    char* base, const WsLayout& w) {
  const Ctx& C = g->C;
  double* F = (double*)(base + w.F);
  double* emf = (double*)(base + w.emf);
  double* vch = (double*)(base + w.vch);
  double* Ue = (double*)(base + w.Uexp);
  double* Pa = (double*)(base + w.Pa);
  double* Ua = (double*)(base + w.Ua);
  double* err = (double*)(base + w.err);
  int* st = (int*)(base + w.st);
  int* it = (int*)(base + w.it);
  const size_t N = (size_t)C.Ntot;
  // Shu-Osher RK3: U(k) = a U^n + b U(k-1) + c dt (X + M(U(k)))
  const double A[3] = {1.0, 0.75, 1.0 / 3.0}, B[3] = {0.0, 0.25, 2.0 / 3.0},
               Cc[3] = {1.0, 0.25, 2.0 / 3.0};
  int rc;
  // the full cascade's entropy tracer: U_S(P^n), per stage its face fluxes and
  // explicit value (row 12 of the explicit state, free until the fix-ups)
  double* Fs = C.cascade ? (double*)(base + w.Fs) : nullptr;
  double* Sn = C.cascade ? (double*)(base + w.Sn) : nullptr;
  double* Sexp = C.cascade ? Ue + 12 * N : nullptr;
  const long nint = n_interior(C);
  if (C.cascade) {
    hipLaunchKernelGGL(k_entropy_field, dim3(nblocks(nint, 256)), dim3(256), 0, g->stream, C, P, Sn);
    LAUNCHCHK();
  }
  // staggered field: stage inputs Bf, B1, B2; outputs B1, B2, Bf
  double* VF = Bf ? (double*)(base + w.VF) : nullptr;
  double* SP = Bf ? (double*)(base + w.SP) : nullptr;
  const size_t b3 = round256(sizeof(double) * 3 * N);
  double* Bst[3] = {Bf ? (double*)(base + w.Bs) : nullptr, Bf ? (double*)(base + w.Bs + b3) : nullptr,
                    Bf};
  FaceRange RF;
  RF.total = 1;
  for (int e = 0; e < 3; e++) {
    RF.lo[e] = C.ng[e];
    RF.cnt[e] = C.n[e] > 1 ? C.n[e] + 1 : 1;
    RF.total *= RF.cnt[e];
  }
  for (int s = 0; s < 3; s++) {
    double* Pin = (s == 0) ? P : Pa;
    const double* Uprev = (s == 0) ? U : Ua;
    double* Pout = (s == 2) ? P : Pa;
    double* Uout = (s == 2) ? U : Ua;
    double* Bin = Bf ? ((s == 0) ? Bf : Bst[s - 1]) : nullptr;
    if ((rc = launch_bc(g, Pin))) return rc;
    if (Bf) {
      hipLaunchKernelGGL(k_bc_faces, dim3(nblocks(3 * C.Ntot, 256)), dim3(256), 0, g->stream, C,
                         Bin);
      LAUNCHCHK();
    }
    // stage 1 without a fixed dt: the Courant reduction rides on the EMF launch
    // and the update takes dt from it (dtstep alternates between steps)
    const bool red = (s == 0 && !dt_fixed);
    unsigned long long* dmin = red ? g->dtstep[g->dtp] : nullptr;
    unsigned long long* dnext = red ? g->dtstep[g->dtp ^ 1] : nullptr;
    if ((rc = launch_fluxes(g, Pin, chi_abs, chi_es, F, emf, vch, dmin, s > 0, Fs, Bin, VF, SP)))
      return rc;
    if (Bf) {
      // the stage's faces (before the cell update, which averages them)
      hipLaunchKernelGGL(k_face_update, dim3(nblocks(RF.total, 256)), dim3(256), 0, g->stream, C,
                         RF, A[s], B[s], Cc[s], (const double*)dt_dev,
                         (const unsigned long long*)dmin, (const double*)Bf,
                         (const double*)(s > 0 ? Bst[s - 1] : nullptr), (const double*)emf,
                         Bst[s]);
      LAUNCHCHK();
    }
    if ((rc = launch_update(g, A[s], B[s], Cc[s], dt_dev, Pin, U, Uprev, F, emf, Ue, dmin, dnext,
                            nullptr, Bf ? Bst[s] : nullptr)))
      return rc;
    if (red) g->dtp ^= 1;
    if (C.cascade) {
      hipLaunchKernelGGL(k_entropy_update, dim3(nblocks(nint, 256)), dim3(256), 0, g->stream, C,
                         A[s], B[s], Cc[s], (const double*)dt_dev, (const double*)Sn,
                         (const double*)Pin, (const double*)Fs, Sexp);
      LAUNCHCHK();
    }
    if ((rc = launch_implicit(g, Ue, Pin, Cc[s], dt_dev, chi_abs, chi_es, Pout, Uout, it, st, err,
                              Sexp)))
      return rc;
    if ((rc = launch_fixup(g, Pout, Uout, st, Ue, status, it, iters, s > 0))) return rc;
  }
  return 0;
}

static int step_args(grrmhd_grid* g, void* workspace, size_t ws_bytes, WsLayout& w) {
  w = ws_layout(g->C, g->p.scheme);
  if (ws_bytes < w.total) return fail(GRRMHD_EINVAL, "workspace too small");
  if (((uintptr_t)workspace) & 255) return fail(GRRMHD_EINVAL, "workspace must be 256-byte aligned");
  return 0;
}

extern "C" int grrmhd_step(grrmhd_grid* g, double* P, double* U, const double* chi_abs,
                           const double* chi_es, double* dt_dev, int dt_fixed, int* status,
                           int* iters, void* workspace, size_t ws_bytes) {
  NEEDG();
  if (!P || !U || !chi_abs || !chi_es || !dt_dev || !workspace)
    return fail(GRRMHD_EINVAL, "NULL array");
  if (g->C.ct) return fail(GRRMHD_EINVAL, "a staggered-field grid steps with grrmhd_step_staggered");
  WsLayout w;
  int rc = step_args(g, workspace, ws_bytes, w);
  if (rc) return rc;
  char* base = (char*)workspace;
  if (g->p.scheme != GRRMHD_RK3)
    return imex_step(g, P, U, nullptr, chi_abs, chi_es, dt_dev, dt_fixed, status, iters, base, w);
  return rk3_step(g, P, U, nullptr, chi_abs, chi_es, dt_dev, dt_fixed, status, iters, base, w);
}

extern "C" int grrmhd_step_staggered(grrmhd_grid* g, double* P, double* U, double* Bf,
                                     const double* chi_abs, const double* chi_es, double* dt_dev,
                                     int dt_fixed, int* status, int* iters, void* workspace,
                                     size_t ws_bytes) {
  NEEDG();
  if (!P || !U || !Bf || !chi_abs || !chi_es || !dt_dev || !workspace)
    return fail(GRRMHD_EINVAL, "NULL array");
  if (!g->C.ct) return fail(GRRMHD_EINVAL, "grid has the flux-CT field (ct = GRRMHD_CT_FLUX)");
  WsLayout w;
  int rc = step_args(g, workspace, ws_bytes, w);
  if (rc) return rc;
  char* base = (char*)workspace;
  if (g->p.scheme != GRRMHD_RK3)
    return imex_step(g, P, U, Bf, chi_abs, chi_es, dt_dev, dt_fixed, status, iters, base, w);
  return rk3_step(g, P, U, Bf, chi_abs, chi_es, dt_dev, dt_fixed, status, iters, base, w);
}

extern "C" int grrmhd_apply_bc_faces(grrmhd_grid* g, double* Bf) {
  NEEDG();
  if (!Bf) return fail(GRRMHD_EINVAL, "NULL array");
  if (!g->C.ct) return fail(GRRMHD_EINVAL, "grid has the flux-CT field (ct = GRRMHD_CT_FLUX)");
  hipLaunchKernelGGL(k_bc_faces, dim3(nblocks(3 * g->C.Ntot, 256)), dim3(256), 0, g->stream, g->C,
                     Bf);
  LAUNCHCHK();
  return 0;
}

extern "C" int grrmhd_face_to_center(grrmhd_grid* g, const double* Bf, double* P, double* U) {
  NEEDG();
  if (!Bf || (!P && !U)) return fail(GRRMHD_EINVAL, "NULL array");
  if (!g->C.ct) return fail(GRRMHD_EINVAL, "grid has the flux-CT field (ct = GRRMHD_CT_FLUX)");
  hipLaunchKernelGGL(k_face_center, dim3(nblocks(n_interior(g->C), 256)), dim3(256), 0, g->stream,
                     g->C, Bf, P, U);
  LAUNCHCHK();
  return 0;
}

extern "C" int grrmhd_fluxes_staggered(grrmhd_grid* g, const double* P, const double* Bf,
                                       const double* chi_abs, const double* chi_es, double* F,
                                       double* emf, double* vchar, void* workspace,
                                       size_t ws_bytes) {
  NEEDG();
  if (!P || !Bf || !chi_abs || !chi_es || !F || !emf || !vchar || !workspace)
    return fail(GRRMHD_EINVAL, "NULL array");
  if (!g->C.ct) return fail(GRRMHD_EINVAL, "grid has the flux-CT field (ct = GRRMHD_CT_FLUX)");
  WsLayout w;
  int rc = step_args(g, workspace, ws_bytes, w);
  if (rc) return rc;
  const size_t N = (size_t)g->C.Ntot;
  HIPCHK(hipMemsetAsync(F, 0, sizeof(double) * 36 * N, g->stream));
  HIPCHK(hipMemsetAsync(emf, 0, sizeof(double) * 3 * N, g->stream));
  HIPCHK(hipMemsetAsync(vchar, 0, sizeof(double) * 3 * N, g->stream));
  char* base = (char*)workspace;
  return launch_fluxes(g, P, chi_abs, chi_es, F, emf, vchar, nullptr, 0, nullptr, Bf,
                       (double*)(base + w.VF), (double*)(base + w.SP));
}

// ---------------------------------------------------------------------------
// adjoint of one step
// ---------------------------------------------------------------------------
struct AdjLayout {
  size_t F, emf, vch, scr, err, it, Un, Pb, Ue, Pk, Uk, stk, lamP, lamU, lamUe, lamUn, lamPb, lamE,
      G, Gx, Lam, lamPpre, lamUpre, M, lamUs, lamM, lamPg, Pq, FL, GF, LamFl, Lf2, Se, Fs, Sn,
      lamS, lamSn, MS, lamMS, total;
  int ns;   // stages checkpointed
};

// stencil cells per face of the reconstruction (MC 4, PPM 6)
static int adj_slots(const Ctx& C) { return C.recon == GRRMHD_RECON_PPM ? 6 : 4; }

// RK3 keeps three stages; an IMEX scheme its own count, plus the stored
// sources M^k, their cotangents, the per-stage cotangents of U(i) and the
// final inversion's guess cotangent.  PPM adds the flattener of
// every stage, the faces' products with it and two flattener cotangents.
static AdjLayout adj_layout(const Ctx& C, int scheme) {
  AdjLayout w;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t N = (size_t)C.Ntot, D8 = sizeof(double);
  const bool imex = scheme != GRRMHD_RK3;
  const size_t ns = imex ? (size_t)make_scheme(scheme).ns : 3;
  w.ns = (int)ns;
  w.F = take(D8 * 36 * N);
  w.emf = take(D8 * 3 * N);
  w.vch = take(D8 * 3 * N);
  w.scr = take(D8 * 13 * N);
  w.err = take(D8 * N);
  w.it = take(sizeof(int) * N);
  w.Un = take(D8 * 12 * N);
  w.Pb = take(D8 * 12 * ns * N);   // per stage: ghost-filled input primitives
  w.Ue = take(D8 * 12 * ns * N);   // per stage: explicit state U(i)
  w.Pk = take(D8 * 12 * ns * N);   // per stage: output primitives
  w.Uk = take(D8 * 12 * ns * N);   // per stage: output conserved
  w.stk = take(sizeof(int) * ns * N);
  w.lamP = take(D8 * 12 * N);
  w.lamU = take(D8 * 12 * N);
  w.lamUe = take(D8 * 12 * N);
  w.lamUn = take(D8 * 12 * N);
  w.lamPb = take(D8 * 12 * N);
  w.lamE = take(D8 * 3 * N);
  const bool ppm = C.recon == GRRMHD_RECON_PPM;
  w.G = take(D8 * 3 * 12 * adj_slots(C) * N);  // per direction: face products with the stencil cells
  w.Gx = take(D8 * 3 * 2 * N);  // per direction: face products with the 2 face cells' opacity
  w.Lam = take(D8 * 12 * N);
  w.lamPpre = take(D8 * 12 * N);
  w.lamUpre = take(D8 * 12 * N);
  w.M = take(imex ? D8 * 4 * 8 * N : 0);
  w.lamUs = take(imex ? D8 * 12 * ns * N : 0);
  w.lamM = take(imex ? D8 * 4 * 8 * N : 0);
  w.lamPg = take(imex ? D8 * 12 * N : 0);
  w.Pq = take(D8 * 12 * ns * N);   // per stage: output primitives before the fix-ups
  w.FL = take(ppm ? D8 * 6 * ns * N : 0);   // per stage: the flattener its fluxes read
  w.GF = take(ppm ? D8 * 12 * N : 0);       // per direction: face products with the flattener
  w.LamFl = take(ppm ? D8 * 6 * N : 0);     // cotangent of the flattener read, carried back
  w.Lf2 = take(ppm ? D8 * 6 * N : 0);       // cotangent of a stage's own flattener
  // the full cascade's entropy tracer: each stage's explicit value, the face
  // fluxes, U_S(P^n), and the cotangents of a stage's value and of U_S(P^n);
  // an IMEX scheme adds the stored entropy sources and their cotangents
  const bool ent = C.cascade != 0;
  w.Se = take(ent ? D8 * ns * N : 0);
  w.Fs = take(ent ? D8 * 3 * N : 0);
  w.Sn = take(ent ? D8 * N : 0);
  w.lamS = take(ent ? D8 * N : 0);
  w.lamSn = take(ent ? D8 * N : 0);
  w.MS = take(ent && imex ? D8 * 4 * N : 0);
  w.lamMS = take(ent && imex ? D8 * 4 * N : 0);
  w.total = off;
  return w;
}

extern "C" size_t grrmhd_adjoint_workspace_bytes(const grrmhd_grid* g) {
  return g ? adj_layout(g->C, g->p.scheme).total : 0;
}

static int fill_d(grrmhd_grid* g, double* p, size_t n, double v) {
  hipLaunchKernelGGL(k_fill_d, dim3((unsigned)std::min<size_t>((n + 255) / 256, 65536)), dim3(256), 0,
                     g->stream, p, (long)n, v);
  LAUNCHCHK();
  return 0;
}

// lamUe (all cells; zero outside the interior) from the cotangents of the
// implicit solve's outputs
// gchi (nullable, [2][N]): the opacity cotangents are added to it
// Se, lamS (nullable together): the stage's explicit entropy tracer and its
// cotangent out (full cascade)
static int adj_implicit(grrmhd_grid* g, double scale, const double* dt_dev, const double* Ue,
                        const double* Pk, const int* st, const double* ca, const double* ce,
                        const double* lamP, const double* lamU, double* lamUe,
                        double* gchi = nullptr, const double* Se = nullptr,
                        double* lamS = nullptr) {
  const Ctx& C = g->C;
  int rc;
  if ((rc = fill_d(g, lamUe, 12 * (size_t)C.Ntot, 0.0))) return rc;
  if (Se && lamS)
    hipLaunchKernelGGL(k_adj_implicit<true>, dim3(nblocks(n_interior(C), 64)), dim3(64), 0,
                       g->stream, C, scale, dt_dev, Ue, Pk, st, ca, ce, lamP, lamU, lamUe, gchi, Se,
                       lamS);
  else
    hipLaunchKernelGGL(k_adj_implicit<false>, dim3(nblocks(n_interior(C), 64)), dim3(64), 0,
                       g->stream, C, scale, dt_dev, Ue, Pk, st, ca, ce, lamP, lamU, lamUe, gchi,
                       nullptr, nullptr);
  LAUNCHCHK();
  return 0;
}

// PPM: the flattener a stage's fluxes read (fl), the one before it in the
// step (prev, null at the first flux evaluation) and the buffers of the
// flattener's transpose (GF [3][4][N], LamFl and Lf2 [3][2][N]).
struct AdjFlat {
  const double* fl;
  const double* prev;
  double *GF, *LamFl, *Lf2;
};

// lamPb (every allocated cell) = (d Ue / d Pb)^T lamUe through the fluxes,
// EMFs, geometric source and (PPM) flattener of a stage with coefficient
// `scale` on dt
// Gx, gchi (nullable together): opacity face products and the cotangents
// they add to gchi [2][N]
// lamS (nullable): the cotangent of the stage's explicit entropy tracer (full
// cascade), whose face fluxes and b U_S(Pb) term (bS) it differentiates too
static int adj_explicit(grrmhd_grid* g, double scale, const double* dt_dev, const double* Pb,
                        const double* ca, const double* ce, const double* lamUe, double* lamE,
                        double* G, double* lamPb, double* Gx, double* gchi, const AdjFlat* FLT,
                        const double* lamS = nullptr, double bS = 0.0) {
  const Ctx& C = g->C;
  const size_t N = (size_t)C.Ntot;
  hipStream_t s = g->stream;
  const bool ppm = C.recon == GRRMHD_RECON_PPM;
  const size_t gs = 12 * (size_t)adj_slots(C) * N;
  if (ppm && !FLT) return fail(GRRMHD_EINVAL, "PPM adjoint without the flattener buffers");
  const double* fl = ppm ? FLT->fl : nullptr;
  double* GF = ppm ? FLT->GF : nullptr;
  int rc;
  if ((rc = fill_d(g, lamE, 3 * N, 0.0))) return rc;
  for (int a = 0; a < 3; a++) {
    if (C.n[(a + 1) % 3] == 1 || C.n[(a + 2) % 3] == 1) continue;
    const FaceRange R = edge_range(C, a);
    hipLaunchKernelGGL(k_adj_emf, dim3(nblocks(R.total, 256)), dim3(256), 0, s, C, a, R, scale,
                       dt_dev, lamUe, lamE);
    LAUNCHCHK();
  }
  FaceRanges FR;
  for (int d = 0; d < 3; d++) FR.r[d] = face_range(C, d);
  for (int d = 0; d < 3; d++) {
    if (C.n[d] == 1) continue;
    const FaceRange& R = FR.r[d];
    double* Gd = G + (size_t)d * gs;
    double* Gxd = Gx ? Gx + (size_t)d * 2 * N : nullptr;
    double* GFd = ppm ? GF + (size_t)d * 4 * N : nullptr;
    const dim3 gr(nblocks(R.total, 64)), bl(64);
#define ADJ_FLUX(D, PPM)                                                                      \
  hipLaunchKernelGGL((k_adj_flux<D, PPM>), gr, bl, 0, s, C, R, scale, dt_dev, Pb, ca, ce, lamUe, \
                     (const double*)lamE, Gd, Gxd, fl, GFd, lamS)
    if (ppm) {
      if (d == 0) ADJ_FLUX(1, true);
      if (d == 1) ADJ_FLUX(2, true);
      if (d == 2) ADJ_FLUX(3, true);
    } else {
      if (d == 0) ADJ_FLUX(1, false);
      if (d == 1) ADJ_FLUX(2, false);
      if (d == 2) ADJ_FLUX(3, false);
    }
#undef ADJ_FLUX
    LAUNCHCHK();
  }
  if (ppm)
    hipLaunchKernelGGL(k_adj_gather<6>, dim3(nblocks(C.Ntot, 256)), dim3(256), 0, s, C, FR,
                       (const double*)G, (const double*)(G + gs), (const double*)(G + 2 * gs),
                       lamPb);
  else
    hipLaunchKernelGGL(k_adj_gather<4>, dim3(nblocks(C.Ntot, 256)), dim3(256), 0, s, C, FR,
                       (const double*)G, (const double*)(G + gs), (const double*)(G + 2 * gs),
                       lamPb);
  LAUNCHCHK();
  if (C.metric != GRRMHD_MINKOWSKI) {
    const long ncell = (long)C.n[0] * C.n[1] * C.n[2];
    hipLaunchKernelGGL(k_adj_geom, dim3(nblocks(ncell, 64)), dim3(64), 0, s, C, scale, dt_dev, Pb,
                       lamUe, lamPb);
    LAUNCHCHK();
  }
  if (Gx && gchi) {
    hipLaunchKernelGGL(k_adj_gather_chi, dim3(nblocks(C.Ntot, 256)), dim3(256), 0, s, C, FR,
                       (const double*)Gx, (const double*)(Gx + 2 * N), (const double*)(Gx + 4 * N),
                       gchi);
    LAUNCHCHK();
  }
  if (ppm) {
    hipLaunchKernelGGL(k_adj_flat_cot, dim3(nblocks(C.Ntot, 256)), dim3(256), 0, s, C, FR,
                       (const double*)GF, fl, FLT->prev, FLT->LamFl, FLT->Lf2);
    LAUNCHCHK();
    // the compression test's velocities (no derivative): on Kerr-Schild the
    // mass fluxes of Pb, formed in the grid's flattener buffer as the forward
    // does
    double* mf = nullptr;
    if (C.metric == GRRMHD_KERR_SCHILD) {
      mf = g->flat + 6 * N;
      hipLaunchKernelGGL(k_mass_flux, dim3(nblocks(C.Ntot, 256)), dim3(256), 0, s, C, Pb, mf);
      LAUNCHCHK();
    }
    hipLaunchKernelGGL(k_adj_flat, dim3(nblocks(C.Ntot, 128)), dim3(128), 0, s, C, Pb, ca, ce,
                       (const double*)mf, (const double*)FLT->Lf2, lamPb, gchi);
    LAUNCHCHK();
  }
  if (lamS && bS != 0.0) {
    hipLaunchKernelGGL(k_adj_entropy_field, dim3(nblocks(n_interior(C), 128)), dim3(128), 0, s, C,
                       bS, Pb, lamS, lamPb);
    LAUNCHCHK();
  }
  return 0;
}

// transpose of the ghost fill, in place
static int adj_bc(grrmhd_grid* g, double* lam) {
  const Ctx& C = g->C;
  for (int d = 2; d >= 0; d--) {
    if (C.ng[d] == 0) continue;
    const long items = 12L * C.N[(d + 1) % 3] * C.N[(d + 2) % 3];   // (quantity, line)
    hipLaunchKernelGGL(k_adj_bc, dim3(nblocks(items, 256)), dim3(256), 0, g->stream, C, d, lam);
    LAUNCHCHK();
  }
  return 0;
}

// Pieces of the adjoint, for callers composing their own sweeps (and for
// checking each piece against finite differences of its forward part).
extern "C" int grrmhd_implicit_vjp(grrmhd_grid* g, const double* Uexp, const double* P_out,
                                   const int* status, double dt_scale, const double* dt_dev,
                                   const double* chi_abs, const double* chi_es,
                                   const double* gP_out, const double* gU_out, double* gUexp) {
  NEEDG();
  if (!Uexp || !P_out || !status || !dt_dev || !chi_abs || !chi_es || !gP_out || !gU_out || !gUexp)
    return fail(GRRMHD_EINVAL, "NULL array");
  if (g->C.cascade)
    return fail(GRRMHD_EINVAL, "implicit_vjp covers the normal cascade (cascade = 0)");
  return adj_implicit(g, dt_scale, dt_dev, Uexp, P_out, status, chi_abs, chi_es, gP_out, gU_out,
                      gUexp);
}

// lamE [3][N], G [3][12 NSL][N]; PPM also GF [3][4][N], LamFl and Lf2
// [3][2][N] (each 256-byte aligned)
static size_t evjp_part(size_t doubles) { return (doubles * sizeof(double) + 255) & ~(size_t)255; }

extern "C" size_t grrmhd_explicit_vjp_workspace_bytes(const grrmhd_grid* g) {
  if (!g) return 0;
  const size_t N = (size_t)g->C.Ntot;
  size_t b = evjp_part(3 * N) + evjp_part(36 * (size_t)adj_slots(g->C) * N);
  if (g->C.recon == GRRMHD_RECON_PPM) b += evjp_part(12 * N) + 2 * evjp_part(6 * N);
  return b;
}

extern "C" int grrmhd_explicit_vjp(grrmhd_grid* g, double c, const double* dt_dev,
                                   const double* P, const double* chi_abs, const double* chi_es,
                                   const double* gUexp, double* gP, void* workspace,
                                   size_t ws_bytes) {
  NEEDG();
  if (!dt_dev || !P || !chi_abs || !chi_es || !gUexp || !gP || !workspace)
    return fail(GRRMHD_EINVAL, "NULL array");
  if (g->C.ct) return fail(GRRMHD_EINVAL, "the flux adjoint covers the flux-CT field");
  if (ws_bytes < grrmhd_explicit_vjp_workspace_bytes(g)) return fail(GRRMHD_EINVAL, "workspace too small");
  if (((uintptr_t)workspace) & 255) return fail(GRRMHD_EINVAL, "workspace must be 256-byte aligned");
  const Ctx& C = g->C;
  const size_t N = (size_t)C.Ntot;
  char* w = (char*)workspace;
  double* lamE = (double*)w;
  w += evjp_part(3 * N);
  double* G = (double*)w;
  w += evjp_part(36 * (size_t)adj_slots(C) * N);
  if (C.recon != GRRMHD_RECON_PPM)
    return adj_explicit(g, c, dt_dev, P, chi_abs, chi_es, gUexp, lamE, G, gP, nullptr, nullptr,
                        nullptr);
  // PPM: the flattener of P alone, as at a step's first flux evaluation
  AdjFlat F;
  F.GF = (double*)w;
  w += evjp_part(12 * N);
  F.LamFl = (double*)w;
  w += evjp_part(6 * N);
  F.Lf2 = (double*)w;
  int rc;
  if ((rc = launch_flattener(g, P, chi_abs, chi_es, 0))) return rc;
  if ((rc = fill_d(g, F.LamFl, 6 * N, 0.0))) return rc;
  F.fl = g->flat;
  F.prev = nullptr;
  return adj_explicit(g, c, dt_dev, P, chi_abs, chi_es, gUexp, lamE, G, gP, nullptr, nullptr, &F);
}

extern "C" int grrmhd_bc_vjp(grrmhd_grid* g, double* gP) {
  NEEDG();
  if (!gP) return fail(GRRMHD_EINVAL, "NULL array");
  return adj_bc(g, gP);
}

extern "C" int grrmhd_fixup_vjp(grrmhd_grid* g, const double* P, const int* status,
                                const double* gP, const double* gU, double* gP_pre,
                                double* gU_pre, double* scratch) {
  NEEDG();
  if (!P || !status || !gP || !gU || !gP_pre || !gU_pre || !scratch)
    return fail(GRRMHD_EINVAL, "NULL array");
  if (g->C.ct) return fail(GRRMHD_EINVAL, "the fix-up adjoint covers the flux-CT field");
  if (gP_pre == gP || gP_pre == gU || gU_pre == gP || gU_pre == gU || scratch == gP ||
      scratch == gU || scratch == gP_pre || scratch == gU_pre || gP_pre == gU_pre)
    return fail(GRRMHD_EINVAL, "fixup_vjp arrays must not alias");
  const Ctx& C = g->C;
  const size_t N12 = 12 * (size_t)C.Ntot;
  const long nint = n_interior(C);
  int rc;
  if ((rc = fill_d(g, gP_pre, N12, 0.0)) || (rc = fill_d(g, gU_pre, N12, 0.0))) return rc;
  hipLaunchKernelGGL(k_adj_fixup_own, dim3(nblocks(nint, 128)), dim3(128), 0, g->stream, C, P,
                     (const double*)nullptr, status, gP, gU, scratch);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_adj_fixup, dim3(nblocks(nint, 256)), dim3(256), 0, g->stream, C, 0, status,
                     (const double*)scratch, gP, gU, gP_pre, gU_pre);
  LAUNCHCHK();
  return 0;
}

extern "C" int grrmhd_con2prim_vjp(grrmhd_grid* g, const double* U, const double* P,
                                   const int* status, const double* gP, double* gU,
                                   double* gPguess) {
  NEEDG();
  if (!U || !P || !status || !gP || !gU || !gPguess) return fail(GRRMHD_EINVAL, "NULL array");
  if (gU == gPguess || gU == gP || gPguess == gP)
    return fail(GRRMHD_EINVAL, "con2prim_vjp outputs must not alias");
  const size_t N12 = 12 * (size_t)g->C.Ntot;
  int rc;
  if ((rc = fill_d(g, gU, N12, 0.0)) || (rc = fill_d(g, gPguess, N12, 0.0))) return rc;
  hipLaunchKernelGGL(k_adj_c2p, dim3(nblocks(n_interior(g->C), 64)), dim3(64), 0, g->stream, g->C,
                     U, P, status, gP, gU, gPguess);
  LAUNCHCHK();
  return 0;
}

// Named views of the adjoint workspace.
struct AdjPtrs {
  double *F, *emf, *vch, *scr, *err, *Un, *Pb, *Ue, *Pk, *Uk;
  double *lamP, *lamU, *lamUe, *lamUn, *lamPb, *lamE, *G, *Gx, *Lam, *lamPpre, *lamUpre;
  double *M, *lamUs, *lamM, *lamPg, *Pq, *FL, *GF, *LamFl, *Lf2, *Se, *Fs, *Sn, *lamS, *lamSn;
  double *MS, *lamMS;
  int *it, *stk;
};

static int adj_ptrs(grrmhd_grid* g, void* workspace, size_t ws_bytes, AdjPtrs& a) {
  if (g->p.cascade != 0 && g->p.scheme != GRRMHD_RK3) {
    // the tracer's b term is the stage input's U_S, the previous stage's
    const Scheme S = make_scheme(g->p.scheme);
    for (int i = 0; i < S.ns; i++)
      if (S.s[i].g > 0.0 && S.s[i].b != 0.0 && S.s[i].j != i - 1)
        return fail(GRRMHD_EINVAL, "entropy tracer: a stage's b term must take the previous stage");
  }
  if (g->C.ct)
    return fail(GRRMHD_EINVAL, "the adjoint covers the flux-CT field (ct = GRRMHD_CT_FLUX)");
  const AdjLayout w = adj_layout(g->C, g->p.scheme);
  if (ws_bytes < w.total) return fail(GRRMHD_EINVAL, "workspace too small");
  if (((uintptr_t)workspace) & 255) return fail(GRRMHD_EINVAL, "workspace must be 256-byte aligned");
  char* base = (char*)workspace;
  a.F = (double*)(base + w.F);
  a.emf = (double*)(base + w.emf);
  a.vch = (double*)(base + w.vch);
  a.scr = (double*)(base + w.scr);
  a.err = (double*)(base + w.err);
  a.it = (int*)(base + w.it);
  a.Un = (double*)(base + w.Un);
  a.Pb = (double*)(base + w.Pb);
  a.Ue = (double*)(base + w.Ue);
  a.Pk = (double*)(base + w.Pk);
  a.Uk = (double*)(base + w.Uk);
  a.stk = (int*)(base + w.stk);
  a.lamP = (double*)(base + w.lamP);
  a.lamU = (double*)(base + w.lamU);
  a.lamUe = (double*)(base + w.lamUe);
  a.lamUn = (double*)(base + w.lamUn);
  a.lamPb = (double*)(base + w.lamPb);
  a.lamE = (double*)(base + w.lamE);
  a.G = (double*)(base + w.G);
  a.Gx = (double*)(base + w.Gx);
  a.Lam = (double*)(base + w.Lam);
  a.lamPpre = (double*)(base + w.lamPpre);
  a.lamUpre = (double*)(base + w.lamUpre);
  a.M = (double*)(base + w.M);
  a.lamUs = (double*)(base + w.lamUs);
  a.lamM = (double*)(base + w.lamM);
  a.lamPg = (double*)(base + w.lamPg);
  a.Pq = (double*)(base + w.Pq);
  a.FL = (double*)(base + w.FL);
  a.GF = (double*)(base + w.GF);
  a.LamFl = (double*)(base + w.LamFl);
  a.Lf2 = (double*)(base + w.Lf2);
  a.Se = (double*)(base + w.Se);
  a.Fs = (double*)(base + w.Fs);
  a.Sn = (double*)(base + w.Sn);
  a.lamS = (double*)(base + w.lamS);
  a.lamSn = (double*)(base + w.lamSn);
  a.MS = (double*)(base + w.MS);
  a.lamMS = (double*)(base + w.lamMS);
  return 0;
}

// PPM: keep the flattener stage k's fluxes read
static int adj_keep_flat(grrmhd_grid* g, const AdjPtrs& a, int k) {
  if (g->C.recon != GRRMHD_RECON_PPM) return 0;
  const size_t N6 = 6 * (size_t)g->C.Ntot;
  HIPCHK(hipMemcpyAsync(a.FL + k * N6, g->flat, sizeof(double) * N6, hipMemcpyDeviceToDevice,
                        g->stream));
  return 0;
}

// PPM: the flattener views of stage k's reverse step (prev_k: the stage of
// the step's previous flux evaluation, -1 at the first)
static AdjFlat adj_flat_of(grrmhd_grid* g, const AdjPtrs& a, int k, int prev_k) {
  const size_t N6 = 6 * (size_t)g->C.Ntot;
  AdjFlat F;
  F.fl = a.FL + k * N6;
  F.prev = prev_k >= 0 ? a.FL + prev_k * N6 : nullptr;
  F.GF = a.GF;
  F.LamFl = a.LamFl;
  F.Lf2 = a.Lf2;
  return F;
}

static const double ADJ_A[3] = {1.0, 0.75, 1.0 / 3.0}, ADJ_B[3] = {0.0, 0.25, 2.0 / 3.0},
                    ADJ_C[3] = {1.0, 0.25, 2.0 / 3.0};

// Forward step with checkpoints (the same launches as grrmhd_step, dt fixed):
// per stage the ghost-filled input P, the explicit state, the output P, U
// and status, and the output P before the fix-ups.  P_next/U_next (nullable) get the result; U_next's ghost
// entries are those of U(P_n), as grrmhd_step leaves them.
static int adj_forward(grrmhd_grid* g, const double* P_n, const double* chi_abs,
                       const double* chi_es, const double* dt_dev, double* P_next, double* U_next,
                       const AdjPtrs& a) {
  const Ctx& C = g->C;
  const size_t N = (size_t)C.Ntot, N12 = 12 * N, B12 = sizeof(double) * N12;
  hipStream_t s = g->stream;
  int rc;
  HIPCHK(hipMemcpyAsync(a.Pb, P_n, B12, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_p2u, dim3(nblocks(C.Ntot, 256)), dim3(256), 0, s, C, a.Pb, a.Un);
  LAUNCHCHK();
  const bool ent = C.cascade != 0;
  if (ent) {
    hipLaunchKernelGGL(k_entropy_field, dim3(nblocks(n_interior(C), 256)), dim3(256), 0, s, C,
                       (const double*)a.Pb, a.Sn);
    LAUNCHCHK();
  }
  for (int k = 0; k < 3; k++) {
    double* Pin = a.Pb + k * N12;
    double* Uek = a.Ue + k * N12;
    double* Pout = a.Pk + k * N12;
    double* Uout = a.Uk + k * N12;
    int* st = a.stk + k * N;
    if (k > 0) HIPCHK(hipMemcpyAsync(Pin, a.Pk + (k - 1) * N12, B12, hipMemcpyDeviceToDevice, s));
    if ((rc = launch_bc(g, Pin))) return rc;
    if ((rc = launch_fluxes(g, Pin, chi_abs, chi_es, a.F, a.emf, a.vch, nullptr, k > 0,
                            ent ? a.Fs : nullptr)))
      return rc;
    if ((rc = adj_keep_flat(g, a, k))) return rc;
    if ((rc = launch_update(g, ADJ_A[k], ADJ_B[k], ADJ_C[k], dt_dev, Pin, a.Un,
                            k == 0 ? a.Un : a.Uk + (k - 1) * N12, a.F, a.emf, Uek)))
      return rc;
    double* Sek = ent ? a.Se + k * N : nullptr;
    if (ent) {
      hipLaunchKernelGGL(k_entropy_update, dim3(nblocks(n_interior(C), 256)), dim3(256), 0, s, C,
                         ADJ_A[k], ADJ_B[k], ADJ_C[k], dt_dev, (const double*)a.Sn,
                         (const double*)Pin, (const double*)a.Fs, Sek);
      LAUNCHCHK();
    }
    HIPCHK(hipMemcpyAsync(Pout, Pin, B12, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(Uout, Uek, B12, hipMemcpyDeviceToDevice, s));
    if ((rc = launch_implicit(g, Uek, Pin, ADJ_C[k], dt_dev, chi_abs, chi_es, Pout, Uout, a.it, st,
                              a.err, Sek)))
      return rc;
    HIPCHK(hipMemcpyAsync(a.Pq + k * N12, Pout, B12, hipMemcpyDeviceToDevice, s));
    if ((rc = launch_fixup(g, Pout, Uout, st, a.scr, nullptr, a.it, nullptr, 0))) return rc;
  }
  if (P_next) HIPCHK(hipMemcpyAsync(P_next, a.Pk + 2 * N12, B12, hipMemcpyDeviceToDevice, s));
  if (U_next) {   // interior of the last stage over U(P_n) (ghost entries kept)
    HIPCHK(hipMemcpyAsync(U_next, a.Un, B12, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_copy_interior12, dim3(nblocks(n_interior(C), 256)), dim3(256), 0, s, C,
                       (const double*)(a.Uk + 2 * N12), U_next);
    LAUNCHCHK();
  }
  return 0;
}

// Reverse sweep over the checkpoints adj_forward left in the workspace.
static int adj_reverse(grrmhd_grid* g, const double* chi_abs, const double* chi_es,
                       const double* dt_dev, const double* gU_next, double* gP_n, double* g_chi,
                       const AdjPtrs& a) {
  const Ctx& C = g->C;
  const size_t N = (size_t)C.Ntot, N12 = 12 * N;
  hipStream_t s = g->stream;
  const long nint = n_interior(C);
  double* Gx = g_chi ? a.Gx : nullptr;
  int rc;
  const unsigned gi = nblocks(nint, 256), ga = nblocks(C.Ntot, 256);
  hipLaunchKernelGGL(k_copy_interior, dim3(ga), dim3(256), 0, s, C, gU_next, a.lamU);
  LAUNCHCHK();
  if ((rc = fill_d(g, a.lamP, N12, 0.0)) || (rc = fill_d(g, a.lamUn, N12, 0.0))) return rc;
  if (g_chi && (rc = fill_d(g, g_chi, 2 * N, 0.0))) return rc;
  const bool ppm = C.recon == GRRMHD_RECON_PPM;
  if (ppm && (rc = fill_d(g, a.LamFl, 6 * N, 0.0))) return rc;
  const bool ent = C.cascade != 0;
  if (ent && ((rc = fill_d(g, a.lamS, N, 0.0)) || (rc = fill_d(g, a.lamSn, N, 0.0)))) return rc;
  for (int k = 2; k >= 0; k--) {
    const double* Pin = a.Pb + k * N12;
    // fix-up of failed and cold cells, then the implicit solve
    const double* Pq = a.Pq + k * N12;   // the solve's output
    hipLaunchKernelGGL(k_adj_fixup_own, dim3(nblocks(nint, 128)), dim3(128), 0, s, C,
                       (const double*)(a.Pk + k * N12), Pq, (const int*)(a.stk + k * N),
                       (const double*)a.lamP, (const double*)a.lamU, a.Lam);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_adj_fixup, dim3(gi), dim3(256), 0, s, C, 1, (const int*)(a.stk + k * N),
                       (const double*)a.Lam, (const double*)a.lamP, (const double*)a.lamU,
                       a.lamPpre, a.lamUpre);
    LAUNCHCHK();
    if ((rc = adj_implicit(g, ADJ_C[k], dt_dev, a.Ue + k * N12, Pq, a.stk + k * N,
                           chi_abs, chi_es, a.lamPpre, a.lamUpre, a.lamUe, g_chi,
                           ent ? a.Se + k * N : nullptr, ent ? a.lamS : nullptr)))
      return rc;
    if (ent) {   // the tracer's a U_S(P^n) term
      hipLaunchKernelGGL(k_adj_axpy1, dim3(gi), dim3(256), 0, s, C, ADJ_A[k], (const double*)a.lamS,
                         a.lamSn);
      LAUNCHCHK();
    }
    hipLaunchKernelGGL(k_adj_stage, dim3(gi), dim3(256), 0, s, C, ADJ_A[k], ADJ_B[k],
                       (const double*)a.lamUe, a.lamUn, a.lamU);
    LAUNCHCHK();
    const AdjFlat F = adj_flat_of(g, a, k, k - 1);
    if ((rc = adj_explicit(g, ADJ_C[k], dt_dev, Pin, chi_abs, chi_es, a.lamUe, a.lamE, a.G,
                           a.lamPb, Gx, g_chi, ppm ? &F : nullptr, ent ? a.lamS : nullptr,
                           ADJ_B[k])))
      return rc;
    if ((rc = adj_bc(g, a.lamPb))) return rc;
    hipLaunchKernelGGL(k_copy_interior, dim3(ga), dim3(256), 0, s, C, (const double*)a.lamPb, a.lamP);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_adj_p2u, dim3(nblocks(nint, 128)), dim3(128), 0, s, C, (const double*)a.Pb,
                     (const double*)a.lamUn, a.lamP);
  LAUNCHCHK();
  if (ent) {   // U_S(P^n) of every stage's tracer
    hipLaunchKernelGGL(k_adj_entropy_field, dim3(nblocks(nint, 128)), dim3(128), 0, s, C, 1.0,
                       (const double*)a.Pb, (const double*)a.lamSn, a.lamP);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_copy_interior, dim3(ga), dim3(256), 0, s, C, (const double*)a.lamP, gP_n);
  LAUNCHCHK();
  return 0;
}

// IMEX schemes.  Forward: the launches of imex_step with dt fixed, keeping
// per stage the input P (ghost-filled where the stage has a flux), the
// explicit state, the output P, U and status, the output P before the
// fix-ups, the stored sources M^k; with the full cascade also
// each implicit stage's explicit entropy tracer and the stored M_S^k.
static int adj_forward_imex(grrmhd_grid* g, const double* P_n, const double* chi_abs,
                            const double* chi_es, const double* dt_dev, double* P_next,
                            double* U_next, const AdjPtrs& a) {
  const Ctx& C = g->C;
  const Scheme S = make_scheme(g->p.scheme);
  const size_t N = (size_t)C.Ntot, N12 = 12 * N, B12 = sizeof(double) * N12;
  const long nint = n_interior(C);
  hipStream_t s = g->stream;
  int rc;
  HIPCHK(hipMemcpyAsync(a.Pb, P_n, B12, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_p2u, dim3(nblocks(C.Ntot, 256)), dim3(256), 0, s, C, a.Pb, a.Un);
  LAUNCHCHK();
  const bool ent = C.cascade != 0;
  if (ent) {
    hipLaunchKernelGGL(k_entropy_field, dim3(nblocks(nint, 256)), dim3(256), 0, s, C,
                       (const double*)a.Pb, a.Sn);
    LAUNCHCHK();
  }
  int nflux = 0;
  for (int i = 0; i < S.ns; i++) {
    const Stage& x = S.s[i];
    double* Pin = a.Pb + i * N12;
    double* Uei = a.Ue + i * N12;
    double* Pout = a.Pk + i * N12;
    double* Uout = a.Uk + i * N12;
    int* st = a.stk + i * N;
    if (i > 0) HIPCHK(hipMemcpyAsync(Pin, a.Pk + (i - 1) * N12, B12, hipMemcpyDeviceToDevice, s));
    if (x.c != 0.0) {
      if ((rc = launch_bc(g, Pin))) return rc;
      if ((rc = launch_fluxes(g, Pin, chi_abs, chi_es, a.F, a.emf, a.vch, nullptr, nflux > 0,
                              ent ? a.Fs : nullptr)))
        return rc;
      if ((rc = adj_keep_flat(g, a, i))) return rc;
      nflux++;
    }
    MTerms MT;
    memset(&MT, 0, sizeof(MT));
    for (int k = 0; k < i && k < 4; k++) {
      if (x.m[k] == 0.0) continue;
      MT.M[MT.n] = a.M + k * 8 * N;
      MT.m[MT.n] = x.m[k];
      MT.n++;
    }
    const double* Uj = (x.j >= 0) ? a.Uk + x.j * N12 : a.Un;
    if ((rc = launch_update(g, x.a, x.b, x.c, dt_dev, Pin, a.Un, Uj, a.F, a.emf, Uei, nullptr,
                            nullptr, &MT)))
      return rc;
    double* Sei = (ent && x.g > 0.0) ? a.Se + i * N : nullptr;
    if (Sei) {
      hipLaunchKernelGGL(k_entropy_update, dim3(nblocks(nint, 256)), dim3(256), 0, s, C, x.a, x.b,
                         x.c, dt_dev, (const double*)a.Sn, (const double*)Pin,
                         (const double*)a.Fs, Sei);
      LAUNCHCHK();
      if (MT.n > 0) {
        MTerms MS = MT;
        for (int q = 0, k = 0; k < i && k < 4; k++)
          if (x.m[k] != 0.0) MS.M[q++] = a.MS + k * N;
        hipLaunchKernelGGL(k_entropy_mterms, dim3(nblocks(nint, 256)), dim3(256), 0, s, C, MS,
                           dt_dev, Sei);
        LAUNCHCHK();
      }
    }
    HIPCHK(hipMemcpyAsync(Pout, Pin, B12, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(Uout, Uei, B12, hipMemcpyDeviceToDevice, s));
    if (x.g > 0.0) {
      if ((rc = launch_implicit(g, Uei, Pin, x.g, dt_dev, chi_abs, chi_es, Pout, Uout, a.it, st,
                                a.err, Sei)))
        return rc;
      HIPCHK(hipMemcpyAsync(a.Pq + i * N12, Pout, B12, hipMemcpyDeviceToDevice, s));
      if (i < 4 && S.keep_m[i]) {
        hipLaunchKernelGGL(k_stage_m, dim3(nblocks(nint, 256)), dim3(256), 0, s, C, Uei, Uout, st,
                           x.g, dt_dev, a.M + i * 8 * N);
        LAUNCHCHK();
        if (ent) {
          hipLaunchKernelGGL(k_stage_ms, dim3(nblocks(nint, 256)), dim3(256), 0, s, C,
                             (const double*)Pout, (const double*)Sei, (const int*)st, x.g, dt_dev,
                             a.MS + i * N);
          LAUNCHCHK();
        }
      }
      if ((rc = launch_fixup(g, Pout, Uout, st, a.scr, nullptr, a.it, nullptr, 0))) return rc;
    } else {
      hipLaunchKernelGGL(k_con2prim, dim3(nblocks(nint, 128)), dim3(128), 0, s, C, Uei,
                         (const double*)Pin, Pout, st, (int)GRRMHD_ST_FAIL);
      LAUNCHCHK();
      HIPCHK(hipMemcpyAsync(a.Pq + i * N12, Pout, B12, hipMemcpyDeviceToDevice, s));
      if ((rc = launch_fixup(g, Pout, Uout, st, a.scr, nullptr, nullptr, nullptr, 0))) return rc;
    }
  }
  const int l = S.ns - 1;
  if (P_next) HIPCHK(hipMemcpyAsync(P_next, a.Pk + l * N12, B12, hipMemcpyDeviceToDevice, s));
  if (U_next) {
    HIPCHK(hipMemcpyAsync(U_next, a.Un, B12, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_copy_interior12, dim3(nblocks(nint, 256)), dim3(256), 0, s, C,
                       (const double*)(a.Uk + l * N12), U_next);
    LAUNCHCHK();
  }
  return 0;
}

// Reverse sweep of an IMEX step.  Per stage, last first: the fix-up's
// transpose; then the implicit solve's (with the stored source's two sides,
// M^i = (U(i) - U_e)/(g dt) taken before the fix-up) or the final
// inversion's; then the stage bracket U_e = a U^n + b U(j) + c dt X(P_in)
// + dt sum_k m_k M^k, which hands cotangents to U^n, U(j), the earlier M^k
// and through the fluxes to the stage input P_in.  The full cascade's
// entropy tracer runs beside it: M_S^i = (U_S(P_out) - S_e)/(g dt) splits
// its cotangent over the solve's output P and its tracer S_e, and the
// tracer's bracket a U_S(P^n) + b U_S(P_in) + c dt (-div F_S) + dt sum_k m_k
// M_S^k hands its cotangent to U_S(P^n), P_in (its b term and face fluxes)
// and the earlier M_S^k.
static int adj_reverse_imex(grrmhd_grid* g, const double* chi_abs, const double* chi_es,
                            const double* dt_dev, const double* gU_next, double* gP_n,
                            double* g_chi, const AdjPtrs& a) {
  const Ctx& C = g->C;
  const Scheme S = make_scheme(g->p.scheme);
  const size_t N = (size_t)C.Ntot, N12 = 12 * N;
  hipStream_t s = g->stream;
  const long nint = n_interior(C);
  double* Gx = g_chi ? a.Gx : nullptr;
  const unsigned gi = nblocks(nint, 256), ga = nblocks(C.Ntot, 256);
  int rc;
  if ((rc = fill_d(g, a.lamUs, (size_t)S.ns * N12, 0.0)) || (rc = fill_d(g, a.lamM, 32 * N, 0.0)) ||
      (rc = fill_d(g, a.lamP, N12, 0.0)) || (rc = fill_d(g, a.lamUn, N12, 0.0)))
    return rc;
  if (g_chi && (rc = fill_d(g, g_chi, 2 * N, 0.0))) return rc;
  const bool ppm = C.recon == GRRMHD_RECON_PPM;
  if (ppm && (rc = fill_d(g, a.LamFl, 6 * N, 0.0))) return rc;
  const bool ent = C.cascade != 0;
  if (ent && ((rc = fill_d(g, a.lamS, N, 0.0)) || (rc = fill_d(g, a.lamSn, N, 0.0)) ||
              (rc = fill_d(g, a.lamMS, 4 * N, 0.0))))
    return rc;
  hipLaunchKernelGGL(k_copy_interior, dim3(ga), dim3(256), 0, s, C, gU_next,
                     a.lamUs + (S.ns - 1) * N12);
  LAUNCHCHK();
  for (int i = S.ns - 1; i >= 0; i--) {
    const Stage& x = S.s[i];
    const double* Pin = a.Pb + i * N12;
    const double* Pk = a.Pk + i * N12;
    const double* Uei = a.Ue + i * N12;
    const int* st = a.stk + i * N;
    const double* lamUo = a.lamUs + i * N12;
    const double* Pq = a.Pq + i * N12;   // the solve's or inversion's output
    hipLaunchKernelGGL(k_adj_fixup_own, dim3(nblocks(nint, 128)), dim3(128), 0, s, C, Pk, Pq, st,
                       (const double*)a.lamP, lamUo, a.Lam);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_adj_fixup, dim3(gi), dim3(256), 0, s, C, 1, st, (const double*)a.Lam,
                       (const double*)a.lamP, lamUo, a.lamPpre, a.lamUpre);
    LAUNCHCHK();
    const bool tr = ent && x.g > 0.0;   // the stage has an entropy tracer
    if (x.g > 0.0) {
      const bool km = i < 4 && S.keep_m[i];
      double* lamMi = a.lamM + i * 8 * N;
      if (km) {
        hipLaunchKernelGGL(k_adj_mscatter, dim3(gi), dim3(256), 0, s, C, 1.0 / x.g, dt_dev, st,
                           (const double*)lamMi, a.lamUpre);
        LAUNCHCHK();
      }
      if (km && ent) {
        hipLaunchKernelGGL(k_adj_stage_ms, dim3(nblocks(nint, 128)), dim3(128), 0, s, C, 0, x.g,
                           dt_dev, st, Pq, (const double*)(a.lamMS + i * N), a.lamPpre, nullptr);
        LAUNCHCHK();
      }
      if ((rc = adj_implicit(g, x.g, dt_dev, Uei, Pq, st, chi_abs, chi_es, a.lamPpre, a.lamUpre,
                             a.lamUe, g_chi, tr ? a.Se + i * N : nullptr, tr ? a.lamS : nullptr)))
        return rc;
      if (km) {
        hipLaunchKernelGGL(k_adj_mscatter, dim3(gi), dim3(256), 0, s, C, -1.0 / x.g, dt_dev, st,
                           (const double*)lamMi, a.lamUe);
        LAUNCHCHK();
      }
      if (km && ent) {
        hipLaunchKernelGGL(k_adj_stage_ms, dim3(nblocks(nint, 128)), dim3(128), 0, s, C, 1, x.g,
                           dt_dev, st, Pq, (const double*)(a.lamMS + i * N), nullptr, a.lamS);
        LAUNCHCHK();
      }
    } else {
      hipLaunchKernelGGL(k_copy_interior, dim3(ga), dim3(256), 0, s, C, (const double*)a.lamUpre,
                         a.lamUe);
      LAUNCHCHK();
      if ((rc = fill_d(g, a.lamPg, N12, 0.0))) return rc;
      hipLaunchKernelGGL(k_adj_c2p, dim3(nblocks(nint, 64)), dim3(64), 0, s, C, Uei,
                         Pq, st, (const double*)a.lamPpre, a.lamUe, a.lamPg);
      LAUNCHCHK();
    }
    hipLaunchKernelGGL(k_adj_axpy12, dim3(gi), dim3(256), 0, s, C, x.a, (const double*)a.lamUe,
                       a.lamUn);
    LAUNCHCHK();
    if (x.b != 0.0) {
      double* lamUj = (x.j >= 0) ? a.lamUs + x.j * N12 : a.lamUn;
      hipLaunchKernelGGL(k_adj_axpy12, dim3(gi), dim3(256), 0, s, C, x.b, (const double*)a.lamUe,
                         lamUj);
      LAUNCHCHK();
    }
    for (int k = 0; k < i && k < 4; k++) {
      if (x.m[k] == 0.0) continue;
      hipLaunchKernelGGL(k_adj_mterm, dim3(gi), dim3(256), 0, s, C, x.m[k], dt_dev,
                         (const double*)a.lamUe, a.lamM + k * 8 * N);
      LAUNCHCHK();
      if (tr) {
        hipLaunchKernelGGL(k_adj_axpy1_dt, dim3(gi), dim3(256), 0, s, C, x.m[k], dt_dev,
                           (const double*)a.lamS, a.lamMS + k * N);
        LAUNCHCHK();
      }
    }
    if (tr) {   // the tracer's a U_S(P^n) term
      hipLaunchKernelGGL(k_adj_axpy1, dim3(gi), dim3(256), 0, s, C, x.a, (const double*)a.lamS,
                         a.lamSn);
      LAUNCHCHK();
    }
    if (x.c != 0.0) {
      int prev = i - 1;   // the step's previous flux evaluation
      while (prev >= 0 && S.s[prev].c == 0.0) prev--;
      const AdjFlat F = adj_flat_of(g, a, i, prev);
      if ((rc = adj_explicit(g, x.c, dt_dev, Pin, chi_abs, chi_es, a.lamUe, a.lamE, a.G, a.lamPb,
                             Gx, g_chi, ppm ? &F : nullptr, tr ? a.lamS : nullptr, x.b)))
        return rc;
      if ((rc = adj_bc(g, a.lamPb))) return rc;
      hipLaunchKernelGGL(k_copy_interior, dim3(ga), dim3(256), 0, s, C, (const double*)a.lamPb,
                         a.lamP);
      LAUNCHCHK();
    } else {
      if ((rc = fill_d(g, a.lamP, N12, 0.0))) return rc;
      if (tr && x.b != 0.0) {   // the tracer's b U_S(P_in) term without a flux
        hipLaunchKernelGGL(k_adj_entropy_field, dim3(nblocks(nint, 128)), dim3(128), 0, s, C, x.b,
                           Pin, (const double*)a.lamS, a.lamP);
        LAUNCHCHK();
      }
    }
    if (x.g <= 0.0) {   // a failed inversion's result was its guess, P_in
      hipLaunchKernelGGL(k_adj_axpy12, dim3(gi), dim3(256), 0, s, C, 1.0, (const double*)a.lamPg,
                         a.lamP);
      LAUNCHCHK();
    }
  }
  hipLaunchKernelGGL(k_adj_p2u, dim3(nblocks(nint, 128)), dim3(128), 0, s, C, (const double*)a.Pb,
                     (const double*)a.lamUn, a.lamP);
  LAUNCHCHK();
  if (ent) {   // U_S(P^n) of every stage's tracer
    hipLaunchKernelGGL(k_adj_entropy_field, dim3(nblocks(nint, 128)), dim3(128), 0, s, C, 1.0,
                       (const double*)a.Pb, (const double*)a.lamSn, a.lamP);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_copy_interior, dim3(ga), dim3(256), 0, s, C, (const double*)a.lamP, gP_n);
  LAUNCHCHK();
  return 0;
}

static int adj_fwd(grrmhd_grid* g, const double* P_n, const double* chi_abs,
                   const double* chi_es, const double* dt_dev, double* P_next, double* U_next,
                   const AdjPtrs& a) {
  return (g->p.scheme == GRRMHD_RK3)
             ? adj_forward(g, P_n, chi_abs, chi_es, dt_dev, P_next, U_next, a)
             : adj_forward_imex(g, P_n, chi_abs, chi_es, dt_dev, P_next, U_next, a);
}

static int adj_rev(grrmhd_grid* g, const double* chi_abs, const double* chi_es,
                   const double* dt_dev, const double* gU_next, double* gP_n, double* g_chi,
                   const AdjPtrs& a) {
  return (g->p.scheme == GRRMHD_RK3)
             ? adj_reverse(g, chi_abs, chi_es, dt_dev, gU_next, gP_n, g_chi, a)
             : adj_reverse_imex(g, chi_abs, chi_es, dt_dev, gU_next, gP_n, g_chi, a);
}

extern "C" int grrmhd_step_adjoint(grrmhd_grid* g, const double* P_n, const double* chi_abs,
                                   const double* chi_es, const double* dt_dev,
                                   const double* gU_next, double* gP_n, double* g_chi,
                                   double* P_next, double* U_next, void* workspace,
                                   size_t ws_bytes) {
  NEEDG();
  if (!P_n || !chi_abs || !chi_es || !dt_dev || !gU_next || !gP_n || !workspace)
    return fail(GRRMHD_EINVAL, "NULL array");
  AdjPtrs a;
  int rc;
  if ((rc = adj_ptrs(g, workspace, ws_bytes, a))) return rc;
  if ((rc = adj_fwd(g, P_n, chi_abs, chi_es, dt_dev, P_next, U_next, a))) return rc;
  return adj_rev(g, chi_abs, chi_es, dt_dev, gU_next, gP_n, g_chi, a);
}

extern "C" int grrmhd_step_checkpointed(grrmhd_grid* g, const double* P_n, const double* chi_abs,
                                        const double* chi_es, const double* dt_dev,
                                        double* P_next, double* U_next, void* workspace,
                                        size_t ws_bytes) {
  NEEDG();
  if (!P_n || !chi_abs || !chi_es || !dt_dev || !workspace) return fail(GRRMHD_EINVAL, "NULL array");
  AdjPtrs a;
  int rc;
  if ((rc = adj_ptrs(g, workspace, ws_bytes, a))) return rc;
  return adj_fwd(g, P_n, chi_abs, chi_es, dt_dev, P_next, U_next, a);
}

extern "C" int grrmhd_step_adjoint_saved(grrmhd_grid* g, const double* chi_abs,
                                         const double* chi_es, const double* dt_dev,
                                         const double* gU_next, double* gP_n, double* g_chi,
                                         void* workspace, size_t ws_bytes) {
  NEEDG();
  if (!chi_abs || !chi_es || !dt_dev || !gU_next || !gP_n || !workspace)
    return fail(GRRMHD_EINVAL, "NULL array");
  AdjPtrs a;
  int rc;
  if ((rc = adj_ptrs(g, workspace, ws_bytes, a))) return rc;
  return adj_rev(g, chi_abs, chi_es, dt_dev, gU_next, gP_n, g_chi, a);
}

// Workspace of the batched solve: [0, 256) counters (list length @0, queue
// cursor @4, two queue lengths @8, cascade cursor @16, deferred and cold
// list lengths @20 and @24, stats @64), then the cascade list and records,
// the deferred (extreme) and cold lists, and for the per-iteration form two
// queues and the lane state.
// workspace of the per-cell batched form: counters and statistics, cascade
// list with first-attempt records, deferred-cell and cold-cell lists
static constexpr size_t batch_ws_bytes(size_t n) {
  return 256 + cascade_bytes(n) + 2 * round256(sizeof(int) * n);
}

extern "C" size_t grrmhd_implicit_source_workspace_bytes_ex(long n, int mode) {
  if (n <= 0) return 0;
  size_t b = batch_ws_bytes((size_t)n);
  if (mode == GRRMHD_IMPLICIT_PER_ITERATION)
    b += 2 * round256(sizeof(int) * (size_t)n) + round256(sizeof(double) * LS_ND * (size_t)n) +
         round256(sizeof(int) * LI_NI * (size_t)n);
  return b;
}

extern "C" size_t grrmhd_implicit_source_workspace_bytes(long n) {
  return grrmhd_implicit_source_workspace_bytes_ex(n, GRRMHD_IMPLICIT_PER_CELL);
}

static int check_batch_args(const grrmhd_params* p, long n, const double* U_expl,
                            const double* P_guess, const double* dt_cell, const double* chi_abs,
                            const double* chi_es, double* P_out, double* U_out, void* workspace,
                            size_t ws_bytes, int mode) {
  int rc = validate(p, false);
  if (rc) return rc;
  if (n < 0 || n > (1L << 31) - 1) return fail(GRRMHD_EINVAL, "n out of range");
  if (n == 0) return 0;
  if (!U_expl || !P_guess || !dt_cell || !chi_abs || !chi_es || !P_out || !U_out || !workspace)
    return fail(GRRMHD_EINVAL, "NULL array");
  if (mode < GRRMHD_IMPLICIT_PER_CELL || mode > GRRMHD_IMPLICIT_PERSISTENT)
    return fail(GRRMHD_EINVAL, "bad implicit mode");
  // the persistent queue cursor runs past n by up to one fetch per lane
  if (mode == GRRMHD_IMPLICIT_PERSISTENT && n > (1L << 30))
    return fail(GRRMHD_EINVAL, "n above 2^30 for the persistent form");
  if (ws_bytes < grrmhd_implicit_source_workspace_bytes_ex(n, mode))
    return fail(GRRMHD_EINVAL, "workspace too small");
  if (((uintptr_t)workspace) & 255) return fail(GRRMHD_EINVAL, "workspace must be 256-byte aligned");
  if (p->metric != GRRMHD_MINKOWSKI) return fail(GRRMHD_EINVAL, "batched cells use the Minkowski metric");
  return 0;
}

static int launch_batch(const Ctx& C, long n, const double* U_expl, const double* P_guess,
                        const double* dt_cell, const double* chi_abs, const double* chi_es,
                        double* P_out, double* U_out, int* iters, int* status, double* err,
                        int mode, int block, int waves_per_cu, void* workspace, hipStream_t s) {
  char* base = (char*)workspace;
  Work W;
  W.counter = (int*)base;
  W.counter_next = nullptr;
  int* next = W.counter + 1;          // persistent queue cursor
  int* qc = W.counter + 2;            // per-iteration queue lengths (2)
  int* cursor = W.counter + 4;        // cascade queue cursor
  W.stats = (unsigned long long*)(base + 64);
  cascade_layout(base + 256, (size_t)n, W);
  // deferred (extreme) cells of the cascade
  Work D = W;
  D.counter = W.counter + 5;
  D.list = (int*)(base + 256 + cascade_bytes((size_t)n));
  // cells the cascade leaves without an energy solution, for the cold limit
  Work K = W;
  K.counter = W.counter + 6;
  K.list = (int*)((char*)D.list + round256(sizeof(int) * (size_t)n));
  char* extra = (char*)K.list + round256(sizeof(int) * (size_t)n);
  if (mode == GRRMHD_IMPLICIT_PERSISTENT) {
    if (block != 64 && block != 128 && block != 256) return fail(GRRMHD_EINVAL, "block must be 64, 128 or 256");
    if (waves_per_cu < 1 || waves_per_cu > 64) return fail(GRRMHD_EINVAL, "waves_per_cu out of [1, 64]");
  }
  // counters, cursors and the four statistics (bytes 0..95)
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, W.counter, 24);
  LAUNCHCHK();
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  if (mode == GRRMHD_IMPLICIT_PER_CELL) {
    hipLaunchKernelGGL(k_implicit_batch, dim3(nblocks(n, 64)), dim3(64), 0, s, C, n, U_expl, P_guess,
                       dt_cell, chi_abs, chi_es, P_out, U_out, iters, status, err, W);
    LAUNCHCHK();
  } else if (mode == GRRMHD_IMPLICIT_PERSISTENT) {
    const long waves = (long)ncu * waves_per_cu;
    const long blocks = std::max<long>(1, std::min<long>(waves * 64 / block, nblocks(n, block)));
    hipLaunchKernelGGL(k_implicit_persist, dim3((unsigned)blocks), dim3(block), 0, s, C, n, U_expl,
                       P_guess, dt_cell, chi_abs, chi_es, P_out, U_out, iters, status, err, next, W);
    LAUNCHCHK();
  } else {
    const size_t qb = round256(sizeof(int) * (size_t)n);
    int* q0 = (int*)extra;
    int* q1 = (int*)(extra + qb);
    double* sd = (double*)(extra + 2 * qb);
    int* si = (int*)(extra + 2 * qb + round256(sizeof(double) * LS_ND * (size_t)n));
    hipLaunchKernelGGL(k_iter_start, dim3(nblocks(n, 64)), dim3(64), 0, s, C, n, U_expl, P_guess,
                       dt_cell, chi_abs, chi_es, sd, si, qc, q0, W);
    LAUNCHCHK();
    // every attempt ends within max_iter trips (+3 round-off trips are inside it)
    for (int t = 0; t <= C.max_iter; t++) {
      int* qin = (t % 2 == 0) ? q0 : q1;
      int* qout = (t % 2 == 0) ? q1 : q0;
      int* cin = qc + (t % 2);
      int* cout = qc + 1 - (t % 2);
      hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, cout, 1);
      LAUNCHCHK();
      hipLaunchKernelGGL(k_iter_step, dim3(list_blocks(n)), dim3(64), 0, s, C, n, U_expl, dt_cell,
                         chi_abs, chi_es, sd, si, (const int*)cin, (const int*)qin, cout, qout,
                         P_out, U_out, iters, status, err, W);
      LAUNCHCHK();
    }
  }
  // the rest of the cascade: URAD attempts in a compacting persistent grid
  // (one wavefront per SIMD: the kernel holds ~470 registers per lane), then
  // the deferred extreme cells one thread each
  const long cwaves = std::max<long>(1, std::min<long>(4L * ncu, nblocks(n, 64)));
  hipLaunchKernelGGL(k_cascade_urad, dim3((unsigned)cwaves), dim3(64), 0, s, C, n, U_expl, P_guess,
                     dt_cell, chi_abs, chi_es, P_out, U_out, iters, status, err, W, cursor, D, K);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_implicit_batch_list, dim3(list_blocks(n)), dim3(64), 0, s, C, n, U_expl,
                     P_guess, dt_cell, chi_abs, chi_es, P_out, U_out, iters, status, err, D, K);
  LAUNCHCHK();
  // the full cascade's rest for the cells the PMHD and URAD attempts left
  // unaccepted (K holds their record slots), the cold limit inline
  if (C.cascade) {
    hipLaunchKernelGGL(k_rest_batch_list, dim3(list_blocks(n)), dim3(64), 0, s, C, n, U_expl,
                       P_guess, dt_cell, chi_abs, chi_es, P_out, U_out, iters, status, err, W, K);
    LAUNCHCHK();
  } else if (C.cold && C.u_floor > 0.0) {
    // cells with no energy solution: the cold MHD limit, one thread each
    hipLaunchKernelGGL(k_cold_batch_list, dim3(list_blocks(n)), dim3(64), 0, s, C, n, U_expl,
                       P_guess, dt_cell, chi_abs, chi_es, P_out, U_out, iters, status, err, K);
    LAUNCHCHK();
  }
  return 0;
}

// stats[0..1] at `src` and the list length at `cnt` into out[0..2]
static int read_stats(const unsigned long long* src, const int* cnt, unsigned long long out[3],
                      hipStream_t s) {
  unsigned long long st[2];
  int c = 0;
  HIPCHK(hipMemcpyAsync(st, src, sizeof(st), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&c, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  out[0] = st[0];
  out[1] = st[1];
  out[2] = (unsigned long long)c;
  return 0;
}

extern "C" int grrmhd_time_implicit(grrmhd_grid* g, int on) {
  if (!g) return fail(GRRMHD_EINVAL, "grid is NULL");
  HIPCHK(hipSetDevice(g->device));
  if (on && !g->ev) {
    g->ev = new hipEvent_t[2 * grrmhd_grid::TCAP];
    for (int i = 0; i < 2 * grrmhd_grid::TCAP; i++) HIPCHK(hipEventCreate(&g->ev[i]));
  }
  if (on) {
    g->nt = 0;
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, g->stream, (int*)g->W.stats, 4);
    LAUNCHCHK();
  }
  g->timing = on ? 1 : 0;
  return 0;
}

extern "C" int grrmhd_implicit_time(grrmhd_grid* g, double* total_ms, int* launches) {
  if (!g || !total_ms || !launches) return fail(GRRMHD_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(g->device));
  HIPCHK(hipStreamSynchronize(g->stream));
  double t = 0.0;
  for (int i = 0; i < g->nt; i++) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, g->ev[2 * i], g->ev[2 * i + 1]));
    t += ms;
  }
  *total_ms = t;
  *launches = g->nt;
  return 0;
}

extern "C" int grrmhd_implicit_stats(grrmhd_grid* g, unsigned long long out[3]) {
  if (!g || !out) return fail(GRRMHD_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(g->device));
  return read_stats(g->W.stats, g->W.counter, out, g->stream);
}

extern "C" int grrmhd_implicit_source_stats(const void* workspace, unsigned long long out[3],
                                            void* hip_stream) {
  if (!workspace || !out) return fail(GRRMHD_EINVAL, "NULL argument");
  if (((uintptr_t)workspace) & 255) return fail(GRRMHD_EINVAL, "workspace must be 256-byte aligned");
  const char* base = (const char*)workspace;
  return read_stats((const unsigned long long*)(base + 64), (const int*)base, out,
                    (hipStream_t)hip_stream);
}

extern "C" int grrmhd_implicit_source_cascade_stats(const void* workspace,
                                                    unsigned long long out[2], void* hip_stream) {
  if (!workspace || !out) return fail(GRRMHD_EINVAL, "NULL argument");
  if (((uintptr_t)workspace) & 255) return fail(GRRMHD_EINVAL, "workspace must be 256-byte aligned");
  HIPCHK(hipMemcpyAsync(out, (const char*)workspace + 80, 2 * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, (hipStream_t)hip_stream));
  HIPCHK(hipStreamSynchronize((hipStream_t)hip_stream));
  return 0;
}

extern "C" int grrmhd_implicit_source_ex(const grrmhd_params* p, long n, const double* U_expl,
                                         const double* P_guess, const double* dt_cell,
                                         const double* chi_abs, const double* chi_es,
                                         double* P_out, double* U_out, int* iters, int* status,
                                         double* err, int mode, int block, int waves_per_cu,
                                         void* workspace, size_t ws_bytes, void* hip_stream) {
  int rc = check_batch_args(p, n, U_expl, P_guess, dt_cell, chi_abs, chi_es, P_out, U_out,
                            workspace, ws_bytes, mode);
  if (rc || n == 0) return rc;
  Ctx C;
  fill_ctx(p, C);
  return launch_batch(C, n, U_expl, P_guess, dt_cell, chi_abs, chi_es, P_out, U_out, iters, status,
                      err, mode, block, waves_per_cu, workspace, (hipStream_t)hip_stream);
}

extern "C" int grrmhd_autotune_implicit_source(const grrmhd_params* p, long n,
                                               const double* U_expl, const double* P_guess,
                                               const double* dt_cell, const double* chi_abs,
                                               const double* chi_es, double* P_out,
                                               double* U_out, int* iters, int* status,
                                               double* err, void* workspace, size_t ws_bytes,
                                               void* hip_stream, grrmhd_tuning* best,
                                               grrmhd_tuning* all, int n_all) {
  if (!best) return fail(GRRMHD_EINVAL, "best is NULL");
  int rc = check_batch_args(p, n, U_expl, P_guess, dt_cell, chi_abs, chi_es, P_out, U_out,
                            workspace, ws_bytes, GRRMHD_IMPLICIT_PER_ITERATION);
  if (rc) return rc;
  if (n == 0) return fail(GRRMHD_EINVAL, "n must be positive");
  if (n > (1L << 30)) return fail(GRRMHD_EINVAL, "n above 2^30 for the persistent form");
  Ctx C;
  fill_ctx(p, C);
  hipStream_t s = (hipStream_t)hip_stream;
  const int cands[GRRMHD_TUNE_CANDIDATES][3] = {
      {GRRMHD_IMPLICIT_PER_CELL, 64, 0},    {GRRMHD_IMPLICIT_PER_ITERATION, 64, 0},
      {GRRMHD_IMPLICIT_PERSISTENT, 64, 4},  {GRRMHD_IMPLICIT_PERSISTENT, 64, 8},
      {GRRMHD_IMPLICIT_PERSISTENT, 128, 4}, {GRRMHD_IMPLICIT_PERSISTENT, 128, 8},
      {GRRMHD_IMPLICIT_PERSISTENT, 256, 4}, {GRRMHD_IMPLICIT_PERSISTENT, 256, 8},
      {GRRMHD_IMPLICIT_PERSISTENT, 256, 16}};
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  best->ms = 1e30f;
  int k = 0;
  for (const auto& cd : cands) {
    float tbest = 1e30f;
    for (int rep = 0; rep < 2; rep++) {   // first run warms caches and code objects
      HIPCHK(hipEventRecord(e0, s));
      rc = launch_batch(C, n, U_expl, P_guess, dt_cell, chi_abs, chi_es, P_out, U_out, iters,
                        status, err, cd[0], cd[1], cd[2], workspace, s);
      if (rc) return rc;
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) tbest = ms;
    }
    if (all && k < n_all) {
      all[k].mode = cd[0];
      all[k].block = cd[1];
      all[k].waves_per_cu = cd[2];
      all[k].ms = tbest;
    }
    k++;
    if (tbest < best->ms) {
      best->ms = tbest;
      best->mode = cd[0];
      best->block = cd[1];
      best->waves_per_cu = cd[2];
    }
  }
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  return 0;
}

extern "C" int grrmhd_implicit_source(const grrmhd_params* p, long n, const double* U_expl,
                                      const double* P_guess, const double* dt_cell,
                                      const double* chi_abs, const double* chi_es, double* P_out,
                                      double* U_out, int* iters, int* status, double* err,
                                      void* workspace, size_t ws_bytes, void* hip_stream) {
  return grrmhd_implicit_source_ex(p, n, U_expl, P_guess, dt_cell, chi_abs, chi_es, P_out, U_out,
                                   iters, status, err, GRRMHD_IMPLICIT_PER_CELL, 64, 0, workspace,
                                   ws_bytes, hip_stream);
}

// ---- the batched solve without allocation ----
// Scratch memory of grrmhd_implicit_source_noalloc: the per-cell form's
// workspace for GRRMHD_NOALLOC_MAX_CELLS cells (counters, lane statistics,
// cascade list with first-attempt records, deferred and cold lists).  Each
// device the library runs on holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in, never a device address:
// kernels get the per-device address from hipGetSymbolAddress below.
static constexpr size_t NOALLOC_BYTES = batch_ws_bytes((size_t)GRRMHD_NOALLOC_MAX_CELLS);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

static const int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[NOALLOC_MAX_DEVICES];

// device address of the current device's scratch array, looked up once per
// device (with that device current) and kept
static int scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(GRRMHD_EINVAL, "device ordinal above the allocation-free solve's device table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || (((uintptr_t)ptr) & 255))
      return fail(GRRMHD_EHIP, "scratch array address missing or not 256-byte aligned");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return 0;
}

extern "C" int grrmhd_implicit_source_noalloc(const grrmhd_params* p, long n,
                                              const double* U_expl, const double* P_guess,
                                              const double* dt_cell, const double* chi_abs,
                                              const double* chi_es, double* P_out, double* U_out,
                                              int* iters, int* status, double* err,
                                              void* hip_stream) {
  if (n > GRRMHD_NOALLOC_MAX_CELLS)
    return fail(GRRMHD_EINVAL, "n above GRRMHD_NOALLOC_MAX_CELLS for the allocation-free solve");
  void* ws = nullptr;
  if (n > 0) {
    int rc = scratch_address(&ws);
    if (rc) return rc;
  }
  int rc = check_batch_args(p, n, U_expl, P_guess, dt_cell, chi_abs, chi_es, P_out, U_out, ws,
                            NOALLOC_BYTES, GRRMHD_IMPLICIT_PER_CELL);
  if (rc || n == 0) return rc;
  Ctx C;
  fill_ctx(p, C);
  // launch_batch clears the counters and statistics it uses with a kernel;
  // the lists and records are written before they are read
  return launch_batch(C, n, U_expl, P_guess, dt_cell, chi_abs, chi_es, P_out, U_out, iters, status,
                      err, GRRMHD_IMPLICIT_PER_CELL, 64, 0, ws, (hipStream_t)hip_stream);
}
