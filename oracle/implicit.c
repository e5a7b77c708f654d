/*
 * Oracle implicit radiation 4-force solve for one cell (Sec. 4.7-4.11).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Solves the energy-momentum exchange between gas and radiation over one
 * implicit sub-step of size dt with rho0 u^t and B^i held fixed (Sec. 4.7):
 *   T^t_nu(new) - T^t_nu(i) = dt G_nu(new)   (eq. source3, PMHD iteration)
 *   R^t_nu(new) - R^t_nu(i) = -dt G_nu(new)  (eq. source4, URAD iteration)
 * with the radiation (gas) part following from total conservation.
 *
 * PMHD iterates x = (u_g, u~^i_gas); its Jacobian here is a centred finite
 * difference.  URAD iterates x = R^t_nu with an MHD inversion inside each
 * residual and a one-sided finite-difference Jacobian (Sec. 4.9); PRAD
 * iterates the radiation primitives (Ebar, u~^i_rad), the gas from the MHD
 * inversion of T^t_nu(i) - Delta R.  With the full cascade the same methods
 * also run in the staged form (one momentum step, energy-only steps, then
 * the 4-D solve, damped on entering each stage) and with the entropy
 * equation (eq. source6, weighted by T_gas) in place of the gas energy
 * equation.  Method order, guesses, pre/post-step checks, stopping rules and
 * the acceptance cascade follow Sec. 4.10-4.11 in the order given there.
 */
#include <float.h>
#include <math.h>
#include <string.h>
#include "oracle.h"
#include "oracle_internal.h"

#define EPS_M DBL_EPSILON
#define MAXH 64

typedef struct {
  const orc_params *p;
  const orc_geom *g;
  double gij[3][3];
  double rhout, B[3];
  double Tgi[4]; /* explicit gas  (T^t_t + rho u^t, T^t_i), per sqrt(-g) */
  double Ri[4];  /* explicit radiation R^t_nu, per sqrt(-g) */
  double dt, chi_abs, chi_es;
  int cold;    /* cold MHD: energy residuals left out of the errors */
  int entropy; /* entropy equation in place of the gas energy equation */
  double Si;   /* explicit [S u^t]_(i) per sqrt(-g) (NAN: not available) */
} ictx;

typedef struct {
  double x[4];
  double P[12];
  double Tg[4], Rr[4], G[4];
  double Eg[4], Er[4];
  double eT, eIg, eIr;
  double Sut, Tgas, Gu, Es; /* entropy methods: S u^t, T_gas, G^mu u_mu, residual */
  double e0g, e0r;          /* normalised error of the energy (entropy) equation */
  int radflags;
  int ok;
} ieval;

enum { M_PMHD = 0, M_URAD = 1, M_PRAD = 2 };

double orc_entropy(const orc_params *p, const double *P) {
  const double rho = P[0], pg = (p->gam - 1.0) * P[1];
  if (!(rho > 0.0) || !(pg > 0.0)) return NAN;
  const double n = 1.0 / (p->gam - 1.0);
  return rho * (n * log(pg) - (n + 1.0) * log(rho)); /* rho0 ln(p^n / rho0^(n+1)) */
}

static void gas_cons(const ictx *c, const double *P, double Tg[4]) {
  orc_gas s;
  orc_gas_state(c->p, c->g, P, &s);
  Tg[0] = orc_gas_energy_flux(&s, 0);
  for (int i = 0; i < 3; i++) Tg[1 + i] = s.T[0][1 + i];
}

static void rad_cons(const ictx *c, const double *P, double Rr[4]) {
  orc_rad r;
  orc_rad_state(c->g, P, &r);
  for (int m = 0; m < 4; m++) Rr[m] = r.R[0][m];
}

static double snorm(const ictx *c, const double V[4]) {
  double s = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) s += c->gij[i][j] * V[1 + i] * V[1 + j];
  return sqrt(s > 0.0 ? s : 0.0);
}

/* Normalised errors (Sec. 4.8): each residual component is divided by the
 * sum of magnitudes of the terms that build it and its sub-expressions.  The
 * gas residual T - T(i) - dt G is normalised by gas-scale terms and dt|G|, the
 * radiation residual R - R(i) + dt G by radiation-scale terms and dt|G|; the
 * spatial components are merged in the normal observer's orthonormal basis
 * and also carry the energy scale (so a state at rest is not 0/0).
 * e_T = (1/4) sum over the four equations of the larger of the two. */
static void errors(const ictx *c, ieval *e) {
  double Gdt[4];
  for (int m = 0; m < 4; m++) Gdt[m] = c->dt * e->G[m];
  const double nG0 = fabs(Gdt[0]), nGs = snorm(c, Gdt);
  double Ntg = fabs(e->Tg[0]) + fabs(c->Tgi[0]) + nG0;
  double Ntr = fabs(e->Rr[0]) + fabs(c->Ri[0]) + nG0;
  if (!(Ntg > 0.0)) Ntg = 1e-300;
  if (!(Ntr > 0.0)) Ntr = 1e-300;
  const double Nsg = snorm(c, e->Tg) + snorm(c, c->Tgi) + nGs + Ntg;
  const double Nsr = snorm(c, e->Rr) + snorm(c, c->Ri) + nGs + Ntr;
  double eg[4], er[4];
  eg[0] = fabs(e->Eg[0]) / Ntg;
  er[0] = fabs(e->Er[0]) / Ntr;
  for (int i = 0; i < 3; i++) {
    const double w = sqrt(c->gij[i][i]);
    eg[1 + i] = fabs(e->Eg[1 + i]) * w / Nsg;
    er[1 + i] = fabs(e->Er[1 + i]) * w / Nsr;
  }
  if (c->entropy) {
    /* the entropy equation (weighted by T_gas) replaces the energy equation
     * on both sides; its norm carries the energy norm (Sec. 4.8) */
    const double Ns = fabs(e->Tgas * e->Sut) + fabs(e->Tgas * c->Si) + fabs(c->dt * e->Gu) + Ntg;
    eg[0] = er[0] = fabs(e->Es) / Ns;
  }
  /* TYPE2 met E_rad <= 0, or cold: the energy (entropy) equation excluded */
  if ((e->radflags & 1) || c->cold) eg[0] = er[0] = 0.0;
  e->e0g = eg[0];
  e->e0r = er[0];
  double eT = 0.0, eIg = 0.0, eIr = 0.0;
  for (int m = 0; m < 4; m++) {
    eT += (eg[m] > er[m] ? eg[m] : er[m]);
    eIg += eg[m];
    eIr += er[m];
  }
  e->eT = 0.25 * eT;
  e->eIg = 0.25 * eIg;
  e->eIr = 0.25 * eIr;
  if (!isfinite(e->eT)) {
    e->eT = INFINITY;
    e->ok = 0;
  }
}

static void finish_eval(const ictx *c, ieval *e) {
  const double rho = e->P[0];
  orc_four_force(c->p, c->g, e->P, c->chi_abs * rho, c->chi_es * rho, e->G);
  for (int m = 0; m < 4; m++) {
    e->Eg[m] = (e->Tg[m] - c->Tgi[m]) - c->dt * e->G[m];
    e->Er[m] = (e->Rr[m] - c->Ri[m]) + c->dt * e->G[m];
  }
  if (c->entropy) {
    /* eq. source6 with G_S = -G^mu u_mu / T_gas (eq. GS), times T_gas:
     * T_gas ([S u^t] - [S u^t]_(i)) + dt G^mu u_mu */
    double ucon[4];
    orc_ucon(c->g, e->P + 2, ucon);
    e->Sut = orc_entropy(c->p, e->P) * ucon[0];
    e->Tgas = (c->p->gam - 1.0) * e->P[1] / rho;
    e->Gu = 0.0;
    for (int m = 0; m < 4; m++) e->Gu += e->G[m] * ucon[m];
    e->Es = e->Tgas * (e->Sut - c->Si) + c->dt * e->Gu;
    if (!isfinite(e->Es)) e->ok = 0;
  }
  errors(c, e);
  if (!e->ok) e->eT = INFINITY;
}

/* PMHD residual (Sec. 4.8, PMHD steps in the listed order) */
static void eval_pmhd(const ictx *c, const double x[4], ieval *e) {
  memset(e, 0, sizeof(*e));
  memcpy(e->x, x, sizeof(double) * 4);
  e->ok = 1;
  double *P = e->P;
  P[1] = x[0];
  for (int i = 0; i < 3; i++) {
    P[2 + i] = x[1 + i];
    P[5 + i] = c->B[i];
  }
  double ucon[4];
  orc_ucon(c->g, P + 2, ucon);
  P[0] = c->rhout / ucon[0];                       /* rho0 = U_1/u^t */
  gas_cons(c, P, e->Tg);                           /* T^t_mu from gas P */
  double U[12];
  memset(U, 0, sizeof(U));
  for (int m = 0; m < 4; m++)                      /* Delta R = -Delta T */
    U[8 + m] = c->g->gdet * (c->Ri[m] - (e->Tg[m] - c->Tgi[m]));
  e->radflags = orc_rad_invert(c->p, c->g, U, 1, P); /* TYPE2 while iterating */
  rad_cons(c, P, e->Rr);                           /* recompute R for consistency */
  finish_eval(c, e);
}

/* URAD residual (Sec. 4.8, URAD steps) */
static void eval_urad(const ictx *c, const double x[4], const double *Pgas_guess, ieval *e) {
  memset(e, 0, sizeof(*e));
  memcpy(e->x, x, sizeof(double) * 4);
  e->ok = 1;
  double *P = e->P;
  double U[12];
  const double gd = c->g->gdet;
  U[0] = gd * c->rhout;
  for (int m = 0; m < 4; m++) U[1 + m] = gd * (c->Tgi[m] - (x[m] - c->Ri[m])); /* Delta T = -Delta R */
  for (int i = 0; i < 3; i++) U[5 + i] = gd * c->B[i];
  for (int m = 0; m < 4; m++) U[8 + m] = gd * x[m];
  const int rc = orc_mhd_invert(c->p, c->g, U, Pgas_guess, P);
  if (rc != 0) {
    e->ok = 0;
    e->eT = INFINITY;
    return;
  }
  e->radflags = orc_rad_invert(c->p, c->g, U, 1, P);
  gas_cons(c, P, e->Tg);
  rad_cons(c, P, e->Rr);
  finish_eval(c, e);
}

/* PRAD residual (Sec. 4.8, PRAD steps): R^t_nu from the iterated radiation
 * primitives, Delta T = -Delta R, the gas from the MHD inversion of the
 * result (Pgas_guess starts it), T^t_nu recomputed from the gas. */
static void eval_prad(const ictx *c, const double x[4], const double *Pgas_guess, ieval *e) {
  memset(e, 0, sizeof(*e));
  memcpy(e->x, x, sizeof(double) * 4);
  e->ok = 1;
  double *P = e->P;
  memcpy(P, Pgas_guess, sizeof(double) * 12);
  P[8] = x[0];
  for (int i = 0; i < 3; i++) P[9 + i] = x[1 + i];
  rad_cons(c, P, e->Rr);
  double U[12];
  const double gd = c->g->gdet;
  U[0] = gd * c->rhout;
  for (int m = 0; m < 4; m++) U[1 + m] = gd * (c->Tgi[m] - (e->Rr[m] - c->Ri[m]));
  for (int i = 0; i < 3; i++) U[5 + i] = gd * c->B[i];
  for (int m = 0; m < 4; m++) U[8 + m] = gd * e->Rr[m];
  if (orc_mhd_invert(c->p, c->g, U, Pgas_guess, P) != 0) {
    e->ok = 0;
    e->eT = INFINITY;
    return;
  }
  gas_cons(c, P, e->Tg);
  e->radflags = 0;
  finish_eval(c, e);
}

static void eval_method(const ictx *c, int method, const double x[4], const double *Pg, ieval *e) {
  if (method == M_PMHD) eval_pmhd(c, x, e);
  else if (method == M_URAD) eval_urad(c, x, Pg, e);
  else eval_prad(c, x, Pg, e);
}

/* the residual a method iterates on: the gas equations for PMHD, the
 * radiation equations for URAD and PRAD; with the entropy equation in the
 * energy slot for the entropy-based methods (Sec. 4.9) */
static void method_residual(const ictx *c, int method, const ieval *e, double r[4]) {
  const double *E = (method == M_PMHD) ? e->Eg : e->Er;
  for (int m = 0; m < 4; m++) r[m] = E[m];
  if (c->entropy) r[0] = e->Es;
}

/* Gaussian elimination with partial pivoting: solves J dx = r. 0 on success */
static int solve4(double J[4][4], const double r[4], double dx[4]) {
  double A[4][5];
  for (int i = 0; i < 4; i++) {
    for (int j = 0; j < 4; j++) A[i][j] = J[i][j];
    A[i][4] = r[i];
  }
  for (int k = 0; k < 4; k++) {
    int piv = k;
    for (int i = k + 1; i < 4; i++)
      if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
    if (!(fabs(A[piv][k]) > 0.0) || !isfinite(A[piv][k])) return 1;
    if (piv != k)
      for (int j = 0; j < 5; j++) {
        const double t = A[k][j];
        A[k][j] = A[piv][j];
        A[piv][j] = t;
      }
    for (int i = k + 1; i < 4; i++) {
      const double f = A[i][k] / A[k][k];
      for (int j = k; j < 5; j++) A[i][j] -= f * A[k][j];
    }
  }
  for (int i = 3; i >= 0; i--) {
    double s = A[i][4];
    for (int j = i + 1; j < 4; j++) s -= A[i][j] * dx[j];
    dx[i] = s / A[i][i];
  }
  for (int i = 0; i < 4; i++)
    if (!isfinite(dx[i])) return 1;
  return 0;
}

static double rad_energy_of(const ictx *c, const double R[4]) {
  const double al = c->g->alpha;
  double s = 0.0;
  for (int i = 0; i < 3; i++) s += c->g->gcon[0][1 + i] * R[1 + i];
  return -R[0] + al * al * s;
}

/* one-sided difference Jacobian of a radiation-side method (URAD, PRAD;
 * Sec. 4.9) at x with residual ev: offsets of a fixed normalised size delta
 * relative to the iterated quantities, floored at 1e4 eps of the radiation
 * residual's own scale (|R_t| + |R_t(i)| + dt |G_t|; a smaller offset is
 * lost in the residual's rounding where the iterated radiation is tiny
 * against it), the energy-like offset in the direction that raises the
 * radiation energy (lowering a floor-sized energy through zero makes the
 * TYPE2 limiter hold R fixed and the column vanish); on an inversion failure
 * the other side, then 10x larger, up to 0.3 of the scale.  Returns 1 when a
 * column cannot be formed. */
static int jacobian_rad(const ictx *c, int method, const double x[4], const ieval *ev, double delta,
                        double J[4][4]) {
  const double Nres = fabs(ev->Rr[0]) + fabs(c->Ri[0]) + fabs(c->dt * ev->G[0]);
  double r0[4];
  method_residual(c, method, ev, r0);
  for (int j = 0; j < 4; j++) {
    double Nx;
    if (method == M_URAD)
      Nx = (j == 0) ? fabs(x[0]) : fabs(x[j]) + fabs(x[0]) / sqrt(c->gij[j - 1][j - 1]);
    else
      Nx = (j == 0) ? fabs(x[0]) : 1.0 + fabs(x[j]);
    const double N = fmax(Nx, 1e4 * EPS_M * Nres / delta);
    /* URAD x_0 = R^t_t = -(energy): lower it; PRAD x_0 = Ebar: raise it */
    double h = (j == 0) ? ((method == M_URAD) ? -delta * N : delta * N) : delta * N;
    int got = 0;
    for (int tries = 0; tries < 12 && !got; tries++) {
      double xp[4];
      memcpy(xp, x, sizeof(xp));
      xp[j] += h;
      ieval ep;
      eval_method(c, method, xp, ev->P, &ep);
      if (ep.ok) {
        double rp[4];
        method_residual(c, method, &ep, rp);
        for (int i = 0; i < 4; i++) J[i][j] = (rp[i] - r0[i]) / h;
        got = 1;
      } else {
        h = (tries % 2 == 0) ? -h : -10.0 * h; /* other side, then larger */
        if (fabs(h) > 0.3 * N) break;
      }
    }
    if (!got) return 1;
  }
  return 0;
}

/* centred difference Jacobian of PMHD (Sec. 4.9) */
static void jacobian_pmhd(const ictx *c, const double x[4], double delta, double J[4][4]) {
  for (int j = 0; j < 4; j++) {
    const double h = (j == 0) ? delta * fabs(x[0]) : delta * (1.0 + fabs(x[j]));
    double xp[4], xm[4];
    memcpy(xp, x, sizeof(xp));
    memcpy(xm, x, sizeof(xm));
    xp[j] += h;
    xm[j] -= h;
    ieval ep, em;
    eval_pmhd(c, xp, &ep);
    eval_pmhd(c, xm, &em);
    double rp[4], rm[4];
    method_residual(c, M_PMHD, &ep, rp);
    method_residual(c, M_PMHD, &em, rm);
    for (int i = 0; i < 4; i++) J[i][j] = (rp[i] - rm[i]) / (2.0 * h);
  }
}

/* post-step check (Sec. 4.10): a negative u_g (PMHD), lab radiation energy
 * (URAD) or Ebar (PRAD) is replaced by half its magnitude; returns 1 when it
 * acted */
static int post_step(const ictx *c, int method, double xn[4]) {
  if (method == M_PMHD || method == M_PRAD) {
    if (xn[0] < 0.0) {
      xn[0] = 0.5 * fabs(xn[0]);
      return 1;
    }
    return 0;
  }
  const double Er = rad_energy_of(c, xn);
  if (Er <= 0.0) {
    const double al = c->g->alpha;
    double s = 0.0;
    for (int i = 0; i < 3; i++) s += c->g->gcon[0][1 + i] * xn[1 + i];
    xn[0] = -0.5 * fabs(Er) + al * al * s;
    return 1;
  }
  return 0;
}

/* one Newton attempt with one method (Sec. 4.9-4.10 "normal" Newton, D = 1) */
static void newton(const ictx *c, int method, const double x0[4], const double *Pgas0, ieval *best,
                   int *iters) {
  const orc_params *p = c->p;
  const double tol = (method == M_PMHD) ? p->tol_pmhd : p->tol_urad;
  double x[4];
  memcpy(x, x0, sizeof(x));
  double Pgas[12];
  memcpy(Pgas, Pgas0, sizeof(Pgas));
  ieval ev;
  eval_method(c, method, x, Pgas, &ev);
  *best = ev;
  if (!ev.ok) return;
  double hist[MAXH];
  int nh = 0;
  hist[nh++] = ev.eT;
  int nrise = 0, extra = 0, conv = 0, nneg = 0;
  for (int it = 0; it < p->max_iter && nh < MAXH - 1; it++) {
    /* pre-step checks (Sec. 4.10) */
    if (ev.eT < tol) conv = 1;
    if (conv) {
      if (!p->roundoff || extra >= 3) break;
      extra++;
    }
    if (!conv && it >= 5) {
      const double avg = (hist[nh - 5] + hist[nh - 4] + hist[nh - 3]) / 3.0;
      if (ev.eT > 0.5 * avg) break;
    }
    /* Jacobian */
    const double eI = (method == M_PMHD) ? ev.eIg : ev.eIr;
    const double delta = (eI < 1e-9) ? 1e-10 : 1e-8;
    double J[4][4];
    if (method == M_PMHD) jacobian_pmhd(c, x, delta, J);
    else if (jacobian_rad(c, method, x, &ev, delta, J)) break;
    double dx[4], res[4];
    method_residual(c, method, &ev, res);
    if (solve4(J, res, dx)) break;
    double xn[4];
    for (int i = 0; i < 4; i++) xn[i] = x[i] - dx[i];
    /* post-step checks (Sec. 4.10) */
    post_step(c, method, xn);
    ieval en;
    if (method == M_PMHD) {
      eval_pmhd(c, xn, &en);
    } else {
      eval_method(c, method, xn, ev.P, &en);
      int back = 0;
      while (!en.ok && back < 20) { /* back up half-way until the inversion succeeds */
        nneg++;
        for (int i = 0; i < 4; i++) xn[i] = 0.5 * (x[i] + xn[i]);
        eval_method(c, method, xn, ev.P, &en);
        back++;
      }
      if (!en.ok || nneg > 3) {
        (*iters)++;
        break;
      }
    }
    (*iters)++;
    int small = 1;
    for (int i = 0; i < 4; i++)
      if (fabs(xn[i] - x[i]) > 10.0 * EPS_M * fabs(x[i])) small = 0;
    memcpy(x, xn, sizeof(x));
    const double prev = hist[nh - 1];
    ev = en;
    hist[nh++] = ev.eT;
    if (ev.eT < best->eT) *best = ev;
    if (it >= 5 && ev.eT > prev) {
      nrise++;
      if (nrise >= 5) break;
    }
    if (small) break;
  }
}

/* The staged attempt of one method (Sec. 4.10): stage 1 one momentum-only
 * Newton step (the 3x3 momentum block, x_0 held), damped by 1/2; stage 2
 * energy-only (entropy-only) Newton steps on x_0 with the momenta held, the
 * first damped by 1/2, until that equation's error is below the method's
 * tolerance, the step is at round-off or max_iter steps; stage 3 the full
 * 4-D Newton for up to 40 steps, the first damped by 1/4, with the stopping
 * rules of newton().  A post-step correction of u_g, the radiation energy or
 * Ebar that recurs 2 times (4 for the entropy equation) within stage 1 or 2
 * holds the prior value and moves on to the next stage. */
static void newton_staged(const ictx *c, int method, const double x0[4], const double *Pgas0,
                          ieval *best, int *iters) {
  const orc_params *p = c->p;
  const double tol = (method == M_PMHD) ? p->tol_pmhd : p->tol_urad;
  const int nmod_max = c->entropy ? 4 : 2;
  double x[4];
  memcpy(x, x0, sizeof(x));
  double Pgas[12];
  memcpy(Pgas, Pgas0, sizeof(Pgas));
  ieval ev;
  eval_method(c, method, x, Pgas, &ev);
  *best = ev;
  if (!ev.ok) return;
  for (int stage = 1; stage <= 2; stage++) {
    const int nmax = (stage == 1) ? 1 : p->max_iter;
    int nmod = 0;
    for (int it = 0; it < nmax; it++) {
      const double eI = (method == M_PMHD) ? ev.eIg : ev.eIr;
      /* stage 2 converges the energy (entropy) equation's own error */
      if (stage == 2 && ((method == M_PMHD) ? ev.e0g : ev.e0r) < tol) break;
      const double delta = (eI < 1e-9) ? 1e-10 : 1e-8;
      double J[4][4];
      if (method == M_PMHD) jacobian_pmhd(c, x, delta, J);
      else if (jacobian_rad(c, method, x, &ev, delta, J)) break;
      double res[4], xn[4];
      method_residual(c, method, &ev, res);
      memcpy(xn, x, sizeof(xn));
      const double D = (it == 0) ? 0.5 : 1.0;
      if (stage == 1) {
        double A[4][4] = {{1.0, 0.0, 0.0, 0.0}, {0.0}, {0.0}, {0.0}};
        for (int i = 1; i < 4; i++)
          for (int j = 1; j < 4; j++) A[i][j] = J[i][j];
        const double r[4] = {0.0, res[1], res[2], res[3]};
        double dx[4];
        if (solve4(A, r, dx)) break;
        for (int i = 1; i < 4; i++) xn[i] = x[i] - D * dx[i];
      } else {
        if (!(fabs(J[0][0]) > 0.0) || !isfinite(J[0][0])) break;
        xn[0] = x[0] - D * res[0] / J[0][0];
      }
      if (post_step(c, method, xn)) {
        if (++nmod >= nmod_max) break; /* hold the prior value, next stage */
      }
      ieval en;
      eval_method(c, method, xn, ev.P, &en);
      (*iters)++;
      if (!en.ok) break;
      int small = 1;
      for (int i = 0; i < 4; i++)
        if (fabs(xn[i] - x[i]) > 10.0 * EPS_M * fabs(x[i])) small = 0;
      memcpy(x, xn, sizeof(x));
      ev = en;
      if (ev.eT < best->eT) *best = ev;
      if (small) break;
    }
  }
  /* stage 3: the full 4-D solve, at most 40 steps, the first damped by 1/4 */
  double hist[MAXH];
  int nh = 0;
  hist[nh++] = ev.eT;
  int nrise = 0, extra = 0, conv = 0, nneg = 0;
  for (int it = 0; it < 40 && nh < MAXH - 1; it++) {
    if (ev.eT < tol) conv = 1;
    if (conv) {
      if (!p->roundoff || extra >= 3) break;
      extra++;
    }
    if (!conv && it >= 5) {
      const double avg = (hist[nh - 5] + hist[nh - 4] + hist[nh - 3]) / 3.0;
      if (ev.eT > 0.5 * avg) break;
    }
    const double eI = (method == M_PMHD) ? ev.eIg : ev.eIr;
    const double delta = (eI < 1e-9) ? 1e-10 : 1e-8;
    double J[4][4];
    if (method == M_PMHD) jacobian_pmhd(c, x, delta, J);
    else if (jacobian_rad(c, method, x, &ev, delta, J)) break;
    double dx[4], res[4];
    method_residual(c, method, &ev, res);
    if (solve4(J, res, dx)) break;
    const double D = (it == 0) ? 0.25 : 1.0;
    double xn[4];
    for (int i = 0; i < 4; i++) xn[i] = x[i] - D * dx[i];
    post_step(c, method, xn);
    ieval en;
    eval_method(c, method, xn, ev.P, &en);
    if (method != M_PMHD) {
      int back = 0;
      while (!en.ok && back < 20) {
        nneg++;
        for (int i = 0; i < 4; i++) xn[i] = 0.5 * (x[i] + xn[i]);
        eval_method(c, method, xn, ev.P, &en);
        back++;
      }
      if (!en.ok || nneg > 3) {
        (*iters)++;
        break;
      }
    }
    (*iters)++;
    if (!en.ok) break;
    int small = 1;
    for (int i = 0; i < 4; i++)
      if (fabs(xn[i] - x[i]) > 10.0 * EPS_M * fabs(x[i])) small = 0;
    memcpy(x, xn, sizeof(x));
    const double prev = hist[nh - 1];
    ev = en;
    hist[nh++] = ev.eT;
    if (ev.eT < best->eT) *best = ev;
    if (it >= 5 && ev.eT > prev) {
      nrise++;
      if (nrise >= 5) break;
    }
    if (small) break;
  }
}

/* Cold MHD attempt (Sec. 4.7: when neither the energy nor the entropy
 * equation has a solution, energy and entropy conservation are dropped).
 * The gas internal energy is held at x0[0] and the three gas momentum
 * equations are solved for u~^i with the PMHD residual, the radiation
 * following from total energy-momentum conservation as in PMHD; the energy
 * residuals are left out of e_T (c->cold).  Centred-difference Jacobian of
 * the 3 momentum residuals in u~^i, the stopping rules of newton(). */
static void newton_cold(const ictx *c, const double x0[4], ieval *best, int *iters) {
  const orc_params *p = c->p;
  double x[4];
  memcpy(x, x0, sizeof(x));
  ieval ev;
  eval_pmhd(c, x, &ev);
  *best = ev;
  if (!ev.ok) return;
  double hist[MAXH];
  int nh = 0;
  hist[nh++] = ev.eT;
  int nrise = 0, extra = 0, conv = 0;
  for (int it = 0; it < p->max_iter && nh < MAXH - 1; it++) {
    if (ev.eT < p->tol_pmhd) conv = 1;
    if (conv) {
      if (!p->roundoff || extra >= 3) break;
      extra++;
    }
    if (!conv && it >= 5) {
      const double avg = (hist[nh - 5] + hist[nh - 4] + hist[nh - 3]) / 3.0;
      if (ev.eT > 0.5 * avg) break;
    }
    const double delta = (ev.eIg < 1e-9) ? 1e-10 : 1e-8;
    /* 4x4 system with u_g pinned: row 0 reads dx_0 = 0 */
    double J[4][4] = {{1.0, 0.0, 0.0, 0.0}, {0.0}, {0.0}, {0.0}};
    for (int j = 1; j < 4; j++) {
      const double h = delta * (1.0 + fabs(x[j]));
      double xp[4], xm[4];
      memcpy(xp, x, sizeof(x));
      memcpy(xm, x, sizeof(x));
      xp[j] += h;
      xm[j] -= h;
      ieval ep, em;
      eval_pmhd(c, xp, &ep);
      eval_pmhd(c, xm, &em);
      for (int i = 1; i < 4; i++) J[i][j] = (ep.Eg[i] - em.Eg[i]) / (2.0 * h);
    }
    const double res[4] = {0.0, ev.Eg[1], ev.Eg[2], ev.Eg[3]};
    double dx[4];
    if (solve4(J, res, dx)) break;
    double xn[4];
    for (int i = 0; i < 4; i++) xn[i] = x[i] - dx[i];
    ieval en;
    eval_pmhd(c, xn, &en);
    (*iters)++;
    int small = 1;
    for (int i = 0; i < 4; i++)
      if (fabs(xn[i] - x[i]) > 10.0 * EPS_M * fabs(x[i])) small = 0;
    memcpy(x, xn, sizeof(x));
    const double prev = hist[nh - 1];
    ev = en;
    hist[nh++] = ev.eT;
    if (ev.ok && ev.eT < best->eT) *best = ev;
    if (!ev.ok) break;
    if (it >= 5 && ev.eT > prev) {
      nrise++;
      if (nrise >= 5) break;
    }
    if (small) break;
  }
}

static void cell_context(const orc_params *p, const orc_geom *g, const double *Ui, double dt,
                         double chi_abs, double chi_es, ictx *c) {
  c->p = p;
  c->g = g;
  orc_spatial_gcon(g, c->gij);
  const double gd = g->gdet;
  c->rhout = Ui[0] / gd;
  for (int i = 0; i < 3; i++) c->B[i] = Ui[5 + i] / gd;
  for (int m = 0; m < 4; m++) {
    c->Tgi[m] = Ui[1 + m] / gd;
    c->Ri[m] = Ui[8 + m] / gd;
  }
  c->dt = dt;
  c->chi_abs = chi_abs;
  c->chi_es = chi_es;
  c->cold = 0;
  c->entropy = 0;
  c->Si = NAN;
}

/* Outputs and status of an accepted (or best) solution of one method
 * (Sec. 4.10-4.11): the iterated side's conserved quantities from the
 * solution, the other side's from total conservation, the BASIC re-inversion
 * where TYPE2 met E_rad <= 0, radiation recomputed where a limiter acted. */
static int emit(const ictx *c, const ieval *best, int method, int status, const double *Ui,
                double *Pout, double *Uout) {
  const orc_params *p = c->p;
  const orc_geom *g = c->g;
  const double gd = g->gdet;
  status |= (method == M_PMHD) ? ORC_ST_PMHD : (method == M_URAD) ? ORC_ST_URAD : ORC_ST_PRAD;
  if (best->eT > p->tol_fail) status |= ORC_ST_FAIL;
  else if (best->eT > p->tol_accept) status |= ORC_ST_NOT_ACCEPT;
  if (best->radflags & 1) status |= ORC_ST_TYPE2_NEG;
  memcpy(Pout, best->P, sizeof(double) * 12);
  double Ucons_rad[4], Ucons_gas[4];
  for (int m = 0; m < 4; m++) {
    if (method == M_PMHD) {
      Ucons_gas[m] = best->Tg[m];
      Ucons_rad[m] = c->Ri[m] - (best->Tg[m] - c->Tgi[m]);
    } else if (method == M_PRAD) {
      Ucons_rad[m] = best->Rr[m];
      Ucons_gas[m] = c->Tgi[m] - (best->Rr[m] - c->Ri[m]);
    } else {
      Ucons_rad[m] = best->x[m];
      Ucons_gas[m] = c->Tgi[m] - (best->x[m] - c->Ri[m]);
    }
  }
  int rad_changed = (best->radflags != 0);
  if (method == M_PMHD && (best->radflags & 1)) {
    /* the accepted solution met E_rad < 0 under TYPE2: re-invert with BASIC */
    double U[12];
    memset(U, 0, sizeof(U));
    for (int m = 0; m < 4; m++) U[8 + m] = gd * Ucons_rad[m];
    orc_rad_invert(p, g, U, 0, Pout);
    status |= ORC_ST_BASIC;
    rad_changed = 1;
  }
  if (rad_changed) rad_cons(c, Pout, Ucons_rad);
  Uout[0] = Ui[0];
  for (int m = 0; m < 4; m++) {
    Uout[1 + m] = gd * Ucons_gas[m];
    Uout[8 + m] = gd * Ucons_rad[m];
  }
  for (int i = 0; i < 3; i++) Uout[5 + i] = Ui[5 + i];
  if (!(Pout[1] > 0.0)) status |= ORC_ST_FAIL;
  return status;
}

/* Conditions of the cold MHD attempt (Sec. 4.11, backups), on the prior
 * primitives and the explicit gas state t^t_mu = T^t_mu + rho0 u^t delta^t_mu:
 * u_g < 0.1 rho0 u^i u_i (the gas cold against its motion) and
 * |t^t_t t^{tt}| < 0.1 |t^t_i t^{ti}| (its energy small against its
 * momentum).  The paper's third condition, on R^t_t R^{tt} against
 * R^t_i R^{ti}, cannot hold for an M1 state (|F| <= E) and is not applied. */
static int cold_allowed(const ictx *c, const double *Pguess) {
  const orc_geom *g = c->g;
  double ucon[4], ucov[4];
  orc_ucon(g, Pguess + 2, ucon);
  for (int a = 0; a < 4; a++) {
    ucov[a] = 0.0;
    for (int b = 0; b < 4; b++) ucov[a] += g->gcov[a][b] * ucon[b];
  }
  double usp = 0.0;
  for (int i = 1; i < 4; i++) usp += ucon[i] * ucov[i];
  if (!(Pguess[1] < 0.1 * Pguess[0] * fabs(usp))) return 0;
  double tup[4];
  for (int a = 0; a < 4; a++) {
    tup[a] = 0.0;
    for (int b = 0; b < 4; b++) tup[a] += g->gcon[a][b] * c->Tgi[b];
  }
  double en = c->Tgi[0] * tup[0], mo = 0.0;
  for (int i = 1; i < 4; i++) mo += c->Tgi[i] * tup[i];
  return fabs(en) < 0.1 * fabs(mo);
}

/* Cold MHD solve with u_g held at u_c, guess u~^i from Pguess; returns 0
 * and fills the outputs (status bit ORC_ST_COLD in place of ORC_ST_PMHD)
 * when e_T of the momentum equations is within tol_fail, 1 otherwise. */
static int cold_cell(const ictx *c0, const double *Ui, const double *Pguess, double u_c,
                     int status, double *Pout, double *Uout, orc_implicit_info *info) {
  ictx c = *c0;
  c.cold = 1;
  const double x0[4] = {u_c, Pguess[2], Pguess[3], Pguess[4]};
  ieval best;
  int iters = 0;
  newton_cold(&c, x0, &best, &iters);
  info->iters += iters;
  if (!best.ok || !(best.eT <= c.p->tol_fail)) return 1;
  const int st = emit(&c, &best, M_PMHD, status, Ui, Pout, Uout);
  info->status = (st & ~ORC_ST_PMHD) | ORC_ST_COLD;
  info->err = best.eT;
  return 0;
}

void orc_implicit_cold(const orc_params *p, const orc_geom *g, const double *Ui,
                       const double *Pguess, double dt, double chi_abs, double chi_es, double u_c,
                       double *Pout, double *Uout, orc_implicit_info *info) {
  ictx c;
  cell_context(p, g, Ui, dt, chi_abs, chi_es, &c);
  info->iters = 0;
  if (cold_cell(&c, Ui, Pguess, u_c, 0, Pout, Uout, info)) {
    memcpy(Pout, Pguess, sizeof(double) * 12);
    memcpy(Uout, Ui, sizeof(double) * 12);
    info->status = ORC_ST_FAIL;
    info->err = INFINITY;
  }
}

/* one phase of the full cascade (Sec. 4.10) with the energy or, with
 * c->entropy, the entropy equation: the normal attempts (PMHD, URAD, PRAD;
 * URAD and PRAD first in the extreme regime) until one is acceptable, then
 * the staged attempts of PMHD, URAD and PRAD (reading: for every cell the
 * normal attempts leave without an acceptable solution; the printed
 * restriction to the extreme regime is read as garbled).
 * Each attempt starts from the previous attempts' best solution when its
 * e_T < 1e-4, otherwise from the method's own guess: PMHD the thin-limit
 * primitives Pthin (staged: u_g from the explicit entropy where it exists),
 * URAD R^t_nu(P_n), PRAD the thin-limit radiation primitives Pradthin. */
static void run_phase(const ictx *c, int extreme, const double *Pguess, const double *Pthin,
                      const double *Pradthin, ieval *best, int *best_method, int *staged,
                      int *iters) {
  const orc_params *p = c->p;
  const double acc = p->roundoff ? 10.0 * p->tol_pmhd : p->tol_accept;
  const int normal[3] = {extreme ? M_URAD : M_PMHD, extreme ? M_PRAD : M_URAD,
                         extreme ? M_PMHD : M_PRAD};
  const int stages[3] = {M_PMHD, M_URAD, M_PRAD};
  memset(best, 0, sizeof(*best));
  best->eT = INFINITY;
  *best_method = -1;
  *staged = 0;
  for (int pass = 0; pass < 2; pass++) {
    for (int mi = 0; mi < 3; mi++) {
      const int method = pass ? stages[mi] : normal[mi];
      const int use_prev = (*best_method >= 0 && best->eT < 1e-4);
      double x0[4], Pg[12];
      if (method == M_PMHD) {
        const double *src = use_prev ? best->P : Pthin;
        memcpy(Pg, src, sizeof(Pg));
        x0[0] = src[1];
        for (int i = 0; i < 3; i++) x0[1 + i] = src[2 + i];
        if (pass == 1 && !use_prev && isfinite(c->Si) && c->rhout > 0.0) {
          /* u_g from the specific entropy Si/(rho0 u^t) at the prior rho0 */
          const double sp = c->Si / c->rhout, rho = Pthin[0], n = 1.0 / (p->gam - 1.0);
          const double pg = exp((sp + (n + 1.0) * log(rho)) / n);
          if (isfinite(pg) && pg > 0.0) x0[0] = pg / (p->gam - 1.0);
        }
      } else if (method == M_URAD) {
        if (use_prev) {
          memcpy(x0, best->Rr, sizeof(x0));
          memcpy(Pg, best->P, sizeof(Pg));
        } else {
          rad_cons(c, Pguess, x0);
          memcpy(Pg, Pguess, sizeof(Pg));
        }
      } else {
        const double *src = use_prev ? best->P : Pradthin;
        memcpy(Pg, src, sizeof(Pg));
        x0[0] = src[8];
        for (int i = 0; i < 3; i++) x0[1 + i] = src[9 + i];
      }
      ieval bm;
      if (pass == 0) newton(c, method, x0, Pg, &bm, iters);
      else newton_staged(c, method, x0, Pg, &bm, iters);
      if (bm.ok && bm.eT < best->eT) {
        *best = bm;
        *best_method = method;
        *staged = pass;
      }
      if (best->eT < acc) return;
    }
  }
}

/* The full cascade (Sec. 4.10-4.11): the energy phase; when it finds no
 * acceptable solution or one with u_g <= 0, the entropy phase (explicit
 * entropy Si needed); the entropy solution is taken when acceptable,
 * otherwise the smaller e_T of the two within tol_fail (u_g > 0); with
 * neither, the cold MHD limit where its conditions hold. */
static void cascade_full(ictx *c, int extreme, const double *Ui, const double *Pguess,
                         const double *Pthin, int status, double *Pout, double *Uout,
                         orc_implicit_info *info) {
  const orc_params *p = c->p;
  const double acc = p->roundoff ? 10.0 * p->tol_pmhd : p->tol_accept;
  int iters = 0;
  /* PRAD's thin-limit guess: the radiation inversion of R(i) when
   * dt kappa_tot(P_n) < 2/3 */
  double Pradthin[12];
  memcpy(Pradthin, Pguess, sizeof(Pradthin));
  if (c->dt * (c->chi_abs + c->chi_es) * Pguess[0] < 2.0 / 3.0) {
    double U[12];
    memset(U, 0, sizeof(U));
    for (int m = 0; m < 4; m++) U[8 + m] = c->g->gdet * c->Ri[m];
    double Pr[12];
    memcpy(Pr, Pguess, sizeof(Pr));
    orc_rad_invert(p, c->g, U, 0, Pr);
    if (Pr[8] > 0.0 && isfinite(Pr[8])) memcpy(Pradthin + 8, Pr + 8, sizeof(double) * 4);
  }
  ieval bE, bS;
  int mE, mS, sE, sS;
  c->entropy = 0;
  run_phase(c, extreme, Pguess, Pthin, Pradthin, &bE, &mE, &sE, &iters);
  const int energy_ok = mE >= 0 && bE.P[1] > 0.0;
  int use = -1; /* 0 energy, 1 entropy */
  if (energy_ok && bE.eT < acc) {
    use = 0;
  } else {
    mS = -1;
    if (isfinite(c->Si)) {
      c->entropy = 1;
      run_phase(c, extreme, Pguess, Pthin, Pradthin, &bS, &mS, &sS, &iters);
      c->entropy = 0;
    }
    const int entropy_ok = mS >= 0 && bS.P[1] > 0.0;
    if (entropy_ok && bS.eT < acc) use = 1;
    else {
      const int eo = energy_ok && bE.eT <= p->tol_fail, so = entropy_ok && bS.eT <= p->tol_fail;
      if (eo && so) use = (bS.eT < bE.eT) ? 1 : 0;
      else if (eo) use = 0;
      else if (so) use = 1;
    }
  }
  const int status0 = status;
  if (use == 0) {
    status = emit(c, &bE, mE, status, Ui, Pout, Uout) | (sE ? ORC_ST_STAGED : 0);
    info->err = bE.eT;
  } else if (use == 1) {
    status = emit(c, &bS, mS, status, Ui, Pout, Uout) | ORC_ST_ENTROPY | (sS ? ORC_ST_STAGED : 0);
    info->err = bS.eT;
  } else if (mE >= 0) {
    status = emit(c, &bE, mE, status, Ui, Pout, Uout) | ORC_ST_FAIL;
    info->err = bE.eT;
  } else {
    memcpy(Pout, Pguess, sizeof(double) * 12);
    for (int i = 0; i < 12; i++) Uout[i] = Ui[i];
    status |= ORC_ST_FAIL;
    info->err = INFINITY;
  }
  info->status = status;
  info->iters = iters;
  if ((status & ORC_ST_FAIL) && p->cold && p->u_floor > 0.0 && cold_allowed(c, Pguess)) {
    double Pc[12], Uc[12];
    orc_implicit_info ic = *info;
    if (cold_cell(c, Ui, Pguess, p->u_floor, status0, Pc, Uc, &ic) == 0) {
      memcpy(Pout, Pc, sizeof(Pc));
      memcpy(Uout, Uc, sizeof(Uc));
      *info = ic;
    } else {
      info->iters = ic.iters;
    }
  }
}

void orc_implicit_cell(const orc_params *p, const orc_geom *g, const double *Ui,
                       const double *Pguess, double dt, double chi_abs, double chi_es,
                       double *Pout, double *Uout, orc_implicit_info *info) {
  /* a cell without a grid: its explicit entropy is that of its prior
   * primitives (no flux divergence, and the entropy has no other explicit
   * source) */
  double ucon[4];
  orc_ucon(g, Pguess + 2, ucon);
  const double Si = g->gdet * orc_entropy(p, Pguess) * ucon[0];
  orc_implicit_cell_s(p, g, Ui, Si, Pguess, dt, chi_abs, chi_es, Pout, Uout, info);
}

void orc_implicit_cell_s(const orc_params *p, const orc_geom *g, const double *Ui, double Si,
                         const double *Pguess, double dt, double chi_abs, double chi_es,
                         double *Pout, double *Uout, orc_implicit_info *info) {
  ictx c;
  cell_context(p, g, Ui, dt, chi_abs, chi_es, &c);
  c.Si = Si / g->gdet;
  int status = 0, iters = 0;

  /* extreme radiation sub-dominance (Sec. 4.10): radiation energy, or the
   * fluid-frame radiation energy against u_g, below 10 eps */
  double Ehat;
  {
    orc_gas s;
    orc_rad r;
    orc_gas_state(p, g, Pguess, &s);
    orc_rad_state(g, Pguess, &r);
    Ehat = 0.0;
    for (int a = 0; a < 4; a++)
      for (int b = 0; b < 4; b++) Ehat += r.R[a][b] * s.ucov[a] * s.ucon[b];
  }
  const int extreme = (fabs(c.Ri[0]) <= 10.0 * EPS_M * (fabs(c.Tgi[0]) + fabs(c.Ri[0]))) ||
                      (fabs(Ehat) <= 10.0 * EPS_M * (fabs(Pguess[1]) + fabs(Ehat)));
  if (extreme) status |= ORC_ST_EXTREME;

  /* PMHD guess: prior primitives, or the thin-limit inversion of U_(i) when
   * the temporal optical depth dt kappa_tot(P_n) < 2/3 (Sec. 4.10) */
  double Pthin[12];
  memcpy(Pthin, Pguess, sizeof(Pthin));
  const double tau = dt * (chi_abs + chi_es) * Pguess[0];
  if (tau < 2.0 / 3.0) {
    double Pt[12];
    memcpy(Pt, Pguess, sizeof(Pt));
    if (orc_mhd_invert(p, g, Ui, Pguess, Pt) == 0) memcpy(Pthin, Pt, sizeof(double) * 8);
    else status |= ORC_ST_C2P_FAIL;
  }

  if (p->cascade) {
    cascade_full(&c, extreme, Ui, Pguess, Pthin, status, Pout, Uout, info);
    return;
  }
  const int order[2] = {extreme ? M_URAD : M_PMHD, extreme ? M_PMHD : M_URAD};
  ieval best;
  memset(&best, 0, sizeof(best));
  best.eT = INFINITY;
  int best_method = -1;
  for (int mi = 0; mi < 2; mi++) {
    const int method = order[mi];
    double x0[4];
    double Pg[12];
    const int use_prev = (best_method >= 0 && best.eT < 1e-4);
    if (method == M_PMHD) {
      const double *src = use_prev ? best.P : Pthin;
      x0[0] = src[1];
      for (int i = 0; i < 3; i++) x0[1 + i] = src[2 + i];
      memcpy(Pg, src, sizeof(Pg));
    } else {
      if (use_prev) {
        memcpy(x0, best.Rr, sizeof(x0));
        memcpy(Pg, best.P, sizeof(Pg));
      } else {
        rad_cons(&c, Pguess, x0);
        memcpy(Pg, Pguess, sizeof(Pg));
      }
    }
    ieval bm;
    newton(&c, method, x0, Pg, &bm, &iters);
    if (bm.ok && bm.eT < best.eT) {
      best = bm;
      best_method = method;
    }
    /* acceptable: no further method (Sec. 4.10); when iterating to round-off
     * the next method is tried unless one came within 10x the PMHD
     * tolerance (a method stalled at its own precision floor is kept) */
    if (best.eT < (p->roundoff ? 10.0 * p->tol_pmhd : p->tol_accept)) break;
  }

  /* status bits of the set-up (EXTREME, C2P_FAIL) */
  const int status0 = status;
  if (best_method < 0) {
    memcpy(Pout, Pguess, sizeof(double) * 12);
    for (int i = 0; i < 12; i++) Uout[i] = Ui[i];
    status |= ORC_ST_FAIL;
    info->err = INFINITY;
  } else {
    status = emit(&c, &best, best_method, status, Ui, Pout, Uout);
    info->err = best.eT;
  }
  info->status = status;
  info->iters = iters;
  /* no energy solution: the cold MHD limit (the entropy equation, tried
   * before it in the paper's cascade, needs an evolved entropy tracer that
   * this step does not carry) */
  if ((status & ORC_ST_FAIL) && p->cold && p->u_floor > 0.0 && cold_allowed(&c, Pguess)) {
    double Pc[12], Uc[12];
    orc_implicit_info ic = *info;
    if (cold_cell(&c, Ui, Pguess, p->u_floor, status0, Pc, Uc, &ic) == 0) {
      memcpy(Pout, Pc, sizeof(Pc));
      memcpy(Uout, Uc, sizeof(Uc));
      *info = ic;
    } else {
      info->iters = ic.iters;
    }
  }
}

void orc_implicit_batch(const orc_params *p, long n, const double *Ui, const double *Pg,
                        const double *dtc, const double *chi_abs, const double *chi_es,
                        double *Pout, double *Uout, int *iters, int *status) {
  orc_geom g;
  orc_geom_point(p, 0.0, 0.5, &g);
#pragma omp parallel for schedule(dynamic, 256)
  for (long c = 0; c < n; c++) {
    double U[12], P[12], Po[12], Uo[12];
    for (int q = 0; q < 12; q++) {
      U[q] = Ui[q * n + c];
      P[q] = Pg[q * n + c];
    }
    orc_implicit_info info;
    orc_implicit_cell(p, &g, U, P, dtc[c], chi_abs[c], chi_es[c], Po, Uo, &info);
    for (int q = 0; q < 12; q++) {
      Pout[q * n + c] = Po[q];
      Uout[q * n + c] = Uo[q];
    }
    if (iters) iters[c] = info.iters;
    if (status) status[c] = info.status;
  }
}

/* One attempt of one method alone, for tests: method 0 PMHD, 1 URAD, 2 PRAD;
 * staged != 0 the staged form; entropy != 0 the entropy equation (Si =
 * sqrt(-g) [S u^t]_(i)); each method from its own guess as in the cascade's
 * first attempt.  Status: the method bit, ORC_ST_FAIL above tol_fail. */
void orc_implicit_attempt(const orc_params *p, const orc_geom *g, const double *Ui, double Si,
                          const double *Pguess, double dt, double chi_abs, double chi_es,
                          int method, int staged, int entropy, double *Pout, double *Uout,
                          orc_implicit_info *info) {
  ictx c;
  cell_context(p, g, Ui, dt, chi_abs, chi_es, &c);
  c.Si = Si / g->gdet;
  c.entropy = entropy;
  double Pthin[12], Pradthin[12];
  memcpy(Pthin, Pguess, sizeof(Pthin));
  memcpy(Pradthin, Pguess, sizeof(Pradthin));
  if (dt * (chi_abs + chi_es) * Pguess[0] < 2.0 / 3.0) {
    double Pt[12];
    memcpy(Pt, Pguess, sizeof(Pt));
    if (orc_mhd_invert(p, g, Ui, Pguess, Pt) == 0) memcpy(Pthin, Pt, sizeof(double) * 8);
    double U[12];
    memset(U, 0, sizeof(U));
    for (int m = 0; m < 4; m++) U[8 + m] = Ui[8 + m];
    double Pr[12];
    memcpy(Pr, Pguess, sizeof(Pr));
    orc_rad_invert(p, g, U, 0, Pr);
    if (Pr[8] > 0.0 && isfinite(Pr[8])) memcpy(Pradthin + 8, Pr + 8, sizeof(double) * 4);
  }
  double x0[4], Pg[12];
  if (method == M_PMHD) {
    memcpy(Pg, Pthin, sizeof(Pg));
    x0[0] = Pthin[1];
    for (int i = 0; i < 3; i++) x0[1 + i] = Pthin[2 + i];
  } else if (method == M_URAD) {
    rad_cons(&c, Pguess, x0);
    memcpy(Pg, Pguess, sizeof(Pg));
  } else {
    memcpy(Pg, Pradthin, sizeof(Pg));
    x0[0] = Pradthin[8];
    for (int i = 0; i < 3; i++) x0[1 + i] = Pradthin[9 + i];
  }
  ieval best;
  int iters = 0;
  if (staged) newton_staged(&c, method, x0, Pg, &best, &iters);
  else newton(&c, method, x0, Pg, &best, &iters);
  info->iters = iters;
  if (!best.ok) {
    memcpy(Pout, Pguess, sizeof(double) * 12);
    for (int i = 0; i < 12; i++) Uout[i] = Ui[i];
    info->status = ORC_ST_FAIL;
    info->err = INFINITY;
    return;
  }
  info->status = emit(&c, &best, method, 0, Ui, Pout, Uout) | (entropy ? ORC_ST_ENTROPY : 0);
  info->err = best.eT;
}
