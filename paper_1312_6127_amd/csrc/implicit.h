// Implicit radiation 4-force solve for one cell on the device (Sec. 4.7-4.11).
//
// Unknowns are iterated with an undamped Newton method ("normal" Newton of
// Sec. 4.10).  PMHD iterates the gas primitives (u_g, u~^i); its 4x4
// Jacobian is exact, built from dual-number evaluations of the residual in
// passes of NJ directions (fewer live registers per pass).  URAD iterates
// R^t_nu, inverts T^t_nu = T(i) - Delta R to gas primitives inside every
// residual and uses a one-sided finite-difference Jacobian (Sec. 4.9).
// Pre-step checks, post-step checks, stopping rules, guesses, method order
// and acceptance follow Sec. 4.10-4.11.
//
// The work is split for the GPU: a lean kernel runs the common case (PMHD
// first, accepted) and appends every other cell to a work list; a second
// kernel runs the full cascade on the list.  Both run the same first PMHD
// attempt from the same guess, so results equal those of one cascade.
#pragma once
#include <float.h>

#include <type_traits>

#include "invert.h"

#ifndef GRRMHD_NJ
#define GRRMHD_NJ 4   // Jacobian directions per dual-number pass (4: one pass)
#endif
#ifndef GRRMHD_URAD_EXACT
#define GRRMHD_URAD_EXACT 1   // URAD Jacobian: 1 exact (dual numbers), 0 one-sided differences
#endif

enum { M_PMHD = 0, M_URAD = 1, M_PRAD = 2 };

struct Cell {
  Metric m;
  double rhout, B[3];
  double Tgi[4], Ri[4];   // explicit gas (T^t_t + rho u^t, T^t_i) and radiation R^t_nu
  double dt, chi_abs, chi_es;
  int cold;               // cold MHD: energy residuals left out of the errors
  double Si;              // explicit [S u^t]_(i) per sqrt(-g) (NAN: none); entropy methods
};

struct Eval {
  double x[4];
  double P[12];
  double Eg[4], Er[4];
  double eT, eIg, eIr;
  double e0g, e0r;        // normalised errors of the energy (entropy) equation
  double Es;              // entropy residual (entropy methods)
  int radflags, ok;
};

struct Phys {
  double gam, arad, gamma_max, ymax;
};

struct Opts {
  double tol_pmhd, tol_urad, tol_accept, tol_fail;
  int max_iter, roundoff;
  int cold;         // try the cold MHD limit where no energy solution is found
  double u_floor;   // u_g of the cold limit
};

DEV double snorm3(const Metric& m, const double V[4]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) s += gamup(m, i, j) * V[1 + i] * V[1 + j];
  return ::sqrt(fmax(s, 0.0));
}

// Normalised errors (Sec. 4.8): gas residual over gas-scale terms and
// dt|G|, radiation residual over radiation-scale terms and dt|G|; spatial
// parts merged in the normal observer's orthonormal basis plus the energy
// scale; e_T = 1/4 sum over equations of the larger of the two.
DEV void norm_errors(const Cell& c, const double Tg[4], const double Rr[4], const double G[4],
                     Eval& e, double es = -1.0) {
  double Gdt[4];
#pragma unroll
  for (int k = 0; k < 4; k++) Gdt[k] = c.dt * G[k];
  const double g0 = ::fabs(Gdt[0]), gs = snorm3(c.m, Gdt);
  double ntg = ::fabs(Tg[0]) + ::fabs(c.Tgi[0]) + g0;
  double ntr = ::fabs(Rr[0]) + ::fabs(c.Ri[0]) + g0;
  if (!(ntg > 0.0)) ntg = 1e-300;
  if (!(ntr > 0.0)) ntr = 1e-300;
  const double nsg = snorm3(c.m, Tg) + snorm3(c.m, c.Tgi) + gs + ntg;
  const double nsr = snorm3(c.m, Rr) + snorm3(c.m, c.Ri) + gs + ntr;
  double eg[4], er[4];
  eg[0] = ::fabs(e.Eg[0]) / ntg;
  er[0] = ::fabs(e.Er[0]) / ntr;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    const double w = ::sqrt(gamup(c.m, i, i));
    eg[1 + i] = ::fabs(e.Eg[1 + i]) * w / nsg;
    er[1 + i] = ::fabs(e.Er[1 + i]) * w / nsr;
  }
  // entropy methods: the entropy equation's error in the energy slot
  if (es >= 0.0) eg[0] = er[0] = es;
  if ((e.radflags & 1) || c.cold) eg[0] = er[0] = 0.0;
  e.e0g = eg[0];
  e.e0r = er[0];
  double t = 0.0, ig = 0.0, ir = 0.0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    t += fmax(eg[k], er[k]);
    ig += eg[k];
    ir += er[k];
  }
  e.eT = 0.25 * t;
  e.eIg = 0.25 * ig;
  e.eIr = 0.25 * ir;
  if (!isfinite(e.eT)) {
    e.eT = INFINITY;
    e.ok = 0;
  }
}

// Entropy equation (eq. source6 with G_S = -G^mu u_mu / T_gas, eq. GS),
// weighted by T_gas: E_S = T_gas ([S u^t] - [S u^t]_(i)) + dt G^mu u_mu with
// S = rho0 ln(p^n / rho0^(n+1)), n = 1/(gam - 1); its norm (returned in ns)
// is the sum of its terms' magnitudes plus the gas energy scale.
template <class D>
DEV D entropy_residual(const Cell& c, double gam, const Gas<D>& s, const D G[4], double ntg,
                       double& ns) {
  const double n = 1.0 / (gam - 1.0);
  const D S = s.rho * (n * log(s.pg) - (n + 1.0) * log(s.rho));
  const D Sut = S * s.v.ucon[0];
  const D T = s.pg / s.rho;
  D Gu = G[0] * s.v.ucon[0];
#pragma unroll
  for (int k = 1; k < 4; k++) Gu = Gu + G[k] * s.v.ucon[k];
  const D TS = T * Sut, TSi = T * c.Si, dGu = c.dt * Gu;
  ns = ::fabs(val(TS)) + ::fabs(val(TSi)) + ::fabs(val(dGu)) + ntg;
  return (TS - TSi) + dGu;
}

// gas energy norm |T^t_t + rho u^t| + |its explicit value| + dt |G_t| (Sec. 4.8)
DEV double gas_energy_norm(const Cell& c, double Tg0, double G0) {
  const double n = ::fabs(Tg0) + ::fabs(c.Tgi[0]) + ::fabs(c.dt * G0);
  return (n > 0.0) ? n : 1e-300;
}

// PMHD residual (Sec. 4.8, PMHD steps in order): rho0 = (rho u^t)/u^t;
// T^t_nu from the gas; Delta R = -Delta T; TYPE2 radiation inversion; R
// recomputed; G; residuals.  With D = Dual<N> one pass seeds Jacobian
// columns k0..k0+N-1; with D = double it evaluates the residual alone.
template <class D, bool ENT = false>
DEV void pmhd_pass(const Cell& c, const Phys& ph, const double x[4], int k0, Eval& e,
                   double J[4][4]) {
  D ug(x[0]), ut[3] = {D(x[1]), D(x[2]), D(x[3])};
  if constexpr (!std::is_same<D, double>::value) {
    constexpr int N = sizeof(D::d) / sizeof(double);
#pragma unroll
    for (int j = 0; j < N; j++) {
      const int k = k0 + j;
      if (k == 0) ug.d[j] = 1.0;
      if (k == 1) ut[0].d[j] = 1.0;
      if (k == 2) ut[1].d[j] = 1.0;
      if (k == 3) ut[2].d[j] = 1.0;
    }
  }
  D B[3] = {D(c.B[0]), D(c.B[1]), D(c.B[2])};
  Gas<D> s;
  {
    Vel<D> v;
    make_vel(c.m, ut, v);
    const D rho = c.rhout / v.ucon[0];
    make_gas(c.m, ph.gam, rho, ug, ut, B, s);
  }
  D row[8];
  gas_row(s, B, 0, row);
  D R[4];
#pragma unroll
  for (int k = 0; k < 4; k++) R[k] = c.Ri[k] - (row[1 + k] - c.Tgi[k]);
  D Eb, utr[3];
  e.radflags = rad_invert(c.m, ph.gamma_max, ph.ymax, 1, R, Eb, utr);
  Vel<D> r;
  make_vel(c.m, utr, r);
  const D Tgas = s.pg / s.rho;
  const D T2 = Tgas * Tgas;
  const D kabs = c.chi_abs * s.rho, kes = c.chi_es * s.rho;
  const D lam = kabs * ph.arad * (T2 * T2);
  D G[4];
  four_force(s.v, r, Eb, kabs, kes, lam, G);
  double Tg[4], Rr[4], Gv[4];
  D Rrow[4];
  rad_row(r, Eb, 0, Rrow);
  double es = -1.0;
  D Es(0.0);
  if constexpr (ENT) {
    double ns;
    Es = entropy_residual(c, ph.gam, s, G, gas_energy_norm(c, val(row[1]), val(G[0])), ns);
    es = ::fabs(val(Es)) / ns;
    e.Es = val(Es);
    if (!isfinite(e.Es)) es = INFINITY;
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const D Egk = (row[1 + k] - c.Tgi[k]) - c.dt * G[k];
    Tg[k] = val(row[1 + k]);
    Rr[k] = val(Rrow[k]);
    Gv[k] = val(G[k]);
    e.Eg[k] = val(Egk);
    e.Er[k] = (Rr[k] - c.Ri[k]) + c.dt * Gv[k];
    if constexpr (!std::is_same<D, double>::value) {
      constexpr int N = sizeof(D::d) / sizeof(double);
#pragma unroll
      for (int j = 0; j < N; j++) J[k][k0 + j] = (ENT && k == 0) ? Es.d[j] : Egk.d[j];
    }
  }
  if (k0 == 0) {
#pragma unroll
    for (int k = 0; k < 4; k++) e.x[k] = x[k];
    e.P[0] = val(s.rho);
    e.P[1] = x[0];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      e.P[2 + i] = x[1 + i];
      e.P[5 + i] = c.B[i];
      e.P[9 + i] = val(utr[i]);
    }
    e.P[8] = val(Eb);
    e.ok = 1;
    norm_errors(c, Tg, Rr, Gv, e, es);
  }
}

template <bool ENT = false>
DEV void eval_pmhd(const Cell& c, const Phys& ph, const double x[4], Eval& e, double J[4][4]) {
#pragma unroll
  for (int k0 = 0; k0 < 4; k0 += GRRMHD_NJ) pmhd_pass<Dual<GRRMHD_NJ>, ENT>(c, ph, x, k0, e, J);
}

// Residual alone: a Newton step close to the root reuses the factorised
// Jacobian of the previous evaluation (chord step).
template <bool ENT = false>
DEV void eval_pmhd_value(const Cell& c, const Phys& ph, const double x[4], Eval& e) {
  pmhd_pass<double, ENT>(c, ph, x, 0, e, nullptr);
}

// gas (T^t_t + rho u^t, T^t_i) of primitives P, without sqrt(-g)
DEV void gas_cons4(const Metric& m, double gam, const double* P, double Tg[4]) {
  Gas<double> s;
  make_gas(m, gam, P[0], P[1], P + 2, P + 5, s);
  double row[8];
  gas_row(s, P + 5, 0, row);
#pragma unroll
  for (int k = 0; k < 4; k++) Tg[k] = row[1 + k];
}

DEV void rad_cons4(const Metric& m, const double* P, double Rr[4]) {
  Vel<double> r;
  make_vel(m, P + 9, r);
  rad_row(r, P[8], 0, Rr);
}

// URAD residual (Sec. 4.8, URAD steps): gas from inverting T(i) - Delta R,
// radiation from TYPE2 inversion of x, both recomputed for consistency.
// Pgas (rho, u_g, u~^i) is the starting guess of the MHD iteration.
DEV void eval_urad(const Cell& c, const Phys& ph, const double x[4], const double Pgas[5],
                   Eval& e) {
  e.ok = 1;
#pragma unroll
  for (int k = 0; k < 4; k++) e.x[k] = x[k];
  double Tt[3] = {c.Tgi[1] - (x[1] - c.Ri[1]), c.Tgi[2] - (x[2] - c.Ri[2]),
                  c.Tgi[3] - (x[3] - c.Ri[3])};
  const double Eg = c.Tgi[0] - (x[0] - c.Ri[0]);
  double rho = Pgas[0], ug = Pgas[1], ut[3] = {Pgas[2], Pgas[3], Pgas[4]};
  if (mhd_invert(c.m, ph.gam, c.rhout, Eg, Tt, c.B, rho, ug, ut)) {
    e.ok = 0;
    e.eT = INFINITY;
    return;
  }
  double Eb, utr[3];
  e.radflags = rad_invert(c.m, ph.gamma_max, ph.ymax, 1, x, Eb, utr);
  Gas<double> s;
  make_gas(c.m, ph.gam, rho, ug, ut, c.B, s);
  double row[8];
  gas_row(s, c.B, 0, row);
  Vel<double> r;
  make_vel(c.m, utr, r);
  double Rr[4], Tg[4];
  rad_row(r, Eb, 0, Rr);
  const double Tgas = s.pg / rho;
  const double kabs = c.chi_abs * rho, kes = c.chi_es * rho;
  const double lam = kabs * ph.arad * (Tgas * Tgas) * (Tgas * Tgas);
  double G[4];
  four_force(s.v, r, Eb, kabs, kes, lam, G);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    Tg[k] = row[1 + k];
    e.Eg[k] = (row[1 + k] - c.Tgi[k]) - c.dt * G[k];
    e.Er[k] = (Rr[k] - c.Ri[k]) + c.dt * G[k];
  }
  e.P[0] = rho;
  e.P[1] = ug;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    e.P[2 + i] = ut[i];
    e.P[5 + i] = c.B[i];
    e.P[9 + i] = utr[i];
  }
  e.P[8] = Eb;
  norm_errors(c, Tg, Rr, G, e);
}

// URAD residual and its exact Jacobian dE_rad/dx in one dual-number pass:
// the same steps as eval_urad, the gas inversion differentiated by the
// implicit-function theorem (mhd_invert_dual).  Values equal eval_urad's.
template <bool ENT = false>
DEV void eval_urad_jac(const Cell& c, const Phys& ph, const double x[4], const double Pgas[5],
                       Eval& e, double J[4][4]) {
  using D = Dual<4>;
  e.ok = 1;
  D xd[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    e.x[k] = x[k];
    xd[k] = D::var(x[k], k);
  }
  const D Tt[3] = {c.Tgi[1] - (xd[1] - c.Ri[1]), c.Tgi[2] - (xd[2] - c.Ri[2]),
                   c.Tgi[3] - (xd[3] - c.Ri[3])};
  const D Eg = c.Tgi[0] - (xd[0] - c.Ri[0]);
  D rho, ug, ut[3];
  if (mhd_invert_dual<4>(c.m, ph.gam, c.rhout, Eg, Tt, c.B, Pgas[1], Pgas + 2, rho, ug, ut)) {
    e.ok = 0;
    e.eT = INFINITY;
    return;
  }
  D Eb, utr[3];
  e.radflags = rad_invert(c.m, ph.gamma_max, ph.ymax, 1, xd, Eb, utr);
  const D B[3] = {D(c.B[0]), D(c.B[1]), D(c.B[2])};
  Gas<D> s;
  make_gas(c.m, ph.gam, rho, ug, ut, B, s);
  D row[8];
  gas_row(s, B, 0, row);
  Vel<D> r;
  make_vel(c.m, utr, r);
  D Rr[4];
  rad_row(r, Eb, 0, Rr);
  const D Tgas = s.pg / rho;
  const D kabs = c.chi_abs * rho, kes = c.chi_es * rho;
  const D lam = kabs * ph.arad * (Tgas * Tgas) * (Tgas * Tgas);
  D G[4];
  four_force(s.v, r, Eb, kabs, kes, lam, G);
  double Tg[4], Rv[4], Gv[4];
  double es = -1.0;
  D Es(0.0);
  if constexpr (ENT) {
    double ns;
    Es = entropy_residual(c, ph.gam, s, G, gas_energy_norm(c, row[1].v, G[0].v), ns);
    es = ::fabs(Es.v) / ns;
    e.Es = Es.v;
    if (!isfinite(e.Es)) es = INFINITY;
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const D Erk = (Rr[k] - c.Ri[k]) + c.dt * G[k];
#pragma unroll
    for (int j = 0; j < 4; j++) J[k][j] = (ENT && k == 0) ? Es.d[j] : Erk.d[j];
    Tg[k] = row[1 + k].v;
    Rv[k] = Rr[k].v;
    Gv[k] = G[k].v;
    e.Eg[k] = (Tg[k] - c.Tgi[k]) - c.dt * Gv[k];
    e.Er[k] = Erk.v;
  }
  e.P[0] = rho.v;
  e.P[1] = ug.v;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    e.P[2 + i] = ut[i].v;
    e.P[5 + i] = c.B[i];
    e.P[9 + i] = utr[i].v;
  }
  e.P[8] = Eb.v;
  norm_errors(c, Tg, Rv, Gv, e, es);
}

// PRAD residual and its exact Jacobian dE_rad/dx in one dual-number pass
// (Sec. 4.8, PRAD steps): x = (Ebar, u~^i_rad); R^t_nu from the radiation
// primitives; the gas from the MHD inversion of T(i) - Delta R (Pgas starts
// it; its derivatives by the implicit-function theorem); G; residuals.
template <bool ENT = false>
DEV void eval_prad_jac(const Cell& c, const Phys& ph, const double x[4], const double Pgas[5],
                       Eval& e, double J[4][4]) {
  using D = Dual<4>;
  e.ok = 1;
  D Eb = D::var(x[0], 0), utr[3];
#pragma unroll
  for (int k = 0; k < 4; k++) e.x[k] = x[k];
#pragma unroll
  for (int i = 0; i < 3; i++) utr[i] = D::var(x[1 + i], 1 + i);
  Vel<D> r;
  make_vel(c.m, utr, r);
  D Rr[4];
  rad_row(r, Eb, 0, Rr);
  const D Tt[3] = {c.Tgi[1] - (Rr[1] - c.Ri[1]), c.Tgi[2] - (Rr[2] - c.Ri[2]),
                   c.Tgi[3] - (Rr[3] - c.Ri[3])};
  const D Eg = c.Tgi[0] - (Rr[0] - c.Ri[0]);
  D rho, ug, ut[3];
  if (mhd_invert_dual<4>(c.m, ph.gam, c.rhout, Eg, Tt, c.B, Pgas[1], Pgas + 2, rho, ug, ut)) {
    e.ok = 0;
    e.eT = INFINITY;
    return;
  }
  e.radflags = 0;
  const D B[3] = {D(c.B[0]), D(c.B[1]), D(c.B[2])};
  Gas<D> s;
  make_gas(c.m, ph.gam, rho, ug, ut, B, s);
  D row[8];
  gas_row(s, B, 0, row);
  const D Tgas = s.pg / rho;
  const D kabs = c.chi_abs * rho, kes = c.chi_es * rho;
  const D lam = kabs * ph.arad * (Tgas * Tgas) * (Tgas * Tgas);
  D G[4];
  four_force(s.v, r, Eb, kabs, kes, lam, G);
  double Tg[4], Rv[4], Gv[4];
  double es = -1.0;
  D Es(0.0);
  if constexpr (ENT) {
    double ns;
    Es = entropy_residual(c, ph.gam, s, G, gas_energy_norm(c, row[1].v, G[0].v), ns);
    es = ::fabs(Es.v) / ns;
    e.Es = Es.v;
    if (!isfinite(e.Es)) es = INFINITY;
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const D Erk = (Rr[k] - c.Ri[k]) + c.dt * G[k];
#pragma unroll
    for (int j = 0; j < 4; j++) J[k][j] = (ENT && k == 0) ? Es.d[j] : Erk.d[j];
    Tg[k] = row[1 + k].v;
    Rv[k] = Rr[k].v;
    Gv[k] = G[k].v;
    e.Eg[k] = (Tg[k] - c.Tgi[k]) - c.dt * Gv[k];
    e.Er[k] = Erk.v;
  }
  e.P[0] = rho.v;
  e.P[1] = ug.v;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    e.P[2 + i] = ut[i].v;
    e.P[5 + i] = c.B[i];
    e.P[9 + i] = x[1 + i];
  }
  e.P[8] = x[0];
  norm_errors(c, Tg, Rv, Gv, e, es);
}

// 4x4 solve with partial pivoting; 0 on success
DEV int solve4(double A[4][4], double b[4], double xo[4]) {
#pragma unroll
  for (int k = 0; k < 4; k++) {
    int p = k;
    double best = ::fabs(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < 4; i++)
      if (::fabs(A[i][k]) > best) { best = ::fabs(A[i][k]); p = i; }
    if (!(best > 0.0) || !isfinite(best)) return 1;
#pragma unroll
    for (int i = k + 1; i < 4; i++) {   // row swap with static indices only
      if (i == p) {
#pragma unroll
        for (int j = 0; j < 4; j++) { const double t = A[k][j]; A[k][j] = A[i][j]; A[i][j] = t; }
        const double t = b[k]; b[k] = b[i]; b[i] = t;
      }
    }
    const double inv = 1.0 / A[k][k];
#pragma unroll
    for (int i = k + 1; i < 4; i++) {
      const double f = A[i][k] * inv;
#pragma unroll
      for (int j = k; j < 4; j++) A[i][j] -= f * A[k][j];
      b[i] -= f * b[k];
    }
  }
#pragma unroll
  for (int i = 3; i >= 0; i--) {
    double s = b[i];
#pragma unroll
    for (int j = i + 1; j < 4; j++) s -= A[i][j] * xo[j];
    xo[i] = s / A[i][i];
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
    if (!isfinite(xo[i])) return 1;
  return 0;
}

// The same elimination split in two: LU with partial pivoting in place
// (multipliers stored below the diagonal in the row positions of their own
// step), then the solve; lu4 + lu_solve4 give solve4's result bit for bit,
// and the factors can be reused for further right-hand sides.
DEV int lu4(double A[4][4], int piv[4]) {
#pragma unroll
  for (int k = 0; k < 4; k++) {
    int p = k;
    double best = ::fabs(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < 4; i++)
      if (::fabs(A[i][k]) > best) { best = ::fabs(A[i][k]); p = i; }
    if (!(best > 0.0) || !isfinite(best)) return 1;
    piv[k] = p;
    // row swap with static indices only (a register-resident matrix)
#pragma unroll
    for (int i = k + 1; i < 4; i++) {
      if (i == p) {
#pragma unroll
        for (int j = k; j < 4; j++) { const double t = A[k][j]; A[k][j] = A[i][j]; A[i][j] = t; }
      }
    }
    const double inv = 1.0 / A[k][k];
#pragma unroll
    for (int i = k + 1; i < 4; i++) {
      const double f = A[i][k] * inv;
#pragma unroll
      for (int j = k + 1; j < 4; j++) A[i][j] -= f * A[k][j];
      A[i][k] = f;
    }
  }
  return 0;
}

DEV int lu_solve4(const double A[4][4], const int piv[4], double b[4], double xo[4]) {
#pragma unroll
  for (int k = 0; k < 4; k++) {
    if (piv[k] != k) {
#pragma unroll
      for (int p = k + 1; p < 4; p++)
        if (p == piv[k]) { const double t = b[k]; b[k] = b[p]; b[p] = t; }
    }
#pragma unroll
    for (int i = k + 1; i < 4; i++) b[i] -= A[i][k] * b[k];
  }
#pragma unroll
  for (int i = 3; i >= 0; i--) {
    double s = b[i];
#pragma unroll
    for (int j = i + 1; j < 4; j++) s -= A[i][j] * xo[j];
    xo[i] = s / A[i][i];
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
    if (!isfinite(xo[i])) return 1;
  return 0;
}

// Below this error the PMHD Newton step keeps the factorised Jacobian of the
// last full evaluation and evaluates the residual alone (chord step): near
// the root the Jacobian changes by O(e_T) between iterates.
#ifndef GRRMHD_CHORD_TOL
#define GRRMHD_CHORD_TOL 1e-4
#endif

DEV double rad_energy_lab(const Metric& m, const double R[4]) {
  return -R[0] + m.alpha * m.alpha * (m.up(0, 1) * R[1] + m.up(0, 2) * R[2] + m.up(0, 3) * R[3]);
}

struct Best {
  double x[4], P[12], eT;
  int radflags, ok;
};

DEV void keep(Best& b, const Eval& e) {
#pragma unroll
  for (int k = 0; k < 4; k++) b.x[k] = e.x[k];
#pragma unroll
  for (int q = 0; q < 12; q++) b.P[q] = e.P[q];
  b.eT = e.eT;
  b.radflags = e.radflags;
  b.ok = e.ok;
}

// One "normal" Newton attempt (D = 1) with one method.  A single Eval
// record is live: the new iterate is evaluated into it once the step is
// taken (PMHD needs only x; URAD keeps the five gas values that seed its
// inner inversion).
template <int METHOD, bool ENT = false>
DEV void newton(const Cell& c, const Phys& ph, const Opts& o, const double x0[4],
                const double Pg0[5], Best& best, int& iters) {
  static_assert(METHOD != M_PRAD || GRRMHD_URAD_EXACT, "PRAD uses exact Jacobians only");
  const double tol = (METHOD == M_PMHD) ? o.tol_pmhd : o.tol_urad;
  double x[4] = {x0[0], x0[1], x0[2], x0[3]};
  Eval ev;
  double J[4][4];
  int piv[4] = {0, 1, 2, 3};
  bool fresh = true;   // PMHD: J holds a new Jacobian, not yet factorised
  bool jok = true;      // URAD (exact): J holds the Jacobian at x
  if (METHOD == M_PMHD) eval_pmhd<ENT>(c, ph, x, ev, J);
  else if (METHOD == M_PRAD) eval_prad_jac<ENT>(c, ph, x, Pg0, ev, J);
  else if (GRRMHD_URAD_EXACT) eval_urad_jac<ENT>(c, ph, x, Pg0, ev, J);
  else eval_urad(c, ph, x, Pg0, ev);
  keep(best, ev);
  if (!ev.ok) return;
  double h[5];           // last five e_T, h[4] newest
#pragma unroll
  for (int k = 0; k < 4; k++) h[k] = INFINITY;
  h[4] = ev.eT;
  int nrise = 0, extra = 0, conv = 0, nfail = 0;
  for (int it = 0; it < o.max_iter; it++) {
    if (ev.eT < tol) conv = 1;
    if (conv) {
      if (!o.roundoff || extra >= 3) break;
      extra++;
    }
    if (!conv && it >= 5 && ev.eT > 0.5 * (h[0] + h[1] + h[2]) * (1.0 / 3.0)) break;
    double r[4];
    double Pn[5];
#pragma unroll
    for (int q = 0; q < 5; q++) Pn[q] = ev.P[q];
    if (METHOD != M_PMHD && GRRMHD_URAD_EXACT) {
      if (!jok) {                       // after a back-off: the Jacobian at x
        Eval ej;
        if (METHOD == M_PRAD) eval_prad_jac<ENT>(c, ph, x, Pn, ej, J);
        else eval_urad_jac<ENT>(c, ph, x, Pn, ej, J);
        if (!ej.ok) break;
        jok = true;
      }
#pragma unroll
      for (int i = 0; i < 4; i++) r[i] = ev.Er[i];
    } else if (METHOD == M_URAD) {
      const double delta = (ev.eIr < 1e-9) ? 1e-10 : 1e-8;
      int jfail = 0;
      // offsets relative to the iterated radiation, floored at 1e4 eps of
      // the radiation residual's scale; the energy offset raises the energy
      // (|R_t| + |R_t(i)| + dt |G_t|, with R_t = x_0 and dt G_t from the residual)
      const double Nres = ::fabs(x[0]) + ::fabs(c.Ri[0]) + ::fabs(ev.Er[0] - (x[0] - c.Ri[0]));
      for (int j = 0; j < 4 && !jfail; j++) {
        const double Nx = (j == 0) ? ::fabs(x[0]) : ::fabs(x[j]) + ::fabs(x[0]) / ::sqrt(gamup(c.m, j - 1, j - 1));
        const double N = fmax(Nx, 1e4 * DBL_EPSILON * Nres / delta);
        double hh = (j == 0) ? -delta * N : delta * N;
        int got = 0;
        for (int tries = 0; tries < 12 && !got; tries++) {
          double xp[4] = {x[0], x[1], x[2], x[3]};
          xp[j] += hh;
          Eval ep;
          eval_urad(c, ph, xp, Pn, ep);
          if (ep.ok) {
            const double ih = 1.0 / hh;
#pragma unroll
            for (int i = 0; i < 4; i++) J[i][j] = (ep.Er[i] - ev.Er[i]) * ih;
            got = 1;
          } else {
            hh = (tries % 2 == 0) ? -hh : -10.0 * hh;
            if (::fabs(hh) > 0.3 * N) break;
          }
        }
        if (!got) jfail = 1;
      }
      if (jfail) break;
#pragma unroll
      for (int i = 0; i < 4; i++) r[i] = ev.Er[i];
    } else {
#pragma unroll
      for (int i = 0; i < 4; i++) r[i] = ev.Eg[i];
    }
    if (ENT) r[0] = ev.Es;   // the entropy equation in the energy slot
    double dx[4];
    if (METHOD == M_PMHD) {
      if (fresh) {
        if (lu4(J, piv)) break;
        fresh = false;
      }
      if (lu_solve4(J, piv, r, dx)) break;
    } else {
      if (solve4(J, r, dx)) break;
    }
    double xn[4];
#pragma unroll
    for (int i = 0; i < 4; i++) xn[i] = x[i] - dx[i];
    if (METHOD == M_PMHD) {
      if (xn[0] < 0.0) xn[0] = 0.5 * ::fabs(xn[0]);            // one-sided bisection of u_g
      if (ev.eT < GRRMHD_CHORD_TOL) {
        eval_pmhd_value<ENT>(c, ph, xn, ev);
      } else {
        eval_pmhd<ENT>(c, ph, xn, ev, J);
        fresh = true;
      }
    } else {
      if (METHOD == M_PRAD) {
        if (xn[0] < 0.0) xn[0] = 0.5 * ::fabs(xn[0]);          // the same for Ebar
      } else {
        const double Erl = rad_energy_lab(c.m, xn);
        if (Erl <= 0.0) {                                     // same for the radiation energy
          const double a2 = c.m.alpha * c.m.alpha;
          xn[0] = -0.5 * ::fabs(Erl) + a2 * (c.m.up(0, 1) * xn[1] + c.m.up(0, 2) * xn[2] + c.m.up(0, 3) * xn[3]);
        }
      }
      if (METHOD == M_PRAD) {
        eval_prad_jac<ENT>(c, ph, xn, Pn, ev, J);
        jok = ev.ok;
      } else if (GRRMHD_URAD_EXACT) {
        eval_urad_jac<ENT>(c, ph, xn, Pn, ev, J);
        jok = ev.ok;
      } else {
        eval_urad(c, ph, xn, Pn, ev);
      }
      int back = 0;
      while (!ev.ok && back < 20) {                           // back up half-way
        nfail++;
        if (GRRMHD_URAD_EXACT && nfail > 3) break;            // ends below either way
#pragma unroll
        for (int i = 0; i < 4; i++) xn[i] = 0.5 * (x[i] + xn[i]);
        if (METHOD == M_PRAD) {
          eval_prad_jac<ENT>(c, ph, xn, Pn, ev, J);
          jok = ev.ok;
        } else if (GRRMHD_URAD_EXACT) {
          eval_urad_jac<ENT>(c, ph, xn, Pn, ev, J);
          jok = ev.ok;
        } else {
          eval_urad(c, ph, xn, Pn, ev);
        }
        back++;
      }
      if (!ev.ok || nfail > 3) {
        iters++;
        break;
      }
    }
    iters++;
    bool small = true;
#pragma unroll
    for (int i = 0; i < 4; i++)
      if (::fabs(xn[i] - x[i]) > 10.0 * DBL_EPSILON * ::fabs(x[i])) small = false;
#pragma unroll
    for (int i = 0; i < 4; i++) x[i] = xn[i];
    const double prev = h[4];
#pragma unroll
    for (int k = 0; k < 4; k++) h[k] = h[k + 1];
    h[4] = ev.eT;
    if (ev.eT < best.eT) keep(best, ev);
    if (it >= 5 && ev.eT > prev) {
      nrise++;
      if (nrise >= 5) break;
    }
    if (small) break;
  }
}

struct CellOut {
  double P[12], U[12];
  int status, iters;
  double err;
};

// Cell set-up shared by both kernels: explicit state, regime and guess.
struct Prep {
  double Pthin[5];
  int status;
  bool extreme;
};

// The cell's explicit state per sqrt(-g) and its coefficients.
DEV void cell_setup(const Metric& m, const double Ui[12], double dt, double chi_abs,
                    double chi_es, Cell& c) {
  c.m = m;
  const double igd = 1.0 / m.gdet;
  c.rhout = Ui[0] * igd;
#pragma unroll
  for (int i = 0; i < 3; i++) c.B[i] = Ui[5 + i] * igd;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    c.Tgi[k] = Ui[1 + k] * igd;
    c.Ri[k] = Ui[8 + k] * igd;
  }
  c.dt = dt;
  c.chi_abs = chi_abs;
  c.chi_es = chi_es;
  c.cold = 0;
  c.Si = NAN;
}

DEV void prepare(const Metric& m, const Phys& ph, const double Ui[12], const double Pg[12], double dt,
                 double chi_abs, double chi_es, Cell& c, Prep& pr) {
  cell_setup(m, Ui, dt, chi_abs, chi_es, c);
  pr.status = 0;
  // extreme radiation sub-dominance: R^t_t against the gas energy, or the
  // gas-frame radiation energy of the guess against u_g, below 10 eps
  double Ehat;
  {
    Vel<double> u, r;
    make_vel(m, Pg + 2, u);
    make_vel(m, Pg + 9, r);
    double w = 0.0;
#pragma unroll
    for (int a = 0; a < 4; a++) w += r.ucon[a] * u.ucov[a];
    Ehat = (4.0 / 3.0) * Pg[8] * w * w - Pg[8] * (1.0 / 3.0);
  }
  const double tenEps = 10.0 * DBL_EPSILON;
  pr.extreme = (::fabs(c.Ri[0]) <= tenEps * (::fabs(c.Tgi[0]) + ::fabs(c.Ri[0]))) ||
               (::fabs(Ehat) <= tenEps * (::fabs(Pg[1]) + ::fabs(Ehat)));
  if (pr.extreme) pr.status |= GRRMHD_ST_EXTREME;
  // PMHD guess: prior primitives, or the MHD inversion of U(i) when the
  // temporal optical depth dt kappa_tot(P_n) < 2/3
#pragma unroll
  for (int q = 0; q < 5; q++) pr.Pthin[q] = Pg[q];
  if (dt * (chi_abs + chi_es) * Pg[0] < 2.0 / 3.0) {
    double rho = Pg[0], ug = Pg[1], ut[3] = {Pg[2], Pg[3], Pg[4]};
    if (mhd_invert(m, ph.gam, c.rhout, c.Tgi[0], c.Tgi + 1, c.B, rho, ug, ut) == 0) {
      pr.Pthin[0] = rho; pr.Pthin[1] = ug; pr.Pthin[2] = ut[0]; pr.Pthin[3] = ut[1]; pr.Pthin[4] = ut[2];
    } else {
      pr.status |= GRRMHD_ST_C2P_FAIL;
    }
  }
}

// Acceptance without trying a further method (Sec. 4.10: e_T < tol_accept);
// when iterating to round-off, within 10x the PMHD tolerance.
DEV double accept_threshold(const Opts& o) { return o.roundoff ? 10.0 * o.tol_pmhd : o.tol_accept; }

// Conserved output and status from the best solution (Sec. 4.10-4.11).
DEV void finalize(const Cell& c, const Phys& ph, const Opts& o, const Best& best, int method,
                  int status, int iters, const double Ui[12], CellOut& out) {
  const Metric& m = c.m;
  out.iters = iters;
  status |= (method == M_PMHD) ? GRRMHD_ST_PMHD : (method == M_URAD) ? GRRMHD_ST_URAD : GRRMHD_ST_PRAD;
  if (best.eT > o.tol_fail) status |= GRRMHD_ST_FAIL;
  else if (best.eT > o.tol_accept) status |= GRRMHD_ST_NOT_ACCEPT;
  if (best.radflags & 1) status |= GRRMHD_ST_TYPE2_NEG;
#pragma unroll
  for (int q = 0; q < 12; q++) out.P[q] = best.P[q];
  double Ug[4], Ur[4];
  if (method == M_PMHD) {
    gas_cons4(m, ph.gam, best.P, Ug);
#pragma unroll
    for (int k = 0; k < 4; k++) Ur[k] = c.Ri[k] - (Ug[k] - c.Tgi[k]);
  } else if (method == M_PRAD) {
    rad_cons4(m, best.P, Ur);
#pragma unroll
    for (int k = 0; k < 4; k++) Ug[k] = c.Tgi[k] - (Ur[k] - c.Ri[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      Ur[k] = best.x[k];
      Ug[k] = c.Tgi[k] - (best.x[k] - c.Ri[k]);
    }
  }
  bool radchg = best.radflags != 0;
  if (method == M_PMHD && (best.radflags & 1)) {
    double Eb, utr[3];
    rad_invert(m, ph.gamma_max, ph.ymax, 0, Ur, Eb, utr);
    out.P[8] = Eb;
    out.P[9] = utr[0]; out.P[10] = utr[1]; out.P[11] = utr[2];
    status |= GRRMHD_ST_BASIC;
    radchg = true;
  }
  if (radchg) rad_cons4(m, out.P, Ur);
  const double gd = m.gdet;
  out.U[0] = Ui[0];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    out.U[1 + k] = gd * Ug[k];
    out.U[8 + k] = gd * Ur[k];
  }
#pragma unroll
  for (int i = 0; i < 3; i++) out.U[5 + i] = Ui[5 + i];
  if (!(out.P[1] > 0.0)) status |= GRRMHD_ST_FAIL;
  out.status = status;
  out.err = best.eT;
}

DEV void failed_out(const double Ui[12], const double Pg[12], int status, int iters, CellOut& out) {
#pragma unroll
  for (int q = 0; q < 12; q++) {
    out.P[q] = Pg[q];
    out.U[q] = Ui[q];
  }
  out.iters = iters;
  out.status = status | GRRMHD_ST_FAIL;
  out.err = INFINITY;
}

// Cold MHD limit (Sec. 4.7: with no solution of the energy or the entropy
// equation, both conservation laws are dropped): u_g held at x0[0], the
// three gas momentum equations solved for u~^i with the PMHD residual and
// its exact Jacobian, the radiation following from total conservation; the
// energy residuals leave e_T (c.cold).  The u_g row and column of the 4x4
// system are pinned (dx_0 = 0); the stopping rules are newton()'s.
DEV void newton_cold(const Cell& c, const Phys& ph, const Opts& o, const double x0[4], Best& best,
                     int& iters) {
  double x[4] = {x0[0], x0[1], x0[2], x0[3]};
  Eval ev;
  double J[4][4];
  eval_pmhd(c, ph, x, ev, J);
  keep(best, ev);
  if (!ev.ok) return;
  double h[5];
#pragma unroll
  for (int k = 0; k < 4; k++) h[k] = INFINITY;
  h[4] = ev.eT;
  int nrise = 0, extra = 0, conv = 0;
  for (int it = 0; it < o.max_iter; it++) {
    if (ev.eT < o.tol_pmhd) conv = 1;
    if (conv) {
      if (!o.roundoff || extra >= 3) break;
      extra++;
    }
    if (!conv && it >= 5 && ev.eT > 0.5 * (h[0] + h[1] + h[2]) * (1.0 / 3.0)) break;
    J[0][0] = 1.0;
#pragma unroll
    for (int k = 1; k < 4; k++) J[0][k] = J[k][0] = 0.0;
    double r[4] = {0.0, ev.Eg[1], ev.Eg[2], ev.Eg[3]};
    double dx[4];
    if (solve4(J, r, dx)) break;
    double xn[4];
#pragma unroll
    for (int i = 0; i < 4; i++) xn[i] = x[i] - dx[i];
    eval_pmhd(c, ph, xn, ev, J);
    iters++;
    bool small = true;
#pragma unroll
    for (int i = 0; i < 4; i++)
      if (::fabs(xn[i] - x[i]) > 10.0 * DBL_EPSILON * ::fabs(x[i])) small = false;
#pragma unroll
    for (int i = 0; i < 4; i++) x[i] = xn[i];
    const double prev = h[4];
#pragma unroll
    for (int k = 0; k < 4; k++) h[k] = h[k + 1];
    h[4] = ev.eT;
    if (ev.ok && ev.eT < best.eT) keep(best, ev);
    if (!ev.ok) break;
    if (it >= 5 && ev.eT > prev) {
      nrise++;
      if (nrise >= 5) break;
    }
    if (small) break;
  }
}

// Conditions of the cold attempt (Sec. 4.11, backups), on the prior
// primitives and the explicit gas state t^t_mu (T^t_mu with rho0 u^t in the
// energy slot): u_g < 0.1 rho0 u^i u_i and |t^t_t t^{tt}| < 0.1 |t^t_i t^{ti}|
// (the gas cold against its motion, its energy small against its momentum).
// The paper's condition on R^t_t R^{tt} against R^t_i R^{ti} cannot hold for
// an M1 state (|F| <= E) and is not applied.
DEV bool cold_allowed(const Cell& c, const double Pg[12]) {
  Vel<double> u;
  make_vel(c.m, Pg + 2, u);
  const double usp = u.ucon[1] * u.ucov[1] + u.ucon[2] * u.ucov[2] + u.ucon[3] * u.ucov[3];
  if (!(Pg[1] < 0.1 * Pg[0] * ::fabs(usp))) return false;
  double en = 0.0, mo = 0.0;
#pragma unroll
  for (int a = 0; a < 4; a++) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < 4; b++) t += c.m.up(a, b) * c.Tgi[b];
    if (a == 0) en = c.Tgi[0] * t;
    else mo += c.Tgi[a] * t;
  }
  return ::fabs(en) < 0.1 * ::fabs(mo);
}

// Cold attempt for a cell with no energy solution that meets the
// conditions above: u_g at the floor, u~^i from the prior primitives.  On
// success (e_T within tol_fail) `out` holds
// the solution with the set-up's status bits (EXTREME, C2P_FAIL) and COLD
// (TYPE2/BASIC/NOT_ACCEPT as for PMHD); iters accumulates either way.
DEV bool cold_cell(const Metric& m, const Phys& ph, const Opts& o, const double Ui[12],
                   const double Pg[12], double dt, double chi_abs, double chi_es, int& iters,
                   CellOut& out) {
  Cell c;
  cell_setup(m, Ui, dt, chi_abs, chi_es, c);
  if (!cold_allowed(c, Pg)) return false;
  Prep pr;   // the set-up's status bits (EXTREME, C2P_FAIL) for the output
  prepare(m, ph, Ui, Pg, dt, chi_abs, chi_es, c, pr);
  c.cold = 1;
  const double x0[4] = {o.u_floor, Pg[2], Pg[3], Pg[4]};
  Best b;
  b.eT = INFINITY;
  b.ok = 0;
  newton_cold(c, ph, o, x0, b, iters);
  if (!b.ok || !(b.eT <= o.tol_fail)) return false;
  finalize(c, ph, o, b, M_PMHD, pr.status, iters, Ui, out);
  out.status = (out.status & ~GRRMHD_ST_PMHD) | GRRMHD_ST_COLD;
  return true;
}

// After the energy cascade: a cell left failed takes the cold limit.
DEV void cold_fallback(const Metric& m, const Phys& ph, const Opts& o, const double Ui[12],
                       const double Pg[12], double dt, double chi_abs, double chi_es,
                       CellOut& out) {
  if (!(out.status & GRRMHD_ST_FAIL) || !o.cold || !(o.u_floor > 0.0)) return;
  int iters = out.iters;
  CellOut oc;
  if (cold_cell(m, ph, o, Ui, Pg, dt, chi_abs, chi_es, iters, oc)) out = oc;
  out.iters = iters;
}

// Result of a cell's first PMHD attempt, kept per cascade-list slot so that
// the cascade resumes where the first attempt ended: field-major [f][cap],
// d = P[12], e_T; i = radiation flags, ok, iterations.
struct RecBuf {
  double* d;
  int* i;
  long cap;
};

DEV void rec_store(const RecBuf& R, long slot, const Best& b, int iters) {
#pragma unroll
  for (int q = 0; q < 12; q++) R.d[q * R.cap + slot] = b.P[q];
  R.d[12 * R.cap + slot] = b.eT;
  R.i[slot] = b.radflags;
  R.i[R.cap + slot] = b.ok;
  R.i[2 * R.cap + slot] = iters;
}

DEV void rec_load(const RecBuf& R, long slot, Best& b, int& iters) {
#pragma unroll
  for (int k = 0; k < 4; k++) b.x[k] = 0.0;
#pragma unroll
  for (int q = 0; q < 12; q++) b.P[q] = R.d[q * R.cap + slot];
  b.eT = R.d[12 * R.cap + slot];
  b.radflags = R.i[slot];
  b.ok = R.i[R.cap + slot];
  iters = R.i[2 * R.cap + slot];
}

// Common case: not extreme, first PMHD attempt accepted.  Returns false when
// the cell needs the full cascade; b and iters then hold the first attempt
// (none when the cell is extreme), trips the residual evaluations it took.
DEV bool implicit_fast(const Metric& m, const Phys& ph, const Opts& o, const double Ui[12],
                       const double Pg[12], double dt, double chi_abs, double chi_es,
                       CellOut& out, Best& b, int& iters, bool& extreme, int& trips) {
  Cell c;
  Prep pr;
  prepare(m, ph, Ui, Pg, dt, chi_abs, chi_es, c, pr);
  b.eT = INFINITY;
  b.ok = 0;
  iters = 0;
  trips = 0;
  extreme = pr.extreme;
  if (pr.extreme) return false;
  const double x0[4] = {pr.Pthin[1], pr.Pthin[2], pr.Pthin[3], pr.Pthin[4]};
  newton<M_PMHD>(c, ph, o, x0, pr.Pthin, b, iters);
  trips = iters + 1;
  if (!(b.ok && b.eT < accept_threshold(o))) return false;
  finalize(c, ph, o, b, M_PMHD, pr.status, iters, Ui, out);
  return true;
}

// Full cascade for one cell (Sec. 4.10-4.11).  With R, a non-extreme cell
// resumes after its first PMHD attempt, stored at list slot `slot` by the
// kernel that ran it (that attempt was not accepted, else the cell would not
// be in the cascade).
DEV void implicit_cell(const Metric& m, const Phys& ph, const Opts& o, const double Ui[12],
                       const double Pg[12], double dt, double chi_abs, double chi_es,
                       CellOut& out, const RecBuf* R = nullptr, long slot = 0,
                       bool try_cold = true) {
  Cell c;
  Prep pr;
  prepare(m, ph, Ui, Pg, dt, chi_abs, chi_es, c, pr);
  Best best;
  best.eT = INFINITY;
  best.ok = 0;
  int bm = -1, iters = 0, k0 = 0;
  if (R && !pr.extreme) {
    Best b;
    rec_load(*R, slot, b, iters);
    if (b.ok && b.eT < best.eT) {
      best = b;
      bm = M_PMHD;
    }
    k0 = 1;
  }
  for (int k = k0; k < 2; k++) {
    const int method = (k == 0) == pr.extreme ? M_URAD : M_PMHD;
    double x0[4], P0[5];
    const bool prev = (bm >= 0 && best.eT < 1e-4);
    Best b;
    b.eT = INFINITY;
    b.ok = 0;
    if (method == M_PMHD) {
      const double* src = prev ? best.P : pr.Pthin;
      x0[0] = src[1]; x0[1] = src[2]; x0[2] = src[3]; x0[3] = src[4];
#pragma unroll
      for (int q = 0; q < 5; q++) P0[q] = src[q];
      newton<M_PMHD>(c, ph, o, x0, P0, b, iters);
    } else {
      if (prev) {
        rad_cons4(m, best.P, x0);
#pragma unroll
        for (int q = 0; q < 5; q++) P0[q] = best.P[q];
      } else {
        rad_cons4(m, Pg, x0);
#pragma unroll
        for (int q = 0; q < 5; q++) P0[q] = Pg[q];
      }
      newton<M_URAD>(c, ph, o, x0, P0, b, iters);
    }
    if (b.ok && b.eT < best.eT) {
      best = b;
      bm = method;
    }
    if (best.eT < accept_threshold(o)) break;
  }
  if (bm < 0) failed_out(Ui, Pg, pr.status, iters, out);
  else finalize(c, ph, o, best, bm, pr.status, iters, Ui, out);
  if (try_cold) cold_fallback(m, ph, o, Ui, Pg, dt, chi_abs, chi_es, out);
}

// ---------------------------------------------------------------------------
// The paper's full cascade (params.cascade = 1; Sec. 4.10-4.11): PMHD, URAD
// and PRAD, their staged forms for cells still without an acceptable
// solution, the same with the entropy equation in place of the gas energy
// equation, then the cold limit.  Exact dual-number Jacobians throughout.
// ---------------------------------------------------------------------------

// residual and exact Jacobian of one method at x (Pn starts the inner MHD
// inversion of URAD and PRAD)
template <int METHOD, bool ENT>
DEV void eval_jac(const Cell& c, const Phys& ph, const double x[4], const double Pn[5], Eval& e,
                  double J[4][4]) {
  if (METHOD == M_PMHD) eval_pmhd<ENT>(c, ph, x, e, J);
  else if (METHOD == M_PRAD) eval_prad_jac<ENT>(c, ph, x, Pn, e, J);
  else eval_urad_jac<ENT>(c, ph, x, Pn, e, J);
}

template <int METHOD, bool ENT>
DEV void method_res(const Eval& e, double r[4]) {
  const double* E = (METHOD == M_PMHD) ? e.Eg : e.Er;
#pragma unroll
  for (int k = 0; k < 4; k++) r[k] = E[k];
  if (ENT) r[0] = e.Es;
}

// post-step check (Sec. 4.10): a negative u_g (PMHD), lab radiation energy
// (URAD) or Ebar (PRAD) becomes half its magnitude; true when it acted
template <int METHOD>
DEV bool post_step(const Cell& c, double xn[4]) {
  if (METHOD != M_URAD) {
    if (xn[0] < 0.0) {
      xn[0] = 0.5 * ::fabs(xn[0]);
      return true;
    }
    return false;
  }
  const double Erl = rad_energy_lab(c.m, xn);
  if (Erl <= 0.0) {
    const double a2 = c.m.alpha * c.m.alpha;
    xn[0] = -0.5 * ::fabs(Erl) + a2 * (c.m.up(0, 1) * xn[1] + c.m.up(0, 2) * xn[2] + c.m.up(0, 3) * xn[3]);
    return true;
  }
  return false;
}

// The staged attempt (Sec. 4.10): stage 1 one momentum-only step (x_0
// held) damped by 1/2; stage 2 energy-only (entropy-only) steps on x_0, the
// first damped by 1/2, until that equation's own error is below the
// method's tolerance, the step is at round-off or max_iter steps; a
// post-step correction recurring 2 times (4 with the entropy equation)
// holds the prior value and ends the stage; stage 3 the 4-D Newton for at
// most 40 steps, the first damped by 1/4, with newton()'s stopping rules.
template <int METHOD, bool ENT>
DEV void newton_staged(const Cell& c, const Phys& ph, const Opts& o, const double x0[4],
                       const double Pg0[5], Best& best, int& iters) {
  const double tol = (METHOD == M_PMHD) ? o.tol_pmhd : o.tol_urad;
  const int nmod_max = ENT ? 4 : 2;
  double x[4] = {x0[0], x0[1], x0[2], x0[3]};
  double Pn[5] = {Pg0[0], Pg0[1], Pg0[2], Pg0[3], Pg0[4]};
  Eval ev;
  double J[4][4];
  eval_jac<METHOD, ENT>(c, ph, x, Pn, ev, J);
  keep(best, ev);
  if (!ev.ok) return;
  for (int stage = 1; stage <= 2; stage++) {
    const int nmax = (stage == 1) ? 1 : o.max_iter;
    int nmod = 0;
    for (int it = 0; it < nmax; it++) {
      if (stage == 2 && ((METHOD == M_PMHD) ? ev.e0g : ev.e0r) < tol) break;
      double r[4], xn[4] = {x[0], x[1], x[2], x[3]};
      method_res<METHOD, ENT>(ev, r);
      const double D = (it == 0) ? 0.5 : 1.0;
      if (stage == 1) {
        double A[4][4], dx[4];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++) A[i][j] = (i == 0 || j == 0) ? (i == j ? 1.0 : 0.0) : J[i][j];
        double rm[4] = {0.0, r[1], r[2], r[3]};
        if (solve4(A, rm, dx)) break;
#pragma unroll
        for (int i = 1; i < 4; i++) xn[i] = x[i] - D * dx[i];
      } else {
        if (!(::fabs(J[0][0]) > 0.0) || !isfinite(J[0][0])) break;
        xn[0] = x[0] - D * r[0] / J[0][0];
      }
      if (post_step<METHOD>(c, xn)) {
        if (++nmod >= nmod_max) break;
      }
#pragma unroll
      for (int q = 0; q < 5; q++) Pn[q] = ev.P[q];
      Eval en;
      eval_jac<METHOD, ENT>(c, ph, xn, Pn, en, J);
      iters++;
      if (!en.ok) {
        eval_jac<METHOD, ENT>(c, ph, x, Pn, ev, J);   // the Jacobian at the held x
        break;
      }
      bool small = true;
#pragma unroll
      for (int i = 0; i < 4; i++)
        if (::fabs(xn[i] - x[i]) > 10.0 * DBL_EPSILON * ::fabs(x[i])) small = false;
#pragma unroll
      for (int i = 0; i < 4; i++) x[i] = xn[i];
      ev = en;
      if (ev.eT < best.eT) keep(best, ev);
      if (small) break;
    }
  }
  double h[5];
#pragma unroll
  for (int k = 0; k < 4; k++) h[k] = INFINITY;
  h[4] = ev.eT;
  int nrise = 0, extra = 0, conv = 0, nfail = 0;
  for (int it = 0; it < 40; it++) {
    if (ev.eT < tol) conv = 1;
    if (conv) {
      if (!o.roundoff || extra >= 3) break;
      extra++;
    }
    if (!conv && it >= 5 && ev.eT > 0.5 * (h[0] + h[1] + h[2]) * (1.0 / 3.0)) break;
    double r[4], dx[4];
    method_res<METHOD, ENT>(ev, r);
    if (solve4(J, r, dx)) break;
    const double D = (it == 0) ? 0.25 : 1.0;
    double xn[4];
#pragma unroll
    for (int i = 0; i < 4; i++) xn[i] = x[i] - D * dx[i];
    post_step<METHOD>(c, xn);
#pragma unroll
    for (int q = 0; q < 5; q++) Pn[q] = ev.P[q];
    Eval en;
    double Jn[4][4];
    eval_jac<METHOD, ENT>(c, ph, xn, Pn, en, Jn);
    if (METHOD != M_PMHD) {
      int back = 0;
      while (!en.ok && back < 20) {
        nfail++;
        if (nfail > 3) break;
#pragma unroll
        for (int i = 0; i < 4; i++) xn[i] = 0.5 * (x[i] + xn[i]);
        eval_jac<METHOD, ENT>(c, ph, xn, Pn, en, Jn);
        back++;
      }
      if (!en.ok || nfail > 3) {
        iters++;
        break;
      }
    }
    iters++;
    if (!en.ok) break;
    bool small = true;
#pragma unroll
    for (int i = 0; i < 4; i++)
      if (::fabs(xn[i] - x[i]) > 10.0 * DBL_EPSILON * ::fabs(x[i])) small = false;
#pragma unroll
    for (int i = 0; i < 4; i++) x[i] = xn[i];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = 0; j < 4; j++) J[i][j] = Jn[i][j];
    const double prev = h[4];
#pragma unroll
    for (int k = 0; k < 4; k++) h[k] = h[k + 1];
    h[4] = en.eT;
    ev = en;
    if (ev.eT < best.eT) keep(best, ev);
    if (it >= 5 && ev.eT > prev) {
      nrise++;
      if (nrise >= 5) break;
    }
    if (small) break;
  }
}

// One attempt of one method, normal or staged (run-time choice over the
// compile-time forms).
template <bool ENT>
DEV void attempt(int method, bool staged, const Cell& c, const Phys& ph, const Opts& o,
                 const double x0[4], const double P0[5], Best& b, int& iters) {
  if (staged) {
    if (method == M_PMHD) newton_staged<M_PMHD, ENT>(c, ph, o, x0, P0, b, iters);
    else if (method == M_URAD) newton_staged<M_URAD, ENT>(c, ph, o, x0, P0, b, iters);
    else newton_staged<M_PRAD, ENT>(c, ph, o, x0, P0, b, iters);
  } else {
    if (method == M_PMHD) newton<M_PMHD, ENT>(c, ph, o, x0, P0, b, iters);
    else if (method == M_URAD) newton<M_URAD, ENT>(c, ph, o, x0, P0, b, iters);
    else newton<M_PRAD, ENT>(c, ph, o, x0, P0, b, iters);
  }
}

// One phase (energy or, with ENT, entropy equation): the normal attempts
// (PMHD, URAD, PRAD; URAD and PRAD first in the extreme regime) until one
// is acceptable, then the staged attempts of PMHD, URAD and PRAD.  The
// first `skip` normal attempts already ran (their best is in best/bm).  Each
// attempt starts from the best so far when its e_T < 1e-4, else from its
// own guess: PMHD the thin-limit primitives (staged: u_g from the explicit
// entropy at the prior rho0), URAD R(P_n), PRAD the thin-limit radiation.
template <bool ENT>
DEV void run_phase(const Cell& c, const Phys& ph, const Opts& o, const Prep& pr,
                   const double Pg[12], const double Pradthin[12], int skip, Best& best, int& bm,
                   int& staged, int& iters) {
  const double acc = accept_threshold(o);
  for (int k = skip; k < 6; k++) {
    if (best.eT < acc) return;
    const bool stg = k >= 3;
    const int kk = k % 3;
    const int method = stg ? kk : (pr.extreme ? (kk == 0 ? M_URAD : (kk == 1 ? M_PRAD : M_PMHD)) : kk);
    const bool prev = (bm >= 0 && best.eT < 1e-4);
    double x0[4], P0[5];
    if (method == M_PMHD) {
      const double* src = prev ? best.P : pr.Pthin;
      x0[0] = src[1]; x0[1] = src[2]; x0[2] = src[3]; x0[3] = src[4];
#pragma unroll
      for (int q = 0; q < 5; q++) P0[q] = src[q];
      if (stg && !prev && isfinite(c.Si) && c.rhout > 0.0) {
        // u_g from the specific entropy Si/(rho0 u^t) at the prior rho0
        const double n = 1.0 / (ph.gam - 1.0), rho = pr.Pthin[0];
        const double pg = ::exp((c.Si / c.rhout + (n + 1.0) * ::log(rho)) / n);
        if (isfinite(pg) && pg > 0.0) x0[0] = pg / (ph.gam - 1.0);
      }
    } else if (method == M_URAD) {
      const double* src = prev ? best.P : Pg;
      rad_cons4(c.m, src, x0);
#pragma unroll
      for (int q = 0; q < 5; q++) P0[q] = src[q];
    } else {
      const double* src = prev ? best.P : Pradthin;
      x0[0] = src[8]; x0[1] = src[9]; x0[2] = src[10]; x0[3] = src[11];
#pragma unroll
      for (int q = 0; q < 5; q++) P0[q] = src[q];
    }
    Best b;
    b.eT = INFINITY;
    b.ok = 0;
    attempt<ENT>(method, stg, c, ph, o, x0, P0, b, iters);
    if (b.ok && b.eT < best.eT) {
      best = b;
      bm = method;
      staged = stg;
    }
  }
}

// Full cascade for one cell.  Si: the explicit entropy sqrt(-g) [S u^t]_(i)
// (NAN: no entropy phase).  resume 1: the first PMHD attempt ran (record R
// at `slot`), 2: PMHD and URAD ran (the record holds the better of the two,
// its method in the record's ok field); 0 from scratch.
DEV void implicit_cell_full(const Metric& m, const Phys& ph, const Opts& o, const double Ui[12],
                            double Si, const double Pg[12], double dt, double chi_abs,
                            double chi_es, CellOut& out, const RecBuf* R = nullptr,
                            long slot = 0, int resume = 0) {
  Cell c;
  Prep pr;
  prepare(m, ph, Ui, Pg, dt, chi_abs, chi_es, c, pr);
  c.Si = Si / m.gdet;
  const double acc = accept_threshold(o);
  double Pradthin[12];
#pragma unroll
  for (int q = 0; q < 12; q++) Pradthin[q] = Pg[q];
  if (dt * (chi_abs + chi_es) * Pg[0] < 2.0 / 3.0) {
    double Eb, utr[3];
    rad_invert(m, ph.gamma_max, ph.ymax, 0, c.Ri, Eb, utr);
    if (Eb > 0.0 && isfinite(Eb)) {
      Pradthin[8] = Eb; Pradthin[9] = utr[0]; Pradthin[10] = utr[1]; Pradthin[11] = utr[2];
    }
  }
  Best bE;
  bE.eT = INFINITY;
  bE.ok = 0;
  int mE = -1, sE = 0, iters = 0, skip = 0;
  if (R && resume && !pr.extreme) {
    Best b;
    rec_load(*R, slot, b, iters);
    const int meth = b.ok >> 1;
    b.ok &= 1;
    if (b.ok) {
      bE = b;
      mE = meth;
    }
    skip = resume;
  }
  run_phase<false>(c, ph, o, pr, Pg, Pradthin, skip, bE, mE, sE, iters);
  const bool eok = mE >= 0 && bE.P[1] > 0.0;
  int use = -1;
  Best bS;
  int mS = -1, sS = 0;
  if (eok && bE.eT < acc) {
    use = 0;
  } else {
    bS.eT = INFINITY;
    bS.ok = 0;
    if (isfinite(c.Si)) run_phase<true>(c, ph, o, pr, Pg, Pradthin, 0, bS, mS, sS, iters);
    const bool sok = mS >= 0 && bS.P[1] > 0.0;
    if (sok && bS.eT < acc) use = 1;
    else {
      const bool e2 = eok && bE.eT <= o.tol_fail, s2 = sok && bS.eT <= o.tol_fail;
      if (e2 && s2) use = (bS.eT < bE.eT) ? 1 : 0;
      else if (e2) use = 0;
      else if (s2) use = 1;
    }
  }
  if (use == 1) {
    finalize(c, ph, o, bS, mS, pr.status, iters, Ui, out);
    out.status |= GRRMHD_ST_ENTROPY | (sS ? GRRMHD_ST_STAGED : 0);
  } else if (mE >= 0) {
    finalize(c, ph, o, bE, mE, pr.status, iters, Ui, out);
    if (use == 0 && sE) out.status |= GRRMHD_ST_STAGED;
    if (use < 0) out.status |= GRRMHD_ST_FAIL;
  } else {
    failed_out(Ui, Pg, pr.status, iters, out);
  }
  cold_fallback(m, ph, o, Ui, Pg, dt, chi_abs, chi_es, out);
}

// ---------------------------------------------------------------------------
// Resumable PMHD attempt for the persistent and per-iteration kernels.
//
// The first PMHD attempt of the fast path as a state machine: every trip
// evaluates the residual once, either at a new cell's guess or at the next
// Newton iterate, so lanes that start a cell and lanes that continue one run
// the same expensive code.  The decisions are exactly those of newton<PMHD>,
// so results equal those of k_implicit bit for bit.
// ---------------------------------------------------------------------------
struct Lane {
  double x[4];
  double Eg[4], eT;        // residual and error of the current iterate
  double J[4][4];          // Jacobian, or its LU factors once factorised
  Best best;
  double h[5];
  int it, nrise, extra, conv, iters, status;
  int piv[4], fresh, chord;  // pivots; J not yet factorised; next evaluation is a chord step
};

enum { TRIP_CONTINUE = 0, TRIP_DONE = 1, TRIP_CASCADE = 2 };

// Part A of a Newton trip: loop-top checks and the step.  Returns true when
// the attempt ends here.
DEV bool lane_step(const Cell& c, const Opts& o, Lane& L) {
  if (L.it >= o.max_iter) return true;
  if (L.eT < o.tol_pmhd) L.conv = 1;
  if (L.conv) {
    if (!o.roundoff || L.extra >= 3) return true;
    L.extra++;
  }
  if (!L.conv && L.it >= 5 && L.eT > 0.5 * (L.h[0] + L.h[1] + L.h[2]) * (1.0 / 3.0)) return true;
  double r[4] = {L.Eg[0], L.Eg[1], L.Eg[2], L.Eg[3]}, dx[4];
  if (L.fresh) {
    if (lu4(L.J, L.piv)) return true;
    L.fresh = 0;
  }
  if (lu_solve4(L.J, L.piv, r, dx)) return true;
#pragma unroll
  for (int i = 0; i < 4; i++) L.x[i] -= dx[i];
  if (L.x[0] < 0.0) L.x[0] = 0.5 * ::fabs(L.x[0]);
  L.chord = L.eT < GRRMHD_CHORD_TOL;
  return false;
}

// The evaluation at the lane's new iterate: residual alone on a chord step,
// else residual and Jacobian.
DEV void lane_eval(const Cell& c, const Phys& ph, Lane& L, Eval& ev) {
  if (L.chord) {
    eval_pmhd_value(c, ph, L.x, ev);
  } else {
    eval_pmhd(c, ph, L.x, ev, L.J);
    L.fresh = 1;
  }
}

// Part B after evaluating at the new iterate (xprev: the previous iterate).
// Returns true when the attempt ends here.
DEV bool lane_after(const Eval& ev, const double xprev[4], Lane& L) {
  L.iters++;
  bool small = true;
#pragma unroll
  for (int i = 0; i < 4; i++)
    if (::fabs(L.x[i] - xprev[i]) > 10.0 * DBL_EPSILON * ::fabs(xprev[i])) small = false;
  const double prev = L.h[4];
#pragma unroll
  for (int k = 0; k < 4; k++) L.h[k] = L.h[k + 1];
  L.h[4] = ev.eT;
  if (ev.eT < L.best.eT) keep(L.best, ev);
  bool done = false;
  if (L.it >= 5 && ev.eT > prev) {
    L.nrise++;
    if (L.nrise >= 5) done = true;
  }
  if (small) done = true;
  L.it++;
  return done;
}

DEV void lane_take(const Eval& ev, Lane& L) {
#pragma unroll
  for (int k = 0; k < 4; k++) L.Eg[k] = ev.Eg[k];
  L.eT = ev.eT;
}

DEV void lane_start(const Eval& ev, Lane& L) {
  L.fresh = 1;
  L.chord = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) L.piv[k] = k;
  keep(L.best, ev);
#pragma unroll
  for (int k = 0; k < 4; k++) L.h[k] = INFINITY;
  L.h[4] = ev.eT;
  L.it = L.nrise = L.extra = L.conv = L.iters = 0;
  lane_take(ev, L);
}

// ---------------------------------------------------------------------------
// The URAD attempt (exact Jacobians) as a lane state machine with one
// residual evaluation per trip, so that lanes of a wavefront can hold cells
// at different stages: START evaluates the guess, STEP takes the Newton step
// from x and evaluates the new point, BACK evaluates half-way back towards x
// after a failed evaluation.  The evaluation points, guesses and decisions
// are those of newton<M_URAD>.
// ---------------------------------------------------------------------------
enum { UM_START = 0, UM_STEP = 1, UM_BACK = 2 };

struct UradLane {
  double x[4], p[4];     // iterate; point of this trip's evaluation
  double Er[4], eT;      // residual and error at x
  double J[4][4];        // Jacobian at x (the solve overwrites it)
  double Pn[5];          // gas primitives at x: guess of the inner MHD inversion
  double h[5];
  Best best;
  int it, nrise, extra, conv, nfail, iters, mode;
};

// Before the evaluation: STEP's loop-top checks and step (true: the attempt
// ends here), BACK's half-way point.
DEV bool urad_before(const Cell& c, const Opts& o, UradLane& L) {
  if (L.mode == UM_BACK) {
#pragma unroll
    for (int i = 0; i < 4; i++) L.p[i] = 0.5 * (L.x[i] + L.p[i]);
    return false;
  }
  if (L.mode != UM_STEP) return false;
  if (L.it >= o.max_iter) return true;
  if (L.eT < o.tol_urad) L.conv = 1;
  if (L.conv) {
    if (!o.roundoff || L.extra >= 3) return true;
    L.extra++;
  }
  if (!L.conv && L.it >= 5 && L.eT > 0.5 * (L.h[0] + L.h[1] + L.h[2]) * (1.0 / 3.0)) return true;
  double r[4] = {L.Er[0], L.Er[1], L.Er[2], L.Er[3]}, dx[4];
  if (solve4(L.J, r, dx)) return true;
#pragma unroll
  for (int i = 0; i < 4; i++) L.p[i] = L.x[i] - dx[i];
  const double Erl = rad_energy_lab(c.m, L.p);
  if (Erl <= 0.0) {
    const double a2 = c.m.alpha * c.m.alpha;
    L.p[0] = -0.5 * ::fabs(Erl) + a2 * (c.m.up(0, 1) * L.p[1] + c.m.up(0, 2) * L.p[2] + c.m.up(0, 3) * L.p[3]);
  }
  return false;
}

DEV void urad_take(const Eval& ev, const double Jn[4][4], UradLane& L) {
#pragma unroll
  for (int i = 0; i < 4; i++) {
    L.x[i] = L.p[i];
    L.Er[i] = ev.Er[i];
#pragma unroll
    for (int j = 0; j < 4; j++) L.J[i][j] = Jn[i][j];
  }
#pragma unroll
  for (int q = 0; q < 5; q++) L.Pn[q] = ev.P[q];
  L.eT = ev.eT;
}

// After the evaluation at L.p (true: the attempt ends here).
DEV bool urad_after(const Eval& ev, const double Jn[4][4], UradLane& L) {
  if (L.mode == UM_START) {
    keep(L.best, ev);
    if (!ev.ok) return true;
    urad_take(ev, Jn, L);
#pragma unroll
    for (int k = 0; k < 4; k++) L.h[k] = INFINITY;
    L.h[4] = ev.eT;
    L.it = L.nrise = L.extra = L.conv = L.nfail = 0;
    L.mode = UM_STEP;
    return false;
  }
  if (!ev.ok) {
    L.nfail++;
    if (L.nfail > 3) {
      L.iters++;
      return true;
    }
    L.mode = UM_BACK;
    return false;
  }
  L.iters++;
  bool small = true;
#pragma unroll
  for (int i = 0; i < 4; i++)
    if (::fabs(L.p[i] - L.x[i]) > 10.0 * DBL_EPSILON * ::fabs(L.x[i])) small = false;
  urad_take(ev, Jn, L);
  const double prev = L.h[4];
#pragma unroll
  for (int k = 0; k < 4; k++) L.h[k] = L.h[k + 1];
  L.h[4] = ev.eT;
  if (ev.eT < L.best.eT) keep(L.best, ev);
  bool done = false;
  if (L.it >= 5 && ev.eT > prev) {
    L.nrise++;
    if (L.nrise >= 5) done = true;
  }
  if (small) done = true;
  L.it++;
  L.mode = UM_STEP;
  return done;
}
