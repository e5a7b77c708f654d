// Adjoint of one RK3-IMEX step: the vector-Jacobian product dL/dP^n of
// L = sum(gU . U^{n+1}(P^n)) with dt held fixed and U^n = U(P^n).
//
// The forward step is recomputed with every stage's inputs and outputs kept
// (checkpoints); the reverse sweep then runs, per stage, from last to first:
//   implicit solve   implicit-function theorem on the PMHD residual at the
//                    converged state: J_x^T mu = (dOut/dx)^T lambda, then
//                    lambda_Ue = (dOut/dUe)^T lambda - (dE/dUe)^T mu
//                    (one transposed 4x4 solve per cell, no unrolled Newton);
//   stage update     U(k) = a U^n + b U(k-1) + c dt (S(P) - div F): linear
//                    parts exact, the geometric source S by its local
//                    Jacobian;
//   fluxes           corner EMFs (linear), then per face the Jacobian of the
//                    Riemann flux with respect to its stencil cells (four
//                    for MC, six for PPM) and, for PPM, to the flattener of
//                    its two cells (face states, HLL / LAXF);
//   PPM flattener    the flattener a stage read is the largest over the
//                    step's sub-steps so far: its cotangent goes to the
//                    sub-step whose value it was, and there through the
//                    flattener's pressures and weights to the primitives
//                    and opacities of its seven-cell stencil;
//   ghost cells      the transpose of the boundary copies (ghost cotangents
//                    folded into their source cells, dimensions in reverse).
// Local Jacobians come from Dual<4> passes of the same templated physics as
// the forward kernels, so each piecewise choice (limiter branch, wave-speed
// extremum, radiation limiter) is differentiated on the branch the forward
// step took.  A failed cell's fix-up (the mean of its neighbours) and the
// floors are differentiated as such, at the state before the fix-ups.
#pragma once
#include "kernels.h"

typedef Dual<4> D4;

// Seed the four inputs k0..k0+3 of an input vector of n doubles.
template <int NI>
DEV void seed4(const double v[NI], int k0, D4 out[NI]) {
#pragma unroll
  for (int q = 0; q < NI; q++) {
    out[q] = D4(v[q]);
#pragma unroll
    for (int j = 0; j < 4; j++)
      if (q == k0 + j) out[q].d[j] = 1.0;
  }
}

DEV void interior_cell(const Ctx& C, long t, int& i, int& j, int& k) {
  i = C.ng[0] + t % C.n[0];
  const long t2 = t / C.n[0];
  j = C.ng[1] + t2 % C.n[1];
  k = C.ng[2] + t2 / C.n[1];
}

// ---------------------------------------------------------------------------
// U^n = U(P^n): lamP += (dU/dP)^T lamU at interior cells
// ---------------------------------------------------------------------------
DEV void adj_p2u_at(Ctx C, const double* __restrict__ P,
                                  const double* __restrict__ lamU, double* __restrict__ lamP, long t) {
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int i, j, k;
  interior_cell(C, t, i, j, k);
  const long c = cell_index(C, i, j, k);
  Metric m;
  load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
  double p[12], lu[12];
#pragma unroll
  for (int q = 0; q < 12; q++) {
    p[q] = P[q * C.Ntot + c];
    lu[q] = lamU[q * C.Ntot + c];
  }
  for (int pass = 0; pass < 3; pass++) {
    D4 pd[12], ud[12];
    seed4<12>(p, 4 * pass, pd);
    prim_to_cons_cell(m, C.gam, pd, ud);
#pragma unroll
    for (int jj = 0; jj < 4; jj++) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 12; q++) s += lu[q] * ud[q].d[jj];
      lamP[(4 * pass + jj) * C.Ntot + c] += s;
    }
  }
}

__global__ void LB(128) k_adj_p2u(Ctx C, const double* __restrict__ P,
                                  const double* __restrict__ lamU, double* __restrict__ lamP) {
  adj_p2u_at(C, P, lamU, lamP, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Implicit solve.  The PMHD map at (x, theta): x = (u_g, u~^i), theta = the
// explicit conserved state U(i) (with sqrt(-g)); E the residual, P and U the
// outputs exactly as the forward step finalises a PMHD solution.  ent: an
// entropy-method solution (Sec. 4.11): E[0] is the entropy equation
// (eq. source6 with G_S of eq. GS, weighted by T_gas as the forward) with
// the explicit tracer Se = sqrt(-g) [S u^t]_(i); P and U as for PMHD.
// ---------------------------------------------------------------------------
template <class T>
DEV void pmhd_map(const Metric& m, const Phys& ph, double dtc, const T& chi_abs, const T& chi_es,
                  const T x[4], const T th[12], T E[4], T P[12], T U[12], bool ent = false,
                  const T& Se = T(0.0)) {
  const double igd = 1.0 / m.gdet;
  const T rhout = th[0] * igd;
  T B[3], Tgi[4], Ri[4];
#pragma unroll
  for (int i = 0; i < 3; i++) B[i] = th[5 + i] * igd;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    Tgi[k] = th[1 + k] * igd;
    Ri[k] = th[8 + k] * igd;
  }
  Gas<T> s;
  {
    Vel<T> v;
    make_vel(m, x + 1, v);
    const T rho = rhout / v.ucon[0];
    make_gas(m, ph.gam, rho, x[0], x + 1, B, s);
  }
  T row[8];
  gas_row(s, B, 0, row);
  T R[4];
#pragma unroll
  for (int k = 0; k < 4; k++) R[k] = Ri[k] - (row[1 + k] - Tgi[k]);
  T Eb, utr[3];
  const int flags = rad_invert(m, ph.gamma_max, ph.ymax, 1, R, Eb, utr);
  Vel<T> r;
  make_vel(m, utr, r);
  const T Tgas = s.pg / s.rho;
  const T T2 = Tgas * Tgas;
  const T kabs = chi_abs * s.rho, kes = chi_es * s.rho;
  const T lam = kabs * ph.arad * (T2 * T2);
  T G[4];
  four_force(s.v, r, Eb, kabs, kes, lam, G);
#pragma unroll
  for (int k = 0; k < 4; k++) E[k] = (row[1 + k] - Tgi[k]) - dtc * G[k];
  if (ent) {
    const double n = 1.0 / (ph.gam - 1.0);
    const T S = s.rho * (n * log(s.pg) - (n + 1.0) * log(s.rho));
    const T Sut = S * s.v.ucon[0];
    const T Tg = s.pg / s.rho;
    T Gu = G[0] * s.v.ucon[0];
#pragma unroll
    for (int k = 1; k < 4; k++) Gu = Gu + G[k] * s.v.ucon[k];
    E[0] = (Tg * Sut - Tg * (Se * igd)) + dtc * Gu;
  }
  P[0] = s.rho;
  P[1] = x[0];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    P[2 + i] = x[1 + i];
    P[5 + i] = B[i];
    P[9 + i] = utr[i];
  }
  P[8] = Eb;
  T Ur[4];
#pragma unroll
  for (int k = 0; k < 4; k++) Ur[k] = R[k];
  if (flags & 1) {   // E_rad <= 0 met: BASIC re-inversion of the radiation
    T Eb2, ut2[3];
    rad_invert(m, ph.gamma_max, ph.ymax, 0, R, Eb2, ut2);
    P[8] = Eb2;
#pragma unroll
    for (int i = 0; i < 3; i++) P[9 + i] = ut2[i];
  }
  if (flags) {       // a limiter acted: radiation recomputed from its primitives
    Vel<T> r2;
    make_vel(m, P + 9, r2);
    rad_row(r2, P[8], 0, Ur);
  }
  U[0] = th[0];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    U[1 + k] = m.gdet * row[1 + k];
    U[8 + k] = m.gdet * Ur[k];
  }
#pragma unroll
  for (int i = 0; i < 3; i++) U[5 + i] = th[5 + i];
}

// ENT (full cascade): Se, the stage's explicit entropy tracer sqrt(-g)
// [S u^t]_(i); lamS [Ntot] out: its cotangent at interior cells (zero where
// the solution is not an entropy-method one).  Without ENT both are unused
// and the entropy row is not compiled in.
template <bool ENT>
DEV void adj_implicit_at(Ctx C, double scale, const double* __restrict__ dt_dev,
                                      const double* __restrict__ Ue, const double* __restrict__ Pk,
                                      const int* __restrict__ status,
                                      const double* __restrict__ chi_abs,
                                      const double* __restrict__ chi_es,
                                      const double* __restrict__ lamP,
                                      const double* __restrict__ lamU, double* __restrict__ lamUe,
                                      double* __restrict__ gchi, const double* __restrict__ Se,
                                      double* __restrict__ lamS, long t) {
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int i, j, k;
  interior_cell(C, t, i, j, k);
  const long c = cell_index(C, i, j, k);
  double lp[12], lu[12], th[12], x[4];
#pragma unroll
  for (int q = 0; q < 12; q++) {
    lp[q] = lamP[q * C.Ntot + c];
    lu[q] = lamU[q * C.Ntot + c];
    th[q] = Ue[q * C.Ntot + c];
  }
  bool ok = !(status[c] & GRRMHD_ST_FAIL);
  const bool ent = ENT && ok && (status[c] & GRRMHD_ST_ENTROPY) && !(status[c] & GRRMHD_ST_COLD);
  const double se = ent ? Se[c] : 0.0;
  if (ENT) lamS[c] = 0.0;
  double mu[4];
  Metric m;
  load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
  Phys ph;
  ph.gam = C.gam;
  ph.arad = C.arad;
  ph.gamma_max = C.gamma_max;
  ph.ymax = C.ymax;
  const double dtc = scale * (*dt_dev);
  const double ca = chi_abs[c], ce = chi_es[c];
  if (ok) {
#pragma unroll
    for (int q = 0; q < 4; q++) x[q] = Pk[(1 + q) * C.Ntot + c];
    D4 xd[4], thd[12], E[4], Po[12], Uo[12];
    seed4<4>(x, 0, xd);
#pragma unroll
    for (int q = 0; q < 12; q++) thd[q] = D4(th[q]);
    pmhd_map(m, ph, dtc, D4(ca), D4(ce), xd, thd, E, Po, Uo, ent, D4(se));
    double JT[4][4], gx[4];
#pragma unroll
    for (int jj = 0; jj < 4; jj++) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 12; q++) s += lp[q] * Po[q].d[jj] + lu[q] * Uo[q].d[jj];
      gx[jj] = s;
#pragma unroll
      for (int kk = 0; kk < 4; kk++) JT[jj][kk] = E[kk].d[jj];
    }
    if (status[c] & GRRMHD_ST_COLD) {   // cold limit: u_g held, the energy equation dropped
      gx[0] = 0.0;
      JT[0][0] = 1.0;
#pragma unroll
      for (int k = 1; k < 4; k++) JT[0][k] = JT[k][0] = 0.0;
    }
    ok = solve4(JT, gx, mu) == 0;
    // the explicit tracer enters E[0] alone, as -T_gas Se/sqrt(-g)
    if (ENT && ok && ent) lamS[c] = mu[0] * ((ph.gam - 1.0) * x[0] / Po[0].v) / m.gdet;
  }
  if (!ok) {   // failed cell (or singular Jacobian): U passes through unchanged
#pragma unroll
    for (int q = 0; q < 12; q++) lamUe[q * C.Ntot + c] = lu[q];
    return;
  }
  // passes over the 12 conserved inputs, four at a time; the values are kept
  // opaque per pass (empty asm) so the compiler recomputes them rather than
  // hoisting the whole value chain out of the loop and spilling it
#pragma unroll 1
  for (int pass = 0; pass < 3; pass++) {
    D4 xd[4], thd[12], E[4], Po[12], Uo[12];
    double xv[4], tv[12];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      xv[q] = x[q];
      asm volatile("" : "+v"(xv[q]));
      xd[q] = D4(xv[q]);
    }
#pragma unroll
    for (int q = 0; q < 12; q++) {
      tv[q] = th[q];
      asm volatile("" : "+v"(tv[q]));
    }
    seed4<12>(tv, 4 * pass, thd);
    pmhd_map(m, ph, dtc, D4(ca), D4(ce), xd, thd, E, Po, Uo, ent, D4(se));
#pragma unroll
    for (int jj = 0; jj < 4; jj++) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 12; q++) s += lp[q] * Po[q].d[jj] + lu[q] * Uo[q].d[jj];
#pragma unroll
      for (int kk = 0; kk < 4; kk++) s -= mu[kk] * E[kk].d[jj];
      lamUe[(4 * pass + jj) * C.Ntot + c] = s;
    }
  }
  if (gchi) {   // the opacities: they enter the residual only (kappa = chi rho0)
    D4 xd[4], thd[12], E[4], Po[12], Uo[12];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      double v = x[q];
      asm volatile("" : "+v"(v));
      xd[q] = D4(v);
    }
#pragma unroll
    for (int q = 0; q < 12; q++) {
      double v = th[q];
      asm volatile("" : "+v"(v));
      thd[q] = D4(v);
    }
    pmhd_map(m, ph, dtc, D4::var(ca, 0), D4::var(ce, 1), xd, thd, E, Po, Uo, ent, D4(se));
#pragma unroll
    for (int jj = 0; jj < 2; jj++) {
      double s = 0.0;
#pragma unroll
      for (int kk = 0; kk < 4; kk++) s -= mu[kk] * E[kk].d[jj];
      gchi[jj * C.Ntot + c] += s;
    }
  }
}

template <bool ENT>
__global__ void LB(64) k_adj_implicit(Ctx C, double scale, const double* __restrict__ dt_dev,
                                      const double* __restrict__ Ue, const double* __restrict__ Pk,
                                      const int* __restrict__ status,
                                      const double* __restrict__ chi_abs,
                                      const double* __restrict__ chi_es,
                                      const double* __restrict__ lamP,
                                      const double* __restrict__ lamU, double* __restrict__ lamUe,
                                      double* __restrict__ gchi, const double* __restrict__ Se,
                                      double* __restrict__ lamS) {
  adj_implicit_at<ENT>(C, scale, dt_dev, Ue, Pk, status, chi_abs, chi_es, lamP, lamU, lamUe, gchi,
                       Se, lamS, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Fix-ups: a failed cell takes P_f = mean of its face neighbours' P (those
// with a good energy solution, neither failed nor cold; all of them when none
// is good), a cold cell the same mean for u_g alone; then the floors F
// (rho0, u_g from below, u_g/rho0 from above, Ebar from below); then U = U(P)
// where P changed.  Transpose: Lam = J_F^T (lamP + (dU/dP)^T lamU) at a
// changed or floored cell (J_F at the state the floors met: the mean, or the
// solve's own output), spread back over the neighbours that were averaged
// (all fields from a failed cell, u_g from a cold one); a failed cell's own
// solve receives nothing, a cold cell's keeps Lam except for u_g, a floored
// cell's keeps Lam, and U before the fix-up receives nothing where P
// changed.  A cell with no interior neighbour is not averaged.  Without the
// state before the fix-ups (Ppre null) floors are taken as the identity.
// ---------------------------------------------------------------------------
DEV bool failed_at(const int* st, long c) { return (st[c] & GRRMHD_ST_FAIL) != 0; }
DEV bool bad_at(const int* st, long c) { return (st[c] & (GRRMHD_ST_FAIL | GRRMHD_ST_COLD)) != 0; }

DEV bool interior_idx(const Ctx& C, const int idx[3]) {
  for (int d = 0; d < 3; d++)
    if (idx[d] < C.ng[d] || idx[d] >= C.ng[d] + C.n[d]) return false;
  return true;
}

// neighbours the fix-up averaged for cell idx: good ones (good_pass) or all
DEV int fixup_count(const Ctx& C, const int* st, const int idx[3], bool& good_pass) {
  int good = 0, all = 0;
  const long c = cell_index(C, idx[0], idx[1], idx[2]);
  for (int d = 0; d < 3; d++) {
    if (C.n[d] == 1) continue;
    for (int s = -1; s <= 1; s += 2) {
      const int nid = idx[d] + s;
      if (nid < C.ng[d] || nid >= C.ng[d] + C.n[d]) continue;
      all++;
      if (!bad_at(st, c + s * C.st[d])) good++;
    }
  }
  good_pass = good > 0;
  return good_pass ? good : all;
}

// a failed or cold cell that had neighbours to average (so P and U changed)
DEV bool fixed_at(const Ctx& C, const int* st, const int idx[3]) {
  if (!bad_at(st, cell_index(C, idx[0], idx[1], idx[2]))) return false;
  bool gp;
  return fixup_count(C, st, idx, gp) > 0;
}

// the fix-up's floors on primitives p, in place (as the forward fix-up)
template <class T>
DEV void floor_map(const Ctx& C, const Metric& m, T p[12]) {
  Gas<T> s;
  make_gas(m, C.gam, p[0], p[1], p + 2, p + 5, s);
  const T br = s.bsq / C.bsq_rho_max, bu = s.bsq / C.bsq_u_max;
  const T rmin = (val(br) > C.rho_floor) ? br : T(C.rho_floor);
  const T umin = (val(bu) > C.u_floor) ? bu : T(C.u_floor);
  if (val(p[0]) < val(rmin)) p[0] = rmin;
  if (val(p[1]) < val(umin)) p[1] = umin;
  if (val(p[1]) > C.u_rho_max * val(p[0])) p[1] = C.u_rho_max * p[0];
  if (!(val(p[8]) >= C.erad_floor)) p[8] = T(C.erad_floor);
}

// a changed cell: Lam; a floored cell (with Ppre) too
DEV bool touched_at(const Ctx& C, const int* st, const int idx[3], bool exact_floors) {
  return fixed_at(C, st, idx) ||
         (exact_floors && (st[cell_index(C, idx[0], idx[1], idx[2])] & GRRMHD_ST_FLOOR));
}

DEV void adj_fixup_own_at(Ctx C, const double* __restrict__ P, const double* __restrict__ Ppre,
                          const int* __restrict__ st, const double* __restrict__ lamP,
                          const double* __restrict__ lamU, double* __restrict__ Lam, long t) {
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int idx[3];
  interior_cell(C, t, idx[0], idx[1], idx[2]);
  const long c = cell_index(C, idx[0], idx[1], idx[2]);
  const bool fixed = fixed_at(C, st, idx);
  const bool floored = Ppre && (st[c] & GRRMHD_ST_FLOOR);
  if (!fixed && !floored) return;
  Metric m;
  load_metric(C.geo_c, C.npos, idx[0] + C.N[0] * idx[1], m);
  double p[12], lu[12], lo[12];
#pragma unroll
  for (int q = 0; q < 12; q++) {
    p[q] = P[q * C.Ntot + c];
    lu[q] = lamU[q * C.Ntot + c];
  }
  for (int pass = 0; pass < 3; pass++) {
    D4 pd[12], ud[12];
    seed4<12>(p, 4 * pass, pd);
    prim_to_cons_cell(m, C.gam, pd, ud);
#pragma unroll
    for (int jj = 0; jj < 4; jj++) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 12; q++) s += lu[q] * ud[q].d[jj];
      lo[4 * pass + jj] = lamP[(4 * pass + jj) * C.Ntot + c] + s;
    }
  }
  if (!floored) {
#pragma unroll
    for (int q = 0; q < 12; q++) Lam[q * C.Ntot + c] = lo[q];
    return;
  }
  // the state the floors met: the solve's output, with the neighbours' mean
  // where the cell was averaged (as the forward: the same neighbours, sum
  // then times 1/count)
  double pp[12];
#pragma unroll
  for (int q = 0; q < 12; q++) pp[q] = Ppre[q * C.Ntot + c];
  if (fixed) {
    bool good_pass;
    const int cnt = fixup_count(C, st, idx, good_pass);
    double acc[12];
#pragma unroll
    for (int q = 0; q < 12; q++) acc[q] = 0.0;
    for (int d = 0; d < 3; d++) {
      if (C.n[d] == 1) continue;
      for (int s = -1; s <= 1; s += 2) {
        const int nid = idx[d] + s;
        if (nid < C.ng[d] || nid >= C.ng[d] + C.n[d]) continue;
        const long nb = c + s * C.st[d];
        if (good_pass && bad_at(st, nb)) continue;
#pragma unroll
        for (int q = 0; q < 12; q++) acc[q] += Ppre[q * C.Ntot + nb];
      }
    }
    const double w = 1.0 / cnt;
    const bool fc = failed_at(st, c);
#pragma unroll
    for (int q = 0; q < 12; q++)
      if (fc || q == 1) pp[q] = acc[q] * w;
  }
  for (int pass = 0; pass < 3; pass++) {
    D4 pd[12];
    seed4<12>(pp, 4 * pass, pd);
    floor_map(C, m, pd);
#pragma unroll
    for (int jj = 0; jj < 4; jj++) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 12; q++) s += lo[q] * pd[q].d[jj];
      Lam[(4 * pass + jj) * C.Ntot + c] = s;
    }
  }
}

// Ppre (nullable): the state before the fix-ups (the floors' transpose)
__global__ void LB(128) k_adj_fixup_own(Ctx C, const double* __restrict__ P,
                                        const double* __restrict__ Ppre,
                                        const int* __restrict__ st, const double* __restrict__ lamP,
                                        const double* __restrict__ lamU, double* __restrict__ Lam) {
  adj_fixup_own_at(C, P, Ppre, st, lamP, lamU, Lam, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

DEV void adj_fixup_at(Ctx C, int exact_floors, const int* __restrict__ st,
                      const double* __restrict__ Lam, const double* __restrict__ lamP,
                      const double* __restrict__ lamU, double* __restrict__ lamPpre,
                      double* __restrict__ lamUpre, long t) {
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int idx[3];
  interior_cell(C, t, idx[0], idx[1], idx[2]);
  const long c = cell_index(C, idx[0], idx[1], idx[2]);
  const bool fixed = fixed_at(C, st, idx);
  const bool touched = touched_at(C, st, idx, exact_floors != 0);
  const bool fc = fixed && failed_at(st, c);
  const bool bc = bad_at(st, c);
  double acc[12];
#pragma unroll
  for (int q = 0; q < 12; q++)
    acc[q] = !touched ? lamP[q * C.Ntot + c]
                      : ((fixed && (fc || q == 1)) ? 0.0 : Lam[q * C.Ntot + c]);
  for (int d = 0; d < 3; d++) {
    if (C.n[d] == 1) continue;
    for (int s = -1; s <= 1; s += 2) {
      int nb[3] = {idx[0], idx[1], idx[2]};
      nb[d] += s;
      if (!interior_idx(C, nb)) continue;
      const long f = c + s * C.st[d];
      if (!bad_at(st, f)) continue;
      bool good_pass;
      const int cnt = fixup_count(C, st, nb, good_pass);
      if (cnt == 0 || (good_pass && bc)) continue;
      const double w = 1.0 / cnt;
      if (failed_at(st, f)) {
#pragma unroll
        for (int q = 0; q < 12; q++) acc[q] += w * Lam[q * C.Ntot + f];
      } else {
        acc[1] += w * Lam[1 * C.Ntot + f];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 12; q++) {
    lamPpre[q * C.Ntot + c] = acc[q];
    lamUpre[q * C.Ntot + c] = touched ? 0.0 : lamU[q * C.Ntot + c];
  }
}

// exact_floors: Lam holds the floors' transpose (k_adj_fixup_own with Ppre)
__global__ void LB(256) k_adj_fixup(Ctx C, int exact_floors, const int* __restrict__ st,
                                    const double* __restrict__ Lam,
                                    const double* __restrict__ lamP, const double* __restrict__ lamU,
                                    double* __restrict__ lamPpre, double* __restrict__ lamUpre) {
  adj_fixup_at(C, exact_floors, st, Lam, lamP, lamU, lamPpre, lamUpre,
               (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Linear parts of the stage combination: lamUn += a lamUe, lamUprev = b lamUe
// ---------------------------------------------------------------------------
DEV void adj_stage_at(Ctx C, double a, double b, const double* __restrict__ lamUe,
                                    double* __restrict__ lamUn, double* __restrict__ lamUprev, long t) {
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int i, j, k;
  interior_cell(C, t, i, j, k);
  const long c = cell_index(C, i, j, k);
#pragma unroll
  for (int q = 0; q < 12; q++) {
    const double l = lamUe[q * C.Ntot + c];
    lamUn[q * C.Ntot + c] += a * l;
    lamUprev[q * C.Ntot + c] = b * l;
  }
}

__global__ void LB(256) k_adj_stage(Ctx C, double a, double b, const double* __restrict__ lamUe,
                                    double* __restrict__ lamUn, double* __restrict__ lamUprev) {
  adj_stage_at(C, a, b, lamUe, lamUn, lamUprev, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Corner EMFs: cotangent of E_a at the edges of edge range R, gathered from
// the stage cotangent lamUe (zero outside the interior) through the face
// induction fluxes the update builds from the EMFs.
// ---------------------------------------------------------------------------
DEV void adj_emf_at(Ctx C, int a, FaceRange R, double scale,
                                  const double* __restrict__ dt_dev,
                                  const double* __restrict__ lamUe, double* __restrict__ lamE, long t) {
  if (t >= R.total) return;
  const int i = R.lo[0] + t % R.cnt[0];
  const long t2 = t / R.cnt[0];
  const int j = R.lo[1] + t2 % R.cnt[1];
  const int k = R.lo[2] + t2 / R.cnt[1];
  const long e = cell_index(C, i, j, k);
  const int b = (a + 1) % 3, cd = (a + 2) % 3;
  double acc = 0.0;
  bool zero = false;
  if (C.metric == GRRMHD_KERR_SCHILD && (b == 1 || cd == 1)) {
    const bool lo = j == C.ng[1] && (C.bc_lo[1] == GRRMHD_BC_REFLECT || C.bc_lo[1] == GRRMHD_BC_POLAR);
    const bool hi = j == C.ng[1] + C.n[1] && (C.bc_hi[1] == GRRMHD_BC_REFLECT || C.bc_hi[1] == GRRMHD_BC_POLAR);
    zero = lo || hi;
  }
  if (!zero) {
    const double cdt = scale * (*dt_dev);
    for (int pair = 0; pair < 2; pair++) {
      const int d = pair ? cd : b;        // flux direction
      const int bb = pair ? b : cd;       // field component
      const double sgn = ((a + 1) % 3 == bb) ? 1.0 : -1.0;
      const double coef = -cdt / C.dx[d] * 0.5 * sgn;
      const double* L = lamUe + (5 + bb) * C.Ntot;
      const long sd = C.st[d], sb = C.st[bb];
      acc += coef * ((L[e - sd] + L[e - sd - sb]) - (L[e] + L[e - sb]));
    }
  }
  lamE[(long)a * C.Ntot + e] = acc;
}

__global__ void LB(256) k_adj_emf(Ctx C, int a, FaceRange R, double scale,
                                  const double* __restrict__ dt_dev,
                                  const double* __restrict__ lamUe, double* __restrict__ lamE) {
  adj_emf_at(C, a, R, scale, dt_dev, lamUe, lamE, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// A face state reduced to what the flux cotangent needs: the sums
// sum_q lF[q] U_q and sum_q lF[q] F_q over the gas components (q < 8, the
// normal field left out; with the entropy tracer's flux, which takes the gas
// speeds, weighted by lFs) and over the radiation components (q >= 8), and
// the four characteristic speeds.  The flux is linear in U and F once the
// speeds are fixed, so these sums carry all of it.
template <class T>
struct FaceSums {
  T gU, gF, rU, rF;
  T gm, gp, rm, rp;
};

template <class T>
DEV void face_sums(const Ctx& C, const Metric& m, int d, const T* P, T chi_tot, const double lF[12],
                   FaceSums<T>& o, double lFs = 0.0) {
  Gas<T> s;
  make_gas(m, C.gam, P[0], P[1], P + 2, P + 5, s);
  T row[8];
  T acc;
  gas_row(s, P + 5, 0, row);
  acc = T(0.0);
#pragma unroll
  for (int q = 0; q < 8; q++)
    if (q != 4 + d) acc = acc + lF[q] * row[q];
  o.gU = m.gdet * acc;
  gas_row(s, P + 5, d, row);
  acc = T(0.0);
#pragma unroll
  for (int q = 0; q < 8; q++)
    if (q != 4 + d) acc = acc + lF[q] * row[q];
  o.gF = m.gdet * acc;
  if (lFs != 0.0) {
    // the tracer sqrt(-g) S u^t and its flux sqrt(-g) S u^d (as entropy_face)
    const double n = 1.0 / (C.gam - 1.0);
    const T S = P[0] * (n * log(s.pg) - (n + 1.0) * log(P[0]));
    o.gU = o.gU + lFs * (m.gdet * S * s.v.ucon[0]);
    o.gF = o.gF + lFs * (m.gdet * S * s.v.ucon[d]);
  }
  Vel<T> r;
  make_vel(m, P + 9, r);
  T rr[4];
  rad_row(r, P[8], 0, rr);
  acc = T(0.0);
#pragma unroll
  for (int q = 0; q < 4; q++) acc = acc + lF[8 + q] * rr[q];
  o.rU = m.gdet * acc;
  rad_row(r, P[8], d, rr);
  acc = T(0.0);
#pragma unroll
  for (int q = 0; q < 4; q++) acc = acc + lF[8 + q] * rr[q];
  o.rF = m.gdet * acc;
  face_speeds(C, m, d, P, chi_tot, s, r, o.gm, o.gp, o.rm, o.rp);
}

// The contracted Riemann flux sum_q lF[q] flux_q of one face (HLL or LAXF,
// as the forward step), its derivative carried by whichever side is a Dual,
// the other side a constant.  Speed extrema take their operands in the
// forward order, so a tie between the two sides takes the forward branch.
template <int N, class TL, class TR>
DEV void flux_contract(const Ctx& C, const FaceSums<TL>& L, const FaceSums<TR>& R, double acc[N]) {
  typedef Dual<N> T;
  const T gmin = -fmin(0.0, fmin(L.gm, R.gm)), gmax = fmax(0.0, fmax(L.gp, R.gp));
  const T rmin = -fmin(0.0, fmin(L.rm, R.rm)), rmax = fmax(0.0, fmax(L.rp, R.rp));
  T fl[2];
#pragma unroll
  for (int grp = 0; grp < 2; grp++) {
    const T vmin = grp ? rmin : gmin, vmax = grp ? rmax : gmax;
    const TL LU = grp ? L.rU : L.gU, LF = grp ? L.rF : L.gF;
    const TR RU = grp ? R.rU : R.gU, RF = grp ? R.rF : R.gF;
    if (C.flux == GRRMHD_FLUX_HLL) {
      const T den = vmin + vmax;
      fl[grp] = (den.v > 0.0) ? (vmin * RF + vmax * LF - vmin * vmax * (RU - LU)) / den
                              : 0.5 * (LF + RF);
    } else {
      fl[grp] = 0.5 * (RF + LF - fmax(vmin, vmax) * (RU - LU));
    }
  }
#pragma unroll
  for (int jj = 0; jj < N; jj++) acc[jj] = fl[0].d[jj] + fl[1].d[jj];
}

// One side S (0 left, 1 right) of a face: its 12 reconstructed primitives
// seeded NS at a time with the other side's state held fixed, giving
// lS[q] = sum_p lF[p] d(flux_p)/d(P_S[q]); with gx, also the derivative with
// respect to side S's total opacity (radiation speed limiter).
//
// Every pass recomputes the same values under different seeds.  Left alone,
// the compiler hoists that value chain out of the pass loop and keeps its
// hundreds of intermediates live across it, which spills; an empty asm
// statement on each input makes the values opaque per pass, so each pass
// recomputes them in registers (measured: the 96x48x24 disk adjoint step
// 5.7 ms -> 3.0 ms).  Two seeds per pass spill least at equal speed.
template <int S>
DEV void adj_face_side(const Ctx& C, const Metric& m, int D, const double PLR[24], double chiL,
                       double chiR, const double lF[12], double lS[12], double* gx,
                       double lFs = 0.0) {
  constexpr int NS = 2;
  typedef Dual<NS> DS;
  const double* own = PLR + 12 * S;
  const double chi_own = S ? chiR : chiL;
  FaceSums<double> O;
  face_sums(C, m, D, PLR + 12 * (1 - S), S ? chiL : chiR, lF, O, lFs);
#pragma unroll 1
  for (int g = 0; g < 12 / NS; g++) {
    DS in[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      double v = own[q];
      asm volatile("" : "+v"(v));   // no instruction: keeps the pass's values from being hoisted
      in[q] = DS(v);
#pragma unroll
      for (int jj = 0; jj < NS; jj++)
        if (q == NS * g + jj) in[q].d[jj] = 1.0;
    }
    FaceSums<DS> F;
    face_sums(C, m, D, in, DS(chi_own), lF, F, lFs);
    double acc[NS];
    if (S == 0)
      flux_contract<NS>(C, F, O, acc);
    else
      flux_contract<NS>(C, O, F, acc);
#pragma unroll
    for (int q = 0; q < 12; q++) lS[q] = (q / NS == g) ? acc[q % NS] : lS[q];
  }
  if (gx) {
    Dual<1> in[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      double v = own[q];
      asm volatile("" : "+v"(v));
      in[q] = Dual<1>(v);
    }
    FaceSums<Dual<1>> F;
    face_sums(C, m, D, in, Dual<1>::var(chi_own, 0), lF, F, lFs);
    double acc[1];
    if (S == 0)
      flux_contract<1>(C, F, O, acc);
    else
      flux_contract<1>(C, O, F, acc);
    *gx = acc[0];
  }
}

// ---------------------------------------------------------------------------
// Faces normal to D: the cotangent of the face flux, then its Jacobian with
// respect to the stencil cells c + (m - NSL/2) s, m = 0..NSL-1 (s the stride
// along D; NSL = 4 for MC, 6 for PPM); the products go to
// G[(m*12 + q)][face].  PPM also reads the flattener fl of the face's two
// cells (this sub-step's, as the forward read it); the face's products with
// those four values (gas and radiation of the left cell, then of the right)
// go to GF[4][face].
// ---------------------------------------------------------------------------
template <int D, bool PPM>
DEV void adj_flux_at(Ctx C, FaceRange R, double scale,
                                                 const double* __restrict__ dt_dev,
                                                 const double* __restrict__ P,
                                                 const double* __restrict__ chi_abs,
                                                 const double* __restrict__ chi_es,
                                                 const double* __restrict__ lamUe,
                                                 const double* __restrict__ lamE,
                                                 double* __restrict__ G, double* __restrict__ Gx,
                                                 const double* __restrict__ fl,
                                                 double* __restrict__ GF,
                                                 const double* __restrict__ lamS, long t) {
  if (t >= R.total) return;
  const int i = R.lo[0] + t % R.cnt[0];
  const long t2 = t / R.cnt[0];
  const int j = R.lo[1] + t2 % R.cnt[1];
  const int k = R.lo[2] + t2 / R.cnt[1];
  const long f = cell_index(C, i, j, k);
  const int d = D - 1;
  const long st = C.st[d];
  const double cdt = scale * (*dt_dev);
  const double idx = 1.0 / C.dx[d];
  double lF[12];
#pragma unroll
  for (int q = 0; q < 12; q++) {
    const double direct = cdt * idx * (lamUe[q * C.Ntot + f] - lamUe[q * C.Ntot + f - st]);
    if (q >= 5 && q <= 7) {
      const int e = q - 5;
      if (e == d) {
        lF[q] = 0.0;                       // normal field: no induction flux
      } else if (C.n[e] > 1) {             // through the corner EMF E_a, a the third axis
        const int a = 3 - d - e;
        const double sgn = (d == (a + 2) % 3) ? 0.25 : -0.25;
        const double* L = lamE + (long)a * C.Ntot;
        lF[q] = sgn * (L[f] + L[f + C.st[e]]);
      } else {
        lF[q] = direct;
      }
    } else {
      lF[q] = direct;
    }
  }
  // PPM: the flattener of the left and right cells (gas, radiation), and on
  // Kerr-Schild along r the sqrt(-g) weights of the vector primitives
  double fgL = 0.0, frL = 0.0, fgR = 0.0, frR = 0.0, gc[6] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
  double gface = 1.0;
  const bool wgt = PPM && (D == 1) && C.metric == GRRMHD_KERR_SCHILD;
  if (PPM) {
    const double* fg = fl + (long)(2 * d) * C.Ntot;
    const double* fr = fg + C.Ntot;
    fgL = fg[f - st];
    frL = fr[f - st];
    fgR = fg[f];
    frR = fr[f];
    if (wgt) {
#pragma unroll
      for (int m = 0; m < 6; m++) gc[m] = C.geo_c[GE_GDET * C.npos + (i + m - 3) + C.N[0] * j];
      gface = C.geo_f1[GE_GDET * C.npos + i + C.N[0] * j];
    }
  }
  double PLR[24];
#pragma unroll
  for (int q = 0; q < 12; q++) {
    const double* p = P + q * C.Ntot;
    if (PPM) {
      const bool vec = wgt && ((q >= 2 && q <= 7) || q >= 9);
      double a[6], l, r;
#pragma unroll
      for (int m = 0; m < 6; m++) a[m] = vec ? p[f + (m - 3) * st] * gc[m] : p[f + (m - 3) * st];
      ppm_cell(a, q < 8 ? fgL : frL, l, PLR[q]);
      ppm_cell(a + 1, q < 8 ? fgR : frR, PLR[12 + q], r);
      if (vec) {
        PLR[q] = PLR[q] / gface;
        PLR[12 + q] = PLR[12 + q] / gface;
      }
    } else {
      const double a = p[f - 2 * st], b = p[f - st], e = p[f], ff = p[f + st];
      PLR[q] = b + 0.5 * mc_slope(b - a, e - b);
      PLR[12 + q] = e - 0.5 * mc_slope(e - b, ff - e);
    }
  }
  Metric m;
  const double* tab = (D == 1) ? C.geo_f1 : ((D == 2) ? C.geo_f2 : C.geo_c);
  load_metric(tab, C.npos, i + C.N[0] * j, m);
  const double chiL = chi_abs[f - st] + chi_es[f - st], chiR = chi_abs[f] + chi_es[f];
  // the entropy tracer's face flux (full cascade): its cotangent as the
  // stage update's divergence gives it
  const double lFs = lamS ? cdt * idx * (lamS[f] - lamS[f - st]) : 0.0;
  double lPLR[24];
  double gxL = 0.0, gxR = 0.0;
  adj_face_side<0>(C, m, D, PLR, chiL, chiR, lF, lPLR, Gx ? &gxL : nullptr, lFs);
  adj_face_side<1>(C, m, D, PLR, chiL, chiR, lF, lPLR + 12, Gx ? &gxR : nullptr, lFs);
  if (Gx) {
    Gx[f] = gxL;                 // d/d chi_tot of cell f - e_d
    Gx[C.Ntot + f] = gxR;        // d/d chi_tot of cell f
  }
  // the reconstruction, per primitive, with respect to the stencil cells
  // (the stencil is read again rather than held through the face passes)
  if (PPM) {
    typedef Dual<8> D8;   // six stencil cells, the left and the right flattener
    double gf[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 12; q++) {
      const double* p = P + q * C.Ntot;
      const bool vec = wgt && ((q >= 2 && q <= 7) || q >= 9);
      D8 a[6];
#pragma unroll
      for (int s = 0; s < 6; s++) {
        a[s] = D8(vec ? p[f + (s - 3) * st] * gc[s] : p[f + (s - 3) * st]);
        a[s].d[s] = vec ? gc[s] : 1.0;
      }
      const D8 fL = D8::var(q < 8 ? fgL : frL, 6), fR = D8::var(q < 8 ? fgR : frR, 7);
      D8 l, r, PL, PR;
      ppm_cell(a, fL, l, PL);
      ppm_cell(a + 1, fR, PR, r);
      const double ig = vec ? 1.0 / gface : 1.0;
#pragma unroll
      for (int s = 0; s < 6; s++)
        G[(s * 12 + q) * C.Ntot + f] = ig * (lPLR[q] * PL.d[s] + lPLR[12 + q] * PR.d[s]);
      gf[q < 8 ? 0 : 1] += ig * lPLR[q] * PL.d[6];
      gf[q < 8 ? 2 : 3] += ig * lPLR[12 + q] * PR.d[7];
    }
#pragma unroll
    for (int s = 0; s < 4; s++) GF[s * C.Ntot + f] = gf[s];
  } else {
#pragma unroll
    for (int q = 0; q < 12; q++) {
      const double* p = P + q * C.Ntot;
      const double v[4] = {p[f - 2 * st], p[f - st], p[f], p[f + st]};
      D4 s[4];
      seed4<4>(v, 0, s);
      const D4 PL = s[1] + 0.5 * mc_slope(s[1] - s[0], s[2] - s[1]);
      const D4 PR = s[2] - 0.5 * mc_slope(s[2] - s[1], s[3] - s[2]);
#pragma unroll
      for (int slot = 0; slot < 4; slot++)
        G[(slot * 12 + q) * C.Ntot + f] = lPLR[q] * PL.d[slot] + lPLR[12 + q] * PR.d[slot];
    }
  }
}

template <int D, bool PPM>
__global__ void __launch_bounds__(64) k_adj_flux(Ctx C, FaceRange R, double scale,
                                                 const double* __restrict__ dt_dev,
                                                 const double* __restrict__ P,
                                                 const double* __restrict__ chi_abs,
                                                 const double* __restrict__ chi_es,
                                                 const double* __restrict__ lamUe,
                                                 const double* __restrict__ lamE,
                                                 double* __restrict__ G, double* __restrict__ Gx,
                                                 const double* __restrict__ fl,
                                                 double* __restrict__ GF,
                                                 const double* __restrict__ lamS) {
  adj_flux_at<D, PPM>(C, R, scale, dt_dev, P, chi_abs, chi_es, lamUe, lamE, G, Gx, fl, GF, lamS,
                      (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Per allocated cell: gather the stencil products of the faces that read it;
// with the geometric source's Jacobian added at interior cells (a kernel of
// its own, the next one), the result is the cotangent of the stage's
// ghost-filled input primitives.  The gather is memory-bound and small in
// registers, the source Jacobian the opposite, hence two kernels.
// ---------------------------------------------------------------------------
struct FaceRanges {
  FaceRange r[3];
};

template <int NSL>
DEV void adj_gather_at(Ctx C, FaceRanges FR, const double* __restrict__ G1,
                       const double* __restrict__ G2, const double* __restrict__ G3,
                       double* __restrict__ lamPb, long c) {
  if (c >= C.Ntot) return;
  int idx[3];
  idx[0] = c % C.N[0];
  idx[1] = (c / C.N[0]) % C.N[1];
  idx[2] = c / ((long)C.N[0] * C.N[1]);
  double acc[12];
#pragma unroll
  for (int q = 0; q < 12; q++) acc[q] = 0.0;
  for (int d = 0; d < 3; d++) {
    if (C.n[d] == 1) continue;
    const double* G = (d == 0) ? G1 : ((d == 1) ? G2 : G3);
    const FaceRange& R = FR.r[d];
    bool trans = true;
    for (int e = 0; e < 3; e++)
      if (e != d && (idx[e] < R.lo[e] || idx[e] >= R.lo[e] + R.cnt[e])) trans = false;
    if (!trans) continue;
    for (int slot = 0; slot < NSL; slot++) {
      const int fd = idx[d] + NSL / 2 - slot;   // face whose slot-th stencil cell is c
      if (fd < R.lo[d] || fd >= R.lo[d] + R.cnt[d]) continue;
      const long f = c + (long)(NSL / 2 - slot) * C.st[d];
#pragma unroll
      for (int q = 0; q < 12; q++) acc[q] += G[(slot * 12 + q) * C.Ntot + f];
    }
  }
#pragma unroll
  for (int q = 0; q < 12; q++) lamPb[q * C.Ntot + c] = acc[q];
}

template <int NSL>
__global__ void LB(256) k_adj_gather(Ctx C, FaceRanges FR, const double* __restrict__ G1,
                                     const double* __restrict__ G2, const double* __restrict__ G3,
                                     double* __restrict__ lamPb) {
  adj_gather_at<NSL>(C, FR, G1, G2, G3, lamPb, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// Interior cell t (curved metric): lamPb += c dt (dS/dP)^T lamUe, the
// geometric source's Jacobian by Dual<4> passes over the 12 primitives.
DEV void adj_geom_at(Ctx C, double scale, const double* __restrict__ dt_dev,
                     const double* __restrict__ P, const double* __restrict__ lamUe,
                     double* __restrict__ lamPb, long t) {
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int i, j, k;
  interior_cell(C, t, i, j, k);
  const long c = cell_index(C, i, j, k);
  const int pos = i + C.N[0] * j;
  Metric m;
  load_metric(C.geo_c, C.npos, pos, m);
  double p[12], lu[12], dg[2][10];
#pragma unroll
  for (int q = 0; q < 12; q++) {
    p[q] = P[q * C.Ntot + c];
    lu[q] = lamUe[q * C.Ntot + c];
  }
  load_dg(C, pos, dg);
  const double cdt = scale * (*dt_dev);
  // values kept opaque per pass (empty asm), as in the face passes
#pragma unroll 1
  for (int pass = 0; pass < 3; pass++) {
    D4 pd[12], S[12];
    double pv[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      pv[q] = p[q];
      asm volatile("" : "+v"(pv[q]));
    }
    seed4<12>(pv, 4 * pass, pd);
    geom_source(m, dg, C.gam, pd, S);
#pragma unroll
    for (int jj = 0; jj < 4; jj++) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 12; q++) s += lu[q] * S[q].d[jj];
      lamPb[(4 * pass + jj) * C.Ntot + c] += cdt * s;
    }
  }
}

__global__ void LB(64) k_adj_geom(Ctx C, double scale, const double* __restrict__ dt_dev,
                                  const double* __restrict__ P, const double* __restrict__ lamUe,
                                  double* __restrict__ lamPb) {
  adj_geom_at(C, scale, dt_dev, P, lamUe, lamPb, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// Opacity cotangents through the fluxes: per allocated cell, the faces that
// read its total opacity (as left cell of face c + e_d, right cell of face c);
// chi_abs and chi_es receive the same amount.  Gx_d: [2][Ntot] per direction.
__global__ void LB(256) k_adj_gather_chi(Ctx C, FaceRanges FR, const double* __restrict__ Gx1,
                                         const double* __restrict__ Gx2,
                                         const double* __restrict__ Gx3,
                                         double* __restrict__ gchi) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.Ntot) return;
  int idx[3];
  idx[0] = c % C.N[0];
  idx[1] = (c / C.N[0]) % C.N[1];
  idx[2] = c / ((long)C.N[0] * C.N[1]);
  double acc = 0.0;
  for (int d = 0; d < 3; d++) {
    if (C.n[d] == 1) continue;
    const double* Gx = (d == 0) ? Gx1 : ((d == 1) ? Gx2 : Gx3);
    const FaceRange& R = FR.r[d];
    bool trans = true;
    for (int e = 0; e < 3; e++)
      if (e != d && (idx[e] < R.lo[e] || idx[e] >= R.lo[e] + R.cnt[e])) trans = false;
    if (!trans) continue;
    const int up = idx[d] + 1;   // face c + e_d: c is its left cell
    if (up >= R.lo[d] && up < R.lo[d] + R.cnt[d]) acc += Gx[c + C.st[d]];
    if (idx[d] >= R.lo[d] && idx[d] < R.lo[d] + R.cnt[d]) acc += Gx[C.Ntot + c];
  }
  gchi[c] += acc;
  gchi[C.Ntot + c] += acc;
}

// ---------------------------------------------------------------------------
// The full cascade's entropy tracer U_S = sqrt(-g) S u^t of the gas
// primitives (rho0, u_g, u~^i; S = rho0 ln(p^n / rho0^(n+1))): lamP[q] +=
// b dU_S/dP_q lamS at interior cells, for a stage's b U_S(P_in) term and
// (b = 1, lamS the a-weighted sum over stages) for a U_S(P^n).  A cell
// whose tracer the forward left undefined (rho0 or u_g not positive) gets
// nothing.
// ---------------------------------------------------------------------------
DEV void adj_entropy_at(const Ctx& C, int i, int j, long c, const double* __restrict__ P,
                       double l, double* __restrict__ lamP) {
  typedef Dual<5> D5;
  D5 pd[5];
#pragma unroll
  for (int q = 0; q < 5; q++) pd[q] = D5::var(P[q * C.Ntot + c], q);
  if (!(pd[0].v > 0.0) || !(pd[1].v > 0.0)) return;
  Metric m;
  load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
  Vel<D5> v;
  make_vel(m, pd + 2, v);
  const double n = 1.0 / (C.gam - 1.0);
  const D5 S = pd[0] * (n * log((C.gam - 1.0) * pd[1]) - (n + 1.0) * log(pd[0]));
  const D5 U = m.gdet * S * v.ucon[0];
#pragma unroll
  for (int q = 0; q < 5; q++) lamP[q * C.Ntot + c] += l * U.d[q];
}

__global__ void LB(128) k_adj_entropy_field(Ctx C, double b, const double* __restrict__ P,
                                            const double* __restrict__ lamS,
                                            double* __restrict__ lamP) {
  int i, j, k;
  if (!interior_ijk(C, (long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
  const long c = cell_index(C, i, j, k);
  const double l = b * lamS[c];
  if (l != 0.0) adj_entropy_at(C, i, j, c, P, l, lamP);
}

// y += alpha x at interior cells, one field
__global__ void LB(256) k_adj_axpy1(Ctx C, double alpha, const double* __restrict__ x,
                                    double* __restrict__ y) {
  int i, j, k;
  if (!interior_ijk(C, (long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
  const long c = cell_index(C, i, j, k);
  y[c] += alpha * x[c];
}

// The IMEX tables' stored entropy source M_S = (U_S(P_out) - Se)/(g dt),
// zero where the solve failed: its cotangent lamMS handed to one side at
// the cells whose solve did not fail, side 0 lamP[q] += dU_S/dP_q lamMS /
// (g dt) (P_out, before the implicit solve's transpose), side 1 lamS -=
// lamMS / (g dt) (Se, after it).
__global__ void LB(128) k_adj_stage_ms(Ctx C, int side, double g, const double* __restrict__ dt_dev,
                                       const int* __restrict__ st, const double* __restrict__ P,
                                       const double* __restrict__ lamMS,
                                       double* __restrict__ lamP, double* __restrict__ lamS) {
  int i, j, k;
  if (!interior_ijk(C, (long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
  const long c = cell_index(C, i, j, k);
  if (st[c] & GRRMHD_ST_FAIL) return;
  const double l = lamMS[c] / (g * (*dt_dev));
  if (l == 0.0) return;
  if (side)
    lamS[c] -= l;
  else
    adj_entropy_at(C, i, j, c, P, l, lamP);
}

// y += m dt x at interior cells, one field (a bracket's dt m_k M_S^k term)
__global__ void LB(256) k_adj_axpy1_dt(Ctx C, double m, const double* __restrict__ dt_dev,
                                       const double* __restrict__ x, double* __restrict__ y) {
  int i, j, k;
  if (!interior_ijk(C, (long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
  const long c = cell_index(C, i, j, k);
  y[c] += m * (*dt_dev) * x[c];
}

// ---------------------------------------------------------------------------
// PPM flattener.  Forward, a sub-step's flux read fl_k = max(fl_{k-1}, f2_k)
// (fl_k = f2_k at the step's first flux evaluation), f2_k the flattener of
// the sub-step's own input.  Per allocated cell, direction and kind: the
// cotangent of fl_k (from the faces that read it, GF, plus what later
// sub-steps passed down in LamFl) goes to f2_k where f2_k was the larger
// (ties: the earlier value, the first argument) and stays in LamFl for the
// earlier sub-steps otherwise.  Lf2: the cotangent of f2_k, zero where f2_k
// has no derivative (both kinds zero at the first evaluation: the
// compression test failed or the ramp is clamped at zero).  prev: fl_{k-1},
// null at the first evaluation.  GF_d: [4][Ntot] per direction.
// ---------------------------------------------------------------------------
__global__ void LB(256) k_adj_flat_cot(Ctx C, FaceRanges FR, const double* __restrict__ GF,
                                       const double* __restrict__ fl,
                                       const double* __restrict__ prev,
                                       double* __restrict__ LamFl, double* __restrict__ Lf2) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.Ntot) return;
  int idx[3];
  idx[0] = c % C.N[0];
  idx[1] = (c / C.N[0]) % C.N[1];
  idx[2] = c / ((long)C.N[0] * C.N[1]);
  for (int d = 0; d < 3; d++) {
    const long xg = (long)(2 * d) * C.Ntot + c, xr = xg + C.Ntot;
    if (C.n[d] == 1) {
      Lf2[xg] = 0.0;
      Lf2[xr] = 0.0;
      continue;
    }
    const double* G = GF + (long)d * 4 * C.Ntot;
    const FaceRange& R = FR.r[d];
    double L[2] = {LamFl[xg], LamFl[xr]};
    bool trans = true;
    for (int e = 0; e < 3; e++)
      if (e != d && (idx[e] < R.lo[e] || idx[e] >= R.lo[e] + R.cnt[e])) trans = false;
    if (trans) {
      const int up = idx[d] + 1;   // face c + e_d: c is its left cell
      const bool left = up >= R.lo[d] && up < R.lo[d] + R.cnt[d];
      const bool right = idx[d] >= R.lo[d] && idx[d] < R.lo[d] + R.cnt[d];
#pragma unroll
      for (int kind = 0; kind < 2; kind++) {
        if (left) L[kind] += G[(long)kind * C.Ntot + c + C.st[d]];
        if (right) L[kind] += G[(long)(2 + kind) * C.Ntot + c];
      }
    }
    const long x[2] = {xg, xr};
    const bool flat0 = !prev && fl[xg] == 0.0 && fl[xr] == 0.0;
#pragma unroll
    for (int kind = 0; kind < 2; kind++) {
      const bool win = !prev || fl[x[kind]] > prev[x[kind]];
      Lf2[x[kind]] = (win && !flat0) ? L[kind] : 0.0;
      LamFl[x[kind]] = win ? 0.0 : L[kind];
    }
  }
}

// Transpose of f2: per allocated cell c, every flattener within three cells
// along a direction whose cotangent Lf2 is not zero, differentiated (one
// Dual<4> pass of the forward's flattener) with respect to c's u_g, Ebar,
// rho and total opacity; added to lamPb and (non-null) to both opacity
// cotangents gchi [2][Ntot].  mf: the mass fluxes of P (k_mass_flux) on a
// Kerr-Schild grid, null in flat space.
__global__ void LB(128) k_adj_flat(Ctx C, const double* __restrict__ P,
                                   const double* __restrict__ chi_abs,
                                   const double* __restrict__ chi_es,
                                   const double* __restrict__ mf,
                                   const double* __restrict__ Lf2, double* __restrict__ lamPb,
                                   double* __restrict__ gchi) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.Ntot) return;
  int idx[3];
  idx[0] = c % C.N[0];
  idx[1] = (c / C.N[0]) % C.N[1];
  idx[2] = c / ((long)C.N[0] * C.N[1]);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  bool any = false;
#pragma unroll 1
  for (int d = 0; d < 3; d++) {
    if (C.n[d] == 1) continue;
    bool trans = true;   // the flattener range: one cell beyond the interior
    for (int e = 0; e < 3; e++)
      if (e != d && C.n[e] > 1 && (idx[e] < C.ng[e] - 1 || idx[e] > C.ng[e] + C.n[e])) trans = false;
    if (!trans) continue;
#pragma unroll 1
    for (int m = -3; m <= 3; m++) {
      const int id = idx[d] - m;   // c is at offset m of cell cp
      if (id < C.ng[d] - 1 || id > C.ng[d] + C.n[d]) continue;
      const long cp = c - (long)m * C.st[d];
      const double Lg = Lf2[(long)(2 * d) * C.Ntot + cp], Lr = Lf2[(long)(2 * d + 1) * C.Ntot + cp];
      if (Lg == 0.0 && Lr == 0.0) continue;
      D4 sd[4];
      sd[0] = D4::var(P[C.Ntot + c], 0);
      sd[1] = D4::var(P[8 * C.Ntot + c], 1);
      sd[2] = D4::var(P[c], 2);
      sd[3] = D4::var(chi_abs[c] + chi_es[c], 3);
      D4 f2[2];
      flat_dir<D4>(C, P, chi_abs, chi_es, mf, cp, d, m, sd, f2);
#pragma unroll
      for (int a = 0; a < 4; a++) acc[a] += Lg * f2[0].d[a] + Lr * f2[1].d[a];
      any = true;
    }
  }
  if (!any) return;
  lamPb[C.Ntot + c] += acc[0];
  lamPb[8 * C.Ntot + c] += acc[1];
  lamPb[c] += acc[2];
  if (gchi) {
    gchi[c] += acc[3];
    gchi[C.Ntot + c] += acc[3];
  }
}

// ---------------------------------------------------------------------------
// Transpose of the ghost fill along d: each ghost's cotangent is added to its
// source cell (sign-flipped where the fill flips), then cleared.  One thread
// per (quantity, line along d) handles both ends of its line, so every cell
// a thread adds into or clears is its own (the polar shift maps lines one to
// one); the lower transverse axis runs fastest for coalesced access.
// ---------------------------------------------------------------------------
DEV void adj_bc_at(Ctx C, int d, double* lam, long t) {
  const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
  const int ng = C.ng[d], n = C.n[d];
  const long lines = (long)C.N[e1] * C.N[e2];
  if (t >= 12 * lines) return;
  const int q = (int)(t / lines);
  const long l = t - q * lines;
  const int a = (int)(l % C.N[e1]);
  const int b = (int)(l / C.N[e1]);
  double* L = lam + (long)q * C.Ntot;
  const bool odd = (q == 2 + d || q == 5 + d || q == 9 + d);   // components along d
  for (int side = 0; side < 2; side++) {
    const int bc = side ? C.bc_hi[d] : C.bc_lo[d];
    const bool flip = odd && (bc == GRRMHD_BC_REFLECT || bc == GRRMHD_BC_POLAR);
    for (int m = 0; m < ng; m++) {
      int cd[3], sd[3];
      cd[d] = side ? ng + n + m : ng - 1 - m;
      if (bc == GRRMHD_BC_OUTFLOW) sd[d] = side ? ng + n - 1 : ng;
      else if (bc == GRRMHD_BC_PERIODIC) sd[d] = side ? ng + m : ng + n - 1 - m;
      else sd[d] = side ? ng + n - 1 - m : ng + m;
      cd[e1] = sd[e1] = a;
      cd[e2] = sd[e2] = b;
      if (bc == GRRMHD_BC_POLAR && d == 1 && C.n[2] > 1) {
        const int g3 = C.ng[2], n3 = C.n[2];
        if (sd[2] < g3 || sd[2] >= g3 + n3) continue;   // filled by the x3 pass
        sd[2] = g3 + (sd[2] - g3 + n3 / 2) % n3;
      }
      const long dst = cell_index(C, cd[0], cd[1], cd[2]);
      const long src = cell_index(C, sd[0], sd[1], sd[2]);
      const double v = L[dst];
      L[src] += flip ? -v : v;
      L[dst] = 0.0;
    }
  }
}

__global__ void LB(256) k_adj_bc(Ctx C, int d, double* lam) {
  adj_bc_at(C, d, lam, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void LB(256) k_fill_d(double* p, long n, double v) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    p[t] = v;
}

// interior entries of src into dst, every other entry of dst cleared
// ---------------------------------------------------------------------------
// Pieces of the IMEX adjoint (stage tables with stored sources M^k).
// ---------------------------------------------------------------------------

// y += alpha x, 12 fields at interior cells
__global__ void LB(256) k_adj_axpy12(Ctx C, double alpha, const double* __restrict__ x,
                                     double* __restrict__ y) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int i, j, k;
  interior_cell(C, t, i, j, k);
  const long c = cell_index(C, i, j, k);
#pragma unroll
  for (int q = 0; q < 12; q++) y[q * C.Ntot + c] += alpha * x[q * C.Ntot + c];
}

// the stored source's rows r = 0..7 are the U slots 1-4 and 8-11
DEV int mslot(int r) { return (r < 4) ? 1 + r : 4 + r; }

// a bracket's dt m_k M^k term: lamM += dt m lamUe (rows of the 8 slots)
__global__ void LB(256) k_adj_mterm(Ctx C, double m, const double* __restrict__ dt_dev,
                                    const double* __restrict__ lamUe, double* __restrict__ lamM) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int i, j, k;
  interior_cell(C, t, i, j, k);
  const long c = cell_index(C, i, j, k);
  const double f = m * (*dt_dev);
#pragma unroll
  for (int r = 0; r < 8; r++) lamM[r * C.Ntot + c] += f * lamUe[mslot(r) * C.Ntot + c];
}

// M = (U_out - U_e)/(g dt) at cells whose solve did not fail: its transpose
// spread into one side, tgt[slot] += scale/dt lamM (scale = 1/g for U_out,
// -1/g for U_e)
__global__ void LB(256) k_adj_mscatter(Ctx C, double scale, const double* __restrict__ dt_dev,
                                       const int* __restrict__ st, const double* __restrict__ lamM,
                                       double* __restrict__ tgt) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int i, j, k;
  interior_cell(C, t, i, j, k);
  const long c = cell_index(C, i, j, k);
  if (st[c] & GRRMHD_ST_FAIL) return;
  const double f = scale / (*dt_dev);
#pragma unroll
  for (int r = 0; r < 8; r++) tgt[mslot(r) * C.Ntot + c] += f * lamM[r * C.Ntot + c];
}

// x = A^-T b for a small dense A, Gaussian elimination with partial
// pivoting on A^T; rows are swapped by selects so every index is static.
// Returns 1 if a pivot vanishes.
template <int N>
DEV int solve_t(const double A[N][N], const double b[N], double x[N]) {
  double M[N][N + 1];
#pragma unroll
  for (int r = 0; r < N; r++) {
#pragma unroll
    for (int c = 0; c < N; c++) M[r][c] = A[c][r];
    M[r][N] = b[r];
  }
#pragma unroll
  for (int k = 0; k < N; k++) {
    double best = ::fabs(M[k][k]);
    int piv = k;
#pragma unroll
    for (int r = k + 1; r < N; r++) {
      const double v = ::fabs(M[r][k]);
      if (v > best) { best = v; piv = r; }
    }
    if (!(best > 0.0) || !isfinite(best)) return 1;
#pragma unroll
    for (int r = k + 1; r < N; r++) {
      const bool sw = (r == piv);
#pragma unroll
      for (int c = k; c <= N; c++) {
        const double a = M[k][c], bb = M[r][c];
        M[k][c] = sw ? bb : a;
        M[r][c] = sw ? a : bb;
      }
    }
    const double ip = 1.0 / M[k][k];
#pragma unroll
    for (int r = k + 1; r < N; r++) {
      const double f = M[r][k] * ip;
#pragma unroll
      for (int c = k; c <= N; c++) M[r][c] -= f * M[k][c];
    }
  }
#pragma unroll
  for (int r = N - 1; r >= 0; r--) {
    double v = M[r][N];
#pragma unroll
    for (int c = r + 1; c < N; c++) v -= M[r][c] * x[c];
    x[r] = v / M[r][r];
  }
#pragma unroll
  for (int r = 0; r < N; r++)
    if (!isfinite(x[r])) return 1;
  return 0;
}

// Transpose of the final inversion P = C2P(U_e) of an IMEX step (the MHD
// inversion, B = U_B/sqrt(-g), the radiation inversion with the BASIC
// limiter) at its result P: lamUe += (dP/dU_e)^T lamP.  The MHD block by the
// implicit-function theorem (P_mhd inverts the 8x8 map U_mhd(P_mhd), so its
// Jacobian is that map's inverse); the radiation block through the limited
// inversion itself.  Where the MHD inversion failed the cell's P_mhd was the
// guess: its cotangent goes to lamPg instead.
DEV void adj_c2p_at(Ctx C, const double* __restrict__ Ue, const double* __restrict__ P,
                    const int* __restrict__ st, const double* __restrict__ lamP,
                    double* __restrict__ lamUe, double* __restrict__ lamPg, long t) {
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return;
  int i, j, k;
  interior_cell(C, t, i, j, k);
  const long c = cell_index(C, i, j, k);
  Metric m;
  load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
  const double igd = 1.0 / m.gdet;
  double lp[12], lu[12];
#pragma unroll
  for (int q = 0; q < 12; q++) {
    lp[q] = lamP[q * C.Ntot + c];
    lu[q] = 0.0;
  }
  {
    D4 ur[4], Eb, utr[3];
#pragma unroll
    for (int b = 0; b < 4; b++) ur[b] = D4::var(Ue[(8 + b) * C.Ntot + c] * igd, b);
    rad_invert(m, C.gamma_max, C.ymax, 0, ur, Eb, utr);
    const D4 pr[4] = {Eb, utr[0], utr[1], utr[2]};
#pragma unroll
    for (int b = 0; b < 4; b++) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 4; a++) s += lp[8 + a] * pr[a].d[b];
      lu[8 + b] = s * igd;
    }
  }
  if (st[c] & GRRMHD_ST_C2P_FAIL) {
#pragma unroll
    for (int q = 0; q < 5; q++) lamPg[q * C.Ntot + c] += lp[q];
#pragma unroll
    for (int q = 5; q < 8; q++) lu[q] = lp[q] * igd;
  } else {
    double p[12], J[8][8];
#pragma unroll
    for (int q = 0; q < 12; q++) p[q] = P[q * C.Ntot + c];
#pragma unroll 1
    for (int pass = 0; pass < 2; pass++) {
      D4 pd[12], ud[12];
      seed4<12>(p, 4 * pass, pd);
      prim_to_cons_cell(m, C.gam, pd, ud);
#pragma unroll
      for (int a = 0; a < 8; a++)
#pragma unroll
        for (int jj = 0; jj < 4; jj++) {
          const double v = ud[a].d[jj];
#pragma unroll
          for (int b = 0; b < 8; b++)
            if (b == 4 * pass + jj) J[a][b] = v;
        }
    }
    double b8[8], x8[8];
#pragma unroll
    for (int q = 0; q < 8; q++) b8[q] = lp[q];
    if (solve_t<8>(J, b8, x8) == 0) {
#pragma unroll
      for (int q = 0; q < 8; q++) lu[q] = x8[q];
    }
  }
#pragma unroll
  for (int q = 0; q < 12; q++) lamUe[q * C.Ntot + c] += lu[q];
}

__global__ void LB(64) k_adj_c2p(Ctx C, const double* __restrict__ Ue, const double* __restrict__ P,
                                 const int* __restrict__ st, const double* __restrict__ lamP,
                                 double* __restrict__ lamUe, double* __restrict__ lamPg) {
  adj_c2p_at(C, Ue, P, st, lamP, lamUe, lamPg, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

DEV void copy_interior_at(Ctx C, const double* __restrict__ src, double* __restrict__ dst, long c) {
  if (c >= C.Ntot) return;
  const int i = c % C.N[0];
  const int j = (c / C.N[0]) % C.N[1];
  const int k = c / ((long)C.N[0] * C.N[1]);
  const bool in = i >= C.ng[0] && i < C.ng[0] + C.n[0] && j >= C.ng[1] && j < C.ng[1] + C.n[1] &&
                  k >= C.ng[2] && k < C.ng[2] + C.n[2];
#pragma unroll
  for (int q = 0; q < 12; q++) dst[q * C.Ntot + c] = in ? src[q * C.Ntot + c] : 0.0;
}

__global__ void LB(256) k_copy_interior(Ctx C, const double* __restrict__ src, double* __restrict__ dst) {
  copy_interior_at(C, src, dst, (long)blockIdx.x * blockDim.x + threadIdx.x);
}
