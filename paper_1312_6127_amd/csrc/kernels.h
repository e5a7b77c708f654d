// HIP kernels of one GRRMHD Runge-Kutta sub-step (Sec. 4.2 steps 1-13).
// All state arrays are field-major SoA over the allocated grid; consecutive
// threads take consecutive i (x1) so every field access is coalesced.
#pragma once
#include "implicit.h"

#define LB(n) __launch_bounds__(n)
#ifndef GRRMHD_FLUX_LB
#define GRRMHD_FLUX_LB __launch_bounds__(128)
#endif

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b to XCD b mod 8)
// and each XCD has its own L2.  This maps b to a work index so that each XCD
// works through one contiguous eighth of the work: neighbouring tiles, which
// share cache lines and stencil rows, then meet in the same L2.  A bijection
// on [0, G): the last G mod 8 workgroups keep their own index.
DEV long xcd_block(long b, long G) {
  const long full = (G / 8) * 8;
  if (b >= full) return b;
  return (b % 8) * (G / 8) + b / 8;
}

#ifndef GRRMHD_IMP_WAVES
#define GRRMHD_IMP_WAVES 1   // minimum waves per SIMD asked of the implicit kernels
#endif
#define LBI __launch_bounds__(64, GRRMHD_IMP_WAVES)

DEV long cell_index(const Ctx& C, int i, int j, int k) { return i + C.st[1] * j + C.st[2] * k; }

// ---------------------------------------------------------------------------
// geometry (Sec. 2): metric and its x1/x2 derivatives via Dual<2>
// ---------------------------------------------------------------------------
template <class T>
DEV void ks_metric_lower(double a, double R0, const T& x1, const T& x2, T g[10]) {
  const T er = exp(x1);
  const T r = R0 + er;
  const T th = M_PI * x2;
  const T s = sin(th), c = cos(th);
  const T s2 = s * s;
  const T Sig = r * r + (a * a) * (c * c);
  const T z = 2.0 * r / Sig;
  // KS components in (t, r, theta, phi) times the map Jacobian (1, er, pi, 2 pi)
  g[sym(0, 0)] = z - 1.0;
  g[sym(0, 1)] = z * er;
  g[sym(0, 2)] = T(0.0);
  g[sym(0, 3)] = -(a * 2.0 * M_PI) * z * s2;
  g[sym(1, 1)] = (1.0 + z) * er * er;
  g[sym(1, 2)] = T(0.0);
  g[sym(1, 3)] = -(a * 2.0 * M_PI) * (1.0 + z) * s2 * er;
  g[sym(2, 2)] = (M_PI * M_PI) * Sig;
  g[sym(2, 3)] = T(0.0);
  g[sym(3, 3)] = (4.0 * M_PI * M_PI) * s2 * (Sig + (a * a) * (1.0 + z) * s2);
}

DEV void geometry_at(Ctx C, double a, double R0, double* gc, double* gf1, double* gf2, int pos) {
  if (pos >= C.npos) return;
  const int i = pos % C.N[0], j = pos / C.N[0];
  for (int loc = 0; loc < 3; loc++) {
    double* tab = loc == 0 ? gc : (loc == 1 ? gf1 : gf2);
    const double x1 = C.xlo[0] + (i - C.ng[0] + (loc == 1 ? 0.0 : 0.5)) * C.dx[0];
    const double x2 = C.xlo[1] + (j - C.ng[1] + (loc == 2 ? 0.0 : 0.5)) * C.dx[1];
    double gl[10], gu[10], d1[10], d2[10], gdet, alpha;
    if (C.metric == GRRMHD_MINKOWSKI) {
      for (int q = 0; q < 10; q++) gl[q] = gu[q] = d1[q] = d2[q] = 0.0;
      gl[0] = gu[0] = -1.0;
      gl[4] = gu[4] = gl[7] = gu[7] = gl[9] = gu[9] = 1.0;
      gdet = alpha = 1.0;
    } else {
      Dual<2> g[10];
      ks_metric_lower(a, R0, Dual<2>::var(x1, 0), Dual<2>::var(x2, 1), g);
      for (int q = 0; q < 10; q++) {
        gl[q] = g[q].v;
        d1[q] = g[q].d[0];
        d2[q] = g[q].d[1];
      }
      const double er = ::exp(x1), r = R0 + er, th = M_PI * x2;
      const double s = ::sin(th), c = ::cos(th);
      const double Sig = r * r + a * a * c * c, Del = r * r - 2.0 * r + a * a;
      const double z = 2.0 * r / Sig;
      const double J[4] = {1.0, er, M_PI, 2.0 * M_PI};
      for (int q = 0; q < 10; q++) gu[q] = 0.0;
      gu[sym(0, 0)] = -(1.0 + z);
      gu[sym(0, 1)] = z / J[1];
      gu[sym(1, 1)] = Del / Sig / (J[1] * J[1]);
      gu[sym(1, 3)] = a / Sig / (J[1] * J[3]);
      gu[sym(2, 2)] = 1.0 / Sig / (J[2] * J[2]);
      // g^{phi phi} diverges on the axis (only face tables touch it, and
      // nothing there reads it)
      gu[sym(3, 3)] = (s != 0.0) ? 1.0 / (Sig * s * s) / (J[3] * J[3]) : 0.0;
      gdet = Sig * ::fabs(s) * J[1] * J[2] * J[3];
      alpha = 1.0 / ::sqrt(1.0 + z);
    }
    for (int q = 0; q < 10; q++) {
      tab[(GE_GCOV + q) * C.npos + pos] = gl[q];
      tab[(GE_GCON + q) * C.npos + pos] = gu[q];
    }
    tab[GE_GDET * C.npos + pos] = gdet;
    tab[GE_ALPHA * C.npos + pos] = alpha;
    if (loc == 0)
      for (int q = 0; q < 10; q++) {
        tab[(GE_DG1 + q) * C.npos + pos] = d1[q];
        tab[(GE_DG2 + q) * C.npos + pos] = d2[q];
      }
  }
}

__global__ void LB(256) k_geometry(Ctx C, double a, double R0, double* gc, double* gf1,
                                   double* gf2) {
  geometry_at(C, a, R0, gc, gf1, gf2, blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// step 1: ghost cells
// ---------------------------------------------------------------------------
// All ghost cells in one pass: the fill dimension by dimension (x1, then x2,
// then x3, each pass copying whole planes including earlier ghosts) composed
// into one source cell and sign per ghost cell.  Applying the maps from the
// last dimension back to the first gives the cell whose interior value the
// three passes carry into the ghost.
DEV void bc_all_at(Ctx C, double* P, long c) {
  if (c >= C.Ntot) return;
  int idx[3];
  idx[0] = c % C.N[0];
  idx[1] = (c / C.N[0]) % C.N[1];
  idx[2] = c / ((long)C.N[0] * C.N[1]);
  int sd[3] = {idx[0], idx[1], idx[2]};
  int flip = 0;
  bool ghost = false;
  for (int d = 2; d >= 0; d--) {
    const int ng = C.ng[d], n = C.n[d];
    if (ng == 0 || (sd[d] >= ng && sd[d] < ng + n)) continue;
    ghost = true;
    const int side = sd[d] >= ng + n;
    const int m = side ? sd[d] - ng - n : ng - 1 - sd[d];
    const int bc = side ? C.bc_hi[d] : C.bc_lo[d];
    if (bc == GRRMHD_BC_OUTFLOW) sd[d] = side ? ng + n - 1 : ng;
    else if (bc == GRRMHD_BC_PERIODIC) sd[d] = side ? ng + m : ng + n - 1 - m;
    else sd[d] = side ? ng + n - 1 - m : ng + m;
    if (bc == GRRMHD_BC_REFLECT || bc == GRRMHD_BC_POLAR) flip ^= 1 << d;
    if (bc == GRRMHD_BC_POLAR && d == 1 && C.n[2] > 1)   // across the axis: phi + pi
      sd[2] = C.ng[2] + (sd[2] - C.ng[2] + C.n[2] / 2) % C.n[2];
  }
  if (!ghost) return;
  const long src = cell_index(C, sd[0], sd[1], sd[2]);
#pragma unroll
  for (int q = 0; q < 12; q++) {
    double v = P[q * C.Ntot + src];
    const int dq = (q >= 2 && q <= 4) ? q - 2 : ((q >= 5 && q <= 7) ? q - 5 : ((q >= 9) ? q - 9 : -1));
    if (dq >= 0 && (flip >> dq & 1)) v = -v;
    P[q * C.Ntot + c] = v;
  }
}

__global__ void LB(256) k_bc_all(Ctx C, double* P) {
  bc_all_at(C, P, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// steps 2-3 helper and P -> U kernel
// ---------------------------------------------------------------------------
template <class T>
DEV void prim_to_cons_cell(const Metric& m, double gam, const T* P, T* U) {
  Gas<T> s;
  make_gas(m, gam, P[0], P[1], P + 2, P + 5, s);
  T row[8];
  gas_row(s, P + 5, 0, row);
  Vel<T> r;
  make_vel(m, P + 9, r);
  T rr[4];
  rad_row(r, P[8], 0, rr);
#pragma unroll
  for (int q = 0; q < 8; q++) U[q] = m.gdet * row[q];
#pragma unroll
  for (int q = 0; q < 4; q++) U[8 + q] = m.gdet * rr[q];
}

DEV void p2u_at(Ctx C, const double* __restrict__ P, double* __restrict__ U, long c) {
  if (c >= C.Ntot) return;
  const int pos = c % C.npos;
  Metric m;
  load_metric(C.geo_c, C.npos, pos, m);
  double p[12], u[12];
#pragma unroll
  for (int q = 0; q < 12; q++) p[q] = P[q * C.Ntot + c];
  prim_to_cons_cell(m, C.gam, p, u);
#pragma unroll
  for (int q = 0; q < 12; q++) U[q * C.Ntot + c] = u[q];
}

__global__ void LB(256) k_p2u(Ctx C, const double* __restrict__ P, double* __restrict__ U) {
  p2u_at(C, P, U, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// steps 4-7: reconstruction, face physics, wave speeds, HLL / LAXF
// ---------------------------------------------------------------------------
template <class T>
DEV T mc_slope(T dl, T dr) {
  using R = typename RealOf<T>::type;
  if (val(dl) * val(dr) <= R(0.0)) return T(R(0.0));
  const T dc = R(0.5) * (dl + dr);
  return copysign(fmin(fabs(dc), R(2.0) * fmin(fabs(dl), fabs(dr))), dc);
}

// PPM (Colella & Woodward 1984, no contact steepening): interface value
// between the 2nd and 3rd of four cells, the mean less the difference of
// their MC slopes over 6
template <class T>
DEV T ppm_iface(T am, T a0, T a1, T a2) {
  using R = typename RealOf<T>::type;
  return R(0.5) * (a0 + a1) - (mc_slope(a1 - a0, a2 - a1) - mc_slope(a0 - am, a1 - a0)) / R(6.0);
}

// left and right values of the middle of five cells: interface values
// flattened towards the cell value by f, then the monotonicity constraints
template <class T>
DEV void ppm_cell(const T* a, T f, T& aL, T& aR) {
  using R = typename RealOf<T>::type;
  const T a0 = a[2];
  T l = ppm_iface(a[0], a[1], a[2], a[3]);
  T r = ppm_iface(a[1], a[2], a[3], a[4]);
  l = f * a0 + (R(1.0) - f) * l;
  r = f * a0 + (R(1.0) - f) * r;
  if (val((r - a0) * (a0 - l)) <= R(0.0)) {
    l = a0;
    r = a0;
  } else {
    const T d = r - l, m6 = R(6.0) * (a0 - R(0.5) * (l + r));
    if (d * m6 > d * d) l = R(3.0) * a0 - R(2.0) * r;
    else if (-(d * d) > d * m6) r = R(3.0) * a0 - R(2.0) * l;
  }
  aL = l;
  aR = r;
}

template <class T>
struct FaceState {
  T U[12], F[12];
  T gm, gp, rm, rp;   // gas and radiation characteristic speeds
};

// Characteristic speeds along d of one face state: gas (gm, gp) and
// radiation (rm, rp).
template <class T>
DEV void face_speeds(const Ctx& C, const MetricT<typename RealOf<T>::type>& m, int d, const T* P,
                     T chi_tot, const Gas<T>& s, const Vel<T>& r, T& gm, T& gp, T& rm, T& rp) {
  using R = typename RealOf<T>::type;
  // gas: fast magnetosonic speed c_ms^2 = v_A^2 + c_s^2 (1 - v_A^2)
  const T w = s.rho + s.ug + s.pg;
  const T cs2 = R(C.gam) * s.pg / w;
  const T va2 = s.bsq / (w + s.bsq);
  char_speeds(m, s.v.ucon, va2 + cs2 * (R(1.0) - va2), d, gm, gp);
  // radiation: 1/sqrt(3) in the radiation frame, limited to 4/(3 tau) in the gas frame
  char_speeds(m, r.ucon, T(R(1.0 / 3.0)), d, rm, rp);
  const T tau = chi_tot * P[0] * sqrt(m.lo(d, d)) * R(C.dx[d - 1]);
  if (val(tau) > R(0.0)) {
    const T cl = R(4.0) / (R(3.0) * tau);
    if (val(cl) < R(1.0)) {
      T lm, lp;
      char_speeds(m, s.v.ucon, cl * cl, d, lm, lp);
      rp = fmin(rp, lp);
      rm = fmax(rm, lm);
    }
  }
}

// T = double, float on the FP32 face path (metric rounded to float too), or
// Dual<N> for the adjoint
template <class T>
DEV void face_state(const Ctx& C, const MetricT<typename RealOf<T>::type>& m, int d, const T* P,
                    T chi_tot, FaceState<T>& fs) {
  Gas<T> s;
  make_gas(m, C.gam, P[0], P[1], P + 2, P + 5, s);
  T row[8];
  gas_row(s, P + 5, 0, row);
#pragma unroll
  for (int q = 0; q < 8; q++) fs.U[q] = m.gdet * row[q];
  gas_row(s, P + 5, d, row);
#pragma unroll
  for (int q = 0; q < 8; q++) fs.F[q] = m.gdet * row[q];
  Vel<T> r;
  make_vel(m, P + 9, r);
  T rr[4];
  rad_row(r, P[8], 0, rr);
#pragma unroll
  for (int q = 0; q < 4; q++) fs.U[8 + q] = m.gdet * rr[q];
  rad_row(r, P[8], d, rr);
#pragma unroll
  for (int q = 0; q < 4; q++) fs.F[8 + q] = m.gdet * rr[q];
  face_speeds(C, m, d, P, chi_tot, s, r, fs.gm, fs.gp, fs.rm, fs.rp);
}

struct FaceRange {
  int lo[3], cnt[3];
  long total;
};

// Faces normal to D in range R: reconstruction, face states, HLL / LAXF, in
// arithmetic T (double; float for the FP32-mixed path); fluxes and speeds are
// stored as double.
// fl: the PPM flattener [3][gas, radiation][Ntot] (unused for MC)
// sqrt(-g) S u^t and sqrt(-g) S u^D of the entropy tracer at a face state
// (S = rho0 ln(p^n / rho0^(n+1)), n = 1/(gam - 1); Sec. 4 lists of U_q, F_q)
template <int D, class T>
DEV void entropy_face(const Ctx& C, const MetricT<T>& m, const T* P, T& Us, T& Fs) {
  Vel<T> v;
  make_vel(m, P + 2, v);
  const T n = T(1.0 / (C.gam - 1.0));
  const T pg = T(C.gam - 1.0) * P[1];
  const T S = P[0] * (n * log(pg) - (n + T(1.0)) * log(P[0]));
  Us = m.gdet * S * v.ucon[0];
  Fs = m.gdet * S * v.ucon[D];
}

// STAG (staggered face field Bf [3][Ntot], sqrt(-g) B^d on the lower d-face
// of each cell): both states take the face's own normal field, and the face
// velocities v^m = u^m/u^t of each state and the gas v_min, v_max of eq. hll
// go to VF [(2 (D-1) + side) 3 + m][Ntot] and SP [2 (D-1) + {0, 1}][Ntot]
// for the corner EMFs.
// Steps 5-7 at one face from its reconstructed left and right primitives
// (the face's own normal field replaced with the staggered field's): face
// states, wave speeds, HLL / LAXF, the stores.  Shared by flux_at (stencil
// from global memory) and the LDS-staged flux kernel.
template <int D, class T, bool ENTF = false, bool STAG = false>
DEV void flux_states(const Ctx& C, int i, int j, long c, long st, T PL[12], T PR[12],
                     const double* __restrict__ chi_abs, const double* __restrict__ chi_es,
                     double* __restrict__ F, double* __restrict__ vchar,
                     double* __restrict__ Fs = nullptr, const double* __restrict__ Bf = nullptr,
                     double* __restrict__ VF = nullptr, double* __restrict__ SP = nullptr) {
  MetricT<T> m;
  const double* tab = (D == 1) ? C.geo_f1 : ((D == 2) ? C.geo_f2 : C.geo_c);
  load_metric(tab, C.npos, i + C.N[0] * j, m);
  if constexpr (STAG) {
    // the face's own normal field (zero where sqrt(-g) vanishes, the axis)
    const double gd = tab[GE_GDET * C.npos + i + C.N[0] * j];
    const T bn = (T)(gd > 0.0 ? Bf[(long)(D - 1) * C.Ntot + c] / gd : 0.0);
    PL[4 + D] = bn;
    PR[4 + D] = bn;
  }
  FaceState<T> L, Rs;
  face_state(C, m, D, PL, (T)(chi_abs[c - st] + chi_es[c - st]), L);
  face_state(C, m, D, PR, (T)(chi_abs[c] + chi_es[c]), Rs);
  // eq. hll: v_min = -min(0, v-_L, v-_R), v_max = max(0, v+_L, v+_R)
  const T zero = T(0.0);
  const T gmin = -fmin(zero, fmin(L.gm, Rs.gm)), gmax = fmax(zero, fmax(L.gp, Rs.gp));
  const T rmin = -fmin(zero, fmin(L.rm, Rs.rm)), rmax = fmax(zero, fmax(L.rp, Rs.rp));
#pragma unroll
  for (int q = 0; q < 12; q++) {
    const T vmin = q < 8 ? gmin : rmin, vmax = q < 8 ? gmax : rmax;
    T f;
    if (C.flux == GRRMHD_FLUX_HLL) {
      const T den = vmin + vmax;
      f = (den > zero) ? (vmin * Rs.F[q] + vmax * L.F[q] - vmin * vmax * (Rs.U[q] - L.U[q])) / den
                       : T(0.5) * (L.F[q] + Rs.F[q]);
    } else {
      f = T(0.5) * (Rs.F[q] + L.F[q] - fmax(vmin, vmax) * (Rs.U[q] - L.U[q]));
    }
    if (q == 4 + D) f = zero;   // normal field component has no induction flux
    F[q * C.Ntot + c] = (double)f;
  }
  vchar[c] = (double)fmax(fmax(gmin, gmax), fmax(rmin, rmax));
  if constexpr (STAG) {
#pragma unroll
    for (int sd = 0; sd < 2; sd++) {
      Vel<T> v;
      make_vel(m, (sd ? PR : PL) + 2, v);
#pragma unroll
      for (int q = 0; q < 3; q++)
        VF[((long)((2 * (D - 1) + sd) * 3) + q) * C.Ntot + c] = (double)(v.ucon[q + 1] / v.ucon[0]);
    }
    SP[(long)(2 * (D - 1)) * C.Ntot + c] = (double)gmin;
    SP[(long)(2 * (D - 1) + 1) * C.Ntot + c] = (double)gmax;
  }
  if constexpr (ENTF) {
    // the entropy tracer's flux, with the gas speeds
    T UsL, FsL, UsR, FsR, f;
    entropy_face<D, T>(C, m, PL, UsL, FsL);
    entropy_face<D, T>(C, m, PR, UsR, FsR);
    if (C.flux == GRRMHD_FLUX_HLL) {
      const T den = gmin + gmax;
      f = (den > zero) ? (gmin * FsR + gmax * FsL - gmin * gmax * (UsR - UsL)) / den
                       : T(0.5) * (FsL + FsR);
    } else {
      f = T(0.5) * (FsR + FsL - fmax(gmin, gmax) * (UsR - UsL));
    }
    Fs[c] = (double)f;
  }
}

// The face velocity states alone (the staggered field's outer faces): u~^1..3
// reconstructed exactly as in flux_at, v^m = u^m/u^t from the face metric.
template <int D, class T>
DEV void stag_face_velocities(const Ctx& C, const double* __restrict__ P,
                              const double* __restrict__ fl, int i, int j, long c, long st,
                              double* __restrict__ VF) {
  T uL[3], uR[3];
  if (C.recon == GRRMHD_RECON_PPM) {
    const double* fg = fl + (long)(2 * (D - 1)) * C.Ntot;
    const T fgL = (T)fg[c - st], fgR = (T)fg[c];
    const bool wgt = (D == 1) && C.metric == GRRMHD_KERR_SCHILD;
    double gc[6] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0}, gface = 1.0;
    if (wgt) {
#pragma unroll
      for (int m = 0; m < 6; m++) gc[m] = C.geo_c[GE_GDET * C.npos + (i + m - 3) + C.N[0] * j];
      gface = C.geo_f1[GE_GDET * C.npos + i + C.N[0] * j];
    }
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const double* p = P + (2 + q) * C.Ntot;
      T a[6];
#pragma unroll
      for (int m = 0; m < 6; m++) a[m] = (T)(wgt ? p[c + (m - 3) * st] * gc[m] : p[c + (m - 3) * st]);
      T l, r;
      ppm_cell(a, fgL, l, uL[q]);
      ppm_cell(a + 1, fgR, uR[q], r);
      if (wgt) {
        uL[q] = uL[q] / (T)gface;
        uR[q] = uR[q] / (T)gface;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const double* p = P + (2 + q) * C.Ntot;
      const T a = (T)p[c - 2 * st], b = (T)p[c - st], e = (T)p[c], f = (T)p[c + st];
      uL[q] = b + T(0.5) * mc_slope(b - a, e - b);
      uR[q] = e - T(0.5) * mc_slope(e - b, f - e);
    }
  }
  MetricT<T> m;
  const double* tab = (D == 1) ? C.geo_f1 : ((D == 2) ? C.geo_f2 : C.geo_c);
  load_metric(tab, C.npos, i + C.N[0] * j, m);
#pragma unroll
  for (int sd = 0; sd < 2; sd++) {
    Vel<T> v;
    make_vel(m, sd ? uR : uL, v);
#pragma unroll
    for (int q = 0; q < 3; q++)
      VF[((long)((2 * (D - 1) + sd) * 3) + q) * C.Ntot + c] = (double)(v.ucon[q + 1] / v.ucon[0]);
  }
}

template <int D, class T, bool ENTF = false, bool STAG = false>
DEV void flux_at(Ctx C, FaceRange R, const double* __restrict__ P,
                               const double* __restrict__ chi_abs,
                               const double* __restrict__ chi_es, double* __restrict__ F,
                               double* __restrict__ vchar, const double* __restrict__ fl, long t,
                               double* __restrict__ Fs = nullptr,
                               const double* __restrict__ Bf = nullptr,
                               double* __restrict__ VF = nullptr, double* __restrict__ SP = nullptr) {
  if (t >= R.total) return;
  const int i = R.lo[0] + t % R.cnt[0];
  const long t2 = t / R.cnt[0];
  const int j = R.lo[1] + t2 % R.cnt[1];
  const int k = R.lo[2] + t2 / R.cnt[1];
  const long c = cell_index(C, i, j, k);
  const long st = C.st[D - 1];
  if constexpr (STAG) {
    // faces two cells beyond the interior across D feed only the corner
    // interpolation of the velocities: reconstruct u~ and store v there
    const int idx[3] = {i, j, k};
    bool outer = false;
#pragma unroll
    for (int e = 0; e < 3; e++)
      if (e != D - 1 && C.n[e] > 1 && (idx[e] < C.ng[e] - 1 || idx[e] > C.ng[e] + C.n[e]))
        outer = true;
    if (outer) {
      stag_face_velocities<D, T>(C, P, fl, i, j, c, st, VF);
      return;
    }
  }
  T PL[12], PR[12];
  if (C.recon == GRRMHD_RECON_PPM) {
    // left state: right value of cell c - st; right state: left value of c
    const double* fg = fl + (long)(2 * (D - 1)) * C.Ntot;
    const double* fr = fg + C.Ntot;
    const T fgL = (T)fg[c - st], frL = (T)fr[c - st], fgR = (T)fg[c], frR = (T)fr[c];
    // Kerr-Schild, along r: the vector primitives interpolated as sqrt(-g)
    // times the value (Sec. 4.3); along phi sqrt(-g) is constant and the
    // weighting the identity
    const bool wgt = (D == 1) && C.metric == GRRMHD_KERR_SCHILD;
    double gc[6] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0}, gface = 1.0;
    if (wgt) {
#pragma unroll
      for (int m = 0; m < 6; m++) gc[m] = C.geo_c[GE_GDET * C.npos + (i + m - 3) + C.N[0] * j];
      gface = C.geo_f1[GE_GDET * C.npos + i + C.N[0] * j];
    }
#pragma unroll
    for (int q = 0; q < 12; q++) {
      const double* p = P + q * C.Ntot;
      const bool vec = wgt && ((q >= 2 && q <= 7) || q >= 9);
      T a[6];
#pragma unroll
      for (int m = 0; m < 6; m++) a[m] = (T)(vec ? p[c + (m - 3) * st] * gc[m] : p[c + (m - 3) * st]);
      T l, r;
      ppm_cell(a, q < 8 ? fgL : frL, l, PL[q]);
      ppm_cell(a + 1, q < 8 ? fgR : frR, PR[q], r);
      if (vec) {
        PL[q] = PL[q] / (T)gface;
        PR[q] = PR[q] / (T)gface;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 12; q++) {
      const double* p = P + q * C.Ntot;
      const T a = (T)p[c - 2 * st], b = (T)p[c - st], e = (T)p[c], f = (T)p[c + st];
      PL[q] = b + T(0.5) * mc_slope(b - a, e - b);
      PR[q] = e - T(0.5) * mc_slope(e - b, f - e);
    }
  }
  flux_states<D, T, ENTF, STAG>(C, i, j, c, st, PL, PR, chi_abs, chi_es, F, vchar, Fs, Bf, VF, SP);
}


// The faces of all directions in one launch: up to three segments (one per
// direction) laid end to end over the thread index; consecutive threads stay
// within one direction except at the two segment boundaries.
struct FluxSegs {
  FaceRange R[3];
  long start[3];
  int D[3];
  int n;
  long total;
};

template <class T, bool ENTF = false, bool STAG = false>
DEV void flux_all_at(Ctx C, const FluxSegs& S, const double* __restrict__ P,
                     const double* __restrict__ chi_abs, const double* __restrict__ chi_es,
                     double* __restrict__ F, double* __restrict__ vchar,
                     const double* __restrict__ fl, long t, double* __restrict__ Fs = nullptr,
                     const double* __restrict__ Bf = nullptr, double* __restrict__ VF = nullptr,
                     double* __restrict__ SP = nullptr) {
  if (t >= S.total) return;
  int k = 0;
  if (S.n > 1 && t >= S.start[1]) k = 1;
  if (S.n > 2 && t >= S.start[2]) k = 2;
  const long u = t - S.start[k];
  const int D = S.D[k];
  double* Fd = F + (long)(D - 1) * 12 * C.Ntot;
  double* vd = vchar + (long)(D - 1) * C.Ntot;
  double* Fsd = ENTF ? Fs + (long)(D - 1) * C.Ntot : nullptr;
  if (D == 1) flux_at<1, T, ENTF, STAG>(C, S.R[k], P, chi_abs, chi_es, Fd, vd, fl, u, Fsd, Bf, VF, SP);
  else if (D == 2) flux_at<2, T, ENTF, STAG>(C, S.R[k], P, chi_abs, chi_es, Fd, vd, fl, u, Fsd, Bf, VF, SP);
  else flux_at<3, T, ENTF, STAG>(C, S.R[k], P, chi_abs, chi_es, Fd, vd, fl, u, Fsd, Bf, VF, SP);
}

// The same with the staggered field (and, with ENTF, the entropy tracer)
template <class T, bool ENTF>
__global__ void GRRMHD_FLUX_LB k_flux_all_stag(Ctx C, FluxSegs S, const double* __restrict__ P,
                                               const double* __restrict__ chi_abs,
                                               const double* __restrict__ chi_es,
                                               double* __restrict__ F, double* __restrict__ vchar,
                                               const double* __restrict__ fl,
                                               double* __restrict__ Fs,
                                               const double* __restrict__ Bf,
                                               double* __restrict__ VF, double* __restrict__ SP) {
  flux_all_at<T, ENTF, true>(C, S, P, chi_abs, chi_es, F, vchar, fl,
                             xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x, Fs, Bf,
                             VF, SP);
}

template <class T>
__global__ void GRRMHD_FLUX_LB k_flux_all(Ctx C, FluxSegs S, const double* __restrict__ P,
                                          const double* __restrict__ chi_abs,
                                          const double* __restrict__ chi_es,
                                          double* __restrict__ F, double* __restrict__ vchar,
                                          const double* __restrict__ fl) {
  flux_all_at<T>(C, S, P, chi_abs, chi_es, F, vchar, fl,
                 xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
}

// The same with the entropy tracer's face fluxes Fs [3][Ntot] (the full
// implicit cascade's entropy equation)
template <class T>
__global__ void GRRMHD_FLUX_LB k_flux_all_s(Ctx C, FluxSegs S, const double* __restrict__ P,
                                            const double* __restrict__ chi_abs,
                                            const double* __restrict__ chi_es,
                                            double* __restrict__ F, double* __restrict__ vchar,
                                            const double* __restrict__ fl,
                                            double* __restrict__ Fs) {
  flux_all_at<T, true>(C, S, P, chi_abs, chi_es, F, vchar, fl,
                       xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x, Fs);
}

// sqrt(-g) S u^t of one cell's primitives p (the entropy tracer; NAN where
// rho0 or u_g is not positive)
DEV double entropy_cons(double gam, const Metric& m, const double p[5]) {
  if (!(p[0] > 0.0) || !(p[1] > 0.0)) return NAN;
  Vel<double> v;
  make_vel(m, p + 2, v);
  const double n = 1.0 / (gam - 1.0);
  const double S = p[0] * (n * ::log((gam - 1.0) * p[1]) - (n + 1.0) * ::log(p[0]));
  return m.gdet * S * v.ucon[0];
}

DEV bool interior_ijk(const Ctx& C, long t, int& i, int& j, int& k) {
  if (t >= (long)C.n[0] * C.n[1] * C.n[2]) return false;
  i = C.ng[0] + t % C.n[0];
  const long t2 = t / C.n[0];
  j = C.ng[1] + t2 % C.n[1];
  k = C.ng[2] + t2 / C.n[1];
  return true;
}

// the entropy tracer of P at interior cells
__global__ void LB(256) k_entropy_field(Ctx C, const double* __restrict__ P, double* __restrict__ S) {
  int i, j, k;
  if (!interior_ijk(C, (long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
  const long c = cell_index(C, i, j, k);
  Metric m;
  load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
  double p[5];
#pragma unroll
  for (int q = 0; q < 5; q++) p[q] = P[q * C.Ntot + c];
  S[c] = entropy_cons(C.gam, m, p);
}

// the entropy tracer's explicit stage value at interior cells:
// a Sn + b U_S(P) + cc dt (-div Fs), Sn = U_S(P^n), P the stage's input (no
// flux term, and no Fs read, where cc = 0)
__global__ void LB(256) k_entropy_update(Ctx C, double a, double b, double cc,
                                         const double* __restrict__ dt_dev,
                                         const double* __restrict__ Sn,
                                         const double* __restrict__ P,
                                         const double* __restrict__ Fs,
                                         double* __restrict__ Sexp) {
  int i, j, k;
  if (!interior_ijk(C, (long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
  const long c = cell_index(C, i, j, k);
  double sp = 0.0;
  if (b != 0.0) {
    Metric m;
    load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
    double p[5];
#pragma unroll
    for (int q = 0; q < 5; q++) p[q] = P[q * C.Ntot + c];
    sp = entropy_cons(C.gam, m, p);
  }
  double div = 0.0;
  for (int d = 0; d < 3 && cc != 0.0; d++)
    if (C.n[d] > 1)
      div += (Fs[(long)d * C.Ntot + c + C.st[d]] - Fs[(long)d * C.Ntot + c]) / C.dx[d];
  Sexp[c] = a * Sn[c] + (b != 0.0 ? b * sp : 0.0) - (cc != 0.0 ? cc * (*dt_dev) * div : 0.0);
}

// ---------------------------------------------------------------------------
// PPM shock flattener (Sec. 4.3; FLASH form with SP0 = 0.75): per cell within
// one cell of the interior and per active direction d, for gas (pressure
// (gam-1) u_g, velocity the specific mass flux sqrt(-g) u^d) and radiation
// (Ebar/3, sqrt(-g) u^d_rad), each pressure
// raised by w = min(1, 2 tau) times the other, tau = kappa_tot sqrt(g_dd) dx^d:
//   f = clamp(10 (|dp1|/|dp2| - 0.75), 0, 1) where |dp1| = |p(+1) - p(-1)| >
//   0.33 min(p(+1), p(-1)) and the flow converges, else 0; then the larger of
//   f and f at the neighbour on the high-pressure side; finally each kind
//   moves towards the larger of the two by w.  keep: the larger of this and
//   the stored value (earlier sub-steps of the step).
// ---------------------------------------------------------------------------
// f at one cell from the pressures one (p1, m1) and two (p2, m2) cells
// above and below it and the velocities one cell below and above
template <class T>
DEV T flat_raw(const T& p1, const T& m1, const T& p2, const T& m2, double vm, double vp) {
  const T d1 = p1 - m1, d2 = p2 - m2;
  if (!(val(fabs(d1)) > 0.33 * val(fmin(p1, m1))) || !(vm - vp > 0.0)) return T(0.0);
  return fmax(0.0, fmin(1.0, 10.0 * (fabs(d1) / fmax(fabs(d2), 1e-300) - 0.75)));
}

// pp[-3..3], v[-2..2] around the cell: f there, then the larger of it and
// f at the neighbour on the high-pressure side
template <class T>
DEV T flat_tilde(const T* pp, const double* v) {
  const T f0 = flat_raw(pp[1], pp[-1], pp[2], pp[-2], v[-1], v[1]);
  // both neighbours formed, then the one above or below taken: a select of
  // operands would become an indexed load and move the arrays to scratch
  const T fa = flat_raw(pp[2], pp[0], pp[3], pp[-1], v[0], v[2]);
  const T fb = flat_raw(pp[0], pp[-2], pp[1], pp[-3], v[-2], v[0]);
  return fmax(f0, val(pp[1] - pp[-1]) < 0.0 ? fa : fb);
}

// x / 3, the value rounded as the plain division (a dual number's division
// by a constant multiplies by its reciprocal)
DEV double third(double x) { return x / 3.0; }
template <int N>
DEV Dual<N> third(const Dual<N>& x) {
  Dual<N> r;
  r.v = x.v / 3.0;
#pragma unroll
  for (int i = 0; i < N; i++) r.d[i] = x.d[i] / 3.0;
  return r;
}

// The flattener's velocities on a Kerr-Schild grid, once per cell: the
// specific mass fluxes sqrt(-g) u^d of the gas (mf[d]) and the radiation
// (mf[3 + d]), d = 0..2, from the cell's own metric.
__global__ void LB(256) k_mass_flux(Ctx C, const double* __restrict__ P, double* __restrict__ mf) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.Ntot) return;
  Metric met;
  load_metric(C.geo_c, C.npos, (int)(c % C.npos), met);
  double ut[3];
  Vel<double> v;
#pragma unroll
  for (int a = 0; a < 3; a++) ut[a] = P[(2 + a) * C.Ntot + c];
  make_vel(met, ut, v);
#pragma unroll
  for (int d = 0; d < 3; d++) mf[(long)d * C.Ntot + c] = met.gdet * v.ucon[d + 1];
#pragma unroll
  for (int a = 0; a < 3; a++) ut[a] = P[(9 + a) * C.Ntot + c];
  make_vel(met, ut, v);
#pragma unroll
  for (int d = 0; d < 3; d++) mf[(long)(3 + d) * C.Ntot + c] = met.gdet * v.ucon[d + 1];
}

// The flattener's velocity of one kind (0 gas, 1 radiation) along d at cell
// cm: the mass flux of k_mass_flux (mf, Kerr-Schild), u~^d in flat space
// (mf null).
DEV double flat_vel(const Ctx& C, const double* __restrict__ P, const double* __restrict__ mf,
                    long cm, int d, int kind) {
  return mf ? mf[(long)(3 * kind + d) * C.Ntot + cm] : P[(long)((kind ? 9 : 2) + d) * C.Ntot + cm];
}

// Flattener of cell c along d for both kinds (f2[0] gas, f2[1] radiation),
// before the larger-over-sub-steps rule.  With T a dual number, the cell at
// offset ms (-3..3) takes (u_g, Ebar, rho, kappa_tot) from sd and every other
// cell is a constant (the forward passes an ms outside the stencil); the
// velocities enter only through the compression test.
template <class T>
DEV void flat_dir(const Ctx& C, const double* __restrict__ P, const double* __restrict__ chi_abs,
                  const double* __restrict__ chi_es, const double* __restrict__ mf, long c, int d,
                  int ms, const T* sd, T f2[2]) {
  const long st = C.st[d];
  const int sq = sym(d + 1, d + 1);
  T pg7[7], pr7[7], w0 = T(0.0);
  double vg5[5], vr5[5];
#pragma unroll
  for (int m = -3; m <= 3; m++) {
    const long cm = c + m * st;
    const int pos = (int)(cm % ((long)C.N[0] * C.N[1]));
    const double gdd = C.geo_c[(GE_GCOV + sq) * C.npos + pos];
    T ug, E, rho, chi;
    if (m == ms) {
      ug = sd[0];
      E = sd[1];
      rho = sd[2];
      chi = sd[3];
    } else {
      ug = T(P[C.Ntot + cm]);
      E = T(P[8 * C.Ntot + cm]);
      rho = T(P[cm]);
      chi = T(chi_abs[cm] + chi_es[cm]);
    }
    const T tau = chi * rho * ::sqrt(gdd) * C.dx[d];
    const T w = fmin(1.0, 2.0 * tau);
    const T p_g = (C.gam - 1.0) * ug, p_r = third(E);
    pg7[m + 3] = p_g + w * p_r;
    pr7[m + 3] = p_r + w * p_g;
    if (m == 0) w0 = w;
    if (m >= -2 && m <= 2) {
      vg5[m + 2] = flat_vel(C, P, mf, cm, d, 0);
      vr5[m + 2] = flat_vel(C, P, mf, cm, d, 1);
    }
  }
  // centred arrays
  const T fg = flat_tilde(pg7 + 3, vg5 + 2), fr = flat_tilde(pr7 + 3, vr5 + 2);
  const T fm = fmax(fg, fr);
  f2[0] = (1.0 - w0) * fg + w0 * fm;
  f2[1] = (1.0 - w0) * fr + w0 * fm;
}

// One thread per (cell, active direction): t runs over the cells within one
// of the interior for the first active direction, then the next (the
// directions' chains of loads overlap across threads rather than following
// one another in a thread).  mf: the mass fluxes of k_mass_flux
// (Kerr-Schild), null in flat space.
DEV void flatten_at(Ctx C, const double* __restrict__ P, const double* __restrict__ chi_abs,
                    const double* __restrict__ chi_es, double* __restrict__ fl, int keep, long t,
                    const double* __restrict__ mf) {
  int lo[3], cnt[3];
#pragma unroll
  for (int e = 0; e < 3; e++) {
    lo[e] = C.n[e] > 1 ? C.ng[e] - 1 : 0;
    cnt[e] = C.n[e] > 1 ? C.n[e] + 2 : 1;
  }
  const long ncell = (long)cnt[0] * cnt[1] * cnt[2];
  int slot = (int)(t / ncell), d = -1;
  for (int e = 0; e < 3; e++)
    if (C.n[e] > 1 && slot-- == 0) d = e;
  if (d < 0) return;
  t -= (t / ncell) * ncell;
  const int i = lo[0] + t % cnt[0];
  const long t2 = t / cnt[0];
  const int j = lo[1] + t2 % cnt[1];
  const int k = lo[2] + t2 / cnt[1];
  const long c = cell_index(C, i, j, k);
  double f2[2];
  flat_dir<double>(C, P, chi_abs, chi_es, mf, c, d, 99, nullptr, f2);
#pragma unroll
  for (int kind = 0; kind < 2; kind++) {
    double* dst = fl + (long)(2 * d + kind) * C.Ntot + c;
    *dst = keep ? ::fmax(*dst, f2[kind]) : f2[kind];
  }
}

__global__ void LB(256) k_flatten(Ctx C, const double* __restrict__ P,
                                  const double* __restrict__ chi_abs,
                                  const double* __restrict__ chi_es, double* __restrict__ fl,
                                  int keep, const double* __restrict__ mf) {
  flatten_at(C, P, chi_abs, chi_es, fl, keep, (long)blockIdx.x * blockDim.x + threadIdx.x, mf);
}

// ---------------------------------------------------------------------------
// step 9 (flux-CT): corner EMF along a = average of the four adjacent face
// induction fluxes, emf_a = F_c[B_b] = -F_b[B_c] for cyclic (a, b, c)
// ---------------------------------------------------------------------------
template <class T>
DEV void emf_edge(const Ctx& C, int a, int i, int j, int k, const double* __restrict__ F,
                  double* __restrict__ emf) {
  const long c = cell_index(C, i, j, k);
  const int b = (a + 1) % 3, cd = (a + 2) % 3;
  const double* Fb = F + (long)b * 12 * C.Ntot + (long)(5 + cd) * C.Ntot;   // F_b[B_c]
  const double* Fc = F + (long)cd * 12 * C.Ntot + (long)(5 + b) * C.Ntot;   // F_c[B_b]
  T e = T(0.25) * (((T)Fc[c] + (T)Fc[c - C.st[b]]) - ((T)Fb[c] + (T)Fb[c - C.st[cd]]));
  if (C.metric == GRRMHD_KERR_SCHILD && (b == 1 || cd == 1)) {
    // edges on the polar axis carry no EMF
    const bool lo = j == C.ng[1] && (C.bc_lo[1] == GRRMHD_BC_REFLECT || C.bc_lo[1] == GRRMHD_BC_POLAR);
    const bool hi = j == C.ng[1] + C.n[1] && (C.bc_hi[1] == GRRMHD_BC_REFLECT || C.bc_hi[1] == GRRMHD_BC_POLAR);
    if (lo || hi) e = T(0.0);
  }
  emf[(long)a * C.Ntot + c] = (double)e;
}

// Every corner EMF in one pass: position (i, j, k) in the union of the edge
// ranges, each orientation a whose other two axes are active and whose range
// holds the position; FP32 arithmetic from x1 index mixed_i on.
DEV void emf_all_at(Ctx C, FaceRange R, const double* __restrict__ F, double* __restrict__ emf,
                    long t) {
  if (t >= R.total) return;
  const int i = R.lo[0] + t % R.cnt[0];
  const long t2 = t / R.cnt[0];
  const int j = R.lo[1] + t2 % R.cnt[1];
  const int k = R.lo[2] + t2 / R.cnt[1];
  const int idx[3] = {i, j, k};
  for (int a = 0; a < 3; a++) {
    if (C.n[(a + 1) % 3] == 1 || C.n[(a + 2) % 3] == 1) continue;
    if (idx[a] >= C.ng[a] + C.n[a]) continue;
    if (i < C.mixed_i) emf_edge<double>(C, a, i, j, k, F, emf);
    else emf_edge<float>(C, a, i, j, k, F, emf);
  }
}

__global__ void LB(256) k_emf_all(Ctx C, FaceRange R, const double* __restrict__ F,
                                  double* __restrict__ emf) {
  emf_all_at(C, R, F, emf, (long)blockIdx.x * blockDim.x + threadIdx.x);
}


// ---------------------------------------------------------------------------
// step 10: explicit stage combination with flux divergence and geometry
// source.  The source uses sqrt(-g) T^k_l Gamma^l_{nu k} =
// (1/2) sqrt(-g) T^{k m} d_nu g_{k m}; both metrics are independent of t and
// x3, so only nu = 1, 2 contribute.
// ---------------------------------------------------------------------------
template <class T>
DEV T contract_sym(const double* dg, const T u[4], const T v[4]) {
  T s = T(0.0);
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) s = s + u[a] * v[b] * dg[sym(a, b)];
  return s;
}

// Geometric source of the cell with primitives p: S[q] = 0 except the
// x1, x2 momentum slots of gas and radiation (dg: d g_{km}/dx1, d/dx2).
template <class T>
DEV void geom_source(const Metric& m, const double dg[2][10], double gam, const T p[12], T S[12]) {
#pragma unroll
  for (int q = 0; q < 12; q++) S[q] = T(0.0);
  Gas<T> s;
  make_gas(m, gam, p[0], p[1], p + 2, p + 5, s);
  Vel<T> r;
  make_vel(m, p + 9, r);
  const T enth = s.rho + s.ug + s.pg + s.bsq, ptot = s.pg + 0.5 * s.bsq;
  for (int nu = 1; nu <= 2; nu++) {
    const double* g = dg[nu - 1];
    double trace = 0.0;   // g^{km} d_nu g_{km}
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) trace += m.up(a, b) * g[sym(a, b)];
    const T sg = enth * contract_sym(g, s.v.ucon, s.v.ucon) + ptot * trace -
                 contract_sym(g, s.bcon, s.bcon);
    const T sr = (4.0 / 3.0) * p[8] * contract_sym(g, r.ucon, r.ucon) + (1.0 / 3.0) * p[8] * trace;
    S[1 + nu] = 0.5 * m.gdet * sg;
    S[8 + nu] = 0.5 * m.gdet * sr;
  }
}

DEV void load_dg(const Ctx& C, int pos, double dg[2][10]) {
#pragma unroll
  for (int q = 0; q < 10; q++) {
    dg[0][q] = C.geo_c[(GE_DG1 + q) * C.npos + pos];
    dg[1][q] = C.geo_c[(GE_DG2 + q) * C.npos + pos];
  }
}

// The step's Courant reduction spreads its atomics over GRRMHD_DT_SLOTS
// slots, one 128-byte line apart (block b uses slot b mod GRRMHD_DT_SLOTS,
// i.e. one per XCD), so the blocks of different XCDs do not queue on one line.
#define GRRMHD_DT_SLOTS 8
#define GRRMHD_DT_STRIDE 16

DEV double dt_slots_min(const unsigned long long* s) {
  unsigned long long b = s[0];
#pragma unroll
  for (int i = 1; i < GRRMHD_DT_SLOTS; i++) b = ::min(b, s[i * GRRMHD_DT_STRIDE]);
  return __longlong_as_double((long long)b);
}

// Stored 4-force sources of earlier stages added to an explicit bracket:
// dt sum_k m[k] M_k, each M_k an [8][Ntot] array (slots 1-4 and 8-11 of U).
struct MTerms {
  const double* M[4];
  double m[4];
  int n;
};

// dt: *dt_dev, or, when dtmin is set, courant x the minimum over the Courant
// reduction's slots, which thread 0 also stores in *dt_dev while it resets
// dtnext (the slots of the following step's reduction) to +inf.
// cc = 0: no flux or geometric term (F, emf and P are not read).
DEV void update_at(Ctx C, double ca, double cb, double cc, double* dt_dev,
                   const unsigned long long* dtmin, unsigned long long* dtnext,
                   const double* __restrict__ P, const double* __restrict__ Un,
                   const double* __restrict__ Uprev, const double* __restrict__ F,
                   const double* __restrict__ emf, const MTerms& MT, double* __restrict__ Uexp,
                   long t, const double* __restrict__ Bface = nullptr) {
  const long nint = (long)C.n[0] * C.n[1] * C.n[2];
  if (t >= nint) return;
  const int i = C.ng[0] + t % C.n[0];
  const long t2 = t / C.n[0];
  const int j = C.ng[1] + t2 % C.n[1];
  const int k = C.ng[2] + t2 / C.n[1];
  const long c = cell_index(C, i, j, k);
  double dt;
  if (dtmin) {
    dt = C.courant * dt_slots_min(dtmin);
    if (t == 0) {
      *dt_dev = dt;
#pragma unroll
      for (int i = 0; i < GRRMHD_DT_SLOTS; i++) dtnext[i * GRRMHD_DT_STRIDE] = 0x7FF0000000000000ull;
    }
  } else {
    dt = *dt_dev;
  }
  double S[12];
#pragma unroll
  for (int q = 0; q < 12; q++) S[q] = 0.0;
  double div[12];
#pragma unroll
  for (int q = 0; q < 12; q++) div[q] = 0.0;
  if (cc != 0.0 && C.metric != GRRMHD_MINKOWSKI) {
    const int pos = i + C.N[0] * j;
    Metric m;
    load_metric(C.geo_c, C.npos, pos, m);
    double p[12], dg[2][10];
#pragma unroll
    for (int q = 0; q < 12; q++) p[q] = P[q * C.Ntot + c];
    load_dg(C, pos, dg);
    geom_source(m, dg, C.gam, p, S);
  }
  for (int d = 0; d < 3 && cc != 0.0; d++) {
    if (C.n[d] == 1) continue;
    const double idx = 1.0 / C.dx[d];
    const double* Fd = F + (long)d * 12 * C.Ntot;
    const long sd = C.st[d];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      if (q >= 5 && q <= 7) continue;
      div[q] += (Fd[q * C.Ntot + c + sd] - Fd[q * C.Ntot + c]) * idx;
    }
    for (int b = 0; b < 3; b++) {
      if (b == d) continue;
      double fm, fp;
      if (C.n[b] > 1) {
        // face flux = mean of the two corner EMFs adjacent along b
        const int aa = 3 - b - d;
        const double sgn = ((aa + 1) % 3 == b) ? 1.0 : -1.0;
        const double* E = emf + (long)aa * C.Ntot;
        const long sb = C.st[b];
        fm = 0.5 * sgn * (E[c] + E[c + sb]);
        fp = 0.5 * sgn * (E[c + sd] + E[c + sd + sb]);
      } else {
        fm = Fd[(5 + b) * C.Ntot + c];
        fp = Fd[(5 + b) * C.Ntot + c + sd];
      }
      div[5 + b] += (fp - fm) * idx;
    }
  }
#pragma unroll
  for (int q = 0; q < 12; q++) {
    double u = ca * Un[q * C.Ntot + c];
    if (cb != 0.0) u += cb * Uprev[q * C.Ntot + c];
    if (cc != 0.0) u += cc * dt * (S[q] - div[q]);
    if (MT.n > 0 && ((q >= 1 && q <= 4) || q >= 8)) {
      const int r = (q <= 4) ? q - 1 : q - 4;
      double sm = 0.0;
      for (int k = 0; k < MT.n; k++) sm += MT.m[k] * MT.M[k][r * C.Ntot + c];
      u += dt * sm;
    }
    Uexp[q * C.Ntot + c] = u;
  }
  if (Bface) {
    // staggered field: the stage's cell-centred field is the mean of the
    // cell's two new faces (the face itself on an inactive dimension)
#pragma unroll
    for (int q = 0; q < 3; q++) {
      const double* B = Bface + (long)q * C.Ntot;
      Uexp[(5 + q) * C.Ntot + c] = (C.n[q] > 1) ? 0.5 * (B[c] + B[c + C.st[q]]) : B[c];
    }
  }
}

__global__ void LB(256) k_update(Ctx C, double ca, double cb, double cc, double* dt_dev,
                                 const unsigned long long* dtmin, unsigned long long* dtnext,
                                 const double* __restrict__ P, const double* __restrict__ Un,
                                 const double* __restrict__ Uprev, const double* __restrict__ F,
                                 const double* __restrict__ emf, MTerms MT,
                                 double* __restrict__ Uexp, const double* __restrict__ Bface) {
  update_at(C, ca, cb, cc, dt_dev, dtmin, dtnext, P, Un, Uprev, F, emf, MT, Uexp,
            (long)blockIdx.x * blockDim.x + threadIdx.x, Bface);
}

// ---------------------------------------------------------------------------
// Courant time step: per-cell harmonic combination, block min, one atomic
// per block on the ordered bit pattern of a positive double
// ---------------------------------------------------------------------------
__global__ void k_dt_init(unsigned long long* slot, int n, int stride) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) slot[(long)i * stride] = 0x7FF0000000000000ull;
}

// 1 / sum_d (larger face speed along d / dx_d) of interior cell t; +inf past the end
DEV double cell_dt(const Ctx& C, const double* __restrict__ vchar, long t) {
  const long nint = (long)C.n[0] * C.n[1] * C.n[2];
  if (t >= nint) return INFINITY;
  const int i = C.ng[0] + t % C.n[0];
  const long t2 = t / C.n[0];
  const int j = C.ng[1] + t2 % C.n[1];
  const int k = C.ng[2] + t2 / C.n[1];
  const long c = cell_index(C, i, j, k);
  double inv = 0.0;
  for (int d = 0; d < 3; d++) {
    if (C.n[d] == 1) continue;
    const double* v = vchar + (long)d * C.Ntot;
    inv += fmax(v[c], v[c + C.st[d]]) / C.dx[d];
  }
  return 1.0 / inv;
}

// minimum over a block of up to 256 threads (every thread calls it), then
// one atomicMin per block on the ordered bits of a positive double
DEV void block_min_atomic(double v, unsigned long long* slot) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  __shared__ double wmin[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wmin[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = wmin[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); w++) b = fmin(b, wmin[w]);
    atomicMin(slot, (unsigned long long)__double_as_longlong(b));
  }
}

__global__ void LB(256) k_dt_min(Ctx C, const double* __restrict__ vchar,
                                 unsigned long long* slot) {
  block_min_atomic(cell_dt(C, vchar, (long)blockIdx.x * blockDim.x + threadIdx.x), slot);
}

// The same, and the Courant reduction over interior cells into dtmin (the
// grid covers both ranges; R.total = 0 when there are no EMFs)
__global__ void LB(256) k_emf_dt(Ctx C, FaceRange R, const double* __restrict__ F,
                                 double* __restrict__ emf, const double* __restrict__ vchar,
                                 unsigned long long* dtmin) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  emf_all_at(C, R, F, emf, t);
  block_min_atomic(cell_dt(C, vchar, t), dtmin + (blockIdx.x % GRRMHD_DT_SLOTS) * GRRMHD_DT_STRIDE);
}

__global__ void k_dt_final(const unsigned long long* slot, double courant, double* dt_out) {
  *dt_out = courant * __longlong_as_double((long long)*slot);
}

// ---------------------------------------------------------------------------
// steps 11-12: implicit solve per interior cell; and the stand-alone
// con2prim of an explicit state
// ---------------------------------------------------------------------------
DEV Phys make_phys(const Ctx& C) {
  Phys ph;
  ph.gam = C.gam;
  ph.arad = C.arad;
  ph.gamma_max = C.gamma_max;
  ph.ymax = C.ymax;
  return ph;
}
DEV Opts make_opts(const Ctx& C) {
  Opts o;
  o.tol_pmhd = C.tol_pmhd;
  o.tol_urad = C.tol_urad;
  o.tol_accept = C.tol_accept;
  o.tol_fail = C.tol_fail;
  o.max_iter = C.max_iter;
  o.roundoff = C.roundoff;
  o.cold = C.cold;
  o.u_floor = C.u_floor;
  return o;
}

// Append flagged lanes of a wavefront to a work list: one atomic per
// wavefront, slots ordered by lane (ballot + popcount prefix).  Returns the
// lane's slot, or -1.
DEV long wave_append(bool need, int item, int* counter, int* list) {
  const unsigned long long mask = __ballot(need);
  if (mask == 0ull) return -1;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader, 64);
  if (!need) return -1;
  const long slot = (long)base + __popcll(mask & ((1ull << lane) - 1ull));
  list[slot] = item;
  return slot;
}

// wavefront-aggregated queue fetch: one atomic for all lanes asking
DEV long wave_fetch(bool need, int* next) {
  const unsigned long long mask = __ballot(need);
  if (mask == 0ull) return -1;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(next, __popcll(mask));
  base = __shfl(base, leader, 64);
  return need ? (long)base + __popcll(mask & ((1ull << lane) - 1ull)) : -1;
}

// Bookkeeping of one implicit launch: the cascade work list with the first
// attempts' records, and lane statistics: stats[0] residual evaluations of
// first PMHD attempts (Newton trips), stats[1] lane slots the wavefronts
// spent on them (64 per wavefront trip), so stats[0]/stats[1] is the active
// lane fraction.
struct Work {
  int* counter;
  int* counter_next;   // if set: zeroed by the cascade kernel for the next launch
  int* list;
  unsigned long long* stats;
  RecBuf rec;
};

// per-wavefront totals of lanes that each ran `trips` trips in lockstep;
// returns the wavefront's largest count
DEV int wave_stats(int trips, unsigned long long* stats) {
  int s = trips, mx = trips;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    mx = ::max(mx, __shfl_xor(mx, off, 64));
  }
  if ((threadIdx.x & 63) == 0 && s > 0) {
    atomicAdd(&stats[0], (unsigned long long)s);
    atomicAdd(&stats[1], 64ull * (unsigned long long)mx);
  }
  return mx;
}

// Dispatch order of the implicit kernel's tiles: costliest first, by the
// largest Newton-trip count of each tile's first attempts in the previous
// launch (keys), one bucket per count up to GRRMHD_ORDER_BUCKETS - 1.  A
// wavefront costs what its slowest lane costs, and with a few waves per
// SIMD the launch ends on whichever tiles start last: dispatching the long
// ones first leaves the short ones to fill the end.  The sort keeps the
// XCD-aware split (xcd_block: XCD x works through the x-th eighth of the
// tiles, whose neighbours share its L2): each eighth is sorted apart, one
// block each (a ninth takes the remainder tiles), by counting sort (ties in
// any order; every tile's result is independent of it).  order[] maps each
// eighth onto itself.
#define GRRMHD_ORDER_BUCKETS 64
DEV int order_bucket(int key) { return ::min(::max(key, 0), GRRMHD_ORDER_BUCKETS - 1); }

__global__ void __launch_bounds__(1024) k_tile_order(long ntiles, const int* __restrict__ keys,
                                                     int* __restrict__ order) {
  __shared__ int cnt[GRRMHD_ORDER_BUCKETS];
  const long seg = ntiles / 8;
  const long lo = (blockIdx.x < 8) ? (long)blockIdx.x * seg : 8 * seg;
  const long hi = (blockIdx.x < 8) ? lo + seg : ntiles;
  for (int b = threadIdx.x; b < GRRMHD_ORDER_BUCKETS; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  for (long t = lo + threadIdx.x; t < hi; t += blockDim.x) atomicAdd(&cnt[order_bucket(keys[t])], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int sum = 0;   // exclusive prefix, largest bucket first
    for (int b = GRRMHD_ORDER_BUCKETS - 1; b >= 0; b--) {
      const int c = cnt[b];
      cnt[b] = sum;
      sum += c;
    }
  }
  __syncthreads();
  for (long t = lo + threadIdx.x; t < hi; t += blockDim.x)
    order[lo + atomicAdd(&cnt[order_bucket(keys[t])], 1)] = (int)t;
}

__global__ void k_zero_ints(int* p, int k) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) p[i] = 0;
}

DEV void store_out(const CellOut& o, long c, long Nst, double* P, double* U, int* iters,
                   int* status, double* err) {
#pragma unroll
  for (int q = 0; q < 12; q++) {
    P[q * Nst + c] = o.P[q];
    U[q * Nst + c] = o.U[q];
  }
  if (iters) iters[c] = o.iters;
  if (status) status[c] = o.status;
  if (err) err[c] = o.err;
}

// A cell the fast path did not accept: to the work list, with its first
// attempt (extreme cells have none).
DEV void to_cascade(bool need, bool extreme, int item, const Best& b, int iters, const Work& W) {
  const long slot = wave_append(need, item, W.counter, W.list);
  if (slot >= 0 && !extreme) rec_store(W.rec, slot, b, iters);
}

// Common path of the implicit solve at interior cells; cells that need the
// full cascade go to the work list (index into the interior enumeration).
// Cells of one wavefront: a tile of ti x (64 / ti) cells in (x1, x2) at one
// x3, so that its lanes share radius and latitude (and with them the Newton
// count) more than a run of 64 cells along x1 does, while each group of ti
// lanes still reads contiguous memory.
DEV bool tile_cell(const Ctx& C, int ti, long wave, int lane, int& i, int& j, int& k) {
  const int tj = 64 / ti;
  const int nti = (C.n[0] + ti - 1) / ti, ntj = (C.n[1] + tj - 1) / tj;
  const int a = wave % nti;
  const long w2 = wave / nti;
  const int b = w2 % ntj;
  k = w2 / ntj;
  const int ii = a * ti + lane % ti, jj = b * tj + lane / ti;
  if (ii >= C.n[0] || jj >= C.n[1] || k >= C.n[2]) return false;
  i = C.ng[0] + ii;
  j = C.ng[1] + jj;
  k += C.ng[2];
  return true;
}

__global__ void LBI k_implicit(Ctx C, int ti, const double* __restrict__ Uexp, const double* Pguess,
                                  double dt_scale, const double* __restrict__ dt_dev,
                                  const double* __restrict__ chi_abs,
                                  const double* __restrict__ chi_es, double* P,
                                  double* __restrict__ U, int* __restrict__ iters,
                                  int* __restrict__ status, double* __restrict__ err, Work W,
                                  const int* __restrict__ order, int* __restrict__ keys) {
  bool need = false, extreme = false;
  Best b;
  int it = 0, trips = 0;
  int i = 0, j = 0, k = 0;
  long t = 0;   // the cell's index in the interior enumeration (x1 fastest)
  // the tile: XCD-aware, and within each XCD's eighth in the cost order of
  // the previous launch when given
  const long xb = xcd_block(blockIdx.x, gridDim.x);
  const long tile = order ? (long)order[xb] : xb;
  if (tile_cell(C, ti, tile, threadIdx.x, i, j, k)) {
    t = (i - C.ng[0]) + (long)C.n[0] * ((j - C.ng[1]) + (long)C.n[1] * (k - C.ng[2]));
    const long c = cell_index(C, i, j, k);
    Metric m;
    load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
    double Ui[12], Pg[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      Ui[q] = Uexp[q * C.Ntot + c];
      Pg[q] = Pguess[q * C.Ntot + c];
    }
    CellOut o;
    if (implicit_fast(m, make_phys(C), make_opts(C), Ui, Pg, dt_scale * (*dt_dev), chi_abs[c],
                      chi_es[c], o, b, it, extreme, trips))
      store_out(o, c, C.Ntot, P, U, iters, status, err);
    else
      need = true;
  }
  const int mx = wave_stats(trips, W.stats);
  if (keys && threadIdx.x == 0) keys[tile] = mx;
  to_cascade(need, extreme, (int)t, b, it, W);
}

// Rest of the cascade over the work list; grid-stride over a count kept on
// the device.
// FULL: the paper's full cascade (params.cascade = 1), a separate
// instantiation so the normal cascade keeps its smaller register footprint
template <bool FULL>
__global__ void LB(64) k_implicit_list(Ctx C, const double* __restrict__ Uexp,
                                       const double* Pguess, double dt_scale,
                                       const double* __restrict__ dt_dev,
                                       const double* __restrict__ chi_abs,
                                       const double* __restrict__ chi_es, double* P,
                                       double* __restrict__ U, int* __restrict__ iters,
                                       int* __restrict__ status, double* __restrict__ err,
                                       Work W, const double* __restrict__ Sexp) {
  const int n = *W.counter;
  if (W.counter_next && blockIdx.x == 0 && threadIdx.x == 0) *W.counter_next = 0;
  for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < n;
       w += (long)gridDim.x * blockDim.x) {
    const long t = W.list[w];
    const int i = C.ng[0] + t % C.n[0];
    const long t2 = t / C.n[0];
    const int j = C.ng[1] + t2 % C.n[1];
    const int k = C.ng[2] + t2 / C.n[1];
    const long c = cell_index(C, i, j, k);
    Metric m;
    load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
    double Ui[12], Pg[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      Ui[q] = Uexp[q * C.Ntot + c];
      Pg[q] = Pguess[q * C.Ntot + c];
    }
    CellOut o;
    if constexpr (FULL)
      implicit_cell_full(m, make_phys(C), make_opts(C), Ui, Sexp ? Sexp[c] : NAN, Pg,
                         dt_scale * (*dt_dev), chi_abs[c], chi_es[c], o, &W.rec, w, 1);
    else
      implicit_cell(m, make_phys(C), make_opts(C), Ui, Pg, dt_scale * (*dt_dev), chi_abs[c],
                    chi_es[c], o, &W.rec, w);
    store_out(o, c, C.Ntot, P, U, iters, status, err);
  }
}

// Independent flat-space cells: same two-kernel structure.
__global__ void LBI k_implicit_batch(Ctx C, long n, const double* __restrict__ Ui_,
                                        const double* __restrict__ Pg_,
                                        const double* __restrict__ dtc,
                                        const double* __restrict__ chi_abs,
                                        const double* __restrict__ chi_es,
                                        double* __restrict__ Po, double* __restrict__ Uo,
                                        int* __restrict__ iters, int* __restrict__ status,
                                        double* __restrict__ err, Work W) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  bool need = false, extreme = false;
  Best b;
  int it = 0, trips = 0;
  if (c < n) {
    Metric m;
    flat_metric(m);
    double Ui[12], Pg[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      Ui[q] = Ui_[q * n + c];
      Pg[q] = Pg_[q * n + c];
    }
    CellOut o;
    if (implicit_fast(m, make_phys(C), make_opts(C), Ui, Pg, dtc[c], chi_abs[c], chi_es[c], o, b,
                      it, extreme, trips))
      store_out(o, c, n, Po, Uo, iters, status, err);
    else
      need = true;
  }
  wave_stats(trips, W.stats);
  to_cascade(need, extreme, (int)c, b, it, W);
}

__global__ void LB(64) k_implicit_batch_list(Ctx C, long n, const double* __restrict__ Ui_,
                                             const double* __restrict__ Pg_,
                                             const double* __restrict__ dtc,
                                             const double* __restrict__ chi_abs,
                                             const double* __restrict__ chi_es,
                                             double* __restrict__ Po, double* __restrict__ Uo,
                                             int* __restrict__ iters, int* __restrict__ status,
                                             double* __restrict__ err, Work W, Work K) {
  const int cnt = *W.counter;
  for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < cnt;
       w += (long)gridDim.x * blockDim.x) {
    const long c = W.list[w];
    Metric m;
    flat_metric(m);
    double Ui[12], Pg[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      Ui[q] = Ui_[q * n + c];
      Pg[q] = Pg_[q * n + c];
    }
    CellOut o;
    const Opts op = make_opts(C);
    if (C.cascade) {
      // the full cascade from scratch, the cold limit inline; a cell without
      // a grid takes the entropy of its prior primitives
      implicit_cell_full(m, make_phys(C), op, Ui, entropy_cons(C.gam, m, Pg), Pg, dtc[c],
                         chi_abs[c], chi_es[c], o);
      store_out(o, c, n, Po, Uo, iters, status, err);
      continue;
    }
    implicit_cell(m, make_phys(C), op, Ui, Pg, dtc[c], chi_abs[c], chi_es[c], o, &W.rec, w, false);
    store_out(o, c, n, Po, Uo, iters, status, err);
    bool cold = false;
    if ((o.status & GRRMHD_ST_FAIL) && op.cold) {
      Cell cl;
      cell_setup(m, Ui, dtc[c], chi_abs[c], chi_es[c], cl);
      cold = cold_allowed(cl, Pg);
    }
    wave_append(cold, (int)c, K.counter, K.list);
  }
}

// Cells of a batch left without an energy solution that meet the cold
// attempt's conditions (listed in K by the cascade kernels): the cold MHD
// limit, one thread each; the iterations of the cell's energy attempts (in
// `iters`, when kept) are carried on.
__global__ void LB(64) k_cold_batch_list(Ctx C, long n, const double* __restrict__ Ui_,
                                         const double* __restrict__ Pg_,
                                         const double* __restrict__ dtc,
                                         const double* __restrict__ chi_abs,
                                         const double* __restrict__ chi_es,
                                         double* __restrict__ Po, double* __restrict__ Uo,
                                         int* __restrict__ iters, int* __restrict__ status,
                                         double* __restrict__ err, Work K) {
  const int cnt = *K.counter;
  for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < cnt;
       w += (long)gridDim.x * blockDim.x) {
    const long c = K.list[w];
    Metric m;
    flat_metric(m);
    double Ui[12], Pg[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      Ui[q] = Ui_[q * n + c];
      Pg[q] = Pg_[q * n + c];
    }
    int it = iters ? iters[c] : 0;
    CellOut o;
    if (cold_cell(m, make_phys(C), make_opts(C), Ui, Pg, dtc[c], chi_abs[c], chi_es[c], it, o))
      store_out(o, c, n, Po, Uo, iters, status, err);
    else if (iters)
      iters[c] = it;
  }
}

// The full cascade's rest (params.cascade = 1) for batch cells the PMHD and
// URAD attempts left unaccepted: K lists their record slots; each resumes
// after both attempts (one thread per cell).
__global__ void LB(64) k_rest_batch_list(Ctx C, long n, const double* __restrict__ Ui_,
                                         const double* __restrict__ Pg_,
                                         const double* __restrict__ dtc,
                                         const double* __restrict__ chi_abs,
                                         const double* __restrict__ chi_es,
                                         double* __restrict__ Po, double* __restrict__ Uo,
                                         int* __restrict__ iters, int* __restrict__ status,
                                         double* __restrict__ err, Work W, Work K) {
  const int cnt = *K.counter;
  for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < cnt;
       w += (long)gridDim.x * blockDim.x) {
    const long slot = K.list[w];
    const long c = W.list[slot];
    Metric m;
    flat_metric(m);
    double Ui[12], Pg[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      Ui[q] = Ui_[q * n + c];
      Pg[q] = Pg_[q * n + c];
    }
    CellOut o;
    implicit_cell_full(m, make_phys(C), make_opts(C), Ui, entropy_cons(C.gam, m, Pg), Pg, dtc[c],
                       chi_abs[c], chi_es[c], o, &W.rec, slot, 2);
    store_out(o, c, n, Po, Uo, iters, status, err);
  }
}

// The cascade of a batch, compacting: a fixed grid of wavefronts whose lanes
// take list entries from a cursor (one atomic per wavefront) and run the URAD
// attempt as a lane state machine, one residual evaluation per trip, taking
// the next entry as soon as their cell ends.  Extreme cells (URAD first, then
// PMHD from scratch) go to the deferred list D for the per-cell cascade.
// Results equal those of implicit_cell resuming from the same record.
__global__ void LB(64) k_cascade_urad(Ctx C, long n, const double* __restrict__ Ui_,
                                      const double* __restrict__ Pg_,
                                      const double* __restrict__ dtc,
                                      const double* __restrict__ chi_abs,
                                      const double* __restrict__ chi_es,
                                      double* __restrict__ Po, double* __restrict__ Uo,
                                      int* __restrict__ iters, int* __restrict__ status,
                                      double* __restrict__ err, Work W, int* cursor, Work D,
                                      Work K) {
  const Phys ph = make_phys(C);
  const Opts o = make_opts(C);
  Metric m;
  flat_metric(m);
  const int cnt = *W.counter;
  UradLane L;
  Cell c;
  long item = 0, slot = 0;
  int pst = 0;
  bool active = false, exhausted = false;
  unsigned long long useful = 0, slots = 0;
  for (;;) {
    const bool need = !active && !exhausted;
    const long got = wave_fetch(need, cursor);
    bool defer = false;
    if (need) {
      if (got < cnt) {
        slot = got;
        item = W.list[slot];
        double Ui[12], Pg[12];
#pragma unroll
        for (int q = 0; q < 12; q++) {
          Ui[q] = Ui_[q * n + item];
          Pg[q] = Pg_[q * n + item];
        }
        Prep pr;
        prepare(m, ph, Ui, Pg, dtc[item], chi_abs[item], chi_es[item], c, pr);
        pst = pr.status;
        if (pr.extreme) {
          defer = true;
        } else {
          // URAD from the first attempt's solution when it got below 1e-4, else from the guess
          Best b0;
          int it0;
          rec_load(W.rec, slot, b0, it0);
          const bool prev = b0.ok && b0.eT < 1e-4;
          const double* src = prev ? b0.P : Pg;
          rad_cons4(m, src, L.p);
#pragma unroll
          for (int q = 0; q < 5; q++) L.Pn[q] = src[q];
          L.iters = it0;
          L.mode = UM_START;
          active = true;
        }
      } else {
        exhausted = true;
      }
    }
    wave_append(defer, (int)item, D.counter, D.list);
    bool ended = false, doeval = false;
    if (active) {
      ended = urad_before(c, o, L);
      doeval = !ended;
    }
    if (doeval) {
      Eval ev;
      double Jn[4][4];
      eval_urad_jac(c, ph, L.p, L.Pn, ev, Jn);
      ended = urad_after(ev, Jn, L);
    }
    const unsigned long long ev_mask = __ballot(doeval);
    useful += __popcll(ev_mask);
    slots += ev_mask ? 64ull : 0ull;
    bool failed = false;
    if (ended) {
      Best best;
      int it0;
      rec_load(W.rec, slot, best, it0);
      int bm = -1;
      if (best.ok) bm = M_PMHD;
      else best.eT = INFINITY;
      if (L.best.ok && L.best.eT < best.eT) {
        best = L.best;
        bm = M_URAD;
      }
      double Ui[12], Pg[12];
#pragma unroll
      for (int q = 0; q < 12; q++) {
        Ui[q] = Ui_[q * n + item];
        Pg[q] = Pg_[q * n + item];
      }
      CellOut out;
      if (bm < 0) failed_out(Ui, Pg, pst, L.iters, out);
      else finalize(c, ph, o, best, bm, pst, L.iters, Ui, out);
      store_out(out, item, n, Po, Uo, iters, status, err);
      if (C.cascade) {
        // not accepted: the rest of the full cascade resumes from the better of
        // the PMHD and URAD attempts, kept in the cell's record (method in ok)
        failed = !(bm >= 0 && best.eT < accept_threshold(o));
        if (failed) {
          Best kb = best;
          kb.ok = (bm >= 0 ? 1 : 0) | ((bm >= 0 ? bm : 0) << 1);
          rec_store(W.rec, slot, kb, L.iters);
        }
      } else {
        failed = (out.status & GRRMHD_ST_FAIL) && o.cold && cold_allowed(c, Pg);
      }
      active = false;
    }
    // to the cold limit; with the full cascade, the record slot to its rest
    wave_append(failed, C.cascade ? (int)slot : (int)item, K.counter, K.list);
    if (!__any(active) && __all(exhausted)) break;
  }
  if ((threadIdx.x & 63) == 0 && useful) {
    atomicAdd(&W.stats[2], useful);
    atomicAdd(&W.stats[3], slots);
  }
}

// fail_bits: extra status bits of a cell whose MHD inversion fails
__global__ void LB(128) k_con2prim(Ctx C, const double* __restrict__ U, const double* Pguess,
                                   double* P, int* __restrict__ status, int fail_bits) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nint = (long)C.n[0] * C.n[1] * C.n[2];
  if (t >= nint) return;
  const int i = C.ng[0] + t % C.n[0];
  const long t2 = t / C.n[0];
  const int j = C.ng[1] + t2 % C.n[1];
  const int k = C.ng[2] + t2 / C.n[1];
  const long c = cell_index(C, i, j, k);
  Metric m;
  load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
  const double igd = 1.0 / m.gdet;
  double u[12], p[12];
#pragma unroll
  for (int q = 0; q < 12; q++) {
    u[q] = U[q * C.Ntot + c] * igd;
    p[q] = Pguess[q * C.Ntot + c];
  }
  double rho = p[0], ug = p[1], ut[3] = {p[2], p[3], p[4]};
  int st = 0;
  if (mhd_invert(m, C.gam, u[0], u[1], u + 2, u + 5, rho, ug, ut) == 0) {
    p[0] = rho; p[1] = ug; p[2] = ut[0]; p[3] = ut[1]; p[4] = ut[2];
  } else {
    st |= GRRMHD_ST_C2P_FAIL | fail_bits;
  }
#pragma unroll
  for (int q = 0; q < 3; q++) p[5 + q] = u[5 + q];
  double Eb, utr[3];
  rad_invert(m, C.gamma_max, C.ymax, 0, u + 8, Eb, utr);
  p[8] = Eb; p[9] = utr[0]; p[10] = utr[1]; p[11] = utr[2];
#pragma unroll
  for (int q = 0; q < 12; q++) P[q * C.Ntot + c] = p[q];
  if (status) status[c] = st;
}

// the 12 fields of src at interior cells into dst (ghost cells untouched)
__global__ void LB(256) k_copy_interior12(Ctx C, const double* __restrict__ src,
                                          double* __restrict__ dst) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nint = (long)C.n[0] * C.n[1] * C.n[2];
  if (t >= nint) return;
  const int i = C.ng[0] + t % C.n[0];
  const long t2 = t / C.n[0];
  const int j = C.ng[1] + t2 % C.n[1];
  const int k = C.ng[2] + t2 / C.n[1];
  const long c = cell_index(C, i, j, k);
#pragma unroll
  for (int q = 0; q < 12; q++) dst[q * C.Ntot + c] = src[q * C.Ntot + c];
}

// The 4-force source of an implicit stage as its solve found it:
// M = (U_out - U_expl) / (g dt) in the gas and radiation energy-momentum
// slots (rows 0-3: U slots 1-4, rows 4-7: slots 8-11; [8][Ntot]), zero where
// the solve failed.
__global__ void LB(256) k_stage_m(Ctx C, const double* __restrict__ Ue,
                                  const double* __restrict__ Uo, const int* __restrict__ status,
                                  double g, const double* __restrict__ dt_dev,
                                  double* __restrict__ M) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nint = (long)C.n[0] * C.n[1] * C.n[2];
  if (t >= nint) return;
  const int i = C.ng[0] + t % C.n[0];
  const long t2 = t / C.n[0];
  const int j = C.ng[1] + t2 % C.n[1];
  const int k = C.ng[2] + t2 / C.n[1];
  const long c = cell_index(C, i, j, k);
  const double gdt = g * (*dt_dev);
  const bool bad = (status[c] & GRRMHD_ST_FAIL) != 0;
#pragma unroll
  for (int r = 0; r < 8; r++) {
    const int q = (r < 4) ? 1 + r : 4 + r;
    M[r * C.Ntot + c] = bad ? 0.0 : (Uo[q * C.Ntot + c] - Ue[q * C.Ntot + c]) / gdt;
  }
}

// The entropy tracer in the IMEX tables: a stage's bracket adds
// dt sum_k m_k M_S^k (MT's arrays: [N] each), and an implicit stage stores
// M_S = (U_S(P_out) - explicit)/(g dt) from its solution before the fix-ups
// (zero where the solve failed), as k_stage_m the other sources.
__global__ void LB(256) k_entropy_mterms(Ctx C, MTerms MT, const double* __restrict__ dt_dev,
                                         double* __restrict__ Sexp) {
  int i, j, k;
  if (!interior_ijk(C, (long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
  const long c = cell_index(C, i, j, k);
  double sm = 0.0;
  for (int q = 0; q < MT.n; q++) sm += MT.m[q] * MT.M[q][c];
  Sexp[c] += (*dt_dev) * sm;
}

__global__ void LB(256) k_stage_ms(Ctx C, const double* __restrict__ Po,
                                   const double* __restrict__ Sexp, const int* __restrict__ status,
                                   double g, const double* __restrict__ dt_dev,
                                   double* __restrict__ MS) {
  int i, j, k;
  if (!interior_ijk(C, (long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
  const long c = cell_index(C, i, j, k);
  if (status[c] & GRRMHD_ST_FAIL) {
    MS[c] = 0.0;
    return;
  }
  Metric m;
  load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
  double p[5];
#pragma unroll
  for (int q = 0; q < 5; q++) p[q] = Po[q * C.Ntot + c];
  MS[c] = (entropy_cons(C.gam, m, p) - Sexp[c]) / (g * (*dt_dev));
}

// ---------------------------------------------------------------------------
// step 13 and floors (Sec. 4.11).  Pass 1 averages the face neighbours of
// failed and cold cells into scratch (neighbours with a good energy solution,
// else all); pass 2 applies them (all primitives of a failed cell, u_g alone
// of a cold one) and the floors, and recomputes U where P changed.
// ---------------------------------------------------------------------------
DEV void fixup_avg_at(Ctx C, const double* __restrict__ P,
                                    const int* __restrict__ status, double* __restrict__ scr, long t) {
  const long nint = (long)C.n[0] * C.n[1] * C.n[2];
  if (t >= nint) return;
  int idx[3];
  idx[0] = C.ng[0] + t % C.n[0];
  const long t2 = t / C.n[0];
  idx[1] = C.ng[1] + t2 % C.n[1];
  idx[2] = C.ng[2] + t2 / C.n[1];
  const long c = cell_index(C, idx[0], idx[1], idx[2]);
  if (!(status[c] & (GRRMHD_ST_FAIL | GRRMHD_ST_COLD))) return;
  for (int pass = 0; pass < 2; pass++) {
    double acc[12];
#pragma unroll
    for (int q = 0; q < 12; q++) acc[q] = 0.0;
    int cnt = 0;
    for (int d = 0; d < 3; d++) {
      if (C.n[d] == 1) continue;
      for (int s = -1; s <= 1; s += 2) {
        const int nid = idx[d] + s;
        if (nid < C.ng[d] || nid >= C.ng[d] + C.n[d]) continue;
        const long nb = c + s * C.st[d];
        if (pass == 0 && (status[nb] & (GRRMHD_ST_FAIL | GRRMHD_ST_COLD))) continue;
#pragma unroll
        for (int q = 0; q < 12; q++) acc[q] += P[q * C.Ntot + nb];
        cnt++;
      }
    }
    if (cnt > 0) {
      const double w = 1.0 / cnt;
#pragma unroll
      for (int q = 0; q < 12; q++) scr[q * C.Ntot + c] = acc[q] * w;
      scr[12 * C.Ntot + c] = pass + 1.0;
      return;
    }
  }
  scr[12 * C.Ntot + c] = 0.0;
}

__global__ void LB(256) k_fixup_avg(Ctx C, const double* __restrict__ P,
                                    const int* __restrict__ status, double* __restrict__ scr) {
  fixup_avg_at(C, P, status, scr, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

DEV void fixup_apply_at(Ctx C, double* __restrict__ P, double* __restrict__ U,
                                      int* __restrict__ status, const double* __restrict__ scr,
                                      int* __restrict__ st_acc, const int* __restrict__ it_stage,
                                      int* __restrict__ it_acc, int accumulate, long t) {
  const long nint = (long)C.n[0] * C.n[1] * C.n[2];
  if (t >= nint) return;
  const int i = C.ng[0] + t % C.n[0];
  const long t2 = t / C.n[0];
  const int j = C.ng[1] + t2 % C.n[1];
  const int k = C.ng[2] + t2 / C.n[1];
  const long c = cell_index(C, i, j, k);
  int st = status[c];
  double p[12];
  bool changed = false;
  const bool fail = (st & GRRMHD_ST_FAIL) != 0;
  const bool cold = !fail && (st & GRRMHD_ST_COLD);
  Metric m;
  load_metric(C.geo_c, C.npos, i + C.N[0] * j, m);
  if ((fail || cold) && scr[12 * C.Ntot + c] > 0.0) {
    // failed: the neighbours' mean primitives; cold: their mean u_g alone
#pragma unroll
    for (int q = 0; q < 12; q++) {
      // a staggered field is not a primitive of the solve: the cell keeps its B
      const bool avg = (fail && !(C.ct && q >= 5 && q <= 7)) || q == 1;
      p[q] = avg ? scr[q * C.Ntot + c] : P[q * C.Ntot + c];
    }
    if (scr[12 * C.Ntot + c] > 1.5) st |= GRRMHD_ST_NO_GOOD_NB;
    changed = true;
  } else {
#pragma unroll
    for (int q = 0; q < 12; q++) p[q] = P[q * C.Ntot + c];
  }
  // the staggered field of a failed cell: the stage's own (its conserved
  // field over sqrt(-g), the mean of its new faces), not the guess that a
  // failed solve or inversion returned
  const bool bnew = fail && C.ct;
  if (bnew) {
#pragma unroll
    for (int q = 5; q <= 7; q++) p[q] = U[q * C.Ntot + c] / m.gdet;
  }
  Gas<double> s;
  make_gas(m, C.gam, p[0], p[1], p + 2, p + 5, s);
  const double rmin = fmax(C.rho_floor, s.bsq / C.bsq_rho_max);
  const double umin = fmax(C.u_floor, s.bsq / C.bsq_u_max);
  bool fl = false;
  if (p[0] < rmin) { p[0] = rmin; fl = true; }
  if (p[1] < umin) { p[1] = umin; fl = true; }
  if (p[1] > C.u_rho_max * p[0]) { p[1] = C.u_rho_max * p[0]; fl = true; }
  if (!(p[8] >= C.erad_floor)) { p[8] = C.erad_floor; fl = true; }
  if (fl) st |= GRRMHD_ST_FLOOR;
  if (fl || changed) {
    double u[12];
    prim_to_cons_cell(m, C.gam, p, u);
#pragma unroll
    for (int q = 0; q < 12; q++) {
      P[q * C.Ntot + c] = p[q];
      U[q * C.Ntot + c] = u[q];
    }
  } else if (bnew) {
#pragma unroll
    for (int q = 5; q <= 7; q++) P[q * C.Ntot + c] = p[q];
  }
  status[c] = st;
  if (st_acc) st_acc[c] = accumulate ? (st_acc[c] | st) : st;
  if (it_acc && it_stage) it_acc[c] = accumulate ? it_acc[c] + it_stage[c] : it_stage[c];
}

__global__ void LB(256) k_fixup_apply(Ctx C, double* __restrict__ P, double* __restrict__ U,
                                      int* __restrict__ status, const double* __restrict__ scr,
                                      int* __restrict__ st_acc, const int* __restrict__ it_stage,
                                      int* __restrict__ it_acc, int accumulate) {
  fixup_apply_at(C, P, U, status, scr, st_acc, it_stage, it_acc, accumulate, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Batched implicit solve, persistent and per-iteration forms.
//
// Persistent: a fixed grid of waves; each lane runs the resumable PMHD
// attempt and, whenever its cell ends, takes the next cell from a global
// queue (one atomic per wavefront), so unconverged cells stay packed in the
// lanes whatever the spread of Newton counts.  Per-iteration: one launch per
// Newton trip, the lane state kept in HBM and the still-active cells
// compacted into the next launch's queue.  Cells that need the full cascade
// go to the same work list as in k_implicit_batch.
// ---------------------------------------------------------------------------
#define LBP __launch_bounds__(256, 1)

DEV void setup_cell(const Metric& m, const double Ui[12], double dt, double ca, double ce, Cell& c) {
  cell_setup(m, Ui, dt, ca, ce, c);
}


DEV void finish_lane(const Cell& c, const Phys& ph, const Opts& o, Lane& L, double U0,
                     const double UB[3], long cidx, long nst, double* P, double* U, int* iters,
                     int* status, double* err) {
  double Uk[12];
#pragma unroll
  for (int q = 0; q < 12; q++) Uk[q] = 0.0;
  Uk[0] = U0;
  Uk[5] = UB[0]; Uk[6] = UB[1]; Uk[7] = UB[2];
  CellOut out;
  finalize(c, ph, o, L.best, M_PMHD, L.status, L.iters, Uk, out);
  store_out(out, cidx, nst, P, U, iters, status, err);
}

__global__ void LBP k_implicit_persist(Ctx C, long n, const double* __restrict__ Ui_,
                                       const double* __restrict__ Pg_,
                                       const double* __restrict__ dtc,
                                       const double* __restrict__ chi_abs,
                                       const double* __restrict__ chi_es,
                                       double* __restrict__ Po, double* __restrict__ Uo,
                                       int* __restrict__ iters, int* __restrict__ status,
                                       double* __restrict__ err, int* next, Work W) {
  const Phys ph = make_phys(C);
  const Opts o = make_opts(C);
  const double thr = accept_threshold(o);
  Metric m;
  flat_metric(m);
  Lane L;
  Cell c;
  double U0 = 0.0, UB[3] = {0.0, 0.0, 0.0};
  long item = -1;
  bool active = false, exhausted = false;
  unsigned long long useful = 0, slots = 0;
  for (;;) {
    const bool need = !active && !exhausted;
    const long got = wave_fetch(need, next);
    bool first = false, tolist = false;
    if (need) {
      if (got < n) {
        item = got;
        double Ui[12], Pg[12];
#pragma unroll
        for (int q = 0; q < 12; q++) {
          Ui[q] = Ui_[q * n + item];
          Pg[q] = Pg_[q * n + item];
        }
        Prep pr;
        prepare(m, ph, Ui, Pg, dtc[item], chi_abs[item], chi_es[item], c, pr);
        U0 = Ui[0];
        UB[0] = Ui[5]; UB[1] = Ui[6]; UB[2] = Ui[7];
        L.status = pr.status;
        if (pr.extreme) {
          tolist = true;
        } else {
          L.x[0] = pr.Pthin[1]; L.x[1] = pr.Pthin[2]; L.x[2] = pr.Pthin[3]; L.x[3] = pr.Pthin[4];
          active = true;
          first = true;
        }
      } else {
        exhausted = true;
      }
    }
    bool ended = false, doeval = first;
    double xprev[4] = {L.x[0], L.x[1], L.x[2], L.x[3]};
    if (active && !first) {
      ended = lane_step(c, o, L);
      doeval = !ended;
    }
    if (doeval) {
      // one evaluation call site for new and continuing lanes (a new lane's
      // first evaluation is a full one), so a wave never runs two of them
      Eval ev;
      if (first) L.chord = 0;
      lane_eval(c, ph, L, ev);
      if (first) {
        lane_start(ev, L);
        if (!ev.ok) ended = true;
      } else {
        lane_take(ev, L);
        ended = lane_after(ev, xprev, L);
      }
    }
    const unsigned long long ev_mask = __ballot(doeval);
    useful += __popcll(ev_mask);
    slots += ev_mask ? 64ull : 0ull;
    bool extreme = tolist;
    if (ended) {
      if (L.best.ok && L.best.eT < thr)
        finish_lane(c, ph, o, L, U0, UB, item, n, Po, Uo, iters, status, err);
      else
        tolist = true;
      active = false;
    }
    to_cascade(tolist, extreme, (int)item, L.best, L.iters, W);
    if (!__any(active) && __all(exhausted)) break;
  }
  if ((threadIdx.x & 63) == 0 && useful) {
    atomicAdd(&W.stats[0], useful);
    atomicAdd(&W.stats[1], slots);
  }
}

// Lane state kept in HBM between per-iteration launches, field-major [f][n].
enum { LS_X = 0, LS_EG = 4, LS_ET = 8, LS_J = 9, LS_BX = 25, LS_BP = 29, LS_BET = 41, LS_H = 42,
       LS_ND = 47 };
enum { LI_BRAD = 0, LI_BOK, LI_IT, LI_NRISE, LI_EXTRA, LI_CONV, LI_ITERS, LI_STATUS, LI_PIV,
       LI_FRESH = LI_PIV + 4, LI_NI };

DEV void lane_save(const Lane& L, long c, long n, double* sd, int* si) {
#pragma unroll
  for (int k = 0; k < 4; k++) {
    sd[(LS_X + k) * n + c] = L.x[k];
    sd[(LS_EG + k) * n + c] = L.Eg[k];
    sd[(LS_BX + k) * n + c] = L.best.x[k];
#pragma unroll
    for (int j = 0; j < 4; j++) sd[(LS_J + 4 * k + j) * n + c] = L.J[k][j];
  }
  sd[LS_ET * n + c] = L.eT;
#pragma unroll
  for (int q = 0; q < 12; q++) sd[(LS_BP + q) * n + c] = L.best.P[q];
  sd[LS_BET * n + c] = L.best.eT;
#pragma unroll
  for (int k = 0; k < 5; k++) sd[(LS_H + k) * n + c] = L.h[k];
  si[LI_BRAD * n + c] = L.best.radflags;
  si[LI_BOK * n + c] = L.best.ok;
  si[LI_IT * n + c] = L.it;
  si[LI_NRISE * n + c] = L.nrise;
  si[LI_EXTRA * n + c] = L.extra;
  si[LI_CONV * n + c] = L.conv;
  si[LI_ITERS * n + c] = L.iters;
  si[LI_STATUS * n + c] = L.status;
#pragma unroll
  for (int k = 0; k < 4; k++) si[(LI_PIV + k) * n + c] = L.piv[k];
  si[LI_FRESH * n + c] = L.fresh;
}

DEV void lane_load(Lane& L, long c, long n, const double* sd, const int* si) {
#pragma unroll
  for (int k = 0; k < 4; k++) {
    L.x[k] = sd[(LS_X + k) * n + c];
    L.Eg[k] = sd[(LS_EG + k) * n + c];
    L.best.x[k] = sd[(LS_BX + k) * n + c];
#pragma unroll
    for (int j = 0; j < 4; j++) L.J[k][j] = sd[(LS_J + 4 * k + j) * n + c];
  }
  L.eT = sd[LS_ET * n + c];
#pragma unroll
  for (int q = 0; q < 12; q++) L.best.P[q] = sd[(LS_BP + q) * n + c];
  L.best.eT = sd[LS_BET * n + c];
#pragma unroll
  for (int k = 0; k < 5; k++) L.h[k] = sd[(LS_H + k) * n + c];
  L.best.radflags = si[LI_BRAD * n + c];
  L.best.ok = si[LI_BOK * n + c];
  L.it = si[LI_IT * n + c];
  L.nrise = si[LI_NRISE * n + c];
  L.extra = si[LI_EXTRA * n + c];
  L.conv = si[LI_CONV * n + c];
  L.iters = si[LI_ITERS * n + c];
  L.status = si[LI_STATUS * n + c];
#pragma unroll
  for (int k = 0; k < 4; k++) L.piv[k] = si[(LI_PIV + k) * n + c];
  L.fresh = si[LI_FRESH * n + c];
  L.chord = 0;
}

// first trip of every cell: guess, first evaluation; active cells to queue
__global__ void LB(64) k_iter_start(Ctx C, long n, const double* __restrict__ Ui_,
                                    const double* __restrict__ Pg_, const double* __restrict__ dtc,
                                    const double* __restrict__ chi_abs,
                                    const double* __restrict__ chi_es, double* sd, int* si,
                                    int* qcount, int* queue, Work W) {
  const long cidx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false, tolist = false, extreme = false;
  int trips = 0;
  Lane L;
  if (cidx < n) {
    const Phys ph = make_phys(C);
    Metric m;
    flat_metric(m);
    double Ui[12], Pg[12];
#pragma unroll
    for (int q = 0; q < 12; q++) {
      Ui[q] = Ui_[q * n + cidx];
      Pg[q] = Pg_[q * n + cidx];
    }
    Cell c;
    Prep pr;
    prepare(m, ph, Ui, Pg, dtc[cidx], chi_abs[cidx], chi_es[cidx], c, pr);
    L.status = pr.status;
    if (pr.extreme) {
      tolist = true;
      extreme = true;
    } else {
      L.x[0] = pr.Pthin[1]; L.x[1] = pr.Pthin[2]; L.x[2] = pr.Pthin[3]; L.x[3] = pr.Pthin[4];
      Eval ev;
      eval_pmhd(c, ph, L.x, ev, L.J);
      lane_start(ev, L);
      trips = 1;
      if (ev.ok) act = true;
      else tolist = true;
      lane_save(L, cidx, n, sd, si);
    }
  }
  wave_stats(trips, W.stats);
  wave_append(act, (int)cidx, qcount, queue);
  to_cascade(tolist, extreme, (int)cidx, L.best, L.iters, W);
}

// one Newton trip for every queued cell
__global__ void LB(64) k_iter_step(Ctx C, long n, const double* __restrict__ Ui_,
                                   const double* __restrict__ dtc,
                                   const double* __restrict__ chi_abs,
                                   const double* __restrict__ chi_es, double* sd, int* si,
                                   const int* qin_count, const int* qin, int* qout_count,
                                   int* qout, double* __restrict__ Po, double* __restrict__ Uo,
                                   int* __restrict__ iters, int* __restrict__ status,
                                   double* __restrict__ err, Work W) {
  const int cnt = *qin_count;
  const long stride = (long)gridDim.x * blockDim.x;
  const long rounds = (cnt + stride - 1) / stride;
  for (long r = 0; r < rounds; r++) {
    const long w = r * stride + (long)blockIdx.x * blockDim.x + threadIdx.x;
    bool keepgoing = false, tolist = false;
    long cidx = -1;
    int trips = 0;
    Lane L;
    if (w < cnt) {
      cidx = qin[w];
      const Phys ph = make_phys(C);
      const Opts o = make_opts(C);
      Metric m;
      flat_metric(m);
      double Ui[12];
#pragma unroll
      for (int q = 0; q < 12; q++) Ui[q] = Ui_[q * n + cidx];
      Cell c;
      setup_cell(m, Ui, dtc[cidx], chi_abs[cidx], chi_es[cidx], c);
      lane_load(L, cidx, n, sd, si);
      double xprev[4] = {L.x[0], L.x[1], L.x[2], L.x[3]};
      bool ended = lane_step(c, o, L);
      if (!ended) {
        trips = 1;
        Eval ev;
        lane_eval(c, ph, L, ev);
        lane_take(ev, L);
        ended = lane_after(ev, xprev, L);
      }
      if (ended) {
        if (L.best.ok && L.best.eT < accept_threshold(o)) {
          const double UB[3] = {Ui[5], Ui[6], Ui[7]};
          finish_lane(c, ph, o, L, Ui[0], UB, cidx, n, Po, Uo, iters, status, err);
        } else {
          tolist = true;
        }
      } else {
        lane_save(L, cidx, n, sd, si);
        keepgoing = true;
      }
    }
    wave_stats(trips, W.stats);
    wave_append(keepgoing, (int)cidx, qout_count, qout);
    to_cascade(tolist, false, (int)cidx, L.best, L.iters, W);
  }
}
