// Conserved-to-primitive inversions on the device.
//   MHD (Sec. 4.5): Newton iteration on the single unknown W' = W - D of the
//   energy relation (eq. EMHD with v~^2(W) of eq. vsqeq), derivative by a
//   one-direction dual number; when Newton leaves the admissible region or
//   stalls, a bracket [W'(chi = 0), gam (E' - Bsq/2)] is built and bisected.
//   RAD (Sec. 4.6): analytic y -> gamma_rad^2 -> p_rad -> v~_rad with the
//   BASIC or TYPE2 limiter; templated so derivatives flow through it.
#pragma once
#include <type_traits>

#include "physics.h"

// spatial inverse metric of the normal observer: g^{ij} - g^{ti} g^{tj}/g^{tt}
DEV double gamup(const Metric& m, int i, int j) {
  return m.up(i + 1, j + 1) - m.up(0, i + 1) * m.up(0, j + 1) / m.up(0, 0);
}

// ---------------------------------------------------------------------------
// M1 radiation inversion.  Input R^t_nu (no sqrt(-g)).  Output Ebar, u~_rad.
// Returns bit 0 if E_rad <= 0 was met, bit 1 if y >= y_max.
// ---------------------------------------------------------------------------
template <class T>
DEV int rad_invert(const Metric& m, double gamma_max, double ymax, int type2, const T R[4],
                   T& Ebar, T ut[3]) {
  const double a = m.alpha, a2 = a * a;
  // E_rad = -eta^mu alpha R^t_mu; U~^i = gamma^{ij} alpha R^t_j (eq. RADPRIM2, RADPRIM3)
  const T Erad = -R[0] + a2 * (m.up(0, 1) * R[1] + m.up(0, 2) * R[2] + m.up(0, 3) * R[3]);
  T Ut[3];
#pragma unroll
  for (int i = 0; i < 3; i++) Ut[i] = a * (gamup(m, i, 0) * R[1] + gamup(m, i, 1) * R[2] + gamup(m, i, 2) * R[3]);
  const T Ut2 = a * (Ut[0] * R[1] + Ut[1] * R[2] + Ut[2] * R[3]);
  const double G2 = gamma_max * gamma_max;
  const double Ev = val(Erad), U2v = val(Ut2);
  const double yv = (Ev != 0.0) ? U2v / (Ev * Ev) : 0.0;
  int flags = (Ev <= 0.0) ? 1 : 0;
  if (Ev > 0.0 && yv >= ymax) flags |= 2;
  if (flags) {
    if (!type2 && Ev <= 0.0) {               // BASIC: no radiation left
      Ebar = T(1e-300);
      ut[0] = ut[1] = ut[2] = T(0.0);
      return flags;
    }
    // keep the direction of U~, cap the Lorentz factor at gamma_max.
    // BASIC keeps E_rad; TYPE2 keeps the momentum and sets E_rad so y = y_max.
    if (U2v > 0.0) {
      const T E2 = type2 ? T(1e-150) + sqrt(Ut2 * (1.0 / ymax)) : Erad;
      const T prad = E2 * (1.0 / (4.0 * G2 - 1.0));
      const T s = sqrt((G2 - 1.0) / Ut2);
      Ebar = 3.0 * prad;
#pragma unroll
      for (int i = 0; i < 3; i++) ut[i] = s * Ut[i];
    } else {
      Ebar = T(1e-150);
      ut[0] = ut[1] = ut[2] = T(0.0);
    }
    return flags;
  }
  if (yv <= 0.0) {                            // gamma_rad = 1
    Ebar = Erad;
    if constexpr (std::is_same<T, double>::value) {
      ut[0] = ut[1] = ut[2] = 0.0;
    } else {
      // zero flux: u~ = 3 U~ / (4 E_rad) to first order, so derivatives
      // with respect to the flux survive
#pragma unroll
      for (int i = 0; i < 3; i++) ut[i] = Ut[i] * (0.75 / val(Erad));
    }
    return flags;
  }
  // eq. ysol, gammarvsy, prsol, tvrsol
  const T y = Ut2 / (Erad * Erad);
  const T g2 = (2.0 - y + sqrt(4.0 - 3.0 * y)) / (4.0 * (1.0 - y));
  const T prad = Erad / (4.0 * g2 - 1.0);
  const T f = sqrt(g2) / (4.0 * prad * g2);
  Ebar = 3.0 * prad;
#pragma unroll
  for (int i = 0; i < 3; i++) ut[i] = f * Ut[i];
  return flags;
}

// ---------------------------------------------------------------------------
// MHD inversion
// ---------------------------------------------------------------------------
// Constants of eq. EMHD; those that depend on the conserved energy and
// momentum have the scalar type C (double, or dual numbers carrying their
// derivatives with respect to upstream unknowns).
template <class C>
struct MhdCT {
  double D, Bsq, gam;
  C Ep, Qt2, S;
  C Qt[3];
  double Bz[3];
};
using MhdC = MhdCT<double>;

// residual of eq. EMHD in W' and chi = u + p; templated for the derivative
template <class T, class C>
DEV T mhd_f(const MhdCT<C>& c, const T& Wp, T& chi, T& gamma) {
  const T W = Wp + c.D;
  const T a = c.Bsq + W;
  const T W2 = W * W;
  const T vsq = (c.Qt2 * W2 + c.S * c.S * (c.Bsq + 2.0 * W)) / (a * a * W2);
  const T gsq = 1.0 / (1.0 - vsq);
  gamma = sqrt(gsq);
  chi = (Wp - c.D * (gsq * vsq) / (1.0 + gamma)) / gsq;   // eq. Wprime, gamma-1 = u~^2/(1+gamma)
  const T pg = ((c.gam - 1.0) / c.gam) * chi;
  return Wp - pg + 0.5 * c.Bsq * (1.0 + vsq) - 0.5 * c.S * c.S / W2 - c.Ep;
}

DEV double mhd_vsq(const MhdC& c, double W) {
  const double a = c.Bsq + W;
  return (c.Qt2 * W * W + c.S * c.S * (c.Bsq + 2.0 * W)) / (a * a * W * W);
}

// Narrows a bracket [lo, hi] of the root of g(W') = f (KIND 0) or chi
// (KIND 1), both increasing on the admissible region, by Newton steps from
// the last point (the midpoint whenever a step would leave the bracket);
// the bisection that follows takes it to adjacent doubles as before, in a
// few steps instead of ~60.  KIND 1 keeps chi > 0 at hi (chi = 0 goes low).
template <int KIND>
DEV void mhd_narrow(const MhdC& c, double& lo, double& hi) {
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 40; it++) {
    Dual<1> chi, gm;
    const Dual<1> f = mhd_f<Dual<1>>(c, Dual<1>::var(x, 0), chi, gm);
    const Dual<1> g = (KIND == 0) ? f : chi;
    if (!isfinite(g.v) || !isfinite(g.d[0])) return;
    if (KIND == 0 && g.v == 0.0) {
      lo = hi = x;
      return;
    }
    if (g.v > 0.0) hi = x;
    else lo = x;
    if (!(hi - lo > 8.0 * DBL_EPSILON * ::fabs(hi))) return;
    double xn = (g.d[0] != 0.0) ? x - g.v / g.d[0] : lo;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    x = xn;
  }
}

// Bracketed bisection: the admissible region is v~^2 < 1 and chi > 0; on it
// the root is bracketed by W0' (chi = 0) and gam (E' - Bsq/2).
DEV int mhd_bisect(const MhdC& c, double& Wp_out) {
  double a0 = 0.0;
  if (mhd_vsq(c, c.D) >= 1.0) {
    double lo = 0.0, hi = 1.0 + c.Ep + ::sqrt(c.Qt2) + c.Bsq;
    for (int it = 0; it < 200 && mhd_vsq(c, c.D + hi) >= 1.0; it++) hi *= 2.0;
    for (int it = 0; it < 200; it++) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (mhd_vsq(c, c.D + mid) >= 1.0) lo = mid; else hi = mid;
    }
    a0 = hi;
  }
  double chi, gm;
  double hi = fmax(c.gam * (c.Ep - 0.5 * c.Bsq), 0.0) * (1.0 + 1e-12) + 1e-300;
  if (hi < a0) hi = a0;
  for (int it = 0; it < 200 && mhd_f<double>(c, hi, chi, gm) < 0.0; it++) hi = 2.0 * hi + 1e-300;
  double nb = hi;
  for (int it = 0; it < 200; it++) {
    mhd_f<double>(c, nb, chi, gm);
    if (chi > 0.0) break;
    nb = 2.0 * nb + 1e-300;
  }
  double na = a0;
  mhd_narrow<1>(c, na, nb);
  for (int it = 0; it < 200; it++) {
    const double mid = 0.5 * (na + nb);
    if (mid <= na || mid >= nb) break;
    mhd_f<double>(c, mid, chi, gm);
    if (chi > 0.0) nb = mid; else na = mid;
  }
  double lo = nb;
  if (!(lo <= hi) || !(mhd_f<double>(c, lo, chi, gm) < 0.0)) return 1;
  mhd_narrow<0>(c, lo, hi);
  for (int it = 0; it < 200; it++) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double fm = mhd_f<double>(c, mid, chi, gm);
    if (fm == 0.0) { lo = hi = mid; break; }
    if (fm < 0.0) lo = mid; else hi = mid;
  }
  const double flo = ::fabs(mhd_f<double>(c, lo, chi, gm));
  const double fhi = ::fabs(mhd_f<double>(c, hi, chi, gm));
  Wp_out = (flo <= fhi) ? lo : hi;
  return 0;
}

// Constants of eq. EMHD from rho u^t, E_gas = T^t_t + rho u^t, T^t_i, B^i
// (all without sqrt(-g)), eq. PRIM1 and the normal-observer projections.
template <class C>
DEV void mhd_consts(const Metric& m, double gam, double rhout, const C& Eg, const C Tt[3],
                    const double B[3], MhdCT<C>& c) {
  const double al = m.alpha;
  c.gam = gam;
  c.D = al * rhout;                                                       // eq. PRIM1
  c.Ep = -Eg + rhout * (1.0 - al) + al * al * (m.up(0, 1) * Tt[0] + m.up(0, 2) * Tt[1] + m.up(0, 3) * Tt[2]);
  c.Qt2 = C(0.0);
  c.S = C(0.0);
  c.Bsq = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    c.Qt[i] = al * (gamup(m, i, 0) * Tt[0] + gamup(m, i, 1) * Tt[1] + gamup(m, i, 2) * Tt[2]);
    c.Bz[i] = al * B[i];
  }
#pragma unroll
  for (int i = 0; i < 3; i++) {
    c.Qt2 = c.Qt2 + c.Qt[i] * al * Tt[i];
    c.S = c.S + al * Tt[i] * c.Bz[i];
#pragma unroll
    for (int j = 0; j < 3; j++) c.Bsq += m.lo(i + 1, j + 1) * c.Bz[i] * c.Bz[j];
  }
}

// The root W' of eq. EMHD: Newton from the guess primitives (W' = D u~^2/(1+gamma)
// + chi gamma^2), bracketed bisection when Newton leaves the admissible
// region or stalls.  0 on success (with chi > 0 at the root), 1 otherwise.
DEV int mhd_solve(const Metric& m, const MhdC& c, double ug_g, const double ut_g[3], double& Wp) {
  if (!(c.D > 0.0) || !(c.Ep > 0.0) || !isfinite(c.Ep) || !isfinite(c.Qt2)) return 1;
  {
    double q = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) q += m.lo(i + 1, j + 1) * ut_g[i] * ut_g[j];
    const double g = ::sqrt(1.0 + q);
    Wp = c.D * q / (1.0 + g) + c.gam * ug_g * (1.0 + q);
  }
  bool ok = isfinite(Wp) && Wp > 0.0;
  int conv = 0;
  double dprev = INFINITY;
  if (ok) {
    for (int it = 0; it < 60; it++) {
      Dual<1> chi, gm;
      const Dual<1> f = mhd_f<Dual<1>>(c, Dual<1>::var(Wp, 0), chi, gm);
      if (!(f.d[0] > 0.0) || !isfinite(f.v)) { ok = false; break; }
      double Wn = Wp - f.v / f.d[0];
      if (!(Wn > 0.0) || mhd_vsq(c, Wn + c.D) >= 1.0) {
        Wn = 0.5 * Wp;                                     // stay admissible
        if (mhd_vsq(c, Wn + c.D) >= 1.0) { ok = false; break; }
      }
      const double dW = ::fabs(Wn - Wp);
      Wp = Wn;
      if (dW <= 2.0 * DBL_EPSILON * Wp) { conv++; if (conv >= 2) break; }
      else conv = 0;
      // at the rounding floor of f: a step already below 1e-12 W' that no
      // longer shrinks is noise of the residual, not progress (a few cells
      // otherwise circle the root for all 60 steps and then bisect)
      if (conv == 0 && dW <= 1e-12 * Wp && dW >= dprev) break;
      dprev = dW;
      if (it == 59) ok = false;
    }
  }
  if (ok) {
    double chi, gm;
    mhd_f<double>(c, Wp, chi, gm);
    if (!(chi > 0.0)) ok = false;
  }
  if (!ok && mhd_bisect(c, Wp)) return 1;
  return 0;
}

// Primitives rho, u_g, u~^i at W' (eq. tveq, rho = D/gamma, u_g = chi/gam)
template <class T, class C>
DEV void mhd_prims(const MhdCT<C>& c, const T& Wp, T& rho, T& ug, T ut[3]) {
  T chi, gm;
  mhd_f<T>(c, Wp, chi, gm);
  const T W = Wp + c.D;
  const T iw = 1.0 / (W + c.Bsq);
#pragma unroll
  for (int i = 0; i < 3; i++) ut[i] = gm * (c.Qt[i] + c.S * c.Bz[i] / W) * iw;   // eq. tveq
  rho = c.D / gm;
  ug = chi / c.gam;
}

// Gas primitives from rho u^t, E_gas = T^t_t + rho u^t, T^t_i, B^i (all
// without sqrt(-g)).  The guess supplies the starting W'.  Writes rho, u_g,
// u~^i.  Returns 0 on success, 1 without a physical (u_g > 0) root.
DEV int mhd_invert(const Metric& m, double gam, double rhout, double Eg, const double Tt[3],
                   const double B[3], double& rho_g, double& ug_g, double ut_g[3]) {
  MhdC c;
  mhd_consts(m, gam, rhout, Eg, Tt, B, c);
  double Wp;
  if (mhd_solve(m, c, ug_g, ut_g, Wp)) return 1;
  mhd_prims(c, Wp, rho_g, ug_g, ut_g);
  return (ug_g > 0.0) ? 0 : 1;
}

// The same inversion as a function of upstream unknowns carried by dual
// numbers: the root W' in double precision, then its derivative from the
// implicit-function theorem on eq. EMHD, dW' = -(df/dc . dc) / (df/dW'),
// and the primitives' derivatives through eq. tveq.
template <int N>
DEV int mhd_invert_dual(const Metric& m, double gam, double rhout, const Dual<N>& Eg,
                        const Dual<N> Tt[3], const double B[3], double ug_g, const double ut_g[3],
                        Dual<N>& rho, Dual<N>& ug, Dual<N> ut[3]) {
  using D = Dual<N>;
  MhdCT<D> cd;
  mhd_consts(m, gam, rhout, Eg, Tt, B, cd);
  MhdC cv;
  cv.D = cd.D;
  cv.Bsq = cd.Bsq;
  cv.gam = cd.gam;
  cv.Ep = cd.Ep.v;
  cv.Qt2 = cd.Qt2.v;
  cv.S = cd.S.v;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    cv.Qt[i] = cd.Qt[i].v;
    cv.Bz[i] = cd.Bz[i];
  }
  double Wp;
  if (mhd_solve(m, cv, ug_g, ut_g, Wp)) return 1;
  D chi, gm;
  const D f = mhd_f<D>(cd, D(Wp), chi, gm);            // df/dc . dc at fixed W'
  Dual<1> chi1, gm1;
  const Dual<1> fw = mhd_f<Dual<1>>(cv, Dual<1>::var(Wp, 0), chi1, gm1);
  if (!(fw.d[0] != 0.0) || !isfinite(fw.d[0])) return 1;
  const double ifw = 1.0 / fw.d[0];
  D Wd(Wp);
#pragma unroll
  for (int j = 0; j < N; j++) Wd.d[j] = -f.d[j] * ifw;
  mhd_prims(cd, Wd, rho, ug, ut);
  return (ug.v > 0.0) ? 0 : 1;
}
