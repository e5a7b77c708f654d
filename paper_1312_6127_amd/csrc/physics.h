// Pointwise GRRMHD + M1 physics on the device.  Templated on the scalar so
// the same code yields values (double, or float on the FP32 face path) or
// values with exact derivatives (Dual<N>).  Only the tensor rows a caller
// needs are formed.
#pragma once
#include "common.h"

// ---------------------------------------------------------------------------
// 4-velocity from the normal-observer-relative velocity (Sec. 2 and 4.5):
// gamma = sqrt(1 + g_ij u~^i u~^j); u^t = gamma/alpha; u^i = u~^i - gamma alpha g^{ti}
// ---------------------------------------------------------------------------
template <class T>
struct Vel {
  T ucon[4], ucov[4];
  T gamma;
  T usq;   // g_ij u~^i u~^j
};

template <class T>
DEV void make_vel(const MetricT<typename RealOf<T>::type>& m, const T ut[3], Vel<T>& v) {
  using R = typename RealOf<T>::type;
  T q = T(R(0.0));
#pragma unroll
  for (int i = 0; i < 3; i++) {
    q = q + m.lo(i + 1, i + 1) * ut[i] * ut[i];
#pragma unroll
    for (int j = i + 1; j < 3; j++) q = q + R(2.0) * m.lo(i + 1, j + 1) * ut[i] * ut[j];
  }
  v.usq = q;
  v.gamma = sqrt(R(1.0) + q);
  const T ga = v.gamma * m.alpha;
  v.ucon[0] = v.gamma / m.alpha;
#pragma unroll
  for (int i = 0; i < 3; i++) v.ucon[i + 1] = ut[i] - ga * m.up(0, i + 1);
#pragma unroll
  for (int a = 0; a < 4; a++) {
    T s = m.lo(a, 0) * v.ucon[0];
#pragma unroll
    for (int b = 1; b < 4; b++) s = s + m.lo(a, b) * v.ucon[b];
    v.ucov[a] = s;
  }
}

// gas state: velocity, fluid-frame field b^mu = B^nu h^mu_nu / u^t (Sec. 2)
template <class T>
struct Gas {
  Vel<T> v;
  T rho, ug, pg;
  T bcon[4], bcov[4], bsq;
  T opu;   // 1 + u_t, free of the rest-mass cancellation
};

template <class T>
DEV void make_gas(const MetricT<typename RealOf<T>::type>& m, double gam, const T& rho,
                  const T& ug, const T ut[3], const T B[3], Gas<T>& s) {
  using R = typename RealOf<T>::type;
  make_vel(m, ut, s.v);
  s.rho = rho;
  s.ug = ug;
  s.pg = R(gam - 1.0) * ug;
  T bt = B[0] * s.v.ucov[1] + B[1] * s.v.ucov[2] + B[2] * s.v.ucov[3];
  s.bcon[0] = bt;
  const T iut = R(1.0) / s.v.ucon[0];
#pragma unroll
  for (int i = 0; i < 3; i++) s.bcon[i + 1] = (B[i] + bt * s.v.ucon[i + 1]) * iut;
#pragma unroll
  for (int a = 0; a < 4; a++) {
    T q = m.lo(a, 0) * s.bcon[0];
#pragma unroll
    for (int b = 1; b < 4; b++) q = q + m.lo(a, b) * s.bcon[b];
    s.bcov[a] = q;
  }
  s.bsq = s.bcon[0] * s.bcov[0] + s.bcon[1] * s.bcov[1] + s.bcon[2] * s.bcov[2] +
          s.bcon[3] * s.bcov[3];
  // u_t = g_ti u~^i - alpha gamma  =>  1 + u_t = (1 - alpha) - alpha u~^2/(1 + gamma) + g_ti u~^i
  T gtu = m.lo(0, 1) * ut[0] + m.lo(0, 2) * ut[1] + m.lo(0, 3) * ut[2];
  s.opu = (R(1.0) - m.alpha) - m.alpha * s.v.usq / (R(1.0) + s.v.gamma) + gtu;
}

// Row mu of the gas conserved/flux vector (Sec. 4 lists of U_q and F_q):
// out[0] = rho u^mu, out[1] = T^mu_t + rho u^mu, out[2..4] = T^mu_i,
// out[5..7] = B^i (mu = 0) or b^i u^mu - b^mu u^i, all without sqrt(-g).
template <class T>
DEV void gas_row(const Gas<T>& s, const T B[3], int mu, T out[8]) {
  using R = typename RealOf<T>::type;
  const T um = s.v.ucon[mu];
  const T ptot = s.pg + R(0.5) * s.bsq;
  const T enth = s.rho + s.ug + s.pg + s.bsq;
  out[0] = s.rho * um;
  out[1] = s.rho * um * s.opu + (s.ug + s.pg + s.bsq) * um * s.v.ucov[0] - s.bcon[mu] * s.bcov[0];
  if (mu == 0) out[1] = out[1] + ptot;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    out[2 + i] = enth * um * s.v.ucov[i + 1] - s.bcon[mu] * s.bcov[i + 1];
    if (mu == i + 1) out[2 + i] = out[2 + i] + ptot;
  }
#pragma unroll
  for (int i = 0; i < 3; i++)
    out[5 + i] = (mu == 0) ? B[i] : s.bcon[i + 1] * um - s.bcon[mu] * s.v.ucon[i + 1];
}

// M1 radiation (eq. Rlab): R^mu_nu = (4/3) Ebar u^mu u_nu + (1/3) Ebar delta
template <class T>
DEV void rad_row(const Vel<T>& r, const T& E, int mu, T out[4]) {
  using R = typename RealOf<T>::type;
  const T f = R(4.0 / 3.0) * E * r.ucon[mu];
#pragma unroll
  for (int nu = 0; nu < 4; nu++) {
    out[nu] = f * r.ucov[nu];
    if (nu == mu) out[nu] = out[nu] + E * R(1.0 / 3.0);
  }
}

// Radiation 4-force with a lower index (eq. Gcov) in closed form: with
// w = u_rad . u, E^ = (4/3) Ebar w^2 - Ebar/3 and R^b_nu u_b =
// (4/3) Ebar w u_rad,nu + (1/3) Ebar u_nu,
//   G_nu = -k_abs (R^b_nu u_b + lambda u_nu) - k_es (R^b_nu u_b + E^ u_nu),
// lambda = k_abs a_rad T^4 (Kirchhoff emission, passed in), T = p/rho0.
template <class T>
DEV void four_force(const Vel<T>& u, const Vel<T>& r, const T& E, const T& kabs, const T& kes,
                    const T& lambda, T G[4]) {
  T w = r.ucon[0] * u.ucov[0];
#pragma unroll
  for (int a = 1; a < 4; a++) w = w + r.ucon[a] * u.ucov[a];
  const T c43 = (4.0 / 3.0) * E * w;
  const T Ehat = c43 * w - E * (1.0 / 3.0);
  const T ktot = kabs + kes;
#pragma unroll
  for (int nu = 0; nu < 4; nu++) {
    const T Ru = c43 * r.ucov[nu] + E * (1.0 / 3.0) * u.ucov[nu];
    G[nu] = -(ktot * Ru + (lambda + kes * Ehat) * u.ucov[nu]);
  }
}

// Lab-frame speeds along dir of a wave with frame speed c (c2 = c^2) in a
// frame of 4-velocity u: the two roots of
// [(1-c2)(u^t)^2 - c2 g^tt] v^2 - 2[(1-c2) u^t u^d - c2 g^td] v + [(1-c2)(u^d)^2 - c2 g^dd] = 0
// (the dispersion relation (k.u)^2 = c2 (k.k + (k.u)^2) with k = d(x^d - v t)).
template <class T>
DEV void char_speeds(const MetricT<typename RealOf<T>::type>& m, const T u[4], T c2, int dir,
                     T& vm, T& vp) {
  using R = typename RealOf<T>::type;
  const T A = (R(1.0) - c2) * u[0] * u[0] - c2 * m.up(0, 0);
  const T B = (R(1.0) - c2) * u[0] * u[dir] - c2 * m.up(0, dir);
  // discriminant B^2 - A C = c2 [(1 - c2) h + c2 k]: the (1 - c2)^2 (u^t u^d)^2
  // parts cancel exactly, so a tiny c2 (optically thick limiter) loses nothing
  const T h = u[0] * u[0] * m.up(dir, dir) - R(2.0) * u[0] * u[dir] * m.up(0, dir) +
              u[dir] * u[dir] * m.up(0, 0);
  const R k = m.up(0, dir) * m.up(0, dir) - m.up(0, 0) * m.up(dir, dir);
  const T disc = fmax(c2 * ((R(1.0) - c2) * h + c2 * k), T(R(0.0)));
  const T sq = sqrt(disc);
  const T ia = R(1.0) / A;
  const T v1 = (B + sq) * ia, v2 = (B - sq) * ia;
  vp = fmax(v1, v2);
  vm = fmin(v1, v2);
}
