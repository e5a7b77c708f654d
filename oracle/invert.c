/*
 * Oracle conserved-to-primitive inversions.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * MHD (Sec. 4.5): one nonlinear equation in W' = W - D, the energy relation
 * (eq. EMHD written with W = W' + D), with v~^2(W) from eq. vsqeq, v~^i from
 * eq. tveq, gamma, rho0 = D/gamma (eq. PRIM1), and the gas pressure from the
 * definition of W' (eq. Wprime).  The root is found by plain bisection
 * inside a bracket that is proven on paper, to the last representable bit.
 *
 * RAD (Sec. 4.6): analytic, y = U~^2/E_rad^2 (eq. ysol), gamma_rad^2
 * (eq. gammarvsy), p_rad (eq. prsol), v~_rad (eq. tvrsol), with the BASIC or
 * TYPE2 limiter of that section.
 */
#include <float.h>
#include <math.h>
#include <string.h>
#include "oracle.h"
#include "oracle_internal.h"

void orc_spatial_gcon(const orc_geom *g, double gij[3][3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      gij[i][j] = g->gcon[i + 1][j + 1] - g->gcon[0][i + 1] * g->gcon[0][j + 1] / g->gcon[0][0];
}

typedef struct {
  double D, Ep, Qt2, Bsq, S, gam;
} mhd_fixed;

/* v~^2(W) of eq. vsqeq */
static double vsq_of_W(const mhd_fixed *m, double W) {
  const double a = m->Bsq + W;
  return (m->Qt2 * W * W + m->S * m->S * (m->Bsq + 2.0 * W)) / (a * a * W * W);
}

/* residual of eq. EMHD with W = W' + D, and chi = u + p from eq. Wprime */
static double mhd_residual(const mhd_fixed *m, double Wp, double *chi_out, double *gamma_out) {
  const double W = Wp + m->D;
  const double vsq = vsq_of_W(m, W);
  const double gsq = 1.0 / (1.0 - vsq);
  const double gamma = sqrt(gsq);
  const double usq = gsq * vsq;
  const double chi = (Wp - m->D * usq / (1.0 + gamma)) / gsq;
  const double pg = (m->gam - 1.0) / m->gam * chi;
  if (chi_out) *chi_out = chi;
  if (gamma_out) *gamma_out = gamma;
  return Wp - pg + 0.5 * m->Bsq * (1.0 + vsq) - 0.5 * m->S * m->S / (W * W) - m->Ep;
}

/* Returns 0 on success, 1 when no physical root exists, 2 when the root has
 * u_g <= 0 (P is still filled). Only P[0..7] are written. */
int orc_mhd_invert(const orc_params *p, const orc_geom *g, const double *U, const double *Pguess,
                   double *P) {
  (void)Pguess;
  const double gd = g->gdet, al = g->alpha;
  const double rhout = U[0] / gd;
  const double e1 = U[1] / gd; /* T^t_t + rho u^t */
  double Tt[3], B[3];
  for (int i = 0; i < 3; i++) {
    Tt[i] = U[2 + i] / gd;
    B[i] = U[5 + i] / gd;
  }
  double gij[3][3];
  orc_spatial_gcon(g, gij);
  mhd_fixed m;
  m.gam = p->gam;
  m.D = al * rhout;                                       /* eq. PRIM1 */
  double gtiT = 0.0;
  for (int i = 0; i < 3; i++) gtiT += g->gcon[0][i + 1] * Tt[i];
  m.Ep = -e1 + rhout * (1.0 - al) + al * al * gtiT;       /* E - D, -E = eta^mu Q_mu */
  double Q[3], Qt[3], Bz[3];
  for (int i = 0; i < 3; i++) {
    Q[i] = al * Tt[i];                                    /* Q_i = -eta_nu T^nu_i */
    Bz[i] = al * B[i];                                    /* ZAMO field alpha B^i */
  }
  m.Qt2 = 0.0;
  for (int i = 0; i < 3; i++) {
    Qt[i] = 0.0;
    for (int j = 0; j < 3; j++) Qt[i] += gij[i][j] * Q[j]; /* eq. Qtilde */
    m.Qt2 += Qt[i] * Q[i];
  }
  m.Bsq = 0.0;
  m.S = 0.0;
  for (int i = 0; i < 3; i++) {
    m.S += Q[i] * Bz[i];
    for (int j = 0; j < 3; j++) m.Bsq += g->gcov[i + 1][j + 1] * Bz[i] * Bz[j];
  }
  if (!(m.D > 0.0) || !(m.Ep > 0.0) || !isfinite(m.Ep) || !isfinite(m.Qt2)) return 1;

  /* Bracket.  v~^2(W) decreases with W, so the admissible region v~^2 < 1 is
   * W > W1 (found by bisection when W1 > D).  On it the numerator of chi,
   * N(W') = W' - D u~^2/(1+gamma), increases strictly (gamma falls with W),
   * so chi >= 0 exactly on [W0', inf).  Upper end: p <= (gam-1) W'/gam and the
   * magnetic terms are >= Bsq/2 (Cauchy-Schwarz on S), so the residual is
   * >= 0 once W' >= gam (E' - Bsq/2).  The physical root lies in [W0', hi]. */
  double a0 = 0.0;
  if (vsq_of_W(&m, m.D) >= 1.0) {
    double a = 0.0, b = 1.0 + m.Ep + sqrt(m.Qt2) + m.Bsq;
    while (vsq_of_W(&m, m.D + b) >= 1.0) b *= 2.0;
    for (int it = 0; it < 4000; it++) {
      const double c = 0.5 * (a + b);
      if (c <= a || c >= b) break;
      if (vsq_of_W(&m, m.D + c) >= 1.0) a = c; else b = c;
    }
    a0 = b;
  }
  double hi = m.gam * (m.Ep > 0.5 * m.Bsq ? m.Ep - 0.5 * m.Bsq : 0.0);
  hi = hi * (1.0 + 1e-12) + 1e-300;
  if (hi < a0) hi = a0;
  while (mhd_residual(&m, hi, NULL, NULL) < 0.0) {
    hi = 2.0 * hi + 1e-300;
    if (!isfinite(hi)) return 1;
  }
  /* W0': zero of the chi numerator */
  double chi_hi;
  double nb = hi;
  for (;;) {
    mhd_residual(&m, nb, &chi_hi, NULL);
    if (chi_hi > 0.0) break;
    nb = 2.0 * nb + 1e-300;
    if (!isfinite(nb)) return 1;
  }
  double na = a0;
  for (int it = 0; it < 4000; it++) {
    const double c = 0.5 * (na + nb);
    if (c <= na || c >= nb) break;
    double chic;
    mhd_residual(&m, c, &chic, NULL);
    if (chic > 0.0) nb = c; else na = c;
  }
  double lo = nb; /* smallest W' found with chi > 0 */
  if (lo > hi) return 1;
  if (!(mhd_residual(&m, lo, NULL, NULL) < 0.0)) return 1; /* no root with u_g > 0 */
  for (int it = 0; it < 4000; it++) {
    const double c = 0.5 * (lo + hi);
    if (c <= lo || c >= hi) break;
    const double fc = mhd_residual(&m, c, NULL, NULL);
    if (fc == 0.0) {
      lo = hi = c;
      break;
    }
    if (fc < 0.0) lo = c; else hi = c;
  }
  const double Wp = (fabs(mhd_residual(&m, lo, NULL, NULL)) <= fabs(mhd_residual(&m, hi, NULL, NULL)))
                        ? lo : hi;
  double chi, gamma;
  mhd_residual(&m, Wp, &chi, &gamma);
  const double W = Wp + m.D;
  /* eq. tveq */
  for (int i = 0; i < 3; i++) {
    const double vt = (Qt[i] + m.S * Bz[i] / W) / (W + m.Bsq);
    P[2 + i] = gamma * vt;
  }
  P[0] = m.D / gamma;
  P[1] = chi / m.gam;
  for (int i = 0; i < 3; i++) P[5 + i] = B[i];
  if (!(P[1] > 0.0)) return 2;
  return 0;
}

/* y_max from gamma_max by inverting eq. gammarvsy: y = 16 G (G-1)/(4G-1)^2, G = gamma^2 */
static double orc_ymax(double gmax) {
  const double G = gmax * gmax;
  return 16.0 * G * (G - 1.0) / ((4.0 * G - 1.0) * (4.0 * G - 1.0));
}

/* limiter: 0 BASIC, 1 TYPE2.  Returns bit 0 when E_rad <= 0 was met, bit 1
 * when y >= y_max was met.  Writes P[8..11]. */
int orc_rad_invert(const orc_params *p, const orc_geom *g, const double *U, int limiter,
                   double *P) {
  const double gd = g->gdet, al = g->alpha;
  double Rt[4];
  for (int m = 0; m < 4; m++) Rt[m] = U[8 + m] / gd;
  double gij[3][3];
  orc_spatial_gcon(g, gij);
  /* U_mu = -R^nu_mu eta_nu = alpha R^t_mu (eq. RADPRIM1OLD); -E_rad = eta^mu U_mu (eq. RADPRIM2) */
  double Uc[3];
  for (int i = 0; i < 3; i++) Uc[i] = al * Rt[i + 1];
  double gtiR = 0.0;
  for (int i = 0; i < 3; i++) gtiR += g->gcon[0][i + 1] * Rt[i + 1];
  const double Erad = -Rt[0] + al * al * gtiR;
  double Ut[3], Ut2 = 0.0;
  for (int i = 0; i < 3; i++) {
    Ut[i] = 0.0;
    for (int j = 0; j < 3; j++) Ut[i] += gij[i][j] * Uc[j]; /* eq. RADPRIM3 */
    Ut2 += Ut[i] * Uc[i];
  }
  const double G = p->gamma_max * p->gamma_max;
  const double ymax = orc_ymax(p->gamma_max);
  int flags = 0;
  const double y = (Erad != 0.0) ? Ut2 / (Erad * Erad) : 0.0;
  if (Erad <= 0.0) flags |= 1;
  if (Erad > 0.0 && y >= ymax) flags |= 2;

  if (limiter == 0) {
    if (Erad <= 0.0) {
      P[8] = 1e-300;
      P[9] = P[10] = P[11] = 0.0;
    } else if (y <= 0.0) {
      P[8] = Erad; /* gamma = 1: p_rad = E_rad/3 */
      P[9] = P[10] = P[11] = 0.0;
    } else if (y >= ymax) {
      const double prad = Erad / (4.0 * G - 1.0);
      const double s = sqrt((G - 1.0) / Ut2);
      P[8] = 3.0 * prad;
      for (int i = 0; i < 3; i++) P[9 + i] = s * Ut[i];
    } else {
      const double gsq = (2.0 - y + sqrt(4.0 - 3.0 * y)) / (4.0 * (1.0 - y));
      const double prad = Erad / (4.0 * gsq - 1.0);
      const double gamma = sqrt(gsq);
      P[8] = 3.0 * prad;
      for (int i = 0; i < 3; i++) P[9 + i] = gamma * Ut[i] / (4.0 * prad * gsq);
    }
    return flags;
  }
  /* TYPE2: keep the momentum, raise E_rad to the value that makes y = y_max */
  if (Erad <= 0.0 || y >= ymax) {
    if (Ut2 > 0.0) {
      const double E2 = 1e-150 + sqrt(Ut2 / ymax);
      const double prad = E2 / (4.0 * G - 1.0);
      const double s = sqrt((G - 1.0) / Ut2);
      P[8] = 3.0 * prad;
      for (int i = 0; i < 3; i++) P[9 + i] = s * Ut[i];
    } else {
      P[8] = 1e-150;
      P[9] = P[10] = P[11] = 0.0;
    }
  } else if (y <= 0.0) {
    P[8] = Erad;
    P[9] = P[10] = P[11] = 0.0;
  } else {
    const double gsq = (2.0 - y + sqrt(4.0 - 3.0 * y)) / (4.0 * (1.0 - y));
    const double prad = Erad / (4.0 * gsq - 1.0);
    const double gamma = sqrt(gsq);
    P[8] = 3.0 * prad;
    for (int i = 0; i < 3; i++) P[9 + i] = gamma * Ut[i] / (4.0 * prad * gsq);
  }
  return flags;
}
