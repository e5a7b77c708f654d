/*
 * Oracle pointwise physics: 4-velocities, fluid-frame magnetic field, the
 * gas and radiation stress-energy tensors, conserved variables, fluxes,
 * geometric sources, the radiation 4-force and characteristic speeds.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Every function writes the
 * textbook definition out in full 4x4 tensor form; nothing is fused.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"
#include "oracle_internal.h"

/* u^mu from the velocity relative to the normal observer (Sec. 2, Sec. 4.5):
 * gamma = sqrt(1 + g_ij u~^i u~^j), u^mu = u~^mu + gamma eta^mu with
 * eta^mu = -alpha g^{mu t}, so u^t = gamma/alpha, u^i = u~^i - gamma alpha g^{ti}. */
double orc_ucon(const orc_geom *g, const double ut[3], double ucon[4]) {
  double q = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) q += g->gcov[i + 1][j + 1] * ut[i] * ut[j];
  const double gamma = sqrt(1.0 + q);
  ucon[0] = gamma / g->alpha;
  for (int i = 0; i < 3; i++) ucon[i + 1] = ut[i] - gamma * g->alpha * g->gcon[0][i + 1];
  return gamma;
}

void orc_lower(const orc_geom *g, const double vcon[4], double vcov[4]) {
  for (int m = 0; m < 4; m++) {
    double s = 0.0;
    for (int n = 0; n < 4; n++) s += g->gcov[m][n] * vcon[n];
    vcov[m] = s;
  }
}

/* b^mu = B^nu h^mu_nu / u^t with h = u u + delta (Sec. 2) */
void orc_bcon(const orc_geom *g, const double B[3], const double ucon[4], const double ucov[4],
              double bcon[4]) {
  double bt = 0.0;
  for (int i = 0; i < 3; i++) bt += B[i] * ucov[i + 1];
  bcon[0] = bt;
  for (int i = 0; i < 3; i++) bcon[i + 1] = (B[i] + bt * ucon[i + 1]) / ucon[0];
  (void)g;
}

void orc_gas_state(const orc_params *p, const orc_geom *g, const double *P, orc_gas *s) {
  s->rho = P[0];
  s->u = P[1];
  s->pg = (p->gam - 1.0) * P[1];
  s->gamma = orc_ucon(g, P + 2, s->ucon);
  orc_lower(g, s->ucon, s->ucov);
  orc_bcon(g, P + 5, s->ucon, s->ucov, s->bcon);
  orc_lower(g, s->bcon, s->bcov);
  double bsq = 0.0;
  for (int m = 0; m < 4; m++) bsq += s->bcon[m] * s->bcov[m];
  s->bsq = bsq;
  /* T^mu_nu = (rho + u + p + b^2) u^mu u_nu + (p + b^2/2) delta - b^mu b_nu (eq. MAEM) */
  const double w = s->rho + s->u + s->pg + bsq;
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++)
      s->T[m][n] = w * s->ucon[m] * s->ucov[n] + (m == n ? s->pg + 0.5 * bsq : 0.0) -
                   s->bcon[m] * s->bcov[n];
  /* 1 + u_t without cancellation (Sec. 4.5: gamma - 1 = u~^2/(gamma + 1)):
   * u_t = g_ti u~^i - alpha gamma, so 1 + u_t = (1 - alpha) - alpha u~^2/(1+gamma) + g_ti u~^i */
  double gtu = 0.0, usq = 0.0;
  for (int i = 0; i < 3; i++) {
    gtu += g->gcov[0][i + 1] * P[2 + i];
    for (int j = 0; j < 3; j++) usq += g->gcov[i + 1][j + 1] * P[2 + i] * P[2 + j];
  }
  s->one_plus_ut = (1.0 - g->alpha) - g->alpha * usq / (1.0 + s->gamma) + gtu;
}

/* T^mu_t + rho u^mu with the rest-mass part cancelled analytically */
double orc_gas_energy_flux(const orc_gas *s, int mu) {
  const double h = s->u + s->pg + s->bsq;
  double e = s->rho * s->ucon[mu] * s->one_plus_ut + h * s->ucon[mu] * s->ucov[0] -
             s->bcon[mu] * s->bcov[0];
  if (mu == 0) e += s->pg + 0.5 * s->bsq;
  return e;
}

/* M1 closure: R^mu_nu = (4/3) Ebar u_rad^mu u_rad_nu + (1/3) Ebar delta (eq. R, eq. Rlab) */
void orc_rad_state(const orc_geom *g, const double *P, orc_rad *r) {
  r->E = P[8];
  r->gamma = orc_ucon(g, P + 9, r->ucon);
  orc_lower(g, r->ucon, r->ucov);
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++)
      r->R[m][n] = (4.0 / 3.0) * r->E * r->ucon[m] * r->ucov[n] + (m == n ? r->E / 3.0 : 0.0);
}

void orc_p2u(const orc_params *p, const orc_geom *g, const double *P, double *U) {
  orc_gas s;
  orc_rad r;
  orc_gas_state(p, g, P, &s);
  orc_rad_state(g, P, &r);
  const double gd = g->gdet;
  U[0] = gd * s.rho * s.ucon[0];
  U[1] = gd * orc_gas_energy_flux(&s, 0);
  for (int i = 0; i < 3; i++) U[2 + i] = gd * s.T[0][i + 1];
  for (int i = 0; i < 3; i++) U[5 + i] = gd * P[5 + i];
  U[8] = gd * r.R[0][0];
  for (int i = 0; i < 3; i++) U[9 + i] = gd * r.R[0][i + 1];
}

/* fluxes F_q along direction dir = 1..3 (Sec. 4, list of F_q); the induction
 * flux is b^i u^d - b^d u^i = B^i v^d - B^d v^i */
void orc_flux(const orc_params *p, const orc_geom *g, const double *P, int dir, double *F) {
  orc_gas s;
  orc_rad r;
  orc_gas_state(p, g, P, &s);
  orc_rad_state(g, P, &r);
  const double gd = g->gdet;
  F[0] = gd * s.rho * s.ucon[dir];
  F[1] = gd * orc_gas_energy_flux(&s, dir);
  for (int i = 0; i < 3; i++) F[2 + i] = gd * s.T[dir][i + 1];
  for (int i = 0; i < 3; i++)
    F[5 + i] = gd * (s.bcon[i + 1] * s.ucon[dir] - s.bcon[dir] * s.ucon[i + 1]);
  F[8] = gd * r.R[dir][0];
  for (int i = 0; i < 3; i++) F[9 + i] = gd * r.R[dir][i + 1];
}

/* geometric source sqrt(-g) T^k_l Gamma^l_{nu k} (and the same for R) */
void orc_source_geom(const orc_params *p, const orc_geom *g, const double conn[4][4][4],
                     const double *P, double *S) {
  orc_gas s;
  orc_rad r;
  orc_gas_state(p, g, P, &s);
  orc_rad_state(g, P, &r);
  memset(S, 0, sizeof(double) * ORC_NPRIM);
  for (int nu = 0; nu < 4; nu++) {
    double sg = 0.0, sr = 0.0;
    for (int k = 0; k < 4; k++)
      for (int l = 0; l < 4; l++) {
        sg += s.T[k][l] * conn[l][nu][k];
        sr += r.R[k][l] * conn[l][nu][k];
      }
    if (nu == 0) {
      S[1] = g->gdet * sg;
      S[8] = g->gdet * sr;
    } else {
      S[1 + nu] = g->gdet * sg;
      S[8 + nu] = g->gdet * sr;
    }
  }
}

/* covariant 4-force (eq. Gcov), returned with a lower index:
 * G^mu = -(k_abs R^mu_a u^a + lambda u^mu) - k_es (R^mu_a u^a + R^a_b u_a u^b u^mu),
 * lambda = k_abs a_rad T^4 (Kirchhoff), T = p/rho0 */
void orc_four_force(const orc_params *p, const orc_geom *g, const double *P, double kabs,
                    double kes, double Gcov[4]) {
  orc_gas s;
  orc_rad r;
  orc_gas_state(p, g, P, &s);
  orc_rad_state(g, P, &r);
  const double T = s.pg / s.rho;
  const double lambda = kabs * p->arad * T * T * T * T;
  double Ru[4];
  for (int m = 0; m < 4; m++) {
    double acc = 0.0;
    for (int a = 0; a < 4; a++) acc += r.R[m][a] * s.ucon[a];
    Ru[m] = acc;
  }
  double Ruu = 0.0;
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++) Ruu += r.R[a][b] * s.ucov[a] * s.ucon[b];
  double Gcon[4];
  for (int m = 0; m < 4; m++)
    Gcon[m] = -(kabs * Ru[m] + lambda * s.ucon[m]) - kes * (Ru[m] + Ruu * s.ucon[m]);
  orc_lower(g, Gcon, Gcov);
}

/* Orthonormal tetrad of the gas frame by Gram-Schmidt, then the fluid-frame
 * moments E^ = R^(0)(0), F^i = R^(0)(i), P^ij = R^(i)(j) (Sec. 3). */
void orc_fluid_frame_rad(const orc_geom *g, const double *P, double *Ehat, double Fhat[3],
                         double Phat[3][3]) {
  double u[4];
  orc_ucon(g, P + 2, u);
  double e[4][4];
  memcpy(e[0], u, sizeof(u));
  for (int a = 1; a < 4; a++) {
    double v[4] = {0, 0, 0, 0};
    v[a] = 1.0;
    for (int b = 0; b < a; b++) {
      double dot = 0.0;
      for (int m = 0; m < 4; m++)
        for (int n = 0; n < 4; n++) dot += g->gcov[m][n] * v[m] * e[b][n];
      const double eta = (b == 0) ? -1.0 : 1.0;
      for (int m = 0; m < 4; m++) v[m] -= eta * dot * e[b][m];
    }
    double nrm = 0.0;
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) nrm += g->gcov[m][n] * v[m] * v[n];
    nrm = sqrt(nrm);
    for (int m = 0; m < 4; m++) e[a][m] = v[m] / nrm;
  }
  orc_rad r;
  orc_rad_state(g, P, &r);
  /* R^{mu nu} = R^mu_l g^{l nu}; tetrad components need e^(a)_mu = eta^{aa} g_{mu nu} e_(a)^nu */
  double Rup[4][4];
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) {
      double acc = 0.0;
      for (int l = 0; l < 4; l++) acc += r.R[m][l] * g->gcon[l][n];
      Rup[m][n] = acc;
    }
  double ecov[4][4];
  for (int a = 0; a < 4; a++) {
    orc_lower(g, e[a], ecov[a]);
    if (a == 0)
      for (int m = 0; m < 4; m++) ecov[a][m] = -ecov[a][m];
  }
  double Rt[4][4];
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++) {
      double acc = 0.0;
      for (int m = 0; m < 4; m++)
        for (int n = 0; n < 4; n++) acc += Rup[m][n] * ecov[a][m] * ecov[b][n];
      Rt[a][b] = acc;
    }
  *Ehat = Rt[0][0];
  for (int i = 0; i < 3; i++) {
    Fhat[i] = Rt[0][i + 1];
    for (int j = 0; j < 3; j++) Phat[i][j] = Rt[i + 1][j + 1];
  }
}

/* Lab-frame speeds along dir of a wave moving at speed c (c2 = c^2) in the
 * frame with 4-velocity u: roots v of (k.u)^2 = c^2 (k.k + (k.u)^2) for
 * k_mu = d_mu (x^dir - v t)  (Sec. 4.4, HARM dispersion relation). */
static void orc_char_roots(const orc_geom *g, const double u[4], double c2, int dir, double *vm,
                           double *vp) {
  const double A = (1.0 - c2) * u[0] * u[0] - c2 * g->gcon[0][0];
  const double B = (1.0 - c2) * u[0] * u[dir] - c2 * g->gcon[0][dir];
  /* B^2 - A C with the (1 - c^2)^2 (u^t u^d)^2 terms cancelled analytically,
   * so the root separation keeps full precision when c^2 is tiny */
  const double h = u[0] * u[0] * g->gcon[dir][dir] - 2.0 * u[0] * u[dir] * g->gcon[0][dir] +
                   u[dir] * u[dir] * g->gcon[0][0];
  const double k = g->gcon[0][dir] * g->gcon[0][dir] - g->gcon[0][0] * g->gcon[dir][dir];
  double disc = c2 * ((1.0 - c2) * h + c2 * k);
  if (disc < 0.0) disc = 0.0;
  const double sq = sqrt(disc);
  const double v1 = (B + sq) / A, v2 = (B - sq) / A;
  *vp = v1 > v2 ? v1 : v2;
  *vm = v1 > v2 ? v2 : v1;
}

/* gas fast magnetosonic and M1 radiation characteristic speeds; the
 * radiation ones are limited by 4/(3 tau) in the gas frame (eq. wavespeedlimit) */
void orc_wavespeeds(const orc_params *p, const orc_geom *g, const double *P, int dir,
                    double kappa_tot_dx, double vgas[2], double vrad[2]) {
  orc_gas s;
  orc_rad r;
  orc_gas_state(p, g, P, &s);
  orc_rad_state(g, P, &r);
  const double w = s.rho + s.u + s.pg;
  const double cs2 = p->gam * s.pg / w;
  const double va2 = s.bsq / (w + s.bsq);
  const double cms2 = va2 + cs2 * (1.0 - va2);
  orc_char_roots(g, s.ucon, cms2, dir, &vgas[0], &vgas[1]);
  orc_char_roots(g, r.ucon, 1.0 / 3.0, dir, &vrad[0], &vrad[1]);
  if (kappa_tot_dx > 0.0) {
    const double clim = 4.0 / (3.0 * kappa_tot_dx);
    if (clim < 1.0) {
      double lm, lp;
      orc_char_roots(g, s.ucon, clim * clim, dir, &lm, &lp);
      if (lp < vrad[1]) vrad[1] = lp;
      if (lm > vrad[0]) vrad[0] = lm;
    }
  }
}
