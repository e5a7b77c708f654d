/*
 * Oracle geometry: metric, inverse metric, sqrt(-g), lapse and connection in
 * the internal coordinates x^(1..3) of a uniform grid (Sec. 2: internal
 * coordinates mapped to physical ones; Sec. 6 grid: r = R0 + exp(x1)).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Kerr-Schild metric with M = 1 (textbook form, horizon-penetrating):
 *   Sigma = r^2 + a^2 cos^2 th,  Delta = r^2 - 2 r + a^2
 *   g_tt = -(1 - 2r/Sigma), g_tr = 2r/Sigma, g_tph = -2 a r sin^2 th/Sigma,
 *   g_rr = 1 + 2r/Sigma, g_rph = -a (1 + 2r/Sigma) sin^2 th, g_thth = Sigma,
 *   g_phph = sin^2 th (Sigma + a^2 (1 + 2r/Sigma) sin^2 th)
 *   g^tt = -(1 + 2r/Sigma), g^tr = 2r/Sigma, g^rr = Delta/Sigma, g^rph = a/Sigma,
 *   g^thth = 1/Sigma, g^phph = 1/(Sigma sin^2 th),  sqrt(-g) = Sigma |sin th|
 * Internal coordinates: r = R0 + exp(x1), th = pi x2, ph = 2 pi x3, so each
 * component picks up the diagonal Jacobian J = (1, r - R0, pi, 2 pi).
 *
 * The connection uses complex-step differentiation of the metric
 * (df/dx = Im f(x + i h)/h, exact to rounding for analytic f), then
 * Gamma^l_{mn} = g^{lk} (d_m g_kn + d_n g_km - d_k g_mn)/2.
 */
#include <complex.h>
#include <math.h>
#include <string.h>
#include "oracle.h"

static void ks_gcov_c(double a, double R0, double complex x1, double complex x2,
                      double complex g[4][4]) {
  const double complex er = cexp(x1);
  const double complex r = R0 + er;
  const double complex th = M_PI * x2;
  const double complex s = csin(th), c = ccos(th);
  const double complex s2 = s * s;
  const double complex Sig = r * r + a * a * c * c;
  const double complex z = 2.0 * r / Sig;
  double complex J[4] = {1.0, er, M_PI, 2.0 * M_PI};
  double complex gb[4][4];
  memset(gb, 0, sizeof(gb));
  gb[0][0] = -(1.0 - z);
  gb[0][1] = gb[1][0] = z;
  gb[0][3] = gb[3][0] = -a * z * s2;
  gb[1][1] = 1.0 + z;
  gb[1][3] = gb[3][1] = -a * (1.0 + z) * s2;
  gb[2][2] = Sig;
  gb[3][3] = s2 * (Sig + a * a * (1.0 + z) * s2);
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) g[m][n] = gb[m][n] * J[m] * J[n];
}

void orc_geom_point(const orc_params *p, double x1, double x2, orc_geom *g) {
  memset(g, 0, sizeof(*g));
  if (p->metric == ORC_MINKOWSKI) {
    g->gcov[0][0] = -1.0;
    g->gcon[0][0] = -1.0;
    for (int i = 1; i < 4; i++) {
      g->gcov[i][i] = 1.0;
      g->gcon[i][i] = 1.0;
    }
    g->gdet = 1.0;
    g->alpha = 1.0;
    return;
  }
  const double a = p->a;
  double complex gc[4][4];
  ks_gcov_c(a, p->R0, x1, x2, gc);
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) g->gcov[m][n] = creal(gc[m][n]);

  const double er = exp(x1);
  const double r = p->R0 + er;
  const double th = M_PI * x2;
  const double s = sin(th), c = cos(th);
  const double Sig = r * r + a * a * c * c;
  const double Del = r * r - 2.0 * r + a * a;
  const double J[4] = {1.0, er, M_PI, 2.0 * M_PI};
  double gb[4][4];
  memset(gb, 0, sizeof(gb));
  gb[0][0] = -(1.0 + 2.0 * r / Sig);
  gb[0][1] = gb[1][0] = 2.0 * r / Sig;
  gb[1][1] = Del / Sig;
  gb[1][3] = gb[3][1] = a / Sig;
  gb[2][2] = 1.0 / Sig;
  gb[3][3] = 1.0 / (Sig * s * s); /* infinite exactly on the axis; never used there */
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) g->gcon[m][n] = gb[m][n] / (J[m] * J[n]);
  g->gdet = Sig * fabs(s) * J[1] * J[2] * J[3];
  g->alpha = 1.0 / sqrt(-g->gcon[0][0]);
}

void orc_connection(const orc_params *p, double x1, double x2, double conn[4][4][4]) {
  memset(conn, 0, sizeof(double) * 64);
  if (p->metric == ORC_MINKOWSKI) return;
  const double h = 1e-30;
  double dg[4][4][4]; /* dg[k][m][n] = d_k g_mn */
  memset(dg, 0, sizeof(dg));
  double complex gc[4][4];
  ks_gcov_c(p->a, p->R0, x1 + I * h, x2, gc);
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) dg[1][m][n] = cimag(gc[m][n]) / h;
  ks_gcov_c(p->a, p->R0, x1, x2 + I * h, gc);
  for (int m = 0; m < 4; m++)
    for (int n = 0; n < 4; n++) dg[2][m][n] = cimag(gc[m][n]) / h;

  orc_geom g;
  orc_geom_point(p, x1, x2, &g);
  double low[4][4][4]; /* Gamma_{k m n} */
  for (int k = 0; k < 4; k++)
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++)
        low[k][m][n] = 0.5 * (dg[m][k][n] + dg[n][k][m] - dg[k][m][n]);
  for (int l = 0; l < 4; l++)
    for (int m = 0; m < 4; m++)
      for (int n = 0; n < 4; n++) {
        double s = 0.0;
        for (int k = 0; k < 4; k++) s += g.gcon[l][k] * low[k][m][n];
        conn[l][m][n] = s;
      }
}
