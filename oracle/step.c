/*
 * Oracle grid-level steps of one Runge-Kutta sub-step (Sec. 4.2, steps
 * 1-13) and the third-order Shu-Osher RK3 with identical explicit and
 * implicit coefficients that the paper uses (Sec. 4.1, last paragraphs).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Reconstruction is piecewise linear with monotonised-central slopes; fluxes
 * are HLL (eq. hll) or LAXF (eq. lax) with separate gas and radiation wave
 * speeds (Sec. 4.4); the induction fluxes are corrected by flux-CT (corner
 * EMF = average of the four adjacent face fluxes, face flux = average of the
 * two adjacent corner EMFs); dt follows Sec. 4.4's last paragraph.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "oracle_internal.h"

int orc_ng(const orc_params *p, int d) { return p->n[d] > 1 ? p->ng : 0; }
int orc_nalloc(const orc_params *p, int d) { return p->n[d] + 2 * orc_ng(p, d); }
double orc_dx(const orc_params *p, int d) { return (p->xhi[d] - p->xlo[d]) / p->n[d]; }
long orc_ncell_alloc(const orc_params *p) {
  return (long)orc_nalloc(p, 0) * orc_nalloc(p, 1) * orc_nalloc(p, 2);
}

void orc_cell_x(const orc_params *p, int i, int j, double *x1, double *x2) {
  *x1 = p->xlo[0] + (i - orc_ng(p, 0) + 0.5) * orc_dx(p, 0);
  *x2 = p->xlo[1] + (j - orc_ng(p, 1) + 0.5) * orc_dx(p, 1);
}

void orc_face_x(const orc_params *p, int dir, int i, int j, double *x1, double *x2) {
  orc_cell_x(p, i, j, x1, x2);
  if (dir == 1) *x1 = p->xlo[0] + (i - orc_ng(p, 0)) * orc_dx(p, 0);
  if (dir == 2) *x2 = p->xlo[1] + (j - orc_ng(p, 1)) * orc_dx(p, 1);
}

#define IDX(p, i, j, k) ((long)(i) + (long)orc_nalloc(p, 0) * ((long)(j) + (long)orc_nalloc(p, 1) * (long)(k)))

/* ---- step 1: ghost cells (Sec. 4.2) ---- */
static void copy_cell(double *P, long N, long dst, long src, const int *neg) {
  for (int q = 0; q < 12; q++) P[q * N + dst] = P[q * N + src];
  for (int m = 0; m < 3 && neg[m] >= 0; m++) P[neg[m] * N + dst] = -P[neg[m] * N + dst];
}

void orc_bc(const orc_params *p, double *P) {
  const long N = orc_ncell_alloc(p);
  const int NA[3] = {orc_nalloc(p, 0), orc_nalloc(p, 1), orc_nalloc(p, 2)};
  for (int d = 0; d < 3; d++) {
    const int ng = orc_ng(p, d);
    if (ng == 0) continue;
    const int n = p->n[d];
    for (int side = 0; side < 2; side++) {
      const int bc = side ? p->bc_hi[d] : p->bc_lo[d];
      int neg[3] = {-1, -1, -1};
      if (bc == ORC_BC_REFLECT || bc == ORC_BC_POLAR) {
        neg[0] = 2 + d;
        neg[1] = 5 + d;
        neg[2] = 9 + d;
      }
      for (int a = 0; a < NA[(d + 1) % 3]; a++)
        for (int b = 0; b < NA[(d + 2) % 3]; b++)
          for (int m = 0; m < ng; m++) {
            const int gidx = side ? ng + n + m : ng - 1 - m;
            int sidx;
            if (bc == ORC_BC_OUTFLOW) sidx = side ? ng + n - 1 : ng;
            else if (bc == ORC_BC_PERIODIC) sidx = side ? ng + m : ng + n - 1 - m;
            else sidx = side ? ng + n - 1 - m : ng + m;
            int c[3], s[3];
            c[d] = gidx;
            s[d] = sidx;
            c[(d + 1) % 3] = s[(d + 1) % 3] = a;
            c[(d + 2) % 3] = s[(d + 2) % 3] = b;
            if (bc == ORC_BC_POLAR && d == 1 && p->n[2] > 1) {
              /* across the axis: same theta distance, phi shifted by pi */
              const int ng3 = orc_ng(p, 2), n3 = p->n[2];
              if (s[2] < ng3 || s[2] >= ng3 + n3) continue; /* phi ghosts filled later */
              s[2] = ng3 + ((s[2] - ng3 + n3 / 2) % n3);
            }
            copy_cell(P, N, IDX(p, c[0], c[1], c[2]), IDX(p, s[0], s[1], s[2]),
                      (bc == ORC_BC_REFLECT || bc == ORC_BC_POLAR) ? neg : (int[3]){-1, -1, -1});
          }
    }
  }
}

void orc_prim_to_cons(const orc_params *p, const double *P, double *U) {
  const long N = orc_ncell_alloc(p);
#pragma omp parallel for collapse(2)
  for (int k = 0; k < orc_nalloc(p, 2); k++)
    for (int j = 0; j < orc_nalloc(p, 1); j++)
      for (int i = 0; i < orc_nalloc(p, 0); i++) {
        double x1, x2;
        orc_cell_x(p, i, j, &x1, &x2);
        orc_geom g;
        orc_geom_point(p, x1, x2, &g);
        const long c = IDX(p, i, j, k);
        double Pc[12], Uc[12];
        for (int q = 0; q < 12; q++) Pc[q] = P[q * N + c];
        orc_p2u(p, &g, Pc, Uc);
        for (int q = 0; q < 12; q++) U[q * N + c] = Uc[q];
      }
}

/* monotonised-central limited slope */
static double mc_slope(double l, double c, double r) {
  const double dm = c - l, dp = r - c;
  if (dm * dp <= 0.0) return 0.0;
  const double dc = 0.5 * (dm + dp);
  double s = fmin(fabs(2.0 * dm), fmin(fabs(2.0 * dp), fabs(dc)));
  return dc > 0.0 ? s : -s;
}

/* MC-limited linear reconstruction at the face between a4[1] and a4[2]: the
 * right value of cell a4[1] and the left value of cell a4[2] (Sec. 4.3, the
 * MC slopes that PPM also uses) */
void orc_mc_face(const double a4[4], double *PL, double *PR) {
  *PL = a4[1] + 0.5 * mc_slope(a4[0], a4[1], a4[2]);
  *PR = a4[2] - 0.5 * mc_slope(a4[1], a4[2], a4[3]);
}

/* ---- PPM (Colella & Woodward 1984 without contact steepening) ----
 * interface value between the 2nd and 3rd of four cells: the average minus
 * the difference of the two cells' MC slopes over 6 (their eq. 1.6 with
 * monotonised slopes) */
static double ppm_iface(double am, double a0, double a1, double a2) {
  return 0.5 * (a0 + a1) - (mc_slope(a0, a1, a2) - mc_slope(am, a0, a1)) / 6.0;
}

/* left and right values of the middle cell: interface values, flattened
 * towards the cell value by f, then the monotonicity constraints (their
 * eq. 1.10) */
void orc_ppm_cell(const double a5[5], double f, double *aL, double *aR) {
  const double a0 = a5[2];
  double l = ppm_iface(a5[0], a5[1], a5[2], a5[3]);
  double r = ppm_iface(a5[1], a5[2], a5[3], a5[4]);
  l = f * a0 + (1.0 - f) * l;
  r = f * a0 + (1.0 - f) * r;
  if ((r - a0) * (a0 - l) <= 0.0) {
    l = a0;
    r = a0;
  } else {
    const double d = r - l, m6 = 6.0 * (a0 - 0.5 * (l + r));
    if (d * m6 > d * d) l = 3.0 * a0 - 2.0 * r;
    else if (-d * d > d * m6) r = 3.0 * a0 - 2.0 * l;
  }
  *aL = l;
  *aR = r;
}

/* shock flattener (Sec. 4.3 with the FLASH form): for pressure pp and
 * velocity v along d, f = clamp(w2 (|dp1|/|dp2| - w1), 0, 1) where the
 * pressure jump |dp1| = |p(+1) - p(-1)| exceeds eps min(p(+1), p(-1)) and the
 * flow converges (v(-1) > v(+1)), else 0; w1 = 0.75 (SP0), w2 = 10, eps = 0.33 */
#define PPM_W1 0.75
#define PPM_W2 10.0
#define PPM_EPS 0.33
static double flat_raw(const double *pp, const double *v, long c, long st) {
  const double d1 = pp[c + st] - pp[c - st], d2 = pp[c + 2 * st] - pp[c - 2 * st];
  if (!(fabs(d1) > PPM_EPS * fmin(pp[c + st], pp[c - st])) || !(v[c - st] - v[c + st] > 0.0))
    return 0.0;
  return fmax(0.0, fmin(1.0, PPM_W2 * (fabs(d1) / fmax(fabs(d2), 1e-300) - PPM_W1)));
}

/* the upstream maximum: f of the cell and of its neighbour on the high-
 * pressure side */
static double flat_tilde(const double *pp, const double *v, long c, long st) {
  const double f0 = flat_raw(pp, v, c, st);
  const long up = (pp[c + st] - pp[c - st] < 0.0) ? c + st : c - st;
  return fmax(f0, flat_raw(pp, v, up, st));
}

void orc_flattener(const orc_params *p, const double *P, const double *chi_abs,
                   const double *chi_es, double *fl, int keep) {
  const long N = orc_ncell_alloc(p);
  const int NA[3] = {orc_nalloc(p, 0), orc_nalloc(p, 1), orc_nalloc(p, 2)};
  double *pg = malloc(sizeof(double) * N), *pr = malloc(sizeof(double) * N);
  double *wt = malloc(sizeof(double) * N), *vg = malloc(sizeof(double) * N);
  double *vr = malloc(sizeof(double) * N);
  for (int d = 0; d < 3; d++) {
    if (p->n[d] == 1) continue;
    long st = 1;
    for (int e = 0; e < d; e++) st *= NA[e];
    const double dxd = orc_dx(p, d);
    /* per cell: tau-blended pressures (each kind gains w times the other,
     * w = min(1, 2 tau), tau = kappa_tot sqrt(g_dd) dx^d) and velocities */
    for (int k = 0; k < NA[2]; k++)
      for (int j = 0; j < NA[1]; j++)
        for (int i = 0; i < NA[0]; i++) {
          const long c = IDX(p, i, j, k);
          double x1, x2;
          orc_cell_x(p, i, j, &x1, &x2);
          orc_geom g;
          orc_geom_point(p, x1, x2, &g);
          const double rho = P[0 * N + c];
          const double tau = (chi_abs[c] + chi_es[c]) * rho * sqrt(g.gcov[d + 1][d + 1]) * dxd;
          const double w = fmin(1.0, 2.0 * tau);
          const double p_g = (p->gam - 1.0) * P[1 * N + c], p_r = P[8 * N + c] / 3.0;
          pg[c] = p_g + w * p_r;
          pr[c] = p_r + w * p_g;
          wt[c] = w;
          if (p->metric == ORC_KERR_SCHILD) {
            /* the specific mass fluxes sqrt(-g) u^d of gas and radiation */
            double ut[3], ucon[4];
            for (int m = 0; m < 3; m++) ut[m] = P[(2 + m) * N + c];
            orc_ucon(&g, ut, ucon);
            vg[c] = g.gdet * ucon[d + 1];
            for (int m = 0; m < 3; m++) ut[m] = P[(9 + m) * N + c];
            orc_ucon(&g, ut, ucon);
            vr[c] = g.gdet * ucon[d + 1];
          } else {
            /* flat space: u^d = u~^d and sqrt(-g) = 1 */
            vg[c] = P[(2 + d) * N + c];
            vr[c] = P[(9 + d) * N + c];
          }
        }
    int lo[3], hi[3];
    for (int e = 0; e < 3; e++) {
      lo[e] = (p->n[e] > 1) ? orc_ng(p, e) - 1 : 0;
      hi[e] = (p->n[e] > 1) ? orc_ng(p, e) + p->n[e] : 0;
    }
    for (int k = lo[2]; k <= hi[2]; k++)
      for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
          const long c = IDX(p, i, j, k);
          const double fg = flat_tilde(pg, vg, c, st), fr = flat_tilde(pr, vr, c, st);
          const double fm = fmax(fg, fr), w = wt[c];
          double f2[2] = {(1.0 - w) * fg + w * fm, (1.0 - w) * fr + w * fm};
          for (int kind = 0; kind < 2; kind++) {
            double *dst = fl + (long)(2 * d + kind) * N + c;
            *dst = keep ? fmax(*dst, f2[kind]) : f2[kind];
          }
        }
  }
  free(pg); free(pr); free(wt); free(vg); free(vr);
}

/* ---- steps 4-9: reconstruction, face fluxes, wave speeds, Riemann, CT ---- */
void orc_fluxes(const orc_params *p, const double *P, const double *chi_abs, const double *chi_es,
                double *F, double *emf, double *vchar) {
  double *fl = NULL;
  if (p->recon == ORC_RECON_PPM) {
    fl = calloc(6 * orc_ncell_alloc(p), sizeof(double));
    orc_flattener(p, P, chi_abs, chi_es, fl, 0);
  }
  orc_fluxes_fl(p, P, chi_abs, chi_es, fl, F, emf, vchar);
  free(fl);
}

void orc_fluxes_fl(const orc_params *p, const double *P, const double *chi_abs,
                   const double *chi_es, const double *fl, double *F, double *emf, double *vchar) {
  orc_fluxes_s(p, P, chi_abs, chi_es, fl, F, emf, vchar, NULL);
}

/* sqrt(-g) S u^t and sqrt(-g) S u^dir of primitives P at geometry g (the
 * 13th conserved quantity and its flux, Sec. 4 lists of U_q and F_q) */
static void entropy_cons_flux(const orc_params *p, const orc_geom *g, const double *P, int dir,
                              double *Us, double *Fs) {
  double ucon[4];
  orc_ucon(g, P + 2, ucon);
  const double S = orc_entropy(p, P);
  *Us = g->gdet * S * ucon[0];
  if (Fs) *Fs = g->gdet * S * ucon[dir];
}

/* Bf (staggered field, else NULL): the normal field of both face states is
 * the face's own, the faces extend two cells beyond the interior across
 * their direction, VF and SP receive the face velocities and gas speeds
 * (layout in orc_emf_stag) and the flux-CT EMFs are left to the caller. */
static void fluxes_core(const orc_params *p, const double *P, const double *chi_abs,
                        const double *chi_es, const double *fl, double *F, double *emf,
                        double *vchar, double *Fs, const double *Bf, double *VF, double *SP) {
  const long N = orc_ncell_alloc(p);
  memset(F, 0, sizeof(double) * 3 * 12 * N);
  if (Fs) memset(Fs, 0, sizeof(double) * 3 * N);
  memset(emf, 0, sizeof(double) * 3 * N);
  memset(vchar, 0, sizeof(double) * 3 * N);
  const int NA[3] = {orc_nalloc(p, 0), orc_nalloc(p, 1), orc_nalloc(p, 2)};
  for (int d = 0; d < 3; d++) {
    if (p->n[d] == 1) continue;
    int lo[3], hi[3];
    for (int e = 0; e < 3; e++) {
      const int ng = orc_ng(p, e);
      const int ext = Bf ? 2 : 1;
      if (e == d) { lo[e] = ng; hi[e] = ng + p->n[e]; }
      else if (p->n[e] > 1) { lo[e] = ng - ext; hi[e] = ng + p->n[e] + ext - 1; }
      else { lo[e] = 0; hi[e] = 0; }
    }
    long st = 1;
    for (int e = 0; e < d; e++) st *= NA[e];
    const double dxd = orc_dx(p, d);
    double *Fd = F + (long)d * 12 * N;
    /* PPM on Kerr-Schild along r (x1): the vector primitives interpolated
     * as sqrt(-g) times the value (Sec. 4.3); along phi sqrt(-g) does not
     * vary, so the weighting is the identity there */
    const int wgt = (p->recon == ORC_RECON_PPM && p->metric == ORC_KERR_SCHILD && d == 0);
#pragma omp parallel for collapse(2)
    for (int k = lo[2]; k <= hi[2]; k++)
      for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
          const long c = IDX(p, i, j, k);
          const long m2 = c - 2 * st, m1 = c - st, p1 = c + st;
          /* staggered field: faces two cells beyond the interior across d
           * serve only the corner interpolation of the face velocities */
          int outer = 0;
          {
            const int idx[3] = {i, j, k};
            for (int e = 0; e < 3; e++)
              if (Bf && e != d && p->n[e] > 1 &&
                  (idx[e] < orc_ng(p, e) - 1 || idx[e] > orc_ng(p, e) + p->n[e]))
                outer = 1;
          }
          double PL[12], PR[12];
          double x1, x2;
          orc_face_x(p, d + 1, i, j, &x1, &x2);
          orc_geom g;
          orc_geom_point(p, x1, x2, &g);
          if (p->recon == ORC_RECON_PPM) {
            /* left state: right value of cell c - st; right state: left value of c */
            double gc[6] = {1, 1, 1, 1, 1, 1};   /* sqrt(-g) of cells c-3 .. c+2 */
            if (wgt)
              for (int m = 0; m < 6; m++) {
                double y1, y2;
                orc_cell_x(p, i + m - 3, j, &y1, &y2);
                orc_geom gm;
                orc_geom_point(p, y1, y2, &gm);
                gc[m] = gm.gdet;
              }
            for (int q = 0; q < 12; q++) {
              const int kind = q < 8 ? 0 : 1;
              const int vec = wgt && ((q >= 2 && q <= 7) || q >= 9);
              double a5[5], l, r;
              for (int m = 0; m < 5; m++) a5[m] = P[q * N + c + (m - 3) * st] * (vec ? gc[m] : 1.0);
              orc_ppm_cell(a5, fl[(long)(2 * d + kind) * N + m1], &l, &PL[q]);
              for (int m = 0; m < 5; m++) a5[m] = P[q * N + c + (m - 2) * st] * (vec ? gc[m + 1] : 1.0);
              orc_ppm_cell(a5, fl[(long)(2 * d + kind) * N + c], &PR[q], &r);
              if (vec) {
                PL[q] /= g.gdet;
                PR[q] /= g.gdet;
              }
              (void)l;
              (void)r;
            }
          } else {
            for (int q = 0; q < 12; q++) {
              const double a4[4] = {P[q * N + m2], P[q * N + m1], P[q * N + c], P[q * N + p1]};
              orc_mc_face(a4, &PL[q], &PR[q]);
            }
          }
          if (Bf) {
            /* the face's own normal field (zero where sqrt(-g) vanishes) */
            const double bn = g.gdet > 0.0 ? Bf[(long)d * N + c] / g.gdet : 0.0;
            PL[5 + d] = PR[5 + d] = bn;
          }
          const double sdx = sqrt(g.gcov[d + 1][d + 1]) * dxd;
          double UL[12], UR[12], FL[12], FR[12], vgL[2], vrL[2], vgR[2], vrR[2];
          orc_p2u(p, &g, PL, UL);
          orc_p2u(p, &g, PR, UR);
          orc_flux(p, &g, PL, d + 1, FL);
          orc_flux(p, &g, PR, d + 1, FR);
          orc_wavespeeds(p, &g, PL, d + 1, (chi_abs[m1] + chi_es[m1]) * PL[0] * sdx, vgL, vrL);
          orc_wavespeeds(p, &g, PR, d + 1, (chi_abs[c] + chi_es[c]) * PR[0] * sdx, vgR, vrR);
          /* eq. hll: v_min = -min(0, v-_L, v-_R), v_max = max(0, v+_L, v+_R) */
          const double gmin = -fmin(0.0, fmin(vgL[0], vgR[0])), gmax = fmax(0.0, fmax(vgL[1], vgR[1]));
          const double rmin = -fmin(0.0, fmin(vrL[0], vrR[0])), rmax = fmax(0.0, fmax(vrL[1], vrR[1]));
          for (int q = 0; q < 12 && !outer; q++) {
            const double vmin = q < 8 ? gmin : rmin, vmax = q < 8 ? gmax : rmax;
            double f;
            if (p->flux == ORC_FLUX_HLL) {
              if (vmin + vmax > 0.0)
                f = (vmin * FR[q] + vmax * FL[q] - vmin * vmax * (UR[q] - UL[q])) / (vmin + vmax);
              else
                f = 0.5 * (FL[q] + FR[q]);
            } else {
              const double vt = fmax(vmin, vmax); /* eq. lax */
              f = 0.5 * (FR[q] + FL[q] - vt * (UR[q] - UL[q]));
            }
            Fd[q * N + c] = f;
          }
          if (!outer) {
            Fd[(5 + d) * N + c] = 0.0; /* induction flux of the normal component vanishes */
            vchar[(long)d * N + c] = fmax(fmax(gmin, gmax), fmax(rmin, rmax));
          }
          if (Bf) {
            for (int sd = 0; sd < 2; sd++) {
              double ucon[4];
              orc_ucon(&g, (sd ? PR : PL) + 2, ucon);
              for (int m = 0; m < 3; m++)
                VF[((long)((2 * d + sd) * 3) + m) * N + c] = ucon[m + 1] / ucon[0];
            }
            if (!outer) {
              SP[(long)(2 * d) * N + c] = gmin;
              SP[(long)(2 * d + 1) * N + c] = gmax;
            }
          }
          if (Fs && !outer) {
            /* the entropy tracer's flux, with the gas speeds */
            double UsL, UsR, FsL, FsR, f;
            entropy_cons_flux(p, &g, PL, d + 1, &UsL, &FsL);
            entropy_cons_flux(p, &g, PR, d + 1, &UsR, &FsR);
            if (p->flux == ORC_FLUX_HLL) {
              if (gmin + gmax > 0.0)
                f = (gmin * FsR + gmax * FsL - gmin * gmax * (UsR - UsL)) / (gmin + gmax);
              else
                f = 0.5 * (FsL + FsR);
            } else {
              f = 0.5 * (FsR + FsL - fmax(gmin, gmax) * (UsR - UsL));
            }
            Fs[(long)d * N + c] = f;
          }
        }
  }
  if (Bf) return;
  /* flux-CT corner EMFs: emf_a = F_c[B_b] = -F_b[B_c], (a, b, c) cyclic */
  for (int a = 0; a < 3; a++) {
    const int b = (a + 1) % 3, cdim = (a + 2) % 3;
    if (p->n[b] == 1 || p->n[cdim] == 1) continue;
    int lo[3], hi[3];
    lo[a] = orc_ng(p, a);
    hi[a] = orc_ng(p, a) + p->n[a] - 1;
    lo[b] = orc_ng(p, b); hi[b] = orc_ng(p, b) + p->n[b];
    lo[cdim] = orc_ng(p, cdim); hi[cdim] = orc_ng(p, cdim) + p->n[cdim];
    long stb = 1, stc = 1;
    for (int e = 0; e < b; e++) stb *= NA[e];
    for (int e = 0; e < cdim; e++) stc *= NA[e];
    const double *Fb = F + (long)b * 12 * N, *Fc = F + (long)cdim * 12 * N;
    for (int k = lo[2]; k <= hi[2]; k++)
      for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
          const long c = IDX(p, i, j, k);
          double e = 0.25 * (Fc[(5 + b) * N + c] + Fc[(5 + b) * N + c - stb] -
                             Fb[(5 + cdim) * N + c] - Fb[(5 + cdim) * N + c - stc]);
          if (p->metric == ORC_KERR_SCHILD && (b == 1 || cdim == 1)) {
            /* edges lying on the polar axis carry no EMF */
            const int ng2 = orc_ng(p, 1);
            const int onlo = (j == ng2) && (p->bc_lo[1] == ORC_BC_REFLECT || p->bc_lo[1] == ORC_BC_POLAR);
            const int onhi = (j == ng2 + p->n[1]) &&
                             (p->bc_hi[1] == ORC_BC_REFLECT || p->bc_hi[1] == ORC_BC_POLAR);
            if (onlo || onhi) e = 0.0;
          }
          emf[(long)a * N + c] = e;
        }
  }
}

void orc_fluxes_s(const orc_params *p, const double *P, const double *chi_abs,
                  const double *chi_es, const double *fl, double *F, double *emf, double *vchar,
                  double *Fs) {
  fluxes_core(p, P, chi_abs, chi_es, fl, F, emf, vchar, Fs, NULL, NULL, NULL);
}

void orc_fluxes_stag(const orc_params *p, const double *P, const double *Bf,
                     const double *chi_abs, const double *chi_es, const double *fl, double *F,
                     double *emf, double *vchar, double *Fs) {
  const long N = orc_ncell_alloc(p);
  double *VF = calloc(18 * N, sizeof(double));
  double *SP = calloc(6 * N, sizeof(double));
  fluxes_core(p, P, chi_abs, chi_es, fl, F, emf, vchar, Fs, Bf, VF, SP);
  orc_emf_stag(p, Bf, VF, SP, emf);
  free(VF);
  free(SP);
}

double orc_timestep(const orc_params *p, const double *vchar) {
  const long N = orc_ncell_alloc(p);
  const int NA[3] = {orc_nalloc(p, 0), orc_nalloc(p, 1), orc_nalloc(p, 2)};
  double dtmin = INFINITY;
  for (int k = orc_ng(p, 2); k < orc_ng(p, 2) + p->n[2]; k++)
    for (int j = orc_ng(p, 1); j < orc_ng(p, 1) + p->n[1]; j++)
      for (int i = orc_ng(p, 0); i < orc_ng(p, 0) + p->n[0]; i++) {
        const long c = IDX(p, i, j, k);
        double inv = 0.0;
        long st = 1;
        for (int d = 0; d < 3; d++) {
          if (p->n[d] > 1) {
            const double v = fmax(vchar[(long)d * N + c], vchar[(long)d * N + c + st]);
            inv += v / orc_dx(p, d);
          }
          st *= NA[d];
        }
        const double dtc = 1.0 / inv;
        if (dtc < dtmin) dtmin = dtc;
      }
  return p->courant * dtmin;
}

/* eps(a, b, d) = +1 for cyclic (a, b, d) of (0, 1, 2), -1 otherwise */
static double levi(int a, int b, int d) {
  return ((a + 1) % 3 == b && (b + 1) % 3 == d) ? 1.0 : -1.0;
}

/* ---- step 10: U_(i) = a U^n + b U^(k-1) + c dt (-div F + S_M) ---- */
void orc_explicit_update(const orc_params *p, double a, double b, double c, double dt,
                         const double *P, const double *Un, const double *Uprev, const double *F,
                         const double *emf, double *Uexp) {
  const long N = orc_ncell_alloc(p);
  const int NA[3] = {orc_nalloc(p, 0), orc_nalloc(p, 1), orc_nalloc(p, 2)};
  long st[3] = {1, NA[0], (long)NA[0] * NA[1]};
#pragma omp parallel for collapse(2)
  for (int k = orc_ng(p, 2); k < orc_ng(p, 2) + p->n[2]; k++)
    for (int j = orc_ng(p, 1); j < orc_ng(p, 1) + p->n[1]; j++)
      for (int i = orc_ng(p, 0); i < orc_ng(p, 0) + p->n[0]; i++) {
        const long cc = IDX(p, i, j, k);
        double x1, x2;
        orc_cell_x(p, i, j, &x1, &x2);
        orc_geom g;
        orc_geom_point(p, x1, x2, &g);
        double conn[4][4][4], Pc[12], S[12];
        orc_connection(p, x1, x2, conn);
        for (int q = 0; q < 12; q++) Pc[q] = P[q * N + cc];
        orc_source_geom(p, &g, conn, Pc, S);
        double div[12];
        for (int q = 0; q < 12; q++) {
          div[q] = 0.0;
          if (q >= 5 && q <= 7) continue;
          for (int d = 0; d < 3; d++) {
            if (p->n[d] == 1) continue;
            const double *Fd = F + (long)d * 12 * N;
            div[q] += (Fd[q * N + cc + st[d]] - Fd[q * N + cc]) / orc_dx(p, d);
          }
        }
        for (int bb = 0; bb < 3; bb++) {
          const int q = 5 + bb;
          for (int d = 0; d < 3; d++) {
            if (p->n[d] == 1 || d == bb) continue;
            double fm, fp;
            if (p->n[bb] > 1) {
              /* face flux = average of the two corner EMFs adjacent along bb */
              const int aa = 3 - bb - d;
              const double *E = emf + (long)aa * N;
              const double s = levi(aa, bb, d);
              fm = 0.5 * s * (E[cc] + E[cc + st[bb]]);
              fp = 0.5 * s * (E[cc + st[d]] + E[cc + st[d] + st[bb]]);
            } else {
              const double *Fd = F + (long)d * 12 * N;
              fm = Fd[q * N + cc];
              fp = Fd[q * N + cc + st[d]];
            }
            div[q] += (fp - fm) / orc_dx(p, d);
          }
        }
        for (int q = 0; q < 12; q++) {
          const double un = Un[q * N + cc];
          const double up = (b != 0.0) ? Uprev[q * N + cc] : 0.0;
          Uexp[q * N + cc] = a * un + b * up + c * dt * (-div[q] + S[q]);
        }
      }
}

void orc_con2prim(const orc_params *p, const double *U, const double *Pguess, double *P, int *status) {
  const long N = orc_ncell_alloc(p);
#pragma omp parallel for collapse(2)
  for (int k = orc_ng(p, 2); k < orc_ng(p, 2) + p->n[2]; k++)
    for (int j = orc_ng(p, 1); j < orc_ng(p, 1) + p->n[1]; j++)
      for (int i = orc_ng(p, 0); i < orc_ng(p, 0) + p->n[0]; i++) {
        const long c = IDX(p, i, j, k);
        double x1, x2;
        orc_cell_x(p, i, j, &x1, &x2);
        orc_geom g;
        orc_geom_point(p, x1, x2, &g);
        double Uc[12], Pg[12], Pc[12];
        for (int q = 0; q < 12; q++) {
          Uc[q] = U[q * N + c];
          Pg[q] = Pguess[q * N + c];
          Pc[q] = Pg[q];
        }
        int st = 0;
        if (orc_mhd_invert(p, &g, Uc, Pg, Pc) != 0) st |= ORC_ST_C2P_FAIL;
        /* B^i = U_B^i / sqrt(-g) needs no inversion: set also where the MHD
         * inversion failed and the gas primitives stay at the guess */
        for (int q = 5; q <= 7; q++) Pc[q] = Uc[q] / g.gdet;
        orc_rad_invert(p, &g, Uc, 0, Pc);
        for (int q = 0; q < 12; q++) P[q * N + c] = Pc[q];
        if (status) status[c] = st;
      }
}

void orc_implicit_grid(const orc_params *p, const double *Uexp, const double *Pguess, double dt,
                       const double *chi_abs, const double *chi_es, double *Pout, double *Uout,
                       int *iters, int *status) {
  orc_implicit_grid_s(p, Uexp, NULL, Pguess, dt, chi_abs, chi_es, Pout, Uout, iters, status);
}

void orc_implicit_grid_s(const orc_params *p, const double *Uexp, const double *Sexp,
                         const double *Pguess, double dt, const double *chi_abs,
                         const double *chi_es, double *Pout, double *Uout, int *iters,
                         int *status) {
  const long N = orc_ncell_alloc(p);
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
  for (int k = orc_ng(p, 2); k < orc_ng(p, 2) + p->n[2]; k++)
    for (int j = orc_ng(p, 1); j < orc_ng(p, 1) + p->n[1]; j++)
      for (int i = orc_ng(p, 0); i < orc_ng(p, 0) + p->n[0]; i++) {
        const long c = IDX(p, i, j, k);
        double x1, x2;
        orc_cell_x(p, i, j, &x1, &x2);
        orc_geom g;
        orc_geom_point(p, x1, x2, &g);
        double Uc[12], Pg[12], Po[12], Uo[12];
        for (int q = 0; q < 12; q++) {
          Uc[q] = Uexp[q * N + c];
          Pg[q] = Pguess[q * N + c];
        }
        orc_implicit_info info;
        orc_implicit_cell_s(p, &g, Uc, Sexp ? Sexp[c] : NAN, Pg, dt, chi_abs[c], chi_es[c], Po, Uo,
                            &info);
        for (int q = 0; q < 12; q++) {
          Pout[q * N + c] = Po[q];
          Uout[q * N + c] = Uo[q];
        }
        if (iters) iters[c] = info.iters;
        if (status) status[c] = info.status;
      }
}

/* ---- step 13: backups (Sec. 4.11) and floors ---- */
void orc_fixup(const orc_params *p, double *P, double *U, int *status) {
  const long N = orc_ncell_alloc(p);
  const int NA[3] = {orc_nalloc(p, 0), orc_nalloc(p, 1), orc_nalloc(p, 2)};
  const long st[3] = {1, NA[0], (long)NA[0] * NA[1]};
  double *P0 = malloc(sizeof(double) * 12 * N);
  memcpy(P0, P, sizeof(double) * 12 * N);
  for (int k = orc_ng(p, 2); k < orc_ng(p, 2) + p->n[2]; k++)
    for (int j = orc_ng(p, 1); j < orc_ng(p, 1) + p->n[1]; j++)
      for (int i = orc_ng(p, 0); i < orc_ng(p, 0) + p->n[0]; i++) {
        const long c = IDX(p, i, j, k);
        const int idx[3] = {i, j, k};
        int changed = 0;
        /* a failed cell takes the average primitives of its face neighbours
         * with a good energy solution (neither failed nor cold), or of all
         * interior face neighbours if none is good (Sec. 4.11); a cold cell
         * (Sec. 4.11, backups) takes that average for u_g alone */
        const int fail = (status[c] & ORC_ST_FAIL) != 0;
        const int cold = !fail && (status[c] & ORC_ST_COLD);
        if (fail || cold) {
          for (int pass = 0; pass < 2 && !changed; pass++) {
            double acc[12] = {0};
            int cnt = 0;
            for (int d = 0; d < 3; d++) {
              if (p->n[d] == 1) continue;
              for (int s = -1; s <= 1; s += 2) {
                const int nid = idx[d] + s;
                if (nid < orc_ng(p, d) || nid >= orc_ng(p, d) + p->n[d]) continue;
                const long nb = c + s * st[d];
                if (pass == 0 && (status[nb] & (ORC_ST_FAIL | ORC_ST_COLD))) continue;
                for (int q = 0; q < 12; q++) acc[q] += P0[q * N + nb];
                cnt++;
              }
            }
            if (cnt > 0) {
              if (fail)
                for (int q = 0; q < 12; q++) {
                  /* a staggered field is not a primitive of the solve: the
                   * cell keeps its face-centred B */
                  if (p->ct && q >= 5 && q <= 7) continue;
                  P[q * N + c] = acc[q] / cnt;
                }
              else
                P[1 * N + c] = acc[1] / cnt;
              changed = 1;
              if (pass == 1) status[c] |= ORC_ST_NO_GOOD_NB;
            }
          }
        }
        double x1, x2;
        orc_cell_x(p, i, j, &x1, &x2);
        orc_geom g;
        orc_geom_point(p, x1, x2, &g);
        /* the staggered field of a failed cell: the stage's own (its conserved
         * field over sqrt(-g), the mean of its new faces), not the guess that
         * a failed solve or inversion returned */
        if (fail && p->ct)
          for (int q = 5; q <= 7; q++) P[q * N + c] = U[q * N + c] / g.gdet;
        double Pc[12];
        for (int q = 0; q < 12; q++) Pc[q] = P[q * N + c];
        /* floors: rho >= max(rho_floor, b^2/bsq_rho_max), u >= max(u_floor,
         * b^2/bsq_u_max), u <= u_rho_max rho, Ebar >= erad_floor */
        orc_gas s;
        orc_gas_state(p, &g, Pc, &s);
        const double rmin = fmax(p->rho_floor, s.bsq / p->bsq_rho_max);
        const double umin = fmax(p->u_floor, s.bsq / p->bsq_u_max);
        int fl = 0;
        if (Pc[0] < rmin) { Pc[0] = rmin; fl = 1; }
        if (Pc[1] < umin) { Pc[1] = umin; fl = 1; }
        if (Pc[1] > p->u_rho_max * Pc[0]) { Pc[1] = p->u_rho_max * Pc[0]; fl = 1; }
        if (!(Pc[8] >= p->erad_floor)) { Pc[8] = p->erad_floor; fl = 1; }
        if (fl) status[c] |= ORC_ST_FLOOR;
        if (fl || changed) {
          double Uc[12];
          orc_p2u(p, &g, Pc, Uc);
          for (int q = 0; q < 12; q++) {
            P[q * N + c] = Pc[q];
            U[q * N + c] = Uc[q];
          }
        }
      }
  free(P0);
}

/* ---- the time integrators as stage tables (Sec. 4.1) ----
 * Stage i:  U^i = a U^n + b U^j + c dt F^{i-1} + dt sum_k m_k M^k  + g dt M(U^i)
 * F^{i-1}: flux divergence and geometric source of the previous stage's
 * primitives (of P^n at the first stage); M^k: the 4-force source of stage
 * k as its implicit solve found it, (U^k - [bracket])/(g_k dt) in the gas
 * and radiation energy-momentum slots (zero elsewhere, and where the solve
 * failed).  A stage with g = 0 is the final explicit combination; its
 * primitives come from the MHD and radiation inversions. */
typedef struct {
  double a, b;
  int j;          /* stage of the U^j term, -1 for none */
  double c;
  double m[4];
  double g;
} orc_stage;

typedef struct {
  int ns;
  orc_stage s[5];
} orc_scheme;

static orc_scheme scheme_table(int which) {
  orc_scheme S;
  memset(&S, 0, sizeof(S));
  for (int i = 0; i < 5; i++) S.s[i].j = -1;
  if (which == ORC_IMEX2) {
    /* eq. IMEX2, gamma = 1 - 1/sqrt(2) */
    const double ga = 1.0 - 1.0 / sqrt(2.0);
    S.ns = 3;
    S.s[0].a = 1.0; S.s[0].g = ga;
    S.s[1].a = (3.0 * ga - 1.0) / ga; S.s[1].b = (1.0 - 2.0 * ga) / ga; S.s[1].j = 0;
    S.s[1].c = 1.0; S.s[1].g = ga;
    S.s[2].a = 0.5; S.s[2].b = 0.5; S.s[2].j = 1; S.s[2].c = 0.5;
    S.s[2].m[0] = ga; S.s[2].m[1] = 0.5 * (1.0 - ga);
  } else if (which == ORC_IMEX2B) {
    /* eq. IMEX2B */
    S.ns = 4;
    S.s[0].a = 1.0; S.s[0].g = 0.25;
    S.s[1].a = 1.0; S.s[1].c = 0.5; S.s[1].g = 0.25;
    S.s[2].b = 1.0; S.s[2].j = 1; S.s[2].c = 0.5; S.s[2].m[0] = 1.0 / 3.0;
    S.s[2].m[1] = 1.0 / 12.0; S.s[2].g = 1.0 / 3.0;
    S.s[3].a = 1.0 / 3.0; S.s[3].b = 2.0 / 3.0; S.s[3].j = 2; S.s[3].c = 1.0 / 3.0;
    S.s[3].m[0] = S.s[3].m[1] = S.s[3].m[2] = 1.0 / 9.0;
  } else if (which == ORC_IMEX3) {
    /* eq. IMEX3 with the printed alpha, beta, eta */
    const double al = 0.24169426078821, be = 0.06042356519705, et = 0.12915286960590;
    S.ns = 5;
    S.s[0].a = 1.0; S.s[0].g = al;
    S.s[1].a = 2.0; S.s[1].b = -1.0; S.s[1].j = 0; S.s[1].g = al;
    S.s[2].a = 1.0; S.s[2].c = 1.0; S.s[2].m[1] = 1.0 - al; S.s[2].g = al;
    S.s[3].a = 0.75; S.s[3].b = 0.25; S.s[3].j = 2; S.s[3].c = 0.25;
    S.s[3].m[0] = be; S.s[3].m[1] = (-1.0 + al + 4.0 * et) / 4.0;
    S.s[3].m[2] = (2.0 - 5.0 * al - 4.0 * (be + et)) / 4.0; S.s[3].g = al;
    S.s[4].a = 1.0 / 3.0; S.s[4].b = 2.0 / 3.0; S.s[4].j = 3; S.s[4].c = 2.0 / 3.0;
    S.s[4].m[0] = -2.0 * be / 3.0; S.s[4].m[1] = (1.0 - 4.0 * et) / 6.0;
    S.s[4].m[2] = (-1.0 + 4.0 * al + 4.0 * (be + et)) / 6.0; S.s[4].m[3] = 4.0 * (1.0 - al) / 6.0;
  } else {
    /* RK3 (Shu-Osher) with the same coefficients for the implicit part */
    S.ns = 3;
    S.s[0].a = 1.0; S.s[0].c = 1.0; S.s[0].g = 1.0;
    S.s[1].a = 0.75; S.s[1].b = 0.25; S.s[1].j = 0; S.s[1].c = 0.25; S.s[1].g = 0.25;
    S.s[2].a = 1.0 / 3.0; S.s[2].b = 2.0 / 3.0; S.s[2].j = 1; S.s[2].c = 2.0 / 3.0;
    S.s[2].g = 2.0 / 3.0;
  }
  return S;
}

/* sqrt(-g) S u^t of P at every allocated cell */
static void entropy_field(const orc_params *p, const double *P, double *S) {
  const long N = orc_ncell_alloc(p);
  for (int k = 0; k < orc_nalloc(p, 2); k++)
    for (int j = 0; j < orc_nalloc(p, 1); j++)
      for (int i = 0; i < orc_nalloc(p, 0); i++) {
        double x1, x2;
        orc_cell_x(p, i, j, &x1, &x2);
        orc_geom g;
        orc_geom_point(p, x1, x2, &g);
        const long c = IDX(p, i, j, k);
        double Pc[12];
        for (int q = 0; q < 12; q++) Pc[q] = P[q * N + c];
        entropy_cons_flux(p, &g, Pc, 1, &S[c], NULL);
      }
}

/* the entropy tracer's explicit stage value at interior cells:
 * a Sn + b U_S(Pprev) + c dt (-div Fs); Sn = U_S(P^n); no flux term (Fs may
 * be NULL) where c = 0 */
static void entropy_update(const orc_params *p, double a, double b, double c, double dt,
                           const double *Sn, const double *Pprev, const double *Fs,
                           double *Sexp) {
  const long N = orc_ncell_alloc(p);
  const int NA[3] = {orc_nalloc(p, 0), orc_nalloc(p, 1), orc_nalloc(p, 2)};
  const long st[3] = {1, NA[0], (long)NA[0] * NA[1]};
  double *Sp = malloc(sizeof(double) * N);
  entropy_field(p, Pprev, Sp);
  for (long q = 0; q < N; q++) Sexp[q] = NAN;
  for (int k = orc_ng(p, 2); k < orc_ng(p, 2) + p->n[2]; k++)
    for (int j = orc_ng(p, 1); j < orc_ng(p, 1) + p->n[1]; j++)
      for (int i = orc_ng(p, 0); i < orc_ng(p, 0) + p->n[0]; i++) {
        const long cc = IDX(p, i, j, k);
        double div = 0.0;
        for (int d = 0; d < 3 && c != 0.0; d++)
          if (p->n[d] > 1) div += (Fs[(long)d * N + cc + st[d]] - Fs[(long)d * N + cc]) / orc_dx(p, d);
        Sexp[cc] = a * Sn[cc] + (b != 0.0 ? b * Sp[cc] : 0.0) - (c != 0.0 ? c * dt * div : 0.0);
      }
  free(Sp);
}

/* one full step of the scheme p->scheme (Sec. 4.1); each implicit stage is
 * implicit in its own new value with dt_k = g dt */
int orc_step(const orc_params *p, double *P, double *U, const double *chi_abs, const double *chi_es,
             double *dt, int dt_fixed, int *status, int *iters) {
  if (p->ct) return -1;
  return orc_step_stag(p, P, U, NULL, chi_abs, chi_es, dt, dt_fixed, status, iters);
}

/* Bf (staggered field, p->ct = 1): the face field [3][N] in and out; each
 * stage's faces are a Bf^n + b Bf^(j) + c dt (-curl EMF) with the stage's own
 * coefficients (Sec. 4.1; no EMF term where c = 0, and the implicit part
 * leaves the field alone), and the stage's cell-centred conserved field their
 * mean (Sec. 4.2 steps 8-10) */
int orc_step_stag(const orc_params *p, double *P, double *U, double *Bf, const double *chi_abs,
                  const double *chi_es, double *dt, int dt_fixed, int *status, int *iters) {
  if ((Bf != NULL) != (p->ct != 0)) return -1;
  const orc_scheme S = scheme_table(p->scheme);
  const long N = orc_ncell_alloc(p);
  const size_t B12 = sizeof(double) * 12 * N;
  double *F = malloc(sizeof(double) * 3 * 12 * N);
  double *emf = malloc(sizeof(double) * 3 * N);
  double *vch = malloc(sizeof(double) * 3 * N);
  double *Uexp = malloc(B12);
  double *Un = malloc(B12);
  double *Pk = malloc(B12);
  double *Ust[5], *Mst[5];
  int need_m[5] = {0};
  for (int i = 0; i < S.ns; i++)
    for (int k = 0; k < 4; k++)
      if (S.s[i].m[k] != 0.0) need_m[k] = 1;
  for (int i = 0; i < S.ns; i++) {
    Ust[i] = malloc(B12);
    memcpy(Ust[i], U, B12);   /* ghost cells keep U^n */
    Mst[i] = need_m[i] ? calloc(12 * N, sizeof(double)) : NULL;
  }
  int *st = calloc(N, sizeof(int));
  int *stacc = calloc(N, sizeof(int));
  int *it = calloc(N, sizeof(int));
  memcpy(Un, U, B12);
  memcpy(Pk, P, B12);
  memcpy(Uexp, U, B12);
  int nbad = 0;
  if (iters) memset(iters, 0, sizeof(int) * N);
  int fresh = 0;   /* F holds the fluxes of Pk */
  /* PPM flattener of the step: the largest over its sub-steps so far */
  double *fl = (p->recon == ORC_RECON_PPM) ? calloc(6 * N, sizeof(double)) : NULL;
  int nflux = 0;
  /* staggered field: Bf^n, each stage's faces, the current stage input */
  const size_t B3 = sizeof(double) * 3 * N;
  double *Bn = NULL, *Bst[5] = {NULL}, *Bk = NULL;
  if (Bf) {
    Bn = malloc(B3);
    memcpy(Bn, Bf, B3);
    for (int i = 0; i < S.ns; i++) {
      Bst[i] = malloc(B3);
      memcpy(Bst[i], Bf, B3);
    }
    Bk = Bn;
  }
  /* the full cascade's entropy equation: the explicit entropy of each stage,
   * a U_S(P^n) + b U_S(P^(j)) + c dt (-div F_S) + dt sum_k m_k M_S^k, the
   * tracer taken from the primitives at every sub-step (Sec. 4.2 step 2: all
   * U_q from P_q; in every table the stage j of a b term is the previous
   * one), and an implicit stage's entropy source stored as computed, M_S^k =
   * (U_S(P^k) - explicit)/(g dt) from its solution before the fix-ups (zero
   * where the solve failed), as the other sources M^k */
  const int ent = p->cascade;
  double *Fs = ent ? malloc(sizeof(double) * 3 * N) : NULL;
  double *Sn = ent ? malloc(sizeof(double) * N) : NULL;
  double *Sexp = ent ? malloc(sizeof(double) * N) : NULL;
  double *MS[4] = {NULL};
  if (ent) {
    entropy_field(p, P, Sn);
    for (int k = 0; k < 4; k++) MS[k] = need_m[k] ? calloc(N, sizeof(double)) : NULL;
  }
#define STEP_FLUXES()                                              \
  do {                                                             \
    if (fl) orc_flattener(p, Pk, chi_abs, chi_es, fl, nflux > 0);  \
    if (Bk) {                                                      \
      orc_bc_face(p, Bk);                                          \
      orc_fluxes_stag(p, Pk, Bk, chi_abs, chi_es, fl, F, emf, vch, Fs); \
    } else {                                                       \
      orc_fluxes_s(p, Pk, chi_abs, chi_es, fl, F, emf, vch, Fs);   \
    }                                                              \
    nflux++;                                                       \
  } while (0)
  if (!dt_fixed) {
    /* Courant dt from the wave speeds of P^n (Sec. 4.4) */
    orc_bc(p, Pk);
    STEP_FLUXES();
    *dt = orc_timestep(p, vch);
    fresh = 1;
  }
  for (int i = 0; i < S.ns; i++) {
    const orc_stage *s = &S.s[i];
    const double *Uj = (s->j >= 0) ? Ust[s->j] : Un;
    if (s->c != 0.0) {
      if (!fresh) {
        orc_bc(p, Pk);
        STEP_FLUXES();
      }
      orc_explicit_update(p, s->a, s->b, s->c, *dt, Pk, Un, Uj, F, emf, Uexp);
      if (ent) entropy_update(p, s->a, s->b, s->c, *dt, Sn, Pk, Fs, Sexp);
      if (Bf) {
        orc_face_update(p, s->a, s->b, s->c, *dt, Bn, (s->j >= 0) ? Bst[s->j] : Bn, emf, Bst[i]);
        orc_face_to_center(p, Bst[i], NULL, Uexp);
        Bk = Bst[i];
      }
    } else {
      for (long q = 0; q < 12 * N; q++) Uexp[q] = s->a * Un[q] + (s->b != 0.0 ? s->b * Uj[q] : 0.0);
      if (ent) entropy_update(p, s->a, s->b, 0.0, *dt, Sn, Pk, NULL, Sexp);
      if (Bf) {
        orc_face_update(p, s->a, s->b, 0.0, *dt, Bn, (s->j >= 0) ? Bst[s->j] : Bn, NULL, Bst[i]);
        orc_face_to_center(p, Bst[i], NULL, Uexp);
        Bk = Bst[i];
      }
    }
    for (int k = 0; k < i && k < 4; k++) {
      if (s->m[k] == 0.0) continue;
      for (long q = 0; q < 12 * N; q++) Uexp[q] += *dt * s->m[k] * Mst[k][q];
      if (ent)
        for (long q = 0; q < N; q++) Sexp[q] += *dt * s->m[k] * MS[k][q];
    }
    if (s->g > 0.0) {
      orc_implicit_grid_s(p, Uexp, ent ? Sexp : NULL, Pk, s->g * (*dt), chi_abs, chi_es, Pk, Ust[i],
                          it, st);
      if (i < 4 && need_m[i]) {
        const double gdt = s->g * (*dt);
        for (long c = 0; c < N; c++)
          for (int q = 0; q < 12; q++) {
            const int slot = (q >= 1 && q <= 4) || q >= 8;
            Mst[i][q * N + c] = (slot && !(st[c] & ORC_ST_FAIL))
                                    ? (Ust[i][q * N + c] - Uexp[q * N + c]) / gdt : 0.0;
          }
        if (ent) {
          double *Sk = malloc(sizeof(double) * N);
          entropy_field(p, Pk, Sk);
          for (int k = orc_ng(p, 2); k < orc_ng(p, 2) + p->n[2]; k++)
            for (int j = orc_ng(p, 1); j < orc_ng(p, 1) + p->n[1]; j++)
              for (int ii = orc_ng(p, 0); ii < orc_ng(p, 0) + p->n[0]; ii++) {
                const long c = IDX(p, ii, j, k);
                MS[i][c] = (st[c] & ORC_ST_FAIL) ? 0.0 : (Sk[c] - Sexp[c]) / gdt;
              }
          free(Sk);
        }
      }
    } else {
      /* final explicit combination: inversions; a failed MHD inversion is a
       * failed cell (neighbour average) */
      double *Pg = malloc(B12);
      memcpy(Pg, Pk, B12);
      orc_con2prim(p, Uexp, Pg, Pk, st);
      free(Pg);
      memcpy(Ust[i], Uexp, B12);
      for (long c = 0; c < N; c++) {
        if (st[c] & ORC_ST_C2P_FAIL) st[c] |= ORC_ST_FAIL;
        it[c] = 0;
      }
    }
    orc_fixup(p, Pk, Ust[i], st);
    fresh = 0;
    for (long c = 0; c < N; c++) {
      stacc[c] |= st[c];
      if (iters) iters[c] += it[c];
    }
  }
  if (status) memcpy(status, stacc, sizeof(int) * N);
  /* write back (ghost cells of P keep the last fill) */
  memcpy(P, Pk, B12);
  memcpy(U, Ust[S.ns - 1], B12);
  if (Bf) {
    memcpy(Bf, Bst[S.ns - 1], B3);
    free(Bn);
    for (int i = 0; i < S.ns; i++) free(Bst[i]);
  }
  for (long c = 0; c < N; c++)
    if (stacc[c] & ORC_ST_FAIL) nbad++;
  for (int i = 0; i < S.ns; i++) {
    free(Ust[i]);
    free(Mst[i]);
  }
  free(F); free(emf); free(vch); free(Uexp); free(Un); free(Pk); free(st); free(stacc);
  free(it);
  free(fl);
  free(Fs);
  free(Sn);
  free(Sexp);
  for (int k = 0; k < 4; k++) free(MS[k]);
#undef STEP_FLUXES
  return nbad;
}
