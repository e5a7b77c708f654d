/*
 * Oracle of the staggered magnetic field: face-centred B^i with corner EMFs
 * from a four-state Riemann solution (Sec. 4, the locations of the magnetic
 * P_q, U_q and their fluxes; Sec. 4.2 steps 8-11; Sec. 4.4 on the EMF wave
 * speeds; the four-state HLL/LAXF form of Del Zanna et al. 2007).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Bf[p][c] is sqrt(-g) B^(p+1) on the lower p-face of cell c (on an
 * inactive dimension p the face is the cell itself).  The EMF of edge e of
 * cell c (its lower corner in the other two directions, p = e+1, q = e+2
 * mod 3) is Phi_e = F^q[B^p] = sqrt(-g)(B^p v^q - B^q v^p) = -F^p[B^q], the
 * same orientation the flux-CT EMFs use.  Readings: the corner velocity
 * states come from the face states (Sec. 4.2 step 4) of both in-plane
 * directions, each interpolated along the other with MC slopes and the two
 * averaged; the corner wave speeds are the mean of those of the two faces
 * adjacent to the edge; the face field is sqrt(-g) B interpolated along the
 * other in-plane direction; the cell-centred field is the mean of its two
 * faces.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "oracle_internal.h"

#define IDX(p, i, j, k) ((long)(i) + (long)orc_nalloc(p, 0) * ((long)(j) + (long)orc_nalloc(p, 1) * (long)(k)))

static long stride(const orc_params *p, int d) {
  long s = 1;
  for (int e = 0; e < d; e++) s *= orc_nalloc(p, e);
  return s;
}

/* sqrt(-g) on the lower d-face of the cell at allocated (i, j) */
static double face_gdet(const orc_params *p, int d, int i, int j) {
  double x1, x2;
  orc_face_x(p, d + 1, i, j, &x1, &x2);
  orc_geom g;
  orc_geom_point(p, x1, x2, &g);
  return g.gdet;
}

/* the face value of the primitive B^(q+1) carried from face src to face dst:
 * sqrt(-g) B at dst from B at src */
static double carry(const orc_params *p, int q, const int *dst, const int *src, double v) {
  const double gd = face_gdet(p, q, dst[0], dst[1]), gs = face_gdet(p, q, src[0], src[1]);
  if (gd == gs) return v;
  if (gs == 0.0) return 0.0;
  return v / gs * gd;
}

/* ---- ghost faces (Sec. 4.2 step 1 for the face field) ----
 * Dimension by dimension as for the cell-centred primitives.  Across a
 * dimension d other than the face's own direction q the faces follow the
 * cell rule; along q the evolved faces are [ng, ng+n] (periodic: [ng,
 * ng+n), face ng+n being face ng); outflow copies the boundary face,
 * periodic wraps, REFLECT and POLAR mirror about the boundary face with the
 * sign of B^q flipped.  The primitive B is carried (sqrt(-g) of the ghost
 * face applied). */
void orc_bc_face(const orc_params *p, double *Bf) {
  const long N = orc_ncell_alloc(p);
  const int NA[3] = {orc_nalloc(p, 0), orc_nalloc(p, 1), orc_nalloc(p, 2)};
  for (int d = 0; d < 3; d++) {
    const int ng = orc_ng(p, d);
    if (ng == 0) continue;
    const int n = p->n[d];
    for (int q = 0; q < 3; q++) {
      double *B = Bf + (long)q * N;
      for (int side = 0; side < 2; side++) {
        const int bc = side ? p->bc_hi[d] : p->bc_lo[d];
        const int mirror = (bc == ORC_BC_REFLECT || bc == ORC_BC_POLAR);
        /* ghost positions along d and their sources */
        int gl[16], sl[16], cnt = 0;
        if (q != d) {
          for (int m = 0; m < ng; m++) {
            gl[cnt] = side ? ng + n + m : ng - 1 - m;
            if (bc == ORC_BC_OUTFLOW) sl[cnt] = side ? ng + n - 1 : ng;
            else if (bc == ORC_BC_PERIODIC) sl[cnt] = side ? ng + m : ng + n - 1 - m;
            else sl[cnt] = side ? ng + n - 1 - m : ng + m;
            cnt++;
          }
        } else {
          if (side == 0) {
            for (int f = 0; f < ng; f++) {
              gl[cnt] = f;
              if (bc == ORC_BC_OUTFLOW) sl[cnt] = ng;
              else if (bc == ORC_BC_PERIODIC) sl[cnt] = f + n;
              else sl[cnt] = 2 * ng - f;
              cnt++;
            }
          } else {
            const int first = (bc == ORC_BC_PERIODIC) ? ng + n : ng + n + 1;
            for (int f = first; f < NA[d]; f++) {
              gl[cnt] = f;
              if (bc == ORC_BC_OUTFLOW) sl[cnt] = ng + n;
              else if (bc == ORC_BC_PERIODIC) sl[cnt] = f - n;
              else sl[cnt] = 2 * (ng + n) - f;
              cnt++;
            }
          }
        }
        const double sgn = (mirror && q == d) ? -1.0 : 1.0;
        for (int a = 0; a < NA[(d + 1) % 3]; a++)
          for (int b = 0; b < NA[(d + 2) % 3]; b++)
            for (int m = 0; m < cnt; m++) {
              int c[3], s[3];
              c[d] = gl[m];
              s[d] = sl[m];
              c[(d + 1) % 3] = s[(d + 1) % 3] = a;
              c[(d + 2) % 3] = s[(d + 2) % 3] = b;
              if (bc == ORC_BC_POLAR && d == 1 && p->n[2] > 1) {
                /* across the axis: phi shifted by pi (phi ghosts filled later) */
                const int ng3 = orc_ng(p, 2), n3 = p->n[2];
                if (s[2] < ng3 || s[2] >= ng3 + n3) continue;
                s[2] = ng3 + ((s[2] - ng3 + n3 / 2) % n3);
              }
              const double v = B[IDX(p, s[0], s[1], s[2])];
              B[IDX(p, c[0], c[1], c[2])] = sgn * carry(p, q, c, s, v);
            }
      }
    }
  }
}

/* ---- Sec. 4.2 step 8: the cell-centred field from the faces ----
 * U[5+p] = mean of sqrt(-g) B^p on the cell's two p-faces (the face itself
 * on an inactive dimension), P[5+p] = U[5+p] / sqrt(-g) at the centre;
 * interior cells, other slots untouched (P or U may be NULL). */
void orc_face_to_center(const orc_params *p, const double *Bf, double *P, double *U) {
  const long N = orc_ncell_alloc(p);
  for (int k = orc_ng(p, 2); k < orc_ng(p, 2) + p->n[2]; k++)
    for (int j = orc_ng(p, 1); j < orc_ng(p, 1) + p->n[1]; j++)
      for (int i = orc_ng(p, 0); i < orc_ng(p, 0) + p->n[0]; i++) {
        const long c = IDX(p, i, j, k);
        double x1, x2;
        orc_cell_x(p, i, j, &x1, &x2);
        orc_geom g;
        orc_geom_point(p, x1, x2, &g);
        for (int q = 0; q < 3; q++) {
          const double *B = Bf + (long)q * N;
          const double u = (p->n[q] > 1) ? 0.5 * (B[c] + B[c + stride(p, q)]) : B[c];
          if (U) U[(5 + q) * N + c] = u;
          if (P) P[(5 + q) * N + c] = u / g.gdet;
        }
      }
}

/* MC-limited values on the two sides of the point between a[1] and a[2] */
static void mc_pair(const double a[4], double *lo, double *hi) { orc_mc_face(a, lo, hi); }

/* ---- Sec. 4.2 steps 8-9: corner EMFs from the four-state solution ----
 * VF[((2 d + s) * 3 + m) N + c]: lab-frame v^(m+1) = u^(m+1)/u^t of face
 * state s (0 left, 1 right) on the lower d-face of c; SP[(2 d + s) N + c]:
 * the face's gas v_min (s = 0) and v_max (s = 1) of eq. hll. */
void orc_emf_stag(const orc_params *p, const double *Bf, const double *VF, const double *SP,
                  double *emf) {
  const long N = orc_ncell_alloc(p);
  memset(emf, 0, sizeof(double) * 3 * N);
  for (int e = 0; e < 3; e++) {
    const int pd = (e + 1) % 3, qd = (e + 2) % 3;
    const int act_p = p->n[pd] > 1, act_q = p->n[qd] > 1;
    if (!act_p && !act_q) continue;
    const long sp = stride(p, pd), sq = stride(p, qd);
    int lo[3], hi[3];
    for (int d = 0; d < 3; d++) {
      lo[d] = orc_ng(p, d);
      hi[d] = orc_ng(p, d) + (p->n[d] > 1 ? p->n[d] : 0);   /* inclusive */
    }
    const double *Bp = Bf + (long)pd * N, *Bq = Bf + (long)qd * N;
    for (int k = lo[2]; k <= hi[2]; k++)
      for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
          const long c = IDX(p, i, j, k);
          /* field states: sqrt(-g) B^p along q (S below, N above), sqrt(-g)
           * B^q along p (L below, R above) */
          double bp[2], bq[2];
          if (act_q) {
            const double a[4] = {Bp[c - 2 * sq], Bp[c - sq], Bp[c], Bp[c + sq]};
            mc_pair(a, &bp[0], &bp[1]);
          } else {
            bp[0] = bp[1] = Bp[c];
          }
          if (act_p) {
            const double a[4] = {Bq[c - 2 * sp], Bq[c - sp], Bq[c], Bq[c + sp]};
            mc_pair(a, &bq[0], &bq[1]);
          } else {
            bq[0] = bq[1] = Bq[c];
          }
          /* velocity states v[a][b][0] = v^p, v[a][b][1] = v^q, a the side
           * along p, b along q */
          double v[2][2][2] = {{{0}}};
          int nsrc = 0;
          if (act_p) {
            /* p-face states (sides a) interpolated along q */
            for (int a = 0; a < 2; a++)
              for (int m = 0; m < 2; m++) {
                const double *V = VF + ((long)((2 * pd + a) * 3) + (m ? qd : pd)) * N;
                double s0, s1;
                if (act_q) {
                  const double w[4] = {V[c - 2 * sq], V[c - sq], V[c], V[c + sq]};
                  mc_pair(w, &s0, &s1);
                } else {
                  s0 = s1 = V[c];
                }
                v[a][0][m] += s0;
                v[a][1][m] += s1;
              }
            nsrc++;
          }
          if (act_q) {
            /* q-face states (sides b) interpolated along p */
            for (int b = 0; b < 2; b++)
              for (int m = 0; m < 2; m++) {
                const double *V = VF + ((long)((2 * qd + b) * 3) + (m ? qd : pd)) * N;
                double s0, s1;
                if (act_p) {
                  const double w[4] = {V[c - 2 * sp], V[c - sp], V[c], V[c + sp]};
                  mc_pair(w, &s0, &s1);
                } else {
                  s0 = s1 = V[c];
                }
                v[0][b][m] += s0;
                v[1][b][m] += s1;
              }
            nsrc++;
          }
          if (nsrc == 2)
            for (int a = 0; a < 2; a++)
              for (int b = 0; b < 2; b++)
                for (int m = 0; m < 2; m++) v[a][b][m] *= 0.5;
          /* per-direction weights of the two sides and the dissipation
           * coefficient: HLL (eq. hll) w_lo = v_max/(v_min+v_max), w_hi =
           * v_min/(v_min+v_max), d = v_min v_max/(v_min+v_max); LAXF (eq.
           * lax) 1/2, 1/2, v_tot/2; a single state on an inactive direction */
          double wp[2], wq[2], dp = 0.0, dq = 0.0;
          for (int dir = 0; dir < 2; dir++) {
            const int act = dir ? act_q : act_p;
            double *w = dir ? wq : wp, *dd = dir ? &dq : &dp;
            if (!act) {
              w[0] = 1.0;
              w[1] = 0.0;
              continue;
            }
            const int fd = dir ? qd : pd;           /* the faces' direction  */
            const long so = dir ? sp : sq;          /* along the edge's other axis */
            const int other_act = dir ? act_p : act_q;
            const double *Smin = SP + (long)(2 * fd) * N, *Smax = SP + (long)(2 * fd + 1) * N;
            const double vmin = other_act ? 0.5 * (Smin[c - so] + Smin[c]) : Smin[c];
            const double vmax = other_act ? 0.5 * (Smax[c - so] + Smax[c]) : Smax[c];
            if (p->flux == ORC_FLUX_HLL) {
              if (vmin + vmax > 0.0) {
                w[0] = vmax / (vmin + vmax);
                w[1] = vmin / (vmin + vmax);
                *dd = vmin * vmax / (vmin + vmax);
              } else {
                w[0] = w[1] = 0.5;
              }
            } else {
              w[0] = w[1] = 0.5;
              *dd = 0.5 * fmax(vmin, vmax);
            }
          }
          double phi = 0.0;
          for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
              const double wab = wp[a] * wq[b];
              if (wab == 0.0) continue;
              phi += wab * (bp[b] * v[a][b][1] - bq[a] * v[a][b][0]);
            }
          phi += -dq * (bp[1] - bp[0]) + dp * (bq[1] - bq[0]);
          if (p->metric == ORC_KERR_SCHILD && (pd == 1 || qd == 1)) {
            /* edges lying on the polar axis carry no EMF */
            const int ng2 = orc_ng(p, 1);
            const int onlo = (j == ng2) && (p->bc_lo[1] == ORC_BC_REFLECT || p->bc_lo[1] == ORC_BC_POLAR);
            const int onhi = (j == ng2 + p->n[1]) &&
                             (p->bc_hi[1] == ORC_BC_REFLECT || p->bc_hi[1] == ORC_BC_POLAR);
            if (onlo || onhi) phi = 0.0;
          }
          emf[(long)e * N + c] = phi;
        }
  }
}

/* ---- Sec. 4.2 step 10 for the face field ----
 * Bout^p = a Bn^p + b Bprev^p + c dt (-sum_{d != p} d_d F^d[B^p]) on the
 * evolved faces, F^d[B^p] = +Phi_e (e = 3-p-d) when p = e+1 mod 3, else
 * -Phi_e; by Stokes' theorem each face's change is the circulation of the
 * EMF around it, so the discrete divergence of Bf never changes.  c = 0 (an
 * IMEX stage without explicit fluxes): no EMF term, emf may be NULL. */
void orc_face_update(const orc_params *p, double a, double b, double c, double dt,
                     const double *Bn, const double *Bprev, const double *emf, double *Bout) {
  const long N = orc_ncell_alloc(p);
  for (int pd = 0; pd < 3; pd++) {
    int lo[3], hi[3];
    for (int d = 0; d < 3; d++) {
      lo[d] = orc_ng(p, d);
      hi[d] = orc_ng(p, d) + (p->n[d] > 1 ? p->n[d] : 1) - 1;
      if (d == pd && p->n[d] > 1) hi[d]++;   /* the upper boundary face */
    }
    for (int k = lo[2]; k <= hi[2]; k++)
      for (int j = lo[1]; j <= hi[1]; j++)
        for (int i = lo[0]; i <= hi[0]; i++) {
          const long f = IDX(p, i, j, k);
          double curl = 0.0;
          for (int d = 0; d < 3 && c != 0.0; d++) {
            if (d == pd || p->n[d] == 1) continue;
            const int e = 3 - pd - d;
            const double s = ((e + 1) % 3 == pd) ? 1.0 : -1.0;
            const double *E = emf + (long)e * N;
            curl += s * (E[f + stride(p, d)] - E[f]) / orc_dx(p, d);
          }
          const long o = (long)pd * N + f;
          Bout[o] = a * Bn[o] + (b != 0.0 ? b * Bprev[o] : 0.0) - (c != 0.0 ? c * dt * curl : 0.0);
        }
  }
}
