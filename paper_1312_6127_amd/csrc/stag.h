// Staggered face-centred magnetic field (Sec. 4: the magnetic P_q and U_q
// live on cell faces and their fluxes, the EMFs, on the corners of the
// planes through the cell centre; Sec. 4.2 steps 8-11; Sec. 4.4 last
// paragraph for the EMF wave speeds) with the four-state HLL/LAXF corner EMF
// of Del Zanna et al. (2007).
//
// Bf [3][Ntot]: sqrt(-g) B^(p+1) on the lower p-face of each cell (the cell
// itself on an inactive dimension p).  Edge e of cell c lies at the cell's
// lower corner in p = e+1 and q = e+2 (mod 3); its EMF is
//   Phi_e = F^q[B^p] = sqrt(-g) (B^p v^q - B^q v^p) = -F^p[B^q],
// the orientation the flux-CT EMFs use.  Corner states: sqrt(-g) B^p
// interpolated along q and sqrt(-g) B^q along p from the faces, the face
// velocity states (flux kernel, STAG) of each active in-plane direction
// interpolated along the other, the two averaged; MC slopes throughout.
// Corner speeds: the mean of the gas v_min, v_max of the two faces adjacent
// to the edge.
#pragma once
#include "kernels.h"

// sqrt(-g) on the lower q-face of the cell at table position (i, j)
DEV double face_gdet(const Ctx& C, int q, int i, int j) {
  const double* tab = (q == 0) ? C.geo_f1 : ((q == 1) ? C.geo_f2 : C.geo_c);
  return tab[GE_GDET * C.npos + i + C.N[0] * j];
}

// sqrt(-g) B on face dst from sqrt(-g) B = v on face src (the primitive B
// carried between the faces)
DEV double carry_face(const Ctx& C, int q, const int* dst, const int* src, double v) {
  const double gd = face_gdet(C, q, dst[0], dst[1]), gs = face_gdet(C, q, src[0], src[1]);
  if (gd == gs) return v;
  if (gs == 0.0) return 0.0;
  return v / gs * gd;
}

// ---------------------------------------------------------------------------
// ghost faces (Sec. 4.2 step 1 for the face field).  Thread t: component q
// = t / Ntot at cell c = t mod Ntot.  The fill dimension by dimension (x1,
// x2, x3 passes, each copying whole planes including earlier ghosts) is
// composed into a chain of positions from the source face to the ghost;
// the carry and sign of each pass are applied in pass order.  Across a
// dimension other than q the faces follow the cell rule; along q the
// evolved faces are [ng, ng+n] ([ng, ng+n) when periodic), outflow copies
// the boundary face, periodic wraps, REFLECT and POLAR mirror about the
// boundary face and negate B^q.
// ---------------------------------------------------------------------------
DEV void face_bc_at(const Ctx& C, double* __restrict__ Bf, long t) {
  if (t >= 3 * C.Ntot) return;
  const int q = (int)(t / C.Ntot);
  const long c = t - (long)q * C.Ntot;
  int sd[3];
  sd[0] = c % C.N[0];
  sd[1] = (c / C.N[0]) % C.N[1];
  sd[2] = c / ((long)C.N[0] * C.N[1]);
  int chain[4][3];   // chain[3]: the ghost; chain[d]: after undoing passes 2..d
  double sgn[3] = {1.0, 1.0, 1.0};
  for (int a = 0; a < 3; a++) chain[3][a] = sd[a];
  bool ghost = false;
  for (int d = 2; d >= 0; d--) {
    const int ng = C.ng[d], n = C.n[d];
    if (ng > 0) {
      const int f = sd[d];
      if (d != q) {
        if (!(f >= ng && f < ng + n)) {
          ghost = true;
          const int side = f >= ng + n;
          const int m = side ? f - ng - n : ng - 1 - f;
          const int bc = side ? C.bc_hi[d] : C.bc_lo[d];
          if (bc == GRRMHD_BC_OUTFLOW) sd[d] = side ? ng + n - 1 : ng;
          else if (bc == GRRMHD_BC_PERIODIC) sd[d] = side ? ng + m : ng + n - 1 - m;
          else sd[d] = side ? ng + n - 1 - m : ng + m;
          if (bc == GRRMHD_BC_POLAR && d == 1 && C.n[2] > 1)
            sd[2] = C.ng[2] + (sd[2] - C.ng[2] + C.n[2] / 2) % C.n[2];
        }
      } else {
        const int lo = C.bc_lo[d], hi = C.bc_hi[d];
        const int top = (hi == GRRMHD_BC_PERIODIC) ? ng + n - 1 : ng + n;   // last evolved face
        if (f < ng || f > top) {
          ghost = true;
          const int side = f > top;
          const int bc = side ? hi : lo;
          if (bc == GRRMHD_BC_OUTFLOW) sd[d] = side ? ng + n : ng;
          else if (bc == GRRMHD_BC_PERIODIC) sd[d] = side ? f - n : f + n;
          else {
            sd[d] = side ? 2 * (ng + n) - f : 2 * ng - f;
            sgn[d] = -1.0;
          }
          if (bc == GRRMHD_BC_POLAR && d == 1 && C.n[2] > 1)
            sd[2] = C.ng[2] + (sd[2] - C.ng[2] + C.n[2] / 2) % C.n[2];
        }
      }
    }
    for (int a = 0; a < 3; a++) chain[d][a] = sd[a];
  }
  if (!ghost) return;
  double* B = Bf + (long)q * C.Ntot;
  double v = B[cell_index(C, chain[0][0], chain[0][1], chain[0][2])];
  for (int d = 0; d < 3; d++)   // pass d carries chain[d] to chain[d + 1]
    v = sgn[d] * carry_face(C, q, chain[d + 1], chain[d], v);
  B[c] = v;
}

__global__ void LB(256) k_bc_faces(Ctx C, double* __restrict__ Bf) {
  face_bc_at(C, Bf, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Sec. 4.2 step 8: U[5+q] = mean of the cell's two q-faces (the face itself
// on an inactive q), P[5+q] = U[5+q] / sqrt(-g) at the centre; interior
// cells; P or U may be null
// ---------------------------------------------------------------------------
__global__ void LB(256) k_face_center(Ctx C, const double* __restrict__ Bf, double* __restrict__ P,
                                      double* __restrict__ U) {
  int i, j, k;
  if (!interior_ijk(C, (long)blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
  const long c = cell_index(C, i, j, k);
  const double gd = C.geo_c[GE_GDET * C.npos + i + C.N[0] * j];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    const double* B = Bf + (long)q * C.Ntot;
    const double u = (C.n[q] > 1) ? 0.5 * (B[c] + B[c + C.st[q]]) : B[c];
    if (U) U[(5 + q) * C.Ntot + c] = u;
    if (P) P[(5 + q) * C.Ntot + c] = u / gd;
  }
}

// MC-limited values on the two sides of the point between a1 and a2
DEV void mc_pair(double a0, double a1, double a2, double a3, double& lo, double& hi) {
  lo = a1 + 0.5 * mc_slope(a1 - a0, a2 - a1);
  hi = a2 - 0.5 * mc_slope(a2 - a1, a3 - a2);
}

// ---------------------------------------------------------------------------
// Sec. 4.2 steps 8-9: the four-state corner EMF of edge e of cell c.
// VF [(2 d + side) 3 + m][Ntot]: v^(m+1) of face state side (0 left, 1
// right) on the lower d-face; SP [2 d + {0, 1}][Ntot]: that face's gas v_min,
// v_max.  HLL (eq. hll): weights v_max/(v_min+v_max) on the lower state and
// v_min/(v_min+v_max) on the upper, dissipation v_min v_max/(v_min+v_max);
// LAXF (eq. lax): 1/2, 1/2 and v_tot/2; one state on an inactive direction.
// ---------------------------------------------------------------------------
DEV double emf_stag_edge(const Ctx& C, int e, int j, long c, const double* __restrict__ Bf,
                         const double* __restrict__ VF, const double* __restrict__ SP) {
  const long N = C.Ntot;
  const int pd = (e + 1) % 3, qd = (e + 2) % 3;
  const bool act_p = C.n[pd] > 1, act_q = C.n[qd] > 1;
  const long sp = C.st[pd], sq = C.st[qd];
  const double* Bp = Bf + (long)pd * N;
  const double* Bq = Bf + (long)qd * N;
  double bp[2], bq[2];
  if (act_q) mc_pair(Bp[c - 2 * sq], Bp[c - sq], Bp[c], Bp[c + sq], bp[0], bp[1]);
  else bp[0] = bp[1] = Bp[c];
  if (act_p) mc_pair(Bq[c - 2 * sp], Bq[c - sp], Bq[c], Bq[c + sp], bq[0], bq[1]);
  else bq[0] = bq[1] = Bq[c];
  // v[a][b][m]: a the side along p, b along q; m = 0 v^p, 1 v^q
  double v[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) v[a][b][0] = v[a][b][1] = 0.0;
  if (act_p) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int m = 0; m < 2; m++) {
        const double* V = VF + ((long)((2 * pd + a) * 3) + (m ? qd : pd)) * N;
        double s0, s1;
        if (act_q) mc_pair(V[c - 2 * sq], V[c - sq], V[c], V[c + sq], s0, s1);
        else s0 = s1 = V[c];
        v[a][0][m] += s0;
        v[a][1][m] += s1;
      }
  }
  if (act_q) {
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int m = 0; m < 2; m++) {
        const double* V = VF + ((long)((2 * qd + b) * 3) + (m ? qd : pd)) * N;
        double s0, s1;
        if (act_p) mc_pair(V[c - 2 * sp], V[c - sp], V[c], V[c + sp], s0, s1);
        else s0 = s1 = V[c];
        v[0][b][m] += s0;
        v[1][b][m] += s1;
      }
  }
  if (act_p && act_q) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++) {
        v[a][b][0] *= 0.5;
        v[a][b][1] *= 0.5;
      }
  }
  double wp[2], wq[2], dp = 0.0, dq = 0.0;
#pragma unroll
  for (int dir = 0; dir < 2; dir++) {
    const bool act = dir ? act_q : act_p;
    double* w = dir ? wq : wp;
    double& dd = dir ? dq : dp;
    if (!act) {
      w[0] = 1.0;
      w[1] = 0.0;
      continue;
    }
    const int fd = dir ? qd : pd;
    const long so = dir ? sp : sq;
    const bool other = dir ? act_p : act_q;
    const double* Smin = SP + (long)(2 * fd) * N;
    const double* Smax = SP + (long)(2 * fd + 1) * N;
    const double vmin = other ? 0.5 * (Smin[c - so] + Smin[c]) : Smin[c];
    const double vmax = other ? 0.5 * (Smax[c - so] + Smax[c]) : Smax[c];
    if (C.flux == GRRMHD_FLUX_HLL) {
      if (vmin + vmax > 0.0) {
        w[0] = vmax / (vmin + vmax);
        w[1] = vmin / (vmin + vmax);
        dd = vmin * vmax / (vmin + vmax);
      } else {
        w[0] = w[1] = 0.5;
      }
    } else {
      w[0] = w[1] = 0.5;
      dd = 0.5 * ::fmax(vmin, vmax);
    }
  }
  double phi = 0.0;
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const double wab = wp[a] * wq[b];
      if (wab == 0.0) continue;
      phi += wab * (bp[b] * v[a][b][1] - bq[a] * v[a][b][0]);
    }
  phi += -dq * (bp[1] - bp[0]) + dp * (bq[1] - bq[0]);
  if (C.metric == GRRMHD_KERR_SCHILD && (pd == 1 || qd == 1)) {
    // edges on the polar axis carry no EMF
    const bool lo = j == C.ng[1] && (C.bc_lo[1] == GRRMHD_BC_REFLECT || C.bc_lo[1] == GRRMHD_BC_POLAR);
    const bool hi = j == C.ng[1] + C.n[1] && (C.bc_hi[1] == GRRMHD_BC_REFLECT || C.bc_hi[1] == GRRMHD_BC_POLAR);
    if (lo || hi) phi = 0.0;
  }
  return phi;
}

// every orientation at position t of the union range R ([ng, ng+n] on each
// active axis)
DEV void emf_stag_at(const Ctx& C, const FaceRange& R, const double* __restrict__ Bf,
                     const double* __restrict__ VF, const double* __restrict__ SP,
                     double* __restrict__ emf, long t) {
  if (t >= R.total) return;
  const int i = R.lo[0] + t % R.cnt[0];
  const long t2 = t / R.cnt[0];
  const int j = R.lo[1] + t2 % R.cnt[1];
  const int k = R.lo[2] + t2 / R.cnt[1];
  const long c = cell_index(C, i, j, k);
  for (int e = 0; e < 3; e++) {
    if (C.n[(e + 1) % 3] == 1 && C.n[(e + 2) % 3] == 1) continue;
    emf[(long)e * C.Ntot + c] = emf_stag_edge(C, e, j, c, Bf, VF, SP);
  }
}

__global__ void LB(256) k_emf_stag(Ctx C, FaceRange R, const double* __restrict__ Bf,
                                   const double* __restrict__ VF, const double* __restrict__ SP,
                                   double* __restrict__ emf) {
  emf_stag_at(C, R, Bf, VF, SP, emf, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

// the same with the step's Courant reduction over interior cells (the grid
// covers both ranges)
__global__ void LB(256) k_emf_stag_dt(Ctx C, FaceRange R, const double* __restrict__ Bf,
                                      const double* __restrict__ VF,
                                      const double* __restrict__ SP, double* __restrict__ emf,
                                      const double* __restrict__ vchar,
                                      unsigned long long* dtmin) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  emf_stag_at(C, R, Bf, VF, SP, emf, t);
  block_min_atomic(cell_dt(C, vchar, t), dtmin + (blockIdx.x % GRRMHD_DT_SLOTS) * GRRMHD_DT_STRIDE);
}

// ---------------------------------------------------------------------------
// Sec. 4.2 step 10 for the faces: Bout^p = a Bn^p + b Bprev^p + c dt
// (-sum_{d != p} d_d F^d[B^p]), F^d[B^p] = +Phi_e (e = 3-p-d) when p = e+1
// mod 3, else -Phi_e, on the evolved faces ([ng, ng+n] along p, [ng, ng+n)
// across).  dt: *dt_dev, or courant x the Courant slots' minimum.  cc = 0
// (an IMEX stage without explicit fluxes): no EMF term and no EMF read.
// ---------------------------------------------------------------------------
__global__ void LB(256) k_face_update(Ctx C, FaceRange R, double a, double b, double cc,
                                      const double* __restrict__ dt_dev,
                                      const unsigned long long* __restrict__ dtmin,
                                      const double* Bn, const double* __restrict__ Bprev,
                                      const double* __restrict__ emf, double* Bout) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R.total) return;
  const int idx[3] = {R.lo[0] + (int)(t % R.cnt[0]), R.lo[1] + (int)((t / R.cnt[0]) % R.cnt[1]),
                      R.lo[2] + (int)(t / ((long)R.cnt[0] * R.cnt[1]))};
  const long f = cell_index(C, idx[0], idx[1], idx[2]);
  const double dt = dtmin ? C.courant * dt_slots_min(dtmin) : *dt_dev;
  for (int pd = 0; pd < 3; pd++) {
    bool in = true;
    for (int d = 0; d < 3; d++)
      if (d != pd && C.n[d] > 1 && idx[d] >= C.ng[d] + C.n[d]) in = false;
    if (!in) continue;
    double curl = 0.0;
    for (int d = 0; d < 3 && cc != 0.0; d++) {
      if (d == pd || C.n[d] == 1) continue;
      const int e = 3 - pd - d;
      const double s = ((e + 1) % 3 == pd) ? 1.0 : -1.0;
      const double* E = emf + (long)e * C.Ntot;
      curl += s * (E[f + C.st[d]] - E[f]) / C.dx[d];
    }
    const long o = (long)pd * C.Ntot + f;
    Bout[o] = a * Bn[o] + (b != 0.0 ? b * Bprev[o] : 0.0) - (cc != 0.0 ? cc * dt * curl : 0.0);
  }
}
