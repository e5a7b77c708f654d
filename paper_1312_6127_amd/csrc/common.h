// Internal definitions shared by the HIP kernels and the host side of the
// library: the kernel context passed by value to every launch, geometry
// table layout, and index helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/grrmhd.h"
#include "dual.h"

#ifndef DEV
#define DEV __device__ __forceinline__
#endif

// Geometry tables: 2-D (x1, x2) arrays broadcast over x3, because both
// metrics are independent of x3 (phi).  Field-major [field][j][i].
// Symmetric 4x4 tensors store the 10 components (00,01,02,03,11,12,13,22,23,33).
enum {
  GE_GCOV = 0,     // 10
  GE_GCON = 10,    // 10
  GE_GDET = 20,
  GE_ALPHA = 21,
  GE_NFACE = 22,   // fields stored at faces
  GE_DG1 = 22,     // d g_{mn}/dx1, 10 (cell centres only)
  GE_DG2 = 32,     // d g_{mn}/dx2, 10
  GE_NCENTER = 42
};

DEV constexpr int sym(int a, int b) {
  return (a <= b) ? (a == 0 ? b : (a == 1 ? 3 + b : (a == 2 ? 5 + b : 9)))
                  : (b == 0 ? a : (b == 1 ? 3 + a : (b == 2 ? 5 + a : 9)));
}

struct Ctx {
  int n[3], ng[3], N[3];
  long Ntot;
  long st[3];          // strides of i, j, k
  int npos;            // N1 * N2 (geometry table stride)
  double dx[3], xlo[3];
  int metric;
  int bc_lo[3], bc_hi[3];
  double gam, arad, gamma_max, ymax, courant;
  int flux;
  int recon;           // GRRMHD_RECON_MC or GRRMHD_RECON_PPM
  int cold;            // cold MHD limit for cells with no energy solution
  int cascade;         // 1: the full method cascade (PRAD, staged, entropy)
  int ct;              // 0: flux-CT on the cell-centred field; 1: staggered face field
  int mixed_i;         // FP32-mixed: cells with x1 index >= mixed_i take the FP32 face path
  double tol_pmhd, tol_urad, tol_accept, tol_fail;
  int max_iter, roundoff;
  double rho_floor, u_floor, bsq_rho_max, bsq_u_max, u_rho_max, erad_floor;
  const double* geo_c;   // [GE_NCENTER][npos]
  const double* geo_f1;  // [GE_NFACE][npos] at x1 faces
  const double* geo_f2;  // [GE_NFACE][npos] at x2 faces
};

// Real type of the literals and metric coefficients that go with a scalar
// T: float on the FP32 face path, double otherwise (double and Dual<N>).
template <class T>
struct RealOf {
  using type = double;
};
template <>
struct RealOf<float> {
  using type = float;
};

// Metric at one point, loaded from a table (rounded to R on the FP32 path).
template <class R>
struct MetricT {
  R gcov[10], gcon[10], gdet, alpha;
  DEV R lo(int a, int b) const { return gcov[sym(a, b)]; }
  DEV R up(int a, int b) const { return gcon[sym(a, b)]; }
};
using Metric = MetricT<double>;

template <class R>
DEV void load_metric(const double* tab, int npos, int pos, MetricT<R>& m) {
#pragma unroll
  for (int q = 0; q < 10; q++) m.gcov[q] = (R)tab[(GE_GCOV + q) * npos + pos];
#pragma unroll
  for (int q = 0; q < 10; q++) m.gcon[q] = (R)tab[(GE_GCON + q) * npos + pos];
  m.gdet = (R)tab[GE_GDET * npos + pos];
  m.alpha = (R)tab[GE_ALPHA * npos + pos];
}

DEV void flat_metric(Metric& m) {
#pragma unroll
  for (int q = 0; q < 10; q++) m.gcov[q] = m.gcon[q] = 0.0;
  m.gcov[0] = m.gcon[0] = -1.0;
  m.gcov[4] = m.gcon[4] = 1.0;
  m.gcov[7] = m.gcon[7] = 1.0;
  m.gcov[9] = m.gcon[9] = 1.0;
  m.gdet = 1.0;
  m.alpha = 1.0;
}
