// Host build of the device solver headers: for every cell of a batch file
// that the first PMHD attempt does not accept (and is not extreme), the
// cascade's URAD lane machine (urad_before / eval_urad_jac / urad_after,
// then the choice against the first attempt's record) must give the same
// bits as implicit_cell resuming from that record.  Prints one line:
// "cascade <n> extreme <n> differing <n> trips <n>".
#define DEV __host__ __device__ inline
#include <hip/hip_runtime.h>
#include <cmath>
__host__ inline bool isfinite(double x) { return std::isfinite(x); }
#include "../../paper_1312_6127_amd/csrc/kernels.h"
#include <cstdio>
#include <cstring>
#include <vector>

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  long n;
  double prm[10];
  if (fread(&n, 8, 1, f) != 1 || fread(prm, 8, 10, f) != 10) return 2;
  std::vector<double> Ui(12 * n), Pg(12 * n), dt(n), ca(n), ce(n);
  size_t got = fread(Ui.data(), 8, 12 * n, f) + fread(Pg.data(), 8, 12 * n, f) +
               fread(dt.data(), 8, n, f) + fread(ca.data(), 8, n, f) + fread(ce.data(), 8, n, f);
  fclose(f);
  if (got != (size_t)(27 * n)) return 2;
  Phys ph;
  ph.gam = prm[0];
  ph.arad = prm[1];
  ph.gamma_max = prm[2];
  const double G = prm[2] * prm[2];
  ph.ymax = 16.0 * G * (G - 1.0) / ((4.0 * G - 1.0) * (4.0 * G - 1.0));
  Opts o;
  o.tol_pmhd = prm[3];
  o.tol_urad = prm[4];
  o.tol_accept = prm[5];
  o.tol_fail = prm[6];
  o.max_iter = (int)prm[7];
  o.roundoff = (int)prm[8];
  long ncas = 0, next = 0, diff = 0, trips = 0;
  for (long cc = 0; cc < n; cc++) {
    Metric m;
    flat_metric(m);
    double u[12], p[12];
    for (int q = 0; q < 12; q++) {
      u[q] = Ui[q * n + cc];
      p[q] = Pg[q * n + cc];
    }
    CellOut first;
    Best b;
    int it = 0, tr = 0;
    bool ext = false;
    if (implicit_fast(m, ph, o, u, p, dt[cc], ca[cc], ce[cc], first, b, it, ext, tr)) continue;
    ncas++;
    if (ext) {
      next++;
      continue;
    }
    double rd[13];
    int ri[3];
    RecBuf R;
    R.d = rd;
    R.i = ri;
    R.cap = 1;
    rec_store(R, 0, b, it);
    CellOut ref;
    implicit_cell(m, ph, o, u, p, dt[cc], ca[cc], ce[cc], ref, &R, 0);
    // the lane machine, one evaluation per trip
    Cell c;
    Prep pr;
    prepare(m, ph, u, p, dt[cc], ca[cc], ce[cc], c, pr);
    UradLane L;
    Best b0;
    int it0;
    rec_load(R, 0, b0, it0);
    const double* src = (b0.ok && b0.eT < 1e-4) ? b0.P : p;
    rad_cons4(m, src, L.p);
    for (int q = 0; q < 5; q++) L.Pn[q] = src[q];
    L.iters = it0;
    L.mode = UM_START;
    for (int guard = 0; guard < 1000; guard++) {
      bool ended = urad_before(c, o, L);
      if (!ended) {
        Eval ev;
        double Jn[4][4];
        eval_urad_jac(c, ph, L.p, L.Pn, ev, Jn);
        trips++;
        ended = urad_after(ev, Jn, L);
      }
      if (ended) break;
    }
    Best best;
    rec_load(R, 0, best, it0);
    int bm = -1;
    if (best.ok) bm = M_PMHD;
    else best.eT = INFINITY;
    if (L.best.ok && L.best.eT < best.eT) {
      best = L.best;
      bm = M_URAD;
    }
    CellOut lane;
    if (bm < 0) failed_out(u, p, pr.status, L.iters, lane);
    else finalize(c, ph, o, best, bm, pr.status, L.iters, u, lane);
    bool same = lane.status == ref.status && lane.iters == ref.iters &&
                std::memcmp(&lane.err, &ref.err, 8) == 0;
    for (int q = 0; q < 12; q++)
      same = same && std::memcmp(&lane.P[q], &ref.P[q], 8) == 0 &&
             std::memcmp(&lane.U[q], &ref.U[q], 8) == 0;
    if (!same) diff++;
  }
  printf("cascade %ld extreme %ld differing %ld trips %ld\n", ncas, next, diff, trips);
  return 0;
}
