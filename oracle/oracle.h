/*
 * FP64 CPU oracle for one GRRMHD time step (HARMRAD method, McKinney,
 * Tchekhovskoy, Sadowski & Narayan 2014).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU path is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline timing may load it; the product path never does.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Conventions (all quantities in code units c = G = M = 1):
 *   primitives P[12]: 0 rho0, 1 u_g, 2-4 u~^i (gas velocity relative to the
 *     normal observer, coordinate components), 5-7 B^i, 8 Ebar (radiation
 *     rest-frame energy density), 9-11 u~^i_rad            (Sec. 4, list of P_q)
 *   conserved U[12] = sqrt(-g) * { rho0 u^t, T^t_t + rho0 u^t, T^t_i, B^i,
 *     R^t_t, R^t_i }                                        (Sec. 4, list of U_q)
 *   grid arrays are structure-of-arrays [q][k][j][i], i fastest, ghosts
 *   included; ghosts only along dimensions with more than one cell.
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H

#include <stdint.h>

#define ORC_NPRIM 12

enum { ORC_MINKOWSKI = 0, ORC_KERR_SCHILD = 1 };
enum { ORC_BC_OUTFLOW = 0, ORC_BC_PERIODIC = 1, ORC_BC_REFLECT = 2, ORC_BC_POLAR = 3 };
enum { ORC_FLUX_LLF = 0, ORC_FLUX_HLL = 1 };
/* time integrators (Sec. 4.1): RK3 with equal explicit and implicit
 * coefficients, and the IMEX2, IMEX2B and IMEX3 schemes */
enum { ORC_RK3 = 0, ORC_IMEX2 = 1, ORC_IMEX2B = 2, ORC_IMEX3 = 3 };
/* reconstruction (Sec. 4.3): MC-limited linear (ghost width 2) or PPM with
 * MC slopes and the gas/radiation shock flattener (ghost width 4) */
enum { ORC_RECON_MC = 0, ORC_RECON_PPM = 1 };

/* per-cell status bits of the implicit solve and fix-ups */
enum {
  ORC_ST_PMHD = 1 << 0,        /* accepted solution came from PMHD iteration */
  ORC_ST_URAD = 1 << 1,        /* accepted solution came from URAD iteration */
  ORC_ST_TYPE2_NEG = 1 << 2,   /* TYPE2 limiter met negative radiation energy */
  ORC_ST_BASIC = 1 << 3,       /* radiation re-inverted with BASIC limiter   */
  ORC_ST_C2P_FAIL = 1 << 4,    /* thin-limit MHD inversion had no solution   */
  ORC_ST_FLOOR = 1 << 5,       /* a floor changed the primitives             */
  ORC_ST_NOT_ACCEPT = 1 << 6,  /* best e_T above the acceptance tolerance    */
  ORC_ST_FAIL = 1 << 7,        /* no solution: primitives neighbour-averaged */
  ORC_ST_NO_GOOD_NB = 1 << 8,  /* averaging found no good neighbour          */
  ORC_ST_EXTREME = 1 << 9,     /* radiation extremely sub-dominant: URAD first */
  ORC_ST_COLD = 1 << 10,       /* solution of the cold MHD limit (u_g held)   */
  ORC_ST_PRAD = 1 << 11,       /* solution from iterating the radiation prims */
  ORC_ST_ENTROPY = 1 << 12,    /* entropy equation in place of the energy one */
  ORC_ST_STAGED = 1 << 13      /* solution from the staged Newton approach    */
};

typedef struct {
  int n[3];               /* interior cells per dimension (1 = inactive)      */
  int ng;                 /* ghost width along active dimensions              */
  int metric;             /* ORC_MINKOWSKI or ORC_KERR_SCHILD                 */
  double a;               /* black-hole spin (Kerr-Schild)                    */
  double R0;              /* radial map r = R0 + exp(x1)                      */
  double xlo[3], xhi[3];  /* internal-coordinate extent of the interior       */
  int bc_lo[3], bc_hi[3];
  double gam;             /* adiabatic index                                  */
  double arad;            /* radiation constant                               */
  double gamma_max;       /* radiation Lorentz-factor cap                     */
  double courant;
  int flux;               /* ORC_FLUX_LLF or ORC_FLUX_HLL                     */
  double tol_pmhd, tol_urad, tol_accept, tol_fail;
  int max_iter;           /* Newton steps per method                          */
  int roundoff;           /* keep iterating past tolerance to round-off       */
  double rho_floor, u_floor, bsq_rho_max, bsq_u_max, u_rho_max, erad_floor;
  int scheme;             /* ORC_RK3, ORC_IMEX2, ORC_IMEX2B, ORC_IMEX3         */
  int recon;              /* ORC_RECON_MC or ORC_RECON_PPM                    */
  int cold;               /* 1: cells with no energy solution try cold MHD    */
  int cascade;            /* 0: PMHD, URAD (then cold); 1: the full cascade of
                             Sec. 4.10-4.11: PMHD, URAD, PRAD, the staged
                             approach in the extreme regime, the entropy-based
                             methods, then cold                               */
  int ct;                 /* 0: flux-CT on the cell-centred field; 1: the
                             staggered face field with four-state corner EMFs */
} orc_params;

/* ---- geometry (Sec. 2; metric of the Kerr-Schild form) ---- */
typedef struct {
  double gcov[4][4];
  double gcon[4][4];
  double gdet;            /* sqrt(-g) */
  double alpha;           /* lapse 1/sqrt(-g^tt) */
} orc_geom;

void orc_geom_point(const orc_params *p, double x1, double x2, orc_geom *g);
/* connection Gamma^l_{m n} at internal coordinates (x1, x2) */
void orc_connection(const orc_params *p, double x1, double x2, double conn[4][4][4]);

/* ---- pointwise physics, exported for tests ---- */
void orc_p2u(const orc_params *p, const orc_geom *g, const double *P, double *U);
void orc_flux(const orc_params *p, const orc_geom *g, const double *P, int dir, double *F);
void orc_source_geom(const orc_params *p, const orc_geom *g, const double conn[4][4][4],
                     const double *P, double *S);
void orc_four_force(const orc_params *p, const orc_geom *g, const double *P,
                    double kabs, double kes, double Gcov[4]);
void orc_fluid_frame_rad(const orc_geom *g, const double *P, double *Ehat, double Fhat[3],
                         double Phat[3][3]);
void orc_wavespeeds(const orc_params *p, const orc_geom *g, const double *P, int dir,
                    double kappa_tot_dx, double vgas[2], double vrad[2]);
int orc_mhd_invert(const orc_params *p, const orc_geom *g, const double *U, const double *Pguess,
                   double *P);
int orc_rad_invert(const orc_params *p, const orc_geom *g, const double *U, int limiter,
                   double *P);

/* ---- implicit 4-force solve for one cell (Sec. 4.7-4.11) ---- */
typedef struct {
  int status;
  int iters;
  double err;
} orc_implicit_info;

void orc_implicit_cell(const orc_params *p, const orc_geom *g, const double *Ui,
                       const double *Pguess, double dt, double chi_abs, double chi_es,
                       double *Pout, double *Uout, orc_implicit_info *info);
/* the same with the explicit entropy Si = sqrt(-g) [S u^t]_(i) of the cell
 * (NAN: no entropy-based methods); orc_implicit_cell takes that of Pguess */
void orc_implicit_cell_s(const orc_params *p, const orc_geom *g, const double *Ui, double Si,
                         const double *Pguess, double dt, double chi_abs, double chi_es,
                         double *Pout, double *Uout, orc_implicit_info *info);
/* one attempt of one method alone (tests): method 0 PMHD, 1 URAD, 2 PRAD,
 * staged form, entropy equation (Si = sqrt(-g) [S u^t]_(i)) */
void orc_implicit_attempt(const orc_params *p, const orc_geom *g, const double *Ui, double Si,
                          const double *Pguess, double dt, double chi_abs, double chi_es,
                          int method, int staged, int entropy, double *Pout, double *Uout,
                          orc_implicit_info *info);
/* entropy density S = rho0 ln(p^n / rho0^(n+1)), n = 1/(gam - 1) (Sec. 2,
 * below eq. S), of primitives P; NAN where rho0 or u_g is not positive */
double orc_entropy(const orc_params *p, const double *P);
/* the cold MHD solve alone, u_g held at u_c (for tests) */
void orc_implicit_cold(const orc_params *p, const orc_geom *g, const double *Ui,
                       const double *Pguess, double dt, double chi_abs, double chi_es, double u_c,
                       double *Pout, double *Uout, orc_implicit_info *info);

/* batch of independent Minkowski cells, arrays [12][n] */
void orc_implicit_batch(const orc_params *p, long n, const double *Ui, const double *Pg,
                        const double *dtc, const double *chi_abs, const double *chi_es,
                        double *Pout, double *Uout, int *iters, int *status);

/* ---- grid-level pieces of one Runge-Kutta sub-step (Sec. 4.2) ---- */
long orc_ncell_alloc(const orc_params *p);
void orc_bc(const orc_params *p, double *P);
void orc_prim_to_cons(const orc_params *p, const double *P, double *U);
void orc_fluxes(const orc_params *p, const double *P, const double *chi_abs, const double *chi_es,
                double *F /* [3][12][N] */, double *emf /* [3][N] */, double *vchar /* [3][N] */);
double orc_timestep(const orc_params *p, const double *vchar);
/* PPM flattener of every cell within one cell of the interior, per active
 * direction d, gas and radiation: fl[(2 d + kind) N + c]; with keep != 0 the
 * larger of the new value and the one in fl (earlier sub-steps of the step) */
void orc_flattener(const orc_params *p, const double *P, const double *chi_abs,
                   const double *chi_es, double *fl, int keep);
/* orc_fluxes_fl plus, when Fs is not NULL, the face fluxes Fs [3][N] of the
 * entropy tracer sqrt(-g) S u^t (HLL/LAXF with the gas speeds) */
void orc_fluxes_s(const orc_params *p, const double *P, const double *chi_abs,
                  const double *chi_es, const double *fl, double *F, double *emf, double *vchar,
                  double *Fs);
/* orc_fluxes with the flattener state fl of the step (PPM; unused for MC) */
void orc_fluxes_fl(const orc_params *p, const double *P, const double *chi_abs,
                   const double *chi_es, const double *fl, double *F, double *emf, double *vchar);
/* MC-limited values on both sides of the face between a4[1] and a4[2] */
void orc_mc_face(const double a4[4], double *PL, double *PR);
/* PPM left and right values of the middle cell of a5[5] with flattener f */
void orc_ppm_cell(const double a5[5], double f, double *aL, double *aR);
void orc_explicit_update(const orc_params *p, double a, double b, double c, double dt,
                         const double *P, const double *Un, const double *Uprev, const double *F,
                         const double *emf, double *Uexp);
void orc_con2prim(const orc_params *p, const double *U, const double *Pguess, double *P, int *status);
void orc_implicit_grid(const orc_params *p, const double *Uexp, const double *Pguess, double dt,
                       const double *chi_abs, const double *chi_es, double *Pout, double *Uout,
                       int *iters, int *status);
/* the same with the explicit entropy Sexp [N] (sqrt(-g) [S u^t]_(i); NULL:
 * that of Pguess) */
void orc_implicit_grid_s(const orc_params *p, const double *Uexp, const double *Sexp,
                         const double *Pguess, double dt, const double *chi_abs,
                         const double *chi_es, double *Pout, double *Uout, int *iters,
                         int *status);
void orc_fixup(const orc_params *p, double *P, double *U, int *status);

/* ---- staggered face-centred field (stag.c; layout there) ---- */
void orc_bc_face(const orc_params *p, double *Bf);
void orc_face_to_center(const orc_params *p, const double *Bf, double *P, double *U);
void orc_emf_stag(const orc_params *p, const double *Bf, const double *VF, const double *SP,
                  double *emf);
void orc_face_update(const orc_params *p, double a, double b, double c, double dt,
                     const double *Bn, const double *Bprev, const double *emf, double *Bout);
/* fluxes and four-state corner EMFs of primitives P with face field Bf */
void orc_fluxes_stag(const orc_params *p, const double *P, const double *Bf,
                     const double *chi_abs, const double *chi_es, const double *fl, double *F,
                     double *emf, double *vchar, double *Fs);
int orc_step_stag(const orc_params *p, double *P, double *U, double *Bf, const double *chi_abs,
                  const double *chi_es, double *dt, int dt_fixed, int *status, int *iters);
/* one full step of the scheme p->scheme; dt in/out (computed from P^n
 * unless dt_fixed) */
int orc_step(const orc_params *p, double *P, double *U, const double *chi_abs, const double *chi_es,
             double *dt, int dt_fixed, int *status, int *iters);

#endif
