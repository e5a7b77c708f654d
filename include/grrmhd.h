/*
 * grrmhd.h -- C ABI of the MI355X (gfx950) GRRMHD time-step library.
 *
 * The library advances the general-relativistic radiation MHD equations of
 * the HARMRAD method (McKinney, Tchekhovskoy, Sadowski & Narayan 2014) by one
 * time step on a fixed Minkowski or Kerr-Schild grid: ghost fill, MC-limited
 * reconstruction, HLL/LAXF fluxes with separate gas and M1-radiation wave
 * speeds, flux-CT magnetic EMFs, the third-order Runge-Kutta update with the
 * radiation 4-force treated implicitly per cell, and the conserved-to-
 * primitive inversions (Sec. 4, 4.1-4.11 of the paper).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: c = G = M = 1; gas temperature T = p/rho0 (Sec. 4, code units).
 * Primitives P, 12 per cell (Sec. 4 list of P_q, 13th slot not carried):
 *   0 rho0, 1 u_g, 2-4 u~^i (gas 4-velocity relative to the normal observer,
 *   coordinate components), 5-7 B^i, 8 Ebar (radiation rest-frame energy
 *   density), 9-11 u~^i_rad.
 * Conserved U, 12 per cell (Sec. 4 list of U_q):
 *   sqrt(-g) * { rho0 u^t, T^t_t + rho0 u^t, T^t_i, B^i, R^t_t, R^t_i }.
 * Layout: structure of arrays, field-major [q][k][j][i] with i fastest, over
 *   the ALLOCATED grid, which adds ng ghost cells on both sides of every
 *   dimension that has more than one interior cell.  N = grrmhd_ncell_alloc().
 * Pointers: every array argument is DEVICE memory (hipMalloc or a PyTorch
 *   CUDA/HIP tensor), 8-byte aligned, not aliased with another argument
 *   unless stated.  The caller owns all state, opacity, status and workspace
 *   buffers; the library owns the grid's geometry tables.
 * Opacities: per-mass coefficients chi_abs, chi_es per allocated cell
 *   (ghosts included); the local opacity is kappa = chi * rho0.
 * Streams: all work is enqueued on the grid's HIP stream (set at init or by
 *   grrmhd_set_stream) and is asynchronous; no entry point synchronises
 *   except grrmhd_init_grid and grrmhd_free_grid.
 * Errors: functions return 0 on success and a negative GRRMHD_E* code on
 *   failure, with a message from grrmhd_last_error().  No C++ exception
 *   crosses the ABI.  Launch errors are checked; errors raised later by a
 *   kernel surface at the next synchronisation.
 */
#ifndef GRRMHD_H
#define GRRMHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRRMHD_NPRIM 12

enum { GRRMHD_MINKOWSKI = 0, GRRMHD_KERR_SCHILD = 1 };
enum { GRRMHD_BC_OUTFLOW = 0, GRRMHD_BC_PERIODIC = 1, GRRMHD_BC_REFLECT = 2, GRRMHD_BC_POLAR = 3 };
enum { GRRMHD_FLUX_LLF = 0, GRRMHD_FLUX_HLL = 1 };
enum { GRRMHD_FP64 = 0, GRRMHD_MIXED = 1 };
enum { GRRMHD_RK3 = 0, GRRMHD_IMEX2 = 1, GRRMHD_IMEX2B = 2, GRRMHD_IMEX3 = 3 };
enum { GRRMHD_RECON_MC = 0, GRRMHD_RECON_PPM = 1 };
enum { GRRMHD_CT_FLUX = 0, GRRMHD_CT_STAGGERED = 1 };
enum { GRRMHD_EINVAL = -1, GRRMHD_EHIP = -2, GRRMHD_ENOMEM = -3 };

/* per-cell status bits written by the implicit solve and the fix-ups */
enum {
  GRRMHD_ST_PMHD = 1 << 0,       /* solution from iterating gas primitives      */
  GRRMHD_ST_URAD = 1 << 1,       /* solution from iterating R^t_nu              */
  GRRMHD_ST_TYPE2_NEG = 1 << 2,  /* TYPE2 radiation limiter met E_rad <= 0       */
  GRRMHD_ST_BASIC = 1 << 3,      /* radiation re-inverted with the BASIC limiter */
  GRRMHD_ST_C2P_FAIL = 1 << 4,   /* MHD inversion of the explicit state failed   */
  GRRMHD_ST_FLOOR = 1 << 5,      /* a floor modified the primitives              */
  GRRMHD_ST_NOT_ACCEPT = 1 << 6, /* best error above tol_accept, below tol_fail  */
  GRRMHD_ST_FAIL = 1 << 7,       /* no solution: neighbour-averaged primitives   */
  GRRMHD_ST_NO_GOOD_NB = 1 << 8, /* averaging found no good neighbour            */
  GRRMHD_ST_EXTREME = 1 << 9,    /* radiation extremely sub-dominant: URAD first */
  GRRMHD_ST_COLD = 1 << 10,      /* no energy solution: cold MHD limit (u_g at the
                                    floor, gas momentum equations solved)       */
  GRRMHD_ST_PRAD = 1 << 11,      /* solution from iterating radiation primitives */
  GRRMHD_ST_ENTROPY = 1 << 12,   /* entropy equation in place of the energy one  */
  GRRMHD_ST_STAGED = 1 << 13     /* solution of the staged Newton approach       */
};

/* Numerical parameters.  Defaults (grrmhd_default_params) are the paper's
 * fixed test parameters (Sec. 5 introduction; Sec. 4.10-4.11) except
 * `roundoff`, which defaults to 1 (a departure from the paper's stopping
 * rule, for element-wise comparisons: see the field); roundoff = 0 gives the
 * paper's rule. */
typedef struct {
  int n[3];             /* interior cells per dimension (1 = inactive)        */
  int ng;               /* ghost width on active dimensions: 2 for MC, 4 for
                           PPM                                                */
  int metric;           /* GRRMHD_MINKOWSKI or GRRMHD_KERR_SCHILD             */
  double a;             /* black-hole spin (Kerr-Schild)                      */
  double R0;            /* radial map r = R0 + exp(x1)                        */
  double xlo[3], xhi[3];/* interior extent in internal coordinates; Kerr-
                           Schild: x1 = ln(r - R0), x2 = theta/pi,
                           x3 = phi/(2 pi)                                    */
  int bc_lo[3], bc_hi[3];
  double gam;           /* adiabatic index                                    */
  double arad;          /* radiation constant                                 */
  double gamma_max;     /* cap on the radiation frame's Lorentz factor        */
  double courant;
  int flux;             /* GRRMHD_FLUX_LLF or GRRMHD_FLUX_HLL                 */
  int precision;        /* GRRMHD_FP64, or GRRMHD_MIXED: reconstruction, face
                           states, Riemann fluxes and corner EMFs in FP32
                           arithmetic (state, update, inversions and the
                           implicit solve stay FP64)                          */
  double r_fp64;        /* MIXED on Kerr-Schild: faces and edges next to cells
                           with r < r_fp64 keep FP64 (default 2, which covers
                           the horizon and the ergosphere)                    */
  double tol_pmhd;      /* stop tolerance of PMHD iterations (1e-12)          */
  double tol_urad;      /* stop tolerance of URAD iterations (1e-9)           */
  double tol_accept;    /* accepted without trying the next method (1e-9)     */
  double tol_fail;      /* above this: no solution (1e-7)                     */
  int max_iter;         /* Newton steps per method (20)                       */
  int roundoff;         /* 1: after meeting the tolerance keep stepping (at
                           most 3 steps) until the step is at round-off, and
                           try the next method unless the best error is
                           within 10 tol_pmhd (instead of tol_accept)        */
  double rho_floor, u_floor, bsq_rho_max, bsq_u_max, u_rho_max, erad_floor;
  int scheme;           /* time integrator of grrmhd_step (Sec. 4.1):
                           GRRMHD_RK3 (default; RK3 with the same stages and
                           coefficients for the implicit part), or the IMEX
                           schemes GRRMHD_IMEX2, GRRMHD_IMEX2B, GRRMHD_IMEX3
                           (eq. IMEX2, IMEX2B, IMEX3)                        */
  int recon;            /* reconstruction (Sec. 4.3): GRRMHD_RECON_MC (default;
                           MC-limited linear, ng = 2) or GRRMHD_RECON_PPM
                           (PPM with MC slopes, no contact steepening, the
                           gas and radiation shock flatteners blended by the
                           optical depth, each the largest over the step's
                           sub-steps; ng = 4).  The adjoint covers both.      */
  int cold;             /* 1 (default): a cell whose implicit solve finds no
                           energy solution takes the cold MHD limit (Sec.
                           4.7): u_g held at u_floor, the three gas momentum
                           equations solved for the gas velocity (PMHD
                           residual, energy residuals left out of e_T), the
                           radiation from total energy-momentum conservation;
                           on success GRRMHD_ST_COLD replaces GRRMHD_ST_FAIL.
                           0: such cells fail (and are neighbour-averaged in
                           grrmhd_step).                                     */
  int cascade;          /* implicit solve's method cascade (Sec. 4.10-4.11):
                           0 (default): PMHD, URAD, then the cold limit;
                           1: the paper's full cascade: PMHD, URAD and PRAD
                           (radiation primitives iterated), their staged
                           forms (a damped momentum step, energy-only steps,
                           then the 4-D solve) for cells still without an
                           acceptable solution, the same with the entropy
                           equation in place of the gas energy equation, then
                           the cold limit (GRRMHD_ST_PRAD, GRRMHD_ST_ENTROPY,
                           GRRMHD_ST_STAGED mark the solutions).  The step's
                           entropy equation needs the entropy tracer's
                           explicit state, which grrmhd_step forms for every
                           scheme (the IMEX tables with the tracer's stored
                           sources); the batched solve takes each cell's from
                           its guess primitives.                             */
  int ct;               /* constrained transport of the field (Sec. 4, Sec.
                           4.2 steps 8-11): GRRMHD_CT_FLUX (default): flux-CT
                           on the cell-centred field, stepped by grrmhd_step;
                           GRRMHD_CT_STAGGERED: the face-centred field with
                           four-state corner EMFs (Del Zanna et al. 2007),
                           stepped by grrmhd_step_staggered (every scheme;
                           the adjoint is not available).                   */
} grrmhd_params;

typedef struct grrmhd_grid grrmhd_grid;

void grrmhd_default_params(grrmhd_params *p);
const char *grrmhd_last_error(void);

/* Geometry of the grid (metric, inverse, sqrt(-g), lapse at cell centres and
 * faces, metric derivatives at centres; Sec. 2) is computed on the device by
 * a kernel and kept by the library.  `device` is the HIP device ordinal,
 * `hip_stream` a hipStream_t (NULL = default stream).  Synchronous.
 * Errors: EINVAL for an invalid shape or parameter, ENOMEM, EHIP. */
int grrmhd_init_grid(const grrmhd_params *p, int device, void *hip_stream, grrmhd_grid **out);
int grrmhd_free_grid(grrmhd_grid *g);
int grrmhd_set_stream(grrmhd_grid *g, void *hip_stream);
long grrmhd_ncell_alloc(const grrmhd_grid *g);
/* bytes of caller-provided workspace needed by grrmhd_step */
size_t grrmhd_workspace_bytes(const grrmhd_grid *g);

/* U = U(P) at every allocated cell (Sec. 4: U_q in closed form of P_q).
 * P [12][N] in, U [12][N] out. */
int grrmhd_prim_to_cons(grrmhd_grid *g, const double *P, double *U);

/* Sub-step 1 of Sec. 4.2: fill the ghost cells of P [12][N] in place from
 * the interior, dimension by dimension (x1, x2, x3) so corners are filled.
 * OUTFLOW copies the edge cell, PERIODIC wraps, REFLECT mirrors and negates
 * the normal vector components, POLAR (x2 in 3-D) maps across the axis to
 * phi + pi and negates the theta components. */
int grrmhd_apply_bc(grrmhd_grid *g, double *P);

/* Sub-steps 4-9 of Sec. 4.2 on a P whose ghosts are filled: MC-limited or
 * PPM reconstruction (params.recon; PPM with the flattener of this P alone),
 * face U and F, gas fast-magnetosonic and M1 radiation wave
 * speeds (radiation limited by 4/(3 tau), eq. wavespeedlimit), HLL (eq. hll)
 * or LAXF (eq. lax) fluxes, then flux-CT corner EMFs.
 * F [3][12][N]: direction d face flux at index c = face between c - e_d and
 *   c; the induction fluxes of the normal component are zero.
 * emf [3][N]: EMF along a at the edge with the two other indices at -1/2.
 * vchar [3][N]: largest characteristic speed magnitude at each face.
 * Values outside the computed face ranges are zero. */
int grrmhd_fluxes(grrmhd_grid *g, const double *P, const double *chi_abs, const double *chi_es,
                  double *F, double *emf, double *vchar);

/* Courant step (Sec. 4.4, last paragraph): dt = C min over interior cells of
 * 1/sum_d(v_d/dx^d), v_d the larger face speed of the cell.  Writes one
 * double to dt_dev (device). */
int grrmhd_timestep(grrmhd_grid *g, const double *vchar, double *dt_dev);

/* Sub-step 10: U_exp = a U^n + b U_prev + c dt (-div F + S_M(P)) at interior
 * cells, with flux-CT face fluxes for B rebuilt from the corner EMFs and the
 * geometric source S_M = sqrt(-g) T^k_l Gamma^l_{nu k} (Sec. 4 list of S_M),
 * evaluated as (1/2) sqrt(-g) T^{k m} d_nu g_{k m}.
 * dt_dev is a device scalar.  Uprev is not read when b == 0. */
int grrmhd_explicit_update(grrmhd_grid *g, double a, double b, double c, const double *dt_dev,
                           const double *P, const double *Un, const double *Uprev,
                           const double *F, const double *emf, double *Uexp);

/* Conserved-to-primitive inversion at interior cells (Sec. 4.5 MHD 1-D W'
 * equation; Sec. 4.6 analytic M1 with the BASIC limiter).  Pguess [12][N]
 * starts the MHD iteration; P [12][N] out (may alias Pguess); status [N]
 * gets GRRMHD_ST_C2P_FAIL where the MHD inversion has no physical root. */
int grrmhd_con2prim(grrmhd_grid *g, const double *U, const double *Pguess, double *P, int *status);

/* Sub-steps 11-12: implicit radiation 4-force solve at interior cells with
 * time step dt_scale * (*dt_dev) (eq. source3/source4; PMHD then URAD,
 * Sec. 4.7-4.11; then, where neither has a solution, the cold MHD limit of
 * Sec. 4.7 when params.cold is set).  Uexp [12][N] explicit conserved state; Pguess [12][N]
 * previous primitives (may alias P).  Out: P, U [12][N] (U may not alias
 * Uexp), iters/status/err [N] (each may be NULL): Newton steps, status
 * bits, final total normalised error e_T. */
int grrmhd_implicit_grid(grrmhd_grid *g, const double *Uexp, const double *Pguess,
                         double dt_scale, const double *dt_dev, const double *chi_abs,
                         const double *chi_es, double *P, double *U, int *iters, int *status,
                         double *err);

/* Sub-step 13 and floors (Sec. 4.11): cells whose status has
 * GRRMHD_ST_FAIL take the average primitives of their face neighbours with
 * a good energy solution (neither GRRMHD_ST_FAIL nor GRRMHD_ST_COLD; of all
 * interior face neighbours if none is good, then GRRMHD_ST_NO_GOOD_NB);
 * cells with GRRMHD_ST_COLD take the same average of u_g alone; then floors
 * on rho0, u_g (b^2/rho0, b^2/u_g, u_g/rho0 limits) and Ebar; U is
 * recomputed where P changed.  On a staggered-field grid a failed cell's B
 * is not averaged: it is its own conserved field over sqrt(-g) (the mean of
 * its faces).  `scratch` is device memory of at least 13 N doubles. */
int grrmhd_fixup(grrmhd_grid *g, double *P, double *U, int *status, double *scratch);

/* One full time step of the grid's scheme (Sec. 4.1).  GRRMHD_RK3:
 * third-order Shu-Osher stages with identical explicit and implicit
 * coefficients, stage k implicit in its own value with dt_k = c_k dt.
 * GRRMHD_IMEX2/IMEX2B/IMEX3 (eq. IMEX2, IMEX2B, IMEX3): each implicit stage
 * i solves U^i = [explicit bracket] + g_i dt M(U^i); the brackets combine
 * U^n, one earlier stage, the flux divergence and geometric source of the
 * previous stage and the stored 4-force sources M^k of earlier stages
 * (M^k = (U^k - bracket)/(g_k dt) from stage k's implicit solve, before its
 * fix-ups, zero where it failed); the final
 * combination is explicit and followed by the MHD and radiation (BASIC)
 * inversions, a cell whose MHD inversion fails being a failed cell.  P, U
 * [12][N] in/out: U^n must hold the conserved state of P^n at interior
 * cells; on return both hold the new state at interior cells (ghosts of P
 * are stale).  dt_dev: device scalar, read when dt_fixed != 0, otherwise
 * computed from the wave speeds of P^n and written.  status/iters [N]
 * (nullable): OR of status bits / sum of Newton steps over the stages.
 * workspace: device buffer of grrmhd_workspace_bytes() (which depends on
 * the scheme).  EINVAL on a staggered-field grid (grrmhd_step_staggered
 * steps those), for NULL arrays or a small or misaligned workspace. */
int grrmhd_step(grrmhd_grid *g, double *P, double *U, const double *chi_abs,
                const double *chi_es, double *dt_dev, int dt_fixed, int *status, int *iters,
                void *workspace, size_t ws_bytes);

/* ---- staggered face-centred field (params.ct = GRRMHD_CT_STAGGERED) ----
 * Bf [3][N] device array: sqrt(-g) B^(p+1) on the lower p-face of each cell
 * (the cell itself along an inactive dimension p); the evolved faces are
 * [ng, ng+n] along p ([ng, ng+n) when x_p is periodic) and the interior
 * range across it; the rest are ghost faces.  Edge e of a cell lies at its
 * lower corner in p = e+1 and q = e+2 (mod 3), and its EMF is
 * F^q[B^p] = sqrt(-g)(B^p v^q - B^q v^p) (Sec. 4 list of fluxes).  All
 * calls are asynchronous on the grid's stream; EINVAL on a flux-CT grid or
 * for NULL arrays. */

/* Ghost faces of Bf (Sec. 4.2 step 1): across a dimension the cell rule;
 * along the face's own direction outflow copies the boundary face, periodic
 * wraps, REFLECT and POLAR mirror about the boundary face with B^p negated
 * (POLAR: phi shifted by pi); the primitive B is carried (sqrt(-g) of the
 * ghost face applied). */
int grrmhd_apply_bc_faces(grrmhd_grid *g, double *Bf);

/* Sec. 4.2 step 8: at interior cells U[5+p] = the mean of sqrt(-g) B^p on
 * the cell's two p-faces and P[5+p] = U[5+p]/sqrt(-g) at the centre; other
 * entries untouched.  P or U may be NULL. */
int grrmhd_face_to_center(grrmhd_grid *g, const double *Bf, double *P, double *U);

/* Sub-steps 4-9 with the staggered field: the face fluxes F [3][12][N] and
 * speeds vchar [3][N] as grrmhd_fluxes with each face's own normal field in
 * both states (zero where sqrt(-g) vanishes), and the corner EMFs emf [3][N]
 * from the four-state HLL/LAXF solution (Del Zanna et al. 2007): sqrt(-g) B^p
 * interpolated along q and sqrt(-g) B^q along p from the faces, the face
 * velocity states of each active in-plane direction interpolated along the
 * other (MC slopes) and averaged, the gas speeds the mean of the two faces
 * adjacent to the edge (Sec. 4.4); zero on the polar axis.  P's ghost cells
 * and Bf's ghost faces must be filled.  workspace: as grrmhd_step's
 * (grrmhd_workspace_bytes(), 256-byte aligned). */
int grrmhd_fluxes_staggered(grrmhd_grid *g, const double *P, const double *Bf,
                            const double *chi_abs, const double *chi_es, double *F, double *emf,
                            double *vchar, void *workspace, size_t ws_bytes);

/* One step of the grid's scheme (as grrmhd_step: RK3, or the IMEX tables of
 * Sec. 4.1) with the staggered field: each stage's faces are a Bf^n +
 * b Bf^(j) + c dt (-circulation of the corner EMFs round the face) with the
 * stage's own coefficients (no EMF term in a stage without explicit fluxes;
 * the implicit part leaves the field alone), so the discrete divergence of
 * Bf never changes, and the stage's cell-centred conserved field is the mean
 * of the new faces; a failed cell's neighbour average keeps its own field.
 * Bf in/out (evolved faces; ghost faces are filled in place at the start).
 * P, U, dt, status, iters and workspace as grrmhd_step (the workspace holds
 * the faces of every stage but the last). */
int grrmhd_step_staggered(grrmhd_grid *g, double *P, double *U, double *Bf,
                          const double *chi_abs, const double *chi_es, double *dt_dev,
                          int dt_fixed, int *status, int *iters, void *workspace,
                          size_t ws_bytes);

/* Adjoint of one full step (grrmhd_step with dt_fixed): gP_n = dL/dP^n for
 * L = sum over interior cells and fields of gU_next * U^{n+1}(P^n), with
 * U^n = U(P^n) and dt (*dt_dev) held fixed.  The forward step is recomputed
 * with per-stage checkpoints; the implicit solve is differentiated by the
 * implicit-function theorem on the PMHD residual at the converged state
 * (Sec. 4.8; one transposed 4x4 solve per cell), the fluxes, EMFs, source
 * and ghost fill by their local Jacobians (dual numbers) and transposes.
 * The fix-ups are differentiated at the state before them: a failed cell's
 * neighbour average (its own failed solve receives nothing) and the floors
 * (a floored quantity passes no cotangent back, U recomputed from P passes
 * none to U before the fix-up), with the implicit solve's transpose taken
 * at its own output.  Every scheme
 * (RK3; eq. IMEX2, IMEX2B, IMEX3): on an IMEX grid the stored
 * sources M^k = (U(k) - U_e(k))/(g dt) are transposed with the stages that
 * read them, and the final explicit stage's inversion is differentiated at
 * its result (the MHD block by the implicit-function theorem, one
 * transposed 8x8 solve per cell; the radiation block through the limited
 * inversion itself; where the MHD inversion failed, its guess, the stage
 * input, takes the cotangent).  MC or PPM reconstruction (Sec. 4.3): with
 * PPM the face states' Jacobian covers the six-cell stencil and the shock
 * flattener of the two face cells, and the flattener itself (the largest
 * over the step's flux evaluations) is differentiated at the evaluation
 * that gave it, inside its ramp through the pressures, densities and
 * opacities of its seven cells.  The full cascade (cascade = 1), every
 * scheme: PRAD and staged solutions are roots of the same energy equations;
 * an entropy-method solution is differentiated on its entropy equation
 * (eq. source6), whose explicit tracer a U_S(P^n) + b U_S(P_in) + c dt
 * (-div F_S) (+ dt sum_k m_k M_S^k on an IMEX grid, the stored entropy
 * sources M_S^k = (U_S(P(k)) - S_e(k))/(g dt) taken at the stage's output
 * before its fix-ups) passes its cotangent on through the tracer's face
 * fluxes, U_S of the primitives and the earlier stages' M_S^k.  The flux-CT
 * field only.  EINVAL on a staggered-field grid (grrmhd_explicit_vjp also
 * rejects one, grrmhd_implicit_vjp a full-cascade grid).  The workspace
 * size depends on the scheme, the reconstruction and the cascade.  P_n [12][N] (interior read; not modified), gU_next
 * [12][N] (interior read), gP_n [12][N] out (ghosts zero); g_chi (nullable)
 * [2][N] out: dL/dchi_abs, dL/dchi_es at every allocated cell (the per-mass
 * opacities enter the implicit residual through kappa = chi rho0 and the
 * face fluxes through the radiation speed limiter of the two face cells,
 * ghost cells included); P_next, U_next (nullable) receive the forward
 * result.  workspace: device buffer of
 * grrmhd_adjoint_workspace_bytes() bytes, 256-byte aligned.  Errors: EINVAL,
 * EHIP. */
size_t grrmhd_adjoint_workspace_bytes(const grrmhd_grid *g);
int grrmhd_step_adjoint(grrmhd_grid *g, const double *P_n, const double *chi_abs,
                        const double *chi_es, const double *dt_dev, const double *gU_next,
                        double *gP_n, double *g_chi, double *P_next, double *U_next,
                        void *workspace, size_t ws_bytes);

/* grrmhd_step_adjoint in two halves, for callers that run the forward step
 * anyway (an autograd forward, then its backward): grrmhd_step_checkpointed
 * is its forward step (P_n -> P_next, U_next, both nullable; U_next's ghost
 * entries are U(P_n)'s), keeping the stage checkpoints in `workspace`;
 * grrmhd_step_adjoint_saved is its reverse sweep from those checkpoints,
 * with the same meaning of gU_next, gP_n and g_chi.  The checkpoints stay
 * valid until `workspace` is used for anything else; the reverse sweep must
 * be given the same grid, opacities and dt as the forward.  Workspace as for
 * grrmhd_step_adjoint.  Errors: EINVAL, EHIP. */
int grrmhd_step_checkpointed(grrmhd_grid *g, const double *P_n, const double *chi_abs,
                             const double *chi_es, const double *dt_dev, double *P_next,
                             double *U_next, void *workspace, size_t ws_bytes);
int grrmhd_step_adjoint_saved(grrmhd_grid *g, const double *chi_abs, const double *chi_es,
                              const double *dt_dev, const double *gU_next, double *gP_n,
                              double *g_chi, void *workspace, size_t ws_bytes);

/* Pieces of the adjoint sweep (each the transpose of the Jacobian of a
 * forward entry point; ghosts of inputs are ignored where the forward
 * ignores them):
 *  grrmhd_implicit_vjp   of grrmhd_implicit_grid at its result (P_out,
 *                        status): gUexp = (dP/dUexp)^T gP_out +
 *                        (dU/dUexp)^T gU_out at interior cells (zero at
 *                        ghosts); cold cells (GRRMHD_ST_COLD) through the
 *                        three momentum equations with u_g fixed (normal
 *                        cascade; EINVAL on a full-cascade grid);
 *  grrmhd_explicit_vjp   of grrmhd_fluxes followed by grrmhd_explicit_update
 *                        with stage coefficient c on dt, with respect to the
 *                        ghost-filled P: gP at every allocated cell (PPM:
 *                        the flattener is P's own, as at a step's first
 *                        flux evaluation; the call overwrites the grid's
 *                        flattener buffer); workspace
 *                        grrmhd_explicit_vjp_workspace_bytes();
 *  grrmhd_bc_vjp         of grrmhd_apply_bc, in place (ghost entries folded
 *                        into their source cells and cleared);
 *  grrmhd_fixup_vjp      of grrmhd_fixup (Sec. 4.11) at its result (P,
 *                        status): gP_pre, gU_pre [12][N] = the cotangents of
 *                        its input P and U for output cotangents gP, gU
 *                        (interior cells; zero at ghosts).  Failed cells'
 *                        neighbour averages and cold cells' u_g averages are
 *                        transposed, U = U(P) at changed cells by its local
 *                        Jacobian, floors as the identity (flux-CT grids;
 *                        EINVAL on a staggered-field grid).  scratch: [12][N]
 *                        doubles; no array may alias another;
 *  grrmhd_con2prim_vjp   of grrmhd_con2prim (Sec. 4.5, 4.6) at its result
 *                        (P, status): gU = (dP/dU)^T gP at interior cells
 *                        (zero at ghosts), the MHD block by the implicit-
 *                        function theorem on U(P) (an 8x8 transposed solve),
 *                        the radiation block through the BASIC inversion;
 *                        where GRRMHD_ST_C2P_FAIL is set the MHD result was
 *                        the guess, so gPguess (fields 0-4) gets gP's and
 *                        gU's MHD block only B's; gPguess is zero elsewhere.
 *                        gU, gPguess [12][N] out, overwritten. */
int grrmhd_implicit_vjp(grrmhd_grid *g, const double *Uexp, const double *P_out,
                        const int *status, double dt_scale, const double *dt_dev,
                        const double *chi_abs, const double *chi_es, const double *gP_out,
                        const double *gU_out, double *gUexp);
size_t grrmhd_explicit_vjp_workspace_bytes(const grrmhd_grid *g);
int grrmhd_explicit_vjp(grrmhd_grid *g, double c, const double *dt_dev, const double *P,
                        const double *chi_abs, const double *chi_es, const double *gUexp,
                        double *gP, void *workspace, size_t ws_bytes);
int grrmhd_bc_vjp(grrmhd_grid *g, double *gP);
int grrmhd_fixup_vjp(grrmhd_grid *g, const double *P, const int *status, const double *gP,
                     const double *gU, double *gP_pre, double *gU_pre, double *scratch);
int grrmhd_con2prim_vjp(grrmhd_grid *g, const double *U, const double *P, const int *status,
                        const double *gP, double *gU, double *gPguess);

/* Implicit 4-force solve for n independent cells in flat space (Minkowski
 * metric, no grid), eq. source3/source4 with the PMHD-then-URAD cascade of
 * Sec. 4.10, then the cold MHD limit (Sec. 4.7, params.cold) for cells left
 * without an energy solution.  Arrays [12][n] (U_expl, P_guess, P_out, U_out)
 * and [n] (dt_cell, chi_abs, chi_es, iters, status, err; the last three
 * nullable), device memory; n < 2^31.  workspace: device buffer of at least
 * grrmhd_implicit_source_workspace_bytes(n) bytes, 256-byte aligned (work
 * list of the cells that need the full cascade, with the result of their
 * first attempt; list of deferred extreme cells; list of cells for the cold
 * limit; lane statistics).  Same algorithm as grrmhd_implicit_grid.  The
 * cascade's URAD attempts run in a compacting persistent grid (lanes take
 * the next listed cell as soon as theirs ends); extreme cells (URAD first)
 * and then cold cells run one thread each afterwards. */
size_t grrmhd_implicit_source_workspace_bytes(long n);
int grrmhd_implicit_source(const grrmhd_params *p, long n, const double *U_expl,
                           const double *P_guess, const double *dt_cell, const double *chi_abs,
                           const double *chi_es, double *P_out, double *U_out, int *iters,
                           int *status, double *err, void *workspace, size_t ws_bytes,
                           void *hip_stream);

/* grrmhd_implicit_source without a workspace argument and without any
 * allocation, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * per-cell form's scratch memory (counters, lane statistics, cascade list
 * with first-attempt records, deferred-cell and cold-cell lists, 128 bytes
 * per cell) lives in a static device array sized for GRRMHD_NOALLOC_MAX_CELLS
 * cells (32 MiB); each device the library runs on holds its own copy until
 * the process ends.  Its address is looked up on the first call on each
 * device (the current HIP device, which must own hip_stream); no call
 * allocates, frees or calls an allocating library routine.  Arguments,
 * results and errors as grrmhd_implicit_source; EINVAL for n above
 * GRRMHD_NOALLOC_MAX_CELLS.  Every call on one device shares that device's
 * array, which keeps the last call's contents (the counters are cleared by a
 * kernel at the start of each call): calls stream-ordered on one device are
 * safe, calls that overlap on one device (other streams, other host threads)
 * race and must be serialised by the caller. */
#define GRRMHD_NOALLOC_MAX_CELLS 262144L
int grrmhd_implicit_source_noalloc(const grrmhd_params *p, long n, const double *U_expl,
                                   const double *P_guess, const double *dt_cell,
                                   const double *chi_abs, const double *chi_es, double *P_out,
                                   double *U_out, int *iters, int *status, double *err,
                                   void *hip_stream);

/* Batched implicit solve with an explicit execution form, for batches whose
 * Newton counts are very uneven between cells (optically thin against thick
 * cells, Sec. 4.10).  mode:
 *   GRRMHD_IMPLICIT_PER_CELL       one thread per cell (as grrmhd_implicit_source);
 *   GRRMHD_IMPLICIT_PER_ITERATION  one launch per Newton trip, lane state in
 *                                  HBM, still-active cells compacted into the
 *                                  next launch's queue;
 *   GRRMHD_IMPLICIT_PERSISTENT     a fixed grid of waves_per_cu waves per CU in
 *                                  blocks of `block` (64, 128, 256) threads;
 *                                  each lane takes the next cell from a queue
 *                                  whenever its cell converges.
 * All forms give identical results (same decisions per cell).  workspace:
 * grrmhd_implicit_source_workspace_bytes_ex(n, mode) bytes, 256-byte aligned;
 * EINVAL for a bad mode, block or waves_per_cu, a small or misaligned
 * workspace, or n > 2^30 in the persistent form. */
enum { GRRMHD_IMPLICIT_PER_CELL = 0, GRRMHD_IMPLICIT_PER_ITERATION = 1, GRRMHD_IMPLICIT_PERSISTENT = 2 };
size_t grrmhd_implicit_source_workspace_bytes_ex(long n, int mode);
int grrmhd_implicit_source_ex(const grrmhd_params *p, long n, const double *U_expl,
                              const double *P_guess, const double *dt_cell, const double *chi_abs,
                              const double *chi_es, double *P_out, double *U_out, int *iters,
                              int *status, double *err, int mode, int block, int waves_per_cu,
                              void *workspace, size_t ws_bytes, void *hip_stream);

/* Autotuner: times each of GRRMHD_TUNE_CANDIDATES candidates (per-cell
 * form; one launch per Newton trip; persistent form with block 64/128/256
 * and 4/8/16 waves per CU) on the caller's inputs with HIP events (each
 * candidate run twice, the second timed) and returns the fastest in *best;
 * `all` (nullable) receives up to n_all candidates with their times, in the
 * order tried.  Outputs hold the last candidate's (identical) results.
 * Synchronises the stream.  Workspace as for GRRMHD_IMPLICIT_PER_ITERATION. */
#define GRRMHD_TUNE_CANDIDATES 9
typedef struct {
  int mode, block, waves_per_cu;
  float ms;
} grrmhd_tuning;
int grrmhd_autotune_implicit_source(const grrmhd_params *p, long n, const double *U_expl,
                                    const double *P_guess, const double *dt_cell,
                                    const double *chi_abs, const double *chi_es, double *P_out,
                                    double *U_out, int *iters, int *status, double *err,
                                    void *workspace, size_t ws_bytes, void *hip_stream,
                                    grrmhd_tuning *best, grrmhd_tuning *all, int n_all);

/* Lane statistics of implicit solves: out[0] residual evaluations of the
 * first PMHD attempts (Newton trips over all cells), out[1] lane slots the
 * wavefronts spent on them (64 per wavefront trip), out[2] cells the last
 * launch sent to the rest of the cascade.  out[0]/out[1] is the active-lane
 * fraction.  A grid's out[0..1] accumulate over its implicit launches since
 * its creation or the last grrmhd_time_implicit(g, 1); a batch's cover the
 * last solve that used the workspace.  Synchronises the stream (the grid's,
 * or hip_stream). */
int grrmhd_implicit_stats(grrmhd_grid *g, unsigned long long out[3]);
int grrmhd_implicit_source_stats(const void *workspace, unsigned long long out[3],
                                 void *hip_stream);

/* Lane statistics of a batch's cascade (the URAD attempts of the cells the
 * first attempt did not accept, run by a compacting persistent grid): out[0]
 * residual evaluations, out[1] lane slots (64 per wavefront trip) of the last
 * solve that used the workspace.  Synchronises hip_stream.  EINVAL for a NULL
 * or misaligned workspace. */
int grrmhd_implicit_source_cascade_stats(const void *workspace, unsigned long long out[2],
                                         void *hip_stream);

/* HIP-event timing of the grid's implicit kernel (the first-attempt kernel
 * of every implicit launch, grrmhd_step's three included).  on != 0 clears
 * the record and the grid's lane statistics, then brackets the next
 * launches (up to 256) with events on the grid's stream; on == 0 stops.
 * grrmhd_implicit_time synchronises the stream and returns the summed
 * duration and the number of timed launches. */
int grrmhd_time_implicit(grrmhd_grid *g, int on);
int grrmhd_implicit_time(grrmhd_grid *g, double *total_ms, int *launches);

#ifdef __cplusplus
}
#endif
#endif
