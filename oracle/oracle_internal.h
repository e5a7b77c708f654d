/* Oracle-internal types shared by its own translation units (test
 * infrastructure only). */
#ifndef ORC_INTERNAL_H
#define ORC_INTERNAL_H
#include "oracle.h"

typedef struct {
  double rho, u, pg, bsq, gamma;
  double ucon[4], ucov[4], bcon[4], bcov[4];
  double T[4][4];        /* T^mu_nu */
  double one_plus_ut;    /* 1 + u_t */
} orc_gas;

typedef struct {
  double E, gamma;
  double ucon[4], ucov[4];
  double R[4][4];        /* R^mu_nu */
} orc_rad;

double orc_ucon(const orc_geom *g, const double ut[3], double ucon[4]);
void orc_lower(const orc_geom *g, const double vcon[4], double vcov[4]);
void orc_bcon(const orc_geom *g, const double B[3], const double ucon[4], const double ucov[4],
              double bcon[4]);
void orc_gas_state(const orc_params *p, const orc_geom *g, const double *P, orc_gas *s);
double orc_gas_energy_flux(const orc_gas *s, int mu);
void orc_rad_state(const orc_geom *g, const double *P, orc_rad *r);
/* spatial metric of the normal observer, gamma^{ij} = g^{ij} - g^{ti} g^{tj}/g^{tt} */
void orc_spatial_gcon(const orc_geom *g, double gam_ij[3][3]);

/* cell-centre geometry at allocated index (i, j, k) and face geometry */
void orc_cell_x(const orc_params *p, int i, int j, double *x1, double *x2);
void orc_face_x(const orc_params *p, int dir, int i, int j, double *x1, double *x2);
int orc_ng(const orc_params *p, int d);
int orc_nalloc(const orc_params *p, int d);
double orc_dx(const orc_params *p, int d);

#endif
