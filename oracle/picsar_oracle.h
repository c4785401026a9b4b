/*
 * picsar_oracle.h -- plain FP64 CPU oracle of the 2.5D axisymmetric PIC step
 * of Belyaev, "PICsar: a 2.5D axisymmetric, relativistic, electromagnetic,
 * particle in cell code with a radiation absorbing boundary" (arXiv 1407.1810).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this library: it is used by the test suite, by the entry-point smoke
 * check and by the benchmark's CPU-baseline leg.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * Indexing (build convention): cells i = 0..nr-1 radially, j = 0..nth-1 in
 * the meridional direction; radial nodes i = 0..nr (conductors at 0 and nr),
 * meridional nodes j = 0..nth (poles at 0 and nth).  Staggering follows
 * eq. (offseteq) of Sec. 3.1.  All arrays are row-major [i][j] with j fastest.
 *
 *   comp  name   position      extent (rows x cols)
 *   0     E_r    (i+1/2, j)    nr      x (nth+1)
 *   1     E_th   (i, j+1/2)    (nr+1)  x nth
 *   2     E_ph   (i, j)        (nr+1)  x (nth+1)
 *   3     B_r    (i, j+1/2)    (nr+1)  x nth
 *   4     B_th   (i+1/2, j)    nr      x (nth+1)
 *   5     B_ph   (i+1/2, j+1/2) nr     x nth
 *   6     F_r    face charge at (i+1/2, j), rows i = -g .. nr+g-1
 *   7     F_th   face charge at (i, j+1/2), rows i = -g .. nr+g
 *   8     F_ph   ring charge at (i, j),     rows i = -g .. nr+g
 * with g = 2*n_filt + 3 ghost rows on each radial side of the F arrays.
 */
#ifndef PICSAR_ORACLE_H
#define PICSAR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_R_LOG = 0, ORA_R_LIN = 1 };
enum { ORA_TH_EQAREA = 0, ORA_TH_LIN = 1 };
enum { ORA_VAY = 0, ORA_BORIS = 1 };
enum { ORA_BG_NONE = 0, ORA_BG_UNIFORM_BZ = 1, ORA_BG_MONOPOLE = 2,
       ORA_BG_DIPOLE = 3, ORA_BG_DIPOLE_COROT = 4 };
enum { ORA_OK = 0, ORA_EINVAL = -1, ORA_ENOMEM = -2, ORA_ECFL = -3 };

typedef struct {
    int32_t nr, nth;        /* cells in r and theta */
    double r_in, r_out;     /* conductor radii (code length units) */
    int32_t r_kind;         /* ORA_R_LOG | ORA_R_LIN */
    int32_t th_kind;        /* ORA_TH_EQAREA | ORA_TH_LIN */
    double c;               /* speed of light in length units per step (dt = 1) */
    int32_t n_filt;         /* passes of the 1-2-1 current filter */
    int32_t absorb_cells;   /* width of the lossy layer in cells (0 = off) */
    double sigma_max;       /* sigma* at the outer conductor */
    int32_t mover;          /* ORA_VAY | ORA_BORIS */
    int32_t bg_kind;        /* analytic "initial" field, see enum */
    double B0;              /* field at r_in (monopole/dipole) or uniform B_z */
    double omega;           /* final angular velocity of the conductor */
    double t_spin;          /* spin-up time (0 = none) */
    double q_over_m;        /* |q/m| of every macro-particle (code units) */
    double f_inj;           /* injection fraction, eq. (volinjeq) */
    double q_inj;           /* |charge| of an injected macro-particle */
    int32_t inject;         /* 1 = surface injection on */
    uint64_t seed;          /* key of the injection random stream */
} ora_params;

typedef struct ora_sim ora_sim;

ora_sim *ora_create(const ora_params *p);
void ora_destroy(ora_sim *s);
const char *ora_error(const ora_sim *s);

/* rows, columns and first row index of component comp (see table above) */
int ora_field_shape(const ora_sim *s, int comp, int32_t *rows, int32_t *cols, int32_t *row0);
int ora_set_field(ora_sim *s, int comp, const double *data);
int ora_get_field(const ora_sim *s, int comp, double *out);

/* particles: absolute grid coordinates x (radial), y (meridional); momenta
 * u = gamma v / c in the local (r, theta, phi) basis; w = signed macro charge */
int ora_add_particles(ora_sim *s, int64_t n, const double *x, const double *y,
                      const double *ur, const double *ut, const double *up,
                      const double *w, const uint64_t *id);
/* the same from cell indices (ci radial, cj meridional) and in-cell offsets */
int ora_add_particles_cells(ora_sim *s, int64_t n, const int32_t *ci, const double *fx, const int32_t *cj,
                            const double *fy, const double *ur, const double *ut, const double *up,
                            const double *w, const uint64_t *id);
int64_t ora_num_particles(const ora_sim *s);
int ora_get_particles(const ora_sim *s, double *x, double *y, double *ur, double *ut,
                      double *up, double *w, uint64_t *id);

int ora_step(ora_sim *s, int32_t nsteps);
int64_t ora_step_index(const ora_sim *s);
void ora_set_step_index(ora_sim *s, int64_t n);
void ora_counters(const ora_sim *s, int64_t *injected, int64_t *deleted);
void ora_set_threads(int n);
int ora_get_threads(void);

/* carry of the fractional injection counts, one per theta node (nth+1) */
int ora_get_carry(const ora_sim *s, double *out);
int ora_set_carry(ora_sim *s, const double *in);

/* Gauss diagnostics on nodes (i, j), i = 0..nr, j = 0..nth:
 * G = closed-surface flux of E through the dual cell, Q = filtered node
 * charge of the particles.  Rows i = 0 and i = nr are left at zero. */
int ora_gauss(const ora_sim *s, double *G, double *Q);
/* Poynting luminosity through the sphere of each radial half-node
 * (nr values), total fields at the current time (Sec. 5.4). */
int ora_poynting(const ora_sim *s, double *L);

/* unit-level entry points used by the pin tests */
int ora_geometry(const ora_sim *s, int which, double *out);
void ora_push_cartesian(int mover, const double u[3], const double E[3],
                        const double B[3], double eps, double u_out[3]);
void ora_background(const ora_sim *s, double x, double y, double t,
                    double E[3], double B[3]);
void ora_gather(const ora_sim *s, double x, double y, double E[3], double B[3]);
/* deposit one straight grid-space move of charge Q into the F arrays */
int ora_deposit(ora_sim *s, double x0, double y0, double x1, double y1, double Q, double dphi);
int ora_clear_F(ora_sim *s);
int ora_filter_F(ora_sim *s);
/* n_filt passes of the node (integer i, integer j) filter on an array shaped
 * like component 8 -- the filtered particle shape of App. B */
int ora_filter_nodes(const ora_sim *s, double *rho);
/* node charge (no filter) of one particle into a (nr+1+2g) x (nth+1) array */
int ora_node_charge(const ora_sim *s, double x, double y, double Q, double *rho);
void ora_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
int32_t ora_ghost(const ora_sim *s);

#ifdef __cplusplus
}
#endif
#endif
