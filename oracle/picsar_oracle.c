/*
 * picsar_oracle.c -- plain, slow, FP64 CPU oracle of one PICsar step.
 *
 * TEST INFRASTRUCTURE ONLY: called from the test suite, the smoke check and
 * the benchmark's CPU-baseline leg, never from the product path.  It shares
 * no code with the GPU library; it is written from the paper (Belyaev 2015,
 * arXiv 1407.1810) section by section:
 *
 *   stretch functions ............ Sec. 3.2 (log radius, equal-area theta)
 *   area / line elements ......... App. A, eqs. (rtdefs), (linearea)
 *   Faraday / Ampere update ...... App. A, eq. (discreteeq), polar rows
 *                                  eq. (erpolarupdate), leapfrog Sec. 3.1
 *   conducting walls, lossy layer  Sec. 3.4.1, eq. (EBcond)
 *   particle boundaries .......... Sec. 3.4.2
 *   mover ........................ Sec. 3.3 (Vay / Boris in Cartesian)
 *   charge-conserving deposit .... Sec. 2 eq. (Jcons), Sec. 3.3 (VB)
 *   1-2-1 filter + polar remap ... App. B, eq. (filtereq) and its V tables
 *   initial (vacuum) fields ...... Sec. 5.2 eqs. (initialfields_outside/
 *                                  inside), Sec. 4.3 (dipole + corotation)
 *   spin-up ...................... Sec. 5.2
 *   surface injection ............ Sec. 5.3 eq. (volinjeq)
 *
 * Readings where the paper is silent (gather, loop order, J_phi deposit,
 * injection placement, absorber variable, dipole exterior E) are the ones
 * listed in the design notes; each is marked "reading:" below.
 *
 * Units: Lorentz-Heaviside (Sec. 2), time step dt = 1, c = Courant number in
 * code lengths per step.  Momenta u = gamma v / c.  F arrays hold charge
 * crossing a face during one step (the J of App. B is charge per face per
 * step, cf. the definition Delta Q = J^{i-1} - J^i there).
 */
#include "picsar_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846
#define NCOMP 9

struct ora_sim {
    ora_params p;
    int32_t g;                 /* ghost rows of the F arrays */
    double dxi;                /* LOG: ln(r_out/r_in)/nr, LIN: (r_out-r_in)/nr */
    double *f[NCOMP];
    int32_t rows[NCOMP], cols[NCOMP], row0[NCOMP];
    int64_t n, cap;
    double *x, *y, *ur, *ut, *up, *w;
    double *dp;                /* distance in y to the nearer pole, min(y, nth - y),
                                  kept to full relative precision */
    uint64_t *id;
    double *carry;             /* fractional injection count per theta node */
    int64_t step;
    int64_t n_injected, n_deleted;
    char err[256];
};

static int g_threads = 1;

void ora_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int ora_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------ */
/* Stretch functions f_r, f_theta (Sec. 3.2)                          */
/* ------------------------------------------------------------------ */

/* radius of radial grid coordinate x: xi = r0 ln(r/r0) uniform (LOG) or r
 * uniform (LIN) */
static double f_r(const ora_sim *s, double x)
{
    if (s->p.r_kind == ORA_R_LOG) return s->p.r_in * exp(x * s->dxi);
    return s->p.r_in + x * s->dxi;
}

static double x_of_r(const ora_sim *s, double r)
{
    if (s->p.r_kind == ORA_R_LOG) return log(r / s->p.r_in) / s->dxi;
    return (r - s->p.r_in) / s->dxi;
}

/* equal-area coordinate theta_A = -cos(theta) uniform on [-1, 1]: node y
 * has cos(theta) = 1 - 2 y / nth; linear: theta = pi y / nth */
static double cos_th(const ora_sim *s, double y)
{
    if (s->p.th_kind == ORA_TH_EQAREA) return 1.0 - 2.0 * y / s->p.nth;
    return cos(PI * y / s->p.nth);
}

static double sin_th(const ora_sim *s, double y)
{
    if (s->p.th_kind == ORA_TH_EQAREA) {
        double a = y * (s->p.nth - y);
        return 2.0 / s->p.nth * sqrt(a > 0.0 ? a : 0.0);
    }
    return sin(PI * y / s->p.nth);
}

static double f_th(const ora_sim *s, double y)
{
    if (s->p.th_kind == ORA_TH_EQAREA) {
        double a = y / s->p.nth;
        if (a < 0.0) a = 0.0;
        if (a > 1.0) a = 1.0;
        return 2.0 * asin(sqrt(a)); /* 1 - cos(theta) = 2 sin^2(theta/2) */
    }
    return PI * y / s->p.nth;
}

/* Near a pole the absolute coordinate y (up to nth) cannot resolve the
 * distance to the pole that sin(theta) depends on (Sec. 3.2 writes
 * sin(theta) through both factors y and nth - y so that neither cancels).
 * Every particle therefore also carries dp = min(y, nth - y) to full
 * relative precision; its trigonometric factors come from dp. */
static double pole_dist(const ora_sim *s, double y)
{
    return y <= 0.5 * s->p.nth ? y : s->p.nth - y;
}

static void trig_at(const ora_sim *s, double y, double dp, double *kc, double *sn)
{
    const int nth = s->p.nth;
    const int south = y > 0.5 * nth;
    if (s->p.th_kind == ORA_TH_EQAREA) {
        const double a = dp * (nth - dp);
        *sn = 2.0 / nth * sqrt(a > 0.0 ? a : 0.0);
        *kc = south ? -1.0 + 2.0 * dp / nth : 1.0 - 2.0 * dp / nth;
    } else {
        *sn = sin(PI * dp / nth);
        *kc = south ? -cos(PI * dp / nth) : cos(PI * dp / nth);
    }
}

/* Distance to the nearer pole of the point (R, Z) at radius r, without
 * cancellation: 1 - |cos(theta)| = R^2 / (r (r + |Z|)). */
static double pole_dist_of(const ora_sim *s, double R, double Z, double r)
{
    if (s->p.th_kind == ORA_TH_EQAREA) return 0.5 * s->p.nth * R * R / (r * (r + fabs(Z)));
    return s->p.nth * atan2(R, fabs(Z)) / PI;
}

/* ------------------------------------------------------------------ */
/* Area and line elements, App. A eq. (linearea)                      */
/* ------------------------------------------------------------------ */

static double dA_tp(double r, double cos_a, double cos_b) { return 2.0 * PI * r * r * (cos_a - cos_b); }
static double dA_rp(double ra, double rb, double sin_t) { return PI * (rb * rb - ra * ra) * sin_t; }
static double dA_rt(double ra, double rb, double ta, double tb) { return 0.5 * (rb * rb - ra * ra) * (tb - ta); }
static double dL_r(double ra, double rb) { return rb - ra; }
static double dL_t(double r, double ta, double tb) { return r * (tb - ta); }
static double dL_p(double r, double sin_t) { return 2.0 * PI * r * sin_t; }

/* ------------------------------------------------------------------ */
/* Storage                                                            */
/* ------------------------------------------------------------------ */

static double *fld(const ora_sim *s, int c, int i, int j)
{
    return &s->f[c][(int64_t)(i - s->row0[c]) * s->cols[c] + j];
}
#define ER(i, j) (*fld(s, 0, (i), (j)))
#define ETH(i, j) (*fld(s, 1, (i), (j)))
#define EPH(i, j) (*fld(s, 2, (i), (j)))
#define BR(i, j) (*fld(s, 3, (i), (j)))
#define BTH(i, j) (*fld(s, 4, (i), (j)))
#define BPH(i, j) (*fld(s, 5, (i), (j)))

static void set_err(ora_sim *s, const char *m)
{
    snprintf(s->err, sizeof s->err, "%s", m);
}

const char *ora_error(const ora_sim *s) { return s ? s->err : "null simulation"; }
int32_t ora_ghost(const ora_sim *s) { return s->g; }

ora_sim *ora_create(const ora_params *p)
{
    if (!p || p->nr < 2 || p->nth < 4 || !(p->r_in > 0.0) || !(p->r_out > p->r_in) ||
        !(p->c > 0.0) || p->n_filt < 0 || p->absorb_cells < 0 || p->absorb_cells > p->nr)
        return NULL;
    ora_sim *s = (ora_sim *)calloc(1, sizeof *s);
    if (!s) return NULL;
    s->p = *p;
    s->g = 2 * p->n_filt + 3;
    s->dxi = p->r_kind == ORA_R_LOG ? log(p->r_out / p->r_in) / p->nr : (p->r_out - p->r_in) / p->nr;
    const int nr = p->nr, nth = p->nth, g = s->g;
    const int32_t rows[NCOMP] = {nr, nr + 1, nr + 1, nr + 1, nr, nr, nr + 2 * g, nr + 1 + 2 * g, nr + 1 + 2 * g};
    const int32_t cols[NCOMP] = {nth + 1, nth, nth + 1, nth, nth + 1, nth, nth + 1, nth, nth + 1};
    for (int c = 0; c < NCOMP; ++c) {
        s->rows[c] = rows[c];
        s->cols[c] = cols[c];
        s->row0[c] = c >= 6 ? -g : 0;
        s->f[c] = (double *)calloc((size_t)rows[c] * cols[c], sizeof(double));
        if (!s->f[c]) { ora_destroy(s); return NULL; }
    }
    s->carry = (double *)calloc((size_t)nth + 1, sizeof(double));
    if (!s->carry) { ora_destroy(s); return NULL; }
    return s;
}

static void free_particles(ora_sim *s)
{
    free(s->x); free(s->y); free(s->ur); free(s->ut); free(s->up); free(s->w); free(s->dp); free(s->id);
    s->x = s->y = s->ur = s->ut = s->up = s->w = NULL;
    s->id = NULL;
}

void ora_destroy(ora_sim *s)
{
    if (!s) return;
    for (int c = 0; c < NCOMP; ++c) free(s->f[c]);
    free_particles(s);
    free(s->carry);
    free(s);
}

int ora_field_shape(const ora_sim *s, int comp, int32_t *rows, int32_t *cols, int32_t *row0)
{
    if (!s || comp < 0 || comp >= NCOMP) return ORA_EINVAL;
    if (rows) *rows = s->rows[comp];
    if (cols) *cols = s->cols[comp];
    if (row0) *row0 = s->row0[comp];
    return ORA_OK;
}

int ora_set_field(ora_sim *s, int comp, const double *data)
{
    if (!s || comp < 0 || comp >= NCOMP || !data) return ORA_EINVAL;
    memcpy(s->f[comp], data, sizeof(double) * s->rows[comp] * s->cols[comp]);
    return ORA_OK;
}

int ora_get_field(const ora_sim *s, int comp, double *out)
{
    if (!s || comp < 0 || comp >= NCOMP || !out) return ORA_EINVAL;
    memcpy(out, s->f[comp], sizeof(double) * s->rows[comp] * s->cols[comp]);
    return ORA_OK;
}

static int reserve(ora_sim *s, int64_t need)
{
    if (need <= s->cap) return ORA_OK;
    int64_t cap = s->cap ? s->cap : 1024;
    while (cap < need) cap *= 2;
    double **arr[7] = {&s->x, &s->y, &s->ur, &s->ut, &s->up, &s->w, &s->dp};
    for (int a = 0; a < 7; ++a) {
        double *q = (double *)realloc(*arr[a], sizeof(double) * cap);
        if (!q) return ORA_ENOMEM;
        *arr[a] = q;
    }
    uint64_t *q = (uint64_t *)realloc(s->id, sizeof(uint64_t) * cap);
    if (!q) return ORA_ENOMEM;
    s->id = q;
    s->cap = cap;
    return ORA_OK;
}

int ora_add_particles(ora_sim *s, int64_t n, const double *x, const double *y, const double *ur,
                      const double *ut, const double *up, const double *w, const uint64_t *id)
{
    if (!s || n < 0) return ORA_EINVAL;
    if (reserve(s, s->n + n) != ORA_OK) return ORA_ENOMEM;
    for (int64_t k = 0; k < n; ++k) {
        int64_t d = s->n + k;
        s->x[d] = x[k];
        s->y[d] = y[k];
        s->dp[d] = pole_dist(s, y[k]);
        s->ur[d] = ur[k];
        s->ut[d] = ut[k];
        s->up[d] = up[k];
        s->w[d] = w[k];
        s->id[d] = id ? id[k] : (uint64_t)d;
    }
    s->n += n;
    return ORA_OK;
}

/* The same from cell indices and in-cell offsets (a state stored as cell +
 * offset): the distance to the nearer pole is formed from the offset,
 * min(j + fy, (nth - j) - fy), before the absolute coordinate rounds it. */
int ora_add_particles_cells(ora_sim *s, int64_t n, const int32_t *ci, const double *fx, const int32_t *cj,
                            const double *fy, const double *ur, const double *ut, const double *up,
                            const double *w, const uint64_t *id)
{
    if (!s || n < 0) return ORA_EINVAL;
    if (reserve(s, s->n + n) != ORA_OK) return ORA_ENOMEM;
    const int nth = s->p.nth;
    for (int64_t k = 0; k < n; ++k) {
        int64_t d = s->n + k;
        s->x[d] = ci[k] + fx[k];
        s->y[d] = cj[k] + fy[k];
        const double north = cj[k] + fy[k], south = (double)(nth - cj[k]) - fy[k];
        s->dp[d] = north <= south ? north : south;
        s->ur[d] = ur[k];
        s->ut[d] = ut[k];
        s->up[d] = up[k];
        s->w[d] = w[k];
        s->id[d] = id ? id[k] : (uint64_t)d;
    }
    s->n += n;
    return ORA_OK;
}

int64_t ora_num_particles(const ora_sim *s) { return s ? s->n : -1; }

int ora_get_particles(const ora_sim *s, double *x, double *y, double *ur, double *ut, double *up,
                      double *w, uint64_t *id)
{
    if (!s) return ORA_EINVAL;
    size_t b = sizeof(double) * (size_t)s->n;
    if (x) memcpy(x, s->x, b);
    if (y) memcpy(y, s->y, b);
    if (ur) memcpy(ur, s->ur, b);
    if (ut) memcpy(ut, s->ut, b);
    if (up) memcpy(up, s->up, b);
    if (w) memcpy(w, s->w, b);
    if (id) memcpy(id, s->id, sizeof(uint64_t) * (size_t)s->n);
    return ORA_OK;
}

int64_t ora_step_index(const ora_sim *s) { return s->step; }
void ora_set_step_index(ora_sim *s, int64_t n) { s->step = n; }

void ora_counters(const ora_sim *s, int64_t *injected, int64_t *deleted)
{
    if (injected) *injected = s->n_injected;
    if (deleted) *deleted = s->n_deleted;
}

int ora_get_carry(const ora_sim *s, double *out)
{
    memcpy(out, s->carry, sizeof(double) * (s->p.nth + 1));
    return ORA_OK;
}

int ora_set_carry(ora_sim *s, const double *in)
{
    memcpy(s->carry, in, sizeof(double) * (s->p.nth + 1));
    return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* Field solve, App. A                                                */
/* ------------------------------------------------------------------ */

/* Faraday's law in integral form, eq. (discreteeq) first three lines,
 * advanced by a fraction h of a step.  B_r = 0 on the conductors and
 * B_theta = 0 on the axis (Sec. 3.4.1, App. A). */
static void faraday(ora_sim *s, double h)
{
    const int nr = s->p.nr, nth = s->p.nth;
    const double c = s->p.c * h;
    for (int i = 1; i < nr; ++i) {
        const double r = f_r(s, i);
        for (int j = 0; j < nth; ++j) {
            double circ = EPH(i, j) * dL_p(r, sin_th(s, j)) - EPH(i, j + 1) * dL_p(r, sin_th(s, j + 1));
            BR(i, j) += c * circ / dA_tp(r, cos_th(s, j), cos_th(s, j + 1));
        }
    }
    for (int i = 0; i < nr; ++i) {
        const double ra = f_r(s, i), rb = f_r(s, i + 1);
        for (int j = 1; j < nth; ++j) {
            const double st = sin_th(s, j);
            double circ = EPH(i + 1, j) * dL_p(rb, st) - EPH(i, j) * dL_p(ra, st);
            BTH(i, j) += c * circ / dA_rp(ra, rb, st);
        }
    }
    for (int i = 0; i < nr; ++i) {
        const double ra = f_r(s, i), rb = f_r(s, i + 1);
        for (int j = 0; j < nth; ++j) {
            const double ta = f_th(s, j), tb = f_th(s, j + 1);
            double circ = (ETH(i, j) * dL_t(ra, ta, tb) - ETH(i + 1, j) * dL_t(rb, ta, tb)) -
                          (ER(i, j) - ER(i, j + 1)) * dL_r(ra, rb);
            BPH(i, j) += c * circ / dA_rt(ra, rb, ta, tb);
        }
    }
}

/* Ampere's law in integral form, eq. (discreteeq) last three lines, with the
 * face charges F (current times area times dt) of the deposit; the axis rows
 * of E_r use the polar cap, eq. (erpolarupdate).  E_theta = E_phi = 0 on the
 * conductors and E_phi = 0 on the axis. */
static void ampere(ora_sim *s)
{
    const int nr = s->p.nr, nth = s->p.nth;
    const double c = s->p.c;
    for (int i = 0; i < nr; ++i) {
        const double r = f_r(s, i + 0.5);
        for (int j = 0; j <= nth; ++j) {
            double circ, area;
            if (j == 0) {
                circ = BPH(i, 0) * dL_p(r, sin_th(s, 0.5));
                area = dA_tp(r, 1.0, cos_th(s, 0.5));
            } else if (j == nth) {
                circ = -BPH(i, nth - 1) * dL_p(r, sin_th(s, nth - 0.5));
                area = dA_tp(r, cos_th(s, nth - 0.5), -1.0);
            } else {
                circ = BPH(i, j) * dL_p(r, sin_th(s, j + 0.5)) - BPH(i, j - 1) * dL_p(r, sin_th(s, j - 0.5));
                area = dA_tp(r, cos_th(s, j - 0.5), cos_th(s, j + 0.5));
            }
            ER(i, j) += (c * circ - *fld(s, 6, i, j)) / area;
        }
    }
    for (int i = 1; i < nr; ++i) {
        const double ra = f_r(s, i - 0.5), rb = f_r(s, i + 0.5);
        for (int j = 0; j < nth; ++j) {
            const double st = sin_th(s, j + 0.5);
            double circ = BPH(i - 1, j) * dL_p(ra, st) - BPH(i, j) * dL_p(rb, st);
            ETH(i, j) += (c * circ - *fld(s, 7, i, j)) / dA_rp(ra, rb, st);
        }
    }
    for (int i = 1; i < nr; ++i) {
        const double ra = f_r(s, i - 0.5), rb = f_r(s, i + 0.5);
        for (int j = 1; j < nth; ++j) {
            const double ta = f_th(s, j - 0.5), tb = f_th(s, j + 0.5);
            double circ = (BTH(i, j) * dL_t(rb, ta, tb) - BTH(i - 1, j) * dL_t(ra, ta, tb)) -
                          (BR(i, j) - BR(i, j - 1)) * dL_r(ra, rb);
            EPH(i, j) += (c * circ - *fld(s, 8, i, j)) / dA_rt(ra, rb, ta, tb);
        }
    }
}

/* Lossy layer, eq. (EBcond): sigma* rises linearly from 0 at the inner edge
 * of the layer to sigma_max at the outer conductor.  reading: "linear with
 * radius" is taken in the radial grid coordinate, evaluated at each
 * component's own staggered position rho. */
static double absorb_factor(const ora_sim *s, double rho)
{
    const int L = s->p.absorb_cells;
    if (L <= 0) return 1.0;
    const double edge = (double)(s->p.nr - L);
    if (rho <= edge) return 1.0;
    return 1.0 - s->p.sigma_max * (rho - edge) / L;
}

static void absorb(ora_sim *s)
{
    if (s->p.absorb_cells <= 0) return;
    for (int c = 0; c < 6; ++c) {
        const double sx = (c == 0 || c == 4 || c == 5) ? 0.5 : 0.0;
        for (int i = 0; i < s->rows[c]; ++i) {
            const double a = absorb_factor(s, i + sx);
            if (a == 1.0) continue;
            for (int j = 0; j < s->cols[c]; ++j) *fld(s, c, i, j) *= a;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Analytic initial fields (Sec. 5.2; Sec. 4.3 for the dipole)        */
/* ------------------------------------------------------------------ */

static double omega_at(const ora_sim *s, double t)
{
    if (s->p.t_spin > 0.0 && t < s->p.t_spin) return s->p.omega * t / s->p.t_spin;
    return s->p.omega;
}

/* Local (r, theta, phi) components at grid position (x, y), time t.  Inside
 * the star (x < 0) the corotation form is used; outside, the vacuum form.
 * reading (dipole exterior, not given in the paper): the l = 2 vacuum
 * potential that matches the corotation surface potential with no net
 * charge, the same rule that yields the paper's monopole exterior. */
static void background_at(const ora_sim *s, double x, double r, double k, double sn, double t, double E[3],
                          double B[3])
{
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0;
    const double r0 = s->p.r_in, B0 = s->p.B0;
    const double inv_rl = omega_at(s, t) / s->p.c; /* 1 / R_l */
    switch (s->p.bg_kind) {
    case ORA_BG_UNIFORM_BZ:
        B[0] = B0 * k;
        B[1] = -B0 * sn;
        break;
    case ORA_BG_MONOPOLE:
        B[0] = B0 * (r0 / r) * (r0 / r);
        if (x < 0.0) {
            E[1] = -B0 * r0 * r0 * sn * inv_rl / r;
        } else {
            const double a = B0 * r0 * r0 * r0 * r0 * inv_rl / (r * r * r);
            E[0] = -2.0 * a * k;
            E[1] = -a * sn;
        }
        break;
    case ORA_BG_DIPOLE:
    case ORA_BG_DIPOLE_COROT: {
        const double mu = B0 * r0 * r0 * r0;
        B[0] = 2.0 * mu * k / (r * r * r);
        B[1] = mu * sn / (r * r * r);
        if (x < 0.0 || s->p.bg_kind == ORA_BG_DIPOLE_COROT) {
            E[0] = mu * sn * sn * inv_rl / (r * r);
            E[1] = -mu * 2.0 * sn * k * inv_rl / (r * r);
        } else {
            const double a = 2.0 * mu * r0 * r0 * inv_rl / (r * r * r * r);
            E[0] = -a * 0.5 * (3.0 * k * k - 1.0);
            E[1] = -a * sn * k;
        }
        break;
    }
    default:
        break;
    }
}

void ora_background(const ora_sim *s, double x, double y, double t, double E[3], double B[3])
{
    background_at(s, x, f_r(s, x), cos_th(s, y), sin_th(s, y), t, E, B);
}

/* ------------------------------------------------------------------ */
/* Gather.  reading: each plasma component is interpolated bilinearly  */
/* in grid coordinates from its own staggered lattice (the cell-shaped */
/* particle of Sec. 3.3); across the axis the lattice is continued by  */
/* mirror parity (r components even, theta and phi components odd);   */
/* beyond the conductors the plasma field is zero.                     */
/* ------------------------------------------------------------------ */

static double node_val(const ora_sim *s, int c, int i, int j, int half_j, double parity)
{
    if (i < 0 || i >= s->rows[c]) return 0.0;
    const int nth = s->p.nth;
    double sign = 1.0;
    if (half_j) {
        if (j < 0) { j = -1 - j; sign = parity; }
        else if (j >= nth) { j = 2 * nth - 1 - j; sign = parity; }
    } else {
        if (j < 0) { j = -j; sign = parity; }
        else if (j > nth) { j = 2 * nth - j; sign = parity; }
    }
    return sign * *fld(s, c, i, j);
}

static double interp(const ora_sim *s, int c, double x, double y, double sx, double sy, double parity)
{
    const double u = x - sx, v = y - sy;
    const int i0 = (int)floor(u), j0 = (int)floor(v);
    const double fu = u - i0, fv = v - j0;
    const int hj = sy != 0.0;
    return (1 - fu) * (1 - fv) * node_val(s, c, i0, j0, hj, parity) +
           fu * (1 - fv) * node_val(s, c, i0 + 1, j0, hj, parity) +
           (1 - fu) * fv * node_val(s, c, i0, j0 + 1, hj, parity) +
           fu * fv * node_val(s, c, i0 + 1, j0 + 1, hj, parity);
}

void ora_gather(const ora_sim *s, double x, double y, double E[3], double B[3])
{
    E[0] = interp(s, 0, x, y, 0.5, 0.0, 1.0);
    E[1] = interp(s, 1, x, y, 0.0, 0.5, -1.0);
    E[2] = interp(s, 2, x, y, 0.0, 0.0, -1.0);
    B[0] = interp(s, 3, x, y, 0.0, 0.5, 1.0);
    B[1] = interp(s, 4, x, y, 0.5, 0.0, -1.0);
    B[2] = interp(s, 5, x, y, 0.5, 0.5, -1.0);
}

/* ------------------------------------------------------------------ */
/* Movers (Sec. 3.3): Vay (2008) and Boris (1970), in Cartesian form,  */
/* u = gamma v / c, eps = q dt / (2 m c)                                */
/* ------------------------------------------------------------------ */

static void cross(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

void ora_push_cartesian(int mover, const double u[3], const double E[3], const double B[3], double eps,
                        double out[3])
{
    if (mover == ORA_BORIS) {
        double um[3], t[3], sv[3], c1[3], up[3], c2[3];
        for (int a = 0; a < 3; ++a) um[a] = u[a] + eps * E[a];
        const double gm = sqrt(1.0 + dot(um, um));
        for (int a = 0; a < 3; ++a) t[a] = eps * B[a] / gm;
        const double f = 2.0 / (1.0 + dot(t, t));
        for (int a = 0; a < 3; ++a) sv[a] = f * t[a];
        cross(um, t, c1);
        for (int a = 0; a < 3; ++a) up[a] = um[a] + c1[a];
        cross(up, sv, c2);
        for (int a = 0; a < 3; ++a) out[a] = um[a] + c2[a] + eps * E[a];
        return;
    }
    /* Vay: u' = u + 2 eps E + eps (u / gamma) x B, then solve the implicit
     * rotation for gamma at the new time level */
    const double g = sqrt(1.0 + dot(u, u));
    double vb[3], up[3], tau[3], t[3], c1[3];
    const double v[3] = {u[0] / g, u[1] / g, u[2] / g};
    cross(v, B, vb);
    for (int a = 0; a < 3; ++a) up[a] = u[a] + 2.0 * eps * E[a] + eps * vb[a];
    for (int a = 0; a < 3; ++a) tau[a] = eps * B[a];
    const double tau2 = dot(tau, tau);
    const double ustar = dot(up, tau);
    const double sigma = 1.0 + dot(up, up) - tau2;
    const double gnew = sqrt(0.5 * (sigma + sqrt(sigma * sigma + 4.0 * (tau2 + ustar * ustar))));
    for (int a = 0; a < 3; ++a) t[a] = tau[a] / gnew;
    const double sfac = 1.0 / (1.0 + dot(t, t));
    const double ut = dot(up, t);
    cross(up, t, c1);
    for (int a = 0; a < 3; ++a) out[a] = sfac * (up[a] + ut * t[a] + c1[a]);
}

/* ------------------------------------------------------------------ */
/* Villasenor-Buneman deposit in grid coordinates (Sec. 3.3)          */
/* ------------------------------------------------------------------ */

typedef struct {
    double *Fr, *Ft, *Fp; /* arrays shaped like components 6, 7, 8 */
} fset;

static int cell_j(const ora_sim *s, double y)
{
    int j = (int)floor(y);
    if (j > s->p.nth - 1) j = s->p.nth - 1; /* y = nth belongs to the last cell */
    if (j < 0) j = 0;
    return j;
}

static double *fref(const ora_sim *s, double *a, int c, int i, int j)
{
    return &a[(int64_t)(i - s->row0[c]) * s->cols[c] + j];
}

/* The straight grid-space path is cut where it crosses integer x or y
 * (at most one crossing per axis for a move shorter than a cell); on each
 * piece inside cell (i, j) the charge flux of a cell-sized cloud through the
 * dual faces is the exact integral of the bilinear weights along the piece.
 * reading (J_phi, not given in the paper): the ring rotates by dphi, so the
 * charge Q dphi / 2 pi crosses a meridional half-plane; it is assigned to
 * the nodes with the bilinear weights of the midpoint of the move. */
static void deposit_path(const ora_sim *s, fset *F, double x0, double y0, double x1, double y1, double Q,
                         double dphi)
{
    double px[4], py[4], pt[4];
    int np = 0;
    px[np] = x0; py[np] = y0; pt[np++] = 0.0;
    const int ia = (int)floor(x0), ib = (int)floor(x1);
    const int ja = cell_j(s, y0), jb = cell_j(s, y1);
    double tx = -1.0, ty = -1.0, X = 0.0, Y = 0.0;
    if (ia != ib) { X = (double)(ib > ia ? ib : ia); tx = (X - x0) / (x1 - x0); }
    if (ja != jb) { Y = (double)(jb > ja ? jb : ja); ty = (Y - y0) / (y1 - y0); }
    if (tx >= 0.0 && ty >= 0.0 && tx == ty) {
        px[np] = X; py[np] = Y; pt[np++] = tx;
    } else {
        if (tx >= 0.0 && (ty < 0.0 || tx < ty)) { px[np] = X; py[np] = y0 + tx * (y1 - y0); pt[np++] = tx; }
        if (ty >= 0.0) { px[np] = x0 + ty * (x1 - x0); py[np] = Y; pt[np++] = ty; }
        if (tx >= 0.0 && ty >= 0.0 && tx > ty) { px[np] = X; py[np] = y0 + tx * (y1 - y0); pt[np++] = tx; }
    }
    px[np] = x1; py[np] = y1; pt[np++] = 1.0;
    (void)pt;
    for (int k = 0; k + 1 < np; ++k) {
        const double xa = px[k], ya = py[k], xb = px[k + 1], yb = py[k + 1];
        const double xm = 0.5 * (xa + xb), ym = 0.5 * (ya + yb);
        const int i = (int)floor(xm), j = cell_j(s, ym);
        const double fx = xm - i, fy = ym - j;
        const double dx = xb - xa, dy = yb - ya;
        *fref(s, F->Fr, 6, i, j) += Q * dx * (1.0 - fy);
        *fref(s, F->Fr, 6, i, j + 1) += Q * dx * fy;
        *fref(s, F->Ft, 7, i, j) += Q * dy * (1.0 - fx);
        *fref(s, F->Ft, 7, i + 1, j) += Q * dy * fx;
    }
    const double xm = 0.5 * (x0 + x1), ym = 0.5 * (y0 + y1);
    const int i = (int)floor(xm), j = cell_j(s, ym);
    const double fx = xm - i, fy = ym - j;
    const double q = Q * dphi / (2.0 * PI);
    *fref(s, F->Fp, 8, i, j) += q * (1 - fx) * (1 - fy);
    *fref(s, F->Fp, 8, i + 1, j) += q * fx * (1 - fy);
    *fref(s, F->Fp, 8, i, j + 1) += q * (1 - fx) * fy;
    *fref(s, F->Fp, 8, i + 1, j + 1) += q * fx * fy;
}

int ora_deposit(ora_sim *s, double x0, double y0, double x1, double y1, double Q, double dphi)
{
    fset F = {s->f[6], s->f[7], s->f[8]};
    deposit_path(s, &F, x0, y0, x1, y1, Q, dphi);
    return ORA_OK;
}

int ora_clear_F(ora_sim *s)
{
    for (int c = 6; c < NCOMP; ++c) memset(s->f[c], 0, sizeof(double) * s->rows[c] * s->cols[c]);
    return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* Current filter, App. B eq. (filtereq) with the polar remap tables  */
/* ------------------------------------------------------------------ */

/* meridional weights V_l, l = -1, 0, +1, of the target node j; build index
 * j = paper index - 1.  Integer-j components (r, phi): */
static void vtab_int(int j, int nth, double V[3])
{
    V[0] = 0.25; V[1] = 0.5; V[2] = 0.25;
    if (j == 0) { V[0] = 0.0; V[1] = 0.5; V[2] = 0.25; }
    else if (j == 1) { V[0] = 0.5; V[1] = 0.5; V[2] = 0.25; }
    else if (j == nth - 1) { V[0] = 0.25; V[1] = 0.5; V[2] = 0.5; }
    else if (j == nth) { V[0] = 0.25; V[1] = 0.5; V[2] = 0.0; }
}

/* half-integer-j component (theta), positions j + 1/2, j = 0..nth-1 */
static void vtab_half(int j, int nth, double V[3])
{
    V[0] = 0.25; V[1] = 0.5; V[2] = 0.25;
    if (j == 0) { V[0] = 0.0; V[1] = 0.25; V[2] = 0.25; }
    else if (j == nth - 1) { V[0] = 0.25; V[1] = 0.25; V[2] = 0.0; }
}

/* one pass of J_bar(i,j) = sum_k sum_l W_k V_l J(i+k, j+l) over an array of
 * `rows` rows and `cols` columns; radially the array is continued by zeros
 * (its ghost rows are wide enough that nothing reaches the ends). */
static void filter_pass(double *a, int rows, int cols, int nth, int half_j, double *tmp)
{
    static const double W[3] = {0.25, 0.5, 0.25};
    for (int i = 0; i < rows; ++i) {
        for (int j = 0; j < cols; ++j) {
            double V[3];
            if (half_j) vtab_half(j, nth, V); else vtab_int(j, nth, V);
            double acc = 0.0;
            for (int k = -1; k <= 1; ++k) {
                const int ii = i + k;
                if (ii < 0 || ii >= rows) continue;
                for (int l = -1; l <= 1; ++l) {
                    if (V[l + 1] == 0.0) continue;
                    acc += W[k + 1] * V[l + 1] * a[(int64_t)ii * cols + j + l];
                }
            }
            tmp[(int64_t)i * cols + j] = acc;
        }
    }
    memcpy(a, tmp, sizeof(double) * rows * cols);
}

static int filter_array(double *a, int rows, int cols, int nth, int half_j, int passes)
{
    if (passes <= 0) return ORA_OK;
    double *tmp = (double *)malloc(sizeof(double) * rows * cols);
    if (!tmp) return ORA_ENOMEM;
    for (int p = 0; p < passes; ++p) filter_pass(a, rows, cols, nth, half_j, tmp);
    free(tmp);
    return ORA_OK;
}

int ora_filter_F(ora_sim *s)
{
    const int nth = s->p.nth;
    int rc = filter_array(s->f[6], s->rows[6], s->cols[6], nth, 0, s->p.n_filt);
    if (rc == ORA_OK) rc = filter_array(s->f[7], s->rows[7], s->cols[7], nth, 1, s->p.n_filt);
    if (rc == ORA_OK) rc = filter_array(s->f[8], s->rows[8], s->cols[8], nth, 0, s->p.n_filt);
    return rc;
}

int ora_filter_nodes(const ora_sim *s, double *rho)
{
    return filter_array(rho, s->rows[8], s->cols[8], s->p.nth, 0, s->p.n_filt);
}

/* ------------------------------------------------------------------ */
/* Random numbers for injection: Philox4x64-10 (Salmon et al. 2011)   */
/* ------------------------------------------------------------------ */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void ora_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        uint64_t h0, l0, h1, l1;
        mulhilo64(0xD2E7470EE14C6C93ULL, x0, &h0, &l0);
        mulhilo64(0xCA5A826395121157ULL, x2, &h1, &l1);
        const uint64_t y0 = h1 ^ x1 ^ k0, y2 = h0 ^ x3 ^ k1;
        x0 = y0; x1 = l1; x2 = y2; x3 = l0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------ */
/* Surface injection, Sec. 5.3 eq. (volinjeq)                         */
/* ------------------------------------------------------------------ */

/* reading: sigma_j is the jump of the total E_r across the conductor,
 * taken as E_r at (1/2, j) (inside, E_r = 0); dA_j is the dual face of node
 * j on the conductor surface (polar caps at the poles); a fractional count
 * is carried to the next step; the pairs are placed at rest at x = 1/2,
 * uniformly in y over the node's dual face. */
static int inject(ora_sim *s, double t_new)
{
    if (!s->p.inject || !(s->p.bg_kind == ORA_BG_MONOPOLE || s->p.bg_kind == ORA_BG_DIPOLE)) return ORA_OK;
    const int nth = s->p.nth;
    const double qi = s->p.q_inj;
    for (int j = 0; j <= nth; ++j) {
        double Ea[3], Ba[3];
        ora_background(s, 0.5, j, t_new, Ea, Ba);
        const double sigma = ER(0, j) + Ea[0];
        const double lo = j == 0 ? 1.0 : cos_th(s, j - 0.5);
        const double hi = j == nth ? -1.0 : cos_th(s, j + 0.5);
        s->carry[j] += s->p.f_inj * fabs(sigma) * dA_tp(s->p.r_in, lo, hi) / qi;
        const double m = floor(s->carry[j]);
        s->carry[j] -= m;
        const int64_t npair = (int64_t)m;
        if (npair <= 0) continue;
        if (reserve(s, s->n + 2 * npair) != ORA_OK) return ORA_ENOMEM;
        const double ylo = j - 0.5 < 0.0 ? 0.0 : j - 0.5;
        const double yhi = j + 0.5 > nth ? (double)nth : j + 0.5;
        for (int64_t k = 0; k < npair; ++k) {
            const uint64_t ctr[4] = {(uint64_t)s->step, (uint64_t)j, (uint64_t)k, 0};
            const uint64_t key[2] = {s->p.seed, 0x50494353ULL};
            uint64_t o[4];
            ora_philox4x64_10(ctr, key, o);
            const double U = (double)(o[0] >> 11) * 0x1.0p-53;
            const double yy = ylo + U * (yhi - ylo);
            for (int sgn = 0; sgn < 2; ++sgn) {
                const int64_t d = s->n++;
                s->x[d] = 0.5;
                s->y[d] = yy;
                s->dp[d] = pole_dist(s, yy);
                s->ur[d] = s->ut[d] = s->up[d] = 0.0;
                s->w[d] = sgn == 0 ? qi : -qi;
                s->id[d] = 0x8000000000000000ULL | ((uint64_t)s->step << 36) | ((uint64_t)j << 20) |
                           ((uint64_t)k << 1) | (uint64_t)sgn;
            }
            s->n_injected += 2;
        }
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* One particle: gather, push, move, deposit (Sec. 3.3, 3.4.2)        */
/* ------------------------------------------------------------------ */

/* returns 1 if the particle is to be deleted, -1 on a CFL violation */
static int move_one(const ora_sim *s, int64_t k, double t, fset *F)
{
    const int nr = s->p.nr, nth = s->p.nth;
    const double x = s->x[k], y = s->y[k], w = s->w[k];
    const double r = f_r(s, x);
    double kc, sn;
    trig_at(s, y, s->dp[k], &kc, &sn);
    double E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
    /* particles inside the outer conductor fly ballistically; inside the
     * inner conductor they feel only the corotation field */
    if (x <= nr) {
        double Ea[3], Ba[3];
        if (x >= 0.0) ora_gather(s, x, y, E, B);
        background_at(s, x, r, kc, sn, t, Ea, Ba);
        for (int a = 0; a < 3; ++a) { E[a] += Ea[a]; B[a] += Ba[a]; }
    }
    /* local basis at phi = 0: e_r = (s, 0, k), e_th = (k, 0, -s), e_ph = y */
    const double ul[3] = {s->ur[k], s->ut[k], s->up[k]};
    const double uc[3] = {sn * ul[0] + kc * ul[1], ul[2], kc * ul[0] - sn * ul[1]};
    const double Ec[3] = {sn * E[0] + kc * E[1], E[2], kc * E[0] - sn * E[1]};
    const double Bc[3] = {sn * B[0] + kc * B[1], B[2], kc * B[0] - sn * B[1]};
    const double eps = (w > 0.0 ? 1.0 : (w < 0.0 ? -1.0 : 0.0)) * s->p.q_over_m / (2.0 * s->p.c);
    double un[3];
    if (x <= nr && eps != 0.0) ora_push_cartesian(s->p.mover, uc, Ec, Bc, eps, un);
    else { un[0] = uc[0]; un[1] = uc[1]; un[2] = uc[2]; }
    const double gnew = sqrt(1.0 + dot(un, un));
    const double X[3] = {r * sn + un[0] * s->p.c / gnew, un[1] * s->p.c / gnew, r * kc + un[2] * s->p.c / gnew};
    const double r1 = sqrt(dot(X, X));
    const double R1 = sqrt(X[0] * X[0] + X[1] * X[1]);
    const double k1 = X[2] / r1, s1 = R1 / r1;
    double cph = 1.0, sph = 0.0;
    if (R1 > 0.0) { cph = X[0] / R1; sph = X[1] / R1; }
    /* rotate the momentum back into the meridional plane of the particle */
    const double ux = cph * un[0] + sph * un[1];
    const double uy = -sph * un[0] + cph * un[1];
    const double uz = un[2];
    const double dp1 = pole_dist_of(s, R1, X[2], r1);
    double x1 = x_of_r(s, r1), y1 = X[2] >= 0.0 ? dp1 : nth - dp1;
    if (y1 < 0.0) y1 = 0.0;
    if (y1 > nth) y1 = nth;
    if (fabs(x1 - x) >= 1.0 || fabs(y1 - y) >= 1.0) return -1;
    deposit_path(s, F, x, y, x1, y1, w, atan2(sph, cph));
    s->x[k] = x1;
    s->y[k] = y1;
    s->dp[k] = dp1;
    s->ur[k] = s1 * ux + k1 * uz;
    s->ut[k] = k1 * ux - s1 * uz;
    s->up[k] = uy;
    /* delete once the whole (filtered) shape is inside a conductor */
    const double lim = s->p.n_filt + 1.0;
    return (x1 < -lim || x1 > nr + lim) ? 1 : 0;
}

static int push_particles(ora_sim *s)
{
    const double t = (double)s->step;
    const int64_t n = s->n;
    unsigned char *del = (unsigned char *)calloc(n > 0 ? n : 1, 1);
    if (!del) return ORA_ENOMEM;
    int nt = g_threads;
#ifndef _OPENMP
    nt = 1;
#endif
    if (nt > 1 && n < 4096) nt = 1;
    const size_t sz[3] = {(size_t)s->rows[6] * s->cols[6], (size_t)s->rows[7] * s->cols[7],
                          (size_t)s->rows[8] * s->cols[8]};
    double *buf = NULL;
    if (nt > 1) {
        buf = (double *)calloc((sz[0] + sz[1] + sz[2]) * (size_t)nt, sizeof(double));
        if (!buf) { free(del); return ORA_ENOMEM; }
    }
    int cfl = 0;
    if (nt == 1) {
        fset F = {s->f[6], s->f[7], s->f[8]};
        for (int64_t k = 0; k < n; ++k) {
            int rc = move_one(s, k, t, &F);
            if (rc < 0) { cfl = 1; break; }
            del[k] = (unsigned char)rc;
        }
    } else {
#ifdef _OPENMP
#pragma omp parallel num_threads(nt) reduction(| : cfl)
        {
            const int tid = omp_get_thread_num();
            double *base = buf + (sz[0] + sz[1] + sz[2]) * (size_t)tid;
            fset F = {base, base + sz[0], base + sz[0] + sz[1]};
            /* contiguous blocks so that the reduction below is in a fixed order */
            const int64_t lo = n * tid / nt, hi = n * (tid + 1) / nt;
            for (int64_t k = lo; k < hi; ++k) {
                int rc = move_one(s, k, t, &F);
                if (rc < 0) { cfl = 1; break; }
                del[k] = (unsigned char)rc;
            }
        }
        for (int th = 0; th < nt; ++th) {
            double *base = buf + (sz[0] + sz[1] + sz[2]) * (size_t)th;
            for (size_t q = 0; q < sz[0]; ++q) s->f[6][q] += base[q];
            for (size_t q = 0; q < sz[1]; ++q) s->f[7][q] += base[sz[0] + q];
            for (size_t q = 0; q < sz[2]; ++q) s->f[8][q] += base[sz[0] + sz[1] + q];
        }
#endif
    }
    free(buf);
    if (cfl) {
        free(del);
        return ORA_ECFL;
    }
    int64_t m = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (del[k]) { s->n_deleted++; continue; }
        if (m != k) {
            s->x[m] = s->x[k]; s->y[m] = s->y[k]; s->dp[m] = s->dp[k];
            s->ur[m] = s->ur[k]; s->ut[m] = s->ut[k]; s->up[m] = s->up[k];
            s->w[m] = s->w[k]; s->id[m] = s->id[k];
        }
        ++m;
    }
    s->n = m;
    free(del);
    return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* The step.  reading of the loop order (the paper states only that B */
/* lags E by half a step and that the filtered current feeds the E     */
/* update): half Faraday, particles, half Faraday, filter, Ampere,     */
/* lossy layer, injection.                                            */
/* ------------------------------------------------------------------ */

int ora_step(ora_sim *s, int32_t nsteps)
{
    if (!s || nsteps < 0) return ORA_EINVAL;
    for (int32_t q = 0; q < nsteps; ++q) {
        ora_clear_F(s);
        faraday(s, 0.5);
        int rc = push_particles(s);
        if (rc == ORA_ECFL) { set_err(s, "particle moved a cell or more in one step (CFL)"); return rc; }
        if (rc != ORA_OK) { set_err(s, "out of memory"); return rc; }
        faraday(s, 0.5);
        rc = ora_filter_F(s);
        if (rc != ORA_OK) { set_err(s, "out of memory"); return rc; }
        ampere(s);
        absorb(s);
        rc = inject(s, (double)(s->step + 1));
        if (rc != ORA_OK) { set_err(s, "out of memory"); return rc; }
        s->step++;
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* Gauss diagnostics (Sec. 2 eq. (maxti), App. B eq. (multfiltcharge)) */
/* ------------------------------------------------------------------ */

int ora_node_charge(const ora_sim *s, double x, double y, double Q, double *rho)
{
    const int i0 = (int)floor(x), j0 = cell_j(s, y);
    const double fx = x - i0, fy = y - j0;
    *fref(s, rho, 8, i0, j0) += Q * (1 - fx) * (1 - fy);
    *fref(s, rho, 8, i0 + 1, j0) += Q * fx * (1 - fy);
    *fref(s, rho, 8, i0, j0 + 1) += Q * (1 - fx) * fy;
    *fref(s, rho, 8, i0 + 1, j0 + 1) += Q * fx * fy;
    return ORA_OK;
}

int ora_gauss(const ora_sim *s, double *G, double *Q)
{
    const int nr = s->p.nr, nth = s->p.nth, g = s->g;
    const int rows = s->rows[8], cols = s->cols[8];
    double *rho = (double *)calloc((size_t)rows * cols, sizeof(double));
    if (!rho) return ORA_ENOMEM;
    for (int64_t k = 0; k < s->n; ++k) ora_node_charge(s, s->x[k], s->y[k], s->w[k], rho);
    if (filter_array(rho, rows, cols, nth, 0, s->p.n_filt) != ORA_OK) { free(rho); return ORA_ENOMEM; }
    memset(G, 0, sizeof(double) * (size_t)(nr + 1) * (nth + 1));
    for (int i = 0; i <= nr; ++i)
        for (int j = 0; j <= nth; ++j) Q[(int64_t)i * (nth + 1) + j] = rho[(int64_t)(i + g) * cols + j];
    for (int i = 1; i < nr; ++i) {
        const double ra = f_r(s, i - 0.5), rb = f_r(s, i + 0.5);
        for (int j = 0; j <= nth; ++j) {
            const double lo = j == 0 ? 1.0 : cos_th(s, j - 0.5);
            const double hi = j == nth ? -1.0 : cos_th(s, j + 0.5);
            double flux = ER(i, j) * dA_tp(rb, lo, hi) - ER(i - 1, j) * dA_tp(ra, lo, hi);
            if (j < nth) flux += ETH(i, j) * dA_rp(ra, rb, sin_th(s, j + 0.5));
            if (j > 0) flux -= ETH(i, j - 1) * dA_rp(ra, rb, sin_th(s, j - 0.5));
            G[(int64_t)i * (nth + 1) + j] = flux;
        }
    }
    free(rho);
    return ORA_OK;
}

/* Spindown luminosity (Sec. 5.4, Fig. 8d: the Poynting flux integrated
 * over a sphere).  reading: through the sphere of each radial half-node
 * rbar_i = r(i + 1/2), i = 0..nr-1, with the total fields -- the plasma
 * field plus the analytic initial field at the current time -- at the cell
 * centres (i + 1/2, j + 1/2): E_theta the mean of its two radial nodes,
 * E_phi of its four corners, B_theta of its two meridional nodes, B_phi at
 * its own point.  Each cell contributes c (E_theta B_phi - E_phi B_theta)
 * times its face on the sphere, 2 pi rbar^2 (cos theta_j - cos theta_j+1)
 * (Lorentz-Heaviside units: S = c E x B). */
int ora_poynting(const ora_sim *s, double *L)
{
    const int nr = s->p.nr, nth = s->p.nth;
    const double t = (double)s->step;
    for (int i = 0; i < nr; ++i) {
        const double x = i + 0.5, r = f_r(s, x);
        double sum = 0.0;
        for (int j = 0; j < nth; ++j) {
            const double y = j + 0.5;
            double Eb[3], Bb[3];
            background_at(s, x, r, cos_th(s, y), sin_th(s, y), t, Eb, Bb);
            const double eth = 0.5 * (ETH(i, j) + ETH(i + 1, j)) + Eb[1];
            const double eph = 0.25 * (EPH(i, j) + EPH(i + 1, j) + EPH(i, j + 1) + EPH(i + 1, j + 1)) + Eb[2];
            const double bth = 0.5 * (BTH(i, j) + BTH(i, j + 1)) + Bb[1];
            const double bph = BPH(i, j) + Bb[2];
            sum += (eth * bph - eph * bth) * 2.0 * PI * r * r * (cos_th(s, j) - cos_th(s, j + 1));
        }
        L[i] = s->p.c * sum;
    }
    return ORA_OK;
}

/* geometry tables for the pin tests:
 * 0: r_i (nr+1)   1: rbar_i (nr)   2: cos theta_j (nth+1)   3: theta_j (nth+1)
 * 4: dual face area of node j on the inner conductor, dA_tp(r_in, ...) (nth+1)
 * 5: dual cell volume of node (i, j), i = 1..nr-1 (rows 0 and nr zero),
 *    (nr+1)*(nth+1) */
int ora_geometry(const ora_sim *s, int which, double *out)
{
    const int nr = s->p.nr, nth = s->p.nth;
    switch (which) {
    case 0: for (int i = 0; i <= nr; ++i) out[i] = f_r(s, i); return ORA_OK;
    case 1: for (int i = 0; i < nr; ++i) out[i] = f_r(s, i + 0.5); return ORA_OK;
    case 2: for (int j = 0; j <= nth; ++j) out[j] = cos_th(s, j); return ORA_OK;
    case 3: for (int j = 0; j <= nth; ++j) out[j] = f_th(s, j); return ORA_OK;
    case 4:
        for (int j = 0; j <= nth; ++j) {
            const double lo = j == 0 ? 1.0 : cos_th(s, j - 0.5);
            const double hi = j == nth ? -1.0 : cos_th(s, j + 0.5);
            out[j] = dA_tp(s->p.r_in, lo, hi);
        }
        return ORA_OK;
    case 5:
        memset(out, 0, sizeof(double) * (size_t)(nr + 1) * (nth + 1));
        for (int i = 1; i < nr; ++i) {
            const double ra = f_r(s, i - 0.5), rb = f_r(s, i + 0.5);
            for (int j = 0; j <= nth; ++j) {
                const double lo = j == 0 ? 1.0 : cos_th(s, j - 0.5);
                const double hi = j == nth ? -1.0 : cos_th(s, j + 0.5);
                out[(int64_t)i * (nth + 1) + j] = 2.0 * PI / 3.0 * (rb * rb * rb - ra * ra * ra) * (lo - hi);
            }
        }
        return ORA_OK;
    default: return ORA_EINVAL;
    }
}
