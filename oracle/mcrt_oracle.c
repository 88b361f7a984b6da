/*
 * mcrt_oracle.c - plain FP64 CPU oracle (test infrastructure; see header).
 *
 * The transport follows sect. 2 of Heymann & Siebenmorgen step by step:
 * equal-energy packets (sect. 2, Eq. 1), isotropic emission, optical depth
 * per cell (Eq. 2) against -ln(zeta) with the interaction point of Eq. 3,
 * albedo split, Henyey-Greenstein scattering (Eq. 15), absorption with
 * re-emission from Eq. 5 (iterative scheme) or Eq. 10 (Bjorkman & Wood),
 * temperatures from Eq. 4, Lucy's path-length estimator in thin cells
 * (sect. 3.1, Eq. 9), a modified random walk in very thick cells (sect. 3.2),
 * the PAH two-stage emission (sect. 2.1, Eqs. 6-7), photon counting for the
 * SED and the ray-tracer of sect. 4 (Eqs. 11-17) with its adjoint.
 *
 * Readings of points the paper leaves open are documented at each function.
 * Compiled with -ffp-contract=off: every product and sum is rounded as written.
 */
#include "mcrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define H_PL 6.62607015e-27  /* erg s (exact SI definition) */
#define C_LI 2.99792458e10   /* cm/s */
#define K_BO 1.380649e-16    /* erg/K */
#define PI_D 3.14159265358979323846
#define T_FLOOR 10.0         /* K: emission temperature of a cell with T = 0 */
#define T_MAX 1.0e5          /* K: upper end of the Eq. 4 search */

/* ------------------------------------------------------------------ RNG */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ((x >> 8) + 1/2) 2^-24: exactly representable, strictly inside (0, 1). */
double orc_u24(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

/* Per-packet stream. key = seed; counter = (draw block, pid low 32 bits,
 * pid bits 32..47 | iteration << 16, model << 8 | stream tag). Draw d uses
 * block d >> 2, word d & 3. */
typedef struct {
  uint32_t key[2], c1, c2, c3;
  uint64_t d, blk;
  uint32_t buf[4];
} rng_t;

static void rng_init(rng_t *r, uint64_t seed, uint64_t pid, uint32_t iter,
                     uint32_t model, uint32_t tag) {
  r->key[0] = (uint32_t)seed;
  r->key[1] = (uint32_t)(seed >> 32);
  r->c1 = (uint32_t)pid;
  r->c2 = ((uint32_t)(pid >> 32) & 0xFFFFu) | (iter << 16);
  r->c3 = (model << 8) | (tag & 0xFFu);
  r->d = 0;
  r->blk = UINT64_MAX;
}

static double rng_next(rng_t *r) {
  uint64_t b = r->d >> 2;
  if (b != r->blk) {
    uint32_t ctr[4] = {(uint32_t)b, r->c1, r->c2, r->c3};
    orc_philox4x32_10(ctr, r->key, r->buf);
    r->blk = b;
  }
  double u = orc_u24(r->buf[r->d & 3]);
  r->d++;
  return u;
}

double orc_draw(uint64_t seed, uint64_t pid, uint32_t iter, uint32_t model,
                uint32_t tag, uint64_t d) {
  rng_t r;
  rng_init(&r, seed, pid, iter, model, tag);
  r.d = d;
  return rng_next(&r);
}

/* ------------------------------------------------- frequency quadrature */

/* nu_j = c / lambda_j. Bin j spans the geometric midpoints of its neighbours,
 * end bins extend by half a logarithmic step; w_j is the bin width in Hz
 * (the Delta nu of sect. 2). Every frequency integral of the paper (Eqs. 4,
 * 5, 7, 10) is read as sum_j w_j f(nu_j). */
void orc_freq_grid(int nl, const double *lam, double *nu, double *w) {
  for (int j = 0; j < nl; j++) nu[j] = C_LI / (lam[j] * 1e-4);
  for (int j = 0; j < nl; j++) {
    double lo = (j == 0) ? lam[0] * sqrt(lam[0] / lam[1]) : sqrt(lam[j - 1] * lam[j]);
    double hi = (j == nl - 1) ? lam[nl - 1] * sqrt(lam[nl - 1] / lam[nl - 2])
                              : sqrt(lam[j] * lam[j + 1]);
    w[j] = C_LI / (lo * 1e-4) - C_LI / (hi * 1e-4);
  }
}

/* Planck function B_nu(T) [erg/s/cm^2/Hz/sr]; 0 when h nu / kT > 700. */
double orc_planck(double nu, double T) {
  if (!(T > 0.0)) return 0.0;
  double x = H_PL * nu / (K_BO * T);
  if (x > 700.0) return 0.0;
  return 2.0 * H_PL * nu * nu * nu / (C_LI * C_LI) / expm1(x);
}

/* dB_nu/dT = B (x/T) e^x/(e^x - 1) = B (x/T)(1 + 1/(e^x - 1)). */
double orc_dplanck_dT(double nu, double T) {
  if (!(T > 0.0)) return 0.0;
  double x = H_PL * nu / (K_BO * T);
  if (x > 700.0) return 0.0;
  double em = expm1(x);
  double B = 2.0 * H_PL * nu * nu * nu / (C_LI * C_LI) / em;
  return B * (x / T) * (1.0 + 1.0 / em);
}

/* Model tables derived once per call: quadrature, mixture opacities,
 * albedo, source spectra. Nothing here reorders the method's arithmetic. */
typedef struct {
  const orc_model *m;
  int nl, ns;
  int64_t ncell;
  double V;
  double *nu, *w;
  double *kabs_mix, *ksca_mix, *kext, *alb, kext_max;
  double *ksca_eff, *g_eff; /* [ns][nl] scattering opacity and asymmetry as transported:
                               the model's, or (1 - g) kappa_sca and 0 under the
                               g-factor approximation */
  double *lucy_frac;  /* [ns][nl] f_s kabs_s / kabs_mix */
  double *lnu;        /* [nsrc][nl] L_nu,s,j erg/s/Hz */
  double *src_f;      /* [nsrc][nl] w_j L_nu,s,j */
  double ltot;
  int *imgmap;        /* [nl] -> imaged index or -1 */
  double (*kv)[3];    /* view directions toward the observer */
} tab_t;

static double sum_desc(const double *f, int n) {
  double t = 0.0;
  for (int j = n - 1; j >= 0; j--) t += f[j];
  return t;
}

static int tab_init(tab_t *t, const orc_model *m) {
  memset(t, 0, sizeof(*t));
  t->m = m;
  int nl = m->nl, ns = m->ns;
  t->nl = nl;
  t->ns = ns;
  t->ncell = orc_nleaf(m); /* leaves: every per-cell array runs over them */
  t->V = m->dcell * m->dcell * m->dcell;
  t->nu = malloc(sizeof(double) * nl);
  t->w = malloc(sizeof(double) * nl);
  t->kabs_mix = malloc(sizeof(double) * nl);
  t->ksca_mix = malloc(sizeof(double) * nl);
  t->kext = malloc(sizeof(double) * nl);
  t->alb = malloc(sizeof(double) * nl);
  t->lucy_frac = malloc(sizeof(double) * nl * ns);
  t->lnu = malloc(sizeof(double) * nl * (m->nsrc > 0 ? m->nsrc : 1));
  t->src_f = malloc(sizeof(double) * nl * (m->nsrc > 0 ? m->nsrc : 1));
  t->imgmap = malloc(sizeof(int) * nl);
  t->kv = malloc(sizeof(double[3]) * (m->nview > 0 ? m->nview : 1));
  t->ksca_eff = malloc(sizeof(double) * nl * ns);
  t->g_eff = malloc(sizeof(double) * nl * ns);
  for (int i = 0; i < nl * ns; i++) {
    t->ksca_eff[i] = m->scat_law == 1 ? (1.0 - m->g[i]) * m->ksca[i] : m->ksca[i];
    t->g_eff[i] = m->scat_law == 1 ? 0.0 : m->g[i];
  }
  orc_freq_grid(nl, m->lam_um, t->nu, t->w);
  t->kext_max = 0.0;
  for (int j = 0; j < nl; j++) {
    double a = 0.0, s = 0.0;
    for (int q = 0; q < ns; q++) {
      a += m->mass_frac[q] * m->kabs[q * nl + j];
      s += m->mass_frac[q] * t->ksca_eff[q * nl + j];
    }
    t->kabs_mix[j] = a;
    t->ksca_mix[j] = s;
    t->kext[j] = a + s;
    t->alb[j] = (a + s > 0.0) ? s / (a + s) : 0.0;
    if (t->kext[j] > t->kext_max) t->kext_max = t->kext[j];
    for (int q = 0; q < ns; q++)
      t->lucy_frac[q * nl + j] = (a > 0.0) ? m->mass_frac[q] * m->kabs[q * nl + j] / a : 0.0;
  }
  t->ltot = 0.0;
  double *f = malloc(sizeof(double) * nl);
  for (int s = 0; s < m->nsrc; s++) {
    for (int j = 0; j < nl; j++) {
      double shape = m->src_shape ? m->src_shape[s * nl + j] : orc_planck(t->nu[j], m->src_tbb[s]);
      f[j] = t->w[j] * shape;
    }
    double norm = sum_desc(f, nl);
    for (int j = 0; j < nl; j++) {
      double shape = m->src_shape ? m->src_shape[s * nl + j] : orc_planck(t->nu[j], m->src_tbb[s]);
      t->lnu[s * nl + j] = m->src_lum[s] * shape / norm;
      t->src_f[s * nl + j] = t->w[j] * t->lnu[s * nl + j];
    }
    t->ltot += m->src_lum[s];
  }
  free(f);
  for (int j = 0; j < nl; j++) t->imgmap[j] = -1;
  for (int q = 0; q < m->nimg; q++) t->imgmap[m->img_idx[q]] = q;
  for (int v = 0; v < m->nview; v++) {
    double th = m->view_deg[2 * v] * PI_D / 180.0, ph = m->view_deg[2 * v + 1] * PI_D / 180.0;
    t->kv[v][0] = sin(th) * cos(ph);
    t->kv[v][1] = sin(th) * sin(ph);
    t->kv[v][2] = cos(th);
  }
  return 0;
}

static void tab_free(tab_t *t) {
  free(t->nu); free(t->w); free(t->kabs_mix); free(t->ksca_mix); free(t->kext);
  free(t->alb); free(t->lucy_frac); free(t->lnu); free(t->src_f); free(t->imgmap);
  free(t->ksca_eff); free(t->g_eff);
  free(t->kv);
}

/* Phi_s(T) = sum_j w_j kabs_s,j B_j(T), summed in ascending frequency. */
static double phi_t(const tab_t *t, int s, double T) {
  double sum = 0.0;
  for (int j = t->nl - 1; j >= 0; j--)
    sum += t->w[j] * t->m->kabs[s * t->nl + j] * orc_planck(t->nu[j], T);
  return sum;
}

double orc_phi(const orc_model *m, int s, double T) {
  tab_t t;
  tab_init(&t, m);
  double r = phi_t(&t, s, T);
  tab_free(&t);
  return r;
}

/* Eq. 4: the T with Phi_s(T) = rhs, by bisection on [0, T_MAX] down to a
 * relative bracket of 1e-13. rhs <= 0 gives 0; rhs above Phi(T_MAX) clamps. */
static double invert_t(const tab_t *t, int s, double rhs, int *clamped) {
  if (!(rhs > 0.0)) return 0.0;
  double lo = 0.0, hi = T_MAX;
  if (phi_t(t, s, hi) <= rhs) {
    if (clamped) *clamped = 1;
    return hi;
  }
  for (int it = 0; it < 400; it++) {
    double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (phi_t(t, s, mid) < rhs) lo = mid; else hi = mid;
    if (hi - lo <= 1e-13 * hi) break;
  }
  return 0.5 * (lo + hi);
}

double orc_invert_T(const orc_model *m, int s, double rhs) {
  tab_t t;
  tab_init(&t, m);
  double r = invert_t(&t, s, rhs, NULL);
  tab_free(&t);
  return r;
}

/* Henyey-Greenstein: inverse of the cumulative distribution of cos(beta). */
double orc_hg_mu(double g, double u) {
  if (fabs(g) < 1e-6) return 2.0 * u - 1.0;
  double q = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
  double mu = (1.0 + g * g - q * q) / (2.0 * g);
  if (mu > 1.0) mu = 1.0;
  if (mu < -1.0) mu = -1.0;
  return mu;
}

/* Eq. 15 per steradian. */
double orc_hg_phase(double g, double mu) {
  double den = 1.0 + g * g - 2.0 * g * mu;
  return (1.0 - g * g) / (4.0 * PI_D * den * sqrt(den));
}

/* Real orthonormal spherical harmonics by the associated-Legendre recurrence
 * in x = cos(theta) without the sin^m factor (Q_l^m), the azimuthal terms
 * from (d_x + i d_y)^m = sin^m(theta) e^{i m phi}:
 *   Q_m^m = (2m-1)!!, Q_{m+1}^m = (2m+1) x Q_m^m,
 *   (l-m) Q_l^m = (2l-1) x Q_{l-1}^m - (l+m-1) Q_{l-2}^m,
 *   Y_l0 = N_l0 Q_l^0, Y_l,+-m = sqrt(2) N_lm Q_l^m (Re, Im)(d_x + i d_y)^m,
 *   N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). */
void orc_ylm(int lmax, const double d[3], double *y) {
  double x = d[2];
  double cr = 1.0, ci = 0.0; /* (d_x + i d_y)^m */
  double qmm = 1.0;          /* Q_m^m */
  for (int m = 0; m <= lmax; m++) {
    if (m > 0) {
      double nr = cr * d[0] - ci * d[1], ni = cr * d[1] + ci * d[0];
      cr = nr;
      ci = ni;
      qmm *= (double)(2 * m - 1);
    }
    double q2 = 0.0, q1 = qmm; /* Q_{l-2}^m, Q_{l-1}^m */
    for (int l = m; l <= lmax; l++) {
      double q;
      if (l == m) q = qmm;
      else if (l == m + 1) q = (double)(2 * m + 1) * x * qmm;
      else q = ((double)(2 * l - 1) * x * q1 - (double)(l + m - 1) * q2) / (double)(l - m);
      if (l > m) {
        q2 = q1;
        q1 = q;
      }
      /* (l-m)!/(l+m)! */
      double ratio = 1.0;
      for (int k = l - m + 1; k <= l + m; k++) ratio /= (double)k;
      double n = sqrt((2.0 * l + 1.0) / (4.0 * PI_D) * ratio);
      if (m == 0) {
        y[l * l + l] = n * q;
      } else {
        y[l * l + l + m] = sqrt(2.0) * n * q * cr;
        y[l * l + l - m] = sqrt(2.0) * n * q * ci;
      }
    }
  }
}

void orc_sh_view_sums(const orc_model *m, int sh_order, const double *sh, const double k[3],
                      double *out) {
  int lmax = sh_order - 1, nlm = sh_order * sh_order;
  int64_t nc = orc_nleaf(m);
  double *y = malloc(sizeof(double) * nlm);
  orc_ylm(lmax, k, y);
  for (int q = 0; q < m->nimg; q++)
    for (int64_t c = 0; c < nc; c++) {
      double s = 0.0;
      for (int i = 0; i < nlm; i++) s += y[i] * sh[((int64_t)q * nlm + i) * nc + c];
      out[(int64_t)q * nc + c] = s;
    }
  free(y);
}

/* Survival probability of a diffusing packet started at the centre of a
 * sphere: S = 2 sum_{n>=1} (-1)^{n+1} y^{n^2}, y = exp(-pi^2 D t / R^2). */
double orc_mrw_survival(double y) {
  if (!(y > 0.0)) return 0.0;
  if (y >= 1.0) return 1.0;
  double ly = log(y), sum = 0.0;
  for (int n = 1; n <= 10000; n++) {
    double term = exp((double)n * (double)n * ly);
    sum += (n & 1) ? term : -term;
    if (term < 1e-17 * fabs(sum)) break;
  }
  return 2.0 * sum;
}

static double mrw_dsurv(double y) {
  double ly = log(y), sum = 0.0;
  for (int n = 1; n <= 10000; n++) {
    double nn = (double)n * (double)n;
    double term = nn * exp((nn - 1.0) * ly);
    sum += (n & 1) ? term : -term;
    if (term < 1e-17 * fabs(sum)) break;
  }
  return 2.0 * sum;
}

/* y in (0,1) with S(y) = u: Newton inside a shrinking bracket, bisection
 * whenever Newton leaves it; stops at |dy| <= 1e-15 y. */
double orc_mrw_solve(double u) {
  double lo = 0.0, hi = 1.0, y = 0.5 * u;
  if (!(y > 0.0)) y = 1e-300;
  for (int it = 0; it < 200; it++) {
    double f = orc_mrw_survival(y) - u;
    if (f > 0.0) hi = y; else lo = y;
    double df = mrw_dsurv(y);
    double yn = (df > 0.0) ? y - f / df : 0.5 * (lo + hi);
    if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
    if (fabs(yn - y) <= 1e-15 * y) { y = yn; break; }
    y = yn;
  }
  return y;
}

/* ------------------------------------------------------------ geometry */

static int64_t cidx(const orc_model *m, const int c[3]) {
  return ((int64_t)c[2] * m->ny + c[1]) * m->nx + c[0];
}

static int inside(const orc_model *m, const int c[3]) {
  return c[0] >= 0 && c[0] < m->nx && c[1] >= 0 && c[1] < m->ny && c[2] >= 0 && c[2] < m->nz;
}

/* Cell holding p; a point exactly on a face belongs to the cell that the
 * direction d points into. */
static void start_cell(const orc_model *m, const double p[3], const double d[3], int c[3]) {
  for (int k = 0; k < 3; k++) {
    double q = (p[k] - m->origin[k]) / m->dcell;
    double f = floor(q);
    int ci = (int)f;
    if (q == f && d[k] < 0.0) ci -= 1;
    c[k] = ci;
  }
}

/* distance along d from p0 to the exit plane of cell c on axis k */
static double plane_t(const orc_model *m, const double p0[3], const double d[3],
                      const int c[3], int k) {
  if (d[k] > 0.0) return (m->origin[k] + (double)(c[k] + 1) * m->dcell - p0[k]) / d[k];
  if (d[k] < 0.0) return (m->origin[k] + (double)c[k] * m->dcell - p0[k]) / d[k];
  return INFINITY;
}

static void upd_margin(double *mm, double v) {
  if (v < *mm) *mm = v;
}

/* ----------------------------------------------- leaves (one refinement level) */

static int64_t n_cubes(const orc_model *m) { return (int64_t)m->nx * m->ny * m->nz; }

int64_t orc_nleaf(const orc_model *m) { return n_cubes(m) + (m->ref ? m->nsub : 0); }

/* sub-cubes per edge of cube cc (1: whole) */
static int cube_r(const orc_model *m, int64_t cc) {
  if (!m->ref) return 1;
  int r = m->ref[cc];
  return r > 1 ? r : 1;
}

/* leaf of sub-cube f of cube c (f = 0 for a whole cube) */
static int64_t leaf_id(const orc_model *m, const int c[3], const int f[3]) {
  int64_t cc = cidx(m, c);
  int r = cube_r(m, cc);
  if (r == 1) return cc;
  return n_cubes(m) + m->sub_off[cc] + ((int64_t)f[2] * r + f[1]) * r + f[0];
}

static double leaf_rho(const orc_model *m, int64_t leaf) {
  int64_t nc = n_cubes(m);
  return leaf < nc ? m->rho[leaf] : m->rho_sub[leaf - nc];
}

/* position of face e (0..r) of the sub-cubes of cube coordinate ck on axis
 * k: the cube's own faces are written as for a whole cube, so a walk leaves
 * a divided cube exactly where the coarse grid puts that face */
static double face_pos(const orc_model *m, int k, int ck, int r, int e) {
  if (e == 0) return m->origin[k] + (double)ck * m->dcell;
  if (e == r) return m->origin[k] + (double)(ck + 1) * m->dcell;
  return m->origin[k] + (double)ck * m->dcell + (double)e * (m->dcell / (double)r);
}

/* sub-cube index on axis k of point x inside cube coordinate ck (a point on
 * a face belongs to the sub-cube d points into), clamped to the cube */
static int sub_index(const orc_model *m, int k, int ck, int r, double x, double dk) {
  if (r == 1) return 0;
  double q = (x - m->origin[k] - (double)ck * m->dcell) / (m->dcell / (double)r);
  double fl = floor(q);
  int fi = (int)fl;
  if (q == fl && dk < 0.0) fi -= 1;
  if (fi < 0) fi = 0;
  if (fi > r - 1) fi = r - 1;
  return fi;
}

/* cube c, sub-cube f and sub-cubes per edge r of a leaf */
static void leaf_loc(const orc_model *m, int64_t leaf, int c[3], int f[3], int *r_out) {
  int64_t nc = n_cubes(m);
  int64_t cc = leaf;
  int r = 1;
  f[0] = f[1] = f[2] = 0;
  if (leaf >= nc) {
    /* sub_off is the exclusive prefix sum of r^3 over the divided cubes, so
     * the cube holding sub-cube s is the last cube with sub_off <= s */
    int64_t s = leaf - nc, lo = 0, hi = nc - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) / 2;
      if (m->sub_off[mid] <= s) lo = mid; else hi = mid - 1;
    }
    cc = lo;
    r = cube_r(m, cc);
    int64_t loc = s - m->sub_off[cc];
    f[0] = (int)(loc % r);
    f[1] = (int)((loc / r) % r);
    f[2] = (int)(loc / ((int64_t)r * r));
  }
  c[0] = (int)(cc % m->nx);
  c[1] = (int)((cc / m->nx) % m->ny);
  c[2] = (int)(cc / ((int64_t)m->nx * m->ny));
  *r_out = r;
}

void orc_leaf_box(const orc_model *m, int64_t leaf, double lo[3], double *h, double *rho) {
  int c[3], f[3], r;
  leaf_loc(m, leaf, c, f, &r);
  for (int k = 0; k < 3; k++) lo[k] = face_pos(m, k, c[k], r, f[k]);
  *h = (r == 1) ? m->dcell : m->dcell / (double)r;
  *rho = leaf_rho(m, leaf);
}

/* A voxel walk through the leaves along p0 + t d (Amanatides & Woo on each
 * cube's own lattice): tm[k] is the distance to the current leaf's next face
 * on axis k; leaving a divided cube continues on the next cube's lattice.
 * Whole cubes take the same arithmetic as an undivided grid. */
typedef struct {
  const orc_model *m;
  const double *p0, *d;
  int c[3], f[3], r;
  double tm[3];
} walker_t;

static void walker_faces(walker_t *W) {
  for (int k = 0; k < 3; k++) {
    double dk = W->d[k];
    if (dk > 0.0) W->tm[k] = (face_pos(W->m, k, W->c[k], W->r, W->f[k] + 1) - W->p0[k]) / dk;
    else if (dk < 0.0) W->tm[k] = (face_pos(W->m, k, W->c[k], W->r, W->f[k]) - W->p0[k]) / dk;
    else W->tm[k] = INFINITY;
  }
}

/* enter cube W->c at distance t (entry axis a, or -1 inside a flight start)
 * with sub-cube indices from the position (f given: used as is) */
static void walker_enter(walker_t *W, double t, int a, const int *f) {
  W->r = cube_r(W->m, cidx(W->m, W->c));
  for (int k = 0; k < 3; k++) {
    if (f) W->f[k] = f[k];
    else if (k == a) W->f[k] = (W->d[k] > 0.0) ? 0 : W->r - 1;
    else W->f[k] = sub_index(W->m, k, W->c[k], W->r, W->p0[k] + t * W->d[k], W->d[k]);
  }
  walker_faces(W);
}

static int64_t walker_leaf(const walker_t *W) { return leaf_id(W->m, W->c, W->f); }

/* step across the face on axis a reached at distance t: 1 when the walk
 * leaves the grid */
static int walker_cross(walker_t *W, int a, double t) {
  const orc_model *m = W->m;
  int s = (W->d[a] > 0.0) ? 1 : -1;
  W->f[a] += s;
  if (W->f[a] >= 0 && W->f[a] < W->r) {
    double dk = W->d[a];
    W->tm[a] = (face_pos(m, a, W->c[a], W->r, dk > 0.0 ? W->f[a] + 1 : W->f[a]) - W->p0[a]) / dk;
    return 0;
  }
  W->c[a] += s;
  int n[3] = {m->nx, m->ny, m->nz};
  if (W->c[a] < 0 || W->c[a] >= n[a]) return 1;
  walker_enter(W, t, a, NULL);
  return 0;
}

/* Amanatides & Woo stepping: the smallest exit time wins, ties step the
 * lowest axis first (x < y < z); segment lengths are never negative. */
int orc_dda(const orc_model *m, const double p0[3], const double d[3], int maxseg,
            int64_t *cells, double *lens) {
  walker_t W = {m, p0, d, {0, 0, 0}, {0, 0, 0}, 1, {0, 0, 0}};
  start_cell(m, p0, d, W.c);
  int nseg = 0;
  if (!inside(m, W.c)) return 0;
  walker_enter(&W, 0.0, -1, NULL);
  double t = 0.0;
  for (;;) {
    int a = 0;
    if (W.tm[1] < W.tm[a]) a = 1;
    if (W.tm[2] < W.tm[a]) a = 2;
    double ell = W.tm[a] - t;
    if (ell < 0.0) ell = 0.0;
    if (nseg >= maxseg) return -1;
    cells[nseg] = walker_leaf(&W);
    lens[nseg] = ell;
    nseg++;
    t = W.tm[a] > t ? W.tm[a] : t;
    if (walker_cross(&W, a, t)) return nseg;
  }
}

static void iso_dir(double uphi, double umu, double d[3]) {
  double phi = 2.0 * PI_D * uphi;
  double mu = 1.0 - 2.0 * umu;
  double s = sqrt(fmax(0.0, 1.0 - mu * mu));
  d[0] = s * cos(phi);
  d[1] = s * sin(phi);
  d[2] = mu;
}

/* New direction at polar angle acos(mu), azimuth phi about d (direction
 * cosines); polar special case near |d_z| = 1; renormalised. */
static void rotate_dir(double d[3], double mu, double phi) {
  double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  double cp = cos(phi), sp = sin(phi);
  double nx, ny, nz;
  if (fabs(d[2]) > 1.0 - 1e-10) {
    nx = st * cp;
    ny = st * sp;
    nz = (d[2] > 0.0) ? mu : -mu;
  } else {
    double s = sqrt(1.0 - d[2] * d[2]);
    nx = st * (d[0] * d[2] * cp - d[1] * sp) / s + d[0] * mu;
    ny = st * (d[1] * d[2] * cp + d[0] * sp) / s + d[1] * mu;
    nz = -st * cp * s + d[2] * mu;
  }
  double nn = sqrt(nx * nx + ny * ny + nz * nz);
  d[0] = nx / nn;
  d[1] = ny / nn;
  d[2] = nz / nn;
}

/* Inverse CDF over ascending frequency (descending index): the first bin,
 * counted from nu = 0, whose running sum reaches u times the total
 * ("shortest frequency" of Eqs. 5, 7, 10). */
static int pick_desc(const double *f, int n, double u, double *mm) {
  double tot = sum_desc(f, n);
  double target = u * tot, c = 0.0;
  for (int j = n - 1; j >= 0; j--) {
    double prev = c;
    c += f[j];
    if (c >= target) {
      if (tot > 0.0) {
        upd_margin(mm, (c - target) / tot);
        upd_margin(mm, (target - prev) / tot);
      }
      return j;
    }
  }
  return 0;
}

/* Smallest index whose running sum (ascending) reaches u times the total. */
static int pick_asc(const double *f, int n, double u, double *mm) {
  double tot = 0.0;
  for (int q = 0; q < n; q++) tot += f[q];
  double target = u * tot, c = 0.0;
  for (int q = 0; q < n; q++) {
    double prev = c;
    c += f[q];
    if (c >= target) {
      if (tot > 0.0 && n > 1) {
        upd_margin(mm, (c - target) / tot);
        upd_margin(mm, (target - prev) / tot);
      }
      return q;
    }
  }
  return n - 1;
}

/* ------------------------------------------------------------ transport */

typedef struct {
  const orc_model *m;
  const orc_opts *o;
  tab_t t;
  orc_state *st;
  double xi;
  uint64_t seed;
  uint32_t iter, tag;
  int pass;           /* 1: source + pass 1, 2: PAH re-emission pass */
  double *f;          /* scratch [nl] */
  double *fs;         /* scratch [ns] */
  /* entries (s, cell) whose energy changed or whose epoch temperature was
   * formed since the last epoch start: the only ones an epoch snapshot can
   * change (bookkeeping only; the snapshot's values are those of a sweep
   * over every entry) */
  int64_t *touched;
  uint8_t *is_touched;
  int64_t n_touched;
} run_t;

typedef struct {
  double p[3], d[3];
  int c[3];   /* cube */
  int f[3];   /* sub-cube of a divided cube (0 in a whole cube) */
  int j, status;
  uint64_t n_cross, n_scat, n_abs, n_mrw, n_lucy, n_int;
  double mm;
} pkt_t;

/* Lucy's thin-cell test on the cell's face-to-face depth (edge h) */
static int is_thin(const run_t *R, double rho, double h) {
  return R->o->lucy_tau > 0.0 && rho > 0.0 && rho * R->t.kext_max * h < R->o->lucy_tau;
}

/* edge and volume of the leaf of packet P */
static double pkt_h(const run_t *R, const pkt_t *P) {
  int r = cube_r(R->m, cidx(R->m, P->c));
  return r == 1 ? R->m->dcell : R->m->dcell / (double)r;
}

static double leaf_V(const run_t *R, int64_t leaf) {
  if (leaf < n_cubes(R->m)) return R->t.V;
  double lo[3], h, rho;
  orc_leaf_box(R->m, leaf, lo, &h, &rho);
  return h * h * h;
}

static void touch(run_t *R, int64_t q) {
  if (R->is_touched && !R->is_touched[q]) {
    R->is_touched[q] = 1;
    R->touched[R->n_touched++] = q;
  }
}

static double e_cell(const run_t *R, int s, int64_t c) {
  int64_t q = (int64_t)s * R->t.ncell + c;
  return (double)R->st->k[q] * R->xi + R->st->epath[q];
}

/* Emission temperature of species s in cell c for the current mode:
 * FROZEN - the previous iteration's T (T_FLOOR when it is 0);
 * BW_EPOCH - Eq. 4 with one more packet on top of the energy held at the
 * start of the epoch, i.e. the temperature after this absorption. */
static double mode_T(run_t *R, int s, int64_t c) {
  int64_t q = (int64_t)s * R->t.ncell + c;
  if (R->o->mode == ORC_FROZEN) {
    double T = R->st->T[q];
    return (T > 0.0) ? T : T_FLOOR;
  }
  if (!R->st->tvalid[q]) {
    double rho = leaf_rho(R->m, c);
    double rhs = (R->st->esnap[q] + R->xi) / (4.0 * PI_D * R->m->mass_frac[s] * rho * leaf_V(R, c));
    int cl = 0;
    R->st->tt[q] = invert_t(&R->t, s, rhs, &cl);
    if (cl) R->st->st.clamped_T++;
    R->st->tvalid[q] = 1;
    touch(R, q);
  }
  return R->st->tt[q];
}

/* Lucy's estimator (Eq. 9) on one segment inside a thin cell: absorbed
 * fraction 1 - exp(-tau_abs) of the packet energy, split over the thermal
 * species by their share of kappa_abs. */
static void lucy_deposit(run_t *R, pkt_t *P, int64_t c, double rho, double ell) {
  int nl = R->t.nl, j = P->j;
  double em = -expm1(-(rho * R->t.kabs_mix[j] * ell));
  for (int s = 0; s < R->t.ns; s++) {
    if (s == R->m->pah_species) continue;
    R->st->epath[(int64_t)s * R->t.ncell + c] += R->xi * R->t.lucy_frac[s * nl + j] * em;
    touch(R, (int64_t)s * R->t.ncell + c);
  }
  P->n_lucy++;
}

/* One flight with optical depth tau_star from the current position.
 * Returns 1 when the packet leaves the grid, 0 at an interaction. With a
 * new draw per cell (the footnote to the sect. 2 interaction test) the
 * packet draws zeta on entering each cell (the flight's first cell at its
 * start point) and interacts there iff the cell's segment depth exceeds
 * -ln zeta, at distance -ln zeta / (rho kext) from where the segment
 * begins; tau_star is then unused. */
static int fly(run_t *R, pkt_t *P, double tau_star, rng_t *rg) {
  const int per_cell = R->o->tau_mode == ORC_TAU_PER_CELL;
  const orc_model *m = R->m;
  double p0[3] = {P->p[0], P->p[1], P->p[2]};
  const double *d = P->d;
  walker_t W = {m, p0, d, {P->c[0], P->c[1], P->c[2]}, {0, 0, 0}, 1, {0, 0, 0}};
  walker_enter(&W, 0.0, -1, P->f);
  double t = 0.0, tau = 0.0;
  double kx = R->t.kext[P->j];
  for (;;) {
    int a = 0;
    if (W.tm[1] < W.tm[a]) a = 1;
    if (W.tm[2] < W.tm[a]) a = 2;
    {
      /* distance of the axis choice from a tie */
      double t1 = W.tm[a], t2 = INFINITY;
      for (int k = 0; k < 3; k++)
        if (k != a && W.tm[k] < t2) t2 = W.tm[k];
      if (isfinite(t2) && t2 > 0.0) upd_margin(&P->mm, (t2 - t1) / t2);
    }
    double ell = W.tm[a] - t;
    if (ell < 0.0) ell = 0.0;
    int64_t c = walker_leaf(&W);
    double rho = leaf_rho(m, c);
    double dtau = rho * kx * ell;
    int thin = is_thin(R, rho, W.r == 1 ? m->dcell : m->dcell / (double)W.r);
    if (per_cell) {
      tau = 0.0;
      tau_star = -log(rng_next(rg));
    }
    upd_margin(&P->mm, fabs(tau + dtau - tau_star) / tau_star);
    if (tau + dtau > tau_star) {
      double tint = t + (tau_star - tau) / (rho * kx);
      if (thin) lucy_deposit(R, P, c, rho, tint - t);
      for (int k = 0; k < 3; k++) {
        P->p[k] = p0[k] + tint * d[k];
        P->c[k] = W.c[k];
        P->f[k] = W.f[k];
      }
      return 0;
    }
    if (thin) lucy_deposit(R, P, c, rho, ell);
    tau += dtau;
    if (W.tm[a] > t) t = W.tm[a];
    P->n_cross++;
    if (walker_cross(&W, a, t)) {
      for (int k = 0; k < 3; k++) {
        P->p[k] = p0[k] + t * d[k];
        P->c[k] = W.c[k];
      }
      return 1;
    }
  }
}

/* Rosseland mean of the mixture extinction at T. */
static double rosseland(const run_t *R, double T) {
  double num = 0.0, den = 0.0;
  for (int j = R->t.nl - 1; j >= 0; j--) {
    if (!(R->t.kext[j] > 0.0)) return 0.0;
    double db = R->t.w[j] * orc_dplanck_dT(R->t.nu[j], T);
    num += db;
    den += db / R->t.kext[j];
  }
  return (den > 0.0) ? num / den : 0.0;
}

/* Planck mean of species s absorption at T. */
static double planck_mean(const run_t *R, int s, double T) {
  double num = 0.0, den = 0.0;
  for (int j = R->t.nl - 1; j >= 0; j--) {
    double b = R->t.w[j] * orc_planck(R->t.nu[j], T);
    num += b * R->m->kabs[s * R->t.nl + j];
    den += b;
  }
  return (den > 0.0) ? num / den : 0.0;
}

/* The two means above for a model, at temperature T (exported for tests). */
double orc_rosseland(const orc_model *m, double T) {
  run_t R;
  memset(&R, 0, sizeof(R));
  R.m = m;
  tab_init(&R.t, m);
  double r = rosseland(&R, T);
  tab_free(&R.t);
  return r;
}

double orc_planck_mean(const orc_model *m, int s, double T) {
  run_t R;
  memset(&R, 0, sizeof(R));
  R.m = m;
  tab_init(&R.t, m);
  double r = planck_mean(&R, s, T);
  tab_free(&R.t);
  return r;
}

static int first_thermal(const run_t *R) {
  for (int s = 0; s < R->t.ns; s++)
    if (s != R->m->pah_species) return s;
  return 0;
}

/* Modified random walk (sect. 3.2; Fleck & Canfield diffusion). At the start
 * of a flight in a cell whose Rosseland-mean optical depth (face to face, at
 * the cell's emission temperature) exceeds mrw_tau, a sphere of radius R
 * (distance to the nearest face) is crossed in one step when it spans at
 * least gamma Rosseland mean free paths: the exit time follows the
 * first-passage law of the diffusion equation, the packet moves to a uniform
 * point on the sphere, deposits xi rho f_s kappa_P,s l per species along the
 * path l and leaves with a new thermal wavelength and an isotropic
 * direction. Cells with rho kext_max dcell <= mrw_tau cannot qualify and are
 * skipped before any opacity mean is formed. Returns 1 if a step was taken. */
static int mrw_step(run_t *R, pkt_t *P, rng_t *rg) {
  const orc_model *m = R->m;
  if (!(R->o->mrw_tau > 0.0)) return 0;
  int64_t c = leaf_id(m, P->c, P->f);
  double rho = leaf_rho(m, c);
  const int r = cube_r(m, cidx(m, P->c));
  const double h = r == 1 ? m->dcell : m->dcell / (double)r;
  if (!(rho > 0.0)) return 0;
  if (!(rho * R->t.kext_max * h > R->o->mrw_tau)) return 0;
  int s0 = first_thermal(R);
  double T0 = mode_T(R, s0, c);
  double kr = rosseland(R, T0);
  double taur = rho * kr * h;
  upd_margin(&P->mm, fabs(taur - R->o->mrw_tau) / R->o->mrw_tau);
  if (!(taur > R->o->mrw_tau)) return 0;
  /* sphere radius: distance to the nearest face of the packet's cell */
  double Rs = INFINITY;
  for (int k = 0; k < 3; k++) {
    double lo = P->p[k] - face_pos(m, k, P->c[k], r, P->f[k]);
    double hi = face_pos(m, k, P->c[k], r, P->f[k] + 1) - P->p[k];
    if (lo < Rs) Rs = lo;
    if (hi < Rs) Rs = hi;
  }
  if (Rs < 0.0) Rs = 0.0;
  double crit = rho * kr * Rs;
  upd_margin(&P->mm, fabs(crit - R->o->mrw_gamma) / R->o->mrw_gamma);
  if (!(crit >= R->o->mrw_gamma)) return 0;
  double ut = rng_next(rg), ups = rng_next(rg), ums = rng_next(rg);
  double ul = rng_next(rg), uph = rng_next(rg), umu = rng_next(rg);
  double y = orc_mrw_solve(ut);
  double ell = -3.0 * rho * kr * Rs * Rs * log(y) / (PI_D * PI_D);
  double ds[3];
  iso_dir(ups, ums, ds);
  for (int k = 0; k < 3; k++) P->p[k] = P->p[k] + Rs * ds[k];
  int nl = R->t.nl;
  for (int j = 0; j < nl; j++) R->f[j] = 0.0;
  for (int s = 0; s < R->t.ns; s++) {
    if (s == m->pah_species) continue;
    double Ts = mode_T(R, s, c);
    double kp = planck_mean(R, s, Ts);
    R->st->epath[(int64_t)s * R->t.ncell + c] += R->xi * rho * m->mass_frac[s] * kp * ell;
    touch(R, (int64_t)s * R->t.ncell + c);
    for (int j = 0; j < nl; j++)
      R->f[j] += R->t.w[j] * m->mass_frac[s] * m->kabs[s * nl + j] * orc_planck(R->t.nu[j], Ts);
  }
  P->j = pick_desc(R->f, nl, ul, &P->mm);
  iso_dir(uph, umu, P->d);
  P->n_mrw++;
  R->st->st.mrw_steps++;
  return 1;
}

static int pah_row(const run_t *R, int64_t c) {
  const orc_model *m = R->m;
  double rho = leaf_rho(m, c);
  double q = (double)R->st->kpah[c] * R->xi /
             (4.0 * PI_D * m->mass_frac[m->pah_species] * rho * leaf_V(R, c));
  int r = 0;
  while (r < m->n_pah_rows - 1 && q >= m->pah_edges[r]) r++;
  return r;
}

/* Photodissociation (sect. 2.1, Eq. 8). The cell's PAH absorb kpah xi erg/s
 * (pass 1) shared by its f_pah rho V / m_PAH molecules, m_PAH = N_C 12 amu
 * (carbon only); within the cooling time t_cool each molecule takes
 * E_PAH = kpah xi m_PAH t_cool / (f_pah rho V), and the molecules dissociate
 * when E_PAH >= N_C/2 eV. */
#define AMU_G 1.66053906660e-24
#define EV_ERG 1.602176634e-12
static int pah_dissociates_xi(const orc_model *m, const orc_opts *o, double xi, double V,
                              uint32_t kpah, int64_t c) {
  if (!(o->pah_nc > 0.0) || !(o->pah_tcool > 0.0) || kpah == 0) return 0;
  double rho = leaf_rho(m, c);
  double mp = o->pah_nc * 12.0 * AMU_G;
  double e = (double)kpah * xi * mp * o->pah_tcool / (m->mass_frac[m->pah_species] * rho * V);
  return e >= 0.5 * o->pah_nc * EV_ERG;
}

int orc_pah_dissociates(const orc_model *m, const orc_opts *o, uint32_t kpah, int64_t c) {
  double ltot = 0.0;
  for (int s = 0; s < m->nsrc; s++) ltot += m->src_lum[s];
  double lo[3], h, rho;
  orc_leaf_box(m, c, lo, &h, &rho);
  double V = (c < n_cubes(m)) ? m->dcell * m->dcell * m->dcell : h * h * h;
  return pah_dissociates_xi(m, o, ltot / (double)o->n_total, V, kpah, c);
}

static int pick_pah_lambda(run_t *R, int row, double u, double *mm) {
  int nl = R->t.nl;
  for (int j = 0; j < nl; j++) R->f[j] = R->t.w[j] * R->m->pah_emis[row * nl + j];
  return pick_desc(R->f, nl, u, mm);
}

static void finish(run_t *R, pkt_t *P, uint64_t pid, uint64_t slot) {
  orc_state *st = R->st;
  st->st.crossings += P->n_cross;
  if (P->status == ORC_ESCAPED) {
    st->st.escaped++;
    int nt = R->o->ntheta > 0 ? R->o->ntheta : 1;
    double x = (P->d[2] + 1.0) * 0.5 * (double)nt;
    int b = (int)floor(x);
    if (b < 0) b = 0;
    if (b >= nt) b = nt - 1;
    if (nt > 1) upd_margin(&P->mm, fabs(x - floor(x + 0.5)) / (double)nt);
    st->sed[(int64_t)b * R->t.nl + P->j] += 1;
  } else if (P->status == ORC_KILLED) {
    st->st.killed++;
  } else if (P->status == ORC_PAH_STOP) {
    st->st.pah_stopped++;
  }
  if (R->o->record && st->rec) {
    orc_record *r = &st->rec[slot];
    r->pid = pid;
    for (int k = 0; k < 3; k++) { r->pos[k] = P->p[k]; r->dir[k] = P->d[k]; }
    r->j = P->j;
    r->status = P->status;
    r->weight = R->xi;
    r->n_cross = P->n_cross;
    r->n_scat = P->n_scat;
    r->n_abs = P->n_abs;
    r->n_mrw = P->n_mrw;
    r->n_lucy = P->n_lucy;
    r->min_margin = P->mm;
  }
  st->st.lucy_deposits += P->n_lucy;
}

/* The life of one packet. pass 2 packets start at a uniform point of cell
 * `pcell` with a wavelength from that cell's PAH emissivity row. */
static void run_packet(run_t *R, uint64_t pid, int64_t pcell, uint64_t slot) {
  const orc_model *m = R->m;
  const tab_t *t = &R->t;
  int nl = t->nl, ns = t->ns;
  rng_t rg;
  rng_init(&rg, R->seed, pid, R->iter, (uint32_t)R->o->model_id, R->tag);
  pkt_t P;
  memset(&P, 0, sizeof(P));
  P.mm = INFINITY;
  R->st->st.packets++;
  if (R->pass == 2 &&
      !pah_dissociates_xi(m, R->o, R->xi, leaf_V(R, pcell), R->st->kpah[pcell], pcell)) {
    int64_t c = pcell;
    double ux = rng_next(&rg), uy = rng_next(&rg), uz = rng_next(&rg);
    double ul = rng_next(&rg), uph = rng_next(&rg), umu = rng_next(&rg);
    double uu[3] = {ux, uy, uz};
    if (c < n_cubes(m)) {
      int cc[3] = {(int)(c % m->nx), (int)((c / m->nx) % m->ny), (int)(c / ((int64_t)m->nx * m->ny))};
      for (int k = 0; k < 3; k++) {
        P.c[k] = cc[k];
        P.p[k] = m->origin[k] + ((double)cc[k] + uu[k]) * m->dcell;
      }
    } else {
      /* a sub-cube: uniform inside it */
      int r;
      leaf_loc(m, c, P.c, P.f, &r);
      double h = m->dcell / (double)r;
      for (int k = 0; k < 3; k++) P.p[k] = face_pos(m, k, P.c[k], r, P.f[k]) + uu[k] * h;
    }
    P.j = pick_pah_lambda(R, pah_row(R, c), ul, &P.mm);
    iso_dir(uph, umu, P.d);
  } else {
    double uph = rng_next(&rg), umu = rng_next(&rg);
    double us = rng_next(&rg), ul = rng_next(&rg);
    /* m equal-energy source bins of Eq. 1, each emitting every m-th packet:
     * packet pid draws inside stratum pid mod m of the source spectrum's
     * cumulative distribution */
    if (R->o->src_strata > 0 && R->pass != 2)
      ul = ((double)(pid % R->o->src_strata) + ul) / (double)R->o->src_strata;
    iso_dir(uph, umu, P.d);
    int s = pick_asc(m->src_lum, m->nsrc, us, &P.mm);
    for (int k = 0; k < 3; k++) P.p[k] = m->src_pos[3 * s + k];
    P.j = pick_desc(t->src_f + (int64_t)s * nl, nl, ul, &P.mm);
    start_cell(m, P.p, P.d, P.c);
    if (!inside(m, P.c)) {
      P.status = ORC_ESCAPED;
      finish(R, &P, pid, slot);
      return;
    }
    int r = cube_r(m, cidx(m, P.c));
    for (int k = 0; k < 3; k++) P.f[k] = sub_index(m, k, P.c[k], r, P.p[k], P.d[k]);
  }
  for (;;) {
    while (mrw_step(R, &P, &rg)) {
      P.n_int++;
      if (R->o->max_int > 0 && P.n_int >= R->o->max_int) {
        P.status = ORC_KILLED;
        finish(R, &P, pid, slot);
        return;
      }
    }
    double tau_star = (R->o->tau_mode == ORC_TAU_PER_CELL) ? 0.0 : -log(rng_next(&rg));
    if (fly(R, &P, tau_star, &rg)) {
      P.status = ORC_ESCAPED;
      finish(R, &P, pid, slot);
      return;
    }
    int64_t c = leaf_id(m, P.c, P.f);
    double ualb = rng_next(&rg), usp = rng_next(&rg);
    int j = P.j;
    upd_margin(&P.mm, fabs(ualb - t->alb[j]));
    if (ualb < t->alb[j]) {
      for (int s = 0; s < ns; s++) R->fs[s] = m->mass_frac[s] * t->ksca_eff[s * nl + j];
      int s = pick_asc(R->fs, ns, usp, &P.mm);
      double gg = t->g_eff[s * nl + j];
      double umu = rng_next(&rg), uph = rng_next(&rg);
      double mu = orc_hg_mu(gg, umu);
      int q = t->imgmap[j];
      if (q >= 0) {
        for (int v = 0; v < m->nview; v++) {
          double cb = P.d[0] * t->kv[v][0] + P.d[1] * t->kv[v][1] + P.d[2] * t->kv[v][2];
          R->st->ssca[((int64_t)v * m->nimg + q) * t->ncell + c] += R->xi * orc_hg_phase(gg, cb);
        }
        /* event stored for any observer: P_HG(d.k) = sum_l g^l sum_m Y_lm(d) Y_lm(k) */
        if (R->o->sh_order > 0 && R->st->sh) {
          int L1 = R->o->sh_order, nlm = L1 * L1;
          double y[256];
          orc_ylm(L1 - 1, P.d, y);
          double gl = 1.0;
          for (int l = 0; l < L1; l++) {
            for (int mm = -l; mm <= l; mm++) {
              int i = l * l + l + mm;
              R->st->sh[((int64_t)q * nlm + i) * t->ncell + c] += R->xi * gl * y[i];
            }
            gl *= gg;
          }
        }
      }
      rotate_dir(P.d, mu, 2.0 * PI_D * uph);
      P.n_scat++;
      R->st->st.scatters++;
    } else {
      for (int s = 0; s < ns; s++) R->fs[s] = m->mass_frac[s] * m->kabs[s * nl + j];
      int s = pick_asc(R->fs, ns, usp, &P.mm);
      P.n_abs++;
      R->st->st.absorptions++;
      if (s == m->pah_species) {
        if (R->pass != 2) {
          R->st->kpah[c] += 1;
          P.status = ORC_PAH_STOP;
          finish(R, &P, pid, slot);
          return;
        }
        double ul = rng_next(&rg), uph = rng_next(&rg), umu = rng_next(&rg);
        P.j = pick_pah_lambda(R, pah_row(R, c), ul, &P.mm);
        iso_dir(uph, umu, P.d);
      } else {
        if (!is_thin(R, leaf_rho(m, c), pkt_h(R, &P))) {
          R->st->k[(int64_t)s * t->ncell + c] += 1;
          touch(R, (int64_t)s * t->ncell + c);
        }
        double T = mode_T(R, s, c);
        for (int q = 0; q < nl; q++) {
          double b = (R->o->mode == ORC_FROZEN) ? orc_planck(t->nu[q], T)
                                                 : orc_dplanck_dT(t->nu[q], T);
          R->f[q] = t->w[q] * m->kabs[s * nl + q] * b;
        }
        double ul = rng_next(&rg), uph = rng_next(&rg), umu = rng_next(&rg);
        P.j = pick_desc(R->f, nl, ul, &P.mm);
        iso_dir(uph, umu, P.d);
      }
    }
    P.n_int++;
    if (R->o->max_int > 0 && P.n_int >= R->o->max_int) {
      P.status = ORC_KILLED;
      finish(R, &P, pid, slot);
      return;
    }
  }
}

static void zero_tallies(const run_t *R) {
  const orc_model *m = R->m;
  int64_t nc = R->t.ncell, ns = R->t.ns;
  memset(R->st->k, 0, sizeof(uint64_t) * nc * ns);
  memset(R->st->epath, 0, sizeof(double) * nc * ns);
  memset(R->st->kpah, 0, sizeof(uint32_t) * nc);
  int nt = R->o->ntheta > 0 ? R->o->ntheta : 1;
  memset(R->st->sed, 0, sizeof(uint64_t) * nt * R->t.nl);
  if (m->nview > 0 && m->nimg > 0 && R->st->ssca)
    memset(R->st->ssca, 0, sizeof(double) * nc * m->nview * m->nimg);
  if (R->o->sh_order > 0 && m->nimg > 0 && R->st->sh)
    memset(R->st->sh, 0,
           sizeof(double) * nc * m->nimg * (size_t)R->o->sh_order * (size_t)R->o->sh_order);
}

/* Start of an epoch: cells whose energy changed get a fresh snapshot and
 * lose their cached epoch temperature. The first snapshot of a run visits
 * every entry; later ones visit the touched entries, the only ones whose
 * energy or cached temperature can have changed since. */
static void snap_entry(run_t *R, int64_t q) {
  double e = (double)R->st->k[q] * R->xi + R->st->epath[q];  /* E of Eq. 4 */
  if (e != R->st->esnap[q] || !R->st->tvalid[q]) {
    R->st->esnap[q] = e;
    R->st->tvalid[q] = 0;
  }
}

static void epoch_snapshot(run_t *R, int full) {
  int64_t nc = R->t.ncell;
  if (full || !R->is_touched) {
    for (int64_t q = 0; q < (int64_t)R->t.ns * nc; q++) snap_entry(R, q);
  } else {
    for (int64_t i = 0; i < R->n_touched; i++) snap_entry(R, R->touched[i]);
  }
  if (R->is_touched) {
    for (int64_t i = 0; i < R->n_touched; i++) R->is_touched[R->touched[i]] = 0;
    R->n_touched = 0;
  }
}

static void run_init(run_t *R, const orc_model *m, const orc_opts *o, uint64_t seed,
                     orc_state *st) {
  memset(R, 0, sizeof(*R));
  R->m = m;
  R->o = o;
  tab_init(&R->t, m);
  R->st = st;
  R->seed = seed;
  R->xi = R->t.ltot / (double)o->n_total;
  R->f = malloc(sizeof(double) * m->nl);
  R->fs = malloc(sizeof(double) * m->ns);
  if (o->mode == ORC_BW_EPOCH) {
    int64_t nq = (int64_t)m->ns * R->t.ncell;
    R->touched = malloc(sizeof(int64_t) * (size_t)nq);
    R->is_touched = calloc((size_t)nq, 1);
  }
}

static void run_free(run_t *R) {
  tab_free(&R->t);
  free(R->f);
  free(R->fs);
  free(R->touched);
  free(R->is_touched);
}

void orc_finalize_T(const orc_model *m, const orc_opts *o, orc_state *st) {
  run_t R;
  run_init(&R, m, o, 0, st);
  int64_t nc = R.t.ncell;
  for (int s = 0; s < R.t.ns; s++)
    for (int64_t c = 0; c < nc; c++) {
      double rho = leaf_rho(m, c);
      double T = 0.0;
      if (s != m->pah_species && rho > 0.0 && m->mass_frac[s] > 0.0) {
        double rhs = e_cell(&R, s, c) / (4.0 * PI_D * m->mass_frac[s] * rho * leaf_V(&R, c));
        int cl = 0;
        T = invert_t(&R.t, s, rhs, &cl);
        if (cl) st->st.clamped_T++;
      }
      st->T[(int64_t)s * nc + c] = T;
    }
  run_free(&R);
}

int orc_run(const orc_model *m, const orc_opts *o, uint64_t first, uint64_t n,
            uint64_t seed, orc_state *st) {
  run_t R;
  run_init(&R, m, o, seed, st);
  R.tag = 0;
  R.pass = 1;
  if (o->mode == ORC_FROZEN) {
    for (int it = 0; it < o->n_iter; it++) {
      R.iter = (uint32_t)it;
      zero_tallies(&R);
      for (uint64_t i = 0; i < n; i++) run_packet(&R, first + i, -1, i);
      orc_finalize_T(m, o, st);
    }
  } else {
    R.iter = 0;
    uint64_t P = o->epoch > 0 ? o->epoch : 1;
    for (uint64_t i = 0; i < n; i++) {
      uint64_t pid = first + i;
      if (i == 0 || pid % P == 0) epoch_snapshot(&R, i == 0);
      run_packet(&R, pid, -1, i);
    }
  }
  run_free(&R);
  return 0;
}

int orc_pah_pass(const orc_model *m, const orc_opts *o, uint64_t seed, orc_state *st) {
  if (m->pah_species < 0) return 0;
  run_t R;
  run_init(&R, m, o, seed, st);
  R.tag = 3;
  R.pass = 2;
  R.iter = 0;
  uint64_t P = o->epoch > 0 ? o->epoch : 1;
  /* pass-1 counts fix the packet ids and the emissivity rows */
  int64_t nc = R.t.ncell;
  uint32_t *k1 = malloc(sizeof(uint32_t) * nc);
  memcpy(k1, st->kpah, sizeof(uint32_t) * nc);
  uint64_t idx = 0;
  for (int64_t c = 0; c < nc; c++) {
    for (uint32_t r = 0; r < k1[c]; r++, idx++) {
      if (o->mode == ORC_BW_EPOCH && (idx == 0 || idx % P == 0)) epoch_snapshot(&R, idx == 0);
      run_packet(&R, o->n_total + idx, c, idx);
    }
  }
  free(k1);
  run_free(&R);
  return 0;
}

void orc_init_T(const orc_model *m, double *T) {
  tab_t t;
  tab_init(&t, m);
  int nl = m->nl;
  double *J = malloc(sizeof(double) * nl);
  double *f = malloc(sizeof(double) * nl);
  for (int64_t c = 0; c < t.ncell; c++) {
    double x[3];
    if (c < n_cubes(m)) {
      int cc[3] = {(int)(c % m->nx), (int)((c / m->nx) % m->ny), (int)(c / ((int64_t)m->nx * m->ny))};
      for (int k = 0; k < 3; k++) x[k] = m->origin[k] + ((double)cc[k] + 0.5) * m->dcell;
    } else {
      double lo[3], h, rho;
      orc_leaf_box(m, c, lo, &h, &rho);
      for (int k = 0; k < 3; k++) x[k] = lo[k] + 0.5 * h;
    }
    for (int j = 0; j < nl; j++) J[j] = 0.0;
    for (int s = 0; s < m->nsrc; s++) {
      double dx = x[0] - m->src_pos[3 * s], dy = x[1] - m->src_pos[3 * s + 1],
             dz = x[2] - m->src_pos[3 * s + 2];
      double r2 = dx * dx + dy * dy + dz * dz;
      for (int j = 0; j < nl; j++) J[j] += t.lnu[s * nl + j] / (16.0 * PI_D * PI_D * r2);
    }
    for (int s = 0; s < m->ns; s++) {
      double Tv = 0.0;
      if (s != m->pah_species && leaf_rho(m, c) > 0.0) {
        for (int j = 0; j < nl; j++) f[j] = t.w[j] * m->kabs[s * nl + j] * J[j];
        Tv = invert_t(&t, s, sum_desc(f, nl), NULL);
      }
      T[(int64_t)s * t.ncell + c] = Tv;
    }
  }
  free(J);
  free(f);
  tab_free(&t);
}

/* ----------------------------------------------------------- ray-tracer */

typedef struct {
  double k[3], ex[3], ey[3];
  double ctr[3], fov, dpx, dpy;
} view_t;

static void view_frame(const orc_model *m, int v, int npx, int npy, view_t *vw) {
  double th = m->view_deg[2 * v] * PI_D / 180.0, ph = m->view_deg[2 * v + 1] * PI_D / 180.0;
  vw->k[0] = sin(th) * cos(ph); vw->k[1] = sin(th) * sin(ph); vw->k[2] = cos(th);
  vw->ex[0] = cos(th) * cos(ph); vw->ex[1] = cos(th) * sin(ph); vw->ex[2] = -sin(th);
  vw->ey[0] = -sin(ph); vw->ey[1] = cos(ph); vw->ey[2] = 0.0;
  int n[3] = {m->nx, m->ny, m->nz};
  double L = 0.0;
  for (int k = 0; k < 3; k++) {
    vw->ctr[k] = m->origin[k] + 0.5 * (double)n[k] * m->dcell;
    if ((double)n[k] * m->dcell > L) L = (double)n[k] * m->dcell;
  }
  vw->fov = sqrt(3.0) * L;
  vw->dpx = vw->fov / (double)npx;
  vw->dpy = vw->fov / (double)npy;
}

/* Entry point of the pixel ray (travelling along -k) into the grid box;
 * returns 0 when the ray misses. */
static int ray_entry(const orc_model *m, const view_t *vw, int ix, int iy, double pe[3],
                     double dir[3], int c[3]) {
  double xp = ((double)ix + 0.5) * vw->dpx - 0.5 * vw->fov;
  double yp = ((double)iy + 0.5) * vw->dpy - 0.5 * vw->fov;
  double r0[3];
  for (int k = 0; k < 3; k++) {
    r0[k] = vw->ctr[k] + xp * vw->ex[k] + yp * vw->ey[k] + vw->fov * vw->k[k];
    dir[k] = -vw->k[k];
  }
  int n[3] = {m->nx, m->ny, m->nz};
  double tmin = -INFINITY, tmax = INFINITY;
  for (int k = 0; k < 3; k++) {
    double lo = m->origin[k], hi = m->origin[k] + (double)n[k] * m->dcell;
    if (dir[k] != 0.0) {
      double t1 = (lo - r0[k]) / dir[k], t2 = (hi - r0[k]) / dir[k];
      double a = t1 < t2 ? t1 : t2, b = t1 < t2 ? t2 : t1;
      if (a > tmin) tmin = a;
      if (b < tmax) tmax = b;
    } else if (r0[k] < lo || r0[k] > hi) {
      return 0;
    }
  }
  if (!(tmin < tmax)) return 0;
  for (int k = 0; k < 3; k++) pe[k] = r0[k] + tmin * dir[k];
  start_cell(m, pe, dir, c);
  for (int k = 0; k < 3; k++) {
    if (c[k] < 0) c[k] = 0;
    if (c[k] >= n[k]) c[k] = n[k] - 1;
  }
  return 1;
}

/* Walk the segments of a ray from p0 in cube c (sub-cube from the
 * position): returns the count, fills leaves/lens (sized by max_segs). */
static int walk(const orc_model *m, const double p0[3], const double d[3], int c0[3],
                int64_t *cells, double *lens) {
  walker_t W = {m, p0, d, {c0[0], c0[1], c0[2]}, {0, 0, 0}, 1, {0, 0, 0}};
  if (!inside(m, W.c)) return 0;
  walker_enter(&W, 0.0, -1, NULL);
  double t = 0.0;
  int ns = 0;
  for (;;) {
    int a = 0;
    if (W.tm[1] < W.tm[a]) a = 1;
    if (W.tm[2] < W.tm[a]) a = 2;
    double ell = W.tm[a] - t;
    if (ell < 0.0) ell = 0.0;
    cells[ns] = walker_leaf(&W);
    lens[ns] = ell;
    ns++;
    if (W.tm[a] > t) t = W.tm[a];
    if (walker_cross(&W, a, t)) return ns;
  }
}

/* most segments a straight walk can have: each cube it enters adds at most
 * 3 r - 2 sub-cube segments */
static int max_segs(const orc_model *m) {
  int rmax = 1;
  if (m->ref)
    for (int64_t c = 0; c < n_cubes(m); c++)
      if (cube_r(m, c) > rmax) rmax = cube_r(m, c);
  return (m->nx + m->ny + m->nz + 3) * 3 * rmax;
}

/* Source function per imaged wavelength (sect. 4, Eqs. 14 and 16 read as
 * emissivity over extinction): S = sum_s f_s kabs_s B(T_s)/kext +
 * Ssca/(V dnu rho kext), with rho the model density that produced the
 * scattering events (emissivity per unit mass fixed). */
static double source_fn(const tab_t *t, const orc_model *m, const double *T,
                        const double *ssca, int v, int q, int64_t c) {
  int j = m->img_idx[q], nl = t->nl;
  double em = 0.0;
  for (int s = 0; s < t->ns; s++) {
    if (s == m->pah_species) continue;
    em += m->mass_frac[s] * m->kabs[s * nl + j] * orc_planck(t->nu[j], T[(int64_t)s * t->ncell + c]);
  }
  double S = em / t->kext[j];
  double lo[3], h, rho;
  orc_leaf_box(m, c, lo, &h, &rho);
  double V = (c < n_cubes(m)) ? t->V : h * h * h;
  if (ssca && rho > 0.0)
    S += ssca[((int64_t)v * m->nimg + q) * t->ncell + c] / (V * t->w[j] * rho * t->kext[j]);
  return S;
}

/* Eqs. 13-14 as printed: absorption optical depth K^abs int rho ds (K^abs
 * of the whole mixture), a cell emitting [1 - exp(-tau_cell)] times its
 * source function, with tau_cell = rho K^abs dcell measured face to face,
 * plus the scattered intensity of Eq. 16, sum P_HG xi / dnu spread over
 * the cell's face dcell^2. The mixture's source function is
 * sum_s f_s kabs_s B(T_s) / K^abs (B(T) for one species). Both terms come
 * from the model density; rho_rt enters only the attenuation toward the
 * observer. */
static double kabs_all(const tab_t *t, const orc_model *m, int j) {
  double k = 0.0;
  for (int s = 0; s < t->ns; s++) k += m->mass_frac[s] * m->kabs[s * t->nl + j];
  return k;
}

static double cell_literal(const tab_t *t, const orc_model *m, const double *T,
                           const double *ssca, int v, int q, int64_t c) {
  int j = m->img_idx[q], nl = t->nl;
  double lo[3], h, rho;
  orc_leaf_box(m, c, lo, &h, &rho);
  if (!(rho > 0.0)) return 0.0;
  double ka = kabs_all(t, m, j);
  double em = 0.0;
  for (int s = 0; s < t->ns; s++) {
    if (s == m->pah_species) continue;
    em += m->mass_frac[s] * m->kabs[s * nl + j] * orc_planck(t->nu[j], T[(int64_t)s * t->ncell + c]);
  }
  double I = (ka > 0.0) ? -expm1(-(rho * ka * h)) * (em / ka) : 0.0;
  if (ssca) I += ssca[((int64_t)v * m->nimg + q) * t->ncell + c] / (t->w[j] * h * h);
  return I;
}

int orc_raytrace(const orc_model *m, int rt_mode, const double *T, const double *ssca,
                 const double *rho_rt, int npx, int npy, double *img, double *sed) {
  const int lit = rt_mode == ORC_RT_ABS_LITERAL;
  double *rho_leaf = NULL;
  if (!rho_rt) {
    /* the model's density of every leaf */
    int64_t nlf = orc_nleaf(m);
    rho_leaf = malloc(sizeof(double) * nlf);
    for (int64_t c = 0; c < nlf; c++) rho_leaf[c] = leaf_rho(m, c);
    rho_rt = rho_leaf;
  }
  tab_t t;
  tab_init(&t, m);
  int maxs = max_segs(m);
  int64_t *cells = malloc(sizeof(int64_t) * maxs);
  double *lens = malloc(sizeof(double) * maxs);
  double D2 = m->distance * m->distance;
  for (int v = 0; v < m->nview; v++) {
    view_t vw;
    view_frame(m, v, npx, npy, &vw);
    double apix = vw.dpx * vw.dpy;
    for (int q = 0; q < m->nimg; q++) sed[v * m->nimg + q] = 0.0;
    for (int iy = 0; iy < npy; iy++)
      for (int ix = 0; ix < npx; ix++) {
        double pe[3], dir[3];
        int c[3], nseg = 0;
        if (ray_entry(m, &vw, ix, iy, pe, dir, c)) nseg = walk(m, pe, dir, c, cells, lens);
        for (int q = 0; q < m->nimg; q++) {
          int j = m->img_idx[q];
          double I = 0.0, tr = 1.0;
          for (int s = 0; s < nseg; s++) {
            double rho = rho_rt[cells[s]];
            if (lit) {
              I += tr * cell_literal(&t, m, T, ssca, v, q, cells[s]);
              tr *= exp(-(rho * kabs_all(&t, m, j) * lens[s]));
              continue;
            }
            if (!(rho > 0.0)) continue;
            double dtau = rho * t.kext[j] * lens[s];
            double S = source_fn(&t, m, T, ssca, v, q, cells[s]);
            I += tr * S * (-expm1(-dtau));
            tr *= exp(-dtau);
          }
          double F = apix / D2 * I;
          img[(((int64_t)v * m->nimg + q) * npy + iy) * npx + ix] = F;
          sed[v * m->nimg + q] += F;
        }
      }
    /* attenuated point sources */
    for (int s = 0; s < m->nsrc; s++) {
      const double *ps = m->src_pos + 3 * s;
      int c[3];
      start_cell(m, ps, vw.k, c);
      int nseg = walk(m, ps, vw.k, c, cells, lens);
      double xp = 0.0, yp = 0.0;
      for (int k = 0; k < 3; k++) {
        xp += (ps[k] - vw.ctr[k]) * vw.ex[k];
        yp += (ps[k] - vw.ctr[k]) * vw.ey[k];
      }
      int ix = (int)floor((xp + 0.5 * vw.fov) / vw.dpx), iy = (int)floor((yp + 0.5 * vw.fov) / vw.dpy);
      for (int q = 0; q < m->nimg; q++) {
        int j = m->img_idx[q];
        double kx = lit ? kabs_all(&t, m, j) : t.kext[j];
        double tau = 0.0;
        for (int g = 0; g < nseg; g++) tau += rho_rt[cells[g]] * kx * lens[g];
        double F = t.lnu[s * t.nl + j] / (4.0 * PI_D * D2) * exp(-tau);
        if (ix >= 0 && ix < npx && iy >= 0 && iy < npy)
          img[(((int64_t)v * m->nimg + q) * npy + iy) * npx + ix] += F;
        sed[v * m->nimg + q] += F;
      }
    }
  }
  free(cells);
  free(lens);
  free(rho_leaf);
  tab_free(&t);
  return 0;
}

/* Adjoint of orc_raytrace. With T and the scattering emissivity per unit
 * mass held fixed, S does not depend on rho; only dtau = rho kext l does:
 * dI/d(dtau_i) = T_<i S_i e^{-dtau_i} - (I - A_i), A_i the intensity
 * gathered up to and including cell i. A first sweep gives I, a second
 * recomputes the transmittance and A_i. */
int orc_raytrace_adjoint(const orc_model *m, int rt_mode, const double *T, const double *ssca,
                         const double *rho_rt, int npx, int npy, const double *w_img,
                         const double *w_sed, double *drho) {
  /* printed form: the cell terms C_i do not depend on rho_rt, so
   * dI/d(dtau_i) = -(I - A_i) with A_i the intensity gathered up to and
   * including cell i */
  const int lit = rt_mode == ORC_RT_ABS_LITERAL;
  double *rho_leaf = NULL;
  if (!rho_rt) {
    /* the model's density of every leaf */
    int64_t nlf = orc_nleaf(m);
    rho_leaf = malloc(sizeof(double) * nlf);
    for (int64_t c = 0; c < nlf; c++) rho_leaf[c] = leaf_rho(m, c);
    rho_rt = rho_leaf;
  }
  tab_t t;
  tab_init(&t, m);
  int maxs = max_segs(m);
  int64_t *cells = malloc(sizeof(int64_t) * maxs);
  double *lens = malloc(sizeof(double) * maxs);
  double D2 = m->distance * m->distance;
  for (int64_t c = 0; c < t.ncell; c++) drho[c] = 0.0;
  for (int v = 0; v < m->nview; v++) {
    view_t vw;
    view_frame(m, v, npx, npy, &vw);
    double apix = vw.dpx * vw.dpy;
    for (int iy = 0; iy < npy; iy++)
      for (int ix = 0; ix < npx; ix++) {
        double pe[3], dir[3];
        int c[3], nseg = 0;
        if (ray_entry(m, &vw, ix, iy, pe, dir, c)) nseg = walk(m, pe, dir, c, cells, lens);
        for (int q = 0; q < m->nimg; q++) {
          int j = m->img_idx[q];
          double W = (w_img ? w_img[(((int64_t)v * m->nimg + q) * npy + iy) * npx + ix] : 0.0) +
                     (w_sed ? w_sed[v * m->nimg + q] : 0.0);
          if (W == 0.0) continue;
          double I = 0.0, tr = 1.0;
          if (lit) {
            double ka = kabs_all(&t, m, j);
            for (int s = 0; s < nseg; s++) {
              I += tr * cell_literal(&t, m, T, ssca, v, q, cells[s]);
              tr *= exp(-(rho_rt[cells[s]] * ka * lens[s]));
            }
            double A = 0.0;
            tr = 1.0;
            for (int s = 0; s < nseg; s++) {
              A += tr * cell_literal(&t, m, T, ssca, v, q, cells[s]);
              drho[cells[s]] += W * (apix / D2) * ka * lens[s] * (-(I - A));
              tr *= exp(-(rho_rt[cells[s]] * ka * lens[s]));
            }
            continue;
          }
          for (int s = 0; s < nseg; s++) {
            double rho = rho_rt[cells[s]];
            if (!(rho > 0.0)) continue;
            double dtau = rho * t.kext[j] * lens[s];
            double S = source_fn(&t, m, T, ssca, v, q, cells[s]);
            I += tr * S * (-expm1(-dtau));
            tr *= exp(-dtau);
          }
          double A = 0.0;
          tr = 1.0;
          for (int s = 0; s < nseg; s++) {
            double rho = rho_rt[cells[s]];
            if (!(rho > 0.0)) continue;
            double dtau = rho * t.kext[j] * lens[s];
            double S = source_fn(&t, m, T, ssca, v, q, cells[s]);
            double e = exp(-dtau);
            A += tr * S * (-expm1(-dtau));
            double dI = tr * S * e - (I - A);
            drho[cells[s]] += W * (apix / D2) * t.kext[j] * lens[s] * dI;
            tr *= e;
          }
        }
      }
    for (int s = 0; s < m->nsrc; s++) {
      const double *ps = m->src_pos + 3 * s;
      int c[3];
      start_cell(m, ps, vw.k, c);
      int nseg = walk(m, ps, vw.k, c, cells, lens);
      double xp = 0.0, yp = 0.0;
      for (int k = 0; k < 3; k++) {
        xp += (ps[k] - vw.ctr[k]) * vw.ex[k];
        yp += (ps[k] - vw.ctr[k]) * vw.ey[k];
      }
      int ix = (int)floor((xp + 0.5 * vw.fov) / vw.dpx), iy = (int)floor((yp + 0.5 * vw.fov) / vw.dpy);
      int inimg = ix >= 0 && ix < npx && iy >= 0 && iy < npy;
      for (int q = 0; q < m->nimg; q++) {
        int j = m->img_idx[q];
        double W = (w_sed ? w_sed[v * m->nimg + q] : 0.0) +
                   ((inimg && w_img) ? w_img[(((int64_t)v * m->nimg + q) * npy + iy) * npx + ix] : 0.0);
        if (W == 0.0) continue;
        double kx = lit ? kabs_all(&t, m, j) : t.kext[j];
        double tau = 0.0;
        for (int g = 0; g < nseg; g++) tau += rho_rt[cells[g]] * kx * lens[g];
        double F = t.lnu[s * t.nl + j] / (4.0 * PI_D * D2) * exp(-tau);
        for (int g = 0; g < nseg; g++) drho[cells[g]] += -W * kx * lens[g] * F;
      }
    }
  }
  free(cells);
  free(lens);
  free(rho_leaf);
  tab_free(&t);
  return 0;
}

/* ----------------------------------------------------------- voxelizers */

/* Clumpy torus by the cell-centre test: clump density inside any clump
 * (overlaps keep the single-clump density), inter-clump density inside the
 * wedge r_in <= r <= r_out, |z| <= r sin(theta1), empty elsewhere. Clumps
 * are visited one by one over the cells near them (a box one cell wider
 * than the clump on each side), which selects exactly the cells whose
 * centre passes the distance test. */
void orc_voxelize_torus(int nx, int ny, int nz, const double origin[3], double dcell,
                        int ncl, const double *C, double r_clump, double rho_clump,
                        double rho_inter, double r_in, double r_out, double s1,
                        double *rho) {
  double rc2 = r_clump * r_clump, ri2 = r_in * r_in, ro2 = r_out * r_out, s12 = s1 * s1;
  int64_t nc = (int64_t)nx * ny * nz;
  unsigned char *in = calloc((size_t)nc, 1);
  int n[3] = {nx, ny, nz};
  for (int k = 0; k < ncl; k++) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
      lo[a] = (int)floor((C[3 * k + a] - r_clump - origin[a]) / dcell) - 1;
      hi[a] = (int)floor((C[3 * k + a] + r_clump - origin[a]) / dcell) + 1;
      if (lo[a] < 0) lo[a] = 0;
      if (hi[a] > n[a] - 1) hi[a] = n[a] - 1;
    }
    for (int iz = lo[2]; iz <= hi[2]; iz++)
      for (int iy = lo[1]; iy <= hi[1]; iy++)
        for (int ix = lo[0]; ix <= hi[0]; ix++) {
          double x = origin[0] + ((double)ix + 0.5) * dcell;
          double y = origin[1] + ((double)iy + 0.5) * dcell;
          double z = origin[2] + ((double)iz + 0.5) * dcell;
          double dx = x - C[3 * k], dy = y - C[3 * k + 1], dz = z - C[3 * k + 2];
          if (dx * dx + dy * dy + dz * dz <= rc2) in[((int64_t)iz * ny + iy) * nx + ix] = 1;
        }
  }
  for (int iz = 0; iz < nz; iz++)
    for (int iy = 0; iy < ny; iy++)
      for (int ix = 0; ix < nx; ix++) {
        int64_t c = ((int64_t)iz * ny + iy) * nx + ix;
        double x = origin[0] + ((double)ix + 0.5) * dcell;
        double y = origin[1] + ((double)iy + 0.5) * dcell;
        double z = origin[2] + ((double)iz + 0.5) * dcell;
        double v = 0.0;
        if (in[c]) {
          v = rho_clump;
        } else {
          double r2 = x * x + y * y + z * z;
          if (r2 >= ri2 && r2 <= ro2 && z * z <= r2 * s12) v = rho_inter;
        }
        rho[c] = v;
      }
  free(in);
}

/* Gauss-Legendre nodes/weights on [-1,1] by Newton on P_n. */
static void gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < n; i++) {
    double z = cos(PI_D * ((double)i + 0.75) / ((double)n + 0.5)), pp = 0.0;
    for (int it = 0; it < 100; it++) {
      double p1 = 1.0, p2 = 0.0;
      for (int k = 1; k <= n; k++) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * k - 1.0) * z * p2 - (k - 1.0) * p3) / k;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      double z1 = z;
      z = z1 - p1 / pp;
      if (fabs(z - z1) < 1e-15) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

/* Power-law shell: cell average of rho0 (r_in/r)^power on [r_in, r_out]
 * (power 2: the r^-2 shell; 0: constant density) by an 8^3 Gauss-Legendre
 * rule per cell. */
static double shell_law(double rho0, double r_in, double r, double power) {
  double q = r_in / r;
  if (power == 2.0) return rho0 * q * q;
  if (power == 0.0) return rho0;
  return rho0 * pow(q, power);
}

void orc_voxelize_shell(int nx, int ny, int nz, const double origin[3], double dcell,
                        double rho0, double r_in, double r_out, double power, double *rho) {
  double gx[8], gw[8];
  gauss_legendre(8, gx, gw);
  for (int iz = 0; iz < nz; iz++)
    for (int iy = 0; iy < ny; iy++)
      for (int ix = 0; ix < nx; ix++) {
        double sum = 0.0;
        for (int a = 0; a < 8; a++)
          for (int b = 0; b < 8; b++)
            for (int e = 0; e < 8; e++) {
              double x = origin[0] + ((double)ix + 0.5 + 0.5 * gx[a]) * dcell;
              double y = origin[1] + ((double)iy + 0.5 + 0.5 * gx[b]) * dcell;
              double z = origin[2] + ((double)iz + 0.5 + 0.5 * gx[e]) * dcell;
              double r = sqrt(x * x + y * y + z * z);
              double f = (r >= r_in && r <= r_out) ? shell_law(rho0, r_in, r, power) : 0.0;
              sum += gw[a] * gw[b] * gw[e] * f;
            }
        rho[((int64_t)iz * ny + iy) * nx + ix] = 0.125 * sum;
      }
}
