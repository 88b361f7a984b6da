/*
 * mcrt_oracle.h - plain FP64 CPU oracle for Monte Carlo dust radiative
 * transfer (Heymann & Siebenmorgen, sect. 2-4).
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the CPU-baseline
 * leg of the benchmark are the only callers. It shares no code with the HIP
 * library: it is a slow, sequential, obviously-correct statement of what the
 * GPU path computes, written from the paper's equations.
 *
 * Units: cgs; wavelengths in micrometres. Grid cells are cubes of side
 * `dcell`, linear index (iz*ny + iy)*nx + ix (x fastest).
 */
#ifndef MCRT_ORACLE_H
#define MCRT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FROZEN = 0, ORC_BW_EPOCH = 1 };
/* optical depth of a flight: one draw per flight, or a new draw on entering
 * each cell (the footnote to the sect. 2 interaction test) */
enum { ORC_TAU_FLIGHT = 0, ORC_TAU_PER_CELL = 1 };
/* ray-tracer formal solution: extinction chord form, or Eqs. 13-14 as
 * printed (absorption optical depth, face-to-face cell emission) */
enum { ORC_RT_EXT = 0, ORC_RT_ABS_LITERAL = 1 };
enum { ORC_ALIVE = 0, ORC_ESCAPED = 1, ORC_KILLED = 2, ORC_PAH_STOP = 3 };

typedef struct {
  int32_t nx, ny, nz, pad0;
  double origin[3];
  double dcell;
  const double *rho;             /* [nz][ny][nx] g/cm^3 */
  int32_t nl, ns;
  const double *lam_um;          /* [nl] strictly increasing */
  const double *mass_frac;       /* [ns] */
  const double *kabs, *ksca, *g; /* [ns][nl] cm^2 per g of dust */
  int32_t pah_species, n_pah_rows;
  const double *pah_emis;        /* [rows][nl] */
  const double *pah_edges;       /* [rows-1] */
  int32_t nsrc;
  int32_t scat_law;              /* 0: Henyey-Greenstein (Eq. 15); 1: g-factor approximation,
                                    isotropic scattering with kappa_sca (1 - g) (sect. 4) */
  const double *src_pos;         /* [nsrc][3] */
  const double *src_lum;         /* [nsrc] erg/s */
  const double *src_shape;       /* [nsrc][nl] ~ L_nu, or NULL */
  const double *src_tbb;         /* [nsrc] blackbody K, used when shape NULL */
  int32_t nview, nimg;
  const double *view_deg;        /* [nview][2] (theta, phi) */
  const int32_t *img_idx;        /* [nimg] */
  double distance;               /* cm */
  /* one level of refinement (sect. 2: cubes divided into sub-cubes of their
   * own density): ref[cube] = r >= 2 divides the cube into r^3 sub-cubes of
   * edge dcell / r whose densities start at rho_sub[sub_off[cube]], x fastest
   * inside the cube; 0 or 1 leaves it whole; sub_off is the exclusive prefix
   * sum over the cubes of r^3 (0 for whole cubes). ref NULL: no refinement. Leaf
   * cells (whole cubes, sub-cubes) are numbered cube index for a whole cube,
   * n_cubes + sub_off[cube] + local index for a sub-cube; every per-cell
   * array (tallies, temperatures, scattering sums) runs over the leaves. */
  const uint8_t *ref;
  const int64_t *sub_off;
  const double *rho_sub;
  int64_t nsub;
} orc_model;

typedef struct {
  int32_t mode;       /* ORC_FROZEN or ORC_BW_EPOCH */
  int32_t n_iter;     /* FROZEN iterations */
  uint64_t epoch;     /* packets per epoch (BW_EPOCH); 1 = serial B&W */
  uint64_t n_total;   /* packet count defining xi = L/n_total */
  double lucy_tau;    /* Lucy threshold on max cell optical depth; <=0 off */
  double mrw_tau;     /* MRW trigger on cell optical depth; <=0 off */
  double mrw_gamma;   /* MRW sphere size in Rosseland mean free paths */
  uint64_t max_int;   /* interaction cap per packet; 0 = none */
  int32_t ntheta;     /* SED polar bins (equal in cos theta) */
  int32_t model_id;
  int32_t record;     /* fill per-packet records */
  int32_t tau_mode;   /* ORC_TAU_FLIGHT or ORC_TAU_PER_CELL */
  uint64_t src_strata;/* m > 0: packet pid takes source-spectrum stratum pid mod m
                         (m equal-energy source bins, Eq. 1); 0 = plain draw */
  double pah_nc;      /* carbon atoms per PAH molecule (Eq. 8); <= 0: no dissociation */
  double pah_tcool;   /* PAH cooling time in s over which absorbed energy adds up */
  int32_t sh_order;   /* L + 1 > 0: keep the scattering events of the imaged wavelengths
                         as spherical-harmonic moments up to degree L (sect. 4: scattered
                         light toward any observer after the run); 0 = off */
  int32_t pad2;
} orc_opts;

typedef struct {
  uint64_t pid;
  double pos[3], dir[3];
  int32_t j, status;
  double weight;
  uint64_t n_cross, n_scat, n_abs, n_mrw, n_lucy;
  double min_margin;
} orc_record;

typedef struct {
  uint64_t packets, escaped, killed, pah_stopped, crossings, scatters,
      absorptions, mrw_steps, lucy_deposits, clamped_T;
} orc_stats;

typedef struct {
  uint64_t *k;        /* [ns][cells] absorption counts (non-thin cells) */
  double *epath;      /* [ns][cells] path-length energy (Lucy + MRW) erg/s */
  double *T;          /* [ns][cells] temperatures (frozen input / final) */
  double *esnap;      /* [ns][cells] epoch snapshot of E (BW_EPOCH) */
  double *tt;         /* [ns][cells] epoch temperatures (BW_EPOCH) */
  uint8_t *tvalid;    /* [ns][cells] */
  uint32_t *kpah;     /* [cells] PAH absorptions of pass 1 */
  uint64_t *sed;      /* [ntheta][nl] escaped packet counts */
  double *ssca;       /* [nview][nimg][cells] HG-weighted scattering, erg/s/sr */
  double *sh;         /* [nimg][(L+1)^2][cells] moments sum xi g^l Y_lm(d_in), erg/s
                         (sh_order = L + 1 > 0) */
  orc_record *rec;    /* [n] when record */
  orc_stats st;
} orc_state;

/* Philox4x32-10 (Salmon et al. 2011) and the 24-bit open-interval uniform */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u24(uint32_t x);
/* u_d of the per-packet stream (counter layout in mcrt_oracle.c) */
double orc_draw(uint64_t seed, uint64_t pid, uint32_t iter, uint32_t model,
                uint32_t tag, uint64_t d);

/* frequency grid: nu_j = c/lambda_j, quadrature weights w_j = bin width in Hz */
void orc_freq_grid(int nl, const double *lam_um, double *nu, double *w);
double orc_planck(double nu, double T);
double orc_dplanck_dT(double nu, double T);
double orc_phi(const orc_model *m, int s, double T);            /* sum w kabs B */
double orc_invert_T(const orc_model *m, int s, double rhs);     /* Eq. 4 */
/* Rosseland mean of the mixture extinction and Planck mean of species s
 * absorption at T (sect. 3.2 diffusion step), on the model's quadrature. */
double orc_rosseland(const orc_model *m, double T);
double orc_planck_mean(const orc_model *m, int s, double T);
double orc_hg_mu(double g, double u);                           /* Eq. 15 CDF */
double orc_hg_phase(double g, double mu);                       /* Eq. 15 */
double orc_mrw_survival(double y);
double orc_mrw_solve(double u);

/* Real orthonormal spherical harmonics Y_lm(d) for l <= lmax, m = -l..l,
 * at index l^2 + l + m (m > 0: cos(m phi) terms, m < 0: sin(|m| phi)). */
void orc_ylm(int lmax, const double d[3], double *y);
/* Scattered-light sums toward direction k from the moments of an order
 * sh_order run: out[q][c] = sum_lm Y_lm(k) sh[q][lm][c] (erg/s/sr), the
 * Henyey-Greenstein phase function expanded in Legendre terms g^l. */
void orc_sh_view_sums(const orc_model *m, int sh_order, const double *sh, const double k[3],
                      double *out);

/* Leaf cells of the model (cubes plus sub-cubes) */
int64_t orc_nleaf(const orc_model *m);
/* Leaf geometry: lower corner, edge and density of leaf `leaf`. */
void orc_leaf_box(const orc_model *m, int64_t leaf, double lo[3], double *h, double *rho);

/* Voxel walk from p0 along d through the leaf cells, starting in the leaf
 * that holds p0 (a point on a face belongs to the leaf that d points into).
 * Writes up to maxseg (leaf, length) pairs; returns the number of segments,
 * or -1 if maxseg was too small. */
int orc_dda(const orc_model *m, const double p0[3], const double d[3],
            int maxseg, int64_t *cells, double *lens);

/* 1 if the PAH of cell c (pass-1 count kpah) dissociate under Eq. 8. */
int orc_pah_dissociates(const orc_model *m, const orc_opts *o, uint32_t kpah, int64_t c);
/* Thin-limit initial temperatures at cell centres. */
void orc_init_T(const orc_model *m, double *T);
/* Monte Carlo transport of packets [first, first+n). */
int orc_run(const orc_model *m, const orc_opts *o, uint64_t first, uint64_t n,
            uint64_t seed, orc_state *st);
/* Second PAH stage: cells re-emit their pass-1 PAH absorptions. With
 * pah_nc > 0, a cell whose PAH molecules absorb at least E_crit = N_C/2 eV
 * within a cooling time (Eq. 8) dissociates them: its packets start from
 * the source instead, as source packets. */
int orc_pah_pass(const orc_model *m, const orc_opts *o, uint64_t seed, orc_state *st);
/* Eq. 4 for every cell and species from the current tallies. */
void orc_finalize_T(const orc_model *m, const orc_opts *o, orc_state *st);

/* Ray-tracer (sect. 4): images [nview][nimg][npy][npx], SED [nview][nimg].
 * rho_rt (NULL = model density) is the density used for extinction; the
 * source function keeps the model's values (emissivity per unit mass). */
int orc_raytrace(const orc_model *m, int rt_mode, const double *T, const double *ssca,
                 const double *rho_rt, int npx, int npy, double *img, double *sed);
/* Gradient of sum(w_img*img) + sum(w_sed*sed) with respect to rho_rt [cells]. */
int orc_raytrace_adjoint(const orc_model *m, int rt_mode, const double *T, const double *ssca,
                         const double *rho_rt, int npx, int npy, const double *w_img,
                         const double *w_sed, double *drho);

/* Voxelizers (model set-up). */
void orc_voxelize_torus(int nx, int ny, int nz, const double origin[3], double dcell,
                        int ncl, const double *centres, double r_clump, double rho_clump,
                        double rho_inter, double r_in, double r_out, double sin_theta1,
                        double *rho);
void orc_voxelize_shell(int nx, int ny, int nz, const double origin[3], double dcell,
                        double rho0, double r_in, double r_out, double power, double *rho);

#ifdef __cplusplus
}
#endif
#endif
