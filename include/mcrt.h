/*
 * mcrt.h - C ABI of the MI355X Monte Carlo dust radiative-transfer library.
 *
 * Method: Heymann & Siebenmorgen, "GPU-based Monte Carlo dust radiative
 * transfer scheme applied to AGN". Photon packets of equal energy (sect. 2,
 * Eq. 1) march cell by cell through a Cartesian dust grid, sample optical
 * depth (Eqs. 2-3), scatter with the Henyey-Greenstein phase function
 * (Eq. 15) or are absorbed and re-emitted (Eqs. 4-5 iterative scheme, Eq. 10
 * Bjorkman & Wood), with Lucy's estimator in thin cells (sect. 3.1, Eq. 9),
 * a modified random walk in very thick cells (sect. 3.2) and the PAH
 * two-stage emission (sect. 2.1, Eqs. 6-7). A ray-tracer (sect. 4, Eqs.
 * 11-17) forms images and SEDs; its adjoint gives d(loss)/d(density).
 *
 * Conventions
 *  - cgs units; wavelengths in micrometres, strictly increasing.
 *  - Grid: nx*ny*nz cubic cells of side `dcell` cm, low corner `origin`;
 *    linear index (iz*ny + iy)*nx + ix (x fastest).
 *  - Frequency integrals are sums over the wavelength grid with bin widths
 *    w_j (Hz) spanning the geometric midpoints of neighbouring wavelengths.
 *  - Per-species arrays are [ns][cells] or [ns][nl], species fastest-outer.
 *  - `mem` says where a caller pointer lives: MCRT_HOST or MCRT_DEVICE
 *    (a device pointer from the same GPU, e.g. torch.Tensor.data_ptr()).
 *  - `stream` is a hipStream_t (NULL = default stream). Calls enqueue work
 *    on it and return; results written to caller memory are complete after
 *    the caller synchronises the stream. Host outputs are synchronous.
 *  - Ownership: mcrt_set_* copy their inputs into library-owned device
 *    memory; the library never keeps or frees caller pointers.
 *  - Errors: every call returns an mcrt_status; mcrt_last_error(ctx) holds
 *    the message until the next call on that context. Nothing is printed.
 *  - One context per host thread at a time; calls on one context are not
 *    thread-safe. Floating-point type of grids, images and gradients is the
 *    context precision (MCRT_FP64 -> double, MCRT_FP32 -> float).
 */
#ifndef MCRT_H
#define MCRT_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcrt_ctx mcrt_ctx;

typedef enum {
  MCRT_OK = 0,
  MCRT_EINVAL = -1,  /* bad argument (shape, value, pointer) */
  MCRT_ENOMEM = -2,  /* device allocation failed */
  MCRT_ESTATE = -3,  /* call out of order (e.g. run before grid/dust/sources) */
  MCRT_EDEVICE = -4  /* HIP runtime or kernel launch error */
} mcrt_status;

enum { MCRT_HOST = 0, MCRT_DEVICE = 1 };
enum { MCRT_FP64 = 0, MCRT_FP32 = 1 };
/* Re-emission rule: FROZEN = iterative scheme of sect. 2 (Eq. 5 with the
 * previous pass's temperatures, n_iter passes, Eq. 4 after each);
 * BW_EPOCH = Bjorkman & Wood (Eq. 10) with temperatures refreshed at fixed
 * packet-id epochs (deterministic); BW_TICKET = Bjorkman & Wood with the
 * temperature updated at every absorption (sect. 3.3; order set by the GPU). */
enum { MCRT_FROZEN = 0, MCRT_BW_EPOCH = 1, MCRT_BW_TICKET = 2 };
enum { MCRT_TAU_FLIGHT = 0, MCRT_TAU_PER_CELL = 1 };
enum { MCRT_RT_EXT = 0, MCRT_RT_ABS_LITERAL = 1 };
enum { MCRT_SCAT_HG = 0, MCRT_SCAT_GFACTOR = 1 };
enum { MCRT_SSCA_PEELOFF = 0, MCRT_SSCA_MOMENTS = 1 };
enum { MCRT_ESCAPED = 1, MCRT_KILLED = 2, MCRT_PAH_STOP = 3 };

typedef struct {
  int32_t mode;              /* MCRT_FROZEN / MCRT_BW_EPOCH / MCRT_BW_TICKET */
  int32_t n_iter;            /* FROZEN passes (paper: 3-5) */
  uint64_t epoch_packets;    /* BW_EPOCH epoch length in packet ids (>= 1) */
  uint64_t n_total;          /* packets defining xi = L/n_total (0 -> n) */
  double lucy_tau;           /* Lucy threshold on rho*max(kext)*dcell; <= 0 off (paper 1e-2) */
  double mrw_tau;            /* MRW on cells with Rosseland depth > mrw_tau; <= 0 off */
  double mrw_gamma;          /* MRW sphere >= gamma Rosseland mean free paths */
  uint64_t max_interactions; /* per-packet cap; 0 = none; capped packets are killed */
  int32_t sed_theta_bins;    /* photon-counting SED bins, equal in cos(theta) */
  int32_t record;            /* 1: keep one mcrt_packet_record per packet */
  int32_t blocks_per_cu;     /* 256-thread blocks per compute unit of the emission and
                                interaction kernels of a round (0 = 3 where the FP32 walk
                                takes the fast interaction kernel, else 2; 1..32) */
  int32_t queue_depth;       /* packets per wavefront queue (0 = 2^25; 64..2^26) */
  int32_t walk_blocks_per_cu; /* 256-thread blocks per compute unit of the walk kernel
                                (0 = 4; 1..32) */
  int32_t tau_mode;          /* MCRT_TAU_FLIGHT: one optical-depth draw per flight (Eq. 2);
                                MCRT_TAU_PER_CELL: a new draw on entering each cell, the
                                packet interacting in the cell iff the segment's depth
                                exceeds -ln(draw) (sect. 2, footnote to the interaction
                                test) */
  uint64_t src_strata;       /* m > 0: m equal-energy source bins (Eq. 1), packet id p
                                drawing its source wavelength inside stratum p mod m of
                                the source spectrum's distribution; 0 = plain draw */
  double pah_nc;             /* PAH photodissociation (sect. 2.1, Eq. 8) in mcrt_run_pah:
                                carbon atoms per molecule N_C; <= 0 = off */
  double pah_tcool;          /* cooling time (s): a cell whose molecules (mass N_C 12 amu)
                                absorb E_PAH = kpah xi m_PAH t_cool / (f_pah rho V) >=
                                N_C/2 eV dissociates, and its pass-2 packets start from
                                the sources as source packets */
  int32_t sh_order;          /* L + 1 (0..9): keep every scattering event at an imaged
                                wavelength as moments sum xi g^l Y_lm(d_in), l <= L, per
                                cell (real orthonormal spherical harmonics of the incoming
                                direction), so that scattered light toward any observer is
                                formed after the run (sect. 4); the HG phase function is
                                sum_l g^l sum_m Y_lm(d) Y_lm(k), cut after degree L. 0 = off.
                                Moments are kept until reset or a change of the imaged
                                wavelengths (mcrt_set_views with other indices) */
  int32_t pad_;
} mcrt_run_opts;

typedef struct {
  uint64_t packets, escaped, killed, pah_stopped, crossings, scatters,
      absorptions, mrw_steps, lucy_deposits, clamped_T;
  double kernel_ms;          /* device time of the transport launches */
} mcrt_run_stats;

typedef struct {
  uint64_t pid;
  double pos[3], dir[3];     /* escape/stop point (cm) and direction */
  int32_t j, status;         /* wavelength index, MCRT_ESCAPED/KILLED/PAH_STOP */
  double weight;             /* packet energy xi (erg/s) */
  uint64_t n_cross, n_scat, n_abs, n_mrw, n_lucy;
  double min_margin;         /* distance of the closest decision from a tie */
} mcrt_packet_record;

/* Create a context on HIP device `device` computing in `precision`
 * (MCRT_FP64 or MCRT_FP32; FP32 keeps Eq. 4 and the diffusion solve in
 * FP64 and accumulates energies in FP64). *out is NULL on failure. */
mcrt_status mcrt_create(mcrt_ctx **out, int device, int precision);
/* Free all device memory of the context. NULL is accepted. */
void mcrt_destroy(mcrt_ctx *ctx);
/* Message of the last failed call on ctx ("" if none); NULL ctx -> creation error. */
const char *mcrt_last_error(const mcrt_ctx *ctx);

/* Grid of sect. 2: cubes of constant density rho (g/cm^3, [nz][ny][nx]).
 * dtype MCRT_FP64 (double) or MCRT_FP32 (float); converted to the context
 * precision. EINVAL: n <= 0 or more than 262143 cells on an axis,
 * dcell <= 0, rho negative or not finite. Resets tallies and temperatures. */
mcrt_status mcrt_set_grid(mcrt_ctx *ctx, int nx, int ny, int nz, const double origin[3],
                          double dcell, const void *rho, int dtype, int mem);
/* One level of refinement (sect. 2: each cube divided into sub-cubes of
 * their own density, for a finer sampling where needed): cube c (linear
 * index, x fastest) is divided into ref[c]^3 sub-cubes of edge dcell/ref[c]
 * when ref[c] >= 2 (at most 16), whole when 0 or 1. rho_sub holds the
 * sub-cube densities (g/cm^3, dtype MCRT_FP64 or MCRT_FP32, host memory),
 * cube after cube in linear order, x fastest inside a cube; nsub must equal
 * the sum of ref[c]^3 over the divided cubes. The cells of every per-cell
 * array (tallies, temperatures, scattering sums, densities, gradients)
 * become the leaves: first the cubes (a divided cube's entry is unused),
 * then the sub-cubes in rho_sub's order. Packets and rays walk the leaves,
 * and Lucy's thin test, diffusion steps, Eq. 4 and the source functions use
 * each leaf's own edge, volume and density. ref NULL (nsub 0) removes the
 * refinement. Call after the grid; set_grid and the voxelizers reset it.
 * Resets tallies. EINVAL: bad ref value, nsub mismatch, negative or
 * non-finite density. ESTATE before the grid. */
mcrt_status mcrt_set_refinement(mcrt_ctx *ctx, const uint8_t *ref, const void *rho_sub,
                                uint64_t nsub, int dtype);
/* Clumpy torus of sect. 6 (Eq. 21 clump centres given, host [n][3] cm):
 * a cell takes rho_clump if its centre lies inside any clump (overlaps keep
 * the single-clump density), rho_inter inside the wedge r_in <= r <= r_out,
 * |z| <= r sin_theta1, else 0. Builds the grid on the device (grid limits
 * as for mcrt_set_grid). */
mcrt_status mcrt_voxelize_torus(mcrt_ctx *ctx, int nx, int ny, int nz, const double origin[3],
                                double dcell, int n_clumps, const double *centres,
                                double r_clump, double rho_clump, double rho_inter,
                                double r_in, double r_out, double sin_theta1);
/* Spherical shell rho0 (r_in/r)^power on [r_in, r_out], cell averages by
 * an 8^3 Gauss-Legendre rule: power 2 is the r^-2 shell of sect. 5.1, power
 * 0 the constant-density envelope of the sect. 3.6 run-time comparison
 * (Table 1). EINVAL on rho0 < 0, r_in <= 0, r_out < r_in or a non-finite
 * value, and on the grid limits of mcrt_set_grid. */
mcrt_status mcrt_voxelize_shell(mcrt_ctx *ctx, int nx, int ny, int nz, const double origin[3],
                                double dcell, double rho0, double r_in, double r_out,
                                double power);

/* Dust of sect. 2: n_lambda wavelengths (um, increasing, 2..256), n_species
 * (1..4) with mass fractions and kabs, ksca (cm^2 per g of dust) and HG g,
 * each [ns][nl] (host). pah_species = -1 or the species treated as PAH
 * (sect. 2.1) with n_pah_rows emissivity rows eps_n [rows][nl] and rows-1
 * increasing edges on the absorbed PAH power per PAH mass and steradian. */
mcrt_status mcrt_set_dust(mcrt_ctx *ctx, int n_lambda, const double *lambda_um, int n_species,
                          const double *mass_frac, const double *kabs, const double *ksca,
                          const double *g, int pah_species, int n_pah_rows,
                          const double *pah_emis, const double *pah_row_edges);
/* Point sources of sect. 2 (host arrays): positions [n][3] cm inside the
 * grid, luminosities erg/s, spectral shape ~L_nu [n][nl] or NULL with
 * blackbody temperatures t_bb [n]; 1 <= n <= 8. Each packet of Eq. 1 leaves
 * a source chosen in proportion to its luminosity, with a frequency bin
 * drawn from that source's w_j L_nu,j. Shapes are normalised to sum_j w_j
 * L_nu,j = L. ESTATE before set_dust and the grid; EINVAL for a source
 * outside the grid, a negative luminosity or an empty spectrum. */
mcrt_status mcrt_set_sources(mcrt_ctx *ctx, int n_src, const double *pos_cm, const double *lum,
                             const double *lnu_shape, const double *t_bb);
/* Observer views for scattering events and the ray-tracer (sect. 4):
 * (theta, phi) degrees [n][2] (n <= 16), imaged wavelength indices
 * [n_img] (<= 16, distinct), distance D in cm. */
mcrt_status mcrt_set_views(mcrt_ctx *ctx, int n_views, const double *theta_phi_deg,
                           int n_img, const int32_t *lambda_idx, double distance_cm);

/* Zero counts, energies, PAH counts, SED, scattering events and epoch state. */
mcrt_status mcrt_reset(mcrt_ctx *ctx, void *stream);
/* Initial guess of the iterative scheme: optically thin equilibrium
 * temperature at every cell centre (Eq. 4 with the unattenuated sources). */
mcrt_status mcrt_init_temperatures(mcrt_ctx *ctx, void *stream);
/* Replace temperatures [ns][cells] (FP64). */
mcrt_status mcrt_set_temperatures(mcrt_ctx *ctx, const double *T, int mem, void *stream);
/* Replace the HG-weighted scattering sums [views][n_img][cells] (FP64, erg/s/sr). */
mcrt_status mcrt_set_scattering(mcrt_ctx *ctx, const double *ssca, int mem, void *stream);

/* Transport of sect. 2-3 for packets first .. first+n-1: emission (Eq. 1),
 * optical depth per cell against -ln(zeta) (Eqs. 2-3), albedo split, HG
 * scattering (Eq. 15) with the scattering sums of the views (Eq. 16 source
 * term), absorption with re-emission by Eq. 5 or Eq. 10 (mode), Lucy's
 * estimator in thin cells (sect. 3.1, Eq. 9), the diffusion step of
 * sect. 3.2 in very thick cells, photon counting of escapes (sect. 4).
 * Random numbers: the counter-based stream of `seed` (Philox4x32-10 keyed
 * by seed, counter = draw block, packet id, iteration, model and stream
 * tag). Tallies accumulate across calls, so a run split into consecutive
 * ranges equals the whole run (FROZEN resets per pass). `stats` (nullable)
 * receives counters after the call completes (the call then synchronises
 * the stream). ESTATE before grid, dust and sources are set; EINVAL for bad
 * options or packet ids beyond 2^48; ENOMEM when queues or records do not
 * fit on the device (the context stays usable). */
mcrt_status mcrt_run_packets(mcrt_ctx *ctx, uint64_t first, uint64_t n, uint64_t seed,
                             const mcrt_run_opts *opts, mcrt_run_stats *stats, void *stream);
/* Second PAH stage (sect. 2.1): every cell re-emits its pass-1 PAH
 * absorptions with wavelengths from its eps_n row (Eq. 7) and the packets
 * are transported as in run_packets (ids n_total + prefix). */
mcrt_status mcrt_run_pah(mcrt_ctx *ctx, uint64_t seed, const mcrt_run_opts *opts,
                         mcrt_run_stats *stats, void *stream);
/* Eq. 4 for every cell and thermal species from the tallies: T_out
 * [ns][cells] FP64 (PAH species and empty cells 0); E_out (nullable)
 * absorbed power [ns][cells] FP64 erg/s. */
mcrt_status mcrt_temperatures(mcrt_ctx *ctx, double *T_out, double *E_out, int mem, void *stream);
/* Eq. 4 on the device for n given right-hand sides rhs = E/(4 pi f rho V)
 * (erg/s/g per species mass, host arrays): T_out[i] for species `species`.
 * method 0: bracketed Newton to 1e-14 in ln T (used by Eq. 4 finalisation
 * and epoch temperatures); 1: cubic Hermite table of ln T(ln Phi) (used at
 * every absorption of BW_TICKET), about 1e-10 relative. */
mcrt_status mcrt_invert_temperature(mcrt_ctx *ctx, int species, uint64_t n, const double *rhs,
                                    double *T_out, int method);
/* Copy of the context's temperature field [ns][cells] FP64 as it stands
 * (initial guess, values set by the caller, or the last Eq. 4 result);
 * unlike mcrt_temperatures nothing is recomputed. */
mcrt_status mcrt_get_temperatures(mcrt_ctx *ctx, double *T_out, int mem, void *stream);
/* Copy of the grid density [cells] in the context precision. */
mcrt_status mcrt_density(mcrt_ctx *ctx, void *rho_out, int mem, void *stream);
/* Raw tallies: counts [ns][cells] u64, path energy [ns][cells] FP64,
 * PAH counts [cells] u32 (each nullable). */
mcrt_status mcrt_tallies(mcrt_ctx *ctx, uint64_t *k_out, double *epath_out, uint32_t *kpah_out,
                         int mem, void *stream);
/* Photon-counting SED (sect. 4): flux density [theta_bins][nl] in
 * erg/s/cm^2/Hz at the view distance (counts * xi / (dOmega D^2 w_j)),
 * and raw counts (nullable). */
mcrt_status mcrt_sed(mcrt_ctx *ctx, double *sed_out, uint64_t *counts_out, int mem, void *stream);
/* HG-weighted scattering sums [views][n_img][cells] FP64. */
mcrt_status mcrt_scattering(mcrt_ctx *ctx, double *ssca_out, int mem, void *stream);
/* Copy min(n, recorded) packet records of the last run_packets/run_pah
 * call with record = 1 (host or device destination): each packet's end
 * state (escape point and direction for the photon counting of sect. 4,
 * wavelength bin, packet energy xi of Eq. 1) and its event counts. ESTATE
 * when the last run kept no records. */
mcrt_status mcrt_packet_records(mcrt_ctx *ctx, mcrt_packet_record *out, uint64_t n, int mem);

/* Ray-tracer (sect. 4, Eqs. 11-17): npx*npy parallel rays per view over a
 * square field of side sqrt(3)*max box edge, front to back; per cell
 * S = sum_s f_s kabs_s B(T_s)/kext + Ssca/(V w rho kext) and
 * I += T S (1 - e^-dtau), T *= e^-dtau with dtau = rho kext l; pixel flux
 * A_pix I / D^2 plus attenuated point sources. img_out [views][n_img][npy][npx]
 * (context precision), sed_out [views][n_img] FP64 (nullable).
 * rho_rt (nullable, device, context precision) replaces the grid density in
 * dtau only; S keeps the grid's values (emissivity per unit mass fixed). */
mcrt_status mcrt_raytrace_image(mcrt_ctx *ctx, int npx, int npy, const void *rho_rt,
                                void *img_out, double *sed_out, int mem, void *stream);
/* Formal solution of the ray-tracer and its adjoint. MCRT_RT_EXT (default):
 * the chord form above. MCRT_RT_ABS_LITERAL: Eqs. 13-14 as printed (sect. 4):
 * optical depth K dtau with K = sum_s f_s kabs_s (absorption only), and each
 * cell a ray crosses adds C = (1 - exp(-rho K dcell)) S_e + I_s attenuated
 * from the cell's border to the observer, where tau_cell = rho K dcell is
 * the face-to-face depth, S_e = sum_s f_s kabs_s B(T_s)/K (B(T) for one
 * species) and I_s = Ssca/(dnu dcell^2) is Eq. 16's scattered intensity with
 * the event energies spread over the cell's face. C comes from the grid
 * density; rho_rt enters only the attenuation. Point sources are attenuated
 * with K. EINVAL on another mode. */
mcrt_status mcrt_set_raytrace_mode(mcrt_ctx *ctx, int rt_mode);

/* Scattering law of the transport and the peel-off sums (sect. 4):
 * MCRT_SCAT_HG (default), Henyey-Greenstein with the given g (Eq. 15); or
 * MCRT_SCAT_GFACTOR, the g-factor approximation: isotropic scattering with
 * kappa_sca (1 - g) per species and wavelength (albedo and extinction follow).
 * Rebuilds the tables. EINVAL on another law. */
mcrt_status mcrt_set_scattering_law(mcrt_ctx *ctx, int law);
/* Scattered light of the ray-tracer's source functions (sect. 4, Eq. 16:
 * the scattering events seen from the observer): MCRT_SSCA_PEELOFF
 * (default), the per-view sums of the transport; MCRT_SSCA_MOMENTS, the
 * moments of the last run with sh_order > 0 evaluated toward each view set
 * (any views, set after the run) as sum_lm Y_lm(k_v) M_lm. EINVAL on another
 * value. */
mcrt_status mcrt_set_scattered_light(mcrt_ctx *ctx, int source);
/* Moments of the scattering events (sect. 4: the stored events, kept as
 * sum xi g^l Y_lm(d_in) per cell and imaged wavelength; erg/s),
 * [n_img][order^2][cells] with index l^2 + l + m, FP64, host or device
 * destination (mem); *order (nullable) receives L + 1 (0 when none). out
 * NULL: order only. ESTATE when there are none. */
mcrt_status mcrt_scattering_moments(mcrt_ctx *ctx, double *out, int *order, int mem,
                                    void *stream);

/* mcrt_raytrace_image for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with img_out
 * [views][n_img][npy][npx] (context precision) and sed_out [views][n_img]
 * (FP64, nullable) in device memory only. The source functions go to a
 * static device array of 64 MiB per GPU (held until the process ends), so
 * views * cells * n_img * (4 FP32 | 8 FP64) bytes must fit: EINVAL beyond.
 * ESTATE unless the context's tallies and scattering sums for the current
 * views already exist (after mcrt_reset, a run, or mcrt_set_temperatures
 * with views set). Calls no allocating routine. Every call on one GPU
 * shares its array: calls that overlap on one GPU (several streams or
 * threads) race and must be serialised by the caller. */
mcrt_status mcrt_raytrace_image_noalloc(mcrt_ctx *ctx, int npx, int npy, const void *rho_rt,
                                        void *img_out, double *sed_out, void *stream);
/* Adjoint of mcrt_raytrace_image: given dL/dimg (context precision,
 * nullable) and dL/dsed (FP64, nullable), writes dL/drho_rt [cells]
 * (context precision). Transmittance is recomputed in a second front-to-
 * back sweep per ray; nothing of the forward pass is stored. */
mcrt_status mcrt_raytrace_adjoint(mcrt_ctx *ctx, int npx, int npy, const void *rho_rt,
                                  const void *dL_dimg, const double *dL_dsed, void *dL_drho,
                                  int mem, void *stream);

/* Batched transport: n_models (<= 1024) contexts (same device and
 * precision, each with grid, dust and sources set) run packets
 * 0..n_packets[m]-1 with seeds[m]. Every kernel of a wavefront round covers
 * all models (blocks visit the models in turn and take queue entries of
 * each); eight rounds are captured in one HIP graph on the library's
 * stream and replayed on the caller's stream until no model has packets
 * left. Each model draws the same Philox streams as its own
 * mcrt_run_packets with the same seed (seeds distinguish the models), so
 * FROZEN batches reproduce per-model runs exactly. Modes FROZEN (n_iter =
 * 1) and BW_TICKET. Tallies are reset first and temperatures finalised
 * (Eq. 4, FP64) afterwards. stats (nullable) [n_models]. */
mcrt_status mcrt_run_batch(mcrt_ctx *const *models, int n_models, const uint64_t *n_packets,
                           const uint64_t *seeds, const mcrt_run_opts *opts,
                           mcrt_run_stats *stats, void *stream);

/* Device time in ms of the last ray-tracer forward / adjoint pixel-ray
 * kernel (without the SED reduction and point-source terms) and of the last
 * transport launch sequence (HIP events on the call's stream). */
mcrt_status mcrt_last_timings(const mcrt_ctx *ctx, double *transport_ms, double *rt_fwd_ms,
                              double *rt_adj_ms);
/* Device time in ms of the last build of the ray-tracer's source functions
 * S (sect. 4, Eq. 14 emission plus the Eq. 16 scattering term, per view,
 * cell and imaged wavelength), which mcrt_raytrace_image runs whenever the
 * temperatures or scattering sums changed since the last build; 0 before
 * any build. EINVAL for NULL arguments. */
mcrt_status mcrt_last_source_build_ms(const mcrt_ctx *ctx, double *ms);

/* n draws of the wavelength bin that species `species` (thermal) re-emits
 * at temperature T (K) after an absorption, taken exactly as the transport
 * takes them: mode MCRT_FROZEN gives Eq. 5 (weights w kabs B), the B&W
 * modes Eq. 10 (weights w kabs dB/dT). FP64 contexts walk the inverse CDF;
 * FP32 contexts sample by rejection from a tabulated envelope (exact in
 * distribution). Draw i uses Philox stream (seed, i, tag 7). counts: host
 * [n_lambda], overwritten. For validation of the sampler. */
mcrt_status mcrt_sample_reemission(mcrt_ctx *ctx, int species, int mode, double T, uint64_t n,
                                   uint64_t seed, uint64_t *counts);

/* Device time in ms of the emission, walk and interaction kernels summed
 * over the rounds of the last mcrt_run_packets / mcrt_run_pah call (HIP
 * events around each kernel on the call's stream), and the number of
 * rounds. Any pointer may be NULL. Batched runs are not timed by phase. */
mcrt_status mcrt_phase_timings(const mcrt_ctx *ctx, double *emit_ms, double *walk_ms,
                               double *interact_ms, uint64_t *rounds);

#ifdef __cplusplus
}
#endif
#endif
