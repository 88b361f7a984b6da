// mcrt_transport.hip - Monte Carlo packet transport (sect. 2-3 of Heymann &
// Siebenmorgen) for gfx950 as wavefront rounds over packet queues.
//
// A packet's history is a chain of events: emission (Eq. 1 packets,
// isotropic directions), optional modified random walk steps (sect. 3.2),
// one flight of sampled optical depth through the voxel grid (Eqs. 2-3)
// with Lucy deposits in thin cells (Eq. 9), then an interaction:
// Henyey-Greenstein scattering (Eq. 15) or absorption with re-emission by
// Eq. 5 (iterative scheme) or Eq. 10 (Bjorkman & Wood). A round moves
// every live packet by one flight and one interaction: an emission kernel
// tops the flight-ready queue up with new packets, the walk kernel (small
// register file, high occupancy) takes every queued packet through its
// flight, and the interaction kernel (FP64 Eq. 4, re-emission spectra)
// handles the packets whose flight ended in the grid. Each kernel's blocks
// stage their model's tables in LDS; escapes are counted into an LDS copy
// of the photon-counting SED.
#include <type_traits>

#include "mcrt_internal.h"
#include "mcrt_scatter.h"

namespace mcrt {

template <typename R>
struct Pkt {
  R p[3], d[3];
  int c[3];
  uint32_t fpk;  // sub-cube of a divided cube c (fine_pack), 0 in a whole cube
  int j, status;
  R rho;  // density of cell c after a flight that ends in an interaction
  uint64_t pid;
  Rng rng;
  uint32_t n_cross, n_scat, n_abs, n_mrw, n_lucy, n_int;
  double mm;
};

template <typename R>
struct Ctx {
  const ModelDev *M;
  TabOff o;
  const double *dt;   // LDS double table
  const R *rt;        // LDS R table
  const int *imgmap;  // LDS
  uint32_t *sed;      // LDS SED counts
  const R *rho;
  int64_t nc;
  unsigned long long *st;  // LDS block counters [NSTAT]
  R rho_thin;              // FP32 walk: lucy_tau / (max kext dcell), 0 when Lucy is off
  R og[3], dc;             // grid origin and cell size in the walk precision
  int nx, ny, nz;
  const R *rho_b;          // bricked density (brick_index)
  int nbx, nby;
  const uint32_t *occ;     // walk: LDS copy of the brick-run occupancy bits (else null)
  int osh;                 // bricked-cell index >> osh is its run
};

__device__ __forceinline__ void stat_add(unsigned long long *st, int i, unsigned long long v) {
  atomicAdd(&st[i], v);
}

// Cell of a start point, in FP64 in both precisions: a source on a cell
// vertex must land on the face decision exactly (in FP32, (p - origin) /
// dcell can miss the integer by an ulp and start the packet one cell short,
// adding a zero-length crossing).
template <typename R>
__device__ __forceinline__ void start_cell(const ModelDev &M, const R p[3], const R d[3], int c[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double q = ((double)p[k] - M.origin[k]) / M.dcell;
    const double f = floor(q);
    int ci = (int)f;
    if (q == f && d[k] < (R)0) ci -= 1;
    c[k] = ci;
  }
}

// Isotropic direction, evaluated in FP64 in both precisions (sqrt(1 - mu^2)
// cancels near the poles in FP32) and rounded to the walk type.
template <typename R>
__device__ __forceinline__ void iso_dir(double uphi, double umu, R d[3]) {
  double phi = 2.0 * PI_D * uphi;
  double mu = 1.0 - 2.0 * umu;
  double s = sqrt(fmax(0.0, 1.0 - mu * mu));
  d[0] = (R)(s * cos(phi));
  d[1] = (R)(s * sin(phi));
  d[2] = (R)mu;
}

// Smallest index whose ascending running sum of f[q*stride] reaches u times
// the total (f read from LDS).
template <typename R, bool REC, typename T>
__device__ __forceinline__ int pick_asc(const T *f, int stride, int n, R u, double &mm) {
  R tot = (R)0;
  for (int q = 0; q < n; ++q) tot += (R)f[q * stride];
  R target = u * tot, c = (R)0;
  for (int q = 0; q < n; ++q) {
    R prev = c;
    c += (R)f[q * stride];
    if (c >= target) {
      if (REC && tot > (R)0 && n > 1) {
        upd_margin(mm, (double)((c - target) / tot));
        upd_margin(mm, (double)((target - prev) / tot));
      }
      return q;
    }
  }
  return n - 1;
}

// Inverse CDF over ascending frequency (descending index) of a spectrum
// given by a functor: the first j (from n-1 down) whose running sum reaches
// u times the total, 0 if none does. The running sums are the plain
// sequential ones. A first pass records them at the start of each of NB
// chunks; the second pass re-walks only the chunk that holds the answer,
// from its recorded start, so it adds the same terms in the same order.
// Lanes then differ by at most one chunk of work instead of a whole pass.
template <typename R, bool REC, typename F>
__device__ __forceinline__ int pick_desc_fn(int n, R u, double &mm, F f) {
  constexpr int NB = 8;
  const int ch = (n + NB - 1) / NB;
  R cb[NB + 1];
  R c = (R)0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    cb[b] = c;
    const int hi = n - 1 - b * ch;
    const int lo = hi - ch + 1 > 0 ? hi - ch + 1 : 0;
    for (int j = hi; j >= lo; --j) c += f(j);
  }
  cb[NB] = c;
  const R tot = c, target = u * tot;
  // first chunk whose end sum reaches the target (the last one otherwise)
  int bs = NB - 1;
  R c0 = cb[NB - 1];
#pragma unroll
  for (int b = NB - 2; b >= 0; --b) {
    if (cb[b + 1] >= target) { bs = b; c0 = cb[b]; }
  }
  const int hi = n - 1 - bs * ch;
  const int lo = hi - ch + 1 > 0 ? hi - ch + 1 : 0;
  c = c0;
  for (int j = hi; j >= lo; --j) {
    const R prev = c;
    c += f(j);
    if (c >= target) {
      if (REC && tot > (R)0) {
        upd_margin(mm, (double)((c - target) / tot));
        upd_margin(mm, (double)((target - prev) / tot));
      }
      return j;
    }
  }
  return 0;
}

// The same pick for a fixed spectrum stored as running sums cum[j] (weights
// of j .. n-1 added from n-1 down): the largest j with cum[j] >= u cum[0],
// found by bisection.
template <bool REC>
__device__ __forceinline__ int pick_desc_cum(const double *cum, int n, double u, double &mm) {
  const double tot = cum[0], target = u * tot;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cum[mid] >= target) lo = mid; else hi = mid - 1;
  }
  if (REC && tot > 0.0) {
    const double prev = lo + 1 < n ? cum[lo + 1] : 0.0;
    upd_margin(mm, (cum[lo] - target) / tot);
    upd_margin(mm, (target - prev) / tot);
  }
  return lo;
}

// Lucy's thin-cell test rho max(kext) dcell < lucy_tau; the FP32 walk
// compares rho with the equivalent density threshold.
template <typename R>
__device__ __forceinline__ bool is_thin(const Ctx<R> &X, R rho) {
  const ModelDev &M = *X.M;
  if constexpr (sizeof(R) == 8) {
    return M.lucy_tau > 0.0 && rho > (R)0 && rho * (R)M.kext_max * (R)M.dcell < (R)M.lucy_tau;
  } else {
    return rho > (R)0 && rho < X.rho_thin;
  }
}

// The same test for a leaf of edge h (refined grids).
template <typename R>
__device__ __forceinline__ bool is_thin_h(const Ctx<R> &X, R rho, double h) {
  const ModelDev &M = *X.M;
  return M.lucy_tau > 0.0 && rho > (R)0 && (double)rho * M.kext_max * h < M.lucy_tau;
}

// Leaf (cell index of every per-cell array) of packet P, its edge and volume.
template <typename R>
__device__ __forceinline__ int64_t pkt_leaf(const ModelDev &M, const Pkt<R> &P, double &h,
                                            double &V) {
  if (!M.ref) {
    h = M.dcell;
    V = M.V;
    return ((int64_t)P.c[2] * M.ny + P.c[1]) * M.nx + P.c[0];
  }
  const int64_t c = leaf_of(M, P.c[0], P.c[1], P.c[2], P.fpk, &h);
  V = (c < (int64_t)M.ncube) ? M.V : h * h * h;
  return c;
}

__device__ __forceinline__ double energy_of(const ModelDev &M, int64_t q) {
  return (double)M.k[q] * M.xi + M.epath[q];
}

// Emission temperature of species s in cell c (see mcrt.h for the modes).
template <typename R>
__device__ double mode_T(Ctx<R> &X, int s, int64_t c, double rho, double V) {
  const ModelDev &M = *X.M;
  int64_t q = (int64_t)s * X.nc + c;
  if (M.mode == M_FROZEN) {
    double T = M.T[q];
    return (T > 0.0) ? T : T_FLOOR;
  }
  double frac = X.dt[X.o.frac + s];
  bool cl = false;
  double T;
  if (M.mode == M_BW_EPOCH) {
    T = M.tt[q];
    if (T < 0.0) {
      double rhs = (M.esnap[q] + M.xi) / (4.0 * PI_D * frac * rho * V);
      T = invert_T_exact(M.herm, X.dt, X.o, M.nl, s, rhs, &cl);
      M.tt[q] = T;  // every lane computes the same value from the snapshot
    }
  } else {
    // the tallies as last seen by this CU (other packets update them with
    // atomics while the kernel runs; any value since the kernel began is a
    // valid reading of the cell's energy so far)
    double e = (double)gld(&M.k[q]) * M.xi + gld(&M.epath[q]);
    double rhs = (e + M.xi) / (4.0 * PI_D * frac * rho * V);
    T = invert_T_fast(M.herm, X.dt, X.o, M.nl, s, rhs, &cl);
  }
  if (cl) stat_add(X.st, 9, 1ull);
  return T;
}

// Lucy's estimator (Eq. 9) on one segment inside a thin cell.
template <typename R>
__device__ __forceinline__ void lucy_deposit(Ctx<R> &X, Pkt<R> &P, int64_t c, R rho, R ell) {
  const ModelDev &M = *X.M;
  int nl = M.nl, j = P.j;
  R em = -m_expm1(-(rho * X.rt[X.o.r_kabsm + j] * ell));
  for (int s = 0; s < M.ns; ++s) {
    R f = X.rt[X.o.r_lucy + s * nl + j];
    if (f == (R)0) continue;
    // FP32: the absorbed fraction in the walk precision, the packet energy
    // (up to ~1e40 erg/s, beyond FLT_MAX) applied in FP64
    double dep;
    if constexpr (sizeof(R) == 8) dep = M.xi * f * em;
    else dep = (double)(f * em) * M.xi;
    gatomic_add(&M.epath[(int64_t)s * X.nc + c], dep);
  }
  if (M.mode == M_BW_EPOCH) M.dirty[c] = 1;
  P.n_lucy++;
}

// Density gathers issued ahead per flight: the voxel path does not depend
// on the density, only where the flight stops does, so each lane walks K
// cells ahead, issues K independent loads, then consumes the segments in
// order (same arithmetic and order as a one-cell-at-a-time walk).
template <typename R> struct Ahead { static constexpr int K = 16; };
template <> struct Ahead<double> { static constexpr int K = 2; };

// State of a flight in progress (kept per lane across event cycles). The
// distance from the flight origin p0 to the next face on axis a is worked
// out afresh from that face's index e_a (an exact integer held in R) at
// every crossing, never accumulated:
//   FP64: ((origin_a + e_a dcell) - p0_a) / d_a   (as a plain evaluation)
//   FP32: fma(e_a, dcell, origin_a - p0_a) * (1 / d_a)
// An axis with d_a = 0 keeps distance +inf and is never stepped.
template <typename R>
struct Flight {
  R tx, ty, tz;  // distance to the next face per axis
  R ex, ey, ez;  // index of that face
  R qx, qy, qz;  // FP32: origin - p0 (unused in FP64)
  R ix, iy, iz;  // FP32: 1 / d; FP64: d
  R t, tau, tstar, kx;
  int cx, cy, cz;
  bool out;
};

template <typename R>
__device__ __forceinline__ R face_t(const Ctx<R> &X, R e, R q, R og, R p0, R id) {
  if constexpr (sizeof(R) == 8) return ((og + e * X.dc) - p0) / id;
  else return __builtin_fmaf(e, X.dc, q) * id;
}

template <typename R>
__device__ __forceinline__ void setup_axis(const Ctx<R> &X, int c, R p, R d, R og, R &e, R &q,
                                           R &id, R &t) {
  e = (R)(c + (d > (R)0 ? 1 : 0));
  q = og - p;
  id = (sizeof(R) == 8) ? d : (R)1 / d;
  t = (d != (R)0) ? face_t<R>(X, e, q, og, p, id) : m_inf<R>();
}

template <typename R>
__device__ __forceinline__ void flight_setup(const Ctx<R> &X, const Pkt<R> &P, Flight<R> &F,
                                             R tau_star) {
  F.cx = P.c[0]; F.cy = P.c[1]; F.cz = P.c[2];
  setup_axis<R>(X, P.c[0], P.p[0], P.d[0], X.og[0], F.ex, F.qx, F.ix, F.tx);
  setup_axis<R>(X, P.c[1], P.p[1], P.d[1], X.og[1], F.ey, F.qy, F.iy, F.ty);
  setup_axis<R>(X, P.c[2], P.p[2], P.d[2], X.og[2], F.ez, F.qz, F.iz, F.tz);
  F.kx = X.rt[X.o.r_kext + P.j];
  F.t = (R)0;
  F.tau = (R)0;
  F.tstar = tau_star;
  F.out = false;
}

// One batch of up to K cell crossings of the flight in F, starting at the
// flight origin P.p. Returns 0 to continue, 1 at an interaction (P.p, P.c
// and P.rho set to the interaction point and its cell), 2 on escape (P.p
// at the exit point). Each crossing leaves by the nearest face, ties going
// to x, then y, then z; the step is written with selects so that lanes
// leaving by different axes do not diverge.
// PC: a new optical-depth draw on entering each cell (the footnote to the
// sect. 2 interaction test): the packet interacts in the first cell whose
// segment depth exceeds -ln(draw), at -ln(draw) / (rho kext) past the start
// of that segment; cells are entered, and draw, in flight order.
template <typename R, bool REC, bool I32, bool PC = false>
__device__ int flight_batch(Ctx<R> &X, Pkt<R> &P, Flight<R> &F) {
  constexpr int K = Ahead<R>::K;
  const R p0x = P.p[0], p0y = P.p[1], p0z = P.p[2];
  const R dx = P.d[0], dy = P.d[1], dz = P.d[2];
  const int sx = dx > (R)0 ? 1 : -1, sy = dy > (R)0 ? 1 : -1, sz = dz > (R)0 ? 1 : -1;
  const R fsx = (R)sx, fsy = (R)sy, fsz = (R)sz;
  // the flight state is worked on in locals (selects between struct members
  // would otherwise become address arithmetic and push the struct to scratch)
  R tx = F.tx, ty = F.ty, tz = F.tz, ex = F.ex, ey = F.ey, ez = F.ez;
  const R qx = F.qx, qy = F.qy, qz = F.qz, ix = F.ix, iy = F.iy, iz = F.iz;
  const R ogx = X.og[0], ogy = X.og[1], ogz = X.og[2];
  R t = F.t, tau = F.tau;
  const R tau_star = F.tstar, kx = F.kx;
  int cx = F.cx, cy = F.cy, cz = F.cz;
  bool out = F.out;
  using Idx = typename std::conditional<I32, uint32_t, int64_t>::type;
  Idx cs[K];
  R ts[K + 1], rh[K];  // ts[k]: distance at the start of step k (ts[ns]: at its end)
  int ns = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (!out) {
      const bool b1 = ty < tx;
      const R t01 = b1 ? ty : tx;
      const bool b2 = tz < t01;
      const R tn = b2 ? tz : t01;
      if (REC) {
        R t2 = b2 ? (b1 ? (tx < ty ? tx : ty) : (ty < tx ? ty : tx))
                  : (b1 ? (tx < tz ? tx : tz) : (ty < tz ? ty : tz));
        if (t2 < m_inf<R>() && t2 > (R)0) upd_margin(P.mm, (double)((t2 - tn) / t2));
      }
      if constexpr (I32) cs[k] = brick_index32(cx, cy, cz, X.nbx, X.nby);
      else cs[k] = brick_index(cx, cy, cz, X.nbx, X.nby);
      ts[k] = t;
      ns = k + 1;
      if (tn > t) t = tn;
      // the segment length max(tn - t, 0) is ts[k + 1] - ts[k]
      const bool mx = !(b1 || b2), my = b1 && !b2;
      cx += mx ? sx : 0;
      cy += my ? sy : 0;
      cz += b2 ? sz : 0;
      out = (unsigned)cx >= (unsigned)X.nx || (unsigned)cy >= (unsigned)X.ny ||
            (unsigned)cz >= (unsigned)X.nz;
      if constexpr (sizeof(R) == 4) {
        // FP32: step the face index of the moved axis, then work out all
        // three next-face distances (two operations each) and keep the
        // moved axis' one; cheaper than selecting the operands
        ex += mx ? fsx : 0.0f;
        ey += my ? fsy : 0.0f;
        ez += b2 ? fsz : 0.0f;
        const R nxt = face_t<R>(X, ex, qx, ogx, p0x, ix);
        const R nyt = face_t<R>(X, ey, qy, ogy, p0y, iy);
        const R nzt = face_t<R>(X, ez, qz, ogz, p0z, iz);
        tx = mx ? nxt : tx;
        ty = my ? nyt : ty;
        tz = b2 ? nzt : tz;
      } else {
        const R e = (b2 ? ez : (b1 ? ey : ex)) + (R)(b2 ? sz : (b1 ? sy : sx));
        const R tf = face_t<R>(X, e, b2 ? qz : (b1 ? qy : qx), b2 ? ogz : (b1 ? ogy : ogx),
                               b2 ? p0z : (b1 ? p0y : p0x), b2 ? iz : (b1 ? iy : ix));
        ex = mx ? e : ex; tx = mx ? tf : tx;
        ey = my ? e : ey; ty = my ? tf : ty;
        ez = b2 ? e : ez; tz = b2 ? tf : tz;
      }
    }
  }
  F.tx = tx; F.ty = ty; F.tz = tz; F.ex = ex; F.ey = ey; F.ez = ez;
  F.t = t; F.cx = cx; F.cy = cy; F.cz = cz; F.out = out;
#pragma unroll
  for (int k = 0; k <= K; ++k)
    if (k == ns) ts[k] = t;
  // a brick run whose occupancy bit is clear holds only zero densities: its
  // cells take rho = 0 without a load
  uint32_t ow[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ow[k] = (k < ns) ? X.occ[(uint32_t)(cs[k] >> X.osh) >> 5] : 0u;
#pragma unroll
  for (int k = 0; k < K; ++k)
    rh[k] = ((ow[k] >> ((uint32_t)(cs[k] >> X.osh) & 31u)) & 1u) ? gld(X.rho_b + cs[k]) : (R)0;
  // linear cell index of a bricked index (Lucy deposits)
  auto lin = [&](Idx i) {
    int ux, uy, uz;
    unbrick(i, X.nbx, X.nby, ux, uy, uz);
    return ((int64_t)uz * X.ny + uy) * X.nx + ux;
  };
  // segments in order; the flight stops in the first whose depth reaches
  // tau_star (its slot is kept and its cell recovered from the bricked
  // index once, after the loop)
  int kint = -1;
  R tint = (R)0, rint = (R)0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (k < ns && kint < 0) {
      const R rho = rh[k];
      const R ell = ts[k + 1] - ts[k];
      const R dtau = rho * kx * ell;
      const bool thin = is_thin(X, rho);
      R tcur = tau_star;
      if constexpr (PC) {
        tau = (R)0;
        tcur = -m_log(rng_u<R>(P.rng));
      }
      if (REC) upd_margin(P.mm, (double)(m_fabs(tau + dtau - tcur) / tcur));
      if (tau + dtau > tcur) {
        tint = ts[k] + (tcur - tau) / (rho * kx);
        rint = rho;
        kint = k;
        if (thin) lucy_deposit(X, P, lin(cs[k]), rho, tint - ts[k]);
      } else {
        if (thin) lucy_deposit(X, P, lin(cs[k]), rho, ell);
        tau += dtau;
        P.n_cross++;
      }
    }
  }
  F.tau = tau;
  if (kint >= 0) {
    Idx ci = cs[0];
#pragma unroll
    for (int k = 1; k < K; ++k)
      if (k == kint) ci = cs[k];
    int ux, uy, uz;
    unbrick(ci, X.nbx, X.nby, ux, uy, uz);
    P.p[0] = p0x + tint * dx;
    P.p[1] = p0y + tint * dy;
    P.p[2] = p0z + tint * dz;
    P.c[0] = ux; P.c[1] = uy; P.c[2] = uz;
    P.rho = rint;
    return 1;
  }
  if (!out) return 0;
  P.p[0] = p0x + t * dx;
  P.p[1] = p0y + t * dy;
  P.p[2] = p0z + t * dz;
  P.c[0] = cx; P.c[1] = cy; P.c[2] = cz;
  return 2;
}

// ------------------------------------------------ walk on refined grids
// One level of refinement: the walk steps each cube's own lattice (a whole
// cube is its own single sub-cube), one leaf per crossing, with the face
// distances in FP64 in both precisions; leaving a divided cube happens on
// the cube's own face. No look-ahead gathers: this walk serves refined
// models, the bricked walk above the uniform grids.
template <typename R>
struct FlightRef {
  double tm[3];  // distance to the current leaf's next face per axis
  double t;      // distance walked from the flight origin
  R tau, tstar, kx;
  int c[3], f[3], r;
};

template <typename R>
__device__ __forceinline__ void ref_faces(const ModelDev &M, const Pkt<R> &P, FlightRef<R> &F) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double dk = (double)P.d[k], pk = (double)P.p[k];
    if (dk > 0.0) F.tm[k] = (face_pos(M, k, F.c[k], F.r, F.f[k] + 1) - pk) / dk;
    else if (dk < 0.0) F.tm[k] = (face_pos(M, k, F.c[k], F.r, F.f[k]) - pk) / dk;
    else F.tm[k] = m_inf<double>();
  }
}

template <typename R>
__device__ __forceinline__ void flight_setup_ref(const Ctx<R> &X, const Pkt<R> &P,
                                                 FlightRef<R> &F, R tau_star) {
  const ModelDev &M = *X.M;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    F.c[k] = P.c[k];
    F.f[k] = fine_get(P.fpk, k);
  }
  F.r = cube_r(M, ((int64_t)F.c[2] * M.ny + F.c[1]) * M.nx + F.c[0]);
  ref_faces(M, P, F);
  F.t = 0.0;
  F.tau = (R)0;
  F.tstar = tau_star;
  F.kx = X.rt[X.o.r_kext + P.j];
}

// Up to K leaf crossings of the flight (0: continue, 1: interaction, 2:
// escape), in the order and arithmetic of a one-leaf-at-a-time walk.
template <typename R, bool REC, bool PC>
__device__ int flight_batch_ref(Ctx<R> &X, Pkt<R> &P, FlightRef<R> &F) {
  const ModelDev &M = *X.M;
  constexpr int K = 8;
  for (int it = 0; it < K; ++it) {
    int a = 0;
    if (F.tm[1] < F.tm[a]) a = 1;
    if (F.tm[2] < F.tm[a]) a = 2;
    if (REC) {
      double t2 = m_inf<double>();
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k != a && F.tm[k] < t2) t2 = F.tm[k];
      if (t2 < m_inf<double>() && t2 > 0.0) upd_margin(P.mm, (t2 - F.tm[a]) / t2);
    }
    double ell = F.tm[a] - F.t;
    if (ell < 0.0) ell = 0.0;
    double h;
    const int64_t c = leaf_of(M, F.c[0], F.c[1], F.c[2], fine_pack(F.f[0], F.f[1], F.f[2]), &h);
    const R rho = gld(X.rho + c);
    const R dtau = rho * F.kx * (R)ell;
    const bool thin = is_thin_h(X, rho, h);
    R tcur = F.tstar;
    if constexpr (PC) {
      F.tau = (R)0;
      tcur = -m_log(rng_u<R>(P.rng));
    }
    if (REC) upd_margin(P.mm, (double)(m_fabs(F.tau + dtau - tcur) / tcur));
    if (F.tau + dtau > tcur) {
      const double tint = F.t + (double)((tcur - F.tau) / (rho * F.kx));
      if (thin) lucy_deposit(X, P, c, rho, (R)(tint - F.t));
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        P.p[k] = (R)((double)P.p[k] + tint * (double)P.d[k]);
        P.c[k] = F.c[k];
      }
      P.fpk = fine_pack(F.f[0], F.f[1], F.f[2]);
      P.rho = rho;
      return 1;
    }
    if (thin) lucy_deposit(X, P, c, rho, (R)ell);
    F.tau += dtau;
    if (F.tm[a] > F.t) F.t = F.tm[a];
    P.n_cross++;
    // cross the face on axis a
    const double da = (double)P.d[a];
    const int sa = da > 0.0 ? 1 : -1;
    F.f[a] += sa;
    if (F.f[a] >= 0 && F.f[a] < F.r) {
      F.tm[a] = (face_pos(M, a, F.c[a], F.r, da > 0.0 ? F.f[a] + 1 : F.f[a]) - (double)P.p[a]) / da;
      continue;
    }
    F.c[a] += sa;
    const int na = a == 0 ? M.nx : (a == 1 ? M.ny : M.nz);
    if (F.c[a] < 0 || F.c[a] >= na) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        P.p[k] = (R)((double)P.p[k] + F.t * (double)P.d[k]);
        P.c[k] = F.c[k];
      }
      return 2;
    }
    // enter the next cube on its own lattice
    F.r = cube_r(M, ((int64_t)F.c[2] * M.ny + F.c[1]) * M.nx + F.c[0]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double dk = (double)P.d[k];
      if (k == a) F.f[k] = dk > 0.0 ? 0 : F.r - 1;
      else F.f[k] = sub_index(M, k, F.c[k], F.r, (double)P.p[k] + F.t * dk, dk);
    }
    ref_faces(M, P, F);
  }
  return 0;
}

// Rosseland mean of the mixture opacity at T (sect. 3.2). The FP64 means
// and the MRW spectrum below are kept out of line so that their loops do
// not add registers to the whole transport kernel.
static __device__ __noinline__ double rosseland_mean(const double *w, const double *hnu,
                                                     const double *a, const double *kext, int nl,
                                                     double T) {
  double num = 0.0, den = 0.0;
  for (int j = nl - 1; j >= 0; --j) {
    double ke = kext[j];
    if (!(ke > 0.0)) return 0.0;
    double db = w[j] * dplanck_d(hnu[j], a[j], T);
    num += db;
    den += db / ke;
  }
  return (den > 0.0) ? num / den : 0.0;
}

// Planck mean of one species' absorption opacity at T.
static __device__ __noinline__ double planck_mean(const double *w, const double *hnu,
                                                  const double *a, const double *kabs, int nl,
                                                  double T) {
  double num = 0.0, den = 0.0;
  for (int j = nl - 1; j >= 0; --j) {
    double b = w[j] * planck_d(hnu[j], a[j], T);
    num += b * kabs[j];
    den += b;
  }
  return (den > 0.0) ? num / den : 0.0;
}

// Thermal emission wavelength after an MRW step: inverse CDF of
// sum_s w_j f_s kabs_s,j B_j(T_s) over the thermal species.
struct PickOut {
  int j;
  double mm;
};
template <bool REC>
static __device__ __noinline__ PickOut mrw_pick(const double *wfk, const double *hnu,
                                                const double *a, int nl, int ns, int pah,
                                                double T0, double T1, double T2, double T3,
                                                double u) {
  PickOut r;
  r.mm = 1e300;
  r.j = pick_desc_fn<double, REC>(nl, u, r.mm, [&](int j) {
    double f = 0.0;
#pragma unroll
    for (int s = 0; s < MAX_NS; ++s) {
      if (s >= ns || s == pah) continue;
      const double T = s == 0 ? T0 : (s == 1 ? T1 : (s == 2 ? T2 : T3));
      f += wfk[s * nl + j] * planck_d(hnu[j], a[j], T);
    }
    return f;
  });
  return r;
}

__device__ __forceinline__ int first_thermal(const ModelDev &M) {
  for (int s = 0; s < M.ns; ++s)
    if (s != M.pah) return s;
  return 0;
}

// The packet's cell as the modified random walk sees it.
struct MrwCell {
  int64_t c;
  double rho, hl, Vl;
  int s0;
};

// Temperature-free bounds of a modified random walk step (sect. 3.2) in
// cell c of density rho, edge hl and volume Vl: false when the step can
// never apply there. frac_s0 is the mass fraction of the first thermal
// species. The second bound is used without records only.
template <bool REC>
__device__ __forceinline__ bool mrw_possible_cell(const ModelDev &M, double rho, double hl,
                                                  double Vl, double frac_s0) {
  if (!(M.mrw_tau > 0.0) || !(rho > 0.0)) return false;
  if (!(rho * M.kext_max * hl > M.mrw_tau)) return false;
  if (!REC && M.mode != M_FROZEN) {
    // B&W temperatures come from at least one packet's energy; when that
    // alone reaches Phi(T_TAB_MIN), T lies on the bound table and kappa_R
    // is below its largest entry, which may already rule the step out
    // without the temperature
    const double rmin = M.xi / (4.0 * PI_D * frac_s0 * rho * Vl);
    if (rmin >= 1.001 * M.phi_tmin && !(rho * M.kr_gmax * hl > M.mrw_tau)) return false;
  }
  return true;
}

// Immediate B&W without records: the table interval that Eq. 4 takes for
// the cell's current tallies bounds kappa_R at its temperature (mrw_ub), so
// one lookup may rule the step out before T is inverted (false). The
// right-hand side is mode_T's.
__device__ __forceinline__ bool mrw_possible_now(const ModelDev &M, int64_t c, int s0,
                                                 double rho, double hl, double Vl,
                                                 double frac_s0) {
  if (M.mode != M_BW_TICKET || !M.mrw_ub) return true;
  const int64_t q0 = (int64_t)s0 * (int64_t)M.ncell + c;
  const double e = (double)gld(&M.k[q0]) * M.xi + gld(&M.epath[q0]);
  const double rhs = (e + M.xi) / (4.0 * PI_D * frac_s0 * rho * Vl);
  const double *h = M.herm + (size_t)s0 * (3 + 2 * NH_TAB);
  const float x = (__logf((float)rhs) - (float)h[0]) / (float)h[1];
  if (x >= 1.0f && x < (float)(NH_TAB - 3)) {
    if (!(rho * gld(M.mrw_ub + (int)x) * hl > M.mrw_tau)) return false;
  }
  return true;
}

// Bounds that rule a modified random walk step out before the cell
// temperature is formed: false when the step cannot apply, true when the
// exact test (Rosseland depth at the cell temperature, sphere size) has to
// decide.
template <typename R, bool REC>
__device__ bool mrw_candidate(Ctx<R> &X, const Pkt<R> &P, MrwCell &C) {
  const ModelDev &M = *X.M;
  if (!(M.mrw_tau > 0.0)) return false;
  double hl, Vl;
  const int64_t c = pkt_leaf(M, P, hl, Vl);
  // the density of the cell came with the packet from its last flight
  double rho = P.rho > (R)0 ? (double)P.rho : (double)gld(X.rho + c);
  const int s0 = first_thermal(M);
  const double f0 = X.dt[X.o.frac + s0];
  if (!mrw_possible_cell<REC>(M, rho, hl, Vl, f0)) return false;
  C.c = c; C.rho = rho; C.hl = hl; C.Vl = Vl; C.s0 = s0;
  if (!REC && !mrw_possible_now(M, c, s0, rho, hl, Vl, f0)) return false;
  return true;
}

// Per-cell diffusion flags of the fast interaction kernel, one bit per leaf
// cell in words of 32. k_mrw_cand marks, once per launch, the cells that
// pass the temperature-free bounds; k_mrw_flags sets, before every fast
// interaction kernel, the bits of those cells that the tally bound does not
// rule out at that moment. The fast kernel hands a packet to the slow
// kernel's exact test when its cell's bit is set: the flags read the
// tallies as they stand when the kernel starts, which is one of the
// readings immediate B&W allows (any value since the kernel began).
template <typename R>
__global__ void k_mrw_cand(const ModelDev *__restrict__ models, int nmodels) {
  for (int mm = 0; mm < nmodels; ++mm) {
    const ModelDev &M = models[mm];
    if (!M.mrw_cand) continue;
    const TabOff o = tab_offsets(M.nl, M.ns, M.nsrc, M.nrows);
    const double f0 = M.tab[o.frac + first_thermal(M)];
    const uint64_t nw = (M.ncell + 31) / 32;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw;
         w += (uint64_t)gridDim.x * blockDim.x) {
      uint32_t bits = 0u;
      for (int b = 0; b < 32; ++b) {
        const uint64_t c = w * 32 + (uint64_t)b;
        if (c >= M.ncell) break;
        const double rho = (double)gld((const R *)M.rho + c);
        const double hl = leaf_edge(M, c);
        const double Vl = (c < M.ncube) ? M.V : hl * hl * hl;
        if (mrw_possible_cell<false>(M, rho, hl, Vl, f0)) bits |= 1u << b;
      }
      M.mrw_cand[w] = bits;
      M.mrw_bits[w] = 0u;
    }
  }
}

template <typename R>
__global__ void k_mrw_flags(const ModelDev *__restrict__ models, int nmodels) {
  for (int mm = 0; mm < nmodels; ++mm) {
    const ModelDev &M = models[mm];
    if (!M.mrw_cand || M.ctl->inq == 0u) continue;
    const TabOff o = tab_offsets(M.nl, M.ns, M.nsrc, M.nrows);
    const int s0 = first_thermal(M);
    const double f0 = M.tab[o.frac + s0];
    const uint64_t nw = (M.ncell + 31) / 32;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw;
         w += (uint64_t)gridDim.x * blockDim.x) {
      uint32_t cand = gld(M.mrw_cand + w);
      if (!cand) continue;
      uint32_t bits = 0u;
      while (cand) {
        const int b = __builtin_ctz(cand);
        cand &= cand - 1u;
        const uint64_t c = w * 32 + (uint64_t)b;
        const double rho = (double)gld((const R *)M.rho + c);
        const double hl = leaf_edge(M, c);
        const double Vl = (c < M.ncube) ? M.V : hl * hl * hl;
        if (mrw_possible_now(M, (int64_t)c, s0, rho, hl, Vl, f0)) bits |= 1u << b;
      }
      M.mrw_bits[w] = bits;
    }
  }
}

// Modified random walk step (sect. 3.2): see the public header for the
// trigger. Returns true when a step was taken.
template <typename R, bool REC>
__device__ bool mrw_step(Ctx<R> &X, Pkt<R> &P) {
  const ModelDev &M = *X.M;
  MrwCell C;
  if (!mrw_candidate<R, REC>(X, P, C)) return false;
  const int64_t c = C.c;
  const double rho = C.rho, hl = C.hl, Vl = C.Vl;
  const int s0 = C.s0;
  double T0 = mode_T(X, s0, c, rho, Vl);
  if (!REC) {
    // upper bound of kappa_R(T) on its table interval (build_tables proves
    // it): skip the exact mean when even the bound cannot reach the threshold
    const double lt0 = log(T_TAB_MIN), dlt = (log(T_MAX) - lt0) / (NT_TAB - 1);
    double xk = (log(T0) - lt0) / dlt;
    int k = (xk >= 0.0 && xk < (double)(NT_TAB - 1)) ? (int)xk : NT_TAB - 1;
    if (!(rho * X.dt[X.o.krmax + k] * hl > M.mrw_tau)) return false;
  }
  double kr = rosseland_mean(X.dt + X.o.w, X.dt + X.o.hnu, X.dt + X.o.a, X.dt + X.o.kext, M.nl, T0);
  double taur = rho * kr * hl;
  if (REC) upd_margin(P.mm, fabs(taur - M.mrw_tau) / M.mrw_tau);
  if (!(taur > M.mrw_tau)) return false;
  double Rs = 1e300;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double pk = (double)P.p[k];
    double lo, hi;
    if (!M.ref) {
      lo = pk - (M.origin[k] + (double)P.c[k] * M.dcell);
      hi = (M.origin[k] + (double)(P.c[k] + 1) * M.dcell) - pk;
    } else {
      // the faces of the packet's leaf
      const int r = cube_r(M, ((int64_t)P.c[2] * M.ny + P.c[1]) * M.nx + P.c[0]);
      lo = pk - face_pos(M, k, P.c[k], r, fine_get(P.fpk, k));
      hi = face_pos(M, k, P.c[k], r, fine_get(P.fpk, k) + 1) - pk;
    }
    if (lo < Rs) Rs = lo;
    if (hi < Rs) Rs = hi;
  }
  if (Rs < 0.0) Rs = 0.0;
  double crit = rho * kr * Rs;
  if (REC) upd_margin(P.mm, fabs(crit - M.mrw_gamma) / M.mrw_gamma);
  if (!(crit >= M.mrw_gamma)) return false;
  double ut = rng_u<double>(P.rng), ups = rng_u<double>(P.rng), ums = rng_u<double>(P.rng);
  double ul = rng_u<double>(P.rng), uph = rng_u<double>(P.rng), umu = rng_u<double>(P.rng);
  double y = mrw_solve(ut);
  double ell = -3.0 * rho * kr * Rs * Rs * log(y) / (PI_D * PI_D);
  double ds[3];
  {
    double phi = 2.0 * PI_D * ups, mu = 1.0 - 2.0 * ums;
    double s = sqrt(fmax(0.0, 1.0 - mu * mu));
    ds[0] = s * cos(phi);
    ds[1] = s * sin(phi);
    ds[2] = mu;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) P.p[k] = (R)((double)P.p[k] + Rs * ds[k]);
  const int nl = M.nl;
  double Ts[MAX_NS] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < MAX_NS; ++s) {
    if (s >= M.ns || s == M.pah) continue;
    const double T = mode_T(X, s, c, rho, Vl);
    Ts[s] = T;
    double kp = planck_mean(X.dt + X.o.w, X.dt + X.o.hnu, X.dt + X.o.a, X.dt + X.o.kabs + s * nl,
                            nl, T);
    gatomic_add(&M.epath[(int64_t)s * X.nc + c], M.xi * rho * X.dt[X.o.frac + s] * kp * ell);
  }
  if (M.mode == M_BW_EPOCH) M.dirty[c] = 1;
  const PickOut pk = mrw_pick<REC>(X.dt + X.o.wfk, X.dt + X.o.hnu, X.dt + X.o.a, nl, M.ns, M.pah,
                                   Ts[0], Ts[1], Ts[2], Ts[3], ul);
  P.j = pk.j;
  if (REC) upd_margin(P.mm, pk.mm);
  iso_dir<R>(uph, umu, P.d);
  P.n_mrw++;
  stat_add(X.st, 7, 1ull);
  return true;
}

template <typename R>
__device__ __forceinline__ int pah_row(const Ctx<R> &X, int64_t c, double rho, double V) {
  const ModelDev &M = *X.M;
  double q = (double)M.kpah[c] * M.xi / (4.0 * PI_D * X.dt[X.o.frac + M.pah] * rho * V);
  int r = 0;
  while (r < M.nrows - 1 && q >= X.dt[X.o.pahe + r]) r++;
  return r;
}

template <typename R, bool REC>
__device__ __forceinline__ int pick_pah(const Ctx<R> &X, int row, double u, double &mm) {
  return pick_desc_cum<REC>(X.dt + X.o.pahcum + row * X.M->nl, X.M->nl, u, mm);
}

// Re-emission wavelength of species s at temperature T: Eq. 5 (FROZEN) or
// Eq. 10 (Bjorkman & Wood), in the walk precision.
template <typename R, bool REC>
__device__ __forceinline__ int pick_thermal(const Ctx<R> &X, int s, double T, R u, double &mm) {
  const ModelDev &M = *X.M;
  const int nl = M.nl;
  if (sizeof(R) == 8) {
    const double *wk = X.dt + X.o.wk + s * nl;
    const double *hnu = X.dt + X.o.hnu;
    const double *a = X.dt + X.o.a;
    if (M.mode == M_FROZEN)
      return pick_desc_fn<double, REC>(nl, (double)u, mm,
                                       [&](int j) { return wk[j] * planck_d(hnu[j], a[j], T); });
    return pick_desc_fn<double, REC>(nl, (double)u, mm,
                                     [&](int j) { return wk[j] * dplanck_d(hnu[j], a[j], T); });
  } else {
    const R *wk = X.rt + X.o.r_wk + s * nl;
    const R *hnu = X.rt + X.o.r_hnu;
    const R *a = X.rt + X.o.r_a;
    const R rkT = (R)(1.0 / (K_BO * T));
    const R cut = x_cut<R>();
    // e^x - 1 from the hardware exponential, with a 3-term series below 0.03;
    // weights drop the common factor 1/T of dB/dT (the CDF is normalised)
    auto em1 = [](R x) { return x < (R)0.03 ? x * ((R)1 + x * ((R)0.5 + x * (R)(1.0 / 6.0))) : __expf(x) - (R)1; };
    if (M.mode == M_FROZEN)
      return pick_desc_fn<R, REC>(nl, u, mm, [&](int j) {
        R x = hnu[j] * rkT;
        return x > cut ? (R)0 : wk[j] * a[j] * __builtin_amdgcn_rcpf(em1(x));
      });
    return pick_desc_fn<R, REC>(nl, u, mm, [&](int j) {
      R x = hnu[j] * rkT;
      if (x > cut) return (R)0;
      R r = __builtin_amdgcn_rcpf(em1(x));
      return wk[j] * a[j] * x * r * ((R)1 + r);
    });
  }
}

// End of a packet: escape tally, status counters and its record. The
// crossings and Lucy deposits of the packet are counted here unless the
// caller counts them per flight (walk_tallied).
// Re-emission bin in the FP32 walk by rejection: a proposal from the alias
// table of T's ln T bin (whose spectrum, taken at the bin's upper edge,
// bounds the spectrum at T), accepted with probability p_j(T) / env_j.
// Exact in distribution; about 1.1 proposals per absorption over 512 bins
// from 1 K to 1e5 K. -1 outside the table or after 64 rejections (the
// caller then walks the inverse CDF).
__device__ __forceinline__ int rej_thermal(const Ctx<float> &X, int s, double T, Rng &rng) {
  const ModelDev &M = *X.M;
  if (!M.rej_pe || !(T > 0.0)) return -1;
  const int nl = M.nl;
  const double lt0 = log(T_TAB_MIN), dlt = (log(T_MAX) - lt0) / NK_REJ;
  const double kf = (log(T) - lt0) / dlt;
  if (!(kf >= 0.0 && kf < (double)NK_REJ)) return -1;
  const int k = (int)kf;
  const size_t base = ((size_t)(M.mode == M_FROZEN ? 0 : 1) * M.ns + s) * ((size_t)NK_REJ * nl) +
                      (size_t)k * nl;
  const float *pe = M.rej_pe + 2 * base;
  const uint8_t *al = M.rej_al + base;
  const float *wk = X.rt + X.o.r_wk + s * nl;
  const float *hnu = X.rt + X.o.r_hnu;
  const float *a = X.rt + X.o.r_a;
  const float rkT = (float)(1.0 / (K_BO * T)), rT = (float)(1.0 / T);
  const bool bw = M.mode != M_FROZEN;
  for (int t = 0; t < 64; ++t) {
    const float u1 = rng_u<float>(rng), u2 = rng_u<float>(rng);
    const float xf = u1 * (float)nl;
    int j = (int)xf;
    if (j > nl - 1) j = nl - 1;
    const float fr = xf - (float)j;
    if (!(fr < gld(pe + 2 * j))) j = gld(al + j);
    const float env = gld(pe + 2 * j + 1);
    const float x = hnu[j] * rkT;
    float p = 0.0f;
    if (x <= 80.0f) {
      const float em = x < 0.03f ? x * (1.0f + x * (0.5f + x * (1.0f / 6.0f))) : __expf(x) - 1.0f;
      const float r = __builtin_amdgcn_rcpf(em);
      p = bw ? wk[j] * a[j] * r * x * rT * (1.0f + r) : wk[j] * a[j] * r;
    }
    if (u2 * env <= p) return j;
  }
  return -1;
}

template <typename R, bool REC>
__device__ void finish(Ctx<R> &X, Pkt<R> &P, bool walk_tallied = false) {
  const ModelDev &M = *X.M;
  if (!walk_tallied) {
    stat_add(X.st, 4, P.n_cross);
    if (P.n_lucy) stat_add(X.st, 8, P.n_lucy);
  }
  if (P.status == ST_ESCAPED) {
    stat_add(X.st, 1, 1ull);
    int nt = M.ntheta > 0 ? M.ntheta : 1;
    R x = (P.d[2] + (R)1) * (R)0.5 * (R)nt;
    int b = (int)m_floor(x);
    if (b < 0) b = 0;
    if (b >= nt) b = nt - 1;
    if (REC && nt > 1) upd_margin(P.mm, (double)(m_fabs(x - m_floor(x + (R)0.5)) / (R)nt));
    atomicAdd(&X.sed[b * M.nl + P.j], 1u);
  } else if (P.status == ST_KILLED) {
    stat_add(X.st, 2, 1ull);
  } else if (P.status == ST_PAH_STOP) {
    stat_add(X.st, 3, 1ull);
  }
  if (REC && M.rec) {
    uint64_t slot = P.pid - M.id_base - M.rec_first;
    uint64_t *r = (uint64_t *)M.rec + slot * 15;  // 120-byte mcrt_packet_record
    double *rd = (double *)r;
    r[0] = P.pid;
    rd[1] = (double)P.p[0]; rd[2] = (double)P.p[1]; rd[3] = (double)P.p[2];
    rd[4] = (double)P.d[0]; rd[5] = (double)P.d[1]; rd[6] = (double)P.d[2];
    int32_t *ri = (int32_t *)(r + 7);
    ri[0] = P.j;
    ri[1] = P.status;
    rd[8] = M.xi;
    r[9] = P.n_cross; r[10] = P.n_scat; r[11] = P.n_abs; r[12] = P.n_mrw; r[13] = P.n_lucy;
    rd[14] = P.mm;
  }
}

// Photodissociation of the PAH in cell c (sect. 2.1, Eq. 8): its kpah
// pass-1 absorptions of xi erg/s are shared by f_pah rho V / m_PAH
// molecules (m_PAH = N_C 12 amu); each takes E_PAH = kpah xi m_PAH t_cool /
// (f_pah rho V) within the cooling time, and E_PAH >= N_C/2 eV dissociates.
constexpr double AMU_G = 1.66053906660e-24;
constexpr double EV_ERG = 1.602176634e-12;
template <typename R>
__device__ __forceinline__ bool pah_dissociates(const Ctx<R> &X, int64_t c) {
  const ModelDev &M = *X.M;
  if (!(M.pah_nc > 0.0) || !(M.pah_tcool > 0.0)) return false;
  const uint32_t kp = M.kpah[c];
  if (kp == 0u) return false;
  const double rho = (double)gld(X.rho + c);
  const double mp = M.pah_nc * 12.0 * AMU_G;
  const double e = (double)kp * M.xi * mp * M.pah_tcool /
                   (X.dt[X.o.frac + M.pah] * rho * leaf_volume(M, (uint64_t)c));
  return e >= 0.5 * M.pah_nc * EV_ERG;
}

// Start packet `idx` of the launch: source emission, or a PAH pass-2
// packet born in the cell that owns it (from the sources when that cell's
// PAH dissociate).
template <typename R, bool REC>
__device__ void start_packet(Ctx<R> &X, Pkt<R> &P, uint64_t idx) {
  const ModelDev &M = *X.M;
  const int nl = M.nl;
  P.pid = M.id_base + M.first + idx;
  rng_init(P.rng, M.seed, P.pid, (uint32_t)M.iter, (uint32_t)M.model_id, M.pass == 2 ? 3u : 0u);
  P.status = ST_ALIVE;
  P.rho = (R)0;
  P.n_cross = P.n_scat = P.n_abs = P.n_mrw = P.n_lucy = P.n_int = 0;
  P.mm = 1e300;
  P.fpk = 0u;
  stat_add(X.st, 0, 1ull);
  int64_t c = -1;
  if (M.pass == 2) {
    // cell owning local packet index (first + idx) in the exclusive prefix of PAH counts
    uint64_t li = M.first + idx;
    int64_t lo = 0, hi = X.nc - 1;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) >> 1;
      if (M.kpah_prefix[mid] <= li) lo = mid; else hi = mid - 1;
    }
    c = lo;
  }
  if (c >= 0 && !pah_dissociates(X, c)) {
    R u3[3];
    u3[0] = rng_u<R>(P.rng);
    u3[1] = rng_u<R>(P.rng);
    u3[2] = rng_u<R>(P.rng);
    double ul = rng_u<double>(P.rng), uph = rng_u<double>(P.rng), umu = rng_u<double>(P.rng);
    if (c < (int64_t)M.ncube) {
      int cc[3] = {(int)(c % M.nx), (int)((c / M.nx) % M.ny), (int)(c / ((int64_t)M.nx * M.ny))};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        P.c[k] = cc[k];
        P.p[k] = (R)M.origin[k] + ((R)cc[k] + u3[k]) * (R)M.dcell;
      }
    } else {
      // uniform inside a sub-cube
      int cc[3], ff[3], r;
      leaf_loc(M, (uint64_t)c, cc, ff, &r);
      const double h = M.dcell / (double)r;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        P.c[k] = cc[k];
        P.p[k] = (R)(face_pos(M, k, cc[k], r, ff[k]) + (double)u3[k] * h);
      }
      P.fpk = fine_pack(ff[0], ff[1], ff[2]);
    }
    P.j = pick_pah<R, REC>(X, pah_row(X, c, (double)gld(X.rho + c), leaf_volume(M, (uint64_t)c)),
                           ul, P.mm);
    iso_dir<R>(uph, umu, P.d);
    return;
  }
  double uph = rng_u<double>(P.rng), umu = rng_u<double>(P.rng);
  double us = rng_u<double>(P.rng), ul = rng_u<double>(P.rng);
  // m equal-energy source bins (Eq. 1): packet p draws inside stratum p mod m
  if (M.src_strata > 0 && M.pass != 2)
    ul = ((double)(P.pid % M.src_strata) + ul) / (double)M.src_strata;
  iso_dir<R>(uph, umu, P.d);
  int s = 0;
  if (M.nsrc > 1) s = pick_asc<double, REC>(X.dt + X.o.lum, 1, M.nsrc, us, P.mm);
#pragma unroll
  for (int k = 0; k < 3; ++k) P.p[k] = (R)X.dt[X.o.srcpos + 3 * s + k];
  P.j = pick_desc_cum<REC>(X.dt + X.o.srccum + s * nl, nl, ul, P.mm);
  start_cell<R>(M, P.p, P.d, P.c);
  if (P.c[0] < 0 || P.c[0] >= M.nx || P.c[1] < 0 || P.c[1] >= M.ny || P.c[2] < 0 ||
      P.c[2] >= M.nz) {
    P.status = ST_ESCAPED;
  } else if (M.ref) {
    const int r = cube_r(M, ((int64_t)P.c[2] * M.ny + P.c[1]) * M.nx + P.c[0]);
    P.fpk = fine_pack(sub_index(M, 0, P.c[0], r, (double)P.p[0], (double)P.d[0]),
                      sub_index(M, 1, P.c[1], r, (double)P.p[1], (double)P.d[1]),
                      sub_index(M, 2, P.c[2], r, (double)P.p[2], (double)P.d[2]));
  }
}

// Start of a flight: modified random walk steps while they apply, then the
// optical depth of the flight. Returns a negative depth when the packet is
// killed. FAST (fast interaction kernel): a packet whose cell needs the
// exact diffusion test sets *defer = 2 and returns before any draw; the slow
// kernel then starts its flight with this function (FAST false).
template <typename R, bool REC, bool FAST = false>
__device__ R flight_tau(Ctx<R> &X, Pkt<R> &P, int *defer = nullptr) {
  const ModelDev &M = *X.M;
  if constexpr (FAST) {
    if (M.mrw_tau > 0.0) {
      double hl, Vl;
      const int64_t c = pkt_leaf(M, P, hl, Vl);
      if (!M.mrw_bits || ((gld(M.mrw_bits + (c >> 5)) >> (c & 31)) & 1u)) {
        *defer = 2;
        return (R)-1;
      }
    }
  } else {
    while (mrw_step<R, REC>(X, P)) {
      P.n_int++;
      if (M.max_int > 0 && P.n_int >= M.max_int) {
        P.status = ST_KILLED;
        return (R)-1;
      }
    }
  }
  // per-cell draws are taken by the walk itself, cell by cell
  if (M.tau_mode == 1) return (R)1;
  return -m_log(rng_u<R>(P.rng));
}

// A scattering event kept for any observer (sect. 4): with the HG phase
// function expanded as P(d.k) = sum_l g^l sum_m Y_lm(d) Y_lm(k), the event
// adds w g^l Y_lm(d_in) to the moments row of its cell and wavelength
// (out of line: its loops stay out of the interaction kernel's registers).
template <typename R>
static __device__ __noinline__ void sh_deposit(R *row, int order, double dx, double dy, double dz,
                                               double g, double w) {
  double gp[MAX_SH_ORDER];
  gp[0] = 1.0;
  for (int l = 1; l < order; ++l) gp[l] = gp[l - 1] * g;
  ylm_each(order, dx, dy, dz, [&](int i, int l, double y) {
    gatomic_add(row + i, (R)(w * gp[l] * y));
  });
}

// Eq. 4 for immediate B&W by the Hermite table alone (fast interaction
// kernel): the caller has checked that the right-hand side lies at or above
// the table's lower end; at or above its upper end, Phi(T_MAX), the
// temperature is T_MAX (clamped).
__device__ __forceinline__ double invert_T_table(const double *herm, int s, double rhs,
                                                bool *clamped) {
  const double *h = herm + (size_t)s * (3 + 2 * NH_TAB);
  double x = (log(rhs) - h[0]) / h[1];
  const int n = (int)h[2];
  if (!(x >= 0.0)) x = 0.0;
  if (!(x < (double)(n - 1))) {
    *clamped = true;
    return T_MAX;
  }
  int k = (int)x;
  double t = x - (double)k, t2 = t * t, t3 = t2 * t;
  const double *p = h + 3 + 2 * k;
  double y = (2.0 * t3 - 3.0 * t2 + 1.0) * p[0] + (t3 - 2.0 * t2 + t) * h[1] * p[1] +
             (-2.0 * t3 + 3.0 * t2) * p[2] + (t3 - t2) * h[1] * p[3];
  return exp(y);
}

// Interaction at P.p in cell P.c: albedo split, HG scattering with its
// event sums, or absorption with re-emission (or a PAH stop). FAST (fast
// interaction kernel: immediate B&W, no records, no moments): an absorption
// in a cell where one packet's energy lies below the Eq. 4 table sets
// *defer = 1 and returns before any tally or statistic changes, so that the
// slow kernel can take the whole interaction again from the queued state.
template <typename R, bool REC, bool FAST = false>
__device__ void interact(Ctx<R> &X, Pkt<R> &P, int *defer = nullptr) {
  const ModelDev &M = *X.M;
  const int nl = M.nl, ns = M.ns;
  double hl, Vl;
  const int64_t c = pkt_leaf(M, P, hl, Vl);
  R ualb = rng_u<R>(P.rng), usp = rng_u<R>(P.rng);
  const int j = P.j;
  const R alb = X.rt[X.o.r_alb + j];
  if (REC) upd_margin(P.mm, (double)m_fabs(ualb - alb));
  if (ualb < alb) {
    int s = pick_asc<R, REC>(X.rt + X.o.r_fsca + j, nl, ns, usp, P.mm);
    R g = X.rt[X.o.r_g + s * nl + j];
    R umu = rng_u<R>(P.rng), uph = rng_u<R>(P.rng);
    R mu = hg_mu<R>(g, umu);
    int q = X.imgmap[j];
    if (q >= 0) {
      for (int v = 0; v < M.nview; ++v) {
        R cb = P.d[0] * (R)M.kv[v][0] + P.d[1] * (R)M.kv[v][1] + P.d[2] * (R)M.kv[v][2];
        // sums kept in units of ssca_unit (the packet energy): erg/s sums overflow FP32
        R add = (R)(M.xi / M.ssca_unit) * hg_phase<R>(g, cb);
        gatomic_add((R *)M.ssca + ((int64_t)c * M.nview + v) * M.nimg + q, add);
      }
      if (!FAST && M.sh_order > 0) {
        const int nlm = M.sh_order * M.sh_order;
        sh_deposit<R>((R *)M.sh + ((int64_t)c * M.nimg + q) * nlm, M.sh_order, (double)P.d[0],
                      (double)P.d[1], (double)P.d[2], (double)g, M.xi / M.ssca_unit);
      }
    }
    rotate_dir<R>(P.d, mu, (R)2 * (R)PI_D * uph);
    P.n_scat++;
    stat_add(X.st, 5, 1ull);
  } else {
    int s = pick_asc<R, REC>(X.rt + X.o.r_fabs + j, nl, ns, usp, P.mm);
    if constexpr (FAST) {
      // Eq. 4's right-hand side is at least one packet's energy over the cell
      if (s != M.pah &&
          !(M.xi >= M.herm_pmin[s] * (4.0 * PI_D * X.dt[X.o.frac + s] * (double)P.rho * Vl))) {
        *defer = 1;
        return;
      }
    }
    P.n_abs++;
    stat_add(X.st, 6, 1ull);
    if (s == M.pah) {
      if (M.pass != 2) {
        gatomic_add(&M.kpah[c], 1u);
        P.status = ST_PAH_STOP;
        return;
      }
      double ul = rng_u<double>(P.rng), uph = rng_u<double>(P.rng), umu = rng_u<double>(P.rng);
      P.j = pick_pah<R, REC>(X, pah_row(X, c, (double)P.rho, Vl), ul, P.mm);
      iso_dir<R>(uph, umu, P.d);
    } else {
      const R rho = P.rho;
      const bool thin = M.ref ? is_thin_h(X, rho, hl) : is_thin(X, rho);
      int64_t qk = (int64_t)s * X.nc + c;
      double T = 0.0;
      if (M.mode == M_BW_TICKET) {
        uint64_t kold = thin ? gld(&M.k[qk])
                             : gatomic_add(&M.k[qk], (uint64_t)1);
        double e = (double)kold * M.xi + gld(&M.epath[qk]);  // racy read, as in mode_T
        double rhs = (e + M.xi) / (4.0 * PI_D * X.dt[X.o.frac + s] * (double)rho * Vl);
        bool cl = false;
        if constexpr (FAST) T = invert_T_table(M.herm, s, rhs, &cl);
        else T = invert_T_fast(M.herm, X.dt, X.o, nl, s, rhs, &cl);
        if (cl) stat_add(X.st, 9, 1ull);
      } else if constexpr (!FAST) {
        if (!thin) gatomic_add(&M.k[qk], (uint64_t)1);
        T = mode_T(X, s, c, (double)rho, Vl);
      }
      if (M.mode == M_BW_EPOCH) M.dirty[c] = 1;
      int jr = -1;
      if constexpr (sizeof(R) == 4) jr = rej_thermal(X, s, T, P.rng);
      if (jr < 0) {
        R ul = rng_u<R>(P.rng);
        jr = pick_thermal<R, REC>(X, s, T, ul, P.mm);
      }
      P.j = jr;
      double uph = rng_u<double>(P.rng), umu = rng_u<double>(P.rng);
      iso_dir<R>(uph, umu, P.d);
    }
  }
  P.n_int++;
  if (M.max_int > 0 && P.n_int >= M.max_int) P.status = ST_KILLED;
}

// ------------------------------------------------------------- wavefront
// Per-block set-up shared by the kernels below: the model's constants in
// Ctx and its tables staged in LDS. The walk needs only the R table (it
// reads the extinction of its wavelength and, in thin cells, the Lucy
// factors) and the SED; the other kernels take every table.
template <typename R>
__device__ void stage_model(Ctx<R> &X, const ModelDev &M, unsigned char *lds_raw,
                            unsigned long long *s_stat, bool full, bool with_occ = false) {
  X.M = &M;
  X.o = tab_offsets(M.nl, M.ns, M.nsrc, M.nrows);
  X.nc = (int64_t)M.ncell;
  X.rho = (const R *)M.rho;
  X.rho_thin = (M.lucy_tau > 0.0) ? (R)(M.lucy_tau / (M.kext_max * M.dcell)) : (R)0;
  X.og[0] = (R)M.origin[0]; X.og[1] = (R)M.origin[1]; X.og[2] = (R)M.origin[2];
  X.dc = (R)M.dcell;
  X.nx = M.nx; X.ny = M.ny; X.nz = M.nz;
  X.rho_b = (const R *)M.rho_b;
  X.nbx = M.nbx; X.nby = M.nby;
  X.osh = M.osh;
  double *dt = (double *)lds_raw;
  R *rt = full ? (R *)(dt + X.o.dtotal) : (R *)lds_raw;
  int *im = (int *)(rt + X.o.r_total + (X.o.r_total & 1));
  uint32_t *sed = (uint32_t *)(im + M.nl + (M.nl & 1));
  if (full) {
#pragma unroll 8
    for (int i = threadIdx.x; i < X.o.dtotal; i += blockDim.x) dt[i] = gld(M.tab + i);
  }
#pragma unroll 8
  for (int i = threadIdx.x; i < X.o.r_total; i += blockDim.x) rt[i] = gld((const R *)M.rtab + i);
  for (int i = threadIdx.x; i < M.nl; i += blockDim.x) im[i] = M.imgmap[i];
  const int nsed = (M.ntheta > 0 ? M.ntheta : 1) * M.nl;
  for (int i = threadIdx.x; i < nsed; i += blockDim.x) sed[i] = 0u;
  uint32_t *occ = sed + nsed;
  if (!full || with_occ) {
#pragma unroll 8
    for (int i = threadIdx.x; i < M.ow; i += blockDim.x) occ[i] = gld(M.occ + i);
  }
  if (threadIdx.x < NSTAT) s_stat[threadIdx.x] = 0ull;
  __syncthreads();
  X.occ = (!full || with_occ) ? occ : nullptr;
  X.dt = full ? dt : nullptr;
  X.rt = rt;
  X.imgmap = im;
  X.sed = sed;
  X.st = s_stat;
}

// Block SED and statistics into the model's tallies.
template <typename R>
__device__ void flush_block(const Ctx<R> &X) {
  const ModelDev &M = *X.M;
  __syncthreads();
  const int nsed = (M.ntheta > 0 ? M.ntheta : 1) * M.nl;
  for (int i = threadIdx.x; i < nsed; i += blockDim.x)
    if (X.sed[i]) atomicAdd((unsigned long long *)&M.sed[i], (unsigned long long)X.sed[i]);
  if (threadIdx.x < NSTAT && X.st[threadIdx.x]) atomicAdd(&M.stats[threadIdx.x], X.st[threadIdx.x]);
  __syncthreads();
}

__device__ __forceinline__ uint64_t pack_cj(const int c[3], int j) {
  return (uint64_t)(uint32_t)c[0] | ((uint64_t)(uint32_t)c[1] << CJ_BITS) |
         ((uint64_t)(uint32_t)c[2] << (2 * CJ_BITS)) | ((uint64_t)(uint32_t)j << (3 * CJ_BITS));
}
__device__ __forceinline__ void unpack_cj(uint64_t w, int c[3], int &j) {
  const uint64_t m = (1ull << CJ_BITS) - 1ull;
  c[0] = (int)(w & m);
  c[1] = (int)((w >> CJ_BITS) & m);
  c[2] = (int)((w >> (2 * CJ_BITS)) & m);
  j = (int)(w >> (3 * CJ_BITS));
}

template <typename R, bool REC>
__device__ __forceinline__ void q_store(const QBuf &b, uint32_t i, const Pkt<R> &P, R tau) {
  ((R *)b.px)[i] = P.p[0]; ((R *)b.py)[i] = P.p[1]; ((R *)b.pz)[i] = P.p[2];
  ((R *)b.dx)[i] = P.d[0]; ((R *)b.dy)[i] = P.d[1]; ((R *)b.dz)[i] = P.d[2];
  ((R *)b.rho)[i] = P.rho;
  ((R *)b.tau)[i] = tau;
  b.cj[i] = pack_cj(P.c, P.j);
  b.pid[i] = P.pid;
  b.rngd[i] = P.rng.d;
  b.nint[i] = P.n_int;
  if (b.fine) b.fine[i] = P.fpk;
  if (REC) {
    b.ncross[i] = P.n_cross; b.nscat[i] = P.n_scat; b.nabs[i] = P.n_abs;
    b.nmrw[i] = P.n_mrw; b.nlucy[i] = P.n_lucy;
    b.mm[i] = P.mm;
  }
}

// Loads a queued packet; its RNG stream is re-keyed from the packet id and
// continues at the stored draw index.
template <typename R, bool REC>
__device__ __forceinline__ R q_load(const ModelDev &M, const QBuf &b, uint32_t i, Pkt<R> &P) {
  P.p[0] = gld((const R *)b.px + i); P.p[1] = gld((const R *)b.py + i);
  P.p[2] = gld((const R *)b.pz + i);
  P.d[0] = gld((const R *)b.dx + i); P.d[1] = gld((const R *)b.dy + i);
  P.d[2] = gld((const R *)b.dz + i);
  P.rho = gld((const R *)b.rho + i);
  const R tau = gld((const R *)b.tau + i);
  unpack_cj(gld(b.cj + i), P.c, P.j);
  P.pid = gld(b.pid + i);
  rng_init(P.rng, M.seed, P.pid, (uint32_t)M.iter, (uint32_t)M.model_id, M.pass == 2 ? 3u : 0u);
  P.rng.d = gld(b.rngd + i);
  P.n_int = gld(b.nint + i);
  P.fpk = b.fine ? gld(b.fine + i) : 0u;
  P.status = ST_ALIVE;
  P.n_cross = P.n_scat = P.n_abs = P.n_mrw = P.n_lucy = 0;
  P.mm = 1e300;
  if (REC) {
    P.n_cross = gld(b.ncross + i); P.n_scat = gld(b.nscat + i); P.n_abs = gld(b.nabs + i);
    P.n_mrw = gld(b.nmrw + i); P.n_lucy = gld(b.nlucy + i);
    P.mm = gld(b.mm + i);
  }
  return tau;
}

// ---- segmented queues (see WfCtl)
__device__ __forceinline__ int home_segment() {
  return (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (NSEG - 1));
}

__device__ __forceinline__ uint32_t seg_count(const WfCtl *c, int f, int g, uint32_t S) {
  const uint32_t v = gload_relaxed(&c->nseg[f][g][0]);
  return v < S ? v : S;
}

// Next chunk [lo, hi) of up to 64 entries for this wave from work counter
// k, searching the segments from g on; seg(g, beg, cnt) gives the entries
// of segment g. False once every segment is handed out. Wave-uniform.
template <typename Seg>
__device__ __forceinline__ bool seg_grab(WfCtl *c, int k, int &g, int lane, uint32_t &lo,
                                         uint32_t &hi, Seg seg) {
  for (int t = 0; t < NSEG; ++t) {
    uint32_t beg, cnt;
    seg(g, beg, cnt);
    if (gload_relaxed(&c->work[k][g][0]) < cnt) {
      uint32_t base = 0u;
      if (lane == 0) base = gatomic_add(&c->work[k][g][0], 64u);
      base = (uint32_t)__shfl((int)base, 0);
      if (base < cnt) {
        lo = beg + base;
        hi = beg + (base + 64u < cnt ? base + 64u : cnt);
        return true;
      }
    }
    g = (g + 1) & (NSEG - 1);
  }
  return false;
}

// One slot of queue f per lane with pred: appended to segment g, spilling
// into the next segments when it is full. Every lane of the wave calls;
// returns the slot of a pred lane. The queue's capacity always covers the
// packets appended in a round (at most the packets it started with).
__device__ __forceinline__ uint32_t seg_reserve(WfCtl *c, int f, uint32_t S, int g, bool pred,
                                                int lane, uint64_t lt_mask) {
  const uint64_t m = __ballot(pred);
  const uint32_t k = (uint32_t)__popcll(m), rank = (uint32_t)__popcll(m & lt_mask);
  uint32_t slot = 0xFFFFFFFFu, done = 0u;
  for (int t = 0; t < NSEG && done < k; ++t) {
    uint32_t base = 0u;
    if (lane == 0) base = gatomic_add(&c->nseg[f][g][0], k - done);
    base = (uint32_t)__shfl((int)base, 0);
    const uint32_t room = base < S ? S - base : 0u;
    const uint32_t got = room < k - done ? room : k - done;
    if (pred && rank >= done && rank < done + got) slot = (uint32_t)g * S + base + (rank - done);
    done += got;
    g = (g + 1) & (NSEG - 1);
  }
  return slot;
}

// Queues the packet at its reserved slot. A slot outside the queue cannot
// occur (capacity covers a round's appends); were it to, the packet would be
// ended as killed rather than written out of bounds.
template <typename R, bool REC>
__device__ __forceinline__ void store_or_drop(Ctx<R> &X, const QBuf &q, uint32_t slot, Pkt<R> &P,
                                              R tau) {
  if (slot < X.M->qcap) {
    q_store<R, REC>(q, slot, P, tau);
  } else {
    P.status = ST_KILLED;
    finish<R, REC>(X, P, true);
  }
}

// Round set-up (one block per model): how many new packets to start, and
// the counters of the queue this round fills.
__global__ void k_wf_plan(const ModelDev *__restrict__ models, int nmodels, int fcur) {
  const ModelDev &M = models[blockIdx.x];
  WfCtl *c = M.ctl;
  __shared__ uint32_t s_held;
  if (threadIdx.x == 0) s_held = 0u;
  __syncthreads();
  for (int g = threadIdx.x; g < NSEG; g += blockDim.x) {
    const uint32_t v = c->nseg[fcur][g][0];
    atomicAdd(&s_held, v < M.qseg ? v : M.qseg);
    c->nseg[1 - fcur][g][0] = 0u;
    c->work[0][g][0] = c->work[1][g][0] = c->work[2][g][0] = 0u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t left = M.n > c->emitted ? M.n - c->emitted : 0;
    const uint32_t room = M.qcap > s_held ? M.qcap - s_held : 0u;
    const uint32_t take = left < (uint64_t)room ? (uint32_t)left : room;
    c->first = c->emitted;
    c->emitted += take;
    c->take = take;
    c->inq = s_held + take;
    c->nslow = 0u;
  }
}

// Emission: new packets of the launch are started, sample the optical
// depth of their first flight and join flight-ready queue fcur.
template <typename R, bool REC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_wf_emit(const ModelDev *__restrict__ models, int nmodels, int fcur) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ unsigned long long s_stat[NSTAT];
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int mm = 0; mm < nmodels; ++mm) {
    const ModelDev &M = models[(blockIdx.x + mm) % nmodels];
    WfCtl *c = M.ctl;
    const uint32_t take = c->take;
    if (take == 0u) continue;
    Ctx<R> X;
    stage_model<R>(X, M, lds_raw, s_stat, true);
    const QBuf &qo = M.q[fcur];
    const int home = home_segment();
    int g = home;
    // the round's new packets in NSEG equal slices, one per segment
    auto slice = [&](int s, uint32_t &beg, uint32_t &cnt) {
      beg = (uint32_t)((uint64_t)take * (uint64_t)s / NSEG);
      cnt = (uint32_t)((uint64_t)take * (uint64_t)(s + 1) / NSEG) - beg;
    };
    uint32_t lo, hi;
    while (seg_grab(c, 0, g, lane, lo, hi, slice)) {
      const uint32_t i = lo + (uint32_t)lane;
      Pkt<R> P;
      R tau = (R)-1;
      bool keep = false;
      if (i < hi) {
        start_packet<R, REC>(X, P, c->first + i);
        if (P.status == ST_ALIVE) tau = flight_tau<R, REC>(X, P);
        keep = P.status == ST_ALIVE;
        if (!keep) finish<R, REC>(X, P, true);
      }
      const uint32_t slot = seg_reserve(c, fcur, M.qseg, home, keep, lane, lt_mask);
      if (keep) store_or_drop<R, REC>(X, qo, slot, P, tau);
    }
    flush_block(X);
  }
}

// The walk's share of a queued packet. Without records or per-cell draws a
// flight reads only position, direction, cell and wavelength, sub-cube and
// depth, and at an interaction changes only position, cell (the word it
// shares with the wavelength), sub-cube and density: the id, draw index,
// interaction count, direction and wavelength stay in the entry as the
// interaction kernel reads them, and that kernel does not read the depth.
// With records or per-cell draws the whole packet moves.
template <typename R, bool REC, bool PC>
__device__ __forceinline__ R q_load_walk(const ModelDev &M, const QBuf &b, uint32_t i, Pkt<R> &P) {
  if constexpr (REC || PC) {
    return q_load<R, REC>(M, b, i, P);
  } else {
    P.p[0] = gld((const R *)b.px + i); P.p[1] = gld((const R *)b.py + i);
    P.p[2] = gld((const R *)b.pz + i);
    P.d[0] = gld((const R *)b.dx + i); P.d[1] = gld((const R *)b.dy + i);
    P.d[2] = gld((const R *)b.dz + i);
    const R tau = gld((const R *)b.tau + i);
    unpack_cj(gld(b.cj + i), P.c, P.j);
    P.fpk = b.fine ? gld(b.fine + i) : 0u;
    P.rho = (R)0;
    P.status = ST_ALIVE;
    P.n_cross = P.n_scat = P.n_abs = P.n_mrw = P.n_lucy = 0;
    P.mm = 1e300;
    return tau;
  }
}

template <typename R, bool REC, bool PC>
__device__ __forceinline__ void q_store_walk(const QBuf &b, uint32_t i, const Pkt<R> &P) {
  if constexpr (REC || PC) {
    q_store<R, REC>(b, i, P, (R)0);
  } else {
    ((R *)b.px)[i] = P.p[0]; ((R *)b.py)[i] = P.p[1]; ((R *)b.pz)[i] = P.p[2];
    ((R *)b.rho)[i] = P.rho;
    b.cj[i] = pack_cj(P.c, P.j);
    if (b.fine) b.fine[i] = P.fpk;
  }
}

// Voxel walk of every flight-ready packet of queue fcur to its next
// interaction or out of the grid; the packet is written back to its own
// entry. Lanes refill one by one from a wave-local chunk, so flights of
// different lengths keep the wave busy.
template <typename R, bool REC, bool I32, bool PC, bool REF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_wf_walk(const ModelDev *__restrict__ models, int nmodels, int fcur) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ unsigned long long s_stat[NSTAT];
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int mm = 0; mm < nmodels; ++mm) {
    const ModelDev &M = models[(blockIdx.x + mm) % nmodels];
    WfCtl *c = M.ctl;
    if (c->inq == 0u) continue;
    Ctx<R> X;
    stage_model<R>(X, M, lds_raw, s_stat, false);
    const QBuf &qi = M.q[fcur];
    const uint32_t S = M.qseg;
    auto seg = [&](int s, uint32_t &beg, uint32_t &cnt) {
      beg = (uint32_t)s * S;
      cnt = seg_count(c, fcur, s, S);
    };
    Pkt<R> P;
    typename std::conditional<REF, FlightRef<R>, Flight<R>>::type F;
    uint32_t mine = 0u;         // queue entry of the lane's packet
    uint32_t c0 = 0u, l0 = 0u;  // crossings and Lucy deposits before this flight
    uint32_t plo = 0u, phi = 0u;  // wave-local chunk of entries not yet started
    int g = home_segment();
    bool more = true;           // some segment may still hand out entries
    int state = 0;              // 0 needs a packet, 1 walking, 2 no work left
    for (;;) {
      const uint64_t need = __ballot(state == 0);
      if (need) {
        const uint32_t k = (uint32_t)__popcll(need);
        const uint32_t rank = (uint32_t)__popcll(need & lt_mask);
        const uint32_t avail = phi - plo;
        uint32_t flo = 0u, fhi = 0u;
        if (k > avail && more) more = seg_grab(c, 1, g, lane, flo, fhi, seg);
        if (state == 0) {
          uint32_t i = 0xFFFFFFFFu;
          if (rank < avail) i = plo + rank;
          else if (rank - avail < fhi - flo) i = flo + (rank - avail);
          if (i != 0xFFFFFFFFu) {
            mine = i;
            const R tau = q_load_walk<R, REC, PC>(M, qi, i, P);
            if constexpr (REF) flight_setup_ref<R>(X, P, F, tau);
            else flight_setup<R>(X, P, F, tau);
            c0 = P.n_cross;
            l0 = P.n_lucy;
            state = 1;
          } else if (!more) {
            state = 2;
          }
        }
        if (k > avail) {
          const uint32_t used = k - avail < fhi - flo ? k - avail : fhi - flo;
          plo = flo + used;
          phi = fhi;
        } else {
          plo += k;
        }
      }
      if (!__any(state != 2)) break;
      int r = 0;
      if (state == 1) {
        if constexpr (REF) r = flight_batch_ref<R, REC, PC>(X, P, F);
        else r = flight_batch<R, REC, I32, PC>(X, P, F);
      }
      if (r != 0) {
        stat_add(X.st, 4, (unsigned long long)(P.n_cross - c0));
        if (P.n_lucy != l0) stat_add(X.st, 8, (unsigned long long)(P.n_lucy - l0));
        state = 0;
      }
      // the packet goes back to its own entry, which the interaction kernel
      // reads next; an escape leaves the entry marked free (CJ_FREE)
      if (r == 1) {
        q_store_walk<R, REC, PC>(qi, mine, P);
      } else if (r == 2) {
        qi.cj[mine] = CJ_FREE;
        P.status = ST_ESCAPED;
        finish<R, REC>(X, P, true);
      }
    }
    flush_block(X);
  }
}

// Interactions of the walked queue fcur (entries freed by escapes are
// skipped); survivors sample their next flight and join flight-ready queue
// 1 - fcur. FAST (immediate B&W without records or moments): the rare
// interactions that need the FP64 Newton solve of Eq. 4 or the exact
// diffusion test go to the walked queue's slow list instead (the entry
// keeps the packet: untouched for a whole interaction, rewritten when only
// the next flight's start remains) and k_wf_slow finishes them. Without the
// out-of-line FP64 calls the fast kernel needs 158 VGPRs and no scratch; the
// general one spills at 256.
template <typename R, bool REC, bool FAST>
__device__ __forceinline__ void interact_round(const ModelDev *__restrict__ models, int nmodels,
                                               int fcur, unsigned char *lds_raw,
                                               unsigned long long *s_stat) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int mm = 0; mm < nmodels; ++mm) {
    const ModelDev &M = models[(blockIdx.x + mm) % nmodels];
    WfCtl *c = M.ctl;
    if (c->inq == 0u) continue;
    Ctx<R> X;
    stage_model<R>(X, M, lds_raw, s_stat, true);
    const QBuf &qi = M.q[fcur];
    const QBuf &qo = M.q[1 - fcur];
    const uint32_t S = M.qseg;
    auto seg = [&](int s, uint32_t &beg, uint32_t &cnt) {
      beg = (uint32_t)s * S;
      cnt = seg_count(c, fcur, s, S);
    };
    const int home = home_segment();
    int g = home;
    uint32_t lo, hi;
    while (seg_grab(c, 2, g, lane, lo, hi, seg)) {
      const uint32_t i = lo + (uint32_t)lane;
      Pkt<R> P;
      R tau = (R)-1;
      bool keep = false;
      if (i < hi && gld(qi.cj + i) != CJ_FREE) {
        (void)q_load<R, REC>(M, qi, i, P);
        int defer = 0;
        interact<R, REC, FAST>(X, P, &defer);
        if (P.status == ST_ALIVE && defer == 0) tau = flight_tau<R, REC, FAST>(X, P, &defer);
        if (FAST && defer != 0) {
          if (defer == 2) q_store<R, REC>(qi, i, P, (R)0);
          const uint32_t k = gatomic_add(&c->nslow, 1u);
          qi.slow[k] = defer == 2 ? (i | SLOW_FLIGHT) : i;
        } else {
          keep = P.status == ST_ALIVE;
          if (!keep) finish<R, REC>(X, P, true);
        }
      }
      const uint32_t slot = seg_reserve(c, 1 - fcur, S, home, keep, lane, lt_mask);
      if (keep) store_or_drop<R, REC>(X, qo, slot, P, tau);
    }
    flush_block(X);
  }
}

template <typename R, bool REC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_wf_interact(const ModelDev *__restrict__ models, int nmodels, int fcur) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ unsigned long long s_stat[NSTAT];
  interact_round<R, REC, false>(models, nmodels, fcur, lds_raw, s_stat);
}

template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_wf_interact_fast(const ModelDev *__restrict__ models, int nmodels, int fcur) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ unsigned long long s_stat[NSTAT];
  interact_round<R, false, true>(models, nmodels, fcur, lds_raw, s_stat);
}

// The slow list of the walked queue fcur: whole interactions (the queued
// state as the fast kernel found it) or only the start of the next flight,
// with the general device functions; survivors join queue 1 - fcur like
// the fast kernel's.
template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_wf_slow(const ModelDev *__restrict__ models, int nmodels, int fcur) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ unsigned long long s_stat[NSTAT];
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int mm = 0; mm < nmodels; ++mm) {
    const ModelDev &M = models[(blockIdx.x + mm) % nmodels];
    WfCtl *c = M.ctl;
    const uint32_t n = c->nslow;  // written by the fast kernel before this launch
    if (n == 0u) continue;
    Ctx<R> X;
    stage_model<R>(X, M, lds_raw, s_stat, true);
    const QBuf &qi = M.q[fcur];
    const QBuf &qo = M.q[1 - fcur];
    const uint32_t S = M.qseg;
    const int home = home_segment();
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t nwave = gridDim.x * (blockDim.x >> 6);
    // every lane of a wave runs the same iterations (queue appends are
    // wave-wide)
    for (uint32_t b = wave * 64u; b < n; b += nwave * 64u) {
      const uint32_t k = b + (uint32_t)lane;
      Pkt<R> P;
      R tau = (R)-1;
      bool keep = false;
      if (k < n) {
        const uint32_t e = gld(qi.slow + k);
        const uint32_t i = e & ~SLOW_FLIGHT;
        (void)q_load<R, false>(M, qi, i, P);
        if (!(e & SLOW_FLIGHT)) interact<R, false>(X, P);
        if (P.status == ST_ALIVE) tau = flight_tau<R, false>(X, P);
        keep = P.status == ST_ALIVE;
        if (!keep) finish<R, false>(X, P, true);
      }
      const uint32_t slot = seg_reserve(c, 1 - fcur, S, home, keep, lane, lt_mask);
      if (keep) store_or_drop<R, false>(X, qo, slot, P, tau);
    }
    flush_block(X);
  }
}

size_t walk_lds_bytes(int nl, int ns, int nsrc, int nrows, int ntheta, int occ_words, bool fp64) {
  TabOff o = tab_offsets(nl, ns, nsrc, nrows);
  size_t rs = fp64 ? 8 : 4;
  return (size_t)(o.r_total + (o.r_total & 1)) * rs + (size_t)(nl + (nl & 1)) * 4 +
         (size_t)(ntheta > 0 ? ntheta : 1) * nl * 4 + (size_t)occ_words * 4;
}

template <typename R, bool REC>
static void wf_phases(const ModelDev *d_models, int nmodels, int fcur, int grid_full, int grid_walk,
                      size_t lds_full, size_t lds_walk, bool idx32, bool per_cell, bool refined,
                      int fast, const hipEvent_t *ev, hipStream_t st) {
  if (ev) (void)hipEventRecord(ev[0], st);
  hipLaunchKernelGGL((k_wf_emit<R, REC>), dim3(grid_full), dim3(256), lds_full, st, d_models,
                     nmodels, fcur);
  if (ev) (void)hipEventRecord(ev[1], st);
  // refined grids take the leaf walk; the per-cell draw variant of the
  // bricked walk uses 64-bit cell indices on any grid
  if (refined && per_cell)
    hipLaunchKernelGGL((k_wf_walk<R, REC, false, true, true>), dim3(grid_walk), dim3(256),
                       lds_walk, st, d_models, nmodels, fcur);
  else if (refined)
    hipLaunchKernelGGL((k_wf_walk<R, REC, false, false, true>), dim3(grid_walk), dim3(256),
                       lds_walk, st, d_models, nmodels, fcur);
  else if (per_cell)
    hipLaunchKernelGGL((k_wf_walk<R, REC, false, true, false>), dim3(grid_walk), dim3(256),
                       lds_walk, st, d_models, nmodels, fcur);
  else if (idx32)
    hipLaunchKernelGGL((k_wf_walk<R, REC, true, false, false>), dim3(grid_walk), dim3(256),
                       lds_walk, st, d_models, nmodels, fcur);
  else
    hipLaunchKernelGGL((k_wf_walk<R, REC, false, false, false>), dim3(grid_walk), dim3(256),
                       lds_walk, st, d_models, nmodels, fcur);
  if (ev) (void)hipEventRecord(ev[2], st);
  // the fast interaction kernel serves the FP32 walk (see interact_round)
  if constexpr (!REC && sizeof(R) == 4) {
    if (fast) {
      if (fast == 2)
        hipLaunchKernelGGL((k_mrw_flags<R>), dim3(grid_full), dim3(256), 0, st, d_models, nmodels);
      hipLaunchKernelGGL((k_wf_interact_fast<R>), dim3(grid_full), dim3(256), lds_full, st,
                         d_models, nmodels, fcur);
      hipLaunchKernelGGL((k_wf_slow<R>), dim3(grid_full), dim3(256), lds_full, st, d_models,
                         nmodels, fcur);
      if (ev) (void)hipEventRecord(ev[3], st);
      return;
    }
  }
  hipLaunchKernelGGL((k_wf_interact<R, REC>), dim3(grid_full), dim3(256), lds_full, st, d_models,
                     nmodels, fcur);
  if (ev) (void)hipEventRecord(ev[3], st);
}

// Candidate bits of the per-cell diffusion flags (once per launch, after
// the models are on the device).
hipError_t launch_mrw_cand(const ModelDev *d_models, int nmodels, int ncu, hipStream_t st) {
  hipLaunchKernelGGL(k_mrw_cand<float>, dim3(ncu * 4), dim3(256), 0, st, d_models, nmodels);
  return hipGetLastError();
}

// One round for nmodels models: plan, emit, walk, interact (stream order).
// idx32: every model's bricked grid has fewer than 2^32 cells. ev (null or
// four events) brackets the emission, walk and interaction kernels.
hipError_t launch_wf_round(const ModelDev *d_models, int nmodels, bool fp64, bool rec, int fcur,
                           int grid_full, int grid_walk, size_t lds_full, size_t lds_walk,
                           bool idx32, bool per_cell, bool refined, int fast,
                           const hipEvent_t *ev, hipStream_t st) {
  hipLaunchKernelGGL(k_wf_plan, dim3(nmodels), dim3(64), 0, st, d_models, nmodels, fcur);
  if (fp64) {
    if (rec) wf_phases<double, true>(d_models, nmodels, fcur, grid_full, grid_walk, lds_full, lds_walk, idx32, per_cell, refined, fast, ev, st);
    else wf_phases<double, false>(d_models, nmodels, fcur, grid_full, grid_walk, lds_full, lds_walk, idx32, per_cell, refined, fast, ev, st);
  } else {
    if (rec) wf_phases<float, true>(d_models, nmodels, fcur, grid_full, grid_walk, lds_full, lds_walk, idx32, per_cell, refined, fast, ev, st);
    else wf_phases<float, false>(d_models, nmodels, fcur, grid_full, grid_walk, lds_full, lds_walk, idx32, per_cell, refined, fast, ev, st);
  }
  return hipGetLastError();
}

// Number of models with packets left after a round whose emptied queue
// was fcur (one block; nmodels <= 1024).
// (and, when `left` is not null, the packets queued for the next round
// over all models, or 0xFFFFFFFF while some model has packets not yet
// started)
__global__ void k_wf_busy(const ModelDev *__restrict__ models, int nmodels, int fcur,
                          uint32_t *busy, uint32_t *left) {
  __shared__ uint32_t s_busy, s_left, s_unstarted;
  if (threadIdx.x == 0) s_busy = s_left = s_unstarted = 0u;
  __syncthreads();
  for (int m = threadIdx.x; m < nmodels; m += blockDim.x) {
    const ModelDev &M = models[m];
    const WfCtl *c = M.ctl;
    const bool unstarted = c->emitted < M.n;
    uint32_t q = 0u;
    for (int g = 0; g < NSEG; ++g) q += seg_count(c, 1 - fcur, g, M.qseg);
    if (unstarted || q > 0u) atomicAdd(&s_busy, 1u);
    if (unstarted) atomicAdd(&s_unstarted, 1u);
    atomicAdd(&s_left, q);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *busy = s_busy;
    if (left) *left = s_unstarted ? 0xFFFFFFFFu : s_left;
  }
}

hipError_t launch_wf_busy(const ModelDev *d_models, int nmodels, int fcur, uint32_t *busy,
                          uint32_t *left, hipStream_t st) {
  hipLaunchKernelGGL(k_wf_busy, dim3(1), dim3(256), 0, st, d_models, nmodels, fcur, busy, left);
  return hipGetLastError();
}

// The last packets of a launch, once every packet has been started: each
// lane takes a flight-ready entry of queue fcur and follows its packet
// through every flight and interaction until it ends, with the device
// functions and draw order of the rounds (so each packet's history is the
// same). Late rounds hold few packets and are as long as their longest
// flight; this replaces them by one launch. A packet still going after
// FINISH_MAX_EVENTS flights in this kernel is ended as killed, so every lane
// reaches the end (no physical packet comes near it).
constexpr uint32_t FINISH_MAX_EVENTS = 1u << 22;

template <typename R, bool REC, bool I32, bool PC, bool REF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_wf_finish(const ModelDev *__restrict__ models, int nmodels, int fcur) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ unsigned long long s_stat[NSTAT];
  const int lane = threadIdx.x & 63;
  for (int mm = 0; mm < nmodels; ++mm) {
    const ModelDev &M = models[(blockIdx.x + mm) % nmodels];
    WfCtl *c = M.ctl;
    if (c->inq == 0u) continue;
    Ctx<R> X;
    stage_model<R>(X, M, lds_raw, s_stat, true, true);
    const QBuf &qi = M.q[fcur];
    const uint32_t S = M.qseg;
    auto seg = [&](int s, uint32_t &beg, uint32_t &cnt) {
      beg = (uint32_t)s * S;
      cnt = seg_count(c, fcur, s, S);
    };
    int g = home_segment();
    uint32_t lo, hi;
    while (seg_grab(c, 1, g, lane, lo, hi, seg)) {
      const uint32_t i = lo + (uint32_t)lane;
      if (i >= hi) continue;
      Pkt<R> P;
      typename std::conditional<REF, FlightRef<R>, Flight<R>>::type F;
      R tau = q_load<R, REC>(M, qi, i, P);
      for (uint32_t ev = 0;; ++ev) {
        if (ev >= FINISH_MAX_EVENTS) {
          P.status = ST_KILLED;
          finish<R, REC>(X, P, true);
          break;
        }
        if constexpr (REF) flight_setup_ref<R>(X, P, F, tau);
        else flight_setup<R>(X, P, F, tau);
        const uint32_t c0 = P.n_cross, l0 = P.n_lucy;
        int r;
        do {
          if constexpr (REF) r = flight_batch_ref<R, REC, PC>(X, P, F);
          else r = flight_batch<R, REC, I32, PC>(X, P, F);
        } while (r == 0);
        stat_add(X.st, 4, (unsigned long long)(P.n_cross - c0));
        if (P.n_lucy != l0) stat_add(X.st, 8, (unsigned long long)(P.n_lucy - l0));
        if (r == 2) {
          P.status = ST_ESCAPED;
          finish<R, REC>(X, P, true);
          break;
        }
        interact<R, REC>(X, P);
        if (P.status == ST_ALIVE) tau = flight_tau<R, REC>(X, P);
        if (P.status != ST_ALIVE) {
          finish<R, REC>(X, P, true);
          break;
        }
      }
    }
    flush_block(X);
  }
}

// Plan of the next round (no new packets remain) and the finishing kernel.
hipError_t launch_wf_finish(const ModelDev *d_models, int nmodels, bool fp64, bool rec, int fcur,
                            int grid, size_t lds, bool idx32, bool per_cell, bool refined,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_wf_plan, dim3(nmodels), dim3(64), 0, st, d_models, nmodels, fcur);
#define MCRT_FIN(RT, RC, IX, PC, RF)                                                             \
  hipLaunchKernelGGL((k_wf_finish<RT, RC, IX, PC, RF>), dim3(grid), dim3(256), lds, st,          \
                     d_models, nmodels, fcur)
#define MCRT_FIN2(RT, RC)                                                                        \
  do {                                                                                           \
    if (refined && per_cell) MCRT_FIN(RT, RC, false, true, true);                                \
    else if (refined) MCRT_FIN(RT, RC, false, false, true);                                      \
    else if (per_cell) MCRT_FIN(RT, RC, false, true, false);                                     \
    else if (idx32) MCRT_FIN(RT, RC, true, false, false);                                        \
    else MCRT_FIN(RT, RC, false, false, false);                                                  \
  } while (0)
  if (fp64) {
    if (rec) MCRT_FIN2(double, true);
    else MCRT_FIN2(double, false);
  } else {
    if (rec) MCRT_FIN2(float, true);
    else MCRT_FIN2(float, false);
  }
#undef MCRT_FIN2
#undef MCRT_FIN
  return hipGetLastError();
}

// n draws of the re-emission bin of species s at temperature T, exactly as
// an absorption in the transport takes them (FP32: rejection with the
// inverse CDF as fallback; FP64: the inverse CDF), counted per bin.
template <typename R>
__global__ void __launch_bounds__(256) k_sample_reem(const ModelDev *__restrict__ md, int s, double T,
                                                     uint64_t n, uint64_t seed,
                                                     unsigned long long *counts) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ unsigned long long s_stat[NSTAT];
  __shared__ unsigned int hist[256];
  const ModelDev &M = *md;
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0u;
  Ctx<R> X;
  stage_model<R>(X, M, lds_raw, s_stat, true);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    Rng rng;
    rng_init(rng, seed, i, 0u, 0u, 7u);
    int j = -1;
    if constexpr (sizeof(R) == 4) j = rej_thermal(X, s, T, rng);
    if (j < 0) {
      double mm = 1e300;
      const R u = rng_u<R>(rng);
      j = pick_thermal<R, false>(X, s, T, u, mm);
    }
    atomicAdd(&hist[j], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < M.nl; i += blockDim.x)
    if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
}

hipError_t launch_sample_reem(const ModelDev *d, bool fp64, int s, double T, uint64_t n,
                              uint64_t seed, unsigned long long *counts, size_t lds,
                              hipStream_t st) {
  if (fp64)
    hipLaunchKernelGGL(k_sample_reem<double>, dim3(1024), dim3(256), lds, st, d, s, T, n, seed, counts);
  else
    hipLaunchKernelGGL(k_sample_reem<float>, dim3(1024), dim3(256), lds, st, d, s, T, n, seed, counts);
  return hipGetLastError();
}

// Lane-side layout size of the LDS tables for a model.
size_t transport_lds_bytes(int nl, int ns, int nsrc, int nrows, int ntheta, bool fp64) {
  TabOff o = tab_offsets(nl, ns, nsrc, nrows);
  size_t rs = fp64 ? 8 : 4;
  size_t b = (size_t)o.dtotal * 8 + (size_t)(o.r_total + (o.r_total & 1)) * rs +
             (size_t)(nl + (nl & 1)) * 4 + (size_t)(ntheta > 0 ? ntheta : 1) * nl * 4;
  return b;
}

// ------------------------------------------------------- per-cell kernels

// Start of a B&W epoch: cells touched since the last snapshot get their
// energy re-read and lose the cached epoch temperature.
__global__ void k_epoch_snapshot(const ModelDev *__restrict__ md) {
  const ModelDev &M = *md;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < M.ncell; i += stride) {
    if (!M.dirty[i]) continue;
    for (int s = 0; s < M.ns; ++s) {
      int64_t q = (int64_t)s * M.ncell + i;
      double e = energy_of(M, q);
      if (e != M.esnap[q] || M.tt[q] >= 0.0) {
        M.esnap[q] = e;
        M.tt[q] = -1.0;
      }
    }
    M.dirty[i] = 0;
  }
}

// Copy of the density in 4x4x4 bricks for the walk (padding cells stay 0).
template <typename R>
__global__ void k_brick(const R *__restrict__ rho, R *__restrict__ rb, int nx, int ny, int nz,
                        int nbx, int nby) {
  const uint64_t n = (uint64_t)nx * ny * nz;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const int cx = (int)(i % (uint64_t)nx);
    const uint64_t r = i / (uint64_t)nx;
    const int cy = (int)(r % (uint64_t)ny), cz = (int)(r / (uint64_t)ny);
    rb[brick_index(cx, cy, cz, nbx, nby)] = rho[i];
  }
}

// Occupancy bit of each run of 2^(osh - 6) bricks, i.e. of bricked cells
// [r << osh, (r + 1) << osh): set if any of its densities is non-zero. One
// lane per run; each wave writes the two words its 64 lanes cover.
template <typename R>
__global__ void k_occ(const R *__restrict__ rb, uint32_t *__restrict__ occ, uint64_t ncell_b,
                      int osh) {
  const uint64_t nrun = (ncell_b + (1ull << osh) - 1) >> osh;
  const uint64_t lim = (nrun + 63) / 64 * 64;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < lim; t += stride) {
    bool any = false;
    if (t < nrun) {
      const uint64_t b = t << osh, e = min(b + (1ull << osh), ncell_b);
      for (uint64_t i = b; i < e; ++i) any |= rb[i] != (R)0;
    }
    const uint64_t m = __ballot(any);
    const int lane = threadIdx.x & 63;
    if (lane == 0) occ[t >> 5] = (uint32_t)m;
    if (lane == 32) occ[t >> 5] = (uint32_t)(m >> 32);
  }
}

hipError_t launch_occ(bool fp64, const void *rb, uint32_t *occ, uint64_t ncell_b, int osh,
                      hipStream_t st) {
  const uint64_t nrun = (ncell_b + (1ull << osh) - 1) >> osh;
  const uint64_t nb = (nrun + 255) / 256;
  const unsigned g = (unsigned)(nb < 4096 ? nb : 4096);
  if (fp64)
    hipLaunchKernelGGL(k_occ<double>, dim3(g), dim3(256), 0, st, (const double *)rb, occ, ncell_b,
                       osh);
  else
    hipLaunchKernelGGL(k_occ<float>, dim3(g), dim3(256), 0, st, (const float *)rb, occ, ncell_b,
                       osh);
  return hipGetLastError();
}

hipError_t launch_brick(bool fp64, const void *rho, void *rb, int nx, int ny, int nz, int nbx,
                        int nby, hipStream_t st) {
  const uint64_t n = (uint64_t)nx * ny * nz;
  const uint64_t nb = (n + 255) / 256;
  const unsigned g = (unsigned)(nb < 65536 ? nb : 65536);
  if (fp64)
    hipLaunchKernelGGL(k_brick<double>, dim3(g), dim3(256), 0, st, (const double *)rho,
                       (double *)rb, nx, ny, nz, nbx, nby);
  else
    hipLaunchKernelGGL(k_brick<float>, dim3(g), dim3(256), 0, st, (const float *)rho,
                       (float *)rb, nx, ny, nz, nbx, nby);
  return hipGetLastError();
}

// Eq. 4 for every cell and thermal species; optionally also writes E.
template <typename R>
__global__ void k_finalize_T(const ModelDev *__restrict__ md, double *T, double *E) {
  const ModelDev &M = *md;
  TabOff o = tab_offsets(M.nl, M.ns, M.nsrc, M.nrows);
  const R *rho = (const R *)M.rho;
  uint64_t n = M.ncell * (uint64_t)M.ns;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    int s = (int)(i / M.ncell);
    uint64_t c = i - (uint64_t)s * M.ncell;
    double r = (double)rho[c];
    double e = energy_of(M, i);
    double frac = M.tab[o.frac + s];
    double t = 0.0;
    if (s != M.pah && r > 0.0 && frac > 0.0) {
      bool cl = false;
      double rhs = e / (4.0 * PI_D * frac * r * leaf_volume(M, c));
      t = (sizeof(R) == 8) ? invert_T_exact(M.herm, M.tab, o, M.nl, s, rhs, &cl)
                           : invert_T_fast(M.herm, M.tab, o, M.nl, s, rhs, &cl);
      if (cl) atomicAdd(&M.stats[9], 1ull);
    }
    T[i] = t;
    if (E) E[i] = e;
  }
}

// Thin-limit equilibrium temperature at every cell centre (first guess
// of the iterative scheme): Phi_s(T) = sum_j w_j kabs_s,j J_j with
// J_j = sum_src L_nu,j / (16 pi^2 r^2).
template <typename R>
__global__ void k_init_T(const ModelDev *__restrict__ md, double *T) {
  const ModelDev &M = *md;
  TabOff o = tab_offsets(M.nl, M.ns, M.nsrc, M.nrows);
  const R *rho = (const R *)M.rho;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const int nl = M.nl;
  for (; i < M.ncell; i += stride) {
    double x[3];
    if (i < M.ncube) {
      int cc[3] = {(int)(i % M.nx), (int)((i / M.nx) % M.ny), (int)(i / ((uint64_t)M.nx * M.ny))};
      for (int k = 0; k < 3; ++k) x[k] = M.origin[k] + ((double)cc[k] + 0.5) * M.dcell;
    } else {
      // centre of a sub-cube
      int cc[3], ff[3], r;
      leaf_loc(M, i, cc, ff, &r);
      const double h = M.dcell / (double)r;
      for (int k = 0; k < 3; ++k) x[k] = face_pos(M, k, cc[k], r, ff[k]) + 0.5 * h;
    }
    double r2[MAX_SRC];
    for (int s = 0; s < M.nsrc; ++s) {
      const double *ps = M.tab + o.srcpos + 3 * s;
      double dx = x[0] - ps[0], dy = x[1] - ps[1], dz = x[2] - ps[2];
      r2[s] = dx * dx + dy * dy + dz * dz;
    }
    for (int s = 0; s < M.ns; ++s) {
      double t = 0.0;
      if (s != M.pah && (double)rho[i] > 0.0) {
        double rhs = 0.0;
        for (int j = nl - 1; j >= 0; --j) {
          double J = 0.0;
          for (int q = 0; q < M.nsrc; ++q)
            J += M.tab[o.lnu + q * nl + j] / (16.0 * PI_D * PI_D * r2[q]);
          rhs += M.tab[o.wk + s * nl + j] * J;
        }
        bool cl = false;
        t = invert_T(M.tab, o, nl, s, rhs, &cl);
      }
      T[(uint64_t)s * M.ncell + i] = t;
    }
  }
}

hipError_t launch_epoch_snapshot(const ModelDev *d, hipStream_t st) {
  hipLaunchKernelGGL(k_epoch_snapshot, dim3(2048), dim3(256), 0, st, d);
  return hipGetLastError();
}
hipError_t launch_finalize_T(const ModelDev *d, bool fp64, double *T, double *E, hipStream_t st) {
  if (fp64) hipLaunchKernelGGL(k_finalize_T<double>, dim3(4096), dim3(256), 0, st, d, T, E);
  else hipLaunchKernelGGL(k_finalize_T<float>, dim3(4096), dim3(256), 0, st, d, T, E);
  return hipGetLastError();
}
hipError_t launch_init_T(const ModelDev *d, bool fp64, double *T, hipStream_t st) {
  if (fp64) hipLaunchKernelGGL(k_init_T<double>, dim3(4096), dim3(256), 0, st, d, T);
  else hipLaunchKernelGGL(k_init_T<float>, dim3(4096), dim3(256), 0, st, d, T);
  return hipGetLastError();
}

}  // namespace mcrt
