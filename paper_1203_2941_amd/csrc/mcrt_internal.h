// mcrt_internal.h - device data layout and helpers of the HIP library.
//
// Everything here is internal to libmcrt (include/mcrt.h is the public ABI).
// Units are cgs; both precisions walk the grid in centimetres with the
// integer cell index authoritative, so the FP64 path follows the same
// rounding sequence as a plain sequential evaluation of the method.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcrt {

constexpr int MAX_NL = 256;
// Queued packets keep their cell (CJ_BITS per axis, x lowest) and wavelength
// index (the top 64 - 3 CJ_BITS bits) in one 64-bit word: grids hold at most
// MAX_AXIS cells per axis.
constexpr int CJ_BITS = 18;
constexpr int MAX_AXIS = (1 << CJ_BITS) - 1;
static_assert(MAX_NL <= (1 << (64 - 3 * CJ_BITS)), "wavelength index fits the packed word");
// The word of an entry the walk frees (an escape): all ones, which names no
// cell (an axis index is at most MAX_AXIS - 1).
constexpr uint64_t CJ_FREE = ~0ull;
constexpr int MAX_NS = 4;
constexpr int MAX_SRC = 8;
constexpr int MAX_VIEW = 16;
constexpr int MAX_IMG = 16;
constexpr int NT_TAB = 256;          // points of the ln(Phi) vs ln(T) table per species
constexpr int NH_TAB = 2048;         // nodes of the Hermite table ln T(ln Phi) per species
constexpr double T_HERM_MIN = 3.0;   // K, lower end of the Hermite table
constexpr double T_TAB_MIN = 1.0;    // K
constexpr int NK_REJ = 512;          // T bins of the FP32 re-emission proposal tables
constexpr double T_MAX = 1.0e5;      // K, upper end of the Eq. 4 search
constexpr double T_FLOOR = 10.0;     // K, emission temperature of a cell with T = 0
constexpr double H_PL = 6.62607015e-27;
constexpr double C_LI = 2.99792458e10;
constexpr double K_BO = 1.380649e-16;
constexpr double PI_D = 3.14159265358979323846;

enum { ST_ALIVE = 0, ST_ESCAPED = 1, ST_KILLED = 2, ST_PAH_STOP = 3 };
enum { M_FROZEN = 0, M_BW_EPOCH = 1, M_BW_TICKET = 2 };
enum { NSTAT = 10 };  // packets escaped killed pah crossings scatters absorptions mrw lucy clampedT

// Offsets (in elements) of the packed per-model tables. The double table
// serves FP64 arithmetic of both precisions (temperatures, diffusion solve,
// source spectra); the R table holds what the packet walk reads per event
// in the walk's precision.
struct TabOff {
  int w, hnu, a, kext, wk, wfk, kabs, frac, srccum, lnu, lum, pahcum, pahe, logphi, krmax, srcpos, dtotal;
  int r_kext, r_kabsm, r_alb, r_fsca, r_fabs, r_g, r_lucy, r_hnu, r_a, r_wk, r_total;
};

__host__ __device__ inline TabOff tab_offsets(int nl, int ns, int nsrc, int nrows) {
  TabOff o;
  int p = 0;
  o.w = p; p += nl;
  o.hnu = p; p += nl;
  o.a = p; p += nl;
  o.kext = p; p += nl;
  o.wk = p; p += ns * nl;
  o.wfk = p; p += ns * nl;
  o.kabs = p; p += ns * nl;
  o.frac = p; p += MAX_NS;
  o.srccum = p; p += nsrc * nl;
  o.lnu = p; p += nsrc * nl;
  o.lum = p; p += MAX_SRC;
  o.pahcum = p; p += (nrows > 0 ? nrows : 1) * nl;
  o.pahe = p; p += (nrows > 0 ? nrows : 1);
  o.logphi = p; p += ns * NT_TAB;
  o.krmax = p; p += NT_TAB;
  o.srcpos = p; p += 3 * MAX_SRC;
  o.dtotal = p;
  int q = 0;
  o.r_kext = q; q += nl;
  o.r_kabsm = q; q += nl;
  o.r_alb = q; q += nl;
  o.r_fsca = q; q += ns * nl;
  o.r_fabs = q; q += ns * nl;
  o.r_g = q; q += ns * nl;
  o.r_lucy = q; q += ns * nl;
  o.r_hnu = q; q += nl;
  o.r_a = q; q += nl;
  o.r_wk = q; q += ns * nl;
  o.r_total = q;
  return o;
}

// One model as the kernels see it (a device array of these drives a launch).
// Packet queues of the wavefront transport. A round runs three kernels on
// flight-ready queue f: emission appends new packets to it; the voxel walk
// takes each packet to its next interaction and writes it back to its own
// entry (an escape frees the entry); the interactions read the entries in
// place and append the survivors, with the optical depth of their next
// flight, to queue 1 - f. Queues hold packets as structures of arrays; the
// R arrays are in the walk precision.
struct QBuf {
  void *px, *py, *pz, *dx, *dy, *dz, *rho, *tau;
  uint64_t *cj;  // cell and wavelength in one word (pack_cj)
  uint64_t *pid;
  uint32_t *rngd, *nint;
  uint32_t *ncross, *nscat, *nabs, *nmrw, *nlucy;  // kept for packet records
  double *mm;                                      // kept for packet records
  uint32_t *fine;  // refined grids: the packet's sub-cube (fine_pack); null otherwise
  uint32_t *slow;  // entries of this queue whose interaction left the fast kernel (see WfCtl)
};

// The walk keeps the occupancy bits of the grid in LDS: one bit per run of
// consecutive bricks (in brick_index order), the shortest power-of-two run
// whose bits fit this many words.
constexpr int OCC_MAX_WORDS = 2048;

// Queue counters. Each queue is split into NSEG segments of equal
// capacity; every counter sits on its own 128-byte line. A wave takes work
// from and appends to its home segment and moves on only when that one is
// exhausted or full: device-scope atomics on one address serialise (about
// 11 ns each on this GPU), on distinct lines they do not.
constexpr int NSEG = 64;
constexpr int CLINE = 32;  // uint32 per counter line
constexpr uint32_t SLOW_FLIGHT = 0x80000000u;  // slow-list flag (queue indices stay below 2^31)

struct WfCtl {
  uint64_t emitted;  // packets of the launch started so far (launch-relative)
  uint64_t first;    // launch-relative index of the first packet emitted this round
  uint32_t take;     // packets emitted this round
  uint32_t busy;     // models with packets left (written by k_wf_busy)
  uint32_t inq;      // upper bound of this round's flight-ready packets (plan)
  uint32_t left;     // packets queued for the next round, all models (k_wf_busy)
  uint32_t nslow;    // entries of the walked queue handed to the slow interaction kernel
                     // this round: index, with SLOW_FLIGHT set when only the next
                     // flight's start (diffusion steps, optical depth) remains
  uint32_t pad[23];
  uint32_t nseg[2][NSEG][CLINE];  // entries appended to segment g of queue f (clamp to capacity)
  uint32_t work[3][NSEG][CLINE];  // next entry of segment g handed out by emit, walk, interact
};

struct ModelDev {
  int32_t nx, ny, nz, nl, ns, nsrc, pah, nrows, nview, nimg, ntheta, model_id;
  int32_t mode, record, pass, iter;
  int32_t tau_mode;           // 0: one optical-depth draw per flight; 1: a new draw per cell
  int32_t rt_lit;             // ray-tracer source terms in the printed form of Eqs. 13-14
  uint64_t src_strata;        // m equal-energy source strata (0 = plain source draw)
  double pah_nc, pah_tcool;   // PAH photodissociation (Eq. 8): carbon atoms, cooling time
  int32_t sh_order;           // transport: scattering moments up to degree sh_order - 1 (0 off)
  int32_t sh_read;            // source functions: scattered light from moments of this order
  void *sh;                   // moments [cell][img][sh_order^2], context precision, units of
                              // ssca_unit
  double origin[3];
  double dcell, V, xi, lucy_tau, mrw_tau, mrw_gamma, kext_max;
  double ssca_unit;           // scattering sums are stored in these units (erg/s/sr)
  double kr_gmax;             // largest Rosseland-mean bound of the table over [T_TAB_MIN, T_MAX]
  double phi_tmin;            // Phi(T_TAB_MIN) of the first thermal species
  double herm_pmin[MAX_NS];   // Phi at the lower end of each species' Hermite table (infinity
                              // when the table is empty): Eq. 4 right-hand sides at or above it
                              // are inverted by the table alone
  uint64_t max_int, first, n, id_base, rec_first, seed, ncell;
  uint64_t ncube;             // cubes of the grid (ncell - ncube sub-cubes follow them)
  const uint8_t *ref;         // [ncube] sub-cubes per edge (0/1 whole), null: no refinement
  const uint64_t *sub_off;    // [ncube] first sub-cube of each divided cube
  const void *rho;            // [cells] context precision
  const void *rho_b;          // the same density in 4x4x4 bricks (brick_index), read by the walk
  int32_t nbx, nby, nbz;      // bricks per axis
  const uint32_t *occ;        // bit per run of 2^(osh - 6) consecutive bricks: 1 if any density != 0
  int32_t osh, ow;            // bricked-cell index >> osh is the run; words of occ
  const double *tab;          // packed double table
  const void *rtab;           // packed R table
  const int32_t *imgmap;      // [nl] -> imaged index or -1
  const double *herm;         // [ns][3 + 2*NH_TAB]: u0, du, n, then (ln T, dlnT/dlnPhi) per node
  const double *mrw_ub;       // [NH_TAB - 1] or null: Rosseland bound per node interval of the
                              // first thermal species' herm table (see build_tables)
  uint32_t *mrw_cand;         // fast interactions with diffusion steps armed: per leaf cell, one
  uint32_t *mrw_bits;         // bit each (words of 32): cells past the temperature-free bounds,
                              // and those of them the tally bound leaves open this round; null
                              // otherwise
  const float *rej_pe;        // FP32 walk: [2 modes][ns][NK_REJ][nl] (alias prob, envelope) pairs
  const uint8_t *rej_al;      // FP32 walk: [2 modes][ns][NK_REJ][nl] alias bins
  int32_t img_j[MAX_IMG];     // wavelength index of each imaged wavelength
  uint64_t *k;                // [ns][cells]
  double *epath;              // [ns][cells]
  double *T;                  // [ns][cells]
  double *esnap;              // [ns][cells]
  double *tt;                 // [ns][cells], < 0 = not yet computed this epoch
  uint8_t *dirty;             // [cells]
  uint32_t *kpah;             // [cells]
  const uint64_t *kpah_prefix;// [cells] exclusive prefix of kpah (PAH pass)
  uint64_t *sed;              // [ntheta][nl]
  void *ssca;                 // [cells][nview][nimg] context precision
  void *rec;                  // records [n]
  uint64_t *counter;          // packet counter of the launch
  unsigned long long *stats;  // [NSTAT]
  double kv[MAX_VIEW][3];     // view directions toward the observer
  QBuf q[2];                  // wavefront queues
  WfCtl *ctl;                 // their counters (counter points at ctl->emitted)
  uint32_t qcap;              // capacity of each queue
  uint32_t qseg;              // capacity of each of its NSEG segments
};

// ------------------------------------------ leaves (one refinement level)
// A divided cube (ref[cube] = r >= 2) holds r^3 sub-cubes of edge dcell / r,
// numbered ncube + sub_off[cube] + (fz r + fy) r + fx among the leaves; a
// whole cube is its own leaf. The sub-cube index f of a packet travels packed
// as fx | fy << 8 | fz << 16.
template <class G>
__host__ __device__ __forceinline__ int cube_r(const G &M, int64_t cc) {
  if (!M.ref) return 1;
  const int r = M.ref[cc];
  return r > 1 ? r : 1;
}

__host__ __device__ __forceinline__ int fine_get(uint32_t fpk, int k) {
  return (int)((fpk >> (8 * k)) & 0xFFu);
}

__host__ __device__ __forceinline__ uint32_t fine_pack(int fx, int fy, int fz) {
  return (uint32_t)fx | ((uint32_t)fy << 8) | ((uint32_t)fz << 16);
}

// leaf of sub-cube fpk of cube (cx, cy, cz), and its edge
template <class G>
__host__ __device__ __forceinline__ int64_t leaf_of(const G &M, int cx, int cy, int cz,
                                                    uint32_t fpk, double *h) {
  const int64_t cc = ((int64_t)cz * M.ny + cy) * M.nx + cx;
  const int r = cube_r(M, cc);
  if (r == 1) {
    if (h) *h = M.dcell;
    return cc;
  }
  if (h) *h = M.dcell / (double)r;
  return (int64_t)M.ncube + (int64_t)M.sub_off[cc] +
         ((int64_t)fine_get(fpk, 2) * r + fine_get(fpk, 1)) * r + fine_get(fpk, 0);
}

// Face e (0..r) of the sub-cubes of cube coordinate ck on axis k; the cube's
// own faces are written as for a whole cube, so a walk leaves a divided cube
// exactly where the grid puts that face.
template <class G>
__host__ __device__ __forceinline__ double face_pos(const G &M, int k, int ck, int r, int e) {
  if (e == 0) return M.origin[k] + (double)ck * M.dcell;
  if (e == r) return M.origin[k] + (double)(ck + 1) * M.dcell;
  return M.origin[k] + (double)ck * M.dcell + (double)e * (M.dcell / (double)r);
}

// sub-cube index on axis k of point x in cube coordinate ck (a point on a
// face belongs to the sub-cube that direction component dk points into)
template <class G>
__host__ __device__ __forceinline__ int sub_index(const G &M, int k, int ck, int r, double x,
                                                  double dk) {
  if (r == 1) return 0;
  const double q = (x - M.origin[k] - (double)ck * M.dcell) / (M.dcell / (double)r);
  const double fl = floor(q);
  int fi = (int)fl;
  if (q == fl && dk < 0.0) fi -= 1;
  return fi < 0 ? 0 : (fi > r - 1 ? r - 1 : fi);
}

// cube c, sub-cube f and sub-cubes per edge r of leaf i; a sub-cube's cube
// is the last one whose first sub-cube is at or before it
template <class G>
__host__ __device__ inline void leaf_loc(const G &M, uint64_t i, int c[3], int f[3], int *r) {
  uint64_t cc = i;
  f[0] = f[1] = f[2] = 0;
  *r = 1;
  if (i >= M.ncube) {
    const uint64_t s = i - M.ncube;
    int64_t lo = 0, hi = (int64_t)M.ncube - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (M.sub_off[mid] <= s) lo = mid; else hi = mid - 1;
    }
    cc = (uint64_t)lo;
    const int rr = cube_r(M, (int64_t)cc);
    const uint64_t loc = s - M.sub_off[cc];
    f[0] = (int)(loc % rr);
    f[1] = (int)((loc / rr) % rr);
    f[2] = (int)(loc / ((uint64_t)rr * rr));
    *r = rr;
  }
  c[0] = (int)(cc % M.nx);
  c[1] = (int)((cc / M.nx) % M.ny);
  c[2] = (int)(cc / ((uint64_t)M.nx * M.ny));
}

// edge and volume of leaf i
__host__ __device__ inline double leaf_edge(const ModelDev &M, uint64_t i) {
  if (i < M.ncube) return M.dcell;
  int c[3], f[3], r;
  leaf_loc(M, i, c, f, &r);
  return M.dcell / (double)r;
}
__host__ __device__ inline double leaf_volume(const ModelDev &M, uint64_t i) {
  if (i < M.ncube) return M.V;
  const double h = leaf_edge(M, i);
  return h * h * h;
}

// ---------------------------------------------------------------- bricks
// The voxel walk reads the density from a copy stored in 4x4x4 bricks of 64
// cells (256 B in FP32), x fastest inside a brick and bricks x-fastest. A
// step to a neighbouring cell stays in its brick three times in four, so
// the gathers of one packet share cache lines far more often than in the
// x-fastest layout, where every y or z step lands on a new line.
__host__ __device__ __forceinline__ int64_t brick_index(int cx, int cy, int cz, int nbx, int nby) {
  return ((((int64_t)(cz >> 2) * nby + (cy >> 2)) * nbx + (cx >> 2)) << 6) +
         (((cz & 3) << 4) | ((cy & 3) << 2) | (cx & 3));
}
// The same in 32-bit arithmetic, for bricked grids of fewer than 2^32 cells
// (cells in range, so every coordinate is >= 0).
// 32-bit form with 24-bit multiplies (full rate; the 32-bit multiply is a
// quarter-rate instruction): valid while the bricked grid has fewer than
// 2^32 cells and nby * nbz < 2^24 (see idx32_ok).
__device__ __forceinline__ uint32_t brick_index32(int cx, int cy, int cz, int nbx, int nby) {
  const uint32_t b = __umul24(__umul24((uint32_t)(cz >> 2), (uint32_t)nby) + (uint32_t)(cy >> 2),
                              (uint32_t)nbx) +
                     (uint32_t)(cx >> 2);
  return (b << 6) | (uint32_t)(((cz & 3) << 4) | ((cy & 3) << 2) | (cx & 3));
}

// Cell of bricked index i (the inverse of brick_index / brick_index32).
template <typename Idx>
__host__ __device__ __forceinline__ void unbrick(Idx i, int nbx, int nby, int &cx, int &cy,
                                                 int &cz) {
  const uint32_t w = (uint32_t)i & 63u;
  if constexpr (sizeof(Idx) == 4) {
    const uint32_t b = (uint32_t)i >> 6;
    const uint32_t r = b / (uint32_t)nbx, bx = b - r * (uint32_t)nbx;
    const uint32_t bz = r / (uint32_t)nby, by = r - bz * (uint32_t)nby;
    cx = (int)(bx * 4u + (w & 3u));
    cy = (int)(by * 4u + ((w >> 2) & 3u));
    cz = (int)(bz * 4u + (w >> 4));
  } else {
    const uint64_t b = (uint64_t)i >> 6;
    const uint64_t r = b / (uint64_t)nbx, bx = b - r * (uint64_t)nbx;
    const uint64_t bz = r / (uint64_t)nby, by = r - bz * (uint64_t)nby;
    cx = (int)(bx * 4u + (w & 3u));
    cy = (int)(by * 4u + ((w >> 2) & 3u));
    cz = (int)(bz * 4u + (w >> 4));
  }
}

// ---------------------------------------------------------------- RNG
// Philox4x32-10 (Salmon et al. 2011); key = seed, counter = (draw block,
// packet id low word, packet id bits 32-47 | iteration << 16,
// model << 8 | stream tag). Draw d uses block d >> 2, word d & 3.
__device__ __forceinline__ void philox10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

struct Rng {
  uint32_t k0, k1, c1, c2, c3, d, blk;
  uint32_t b0, b1, b2, b3;
};

__device__ __forceinline__ void rng_init(Rng &r, uint64_t seed, uint64_t pid, uint32_t iter,
                                         uint32_t model, uint32_t tag) {
  r.k0 = (uint32_t)seed;
  r.k1 = (uint32_t)(seed >> 32);
  r.c1 = (uint32_t)pid;
  r.c2 = ((uint32_t)(pid >> 32) & 0xFFFFu) | (iter << 16);
  r.c3 = (model << 8) | (tag & 0xFFu);
  r.d = 0;
  r.blk = 0xFFFFFFFFu;
}

__device__ __forceinline__ uint32_t rng_u32(Rng &r) {
  uint32_t b = r.d >> 2;
  if (b != r.blk) {
    uint32_t c0 = b, c1 = r.c1, c2 = r.c2, c3 = r.c3;
    philox10(c0, c1, c2, c3, r.k0, r.k1);
    r.b0 = c0; r.b1 = c1; r.b2 = c2; r.b3 = c3;
    r.blk = b;
  }
  // word d & 3 of the block, chosen with masks: a select chain between the
  // members would be turned into an indexed load and move r to scratch
  const uint32_t w = r.d & 3u;
  const uint32_t x = (r.b0 & (0u - (uint32_t)(w == 0u))) | (r.b1 & (0u - (uint32_t)(w == 1u))) |
                     (r.b2 & (0u - (uint32_t)(w == 2u))) | (r.b3 & (0u - (uint32_t)(w == 3u)));
  r.d++;
  return x;
}

// ((x >> 8) + 1/2) 2^-24, strictly inside (0, 1). It has 25 significant bits:
// exact in FP64; rounded to nearest in FP32 (draws that set directions or
// pick source wavelengths are taken in FP64 in both precisions).
template <typename R> __device__ __forceinline__ R rng_u(Rng &r) {
  return ((R)(rng_u32(r) >> 8) + (R)0.5) * (R)(1.0 / 16777216.0);
}

// ------------------------------------------------ global-memory access
// Device buffers reached through ModelDev are generic pointers to the
// compiler, which would emit flat_* instructions; flat loads also count
// against LDS waits. These helpers access them as global memory.
#define MCRT_AS_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ T gld(const T *p) {
  return *(const MCRT_AS_GLOBAL T *)p;
}
// Racy read of a value other lanes update with atomics (queue counters, the
// B&W tallies): device scope, relaxed, so it neither tears nor is kept in a
// register across reads, and it may be served by the L2.
template <typename T> __device__ __forceinline__ T gload_relaxed(const T *p) {
  return __hip_atomic_load((const MCRT_AS_GLOBAL T *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ T gatomic_add(T *p, T v) {
  return __hip_atomic_fetch_add((MCRT_AS_GLOBAL T *)p, v, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- math
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float m_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_cos(double x) { return cos(x); }
__device__ __forceinline__ float m_cos(float x) { return cosf(x); }
__device__ __forceinline__ double m_sin(double x) { return sin(x); }
__device__ __forceinline__ float m_sin(float x) { return sinf(x); }
__device__ __forceinline__ double m_floor(double x) { return floor(x); }
__device__ __forceinline__ float m_floor(float x) { return floorf(x); }
__device__ __forceinline__ double m_fabs(double x) { return fabs(x); }
__device__ __forceinline__ float m_fabs(float x) { return fabsf(x); }
template <typename R> __device__ __forceinline__ R m_inf() { return (R)__builtin_huge_val(); }
// largest x of the Planck factor 1/(e^x - 1) kept in each precision
template <typename R> __device__ __forceinline__ R x_cut();
template <> __device__ __forceinline__ double x_cut<double>() { return 700.0; }
template <> __device__ __forceinline__ float x_cut<float>() { return 80.0f; }

__device__ __forceinline__ void upd_margin(double &mm, double v) {
  if (v < mm) mm = v;
}

// Planck pieces (double): B = a/(e^x - 1), dB/dT = B (x/T)(1 + 1/(e^x - 1)),
// x = h nu / kT; zero for x > 700 or T <= 0.
__device__ __forceinline__ double planck_d(double hnu, double a, double T) {
  if (!(T > 0.0)) return 0.0;
  double x = hnu / (K_BO * T);
  if (x > 700.0) return 0.0;
  return a / expm1(x);
}
__device__ __forceinline__ double dplanck_d(double hnu, double a, double T) {
  if (!(T > 0.0)) return 0.0;
  double x = hnu / (K_BO * T);
  if (x > 700.0) return 0.0;
  double em = expm1(x);
  double B = a / em;
  return B * (x / T) * (1.0 + 1.0 / em);
}

// Phi_s(T) = sum_j w_j kabs_s,j B_j(T) (ascending frequency) and dPhi/dT.
__device__ inline double phi_dphi(const double *wk, const double *hnu, const double *a, int nl,
                                  double T, double *dphi) {
  double s = 0.0, ds = 0.0;
  double kT = K_BO * T;
  for (int j = nl - 1; j >= 0; --j) {
    double x = hnu[j] / kT;
    if (x > 700.0) continue;
    double em = expm1(x);
    double B = a[j] / em;
    s += wk[j] * B;
    ds += wk[j] * (B * (x / T) * (1.0 + 1.0 / em));
  }
  *dphi = ds;
  return s;
}

// Eq. 4 inverted in FP64: table bracket in (ln T, ln Phi), then safeguarded
// Newton on ln Phi(ln T) until |d ln T| < 1e-14. rhs <= 0 -> 0; rhs at or
// above Phi(T_MAX) -> T_MAX, flagged as clamped. Kept out of line: its
// FP64 loops would otherwise add their registers to every caller.
struct TInv {
  double T;
  int clamped;
};

static __device__ __noinline__ TInv invert_T_core(const double *lp, const double *wk,
                                                  const double *hnu, const double *a, int nl,
                                                  double rhs, double u_start, int have_start) {
  TInv r{0.0, 0};
  if (!(rhs > 0.0)) return r;
  const double lt0 = log(T_TAB_MIN), dlt = (log(T_MAX) - lt0) / (NT_TAB - 1);
  double lr = log(rhs);
  double dphi;
  if (!(lr < lp[NT_TAB - 1])) {
    double ph = phi_dphi(wk, hnu, a, nl, T_MAX, &dphi);
    if (ph <= rhs) {
      r.T = T_MAX;
      r.clamped = 1;
      return r;
    }
  }
  double ulo, uhi, u;
  if (lr < lp[0]) {
    ulo = -60.0;  // ~1e-26 K: Phi there underflows to 0 on any grid
    uhi = lt0;
    u = lt0 - 1.0;
  } else {
    int lo = 0, hi = NT_TAB - 1;
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (lp[mid] <= lr) lo = mid; else hi = mid;
    }
    ulo = lt0 + lo * dlt;
    uhi = lt0 + hi * dlt;
    double den = lp[hi] - lp[lo];
    u = (den > 0.0 && lp[lo] > -1e300) ? ulo + (lr - lp[lo]) / den * dlt : 0.5 * (ulo + uhi);
    if (have_start && u_start > ulo && u_start < uhi) u = u_start;
  }
  for (int it = 0; it < 100; ++it) {
    double T = exp(u);
    double ph = phi_dphi(wk, hnu, a, nl, T, &dphi);
    double un;
    if (!(ph > 0.0)) {
      ulo = u;
      un = 0.5 * (ulo + uhi);
    } else {
      double g = log(ph) - lr;
      if (g > 0.0) uhi = u; else ulo = u;
      double slope = T * dphi / ph;
      un = (slope > 0.0) ? u - g / slope : 0.5 * (ulo + uhi);
      if (!(un > ulo && un < uhi)) un = 0.5 * (ulo + uhi);
    }
    double du = un - u;
    u = un;
    if (fabs(du) < 1e-14) break;
  }
  r.T = exp(u);
  return r;
}

__device__ inline double invert_T(const double *tab, const TabOff &o, int nl, int s, double rhs,
                                  bool *clamped, double u_start = 0.0, bool have_start = false) {
  if (!(rhs > 0.0)) return 0.0;
  TInv r = invert_T_core(tab + o.logphi + s * NT_TAB, tab + o.wk + s * nl, tab + o.hnu,
                         tab + o.a, nl, rhs, u_start, have_start ? 1 : 0);
  if (r.clamped) *clamped = true;
  return r.T;
}

// Eq. 4 by table: ln T as a cubic Hermite function of ln Phi on a uniform
// ln Phi grid whose node values and slopes are exact (host FP64). Interval
// error ~ du^4/384 |y''''| (about 1e-10 relative in T for 2048 nodes); falls
// back to the Newton solve outside the table.
__device__ inline bool herm_lnT(const double *herm, int s, double rhs, double *lnT) {
  const double *h = herm + (size_t)s * (3 + 2 * NH_TAB);
  double x = (log(rhs) - h[0]) / h[1];
  int n = (int)h[2];
  if (!(x >= 0.0) || !(x < (double)(n - 1))) return false;
  int k = (int)x;
  double t = x - (double)k, t2 = t * t, t3 = t2 * t;
  const double *p = h + 3 + 2 * k;
  *lnT = (2.0 * t3 - 3.0 * t2 + 1.0) * p[0] + (t3 - 2.0 * t2 + t) * h[1] * p[1] +
         (-2.0 * t3 + 3.0 * t2) * p[2] + (t3 - t2) * h[1] * p[3];
  return true;
}

// Eq. 4 in FP64 to 1e-14, Newton started from the Hermite estimate.
__device__ inline double invert_T_exact(const double *herm, const double *tab, const TabOff &o,
                                        int nl, int s, double rhs, bool *clamped) {
  if (!(rhs > 0.0)) return 0.0;
  double u0;
  bool ok = herm && herm_lnT(herm, s, rhs, &u0);
  return invert_T(tab, o, nl, s, rhs, clamped, u0, ok);
}

__device__ inline double invert_T_fast(const double *herm, const double *tab, const TabOff &o,
                                       int nl, int s, double rhs, bool *clamped) {
  if (!(rhs > 0.0)) return 0.0;
  const double *h = herm + (size_t)s * (3 + 2 * NH_TAB);
  double x = (log(rhs) - h[0]) / h[1];
  int n = (int)h[2];
  if (!(x >= 0.0) || !(x < (double)(n - 1))) return invert_T(tab, o, nl, s, rhs, clamped);
  int k = (int)x;
  double t = x - (double)k, t2 = t * t, t3 = t2 * t;
  const double *p = h + 3 + 2 * k;
  double y = (2.0 * t3 - 3.0 * t2 + 1.0) * p[0] + (t3 - 2.0 * t2 + t) * h[1] * p[1] +
             (-2.0 * t3 + 3.0 * t2) * p[2] + (t3 - t2) * h[1] * p[3];
  return exp(y);
}

// Survival in a sphere for diffusion from its centre, S = 2 sum (-1)^{n+1} y^{n^2}.
__device__ inline double mrw_surv(double y) {
  if (!(y > 0.0)) return 0.0;
  if (y >= 1.0) return 1.0;
  double ly = log(y), sum = 0.0;
  for (int n = 1; n <= 10000; ++n) {
    double term = exp((double)n * (double)n * ly);
    sum += (n & 1) ? term : -term;
    if (term < 1e-17 * fabs(sum)) break;
  }
  return 2.0 * sum;
}

__device__ inline double mrw_dsurv(double y) {
  double ly = log(y), sum = 0.0;
  for (int n = 1; n <= 10000; ++n) {
    double nn = (double)n * (double)n;
    double term = nn * exp((nn - 1.0) * ly);
    sum += (n & 1) ? term : -term;
    if (term < 1e-17 * fabs(sum)) break;
  }
  return 2.0 * sum;
}

// y in (0,1) with S(y) = u (FP64): Newton within a shrinking bracket.
static __device__ __noinline__ double mrw_solve(double u) {
  double lo = 0.0, hi = 1.0, y = 0.5 * u;
  if (!(y > 0.0)) y = 1e-300;
  for (int it = 0; it < 200; ++it) {
    double f = mrw_surv(y) - u;
    if (f > 0.0) hi = y; else lo = y;
    double df = mrw_dsurv(y);
    double yn = (df > 0.0) ? y - f / df : 0.5 * (lo + hi);
    if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);
    if (fabs(yn - y) <= 1e-15 * y) {
      y = yn;
      break;
    }
    y = yn;
  }
  return y;
}

// Real orthonormal spherical harmonics Y_lm(d), l < order, handed to
// f(index, value) with index l^2 + l + m: associated Legendre terms in
// x = d_z without their sin^m factor,
//   Q_m^m = (2m-1)!!, Q_{m+1}^m = (2m+1) x Q_m^m,
//   (l-m) Q_l^m = (2l-1) x Q_{l-1}^m - (l+m-1) Q_{l-2}^m,
// and (d_x + i d_y)^m = sin^m e^{i m phi}: Y_l0 = N Q, Y_l,+-m = sqrt(2) N Q
// (Re, Im)(d_x + i d_y)^m with N^2 = (2l+1)/(4 pi) (l-m)!/(l+m)!.
constexpr int MAX_SH_ORDER = 9;
constexpr int MAX_REF = 16;  // sub-cubes per edge of a divided cube
template <typename F>
__host__ __device__ inline void ylm_each(int order, double dx, double dy, double dz, F f) {
  double cr = 1.0, ci = 0.0, qmm = 1.0;
  for (int m = 0; m < order; ++m) {
    if (m > 0) {
      const double nr = cr * dx - ci * dy, ni = cr * dy + ci * dx;
      cr = nr;
      ci = ni;
      qmm *= (double)(2 * m - 1);
    }
    double q2 = 0.0, q1 = qmm;
    for (int l = m; l < order; ++l) {
      double q;
      if (l == m) q = qmm;
      else if (l == m + 1) q = (double)(2 * m + 1) * dz * qmm;
      else q = ((double)(2 * l - 1) * dz * q1 - (double)(l + m - 1) * q2) / (double)(l - m);
      if (l > m) {
        q2 = q1;
        q1 = q;
      }
      double ratio = 1.0;
      for (int k = l - m + 1; k <= l + m; ++k) ratio /= (double)k;
      const double n = sqrt((2.0 * l + 1.0) / (4.0 * PI_D) * ratio);
      if (m == 0) {
        f(l * l + l, l, n * q);
      } else {
        f(l * l + l + m, l, sqrt(2.0) * n * q * cr);
        f(l * l + l - m, l, sqrt(2.0) * n * q * ci);
      }
    }
  }
}

// Device fill (kept as a kernel so that graph captures record no memsets).
template <typename T> __global__ void k_fill(T *p, T v, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

}  // namespace mcrt
