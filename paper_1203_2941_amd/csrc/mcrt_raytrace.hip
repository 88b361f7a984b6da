// mcrt_raytrace.hip - ray-tracer of sect. 4 (Eqs. 11-17) and its adjoint.
//
// One lane per pixel ray. Rays are parallel to -k (k toward the observer)
// through a square field of side sqrt(3) x box edge and march front to back
// with the same voxel walk as the transport. Every imaged wavelength of a
// ray is carried in registers, so a cell crossing reads the density once
// and one contiguous vector of source functions S[view][cell][0..n_img)
// that is built per view before the march (emission plus scattered light,
// both per unit extinction; constant in the traced density).
// Intensities accumulate in FP64 in both precisions; transmittances and
// adjoint weights are in the context precision.
#include "mcrt_rtargs.h"

namespace mcrt {

template <typename R>
__device__ __forceinline__ double plane_d(const RtArgs &A, double p0, double d, int c, int k) {
  if (d > 0.0) return (A.origin[k] + (double)(c + 1) * A.dcell - p0) / d;
  if (d < 0.0) return (A.origin[k] + (double)c * A.dcell - p0) / d;
  return __builtin_huge_val();
}

// Entry of pixel ray (ix, iy) of view v into the box; false when it misses.
__device__ inline bool ray_entry(const RtArgs &A, const RtView &V, int ix, int iy, double pe[3],
                                 double dir[3], int c[3]) {
  double xp = ((double)ix + 0.5) * V.dpx - 0.5 * V.fov;
  double yp = ((double)iy + 0.5) * V.dpy - 0.5 * V.fov;
  double r0[3];
  int n[3] = {A.nx, A.ny, A.nz};
  double tmin = -__builtin_huge_val(), tmax = __builtin_huge_val();
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r0[k] = V.ctr[k] + xp * V.ex[k] + yp * V.ey[k] + V.fov * V.k[k];
    dir[k] = -V.k[k];
    double lo = A.origin[k], hi = A.origin[k] + (double)n[k] * A.dcell;
    if (dir[k] != 0.0) {
      double t1 = (lo - r0[k]) / dir[k], t2 = (hi - r0[k]) / dir[k];
      double a = t1 < t2 ? t1 : t2, b = t1 < t2 ? t2 : t1;
      if (a > tmin) tmin = a;
      if (b < tmax) tmax = b;
    } else if (r0[k] < lo || r0[k] > hi) {
      return false;
    }
  }
  if (!(tmin < tmax)) return false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pe[k] = r0[k] + tmin * dir[k];
    double q = (pe[k] - A.origin[k]) / A.dcell;
    double f = floor(q);
    int ci = (int)f;
    if (q == f && dir[k] < 0.0) ci -= 1;
    if (ci < 0) ci = 0;
    if (ci >= n[k]) ci = n[k] - 1;
    c[k] = ci;
  }
  return true;
}

// Voxel walk calling seg(cell, length) for every segment (FP64 geometry).
template <typename F>
__device__ __forceinline__ void walk(const RtArgs &A, const double p0[3], const double d[3],
                                     int c0[3], F seg) {
  int cx = c0[0], cy = c0[1], cz = c0[2];
  if (cx < 0 || cx >= A.nx || cy < 0 || cy >= A.ny || cz < 0 || cz >= A.nz) return;
  double tx = plane_d<double>(A, p0[0], d[0], cx, 0);
  double ty = plane_d<double>(A, p0[1], d[1], cy, 1);
  double tz = plane_d<double>(A, p0[2], d[2], cz, 2);
  const int sx = d[0] > 0.0 ? 1 : -1, sy = d[1] > 0.0 ? 1 : -1, sz = d[2] > 0.0 ? 1 : -1;
  double t = 0.0;
  int64_t c = ((int64_t)cz * A.ny + cy) * A.nx + cx;
  for (;;) {
    int a = 0;
    double tn = tx;
    if (ty < tn) { a = 1; tn = ty; }
    if (tz < tn) { a = 2; tn = tz; }
    double ell = tn - t;
    if (ell < 0.0) ell = 0.0;
    seg(c, ell);
    if (tn > t) t = tn;
    if (a == 0) {
      cx += sx;
      if (cx < 0 || cx >= A.nx) return;
      c += sx;
      tx = plane_d<double>(A, p0[0], d[0], cx, 0);
    } else if (a == 1) {
      cy += sy;
      if (cy < 0 || cy >= A.ny) return;
      c += (int64_t)sy * A.nx;
      ty = plane_d<double>(A, p0[1], d[1], cy, 1);
    } else {
      cz += sz;
      if (cz < 0 || cz >= A.nz) return;
      c += (int64_t)sz * A.nx * A.ny;
      tz = plane_d<double>(A, p0[2], d[2], cz, 2);
    }
  }
}

// The same walk through the leaves of a refined grid: each cube's own
// lattice (a whole cube is one leaf), leaving a divided cube on the cube's
// own face; the sub-cube of the start from the position.
template <typename F>
__device__ __forceinline__ void walk_leaves(const RtArgs &A, const double p0[3], const double d[3],
                                            int c0[3], F seg) {
  int c[3] = {c0[0], c0[1], c0[2]};
  if (c[0] < 0 || c[0] >= A.nx || c[1] < 0 || c[1] >= A.ny || c[2] < 0 || c[2] >= A.nz) return;
  int f[3];
  int r = cube_r(A, ((int64_t)c[2] * A.ny + c[1]) * A.nx + c[0]);
  double tm[3];
  auto faces = [&]() {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (d[k] > 0.0) tm[k] = (face_pos(A, k, c[k], r, f[k] + 1) - p0[k]) / d[k];
      else if (d[k] < 0.0) tm[k] = (face_pos(A, k, c[k], r, f[k]) - p0[k]) / d[k];
      else tm[k] = __builtin_huge_val();
    }
  };
#pragma unroll
  for (int k = 0; k < 3; ++k) f[k] = sub_index(A, k, c[k], r, p0[k], d[k]);
  faces();
  double t = 0.0;
  const int n[3] = {A.nx, A.ny, A.nz};
  for (;;) {
    int a = 0;
    if (tm[1] < tm[a]) a = 1;
    if (tm[2] < tm[a]) a = 2;
    double ell = tm[a] - t;
    if (ell < 0.0) ell = 0.0;
    seg(leaf_of(A, c[0], c[1], c[2], fine_pack(f[0], f[1], f[2]), nullptr), ell);
    if (tm[a] > t) t = tm[a];
    const int sa = d[a] > 0.0 ? 1 : -1;
    f[a] += sa;
    if (f[a] >= 0 && f[a] < r) {
      tm[a] = (face_pos(A, a, c[a], r, d[a] > 0.0 ? f[a] + 1 : f[a]) - p0[a]) / d[a];
      continue;
    }
    c[a] += sa;
    if (c[a] < 0 || c[a] >= n[a]) return;
    r = cube_r(A, ((int64_t)c[2] * A.ny + c[1]) * A.nx + c[0]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k == a) f[k] = d[k] > 0.0 ? 0 : r - 1;
      else f[k] = sub_index(A, k, c[k], r, p0[k] + t * d[k], d[k]);
    }
    faces();
  }
}

// 1 - e^-x and e^-x of one segment in the walk precision.
__device__ __forceinline__ void absorb_pair(double x, double &om, double &e) {
  om = -expm1(-x);
  e = exp(-x);
}
__device__ __forceinline__ void absorb_pair(float x, float &om, float &e) {
  om = -expm1f(-x);
  e = expf(-x);
}
// The same pair from one exponential (the adjoint's two sweeps): 1 - e^-x by
// its Taylor series below 1/2 (8 terms: truncation under 2e-8 relative) and
// as the difference above (e <= 0.61 there): within 1e-7 relative of the
// exact value, against 6e-8 for a correctly rounded expm1f. FP64 keeps the
// library pair.
__device__ __forceinline__ void absorb_pair1(double x, double &om, double &e) {
  absorb_pair(x, om, e);
}
__device__ __forceinline__ void absorb_pair1(float x, float &om, float &e) {
  e = expf(-x);
  float p = 1.0f / 40320.0f;
  p = fmaf(-x, p, 1.0f / 5040.0f);
  p = fmaf(-x, p, 1.0f / 720.0f);
  p = fmaf(-x, p, 1.0f / 120.0f);
  p = fmaf(-x, p, 1.0f / 24.0f);
  p = fmaf(-x, p, 1.0f / 6.0f);
  p = fmaf(-x, p, 0.5f);
  p = fmaf(-x, p, 1.0f);
  om = x < 0.5f ? x * p : 1.0f - e;
}

// S[v][c][q] = sum_s f_s kabs_s B(T_s)/kext + Ssca/(V w rho kext): one lane
// per cell evaluates the view-independent emission once and writes the
// 16-wide source vector of every view.
// One cell's S row (nq values, contiguous): four 16-byte loads for 16 FP32
// values, else one load per value.
template <typename R>
__device__ __forceinline__ void load_row(const R *sc, int nq, R out[MAX_IMG]) {
  if constexpr (sizeof(R) == 4 && MAX_IMG == 16) {
    if (nq == 16) {
      const float4 *s4 = reinterpret_cast<const float4 *>(sc);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 w = s4[k];
        out[4 * k] = w.x; out[4 * k + 1] = w.y; out[4 * k + 2] = w.z; out[4 * k + 3] = w.w;
      }
      return;
    }
  }
#pragma unroll
  for (int q = 0; q < MAX_IMG; ++q) out[q] = q < nq ? sc[q] : (R)0;
}

// LIT: the printed form of Eqs. 13-14; SH: scattered light formed from the
// moments of the scattering events (else the per-view sums). Separate
// instances keep the moment loop's registers out of the common case.
// B_nu(T) for the source functions in the precision they are stored in:
// FP32 for an FP32 context (expm1f; beyond x = 80 the value is below what an
// FP32 source function resolves, so it is 0), FP64 otherwise.
template <typename R>
__device__ __forceinline__ double planck_r(double hnu, double a, double T) {
  if constexpr (sizeof(R) == 8) {
    return planck_d(hnu, a, T);
  } else {
    if (!(T > 0.0)) return 0.0;
    const float x = (float)hnu / ((float)K_BO * (float)T);
    if (!(x <= 80.0f)) return 0.0;
    return (double)((float)a / expm1f(x));
  }
}

template <typename R, bool LIT, bool SH>
__global__ void k_build_S(const ModelDev *__restrict__ md, R *S) {
  const ModelDev &M = *md;
  TabOff o = tab_offsets(M.nl, M.ns, M.nsrc, M.nrows);
  const R *rho = (const R *)M.rho;
  const R *ss = (const R *)M.ssca;
  const int nq = M.nimg;
  uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; c < M.ncell; c += stride) {
    double T[MAX_NS];
    bool hot = false;
    for (int s = 0; s < M.ns; ++s) {
      T[s] = (s == M.pah) ? 0.0 : M.T[(uint64_t)s * M.ncell + c];
      hot |= T[s] > 0.0;
    }
    double r = (double)rho[c];
    double em[MAX_IMG];
#pragma unroll
    for (int q = 0; q < MAX_IMG; ++q) {
      em[q] = 0.0;
      if (q < nq && hot) {
        int j = M.img_j[q];
        double e = 0.0;
        for (int s = 0; s < M.ns; ++s) {
          if (s == M.pah) continue;
          e += M.tab[o.frac + s] * M.tab[o.kabs + s * M.nl + j] *
               planck_r<R>(M.tab[o.hnu + j], M.tab[o.a + j], T[s]);
        }
        if constexpr (LIT) {
          // printed form: the cell's emergent emission (1 - e^-tau_cell) e/K
          // with K the whole mixture's absorption and tau_cell face to face
          double K = 0.0;
          for (int s = 0; s < M.ns; ++s) K += M.tab[o.frac + s] * M.tab[o.kabs + s * M.nl + j];
          em[q] = (r > 0.0 && K > 0.0) ? -expm1(-(r * K * leaf_edge(M, c))) * (e / K) : 0.0;
        } else {
          em[q] = e / M.tab[o.kext + j];
        }
      }
    }
    // per wavelength, the factor from a scattering sum to its source term
    // (the same for every view)
    double fs[MAX_IMG];
#pragma unroll
    for (int q = 0; q < MAX_IMG; ++q) {
      fs[q] = 0.0;
      if (q < nq && r > 0.0) {
        const int j = M.img_j[q];
        if constexpr (LIT) {  // Eq. 16: scattered intensity over the cell's face
          const double hc = leaf_edge(M, c);
          fs[q] = M.ssca_unit / (M.tab[o.w + j] * hc * hc);
        } else {
          fs[q] = M.ssca_unit / (leaf_volume(M, c) * M.tab[o.w + j] * r * M.tab[o.kext + j]);
        }
      }
    }
    for (int v = 0; v < M.nview; ++v) {
      // S is [view][cell][img]; the scattering sums are [cell][view][img] (a
      // scattering event's view sums share cache lines)
      R *out = S + ((uint64_t)v * M.ncell + c) * nq;
      const R *sc = ss ? ss + ((uint64_t)c * M.nview + v) * nq : nullptr;
      R sv[MAX_IMG];
#pragma unroll
      for (int q = 0; q < MAX_IMG; ++q) sv[q] = (R)0;
      if (SH && r > 0.0) {
        // scattered light toward this view from the moments:
        // sum_lm Y_lm(k_v) M[c][q][lm]
        const int nlm = M.sh_read * M.sh_read;
        const R *mc = (const R *)M.sh + (uint64_t)c * nq * nlm;
        double acc[MAX_IMG];
#pragma unroll
        for (int q = 0; q < MAX_IMG; ++q) acc[q] = 0.0;
        ylm_each(M.sh_read, M.kv[v][0], M.kv[v][1], M.kv[v][2], [&](int i, int, double y) {
#pragma unroll
          for (int q = 0; q < MAX_IMG; ++q)
            if (q < nq) acc[q] += y * (double)mc[q * nlm + i];
        });
#pragma unroll
        for (int q = 0; q < MAX_IMG; ++q) sv[q] = (R)acc[q];
      } else if (sc && r > 0.0) {
        bool vec = false;
        if constexpr (sizeof(R) == 4 && MAX_IMG == 16) {
          if (nq == 16) {
            const float4 *s4 = reinterpret_cast<const float4 *>(sc);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const float4 w = s4[k];
              sv[4 * k] = w.x; sv[4 * k + 1] = w.y; sv[4 * k + 2] = w.z; sv[4 * k + 3] = w.w;
            }
            vec = true;
          }
        }
        if (!vec) {
#pragma unroll
          for (int q = 0; q < MAX_IMG; ++q)
            if (q < nq) sv[q] = sc[q];
        }
      }
      R vals[MAX_IMG];
#pragma unroll
      for (int q = 0; q < MAX_IMG; ++q) {
        double val = em[q];
        if (q < nq && (sc || SH) && r > 0.0) val += (double)sv[q] * fs[q];
        vals[q] = (R)val;
      }
      if constexpr (sizeof(R) == 4 && MAX_IMG == 16) {
        // a cell's 16 values are 64 contiguous bytes (16-byte aligned): four
        // 16-byte stores per lane instead of sixteen 4-byte ones
        if (nq == 16) {
          float4 *o4 = reinterpret_cast<float4 *>(out);
#pragma unroll
          for (int k = 0; k < 4; ++k)
            o4[k] = make_float4(vals[4 * k], vals[4 * k + 1], vals[4 * k + 2], vals[4 * k + 3]);
          continue;
        }
      }
#pragma unroll
      for (int q = 0; q < MAX_IMG; ++q) {
        if (q >= nq) break;
        out[q] = vals[q];
      }
    }
  }
}

// LIT: printed form of Eqs. 13-14: S holds each cell's whole term C, added
// in full (I += T C) whatever the traced density, which only attenuates.
template <typename R, bool LIT, bool REF>
__global__ void __launch_bounds__(256) k_rt_fwd(const RtArgs *__restrict__ Ap, R *img) {
  const RtArgs &A = *Ap;
  const int v = blockIdx.y;
  const int pix = blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= A.npx * A.npy) return;
  const int ix = pix % A.npx, iy = pix / A.npx;
  const RtView &V = A.v[v];
  const int nq = A.nimg;
  const R *rho = (const R *)A.rho;
  const R *S = (const R *)A.S + (uint64_t)v * A.ncell * nq;
  double I[MAX_IMG];
  R tr[MAX_IMG];
#pragma unroll
  for (int q = 0; q < MAX_IMG; ++q) {
    I[q] = 0.0;
    tr[q] = (R)1;
  }
  double pe[3], dir[3];
  int c[3];
  if (ray_entry(A, V, ix, iy, pe, dir, c)) {
    auto seg = [&](int64_t cell, double ell) {
      R r = rho[cell];
      if (!LIT && !(r > (R)0)) return;
      R sc[MAX_IMG];
      load_row(S + (uint64_t)cell * nq, nq, sc);
      R el = (R)ell;
#pragma unroll
      for (int q = 0; q < MAX_IMG; ++q) {
        if (q >= nq) break;
        R dtau = r * (R)A.kext[q] * el;
        R om, e;
        absorb_pair1(dtau, om, e);
        I[q] += (double)tr[q] * (double)sc[q] * (LIT ? 1.0 : (double)om);
        tr[q] *= e;
      }
    };
    if constexpr (REF) walk_leaves(A, pe, dir, c, seg);
    else walk(A, pe, dir, c, seg);
  }
  const uint64_t plane = (uint64_t)A.npx * A.npy;
#pragma unroll
  for (int q = 0; q < MAX_IMG; ++q) {
    if (q >= nq) break;
    img[((uint64_t)v * nq + q) * plane + pix] = (R)(V.apix_d2 * I[q]);
  }
}

// Attenuated point sources: one lane per (view, source, imaged wavelength).
template <typename R>
__global__ void k_rt_star(const RtArgs *__restrict__ Ap, R *img, double *sed) {
  const RtArgs &A = *Ap;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int q = t % A.nimg, s = (t / A.nimg) % A.nsrc, v = t / (A.nimg * A.nsrc);
  if (v >= A.nview) return;
  const RtView &V = A.v[v];
  const R *rho = (const R *)A.rho;
  double p0[3] = {A.srcpos[s][0], A.srcpos[s][1], A.srcpos[s][2]};
  int c[3];
  for (int k = 0; k < 3; ++k) {
    double qq = (p0[k] - A.origin[k]) / A.dcell;
    double f = floor(qq);
    int ci = (int)f;
    if (qq == f && V.k[k] < 0.0) ci -= 1;
    c[k] = ci;
  }
  double tau = 0.0;
  auto acc = [&](int64_t cell, double ell) { tau += (double)rho[cell] * A.kext[q] * ell; };
  if (A.ref) walk_leaves(A, p0, V.k, c, acc);
  else walk(A, p0, V.k, c, acc);
  double F = A.lnu[s][q] / (4.0 * PI_D * A.D2) * exp(-tau);
  double xp = 0.0, yp = 0.0;
  for (int k = 0; k < 3; ++k) {
    xp += (p0[k] - V.ctr[k]) * V.ex[k];
    yp += (p0[k] - V.ctr[k]) * V.ey[k];
  }
  int ix = (int)floor((xp + 0.5 * V.fov) / V.dpx), iy = (int)floor((yp + 0.5 * V.fov) / V.dpy);
  if (ix >= 0 && ix < A.npx && iy >= 0 && iy < A.npy)
    atomicAdd(&img[((uint64_t)v * A.nimg + q) * A.npx * A.npy + (uint64_t)iy * A.npx + ix], (R)F);
  if (sed) atomicAdd(&sed[v * A.nimg + q], F);
}

// SED of the dust: one block per (view, wavelength), fixed-order tree sum.
template <typename R>
__global__ void k_rt_sed(const RtArgs *__restrict__ Ap, const R *img, double *sed) {
  const RtArgs &A = *Ap;
  const int vq = blockIdx.x;
  const uint64_t plane = (uint64_t)A.npx * A.npy;
  const R *p = img + (uint64_t)vq * plane;
  double acc = 0.0;
  for (uint64_t i = threadIdx.x; i < plane; i += blockDim.x) acc += (double)p[i];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sed[vq] = red[0];
}

// Adjoint: first sweep gives I per wavelength, the second recomputes the
// transmittance and the gathered intensity A_i in front of each cell:
// dI/d(dtau_i) = T_<i S_i e^-dtau_i - (I - A_i), d(dtau_i)/d(rho_i) = kext l_i.
// LIT: the cell terms do not depend on the traced density, so
// dI/d(dtau_i) = -(I - A_i).
template <typename R, bool LIT, bool REF>
__global__ void __launch_bounds__(256) k_rt_adj(const RtArgs *__restrict__ Ap, const R *w_img,
                                                const double *w_sed, R *drho) {
  const RtArgs &A = *Ap;
  const int v = blockIdx.y;
  const int pix = blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= A.npx * A.npy) return;
  const int ix = pix % A.npx, iy = pix / A.npx;
  const RtView &V = A.v[v];
  const int nq = A.nimg;
  const R *rho = (const R *)A.rho;
  const R *S = (const R *)A.S + (uint64_t)v * A.ncell * nq;
  const uint64_t plane = (uint64_t)A.npx * A.npy;
  // wk = W kext (the weight of dI in dL/drho per unit length); rem = the
  // intensity that reaches the pixel from behind the current cell (I of the
  // whole ray less what the cells up to here contribute)
  double rem[MAX_IMG];
  R wk[MAX_IMG], tr[MAX_IMG];
  bool any = false;
#pragma unroll
  for (int q = 0; q < MAX_IMG; ++q) {
    double W = 0.0;
    if (q < nq) {
      W = (w_img ? (double)w_img[((uint64_t)v * nq + q) * plane + pix] : 0.0) +
          (w_sed ? w_sed[v * nq + q] : 0.0);
      W *= V.apix_d2;
    }
    any |= (W != 0.0);
    wk[q] = q < nq ? (R)(W * A.kext[q]) : (R)0;
    rem[q] = 0.0;
    tr[q] = (R)1;
  }
  if (!any) return;
  double pe[3], dir[3];
  int c[3];
  if (!ray_entry(A, V, ix, iy, pe, dir, c)) return;
  auto sweep1 = [&](int64_t cell, double ell) {
    R r = rho[cell];
    if (!LIT && !(r > (R)0)) return;
    const R *sc = S + (uint64_t)cell * nq;
    R el = (R)ell;
#pragma unroll
    for (int q = 0; q < MAX_IMG; ++q) {
      if (q >= nq) break;
      R om, e;
      absorb_pair1(r * (R)A.kext[q] * el, om, e);
      rem[q] += (double)tr[q] * (double)sc[q] * (LIT ? 1.0 : (double)om);
      tr[q] *= e;
    }
  };
  if constexpr (REF) walk_leaves(A, pe, dir, c, sweep1);
  else walk(A, pe, dir, c, sweep1);
#pragma unroll
  for (int q = 0; q < MAX_IMG; ++q) tr[q] = (R)1;
  auto sweep2 = [&](int64_t cell, double ell) {
    R r = rho[cell];
    if (!LIT && !(r > (R)0)) return;
    const R *sc = S + (uint64_t)cell * nq;
    R el = (R)ell;
    double g = 0.0;
#pragma unroll
    for (int q = 0; q < MAX_IMG; ++q) {
      if (q >= nq) break;
      R om, e;
      absorb_pair1(r * (R)A.kext[q] * el, om, e);
      double Sq = (double)sc[q];
      rem[q] -= (double)tr[q] * Sq * (LIT ? 1.0 : (double)om);
      double dI = (LIT ? 0.0 : (double)tr[q] * Sq * (double)e) - rem[q];
      g += (double)wk[q] * ell * dI;
      tr[q] *= e;
    }
    if (g != 0.0) atomicAdd(&drho[cell], (R)g);
  };
  if constexpr (REF) walk_leaves(A, pe, dir, c, sweep2);
  else walk(A, pe, dir, c, sweep2);
}

// Adjoint of the attenuated point-source term.
template <typename R>
__global__ void k_rt_star_adj(const RtArgs *__restrict__ Ap, const R *w_img, const double *w_sed,
                              R *drho) {
  const RtArgs &A = *Ap;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int q = t % A.nimg, s = (t / A.nimg) % A.nsrc, v = t / (A.nimg * A.nsrc);
  if (v >= A.nview) return;
  const RtView &V = A.v[v];
  const R *rho = (const R *)A.rho;
  double p0[3] = {A.srcpos[s][0], A.srcpos[s][1], A.srcpos[s][2]};
  int c[3];
  for (int k = 0; k < 3; ++k) {
    double qq = (p0[k] - A.origin[k]) / A.dcell;
    double f = floor(qq);
    int ci = (int)f;
    if (qq == f && V.k[k] < 0.0) ci -= 1;
    c[k] = ci;
  }
  double xp = 0.0, yp = 0.0;
  for (int k = 0; k < 3; ++k) {
    xp += (p0[k] - V.ctr[k]) * V.ex[k];
    yp += (p0[k] - V.ctr[k]) * V.ey[k];
  }
  int ix = (int)floor((xp + 0.5 * V.fov) / V.dpx), iy = (int)floor((yp + 0.5 * V.fov) / V.dpy);
  bool inimg = ix >= 0 && ix < A.npx && iy >= 0 && iy < A.npy;
  double W = (w_sed ? w_sed[v * A.nimg + q] : 0.0) +
             ((inimg && w_img) ? (double)w_img[((uint64_t)v * A.nimg + q) * A.npx * A.npy +
                                               (uint64_t)iy * A.npx + ix]
                               : 0.0);
  if (W == 0.0) return;
  double tau = 0.0;
  auto acc = [&](int64_t cell, double ell) { tau += (double)rho[cell] * A.kext[q] * ell; };
  if (A.ref) walk_leaves(A, p0, V.k, c, acc);
  else walk(A, p0, V.k, c, acc);
  double F = A.lnu[s][q] / (4.0 * PI_D * A.D2) * exp(-tau);
  auto grad = [&](int64_t cell, double ell) {
    atomicAdd(&drho[cell], (R)(-W * A.kext[q] * ell * F));
  };
  if (A.ref) walk_leaves(A, p0, V.k, c, grad);
  else walk(A, p0, V.k, c, grad);
}

template <typename R>
static void build_S_as(const ModelDev *d, bool lit, bool sh, R *S, hipStream_t st) {
  const dim3 g(65536), b(256);
  if (lit && sh) hipLaunchKernelGGL((k_build_S<R, true, true>), g, b, 0, st, d, S);
  else if (lit) hipLaunchKernelGGL((k_build_S<R, true, false>), g, b, 0, st, d, S);
  else if (sh) hipLaunchKernelGGL((k_build_S<R, false, true>), g, b, 0, st, d, S);
  else hipLaunchKernelGGL((k_build_S<R, false, false>), g, b, 0, st, d, S);
}

// lit and sh must match the model's rt_lit and sh_read (> 0).
hipError_t launch_build_S(const ModelDev *d, bool fp64, bool lit, bool sh, void *S,
                          hipStream_t st) {
  if (fp64) build_S_as<double>(d, lit, sh, (double *)S, st);
  else build_S_as<float>(d, lit, sh, (float *)S, st);
  return hipGetLastError();
}

// ev_main (nullable) is recorded right after the pixel-ray kernel, before
// the SED reduction and the point-source terms.
hipError_t launch_rt_fwd(const RtArgs *dA, const RtArgs &hA, bool fp64, void *img, double *sed,
                         hipEvent_t ev_main, hipStream_t st) {
  dim3 grid((hA.npx * hA.npy + 255) / 256, hA.nview);
  int nstar = hA.nview * hA.nsrc * hA.nimg;
  if (fp64) {
    if (hA.ref) {
      if (hA.lit) hipLaunchKernelGGL((k_rt_fwd<double, true, true>), grid, dim3(256), 0, st, dA, (double *)img);
      else hipLaunchKernelGGL((k_rt_fwd<double, false, true>), grid, dim3(256), 0, st, dA, (double *)img);
    } else {
      if (hA.lit) hipLaunchKernelGGL((k_rt_fwd<double, true, false>), grid, dim3(256), 0, st, dA, (double *)img);
      else hipLaunchKernelGGL((k_rt_fwd<double, false, false>), grid, dim3(256), 0, st, dA, (double *)img);
    }
    if (ev_main) (void)hipEventRecord(ev_main, st);
    if (sed) hipLaunchKernelGGL(k_rt_sed<double>, dim3(hA.nview * hA.nimg), dim3(256), 0, st, dA,
                                (const double *)img, sed);
    if (nstar) hipLaunchKernelGGL(k_rt_star<double>, dim3((nstar + 63) / 64), dim3(64), 0, st, dA,
                                  (double *)img, sed);
  } else {
    if (hA.ref) {
      if (hA.lit) hipLaunchKernelGGL((k_rt_fwd<float, true, true>), grid, dim3(256), 0, st, dA, (float *)img);
      else hipLaunchKernelGGL((k_rt_fwd<float, false, true>), grid, dim3(256), 0, st, dA, (float *)img);
    } else {
      if (hA.lit) hipLaunchKernelGGL((k_rt_fwd<float, true, false>), grid, dim3(256), 0, st, dA, (float *)img);
      else hipLaunchKernelGGL((k_rt_fwd<float, false, false>), grid, dim3(256), 0, st, dA, (float *)img);
    }
    if (ev_main) (void)hipEventRecord(ev_main, st);
    if (sed) hipLaunchKernelGGL(k_rt_sed<float>, dim3(hA.nview * hA.nimg), dim3(256), 0, st, dA,
                                (const float *)img, sed);
    if (nstar) hipLaunchKernelGGL(k_rt_star<float>, dim3((nstar + 63) / 64), dim3(64), 0, st, dA,
                                  (float *)img, sed);
  }
  return hipGetLastError();
}

hipError_t launch_rt_adj(const RtArgs *dA, const RtArgs &hA, bool fp64, const void *w_img,
                         const double *w_sed, void *drho, hipEvent_t ev_main, hipStream_t st) {
  dim3 grid((hA.npx * hA.npy + 255) / 256, hA.nview);
  int nstar = hA.nview * hA.nsrc * hA.nimg;
  if (fp64) {
    if (hA.ref) {
      if (hA.lit)
        hipLaunchKernelGGL((k_rt_adj<double, true, true>), grid, dim3(256), 0, st, dA,
                           (const double *)w_img, w_sed, (double *)drho);
      else
        hipLaunchKernelGGL((k_rt_adj<double, false, true>), grid, dim3(256), 0, st, dA,
                           (const double *)w_img, w_sed, (double *)drho);
    } else {
      if (hA.lit)
        hipLaunchKernelGGL((k_rt_adj<double, true, false>), grid, dim3(256), 0, st, dA,
                           (const double *)w_img, w_sed, (double *)drho);
      else
        hipLaunchKernelGGL((k_rt_adj<double, false, false>), grid, dim3(256), 0, st, dA,
                           (const double *)w_img, w_sed, (double *)drho);
    }
    if (ev_main) (void)hipEventRecord(ev_main, st);
    if (nstar) hipLaunchKernelGGL(k_rt_star_adj<double>, dim3((nstar + 63) / 64), dim3(64), 0, st,
                                  dA, (const double *)w_img, w_sed, (double *)drho);
  } else {
    if (hA.ref) {
      if (hA.lit)
        hipLaunchKernelGGL((k_rt_adj<float, true, true>), grid, dim3(256), 0, st, dA,
                           (const float *)w_img, w_sed, (float *)drho);
      else
        hipLaunchKernelGGL((k_rt_adj<float, false, true>), grid, dim3(256), 0, st, dA,
                           (const float *)w_img, w_sed, (float *)drho);
    } else {
      if (hA.lit)
        hipLaunchKernelGGL((k_rt_adj<float, true, false>), grid, dim3(256), 0, st, dA,
                           (const float *)w_img, w_sed, (float *)drho);
      else
        hipLaunchKernelGGL((k_rt_adj<float, false, false>), grid, dim3(256), 0, st, dA,
                           (const float *)w_img, w_sed, (float *)drho);
    }
    if (ev_main) (void)hipEventRecord(ev_main, st);
    if (nstar) hipLaunchKernelGGL(k_rt_star_adj<float>, dim3((nstar + 63) / 64), dim3(64), 0, st,
                                  dA, (const float *)w_img, w_sed, (float *)drho);
  }
  return hipGetLastError();
}

}  // namespace mcrt
