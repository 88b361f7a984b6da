// mcrt_voxel.hip - model set-up kernels: density grids of the clumpy AGN
// torus (sect. 6, Eq. 21 clump centres) and of power-law spherical shells.
#include "mcrt_internal.h"

namespace mcrt {

// Cell-centre test: clump density inside any clump (overlaps keep the
// single-clump value), inter-clump density inside the wedge, else empty.
// All decisions use exact products and sums in FP64.
template <typename R>
__global__ void k_vox_torus(int nx, int ny, int nz, double ox, double oy, double oz, double dc,
                            int ncl, const double *__restrict__ C, double rc2, double rho_cl,
                            double rho_int, double ri2, double ro2, double s12, R *rho) {
  extern __shared__ double cs[];
  uint64_t n = (uint64_t)nx * ny * nz;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((uint64_t)nx * ny));
  double x = ox + ((double)ix + 0.5) * dc;
  double y = oy + ((double)iy + 0.5) * dc;
  double z = oz + ((double)iz + 0.5) * dc;
  bool hit = false;
  // clump centres staged through LDS in tiles
  for (int base = 0; base < ncl; base += 1024) {
    int m = ncl - base < 1024 ? ncl - base : 1024;
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * m; t += blockDim.x) cs[t] = C[3 * base + t];
    __syncthreads();
    if (i < n && !hit) {
      for (int k = 0; k < m; ++k) {
        double dx = x - cs[3 * k], dy = y - cs[3 * k + 1], dz = z - cs[3 * k + 2];
        if (dx * dx + dy * dy + dz * dz <= rc2) {
          hit = true;
          break;
        }
      }
    }
  }
  if (i >= n) return;
  double v = 0.0;
  if (hit) {
    v = rho_cl;
  } else {
    double r2 = x * x + y * y + z * z;
    if (r2 >= ri2 && r2 <= ro2 && z * z <= r2 * s12) v = rho_int;
  }
  rho[i] = (R)v;
}

// Cell average of rho0 (r_in/r)^power on [r_in, r_out] (power 2: r^-2
// shell, 0: constant density) by a product Gauss-Legendre rule with the
// nodes/weights given.
template <typename R>
__global__ void k_vox_shell(int nx, int ny, int nz, double ox, double oy, double oz, double dc,
                            double rho0, double r_in, double r_out, double power, int ng,
                            const double *__restrict__ gx, const double *__restrict__ gw, R *rho) {
  uint64_t n = (uint64_t)nx * ny * nz;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((uint64_t)nx * ny));
  double sum = 0.0;
  for (int a = 0; a < ng; ++a)
    for (int b = 0; b < ng; ++b)
      for (int e = 0; e < ng; ++e) {
        double x = ox + ((double)ix + 0.5 + 0.5 * gx[a]) * dc;
        double y = oy + ((double)iy + 0.5 + 0.5 * gx[b]) * dc;
        double z = oz + ((double)iz + 0.5 + 0.5 * gx[e]) * dc;
        double r = sqrt(x * x + y * y + z * z);
        double f = 0.0;
        if (r >= r_in && r <= r_out) {
          const double q = r_in / r;
          f = power == 2.0 ? rho0 * q * q : (power == 0.0 ? rho0 : rho0 * pow(q, power));
        }
        sum += gw[a] * gw[b] * gw[e] * f;
      }
  rho[i] = (R)(0.125 * sum);
}

hipError_t launch_vox_torus(bool fp64, int nx, int ny, int nz, const double o[3], double dc,
                            int ncl, const double *dC, double r_clump, double rho_cl,
                            double rho_int, double r_in, double r_out, double s1, void *rho,
                            hipStream_t st) {
  uint64_t n = (uint64_t)nx * ny * nz;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  size_t lds = 3 * 1024 * sizeof(double);
  double rc2 = r_clump * r_clump, ri2 = r_in * r_in, ro2 = r_out * r_out, s12 = s1 * s1;
  if (fp64)
    hipLaunchKernelGGL(k_vox_torus<double>, grid, block, lds, st, nx, ny, nz, o[0], o[1], o[2], dc,
                       ncl, dC, rc2, rho_cl, rho_int, ri2, ro2, s12, (double *)rho);
  else
    hipLaunchKernelGGL(k_vox_torus<float>, grid, block, lds, st, nx, ny, nz, o[0], o[1], o[2], dc,
                       ncl, dC, rc2, rho_cl, rho_int, ri2, ro2, s12, (float *)rho);
  return hipGetLastError();
}

hipError_t launch_vox_shell(bool fp64, int nx, int ny, int nz, const double o[3], double dc,
                            double rho0, double r_in, double r_out, double power, int ng,
                            const double *dgx, const double *dgw, void *rho, hipStream_t st) {
  uint64_t n = (uint64_t)nx * ny * nz;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (fp64)
    hipLaunchKernelGGL(k_vox_shell<double>, grid, block, 0, st, nx, ny, nz, o[0], o[1], o[2], dc,
                       rho0, r_in, r_out, power, ng, dgx, dgw, (double *)rho);
  else
    hipLaunchKernelGGL(k_vox_shell<float>, grid, block, 0, st, nx, ny, nz, o[0], o[1], o[2], dc,
                       rho0, r_in, r_out, power, ng, dgx, dgw, (float *)rho);
  return hipGetLastError();
}

}  // namespace mcrt
