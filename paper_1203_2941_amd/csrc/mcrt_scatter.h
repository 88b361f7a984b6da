// mcrt_scatter.h - Henyey-Greenstein scattering (Eq. 15) and the rotation
// of a direction by a scattering angle, for host and device.
//
// Kept apart so that the same FP32 and FP64 code can be exercised on the
// host (tests compile it without a GPU).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace mcrt {

constexpr double PI_SC = 3.14159265358979323846;

// Henyey-Greenstein inverse CDF of cos(beta) and phase function (Eq. 15).
template <typename R> __host__ __device__ inline R hg_mu(R g, R u) {
  if (std::fabs(g) < (R)1e-6) return (R)2 * u - (R)1;
  R q = ((R)1 - g * g) / ((R)1 - g + (R)2 * g * u);
  R mu = ((R)1 + g * g - q * q) / ((R)2 * g);
  if (mu > (R)1) mu = (R)1;
  if (mu < (R)-1) mu = (R)-1;
  return mu;
}
template <typename R> __host__ __device__ inline R hg_phase(R g, R mu) {
  R den = (R)1 + g * g - (R)2 * g * mu;
  return ((R)1 - g * g) / ((R)4 * (R)PI_SC * den * std::sqrt(den));
}

// New direction at polar angle acos(mu) and azimuth phi about d, then
// renormalised. The frame about d is e1 = (dx dz, dy dz, -s^2)/s,
// e2 = (-dy, dx, 0)/s with s the length of d's xy part.
//  - FP64: s = sqrt(1 - dz^2), with the polar case for |dz| > 1 - 1e-10
//    (the evaluation of the reference method, so that both codes round
//    alike).
//  - FP32: 1 - 1e-10 rounds to 1 and 1 - dz^2 cancels near the poles (a
//    direction within ~2e-4 rad of +-z has dz == 1.0f exactly, which made
//    s = 0 and the frame NaN). s is taken as hypot(dx, dy) instead, which
//    keeps e1, e2 orthonormal to d at any tilt; the polar case is left for
//    s == 0 (dx = dy = 0).
template <typename R> __host__ __device__ inline void rotate_dir(R d[3], R mu, R phi) {
  R t = (R)1 - mu * mu;
  R st = std::sqrt(t > (R)0 ? t : (R)0);
  R cp = std::cos(phi), sp = std::sin(phi);
  R nx, ny, nz;
  bool pole;
  R s;
  if constexpr (sizeof(R) == 8) {
    pole = std::fabs(d[2]) > 1.0 - 1e-10;
    s = pole ? 0.0 : std::sqrt(1.0 - d[2] * d[2]);
  } else {
    s = std::sqrt(d[0] * d[0] + d[1] * d[1]);
    pole = !(s > 1e-30f);
  }
  if (pole) {
    nx = st * cp;
    ny = st * sp;
    nz = (d[2] > (R)0) ? mu : -mu;
  } else {
    nx = st * (d[0] * d[2] * cp - d[1] * sp) / s + d[0] * mu;
    ny = st * (d[1] * d[2] * cp + d[0] * sp) / s + d[1] * mu;
    nz = -st * cp * s + d[2] * mu;
  }
  R nn = std::sqrt(nx * nx + ny * ny + nz * nz);
  d[0] = nx / nn;
  d[1] = ny / nn;
  d[2] = nz / nn;
}

}  // namespace mcrt
