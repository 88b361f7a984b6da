// mcrt_rtargs.h - arguments of the ray-tracer kernels (one launch covers
// every view; per-view frames, per-wavelength extinction, point sources).
#pragma once
#include "mcrt_internal.h"

namespace mcrt {

struct RtView {
  double k[3], ex[3], ey[3];
  double ctr[3], fov, dpx, dpy, apix_d2;
};

struct RtArgs {
  int32_t nx, ny, nz, nimg, npx, npy, nview, nsrc;
  double origin[3], dcell;
  uint64_t ncell;
  const void *rho;            // traced density (context precision)
  const void *S;              // [view][cell][nimg] context precision
  double kext[MAX_IMG];       // per imaged wavelength (cgs)
  double lnu[MAX_SRC][MAX_IMG];
  double srcpos[MAX_SRC][3];
  double D2;
  RtView v[MAX_VIEW];
};

}  // namespace mcrt
