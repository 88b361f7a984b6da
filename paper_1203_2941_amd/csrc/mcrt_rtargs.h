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
  int32_t lit, pad_;          // 1: printed form of Eqs. 13-14 (S holds each cell's term C)
  double origin[3], dcell;
  uint64_t ncell;             // leaf cells (per-cell arrays)
  uint64_t ncube;             // cubes of the grid
  const uint8_t *ref;         // refined grids: sub-cubes per edge of each cube (else null)
  const uint64_t *sub_off;    // first sub-cube of each divided cube
  const void *rho;            // traced density (context precision)
  const void *S;              // [view][cell][nimg] context precision
  double kext[MAX_IMG];       // per imaged wavelength (cgs): extinction, or the mixture's
                              // absorption in the printed form
  double lnu[MAX_SRC][MAX_IMG];
  double srcpos[MAX_SRC][3];
  double D2;
  RtView v[MAX_VIEW];
};

}  // namespace mcrt
