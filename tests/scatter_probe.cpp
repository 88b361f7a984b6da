// Host build of the library's scattering rotation (mcrt_scatter.h): reads
// "prec dx dy dz mu phi" lines (prec 4 = FP32, 8 = FP64; values as C
// floating literals, hex allowed), rotates d in that precision and prints
// the new direction in hex.
#include <cstdio>

#include "../paper_1203_2941_amd/csrc/mcrt_scatter.h"

int main() {
  int prec;
  double a[5];
  while (std::scanf("%d %lf %lf %lf %lf %lf", &prec, &a[0], &a[1], &a[2], &a[3], &a[4]) == 6) {
    if (prec == 4) {
      float d[3] = {(float)a[0], (float)a[1], (float)a[2]};
      mcrt::rotate_dir<float>(d, (float)a[3], (float)a[4]);
      std::printf("%a %a %a\n", (double)d[0], (double)d[1], (double)d[2]);
    } else {
      double d[3] = {a[0], a[1], a[2]};
      mcrt::rotate_dir<double>(d, a[3], a[4]);
      std::printf("%a %a %a\n", d[0], d[1], d[2]);
    }
  }
  return 0;
}
