// Host-side checks of the routing helpers in internal.h, driven by
// test_host_logic.py: reads commands from stdin and prints results.
//   w m n score sigma_max alpha beta  -> band_w_for_score
//   r m n W smax_pos drop alpha beta  -> band16_range_ok, band16_bias, ub, lb
//   c                                 -> packed and 32-bit class widths
//   p m n w smax_pos drop alpha beta  -> band_route (packed flag, class, width)
//   f v                               -> FP8 E4M3 code, E5M2 code, E5M2 exactness
#include <cstdio>
#include <cstring>

#include "internal.h"

using namespace asmi;

int main() {
  char cmd[8];
  while (scanf("%7s", cmd) == 1) {
    if (!strcmp(cmd, "w")) {
      int m, n, s, sm, a, b;
      if (scanf("%d %d %d %d %d %d", &m, &n, &s, &sm, &a, &b) != 6) return 2;
      printf("%d\n", band_w_for_score(m, n, s, sm, a, b));
    } else if (!strcmp(cmd, "r")) {
      int m, n, W, sp, dr, a, b;
      if (scanf("%d %d %d %d %d %d %d", &m, &n, &W, &sp, &dr, &a, &b) != 7) return 2;
      printf("%d %d %lld %lld\n", (int)band16_range_ok(m, n, W, sp, dr, a, b), band16_bias(m, n, W, sp, a, b),
             (long long)band16_ub(m, n, W, sp, a, b), (long long)band16_lb(m, n, dr, a, b));
    } else if (!strcmp(cmd, "c")) {
      for (int pc = 0; pc < kBand16Classes; ++pc) printf("%d ", band16_class_width(pc));
      printf("\n");
      for (int kc = 0; kc < kBandClasses; ++kc) printf("%d ", band_class_width(kc));
      printf("\n");
    } else if (!strcmp(cmd, "p")) {
      int m, n, w, sp, dr, a, b;
      if (scanf("%d %d %d %d %d %d %d", &m, &n, &w, &sp, &dr, &a, &b) != 7) return 2;
      bool packed = false;
      const int c = band_route(m, n, w, true, sp, dr, a, b, &packed);
      printf("%d %d %d\n", (int)packed, c, c < 0 ? 0 : (packed ? band16_class_width(c) : band_class_width(c)));
    } else if (!strcmp(cmd, "f")) {
      int v;
      if (scanf("%d", &v) != 1) return 2;
      printf("%u %u %d\n", fp8_e4m3(v), fp8_e5m2(v), (int)e5m2_exact(v));
    } else {
      return 3;
    }
    fflush(stdout);
  }
  return 0;
}
