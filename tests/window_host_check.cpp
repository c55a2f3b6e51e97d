// Host driver for the accurate mode's decision window (oz2_window.h) with the
// library's own tables (oz2_tables.cpp): for N moduli of list `list`, reads
// lines "kp parts bits" (kp: the padded k extent; parts: the k ranges whose
// sums are added; bits: the FP32 bit pattern of a computed line maximum
// r' > 0, in hex) and prints, per line, the window's ends as hex doubles and
// the scale exponents of both ends, exactly as the scale kernel computes them.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oz2_internal.h"
#include "oz2_window.h"

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  const int N = atoi(argv[1]), list = atoi(argv[2]);
  static oz2::Tables tab;
  if (!oz2::build_tables(N, list, &tab)) return 3;
  long long kp;
  int parts;
  unsigned bits;
  while (scanf("%lld %d %x", &kp, &parts, &bits) == 3) {
    float r;
    memcpy(&r, &bits, 4);
    double lo, hi;
    oz2::bound_window((double)r, (int64_t)kp, parts, &lo, &hi);
    int es, el;
    oz2::window_exponents((double)r, (int64_t)kp, parts, tab.D, &es, &el);
    printf("%a %a %d %d\n", lo, hi, es, el);
  }
  return 0;
}
