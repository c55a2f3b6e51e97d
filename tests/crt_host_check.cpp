// Host driver for the CRT arithmetic of the library (oz2_crt_math.h) with the
// library's own tables (oz2_tables.cpp): for N moduli of list `list`, reads
// lines "t u_1 ... u_N" (residues in the symmetric range of the int16 planes)
// and prints, per line, the bits of RN(C' 2^-t) with C' = sum_l w_l u_l mods P,
// computed exactly as the CRT kernel does.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "oz2_crt_math.h"

namespace {

template <int L>
double reconstruct(const oz2::Tables &tab, const int *u, int N, int t) {
  double acc[L];
  for (int q = 0; q < L; ++q) acc[q] = 0.0;
  for (int l = 0; l < N; ++l)
    for (int q = 0; q < L; ++q) acc[q] = fma(tab.wd[l][q], (double)u[l], acc[q]);
  uint32_t mag[L];
  const bool neg = oz2::crt_reduce<L>(acc, &tab, mag);
  const double v = oz2::scaled_rn<L>(mag, t);
  return neg ? -v : v;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  const int N = atoi(argv[1]), list = atoi(argv[2]);
  static oz2::Tables tab;
  if (!oz2::build_tables(N, list, &tab)) return 3;
  std::vector<int> u(N);
  int t;
  while (scanf("%d", &t) == 1) {
    for (int l = 0; l < N; ++l)
      if (scanf("%d", &u[l]) != 1) return 4;
    double r;
    switch (tab.limbs) {
      case 1: r = reconstruct<1>(tab, u.data(), N, t); break;
      case 2: r = reconstruct<2>(tab, u.data(), N, t); break;
      case 3: r = reconstruct<3>(tab, u.data(), N, t); break;
      case 4: r = reconstruct<4>(tab, u.data(), N, t); break;
      case 5: r = reconstruct<5>(tab, u.data(), N, t); break;
      case 6: r = reconstruct<6>(tab, u.data(), N, t); break;
      case 7: r = reconstruct<7>(tab, u.data(), N, t); break;
      case 8: r = reconstruct<8>(tab, u.data(), N, t); break;
      case 9: r = reconstruct<9>(tab, u.data(), N, t); break;
      case 10: r = reconstruct<10>(tab, u.data(), N, t); break;
      default: return 5;
    }
    uint64_t bits;
    memcpy(&bits, &r, 8);
    printf("%016llx\n", (unsigned long long)bits);
  }
  return 0;
}
