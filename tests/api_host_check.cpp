// Host driver for the C ABI's host-side logic (oz2_api.cpp, oz2_tables.cpp):
// argument checks, workspace sizes and layouts, settings.  Built with the
// sanitizers against stub kernel launchers (no device code), it reads one
// command per line and prints one result line, for comparison with the
// library itself:
//   L list                      ozaki2_set_moduli_list
//   B m_blk n_blk               ozaki2_set_blocking
//   M mode                      ozaki2_set_mode
//   S config                    ozaki2_set_schedule
//   K parts                     ozaki2_set_split
//   W m n k N                   ozaki2_workspace_bytes
//   Y m n k N                   ozaki2_workspace_layout (status, 11 offsets, 4 pads)
//   R m n k N                   ozaki2_workspace_parts (status, parts, bound parts)
//   Q N count m n k ...         ozaki2_workspace_bytes_batched
//   D ta tb m n k lda ldb ldc N ozaki2_dgemm on null pointers (argument checks;
//                               valid arguments end at the device check)
//   P N                         ozaki2_moduli
#include <stdio.h>
#include <string.h>

#include <vector>

#include "oz2_internal.h"

namespace oz2 {
// no kernels in this build: every launch succeeds without doing anything
hipError_t launch_quant_family(int, const Problem *, const Group *, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_scale_family(int, const Problem *, const Group *, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_gemm_family(int, const Problem *, const Group *, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_gemm_persistent(int, bool, const WorkList &, int64_t, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_crt_family(const Problem *, const Group *, int, int, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_scal(int64_t, int64_t, double, double *, int64_t, hipStream_t) {
  return hipSuccess;
}
}  // namespace oz2

int main() {
  char cmd[8];
  while (scanf("%7s", cmd) == 1) {
    long long a[12];
    if (!strcmp(cmd, "L")) {
      if (scanf("%lld", &a[0]) != 1) return 2;
      printf("%d\n", ozaki2_set_moduli_list((int)a[0]));
    } else if (!strcmp(cmd, "B")) {
      if (scanf("%lld %lld", &a[0], &a[1]) != 2) return 2;
      printf("%d\n", ozaki2_set_blocking(a[0], a[1]));
    } else if (!strcmp(cmd, "M")) {
      if (scanf("%lld", &a[0]) != 1) return 2;
      printf("%d\n", ozaki2_set_mode((int)a[0]));
    } else if (!strcmp(cmd, "S")) {
      if (scanf("%lld", &a[0]) != 1) return 2;
      printf("%d\n", ozaki2_set_schedule((int)a[0]));
    } else if (!strcmp(cmd, "K")) {
      if (scanf("%lld", &a[0]) != 1) return 2;
      printf("%d\n", ozaki2_set_split((int)a[0]));
    } else if (!strcmp(cmd, "W")) {
      if (scanf("%lld %lld %lld %lld", &a[0], &a[1], &a[2], &a[3]) != 4) return 2;
      printf("%zu\n", ozaki2_workspace_bytes(a[0], a[1], a[2], (int)a[3]));
    } else if (!strcmp(cmd, "Y")) {
      if (scanf("%lld %lld %lld %lld", &a[0], &a[1], &a[2], &a[3]) != 4) return 2;
      int64_t off[11] = {0}, pads[4] = {0};
      const int r = ozaki2_workspace_layout(a[0], a[1], a[2], (int)a[3], off, pads);
      printf("%d", r);
      for (int q = 0; q < 11; ++q) printf(" %lld", r > 0 ? (long long)off[q] : 0ll);
      for (int q = 0; q < 4; ++q) printf(" %lld", r > 0 ? (long long)pads[q] : 0ll);
      printf("\n");
    } else if (!strcmp(cmd, "R")) {
      if (scanf("%lld %lld %lld %lld", &a[0], &a[1], &a[2], &a[3]) != 4) return 2;
      int parts = 0, bparts = 0;
      const int r = ozaki2_workspace_parts(a[0], a[1], a[2], (int)a[3], &parts, &bparts);
      printf("%d %d %d\n", r, r == 0 ? parts : 0, r == 0 ? bparts : 0);
    } else if (!strcmp(cmd, "Q")) {
      long long N, cnt;
      if (scanf("%lld %lld", &N, &cnt) != 2 || cnt < 0 || cnt > 4096) return 2;
      std::vector<int64_t> m(cnt), n(cnt), k(cnt);
      for (long long q = 0; q < cnt; ++q) {
        long long x, y, z;
        if (scanf("%lld %lld %lld", &x, &y, &z) != 3) return 2;
        m[q] = x;
        n[q] = y;
        k[q] = z;
      }
      printf("%zu\n", ozaki2_workspace_bytes_batched((int)cnt, m.data(), n.data(), k.data(),
                                                     (int)N));
    } else if (!strcmp(cmd, "D")) {
      char ta[4], tb[4];
      if (scanf("%3s %3s %lld %lld %lld %lld %lld %lld %lld", ta, tb, &a[0], &a[1], &a[2],
                &a[3], &a[4], &a[5], &a[6]) != 9)
        return 2;
      printf("%d\n", ozaki2_dgemm(ta[0], tb[0], a[0], a[1], a[2], 1.0, nullptr, a[3], nullptr,
                                  a[4], 0.0, nullptr, a[5], (int)a[6]));
    } else if (!strcmp(cmd, "P")) {
      if (scanf("%lld", &a[0]) != 1) return 2;
      int32_t p[64], kinds[64];
      const int r = ozaki2_moduli((int)a[0], p, kinds);
      printf("%d", r);
      if (r == 0)
        for (int q = 0; q < a[0]; ++q) printf(" %d:%d", p[q], kinds[q]);
      printf("\n");
    } else {
      return 3;
    }
  }
  return 0;
}
