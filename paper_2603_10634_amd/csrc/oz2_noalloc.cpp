// ozaki2_dgemm_noalloc: the emulated DGEMM for callers that cannot allocate
// device memory.  Its workspace is a file-scope device array of fixed size,
// and the moduli/CRT tables of every (list, N) sit in a second one; both are
// set up once per device (their device addresses looked up, the tables
// copied in) on the first call on that device, after which a call only
// launches kernels.
#include <mutex>

#include "oz2_internal.h"

namespace {

// The workspace of ozaki2_dgemm_noalloc on each device (held until the
// process ends).  In host code these names stand for host-side shadows, not
// device addresses: the kernels only ever receive the addresses that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[OZ2_NOALLOC_SCRATCH_BYTES];
static __device__ __align__(256) oz2::Tables scratch_tables[3][oz2::kMaxN];

constexpr int kMaxDevices = 64;

struct DeviceScratch {
  bool ready = false;
  uint8_t *ws = nullptr;
  oz2::Tables *tables = nullptr;
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

// Device addresses of the arrays on `dev` (the current device), looked up
// and filled with the tables on the first call on that device.
oz2::FixedResources resources(int dev) {
  oz2::FixedResources r{nullptr, 0, nullptr};
  if (dev < 0 || dev >= kMaxDevices) return r;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceScratch &d = g_dev[dev];
  if (!d.ready) {
    void *ws = nullptr, *tab = nullptr;
    if (hipGetSymbolAddress(&ws, HIP_SYMBOL(scratch)) != hipSuccess ||
        hipGetSymbolAddress(&tab, HIP_SYMBOL(scratch_tables)) != hipSuccess) {
      (void)hipGetLastError();
      return r;
    }
    static oz2::Tables host;
    for (int list = 0; list < 3; ++list)
      for (int N = 1; N <= oz2::kMaxN; ++N) {
        if (!oz2::host_tables_for(N, list, &host)) continue;
        oz2::Tables *dst = (oz2::Tables *)tab + (size_t)list * oz2::kMaxN + (N - 1);
        if (hipMemcpy(dst, &host, sizeof(host), hipMemcpyHostToDevice) != hipSuccess) {
          (void)hipGetLastError();
          return r;
        }
      }
    d.ws = (uint8_t *)ws;
    d.tables = (oz2::Tables *)tab;
    d.ready = true;
  }
  r.ws = d.ws;
  r.ws_bytes = OZ2_NOALLOC_SCRATCH_BYTES;
  r.tables = d.tables;
  return r;
}

}  // namespace

extern "C" int ozaki2_dgemm_noalloc(char transA, char transB, int64_t m, int64_t n, int64_t k,
                                    double alpha, const double *A, int64_t lda, const double *B,
                                    int64_t ldb, double beta, double *C, int64_t ldc,
                                    int num_moduli) {
  return oz2::dgemm_fixed(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                          num_moduli, resources);
}
