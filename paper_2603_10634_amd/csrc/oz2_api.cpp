// C ABI: argument checking, workspace management, per-device tables and the
// launch sequence of one emulated DGEMM (the workflow of Section IV-B).
#include <string.h>

#include <map>
#include <mutex>
#include <utility>

#include "oz2_internal.h"

using namespace oz2;

namespace {

constexpr int kEvents = 7;

struct ThreadState {
  hipStream_t stream = nullptr;
  void *user_ws = nullptr;
  size_t user_ws_bytes = 0;
  void *own_ws = nullptr;
  size_t own_ws_bytes = 0;
  int own_dev = -1;
  bool timing = false;
  bool ev_ready = false;
  int ev_dev = -1;
  hipEvent_t ev[kEvents];
  bool have_times = false;
};

thread_local ThreadState g_ts;

std::mutex g_mu;
std::map<std::pair<int, int>, Tables *> g_tables;  // (device, N) -> device copy
std::map<int, bool> g_is_gfx950;
std::map<int, Tables> g_host_tables;                // N -> host copy

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct Layout {
  int64_t mp, np, kp;
  int M;
  size_t off[17];
  size_t total;
};

// Offsets of every workspace buffer (256-byte aligned).  The zero-initialised
// per-line vectors come first and contiguously so one fill clears them.
bool make_layout(int64_t m, int64_t n, int64_t k, int N, Layout *L) {
  Tables t;
  if (!build_tables(N, &t)) return false;
  L->mp = round_up(m > 0 ? m : 1, kPad);
  L->np = round_up(n > 0 ? n : 1, kPad);
  L->kp = round_up(k > 0 ? k : 1, kPad);
  L->M = t.M;
  const int64_t lines = L->mp + L->np;
  size_t o = 0;
  auto take = [&](int idx, size_t bytes) {
    L->off[idx] = o;
    o += (bytes + 255) / 256 * 256;
  };
  // zero-initialised group
  take(10, sizeof(uint64_t) * lines);          // amax
  take(11, sizeof(uint32_t) * lines);          // flags
  take(12, sizeof(uint32_t) * lines);          // rmax
  take(13, sizeof(uint64_t) * lines);          // rfix
  take(14, sizeof(uint32_t) * (lines + 1));    // amb
  L->off[15] = o;                              // end of the zeroed group
  take(0, sizeof(int32_t) * lines);            // shift
  take(1, sizeof(int32_t) * lines);            // E
  take(2, sizeof(int32_t) * lines);            // e
  take(3, (size_t)(L->mp * L->kp));            // Abar
  take(4, (size_t)(L->np * L->kp));            // Bbar
  take(5, (size_t)t.M * L->mp * L->kp);        // A slices
  take(6, (size_t)t.M * L->np * L->kp);        // B slices
  take(7, sizeof(int16_t) * (size_t)N * L->mp * L->np);  // planes
  L->off[8] = L->off[12];
  L->off[9] = L->off[11];
  L->off[16] = L->off[14];
  L->total = o;
  return true;
}

bool device_ok(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_is_gfx950.find(dev);
  if (it != g_is_gfx950.end()) return it->second;
  hipDeviceProp_t prop;
  bool ok = hipGetDeviceProperties(&prop, dev) == hipSuccess &&
            strncmp(prop.gcnArchName, "gfx950", 6) == 0;
  g_is_gfx950[dev] = ok;
  return ok;
}

const Tables *host_tables(int N) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_host_tables.find(N);
  if (it != g_host_tables.end()) return &it->second;
  Tables t;
  if (!build_tables(N, &t)) return nullptr;
  return &(g_host_tables[N] = t);
}

// Device copy of the tables, created once per (device, N) and kept for the
// life of the process.
const Tables *device_tables(int dev, int N, hipError_t *err) {
  const Tables *h = host_tables(N);
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, N);
  auto it = g_tables.find(key);
  if (it != g_tables.end()) return it->second;
  Tables *d = nullptr;
  *err = hipMalloc((void **)&d, sizeof(Tables));
  if (*err != hipSuccess) return nullptr;
  *err = hipMemcpy(d, h, sizeof(Tables), hipMemcpyHostToDevice);
  if (*err != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  g_tables[key] = d;
  return d;
}

int ensure_events(int dev) {
  ThreadState &ts = g_ts;
  if (ts.ev_ready && ts.ev_dev == dev) return OZ2_SUCCESS;
  if (ts.ev_ready) {
    for (int q = 0; q < kEvents; ++q) (void)hipEventDestroy(ts.ev[q]);
    ts.ev_ready = false;
  }
  for (int q = 0; q < kEvents; ++q)
    if (hipEventCreate(&ts.ev[q]) != hipSuccess) return OZ2_ERR_HIP;
  ts.ev_ready = true;
  ts.ev_dev = dev;
  return OZ2_SUCCESS;
}

bool valid_trans(char c) {
  return c == 'N' || c == 'n' || c == 'T' || c == 't' || c == 'C' || c == 'c';
}

}  // namespace

extern "C" {

const char *ozaki2_status_string(int status) {
  switch (status) {
    case OZ2_SUCCESS: return "success";
    case OZ2_ERR_HIP: return "HIP runtime error";
    case OZ2_ERR_ALLOC: return "workspace allocation failed";
    case OZ2_ERR_WORKSPACE: return "caller workspace too small";
    case OZ2_ERR_UNSUPPORTED: return "unsupported size or state";
    case OZ2_ERR_NO_DEVICE: return "no gfx950 device is current";
    default: return status < 0 ? "invalid argument" : "unknown status";
  }
}

int ozaki2_moduli(int num_moduli, int32_t *p, int32_t *kinds) {
  const Tables *t = host_tables(num_moduli);
  if (!t) return -1;
  for (int l = 0; l < num_moduli; ++l) {
    if (p) p[l] = t->p[l];
    if (kinds) kinds[l] = t->kind[l];
  }
  return 0;
}

size_t ozaki2_workspace_bytes(int64_t m, int64_t n, int64_t k, int num_moduli) {
  if (m < 0 || n < 0 || k < 0 || num_moduli < 1 || num_moduli > OZ2_MAX_MODULI) return 0;
  Layout L;
  if (!make_layout(m, n, k, num_moduli, &L)) return 0;
  return L.total;
}

int ozaki2_workspace_layout(int64_t m, int64_t n, int64_t k, int num_moduli, int64_t *off,
                            int64_t *pads) {
  if (m < 0 || n < 0 || k < 0 || num_moduli < 1 || num_moduli > OZ2_MAX_MODULI) return -1;
  Layout L;
  if (!make_layout(m, n, k, num_moduli, &L)) return -1;
  if (off) {
    for (int q = 0; q < 10; ++q) off[q] = (int64_t)L.off[q];
    off[10] = (int64_t)L.off[16];
  }
  if (pads) {
    pads[0] = L.mp;
    pads[1] = L.np;
    pads[2] = L.kp;
    pads[3] = L.M;
  }
  return 11;
}

int ozaki2_set_stream(void *stream) {
  g_ts.stream = (hipStream_t)stream;
  return OZ2_SUCCESS;
}

int ozaki2_set_workspace(void *ptr, size_t bytes) {
  if (ptr && ((uintptr_t)ptr & 255u)) return -1;
  g_ts.user_ws = ptr;
  g_ts.user_ws_bytes = ptr ? bytes : 0;
  return OZ2_SUCCESS;
}

int ozaki2_set_timing(int on) {
  g_ts.timing = on != 0;
  return OZ2_SUCCESS;
}

int ozaki2_release(void) {
  ThreadState &ts = g_ts;
  if (ts.own_ws) {
    (void)hipFree(ts.own_ws);
    ts.own_ws = nullptr;
    ts.own_ws_bytes = 0;
  }
  if (ts.ev_ready) {
    for (int q = 0; q < kEvents; ++q) (void)hipEventDestroy(ts.ev[q]);
    ts.ev_ready = false;
  }
  ts.have_times = false;
  return OZ2_SUCCESS;
}

int ozaki2_get_kernel_times(float *ms, int count) {
  ThreadState &ts = g_ts;
  if (!ts.have_times || !ts.ev_ready) return -OZ2_ERR_UNSUPPORTED;
  if (hipEventSynchronize(ts.ev[kEvents - 1]) != hipSuccess) return -OZ2_ERR_HIP;
  int w = 0;
  for (int q = 0; q + 1 < kEvents && w < count; ++q, ++w) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, ts.ev[q], ts.ev[q + 1]) != hipSuccess) return -OZ2_ERR_HIP;
    ms[w] = t;
  }
  return w;
}

int ozaki2_get_stage_times(float ms[5]) {
  float k[6];
  int r = ozaki2_get_kernel_times(k, 6);
  if (r < 0) return -r;
  ms[0] = k[0] + k[3];  // quant
  ms[1] = k[1] + k[4];  // gemms
  ms[2] = 0.0f;         // requant: fused into the residue products
  ms[3] = k[5];         // dequant
  ms[4] = k[2];         // others
  return OZ2_SUCCESS;
}

int ozaki2_dgemm(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
                 const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                 double *C, int64_t ldc, int num_moduli) {
  // ---- argument checks (BLAS order) ----
  if (!valid_trans(transA)) return -1;
  if (!valid_trans(transB)) return -2;
  if (m < 0) return -3;
  if (n < 0) return -4;
  if (k < 0) return -5;
  const bool tA = !(transA == 'N' || transA == 'n');
  const bool tB = !(transB == 'N' || transB == 'n');
  const int64_t rowsA = tA ? k : m;
  const int64_t rowsB = tB ? n : k;
  if (lda < (rowsA > 1 ? rowsA : 1)) return -8;
  if (ldb < (rowsB > 1 ? rowsB : 1)) return -10;
  if (ldc < (m > 1 ? m : 1)) return -13;
  if (num_moduli < 1 || num_moduli > OZ2_MAX_MODULI) return -14;

  ThreadState &ts = g_ts;
  hipStream_t st = ts.stream;
  if (m == 0 || n == 0) return OZ2_SUCCESS;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZ2_ERR_NO_DEVICE;
  if (!device_ok(dev)) return OZ2_ERR_NO_DEVICE;
  if (k == 0 || alpha == 0.0)
    return launch_scal(m, n, beta, C, ldc, st) == hipSuccess ? OZ2_SUCCESS : OZ2_ERR_HIP;
  if (k > OZ2_MAX_K) return OZ2_ERR_UNSUPPORTED;

  Layout L;
  if (!make_layout(m, n, k, num_moduli, &L)) return OZ2_ERR_UNSUPPORTED;
  hipError_t herr = hipSuccess;
  const Tables *dt = device_tables(dev, num_moduli, &herr);
  if (!dt) return OZ2_ERR_HIP;
  const Tables *ht = host_tables(num_moduli);

  // ---- workspace ----
  uint8_t *ws = nullptr;
  if (ts.user_ws) {
    if (ts.user_ws_bytes < L.total) return OZ2_ERR_WORKSPACE;
    ws = (uint8_t *)ts.user_ws;
  } else {
    if (ts.own_ws && (ts.own_ws_bytes < L.total || ts.own_dev != dev)) {
      (void)hipFree(ts.own_ws);
      ts.own_ws = nullptr;
      ts.own_ws_bytes = 0;
    }
    if (!ts.own_ws) {
      if (hipMalloc(&ts.own_ws, L.total) != hipSuccess) {
        ts.own_ws = nullptr;
        (void)hipGetLastError();
        return OZ2_ERR_ALLOC;
      }
      ts.own_ws_bytes = L.total;
      ts.own_dev = dev;
    }
    ws = (uint8_t *)ts.own_ws;
  }

  Geometry g{m, n, k, L.mp, L.np, L.kp, num_moduli, L.M};
  Work w;
  w.amax = (uint64_t *)(ws + L.off[10]);
  w.flags = (uint32_t *)(ws + L.off[11]);
  w.rmax = (uint32_t *)(ws + L.off[12]);
  w.rfix = (uint64_t *)(ws + L.off[13]);
  w.amb = (uint32_t *)(ws + L.off[14]);
  w.shift = (int32_t *)(ws + L.off[0]);
  w.E = (int32_t *)(ws + L.off[1]);
  w.e = (int32_t *)(ws + L.off[2]);
  w.Abar = ws + L.off[3];
  w.Bbar = ws + L.off[4];
  w.Asl = ws + L.off[5];
  w.Bsl = ws + L.off[6];
  w.planes = (int16_t *)(ws + L.off[7]);

  Operand opA, opB;
  opA.ptr = A;
  opA.lines = m;
  opA.k = k;
  opA.sr = tA ? lda : 1;
  opA.sh = tA ? 1 : lda;
  opB.ptr = B;
  opB.lines = n;
  opB.k = k;
  opB.sr = tB ? 1 : ldb;
  opB.sh = tB ? ldb : 1;

  const bool timed = ts.timing;
  if (timed) {
    int r = ensure_events(dev);
    if (r != OZ2_SUCCESS) return r;
  }
  int evn = 0;
  auto mark = [&]() {
    if (timed) (void)hipEventRecord(ts.ev[evn++], st);
  };

#define OZ2_TRY(expr)                       \
  do {                                      \
    if ((expr) != hipSuccess) {             \
      ts.have_times = false;                \
      return OZ2_ERR_HIP;                   \
    }                                       \
  } while (0)

  mark();
  // workflow step 1: mu', nu' and the FP8 bound operands
  OZ2_TRY(launch_fill_u32((uint32_t *)(ws + L.off[10]), 0u,
                          (int64_t)((L.off[15] - L.off[10]) / 4), st));
  OZ2_TRY(launch_line_max(opA, w.amax, w.flags, st));
  OZ2_TRY(launch_line_max(opB, w.amax + L.mp, w.flags + L.mp, st));
  OZ2_TRY(launch_bound_operand(opA, L.mp, L.kp, w.amax, w.E, w.flags, w.Abar, st));
  OZ2_TRY(launch_bound_operand(opB, L.np, L.kp, w.amax + L.mp, w.E + L.mp, w.flags + L.mp,
                               w.Bbar, st));
  mark();
  // workflow step 2: the FP8 bound product (its line maxima only)
  OZ2_TRY(launch_bound_gemm(g, w.Abar, w.Bbar, w.rmax, w.rmax + L.mp, st));
  mark();
  // workflow step 3: scale exponents mu, nu
  OZ2_TRY(launch_scale(g, dt, w, st));
  mark();
  // workflow steps 4-6: integers, residues and FP8 digits
  OZ2_TRY(launch_residues(opA, L.mp, L.kp, w.shift, dt, num_moduli, w.Asl, st));
  OZ2_TRY(launch_residues(opB, L.np, L.kp, w.shift + L.mp, dt, num_moduli, w.Bsl, st));
  mark();
  // workflow steps 7-8: residue products and their reduction modulo p
  OZ2_TRY(launch_residue_gemm(g, dt, w.Asl, w.Bsl, w.planes, st));
  mark();
  // workflow steps 9-10: CRT and inverse scaling
  OZ2_TRY(launch_crt(g, dt, w, alpha, beta, C, ldc, ht->limbs, st));
  mark();
#undef OZ2_TRY
  ts.have_times = timed;
  return OZ2_SUCCESS;
}

}  // extern "C"
