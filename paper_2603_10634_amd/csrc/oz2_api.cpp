// C ABI: argument checking, workspace management, per-device tables, the
// launch sequence of one emulated DGEMM (the workflow of Section IV-B), and
// the same sequence over a batch of problems as one grouped launch per
// kernel family, optionally captured in a hipGraph and with an autotuned
// residue-product schedule.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "oz2_internal.h"

using namespace oz2;

namespace {

constexpr int kEvents = 7;

struct Plan;

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
  bool graph = false;                      // capture launch sequences in hipGraphs
  bool autotune = false;                   // tune the grouped residue-product schedule
  int last_schedule = -1;                  // configuration of the last batched call
  int forced = -1;                         // configuration set by ozaki2_set_schedule
  int mode = OZ2_MODE_ACCURATE;            // scaling mode (Section III-E)
  int list = OZ2_MODULI_HYBRID;            // modulus list (Sections III-B, III-D)
  int64_t blk_m = 0, blk_n = 0;            // m/n blocking of ozaki2_dgemm (0: none)
  int split = 0;                           // k parts of ozaki2_dgemm's products (0: the rule)
  hipStream_t cap_stream = nullptr;        // private stream used only for capture
  int cap_dev = -1;
  std::list<std::unique_ptr<Plan>> plans;  // cached plans, most recent first
};

thread_local ThreadState g_ts;

std::mutex g_mu;
std::map<std::tuple<int, int, int>, Tables *> g_tables;  // (device, N, list) -> device copy
std::map<int, bool> g_is_gfx950;
std::map<std::pair<int, int>, Tables> g_host_tables;     // (N, list) -> host copy

// Schedules of the grouped residue products chosen by the autotuner, keyed
// by the shapes of a batch (not its pointers).
std::map<std::vector<int64_t>, int> g_tuned;

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Fault injection for tests of the error paths: with OZ2_FAULT=alloc in the
// environment (read once per process) every device or pinned allocation the
// library would make fails as if the runtime had refused it.
bool fault_alloc() {
  static const bool on = [] {
    const char *f = getenv("OZ2_FAULT");
    return f && strcmp(f, "alloc") == 0;
  }();
  return on;
}

// Split-K in batched calls: a problem with at most kSplitTiles output tiles
// of 256 x 256 per modulus and at least two 256-blocks of k may have its
// residue products split into up to kMaxParts k parts, each written to its
// own copy of the residue planes (the CRT sums them); its batched workspace
// holds kMaxParts copies.
constexpr int kMaxParts = 4;
constexpr int64_t kSplitTiles = 4;

int parts_alloc(int64_t m, int64_t n, int64_t k) {
  const int64_t tiles = (round_up(m, kPad) / kPad) * (round_up(n, kPad) / kPad);
  return tiles <= kSplitTiles && round_up(k, kPad) >= 2 * kPad ? kMaxParts : 1;
}

// Split-K in single calls: each modulus kind's residue products are one
// launch of T tiles x n moduli workgroups (T tiles of 256 x 256 outputs in a
// block), one per CU at a time.  When T n is small against the CU count the
// launch leaves CUs idle for its whole k loop, so k is split into parts that
// run as workgroups of their own, each into its own copy of the planes (the
// CRT sums the copies).  Every part is at most kChunkK long (one exact FP32
// accumulation), so there are at least ceil(kp / kChunkK) parts; above that
// the number minimises the launches' waves of workgroups per unit of k,
// sum over kinds of ceil(T n_kind parts / kCUs) / parts (ties to fewer
// parts), with at least kMinPartK of k in every added part and at most
// kMaxSplit parts (kMaxSplit kChunkK = OZ2_MAX_K).  A fixed CU count keeps
// the workspace size a function of the shape alone.
constexpr int kMaxSplit = 8;
constexpr int64_t kMinPartK = 2048;
constexpr int64_t kCUs = 256;
static_assert((int64_t)kMaxSplit * kChunkK >= OZ2_MAX_K, "parts cannot cover k");

// (k above OZ2_MAX_K is refused before any launch; its workspace size is
// given for kMaxSplit parts)
int min_parts(int64_t kp) {
  return (int)std::min<int64_t>(kMaxSplit, (kp + kChunkK - 1) / kChunkK);
}

int single_parts(int64_t mbp, int64_t nbp, int64_t kp, const Tables &t) {
  const int64_t tiles = (mbp / kGemmTIW) * (nbp / kGemmTJ);
  const int64_t kinds[3] = {t.nsq, t.nka, t.N - t.nsq - t.nka};
  const int lo = min_parts(kp);
  int best = lo;
  double best_cost = 0.0;
  for (int parts = lo; parts <= kMaxSplit && (parts == lo || kp / parts >= kMinPartK); ++parts) {
    double cost = 0.0;
    for (int64_t n : kinds)
      if (n > 0) cost += (double)((tiles * n * parts + kCUs - 1) / kCUs) / parts;
    if (parts == lo || cost < best_cost) {
      best = parts;
      best_cost = cost;
    }
  }
  return best;
}

// Split-K of a single call's bound product (accurate mode): its launch has
// one workgroup per 256 x 256 tile, so an output of few tiles leaves most CUs
// idle through the whole k loop.  With fewer than kCUs / 2 tiles and at
// least 2 kBoundPartK of k, k is cut into up to kMaxBoundSplit parts of at
// least kBoundPartK, enough to give about one workgroup per CU; each part's
// FP32 sums go to a buffer, and one more launch adds them in part order and
// takes the line maxima.  The decision window counts the parts - 1 extra
// additions.  The buffer (4 mp np bytes per part) lies over the residue
// planes, which are written only later in the call.
constexpr int kMaxBoundSplit = 16;
constexpr int64_t kBoundPartK = 4096;

int bound_parts(int64_t mp, int64_t np, int64_t kp) {
  const int64_t tiles = (mp / kGemmTIW) * (np / kGemmTJ);
  if (tiles >= kCUs / 2 || kp < 2 * kBoundPartK) return 1;
  const int64_t want = (kCUs + tiles - 1) / tiles;
  return (int)std::min<int64_t>({want, kp / kBoundPartK, kMaxBoundSplit});
}

struct Layout {
  int64_t mp, np, kp;
  int64_t mbp, nbp;  // padded block extents (mp, np when the call is not blocked)
  int M;
  int parts;         // copies of the residue planes (k parts of the products)
  int bparts;        // k parts of the bound product
  size_t off[17];
  size_t total;
};

const Tables *host_tables(int N, int list) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(N, list);
  auto it = g_host_tables.find(key);
  if (it != g_host_tables.end()) return &it->second;
  Tables t;
  if (!build_tables(N, list, &t)) return nullptr;
  return &(g_host_tables[key] = t);
}

// Offsets of every workspace buffer (256-byte aligned) for N moduli of the
// calling thread's list, for blocks of at most mb x nb outputs (0: whole
// extent).  The per-line vectors and the bound operands cover the whole
// problem; digit slices and residue planes cover one block.  The
// zero-initialised per-line vectors come first and contiguously so one fill
// clears them.  The planes region holds `parts` copies (a batched call's
// split-K allocation; 0 takes the single-call rule, single_parts).
bool make_layout(int64_t m, int64_t n, int64_t k, int N, Layout *L, int64_t mb = 0,
                 int64_t nb = 0, int parts = 0) {
  const Tables *ht = host_tables(N, g_ts.list);
  if (!ht) return false;
  const Tables &t = *ht;
  // extents beyond any device memory are refused before they are padded, and
  // every size below is formed with overflow checks: a wrapped size would
  // pass for a small workspace and let the kernels write past it
  constexpr int64_t kMaxExtent = (int64_t)1 << 40;
  if (m > kMaxExtent || n > kMaxExtent || k > kMaxExtent) return false;
  L->mp = round_up(m > 0 ? m : 1, kPad);
  L->np = round_up(n > 0 ? n : 1, kPad);
  L->kp = round_up(k > 0 ? k : 1, kPad);
  L->mbp = mb > 0 && mb < L->mp ? mb : L->mp;
  L->nbp = nb > 0 && nb < L->np ? nb : L->np;
  L->M = t.M;
  L->bparts = 1;
  if (parts <= 0) {
    parts = g_ts.split > 0
                ? std::max(min_parts(L->kp), (int)std::min<int64_t>(g_ts.split, L->kp / kPad))
                : single_parts(L->mbp, L->nbp, L->kp, t);
    L->bparts = bound_parts(L->mp, L->np, L->kp);
  }
  L->parts = parts;
  const int64_t lines = L->mp + L->np;
  size_t o = 0;
  bool ok = true;
  auto size3 = [&](size_t a, size_t b, size_t c) -> size_t {
    size_t ab = 0, abc = 0;
    if (__builtin_mul_overflow(a, b, &ab) || __builtin_mul_overflow(ab, c, &abc)) ok = false;
    return abc;
  };
  auto take = [&](int idx, size_t bytes) {
    L->off[idx] = o;
    const size_t padded = bytes / 256 * 256 + (bytes % 256 ? 256 : 0);
    if (padded < bytes || __builtin_add_overflow(o, padded, &o)) ok = false;
  };
  // zero-initialised group
  take(10, sizeof(uint64_t) * lines);          // amax
  take(11, sizeof(uint32_t) * lines);          // flags
  take(12, sizeof(uint32_t) * lines);          // rmax
  take(13, sizeof(uint64_t) * lines);          // rfix
  take(14, sizeof(uint32_t) * (lines + 2));    // amb
  L->off[15] = o;                              // end of the zeroed group
  take(0, sizeof(int32_t) * lines);            // shift
  take(1, sizeof(int32_t) * lines);            // E
  take(2, sizeof(int32_t) * lines);            // e
  take(3, size3(L->mp, L->kp, 1));             // Abar
  take(4, size3(L->np, L->kp, 1));             // Bbar
  take(5, size3(t.M, L->mbp, L->kp));          // A slices (one block)
  take(6, size3(t.M, L->nbp, L->kp));          // B slices
  // planes (per k part), or the split bound product's part sums
  take(7, std::max(size3(sizeof(int16_t) * N * L->parts, L->mbp, L->nbp),
                   L->bparts > 1 ? size3(sizeof(float) * L->bparts, L->mp, L->np) : 0));
  L->off[8] = L->off[12];
  L->off[9] = L->off[11];
  L->off[16] = L->off[14];
  L->total = o;
  return ok;
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

// Device copy of the tables, created once per (device, N, list) and kept for
// the life of the process.
const Tables *device_tables(int dev, int N, int list, hipError_t *err) {
  const Tables *h = host_tables(N, list);
  if (!h) {
    *err = hipErrorInvalidValue;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dev, N, list);
  auto it = g_tables.find(key);
  if (it != g_tables.end()) return it->second;
  Tables *d = nullptr;
  *err = fault_alloc() ? hipErrorOutOfMemory : hipMalloc((void **)&d, sizeof(Tables));
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

bool is_trans(char c) { return !(c == 'N' || c == 'n'); }

// Problem descriptor of one call whose workspace starts at ws (layout L).
Problem make_problem(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
                     const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                     double *C, int64_t ldc, int N, uint8_t *ws, const Layout &L,
                     const Tables *dt, const Tables *ht) {
  Problem P;
  memset(&P, 0, sizeof(P));
  const bool tA = is_trans(transA), tB = is_trans(transB);
  P.A.ptr = A;
  P.A.lines = m;
  P.A.k = k;
  P.A.sr = tA ? lda : 1;
  P.A.sh = tA ? 1 : lda;
  P.B.ptr = B;
  P.B.lines = n;
  P.B.k = k;
  P.B.sr = tB ? 1 : ldb;
  P.B.sh = tB ? ldb : 1;
  P.g = Geometry{m, n, k, L.mp, L.np, L.kp, N, L.M, ht->nsq, ht->nka, g_ts.list};
  Work &w = P.w;
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
  w.bpart = (float *)(ws + L.off[7]);
  w.zero = (uint32_t *)(ws + L.off[10]);
  w.zero_words = (int64_t)((L.off[15] - L.off[10]) / 4);
  w.lineB = L.mp;
  P.tab = dt;
  P.alpha = alpha;
  P.beta = beta;
  P.C = C;
  P.ldc = ldc;
  P.limbs = ht->limbs;
  P.mode = g_ts.mode;
  P.parts = L.parts;
  P.bparts = P.mode == OZ2_MODE_FAST ? 1 : L.bparts;
  return P;
}

// Timing marks: event q is recorded after kernel group q - 1.
struct Marks {
  ThreadState *ts;
  hipStream_t st;
  bool on;
  int n = 0;
  void operator()() {
    if (on) (void)hipEventRecord(ts->ev[n++], st);
  }
};

#define OZ2_TRY(expr)                 \
  do {                                \
    if ((expr) != hipSuccess) {       \
      (void)hipGetLastError();        \
      return OZ2_ERR_HIP;             \
    }                                 \
  } while (0)

// Workflow steps 1-3 of Section IV-B for one problem: maxima, bound, scale
// exponents.  Fast mode replaces the bound operands, bound product and its
// decision by the exact line norms of the bound operands (Section III-E).
int enqueue_scaling(const Problem &P, hipStream_t st, Marks &mark) {
  const bool fast = P.mode == OZ2_MODE_FAST;
  mark();
  // step 1: mu', nu' and the FP8 bound operands (fast mode: their line norms)
  for (int f : {kFamFill, kFamLmaxA, kFamLmaxB}) OZ2_TRY(launch_quant_family(f, &P, nullptr, st));
  for (int f : {fast ? kFamNormA : kFamBarA, fast ? kFamNormB : kFamBarB})
    OZ2_TRY(launch_quant_family(f, &P, nullptr, st));
  mark();
  // step 2: the FP8 bound product (its line maxima only; none in fast mode)
  if (!fast) {
    OZ2_TRY(launch_gemm_family(kFamBgemm, &P, nullptr, st));
    if (P.bparts > 1) OZ2_TRY(launch_gemm_family(kFamBreduce, &P, nullptr, st));
  }
  mark();
  // step 3: scale exponents mu, nu
  if (!fast)
    for (int f : {kFamDecide, kFamFixup}) OZ2_TRY(launch_scale_family(f, &P, nullptr, st));
  OZ2_TRY(launch_scale_family(kFamFinal, &P, nullptr, st));
  mark();
  return OZ2_SUCCESS;
}

// Workflow steps 4-10 for one problem or block; res_a / res_b select which
// operand's residues are (re)computed.
int enqueue_products(const Problem &P, hipStream_t st, Marks &mark, bool res_a = true,
                     bool res_b = true) {
  // steps 4-6: integers, residues and FP8 digits
  if (res_a) OZ2_TRY(launch_quant_family(kFamResA, &P, nullptr, st));
  if (res_b) OZ2_TRY(launch_quant_family(kFamResB, &P, nullptr, st));
  mark();
  // steps 7-8: residue products and their reduction modulo p (every k part
  // of a kind in one launch)
  for (int f : {kFamGemmSq, kFamGemmKa, kFamGemmI8})
    OZ2_TRY(launch_gemm_family(f, &P, nullptr, st));
  mark();
  // steps 9-10: CRT and inverse scaling
  OZ2_TRY(launch_crt_family(&P, nullptr, P.limbs, P.g.N, st));
  mark();
  return OZ2_SUCCESS;
}

// The launch sequence of one problem (workflow steps 1-10 of Section IV-B).
int enqueue_single(const Problem &P, hipStream_t st, Marks &mark) {
  const int r = enqueue_scaling(P, st, mark);
  return r != OZ2_SUCCESS ? r : enqueue_products(P, st, mark);
}

// Block (i0.., j0..) of mi x nj outputs of problem P: its operand lines, its
// C entries, and the per-line vectors of P at those lines; digit slices and
// planes are the block buffers of P's workspace.
Problem block_problem(const Problem &P, int64_t i0, int64_t j0, int64_t mi, int64_t nj) {
  Problem B = P;
  B.A.ptr += i0 * P.A.sr;
  B.A.lines = mi;
  B.B.ptr += j0 * P.B.sr;
  B.B.lines = nj;
  B.g.m = mi;
  B.g.n = nj;
  B.g.mp = round_up(mi, kPad);
  B.g.np = round_up(nj, kPad);
  B.w.shift += i0;
  B.w.E += i0;
  B.w.e += i0;
  B.w.flags += i0;
  B.w.amax += i0;
  B.w.lineB = P.g.mp + j0 - i0;
  B.C += i0 + j0 * P.ldc;
  return B;
}

// m/n-blocked launch sequence (the blocking the paper recommends for the
// working memory, Section IV-C): the scale exponents of the whole problem
// first, so that every block is bit-identical to the unblocked call, then
// per block of mb x nb outputs the residues, products and CRT.  A's residues
// are computed once per block row; B's once per block column when there is
// a single block row, else again for every block.
int enqueue_blocked(const Problem &P, int64_t mb, int64_t nb, hipStream_t st) {
  Marks none{nullptr, st, false};
  int r = enqueue_scaling(P, st, none);
  if (r != OZ2_SUCCESS) return r;
  const int64_t m = P.g.m, n = P.g.n;
  const int64_t nJ = (n + nb - 1) / nb;
  for (int64_t i0 = 0; i0 < m; i0 += mb)
    for (int64_t j0 = 0; j0 < n; j0 += nb) {
      const Problem B = block_problem(P, i0, j0, std::min(mb, m - i0), std::min(nb, n - j0));
      r = enqueue_products(B, st, none, j0 == 0, i0 == 0 || nJ > 1);
      if (r != OZ2_SUCCESS) return r;
    }
  return OZ2_SUCCESS;
}

// ---- batched calls ----

// Configurations of the batched residue products, chosen by the autotuner:
// the tile program (config / 3: 0 = eight waves of 128 x 64 outputs per
// 256 x 256 tile, two per SIMD; 1 = four waves of 128 x 128, one per SIMD)
// and the split-K limit (config % 3: at most 1, 2 or 4 k parts for the
// problems that parts_alloc allows to split).  Config 0 is the default.
constexpr int kNumConfigs = 6;
int config_waves(int c) { return c / 3 == 0 ? 8 : 4; }
int config_max_parts(int c) { return c % 3 == 0 ? 1 : (c % 3 == 1 ? 2 : 4); }

// Grouped launches of at most this many blocks carry a block -> problem
// table (4 bytes per block) in the plan.
constexpr int64_t kMaxSegTable = (int64_t)1 << 24;

// The persistent launch of the residue products (not a kernel family of the
// single-problem path).
constexpr int kFamPersist = kNumFamilies;

// One grouped launch of a sub-batch.  The descriptor arrays live in the
// plan's device buffer at the given byte offsets; G (or W for the persistent
// products) is filled in once the buffer exists.  The products and the CRT
// exist once per configuration (they differ in the k parts).
struct GLaunch {
  int fam, config;  // config: -1 for the launches every configuration shares
  size_t off_probs, off_order, off_start, off_seg;  // off_seg: 0 when there is no table
  size_t off_items, off_counters;
  int64_t items;
  bool int8;
  Group G;
  WorkList W;
};

// Problems whose workspaces fit together, run as one set of grouped launches.
struct SubBatch {
  std::vector<GLaunch> launches;
  int limbs;
  int N;  // number of moduli (every problem of a batch has the same)
};

// Everything a batched call (or, in graph mode, a single call) needs beyond
// its arguments: device-resident descriptors and block maps, the split into
// sub-batches, the scale-only problems, and the captured graph.  Keyed by the
// exact argument bytes.
struct Plan {
  std::vector<uint8_t> key;
  int dev = -1;
  void *dbuf = nullptr;  // device: problems, orders, block maps
  void *hbuf = nullptr;  // pinned staging copy of dbuf
  size_t bytes = 0;
  bool uploaded = false;
  std::vector<SubBatch> subs;
  struct Scal {
    int64_t m, n;
    double beta;
    double *C;
    int64_t ldc;
  };
  std::vector<Scal> scal;
  std::vector<int64_t> shape_key;  // N, mode, list, then (m, n, k) of each emulated problem
  std::string bucket;              // the shapes' bucket (the autotuner's cache file key)
  int schedule = -1;               // the residue-product configuration
  bool single = false;
  Problem single_problem;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (dbuf) (void)hipFree(dbuf);
    if (hbuf) (void)hipHostFree(hbuf);
  }
};

// ---- the autotuner's cache file ----
//
// Choices are kept per process by exact shapes (g_tuned) and, when the
// environment names a file in OZ2_AUTOTUNE_CACHE, per shape bucket in that
// file across processes.  A bucket is the number of moduli, the mode, the
// list and the histogram of the problems over (log2 of the output tiles per
// modulus, log2 of the 256-blocks of k).  The file is JSON, one entry per
// line:
//   {"oz2_autotune": 1, "entries": [
//   {"key": "...", "config": 3},
//   ...
//   ]}
// A missing file, or one that does not parse line by line in this form or
// holds a configuration out of range, is ignored: every batch then starts
// from the default configuration (or is tuned again when tuning is on, and
// the file is rewritten).
std::map<std::string, int> g_cache;
bool g_cache_loaded = false;

int ilog2_floor(int64_t v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    ++r;
  }
  return r;
}

std::string bucket_key(const std::vector<int64_t> &shape_key) {
  std::map<std::pair<int, int>, int> hist;
  for (size_t q = 3; q + 2 < shape_key.size(); q += 3) {
    const int64_t tiles = (round_up(shape_key[q], kPad) / kPad) *
                          (round_up(shape_key[q + 1], kPad) / kPad);
    const int64_t kb = round_up(shape_key[q + 2], kPad) / kPad;
    ++hist[{ilog2_floor(tiles), ilog2_floor(kb)}];
  }
  std::string key = "n" + std::to_string(shape_key[0]) + "m" + std::to_string(shape_key[1]) +
                    "l" + std::to_string(shape_key[2]) + ":";
  for (const auto &h : hist)
    key += "t" + std::to_string(h.first.first) + "k" + std::to_string(h.first.second) + "x" +
           std::to_string(h.second) + ";";
  return key;
}

const char *cache_path() {
  const char *p = getenv("OZ2_AUTOTUNE_CACHE");
  return p && *p ? p : nullptr;
}

// Reads the cache file once per process (caller holds g_mu).
void cache_load_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char *path = cache_path();
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  std::map<std::string, int> got;
  char line[4096];
  static const char kHead[] = "{\"oz2_autotune\": 1, \"entries\": [";
  bool ok = fgets(line, sizeof(line), f) && strncmp(line, kHead, sizeof(kHead) - 1) == 0;
  bool closed = false;
  while (ok && fgets(line, sizeof(line), f)) {
    if (strncmp(line, "]}", 2) == 0) {
      closed = true;
      break;
    }
    char key[2048];
    int config = -1, used = 0;
    if (sscanf(line, "{\"key\": \"%2047[^\"]\", \"config\": %d}%n", key, &config, &used) != 2 ||
        used == 0 || config < 0 || config >= kNumConfigs) {
      ok = false;
      break;
    }
    got[key] = config;
  }
  fclose(f);
  if (ok && closed) g_cache = got;
}

int cache_lookup(const std::string &bucket) {
  std::lock_guard<std::mutex> lk(g_mu);
  cache_load_locked();
  auto it = g_cache.find(bucket);
  return it == g_cache.end() ? -1 : it->second;
}

// Records a choice and rewrites the file (through a temporary file renamed
// over it, so a reader never sees half a file).
void cache_store(const std::string &bucket, int config) {
  std::lock_guard<std::mutex> lk(g_mu);
  cache_load_locked();
  g_cache[bucket] = config;
  const char *path = cache_path();
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\"oz2_autotune\": 1, \"entries\": [\n");
  size_t i = 0;
  for (const auto &e : g_cache)
    fprintf(f, "{\"key\": \"%s\", \"config\": %d}%s\n", e.first.c_str(), e.second,
            ++i < g_cache.size() ? "," : "");
  fprintf(f, "]}\n");
  const bool good = fclose(f) == 0;
  if (good) (void)rename(tmp.c_str(), path);
}

struct KeyBuilder {
  std::vector<uint8_t> b;
  template <class T>
  void add(const T &v) {
    const uint8_t *p = (const uint8_t *)&v;
    b.insert(b.end(), p, p + sizeof(T));
  }
};

Plan *find_plan(const std::vector<uint8_t> &key) {
  ThreadState &ts = g_ts;
  for (auto it = ts.plans.begin(); it != ts.plans.end(); ++it) {
    if ((*it)->key == key) {
      ts.plans.splice(ts.plans.begin(), ts.plans, it);  // most recent first
      return ts.plans.front().get();
    }
  }
  return nullptr;
}

Plan *add_plan(std::unique_ptr<Plan> p) {
  ThreadState &ts = g_ts;
  constexpr size_t kMaxPlans = 8;
  if (ts.plans.size() >= kMaxPlans) {
    // a plan being evicted may still be referenced by queued work
    (void)hipStreamSynchronize(ts.stream);
    ts.plans.pop_back();
  }
  ts.plans.push_front(std::move(p));
  return ts.plans.front().get();
}

int capture_stream(int dev, hipStream_t *out) {
  ThreadState &ts = g_ts;
  if (ts.cap_stream && ts.cap_dev != dev) {
    (void)hipStreamDestroy(ts.cap_stream);
    ts.cap_stream = nullptr;
  }
  if (!ts.cap_stream) {
    if (hipStreamCreateWithFlags(&ts.cap_stream, hipStreamNonBlocking) != hipSuccess) {
      ts.cap_stream = nullptr;
      return OZ2_ERR_HIP;
    }
    ts.cap_dev = dev;
  }
  *out = ts.cap_stream;
  return OZ2_SUCCESS;
}

// Runs `enqueue` on st, or (graph mode) replays the plan's graph, capturing
// it first on the private stream if the plan has none yet.
template <class F>
int run_maybe_graph(Plan *plan, int dev, hipStream_t st, F enqueue) {
  if (!plan) return enqueue(st);
  if (!plan->exec) {
    hipStream_t cs;
    int r = capture_stream(dev, &cs);
    if (r != OZ2_SUCCESS) return r;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return OZ2_ERR_HIP;
    }
    const int er = enqueue(cs);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    if (er != OZ2_SUCCESS || ee != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return er != OZ2_SUCCESS ? er : OZ2_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return OZ2_ERR_HIP;
    }
    plan->graph = graph;
    plan->exec = exec;
  }
  OZ2_TRY(hipGraphLaunch(plan->exec, st));
  return OZ2_SUCCESS;
}

// Host image of a plan's device buffer (256-byte aligned pieces).
struct ImageWriter {
  std::vector<uint8_t> img;
  size_t put(const void *src, size_t bytes) {
    const size_t at = (img.size() + 255) / 256 * 256;
    img.resize(at + bytes);
    memcpy(img.data() + at, src, bytes);
    return at;
  }
};

// The grouped launches of one sub-batch: every family over all its problems,
// and per configuration the persistent residue products (one work list over
// every problem, modulus, tile and k part, longest item first) and the CRT
// (over descriptors that carry the configuration's k parts).
void build_subbatch(const std::vector<Problem> &probs, ImageWriter &W, SubBatch *sb) {
  const int np = (int)probs.size();
  const size_t at_probs = W.put(probs.data(), sizeof(Problem) * np);
  std::vector<int32_t> nat(np);
  for (int q = 0; q < np; ++q) nat[q] = q;
  const size_t at_nat = W.put(nat.data(), sizeof(int32_t) * np);
  auto add = [&](int fam, size_t off_probs, int config) {
    std::vector<int64_t> start(np + 1, 0);
    for (int q = 0; q < np; ++q) start[q + 1] = start[q] + family_blocks(fam, probs[q]);
    if (start[np] == 0) return;
    GLaunch L;
    memset(&L, 0, sizeof(L));
    L.fam = fam;
    L.config = config;
    L.off_probs = off_probs;
    L.off_order = at_nat;
    L.off_start = W.put(start.data(), sizeof(int64_t) * (np + 1));
    if (start[np] <= kMaxSegTable) {
      // block -> problem, so that no block searches the prefix sums
      std::vector<int32_t> seg((size_t)start[np]);
      for (int q = 0; q < np; ++q)
        std::fill(seg.begin() + start[q], seg.begin() + start[q + 1], q);
      L.off_seg = W.put(seg.data(), sizeof(int32_t) * seg.size());
    }
    L.G.tab = probs[0].tab;
    L.G.nseg = np;
    L.G.total = start[np];
    sb->launches.push_back(L);
  };
  // every problem of a batch has the calling thread's mode
  if (probs[0].mode == OZ2_MODE_FAST) {
    for (int f : {kFamFill, kFamLmaxA, kFamLmaxB, kFamNormA, kFamNormB, kFamFinal, kFamResA,
                  kFamResB})
      add(f, at_probs, -1);
  } else {
    for (int f : {kFamFill, kFamLmaxA, kFamLmaxB, kFamBarA, kFamBarB, kFamBgemm, kFamDecide,
                  kFamFixup, kFamFinal, kFamResA, kFamResB})
      add(f, at_probs, -1);
  }
  const uint32_t zero2[2] = {0u, 0u};
  const size_t at_counters = W.put(zero2, sizeof(zero2));
  for (int c = 0; c < kNumConfigs; ++c) {
    std::vector<Problem> pc(probs);
    std::vector<ProductItem> items;
    for (int q = 0; q < np; ++q) {
      const Geometry &g = pc[q].g;
      const int64_t nb = g.kp / kPad;  // 256-blocks of k
      int parts = 1;
      if (parts_alloc(g.m, g.n, g.k) > 1) parts = (int)std::min<int64_t>(config_max_parts(c), nb);
      pc[q].parts = parts;
      for (int l = 0; l < g.N; ++l)
        for (int64_t ty = 0; ty < g.np / kGemmTJ; ++ty)
          for (int64_t tx = 0; tx < g.mp / kGemmTIW; ++tx)
            for (int part = 0; part < parts; ++part) {
              ProductItem it;
              it.prob = q;
              it.l = (int16_t)l;
              it.part = (int16_t)part;
              it.tx = (int32_t)tx;
              it.ty = (int32_t)ty;
              int64_t k0, k1;
              part_range(g.kp, parts, part, &k0, &k1);
              it.k0 = (int32_t)k0;
              it.k1 = (int32_t)k1;
              items.push_back(it);
            }
    }
    // longest first (every item costs in proportion to its k extent)
    std::stable_sort(items.begin(), items.end(), [](const ProductItem &a, const ProductItem &b) {
      return a.k1 - a.k0 > b.k1 - b.k0;
    });
    const size_t at_pc = W.put(pc.data(), sizeof(Problem) * np);
    if (!items.empty()) {
      GLaunch L;
      memset(&L, 0, sizeof(L));
      L.fam = kFamPersist;
      L.config = c;
      L.off_probs = at_pc;
      L.off_items = W.put(items.data(), sizeof(ProductItem) * items.size());
      L.off_counters = at_counters;
      L.items = (int64_t)items.size();
      L.int8 = probs[0].g.list == OZ2_MODULI_INT8;
      sb->launches.push_back(L);
    }
    add(kFamCrt, at_pc, c);
  }
}

// Kernel group of a family, as reported by ozaki2_get_kernel_times.
int family_group(int fam) {
  switch (fam) {
    case kFamBgemm: case kFamBreduce: return 1;
    case kFamDecide: case kFamFixup: case kFamFinal: return 2;
    case kFamResA: case kFamResB: return 3;
    case kFamGemmSq: case kFamGemmKa: case kFamGemmI8: case kFamPersist: return 4;
    case kFamCrt: return 5;
    default: return 0;
  }
}

// Enqueues the kernel groups g0..g1 (numbered as in ozaki2_get_kernel_times)
// of sub-batch sb with residue-product configuration `config`.  Marks are
// placed at every group boundary when the whole sequence runs.  With `ev`
// non-null, ev[0] and ev[1] bracket the residue products (group 4).
int enqueue_subbatch(const SubBatch &sb, int config, int cus, hipStream_t st, Marks &mark,
                     hipEvent_t *ev, int g0 = 0, int g1 = 5) {
  int group = -1;
  auto advance = [&](int to) -> int {
    while (group < to) {
      if (group == 3 && ev) OZ2_TRY(hipEventRecord(ev[0], st));
      if (group == 4 && ev) OZ2_TRY(hipEventRecord(ev[1], st));
      mark();
      ++group;
    }
    return OZ2_SUCCESS;
  };
  for (const GLaunch &L : sb.launches) {
    if (L.config >= 0 && L.config != config) continue;
    const int gq = family_group(L.fam);
    if (gq < g0 || gq > g1) continue;
    if (advance(gq) != OZ2_SUCCESS) return OZ2_ERR_HIP;
    if (L.fam == kFamPersist)
      OZ2_TRY(launch_gemm_persistent(config_waves(config), L.int8, L.W, cus, st));
    else if (L.fam == kFamBgemm)
      OZ2_TRY(launch_gemm_family(L.fam, nullptr, &L.G, st));
    else if (L.fam == kFamDecide || L.fam == kFamFixup || L.fam == kFamFinal)
      OZ2_TRY(launch_scale_family(L.fam, nullptr, &L.G, st));
    else if (L.fam == kFamCrt)
      OZ2_TRY(launch_crt_family(nullptr, &L.G, sb.limbs, sb.N, st));
    else
      OZ2_TRY(launch_quant_family(L.fam, nullptr, &L.G, st));
  }
  return advance(g1 + 1);
}

// Argument checks of ozaki2_dgemm in BLAS order: 0, or -i for argument i.
int check_args(char transA, char transB, int64_t m, int64_t n, int64_t k, int64_t lda,
               int64_t ldb, int64_t ldc, int num_moduli) {
  if (!valid_trans(transA)) return -1;
  if (!valid_trans(transB)) return -2;
  if (m < 0) return -3;
  if (n < 0) return -4;
  if (k < 0) return -5;
  const int64_t rowsA = is_trans(transA) ? k : m;
  const int64_t rowsB = is_trans(transB) ? n : k;
  if (lda < (rowsA > 1 ? rowsA : 1)) return -8;
  if (ldb < (rowsB > 1 ? rowsB : 1)) return -10;
  if (ldc < (m > 1 ? m : 1)) return -13;
  if (num_moduli < 1 || num_moduli > OZ2_MAX_MODULI) return -14;
  return 0;
}

}  // namespace

namespace oz2 {

int dgemm_fixed(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
                const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                double *C, int64_t ldc, int num_moduli, FixedResources (*resources)(int dev)) {
  const int bad = check_args(transA, transB, m, n, k, lda, ldb, ldc, num_moduli);
  if (bad) return bad;
  ThreadState &ts = g_ts;
  hipStream_t st = ts.stream;
  ts.have_times = false;
  if (m == 0 || n == 0) return OZ2_SUCCESS;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZ2_ERR_NO_DEVICE;
  if (!device_ok(dev)) return OZ2_ERR_NO_DEVICE;
  if (k == 0 || alpha == 0.0)
    return launch_scal(m, n, beta, C, ldc, st) == hipSuccess ? OZ2_SUCCESS : OZ2_ERR_HIP;
  if (k > OZ2_MAX_K) return OZ2_ERR_UNSUPPORTED;
  Layout L;
  if (!make_layout(m, n, k, num_moduli, &L, ts.blk_m, ts.blk_n)) return OZ2_ERR_UNSUPPORTED;
  const Tables *ht = host_tables(num_moduli, ts.list);
  if (!ht) return OZ2_ERR_UNSUPPORTED;
  const FixedResources res = resources(dev);
  if (!res.ws || !res.tables) return OZ2_ERR_HIP;
  if (L.total > res.ws_bytes) return OZ2_ERR_SCRATCH;
  const Tables *dt = res.tables + (size_t)ts.list * kMaxN + (num_moduli - 1);
  const Problem P = make_problem(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                                 num_moduli, res.ws, L, dt, ht);
  if (L.mbp < L.mp || L.nbp < L.np) return enqueue_blocked(P, L.mbp, L.nbp, st);
  Marks none{&ts, st, false};
  return enqueue_single(P, st, none);
}

bool host_tables_for(int N, int list, Tables *out) {
  const Tables *t = host_tables(N, list);
  if (!t) return false;
  *out = *t;
  return true;
}

}  // namespace oz2

extern "C" {

const char *ozaki2_status_string(int status) {
  switch (status) {
    case OZ2_SUCCESS: return "success";
    case OZ2_ERR_HIP: return "HIP runtime error";
    case OZ2_ERR_ALLOC: return "workspace allocation failed";
    case OZ2_ERR_WORKSPACE: return "caller workspace too small";
    case OZ2_ERR_UNSUPPORTED: return "unsupported size or state";
    case OZ2_ERR_NO_DEVICE: return "no gfx950 device is current";
    case OZ2_ERR_SCRATCH: return "problem needs more than the no-allocation scratch buffer";
    default: return status < 0 ? "invalid argument" : "unknown status";
  }
}

int ozaki2_moduli(int num_moduli, int32_t *p, int32_t *kinds) {
  const Tables *t = host_tables(num_moduli, g_ts.list);
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
  if (!make_layout(m, n, k, num_moduli, &L, g_ts.blk_m, g_ts.blk_n)) return 0;
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

int ozaki2_workspace_parts(int64_t m, int64_t n, int64_t k, int num_moduli, int *parts,
                           int *bound_parts) {
  if (m < 0 || n < 0 || k < 0 || num_moduli < 1 || num_moduli > OZ2_MAX_MODULI) return -1;
  Layout L;
  if (!make_layout(m, n, k, num_moduli, &L, g_ts.blk_m, g_ts.blk_n)) return -1;
  if (parts) *parts = L.parts;
  if (bound_parts) *bound_parts = L.bparts;
  return 0;
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
  if (!ts.plans.empty()) {
    (void)hipDeviceSynchronize();
    ts.plans.clear();
  }
  if (ts.cap_stream) {
    (void)hipStreamDestroy(ts.cap_stream);
    ts.cap_stream = nullptr;
  }
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

// Workspace of the calling thread for `need` bytes (the caller's if set).
static int get_workspace(int dev, size_t need, uint8_t **ws, size_t *have) {
  ThreadState &ts = g_ts;
  if (ts.user_ws) {
    *ws = (uint8_t *)ts.user_ws;
    *have = ts.user_ws_bytes;
    return ts.user_ws_bytes < need ? OZ2_ERR_WORKSPACE : OZ2_SUCCESS;
  }
  if (ts.own_ws && (ts.own_ws_bytes < need || ts.own_dev != dev)) {
    // plans captured over the old workspace must not be replayed
    (void)hipDeviceSynchronize();
    ts.plans.clear();
    (void)hipFree(ts.own_ws);
    ts.own_ws = nullptr;
    ts.own_ws_bytes = 0;
  }
  if (!ts.own_ws) {
    if (fault_alloc() || hipMalloc(&ts.own_ws, need) != hipSuccess) {
      ts.own_ws = nullptr;
      (void)hipGetLastError();
      return OZ2_ERR_ALLOC;
    }
    ts.own_ws_bytes = need;
    ts.own_dev = dev;
  }
  *ws = (uint8_t *)ts.own_ws;
  *have = ts.own_ws_bytes;
  return OZ2_SUCCESS;
}

int ozaki2_dgemm(char transA, char transB, int64_t m, int64_t n, int64_t k, double alpha,
                 const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                 double *C, int64_t ldc, int num_moduli) {
  const int bad = check_args(transA, transB, m, n, k, lda, ldb, ldc, num_moduli);
  if (bad) return bad;

  ThreadState &ts = g_ts;
  hipStream_t st = ts.stream;
  if (m == 0 || n == 0) return OZ2_SUCCESS;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZ2_ERR_NO_DEVICE;
  if (!device_ok(dev)) return OZ2_ERR_NO_DEVICE;
  ts.have_times = false;
  if (k == 0 || alpha == 0.0)
    return launch_scal(m, n, beta, C, ldc, st) == hipSuccess ? OZ2_SUCCESS : OZ2_ERR_HIP;
  if (k > OZ2_MAX_K) return OZ2_ERR_UNSUPPORTED;

  Layout L;
  if (!make_layout(m, n, k, num_moduli, &L, ts.blk_m, ts.blk_n)) return OZ2_ERR_UNSUPPORTED;
  hipError_t herr = hipSuccess;
  const Tables *dt = device_tables(dev, num_moduli, ts.list, &herr);
  if (!dt) return herr == hipErrorOutOfMemory ? OZ2_ERR_ALLOC : OZ2_ERR_HIP;
  const Tables *ht = host_tables(num_moduli, ts.list);

  uint8_t *ws = nullptr;
  size_t have = 0;
  int r = get_workspace(dev, L.total, &ws, &have);
  if (r != OZ2_SUCCESS) return r;
  const Problem P = make_problem(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                                 num_moduli, ws, L, dt, ht);
  const bool blocked = L.mbp < L.mp || L.nbp < L.np;
  const int64_t mb = L.mbp, nb = L.nbp;

  if (ts.graph) {
    KeyBuilder kb;
    kb.add(dev);
    kb.add(P);
    kb.add(mb);
    kb.add(nb);
    Plan *plan = find_plan(kb.b);
    if (!plan) {
      std::unique_ptr<Plan> p(new Plan);
      p->key = kb.b;
      p->dev = dev;
      p->single = true;
      p->single_problem = P;
      plan = add_plan(std::move(p));
    }
    return run_maybe_graph(plan, dev, st, [&](hipStream_t s) {
      if (blocked) return enqueue_blocked(plan->single_problem, mb, nb, s);
      Marks none{&ts, s, false};
      return enqueue_single(plan->single_problem, s, none);
    });
  }
  if (blocked) return enqueue_blocked(P, mb, nb, st);  // not timed
  const bool timed = ts.timing;
  if (timed) {
    r = ensure_events(dev);
    if (r != OZ2_SUCCESS) return r;
  }
  Marks mark{&ts, st, timed};
  r = enqueue_single(P, st, mark);
  ts.have_times = timed && r == OZ2_SUCCESS;
  return r;
}

// Per-problem argument checks of a batched call; returns 0 or -(argument).
static int check_batch(int count, const char *transA, const char *transB, const int64_t *m,
                       const int64_t *n, const int64_t *k, const double *alpha,
                       const double *const *A, const int64_t *lda, const double *const *B,
                       const int64_t *ldb, const double *beta, double *const *C,
                       const int64_t *ldc, int num_moduli) {
  if (count < 0) return -1;
  if (count == 0) return num_moduli < 1 || num_moduli > OZ2_MAX_MODULI ? -15 : 0;
  if (!transA) return -2;
  if (!transB) return -3;
  if (!m) return -4;
  if (!n) return -5;
  if (!k) return -6;
  if (!alpha) return -7;
  if (!A) return -8;
  if (!lda) return -9;
  if (!B) return -10;
  if (!ldb) return -11;
  if (!beta) return -12;
  if (!C) return -13;
  if (!ldc) return -14;
  for (int q = 0; q < count; ++q) {
    if (!valid_trans(transA[q])) return -2;
    if (!valid_trans(transB[q])) return -3;
    if (m[q] < 0) return -4;
    if (n[q] < 0) return -5;
    if (k[q] < 0) return -6;
    const int64_t rowsA = is_trans(transA[q]) ? k[q] : m[q];
    const int64_t rowsB = is_trans(transB[q]) ? n[q] : k[q];
    if (lda[q] < (rowsA > 1 ? rowsA : 1)) return -9;
    if (ldb[q] < (rowsB > 1 ? rowsB : 1)) return -11;
    if (ldc[q] < (m[q] > 1 ? m[q] : 1)) return -14;
  }
  if (num_moduli < 1 || num_moduli > OZ2_MAX_MODULI) return -15;
  return 0;
}

static bool emulated(int64_t m, int64_t n, int64_t k, double alpha) {
  return m > 0 && n > 0 && k > 0 && alpha != 0.0;
}

size_t ozaki2_workspace_bytes_batched(int count, const int64_t *m, const int64_t *n,
                                      const int64_t *k, int num_moduli) {
  if (count < 0 || num_moduli < 1 || num_moduli > OZ2_MAX_MODULI) return 0;
  if (count > 0 && (!m || !n || !k)) return 0;
  size_t total = 0;
  for (int q = 0; q < count; ++q) {
    if (m[q] < 0 || n[q] < 0 || k[q] < 0) return 0;
    if (m[q] == 0 || n[q] == 0 || k[q] == 0) continue;
    Layout L;
    if (!make_layout(m[q], n[q], k[q], num_moduli, &L, 0, 0, parts_alloc(m[q], n[q], k[q])))
      return 0;
    if (__builtin_add_overflow(total, L.total, &total)) return 0;
  }
  return total;
}

int ozaki2_dgemm_batched(int count, const char *transA, const char *transB, const int64_t *m,
                         const int64_t *n, const int64_t *k, const double *alpha,
                         const double *const *A, const int64_t *lda, const double *const *B,
                         const int64_t *ldb, const double *beta, double *const *C,
                         const int64_t *ldc, int num_moduli) {
  int r = check_batch(count, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                      num_moduli);
  if (r != 0) return r;
  ThreadState &ts = g_ts;
  ts.have_times = false;
  if (count == 0) return OZ2_SUCCESS;
  bool any = false;
  for (int q = 0; q < count; ++q) {
    if (m[q] > 0 && n[q] > 0) any = true;
    if (emulated(m[q], n[q], k[q], alpha[q]) && k[q] > OZ2_MAX_K) return OZ2_ERR_UNSUPPORTED;
  }
  if (!any) return OZ2_SUCCESS;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OZ2_ERR_NO_DEVICE;
  if (!device_ok(dev)) return OZ2_ERR_NO_DEVICE;
  hipStream_t st = ts.stream;
  hipError_t herr = hipSuccess;
  const Tables *dt = device_tables(dev, num_moduli, ts.list, &herr);
  if (!dt) return herr == hipErrorOutOfMemory ? OZ2_ERR_ALLOC : OZ2_ERR_HIP;
  const Tables *ht = host_tables(num_moduli, ts.list);

  // workspace: library-owned grows to the whole batch, capped at 16 GiB
  // (or the largest single problem); a caller's is used as given
  std::vector<Layout> lays(count);
  size_t total = 0, largest = 0;
  for (int q = 0; q < count; ++q) {
    if (!emulated(m[q], n[q], k[q], alpha[q])) continue;
    if (!make_layout(m[q], n[q], k[q], num_moduli, &lays[q], 0, 0,
                     parts_alloc(m[q], n[q], k[q])))
      return OZ2_ERR_UNSUPPORTED;
    if (__builtin_add_overflow(total, lays[q].total, &total)) total = SIZE_MAX;
    largest = std::max(largest, lays[q].total);
  }
  uint8_t *ws = nullptr;
  size_t have = 0;
  if (total > 0) {
    size_t want = total;
    if (!ts.user_ws) want = std::max(largest, std::min(total, (size_t)16 << 30));
    r = get_workspace(dev, ts.user_ws ? largest : want, &ws, &have);
    if (r != OZ2_SUCCESS) return r;
  }

  KeyBuilder kb;
  kb.add(dev);
  kb.add(ts.mode);
  kb.add(ts.list);
  kb.add(num_moduli);
  kb.add(ts.forced);
  kb.add(count);
  kb.add(ws);
  kb.add(have);
  for (int q = 0; q < count; ++q) {
    kb.add(transA[q]);
    kb.add(transB[q]);
    kb.add(m[q]);
    kb.add(n[q]);
    kb.add(k[q]);
    kb.add(alpha[q]);
    kb.add(A[q]);
    kb.add(lda[q]);
    kb.add(B[q]);
    kb.add(ldb[q]);
    kb.add(beta[q]);
    kb.add(C[q]);
    kb.add(ldc[q]);
  }
  Plan *plan = find_plan(kb.b);
  if (!plan) {
    std::unique_ptr<Plan> p(new Plan);
    p->key = kb.b;
    p->dev = dev;
    ImageWriter W;
    std::vector<Problem> cur;
    size_t used = 0;
    auto flush = [&]() {
      if (cur.empty()) return;
      SubBatch sb;
      sb.limbs = ht->limbs;
      sb.N = num_moduli;
      build_subbatch(cur, W, &sb);
      p->subs.push_back(std::move(sb));
      cur.clear();
      used = 0;
    };
    p->shape_key.push_back(num_moduli);
    p->shape_key.push_back(ts.mode);
    p->shape_key.push_back(ts.list);
    for (int q = 0; q < count; ++q) {
      if (m[q] == 0 || n[q] == 0) continue;
      if (!emulated(m[q], n[q], k[q], alpha[q])) {
        p->scal.push_back(Plan::Scal{m[q], n[q], beta[q], C[q], ldc[q]});
        continue;
      }
      const Layout &L = lays[q];
      if (used + L.total > have) flush();
      cur.push_back(make_problem(transA[q], transB[q], m[q], n[q], k[q], alpha[q], A[q], lda[q],
                                 B[q], ldb[q], beta[q], C[q], ldc[q], num_moduli, ws + used, L,
                                 dt, ht));
      used += L.total;
      for (int64_t v : {m[q], n[q], k[q]}) p->shape_key.push_back(v);
    }
    flush();
    p->bytes = W.img.size();
    if (p->bytes) {
      if (fault_alloc() || hipMalloc(&p->dbuf, p->bytes) != hipSuccess) {
        (void)hipGetLastError();
        return OZ2_ERR_ALLOC;
      }
      if (hipHostMalloc(&p->hbuf, p->bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return OZ2_ERR_ALLOC;
      }
      memcpy(p->hbuf, W.img.data(), p->bytes);
      uint8_t *base = (uint8_t *)p->dbuf;
      for (SubBatch &sb : p->subs)
        for (GLaunch &L : sb.launches) {
          if (L.fam == kFamPersist) {
            L.W.probs = (const Problem *)(base + L.off_probs);
            L.W.items = (const ProductItem *)(base + L.off_items);
            L.W.count = L.items;
            L.W.counters = (uint32_t *)(base + L.off_counters);
            continue;
          }
          L.G.probs = (const Problem *)(base + L.off_probs);
          L.G.order = (const int32_t *)(base + L.off_order);
          L.G.start = (const int64_t *)(base + L.off_start);
          L.G.seg = L.off_seg ? (const int32_t *)(base + L.off_seg) : nullptr;
        }
    }
    p->bucket = bucket_key(p->shape_key);
    {
      std::lock_guard<std::mutex> lk(g_mu);
      auto it = g_tuned.find(p->shape_key);
      if (it != g_tuned.end()) p->schedule = it->second;
    }
    if (p->schedule < 0) p->schedule = cache_lookup(p->bucket);
    plan = add_plan(std::move(p));
  }
  if (!plan->uploaded && plan->bytes) {
    OZ2_TRY(hipMemcpyAsync(plan->dbuf, plan->hbuf, plan->bytes, hipMemcpyHostToDevice, st));
    plan->uploaded = true;
  }
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);

  // autotuner: on the first call of a new batch shape (no choice for its
  // exact shapes in this process, none for its shape bucket in the cache
  // file), run the first sub-batch's residue products under every
  // configuration (tile program x split-K limit; the products are
  // recomputed from the digit slices each time, into plane copies the CRT of
  // the chosen configuration reads, so the result is the same) and keep the
  // fastest
  if (plan->schedule < 0 && ts.autotune && ts.forced < 0 && !plan->subs.empty()) {
    r = ensure_events(dev);
    if (r != OZ2_SUCCESS) return r;
    const SubBatch &sb = plan->subs[0];
    Marks none{&ts, st, false};
    float best = 0.0f;
    int best_c = 0;
    // the stages before the products once, then the products per
    // configuration (the CRT, which reads C when beta != 0, runs only in the
    // real pass)
    r = enqueue_subbatch(sb, 0, cus, st, none, nullptr, 0, 3);
    if (r != OZ2_SUCCESS) return r;
    for (int c = 0; c < kNumConfigs; ++c) {
      r = enqueue_subbatch(sb, c, cus, st, none, ts.ev, 4, 4);
      if (r != OZ2_SUCCESS) return r;
      float t = 0.0f;
      OZ2_TRY(hipEventSynchronize(ts.ev[1]));
      OZ2_TRY(hipEventElapsedTime(&t, ts.ev[0], ts.ev[1]));
      if (c == 0 || t < best) {
        best = t;
        best_c = c;
      }
    }
    plan->schedule = best_c;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      g_tuned[plan->shape_key] = best_c;
    }
    cache_store(plan->bucket, best_c);
  }
  const int sched = ts.forced >= 0 ? ts.forced : (plan->schedule < 0 ? 0 : plan->schedule);
  ts.last_schedule = sched;

  auto enqueue_all = [&](hipStream_t s, bool timed) -> int {
    for (const Plan::Scal &c : plan->scal)
      OZ2_TRY(launch_scal(c.m, c.n, c.beta, c.C, c.ldc, s));
    for (const SubBatch &sb : plan->subs) {
      Marks mark{&ts, s, timed};
      const int e = enqueue_subbatch(sb, sched, cus, s, mark, nullptr);
      if (e != OZ2_SUCCESS) return e;
    }
    return OZ2_SUCCESS;
  };
  if (ts.graph)
    return run_maybe_graph(plan, dev, st, [&](hipStream_t s) { return enqueue_all(s, false); });
  // timing covers batches that run as one sub-batch
  const bool timed = ts.timing && plan->subs.size() == 1;
  if (timed) {
    r = ensure_events(dev);
    if (r != OZ2_SUCCESS) return r;
  }
  r = enqueue_all(st, timed);
  ts.have_times = timed && r == OZ2_SUCCESS;
  return r;
}

int ozaki2_set_graph(int on) {
  g_ts.graph = on != 0;
  return OZ2_SUCCESS;
}

int ozaki2_set_autotune(int on) {
  g_ts.autotune = on != 0;
  return OZ2_SUCCESS;
}

int ozaki2_get_schedule(void) { return g_ts.last_schedule; }

int ozaki2_set_schedule(int config) {
  if (config < -1 || config >= kNumConfigs) return -1;
  g_ts.forced = config;
  return OZ2_SUCCESS;
}

int ozaki2_set_split(int parts) {
  if (parts < 0 || parts > kMaxSplit) return -1;
  g_ts.split = parts;
  return OZ2_SUCCESS;
}

int ozaki2_set_mode(int mode) {
  if (mode != OZ2_MODE_ACCURATE && mode != OZ2_MODE_FAST) return -1;
  g_ts.mode = mode;
  return OZ2_SUCCESS;
}

int ozaki2_get_mode(void) { return g_ts.mode; }

int ozaki2_set_moduli_list(int list) {
  if (list != OZ2_MODULI_HYBRID && list != OZ2_MODULI_KARATSUBA && list != OZ2_MODULI_INT8)
    return -1;
  g_ts.list = list;
  return OZ2_SUCCESS;
}

int ozaki2_get_moduli_list(void) { return g_ts.list; }

int ozaki2_set_blocking(int64_t m_blk, int64_t n_blk) {
  if (m_blk < 0 || m_blk % kPad) return -1;
  if (n_blk < 0 || n_blk % kPad) return -2;
  g_ts.blk_m = m_blk;
  g_ts.blk_n = n_blk;
  return OZ2_SUCCESS;
}

int ozaki2_get_blocking(int64_t *m_blk, int64_t *n_blk) {
  if (m_blk) *m_blk = g_ts.blk_m;
  if (n_blk) *n_blk = g_ts.blk_n;
  return OZ2_SUCCESS;
}

}  // extern "C"
