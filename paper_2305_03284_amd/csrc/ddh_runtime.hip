// Host runtime behind the C ABI in include/ddh.h: per-stream device state,
// the per-frame launch sequence, HIP-graph capture, batches of streams with
// mixed grid sizes, per-kernel event timing and the FP64 diagnostics.
#include "ddh.h"
#include "ddh_internal.h"

#include <algorithm>
#include <array>
#include <unordered_set>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

using namespace ddh;

// Device list of stream-descriptor pointers for ddh_step_batch_noalloc (the
// batched step for callers that cannot allocate): a file-scope device array,
// of which every device that runs the library holds one copy until the
// process ends.  Host code never uses its name as an address: the address on
// each device is taken once, at the first stream creation on that device
// (ensure_scratch), and only that address reaches kernels.
constexpr int kNoAllocMaxStreams = 4096;
static __device__ __align__(256) StreamDesc* scratch[kNoAllocMaxStreams];

namespace {

constexpr int kMaxDev = 64;
constexpr int kDiagParts = 256;

thread_local std::string g_last_err;
std::mutex g_mu;

// Handles currently alive (streams, batches, servers): a handle is checked by
// membership here, never by reading through a pointer that may be freed.
std::mutex g_live_mu;
std::unordered_set<const void*> g_live;
void live_add(const void* h) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  g_live.insert(h);
}
void live_remove(const void* h) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  g_live.erase(h);
}
bool is_live(const void* h) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  return g_live.count(h) != 0;
}
float2* g_tw[kMaxDev] = {nullptr};

std::mutex g_scratch_mu;
StreamDesc** g_scratch[kMaxDev] = {nullptr};
constexpr int FRAME_CHUNK = 64;  // streams per stats launch filled from stack arrays

int hip_fail(hipError_t e, const char* what);

// The device address of `scratch` on device dev (which must be current).
int ensure_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDev) return DDH_EDEVICE;
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<StreamDesc**>(ptr);
  }
  return DDH_OK;
}

StreamDesc** scratch_of(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return dev >= 0 && dev < kMaxDev ? g_scratch[dev] : nullptr;
}

int hip_fail(hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  g_last_err = buf;
  if (e == hipErrorOutOfMemory) return DDH_ENOMEM;
  return DDH_EDEVICE;
}
#define DDH_CHECK(expr)                              \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool valid_N(int N) { return N == 64 || N == 128 || N == 256 || N == 512; }

// check_diameter: the aperture is the circle of p->pupil_diameter (no
// aperture array given)
int validate(const ddh_params* p, bool check_diameter = true) {
  if (!p) return DDH_EINVAL;
  if (!valid_N(p->N)) return DDH_EINVAL;
  auto fin = [](float x) { return std::isfinite(x); };
  if (check_diameter &&
      (!fin(p->pupil_diameter) || !(p->pupil_diameter > 0.f) || p->pupil_diameter > p->N * 1.41421357f))
    return DDH_EINVAL;
  if (!fin(p->lambda) || p->lambda < 0.f || p->lambda > 1.f) return DDH_EINVAL;
  if (!fin(p->alpha) || p->alpha < 0.f || p->alpha > 1.f) return DDH_EINVAL;
  if (p->n_k < 1 || p->n_k > 1024) return DDH_EINVAL;
  if (!fin(p->sigma_w2) || !(p->sigma_w2 > 0.f)) return DDH_EINVAL;
  if (p->qg_p != 2.0f) return DDH_EINVAL;
  if (!fin(p->qg_q) || p->qg_q < 1.f || p->qg_q > 2.f) return DDH_EINVAL;
  if (!fin(p->qg_T) || !(p->qg_T > 0.f)) return DDH_EINVAL;
  if (!fin(p->qg_sigma) || !(p->qg_sigma > 0.f)) return DDH_EINVAL;
  if (!fin(p->beta_phi) || p->beta_phi < 0.f) return DDH_EINVAL;
  if (!fin(p->r_floor) || !(p->r_floor > 0.f)) return DDH_EINVAL;
  return DDH_OK;
}

// exp(-2 pi i m / N) tables for N = 64..512, computed in double.
int ensure_twiddles(int dev, float2** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev < 0 || dev >= kMaxDev) return DDH_EDEVICE;
  if (!g_tw[dev]) {
    std::vector<float2> h(TWIDDLE_TOTAL);
    for (int N : {64, 128, 256, 512}) {
      const int off = twiddle_offset(N);
      for (int m = 0; m < N; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)N;
        h[off + m] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
    }
    float2* d = nullptr;
    DDH_CHECK(hipMalloc(&d, sizeof(float2) * TWIDDLE_TOTAL));
    DDH_CHECK(hipMemcpy(d, h.data(), sizeof(float2) * TWIDDLE_TOTAL, hipMemcpyHostToDevice));
    g_tw[dev] = d;
  }
  *out = g_tw[dev];
  return DDH_OK;
}

// Per-pixel aperture bytes from the binary aperture inside[] (N*N, 0 or 1):
// the aperture-neighbour weight in twelfths (bits 0-3: 2 per edge and 1 per
// diagonal neighbour in the aperture) and the in-aperture flag (bit 4), zero
// off the aperture.  Every kernel reads the aperture through these bytes.
std::vector<unsigned char> geometry_bytes(int N, const std::vector<unsigned char>& inside) {
  std::vector<unsigned char> geo((size_t)N * N, 0);
  auto inp = [&](int i, int j) { return i >= 0 && i < N && j >= 0 && j < N && inside[(size_t)i * N + j] != 0; };
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      if (!inp(i, j)) continue;
      const int n12 = 2 * (inp(i - 1, j) + inp(i + 1, j) + inp(i, j - 1) + inp(i, j + 1)) + inp(i - 1, j - 1) +
                      inp(i - 1, j + 1) + inp(i + 1, j - 1) + inp(i + 1, j + 1);
      geo[(size_t)i * N + j] = (unsigned char)(n12 | 16);
    }
  return geo;
}

// The circular pupil of diameter^2 d2 centred at ((N-1)/2, (N-1)/2): pixel
// (i, j) is inside iff (2i-N+1)^2 + (2j-N+1)^2 <= d2 (integer arithmetic).
std::vector<unsigned char> circle_mask(int N, float d2) {
  std::vector<unsigned char> m((size_t)N * N, 0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const int di = 2 * i - N + 1, dj = 2 * j - N + 1;
      m[(size_t)i * N + j] = (float)(di * di + dj * dj) <= d2 ? 1 : 0;
    }
  return m;
}

// Aperture bytes of a circular pupil: one read-only N x N byte array per
// device and (N, pupil diameter), shared by every stream of that shape and
// kept until the process ends (like the twiddle table).
int ensure_geometry(int dev, int N, float d2, const unsigned char** out) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, uint32_t>, unsigned char*> cache;
  std::lock_guard<std::mutex> lk(mu);
  uint32_t bits = 0;
  memcpy(&bits, &d2, sizeof bits);
  const auto key = std::make_tuple(dev, N, bits);
  const auto it = cache.find(key);
  if (it != cache.end()) {
    *out = it->second;
    return DDH_OK;
  }
  const std::vector<unsigned char> geo = geometry_bytes(N, circle_mask(N, d2));
  unsigned char* d = nullptr;
  DDH_CHECK(hipMalloc(&d, geo.size()));
  hipError_t e = hipMemcpy(d, geo.data(), geo.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "hipMemcpy(geometry)");
  }
  cache[key] = d;
  *out = d;
  return DDH_OK;
}

TileConfig default_tiles(int N) {
  switch (N) {
    case 64: return {32, 32, 32, 32};
    case 128: return {16, 16, 32, 32};
    case 256: return {16, 16, 32, 32};
    default: return {8, 8, 32, 32};
  }
}

std::map<int, TileConfig>& tile_cache() {
  static std::map<int, TileConfig> m;
  return m;
}

bool tiles_ok(int N, const TileConfig& t) {
  const int T = N / (N == 64 ? 8 : 16);
  auto pow2in = [](int v) { return v == 4 || v == 8 || v == 16 || v == 32; };
  if (!pow2in(t.row_lines) || !pow2in(t.col_width)) return false;
  if (t.row_lines * T > 1024 || t.col_width * T > 1024 || N % t.row_lines || N % t.col_width) return false;
  const bool ms = (t.m_tile_h == 0 && t.m_tile_w == 0) ||
                  (t.m_tile_h == 16 && (t.m_tile_w == 16 || t.m_tile_w == 32 || t.m_tile_w == 64)) ||
                  (t.m_tile_h == 32 && (t.m_tile_w == 32 || t.m_tile_w == 64 || t.m_tile_w == 128)) ||
                  (t.m_tile_h == 64 && t.m_tile_w == 64);
  return ms && (t.m_tile_h == 0 || (N % t.m_tile_h == 0 && N % t.m_tile_w == 0));
}

TileConfig tiles_for(int N) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = tile_cache().find(N);
  return it == tile_cache().end() ? default_tiles(N) : it->second;
}

const char* kKindNames[KK_COUNT] = {"stats", "finalize", "row_ifft", "col_fused", "row_fft", "m_step", "begin",
                                    "frame_worklist", "stats_row_ifft"};

// XCDs of a device (queues of the work-list kernel), cached per device.
int xcd_count(int dev) {
  static std::mutex mu;
  static int cache[kMaxDev] = {0};
  std::lock_guard<std::mutex> lk(mu);
  if (dev < 0 || dev >= kMaxDev) return 1;
  if (!cache[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || n < 1) {
      (void)hipGetLastError();
      n = 1;
    }
    cache[dev] = std::min(n, (int)CTL_MAX_QUEUES);
  }
  return cache[dev];
}

}  // namespace

namespace ddh {
int twiddle_offset(int N) {
  switch (N) {
    case 64: return 0;
    case 128: return 64;
    case 256: return 192;
    case 512: return 448;
    default: return -1;
  }
}
}  // namespace ddh

// ------------------------------------------------------------------ stream
struct ddh_stream_s {
  ddh_params prm{};
  int N = 0;
  int device = 0;
  char* mem = nullptr;
  StreamDesc h{};
  StreamDesc* d = nullptr;       // device descriptor
  StreamDesc** dptr = nullptr;   // device array holding d
  double* diag = nullptr;        // device FP64 partials for diagnostics
  float2* tw = nullptr;          // twiddles for this N on this device
  int parity = 0;                // host mirror of d->cur
  long long n = 0;
  hipStream_t cap = nullptr;     // internal stream for graph capture
  hipGraphExec_t gexec = nullptr;
  bool use_graph = false;
};

// ------------------------------------------------------------------ batch
struct Group {
  int N;
  int off;
  int count;
  TileConfig tc;
  const float2* tw;
  unsigned* ctl0 = nullptr;  // work-list control words of the group's launch (its first stream's)
  float share = 1.0f;        // part of the device its work-list launch fills (lanes running at once)
};

// Work-list (persistent frame kernel) settings of a batch.
constexpr unsigned kSpinLimit = 1u << 20;  // polls before a cross-workgroup wait gives up

struct Worklist {
  int nq = 1;                   // XCD queues
  int lag = 2;                  // slots between consecutive stages of a stream
  unsigned spin = kSpinLimit;   // polls before a wait gives up
  int giveup = 0;               // failure-path test: every wait gives up at once
};

// A lane is a subset of a batch's streams whose launch chain runs on its own
// HIP stream, so that the chains of different lanes overlap on the device.
struct Lane {
  std::vector<Group> groups;
  int off = 0, count = 0;
  hipStream_t s = nullptr;
  hipEvent_t join = nullptr;
};

struct ddh_batch_s {
  std::vector<ddh_stream_t> streams;  // input order
  std::vector<int> pos;               // grouped position of input stream i
  std::vector<Group> groups;          // all groups (every lane), for timing mode
  std::vector<Lane> lanes;
  hipEvent_t fork = nullptr;
  StreamDesc** dptrs = nullptr;       // device array, ordered by lane then N
  int total = 0;
  int n_k = 1;
  int flags = 0;
  int device = 0;
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool capturing = false;             // enqueueing into the graph capture (frame start from descriptors)
  bool worklist = false;              // DDH_BATCH_WORKLIST: persistent frame kernel
  bool fuse_stats = true;             // statistics formed in the first row pass (k_row1s)
  Worklist wl;
  std::vector<const float2*> yord;
  std::vector<int> curord;       // host parity of each stream, in descriptor order
  // timing
  bool timing = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  double acc_ms[KK_COUNT] = {0};
  long long acc_n[KK_COUNT] = {0};
};

// Continuous-batching server: a device list of descriptor pointers, filled per
// call by the stats kernel from its arguments.
struct ddh_server_s {
  int device = 0;
  int max = 0;
  StreamDesc** list = nullptr;  // device, max entries
  bool bound = false;           // calls are bound to the first call's HIP stream
  hipStream_t st = nullptr;
  std::vector<int> order;
  std::vector<const float2*> ys;
  std::vector<int> curs;
  std::vector<StreamDesc*> ds;
  // one internal HIP stream per N group of a call, forked from and joined
  // back into the caller's stream
  hipStream_t lane[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr, join[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

// Rows per block of the fused statistics + first row pass of `count` streams
// of size N whose row passes use row_lines: 32 for batches of 8 or more
// streams at N >= 256 (half the blocks to wait for and to combine; measured
// 25.5 -> 23.4 us at 64 x N = 256 and 27.6 -> 26.6 us at 16 x N = 512),
// row_lines otherwise (a single N = 256 stream was 1.4 us slower with 32).
// The environment variable DDH_FUSED_LINES (4, 8, 16 or 32) overrides.
int fused_lines(int N, int count, int row_lines) {
  static const int env = [] {
    const char* e = getenv("DDH_FUSED_LINES");
    const int x = e ? atoi(e) : 0;
    return (x == 4 || x == 8 || x == 16 || x == 32) ? x : 0;
  }();
  if (env) return env;
  return (N >= 256 && count >= 8) ? 32 : row_lines;
}

// Whether a frame of `lanes` concurrently running lanes forms its statistics
// in the first row pass: with one lane, or when the frame is replayed as a
// HIP graph (measured on the 2:5:1 mixed-size batch: eager launches 376k
// EM iters/s with the separate statistics launch against 370k fused, graph
// replay 383k-385k against 388k fused); DDH_FUSED_STATS=0/1 overrides.
bool fused_stats_for(int lanes, bool graph) {
  static const int env = [] {
    const char* v = getenv("DDH_FUSED_STATS");
    return v && (v[0] == '0' || v[0] == '1') ? v[0] - '0' : -1;
  }();
  return env >= 0 ? env == 1 : (lanes <= 1 || graph);
}

// The EM iterations of one frame (everything after the statistics) for
// `ngroups` groups of streams whose descriptor pointers sit at
// dptrs[g.off, g.off + g.count); `around` wraps every launch (timing).
// first_row1_done: the k = 0 row pass has run (fused with the statistics).
template <class OnLaunch>
int enqueue_iters(StreamDesc** dptrs, const Group* groups, int ngroups, int n_k, int mode, hipStream_t st,
                  OnLaunch&& around, bool first_row1_done = false) {
  hipError_t e;
  const int iters = mode ? n_k : 1;
  for (int k = 0; k < iters; ++k) {
    const int first = (mode && k == 0) ? 1 : 0;
    for (int q = 0; q < ngroups && !(k == 0 && first_row1_done); ++q) {
      const Group& g = groups[q];
      e = around(KK_ROW1,
                 [&] { return launch_row1(dptrs + g.off, g.count, g.N, g.tw, k, first, k == 0, mode, g.tc, st); });
      if (e != hipSuccess) return hip_fail(e, "launch_row1");
    }
    for (int q = 0; q < ngroups; ++q) {
      const Group& g = groups[q];
      e = around(KK_COL, [&] { return launch_col(dptrs + g.off, g.count, g.N, g.tw, k, first, g.tc, st); });
      if (e != hipSuccess) return hip_fail(e, "launch_col");
    }
    for (int q = 0; q < ngroups; ++q) {
      const Group& g = groups[q];
      e = around(KK_ROW2, [&] { return launch_row2(dptrs + g.off, g.count, g.N, g.tw, k, first, g.tc, st); });
      if (e != hipSuccess) return hip_fail(e, "launch_row2");
    }
    for (int q = 0; q < ngroups; ++q) {
      const Group& g = groups[q];
      e = around(KK_MSTEP, [&] { return launch_mstep(dptrs + g.off, g.count, g.N, k, first, first, g.tc, st); });
      if (e != hipSuccess) return hip_fail(e, "launch_mstep");
    }
  }
  return DDH_OK;
}

// Enqueue one frame (mode 1: DDH frame with prologue; mode 0: plain EM) for
// the streams in `dptrs` (grouped by N).  Frame start from ys/curs/ds
// (nullptr: from the descriptors).  fuse: the statistics are formed in the
// first row pass (k_row1s, one launch per group); otherwise by a statistics
// launch before the k = 0 row pass.  Launches of other lanes that run at the
// same time share the device with k_row1s's waiting blocks, so batches with
// several lanes use the separate launch.
template <class OnLaunch>
int enqueue_frame(StreamDesc** dptrs, const std::vector<Group>& groups, int total, int n_k, int mode,
                  hipStream_t st, OnLaunch&& around, const float2* const* ys = nullptr, const int* curs = nullptr,
                  StreamDesc* const* ds = nullptr, bool fuse = true) {
  hipError_t e;
  (void)total;
  if (!fuse) {
    // the statistics as a launch of their own, then the k = 0 row pass
    for (const Group& g : groups) {
      e = around(KK_STATS, [&] {
        return launch_stats(dptrs + g.off, g.count, g.N, mode, ys ? ys + g.off : nullptr,
                            ys ? curs + g.off : nullptr, ds ? ds + g.off : nullptr, st);
      });
      if (e != hipSuccess) return hip_fail(e, "launch_stats");
    }
    return enqueue_iters(dptrs, groups.data(), (int)groups.size(), n_k, mode, st, around);
  }
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const int nq = xcd_count(dev);
  // the statistics and the first row pass as one launch per group
  for (const Group& g : groups) {
    TileConfig tc = g.tc;
    tc.row_lines = fused_lines(g.N, g.count, g.tc.row_lines);
    e = around(KK_ROW1S, [&] {
      return launch_row1s(dptrs + g.off, g.count, g.N, g.tw, mode, ys ? ys + g.off : nullptr,
                          ys ? curs + g.off : nullptr, ds ? ds + g.off : nullptr, kSpinLimit, nq, tc, st);
    });
    if (e != hipSuccess) return hip_fail(e, "launch_row1s");
  }
  return enqueue_iters(dptrs, groups.data(), (int)groups.size(), n_k, mode, st, around, true);
}

// One frame on the work-list path: per EM iteration one persistent launch
// per group (stats at k = 0, row1, column and row2 as one work list), then
// the groups' M-steps.  Frame start from ys/curs/ds at k = 0 (nullptr: from
// the descriptors); later iterations read it from the descriptors.
template <class OnLaunch>
int enqueue_frame_worklist(StreamDesc** dptrs, const Group* groups, int ngroups, int n_k, int mode, hipStream_t st,
                           OnLaunch&& around, const Worklist& wl, const float2* const* ys = nullptr,
                           const int* curs = nullptr, StreamDesc* const* ds = nullptr) {
  hipError_t e;
  const int iters = mode ? n_k : 1;
  for (int k = 0; k < iters; ++k) {
    const int first = (mode && k == 0) ? 1 : 0;
    for (int q = 0; q < ngroups; ++q) {
      const Group& g = groups[q];
      const bool args = k == 0 && ys != nullptr;
      e = around(KK_FRAME, [&] {
        return launch_frame(dptrs + g.off, g.count, g.N, g.tw, k, mode, args ? ys + g.off : nullptr,
                            args ? curs + g.off : nullptr, args && ds ? ds + g.off : nullptr, g.ctl0, wl.nq, wl.lag,
                            wl.spin, wl.giveup, g.tc.m_tile_h == 0, g.share, st);
      });
      if (e != hipSuccess) return hip_fail(e, "launch_frame");
    }
    for (int q = 0; q < ngroups; ++q) {
      const Group& g = groups[q];
      e = around(KK_MSTEP, [&] { return launch_mstep(dptrs + g.off, g.count, g.N, k, first, first, g.tc, st); });
      if (e != hipSuccess) return hip_fail(e, "launch_mstep");
    }
  }
  return DDH_OK;
}

struct NoTiming {
  template <class F>
  hipError_t operator()(int, F&& f) const { return f(); }
};

int check_stream(ddh_stream_t s) {
  if (!s) return DDH_EINVAL;
  if (!is_live(s)) return DDH_ESTATE;
  return DDH_OK;
}

int set_device_of(int dev) {
  int cur = -1;
  DDH_CHECK(hipGetDevice(&cur));
  if (cur != dev) DDH_CHECK(hipSetDevice(dev));
  return DDH_OK;
}

int single_step(ddh_stream_t s, const void* y, hipStream_t st, int mode) {
  const float2* yp = static_cast<const float2*>(y);
  const int iters = mode ? s->prm.n_k : 1;
  std::vector<Group> g{{s->N, 0, 1, tiles_for(s->N), s->tw, s->h.ctl}};
  if (mode && s->use_graph) {
    // the replayed graph reads the frame start from the descriptor
    hipError_t e = launch_begin(s->dptr, &yp, &s->parity, 1, st);
    if (e != hipSuccess) return hip_fail(e, "launch_begin");
    if (!s->gexec) {
      hipGraph_t graph = nullptr;
      DDH_CHECK(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
      int rc = enqueue_frame(s->dptr, g, 1, s->prm.n_k, 1, s->cap, NoTiming{});
      hipError_t ec = hipStreamEndCapture(s->cap, &graph);
      if (rc != DDH_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
      ec = hipGraphInstantiate(&s->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ec != hipSuccess) {
        s->gexec = nullptr;
        return hip_fail(ec, "hipGraphInstantiate");
      }
    }
    DDH_CHECK(hipGraphLaunch(s->gexec, st));
  } else {
    int rc = enqueue_frame(s->dptr, g, 1, s->prm.n_k, mode, st, NoTiming{}, &yp, &s->parity);
    if (rc != DDH_OK) return rc;
  }
  s->parity = (s->parity + iters) & 1;
  if (mode) s->n++;
  return DDH_OK;
}

}  // namespace

extern "C" {

const char* ddh_version(void) { return "ddh-mi355x 0.1 (gfx950)"; }

const char* ddh_error_string(int code) {
  switch (code) {
    case DDH_OK: return "ok";
    case DDH_EINVAL: return "invalid argument";
    case DDH_ENOMEM: return "out of device memory";
    case DDH_EDEVICE: return "HIP runtime error";
    case DDH_EDATA: return "frame rejected: Normalize undefined (zero or non-finite ||y - mean||)";
    case DDH_ESTATE: return "invalid handle state";
    default: return "unknown error";
  }
}

const char* ddh_last_error_message(void) { return g_last_err.c_str(); }

int ddh_default_params(int N, ddh_params* p) {
  if (!p || !valid_N(N)) return DDH_EINVAL;
  p->N = N;
  p->pupil_diameter = (float)N;
  p->lambda = 0.45f;
  p->alpha = 0.025f;
  p->n_k = 1;
  p->sigma_w2 = 0.1f;
  p->qg_p = 2.0f;
  p->qg_q = 1.2f;
  p->qg_T = 0.1f;
  p->qg_sigma = 0.2f;
  p->beta_phi = 0.5f;
  p->r_floor = 1e-8f;
  return DDH_OK;
}

// Device allocation of one stream (one hipMalloc): offsets of its buffers.
struct StreamLayout {
  size_t r0, r1, p0, p1, T, U, bb, part, scal, ctl, desc, dptr, diag, geo, total;
  explicit StreamLayout(int N) {
    const size_t px = (size_t)N * N;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      size_t o = off;
      off = align256(off + bytes);
      return o;
    };
    r0 = take(px * 4);
    r1 = take(px * 4);
    p0 = take(px * 4);
    p1 = take(px * 4);
    T = take(px * 8);
    U = take(px * 8);
    bb = take(px * 4);
    part = take((size_t)N * PART_STRIDE * 4);  // one statistics record per grid row
    scal = take(SC_COUNT * 4);
    ctl = take(CTL_WORDS * 4);  // zeroed with the scratch at creation
    desc = take(sizeof(StreamDesc));
    dptr = take(sizeof(StreamDesc*));
    diag = take(kDiagParts * 3 * sizeof(double) + 64);
    geo = take(px);  // aperture bytes of a stream created with an aperture array
    total = off;
  }
};

int ddh_stream_bytes(int N, unsigned long long* bytes) {
  if (!bytes || !valid_N(N)) return DDH_EINVAL;
  *bytes = StreamLayout(N).total;
  return DDH_OK;
}

// Host copy of an aperture array (host or device memory), validated: every
// value 0 or 1, at least one 1.
static int read_aperture(const float* a, int N, std::vector<unsigned char>* mask) {
  const size_t n = (size_t)N * N;
  std::vector<float> h(n);
  hipPointerAttribute_t at{};
  bool on_device = false;
  if (hipPointerGetAttributes(&at, a) == hipSuccess)
    on_device = at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
  else
    (void)hipGetLastError();  // plain host memory is not known to HIP: not an error here
  if (on_device)
    DDH_CHECK(hipMemcpy(h.data(), a, n * sizeof(float), hipMemcpyDeviceToHost));
  else
    memcpy(h.data(), a, n * sizeof(float));
  mask->assign(n, 0);
  size_t inside = 0;
  for (size_t k = 0; k < n; ++k) {
    if (h[k] == 1.0f) {
      (*mask)[k] = 1;
      ++inside;
    } else if (h[k] != 0.0f) {  // also NaN
      return DDH_EINVAL;
    }
  }
  return inside ? DDH_OK : DDH_EINVAL;
}

// Plane-fit moments over the aperture (exact sums over integer coordinates,
// in double): n, sum di, sum dj, sum di^2, sum di dj, sum dj^2 with
// di = i - c, dj = j - c, c = (N-1)/2, and the inverse of the symmetric
// normal matrix; returns false (inverse left zero) when it is singular.
static bool aperture_moments(int N, const std::vector<unsigned char>& inside, double* mom, double* minv) {
  double m[6] = {0, 0, 0, 0, 0, 0};
  const double c = 0.5 * (N - 1);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      if (!inside[(size_t)i * N + j]) continue;
      const double a = i - c, b = j - c;
      m[0] += 1;
      m[1] += a;
      m[2] += b;
      m[3] += a * a;
      m[4] += a * b;
      m[5] += b * b;
    }
  memcpy(mom, m, sizeof m);
  // symmetric inverse by cofactors (the plane fit's normal equations)
  const double a00 = m[0], a01 = m[1], a02 = m[2], a11 = m[3], a12 = m[4], a22 = m[5];
  const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
  const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
  const double det = a00 * c00 + a01 * c01 + a02 * c02;
  const double inv[6] = {c00 / det, c01 / det, c02 / det, c11 / det, c12 / det, c22 / det};
  for (int q = 0; q < 6; ++q) minv[q] = det != 0.0 ? inv[q] : 0.0;
  return det != 0.0;
}

int ddh_init_stream(const ddh_params* p, const float* aperture, void* hip_stream, ddh_stream_t* out) {
  if (!out) return DDH_EINVAL;
  int rc = validate(p, aperture == nullptr);
  if (rc != DDH_OK) return rc;
  const int N = p->N;
  const float d2 = p->pupil_diameter * p->pupil_diameter;
  // the aperture: the caller's array (validated before any device work) or
  // the circle of the given diameter
  std::vector<unsigned char> inside;
  if (aperture) {
    rc = read_aperture(aperture, N, &inside);
    if (rc != DDH_OK) return rc;
  } else {
    inside = circle_mask(N, d2);
  }
  double mom[6], minv[6];
  // an aperture array must fix the plane of RemoveTipTilt (three pixels not on one line)
  if (!aperture_moments(N, inside, mom, minv) && aperture) return DDH_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  DDH_CHECK(hipGetDevice(&dev));
  float2* tw_all = nullptr;
  rc = ensure_twiddles(dev, &tw_all);
  if (rc != DDH_OK) return rc;
  rc = ensure_scratch(dev);
  if (rc != DDH_OK) return rc;
  const unsigned char* geo = nullptr;
  if (!aperture) {
    rc = ensure_geometry(dev, N, d2, &geo);
    if (rc != DDH_OK) return rc;
  }
  const StreamLayout lay(N);
  const size_t o_r0 = lay.r0, o_r1 = lay.r1, o_p0 = lay.p0, o_p1 = lay.p1, o_T = lay.T, o_U = lay.U, o_bb = lay.bb;
  const size_t o_part = lay.part, o_scal = lay.scal, o_desc = lay.desc, o_dptr = lay.dptr, o_diag = lay.diag;
  char* mem = nullptr;
  hipError_t e = hipMalloc(&mem, lay.total);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(stream)");
  if (aperture) {
    // the stream's own aperture bytes
    const std::vector<unsigned char> g = geometry_bytes(N, inside);
    e = hipMemcpy(mem + lay.geo, g.data(), g.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(mem);
      return hip_fail(e, "hipMemcpy(aperture)");
    }
    geo = (const unsigned char*)(mem + lay.geo);
  }
  ddh_stream_t s = new ddh_stream_s();
  s->prm = *p;
  s->N = N;
  s->device = dev;
  s->mem = mem;
  s->tw = tw_all + twiddle_offset(N);
  StreamDesc& h = s->h;
  h.y = nullptr;
  h.r[0] = (float*)(mem + o_r0);
  h.r[1] = (float*)(mem + o_r1);
  h.phi[0] = (float*)(mem + o_p0);
  h.phi[1] = (float*)(mem + o_p1);
  h.T = (float2*)(mem + o_T);
  h.U = (float2*)(mem + o_U);
  h.bb = (float*)(mem + o_bb);
  h.part = (float*)(mem + o_part);
  h.scal = (float*)(mem + o_scal);
  h.ctl = (unsigned*)(mem + lay.ctl);
  h.geo = geo;
  h.N = N;
  h.cur = 0;
  h.sigma2 = p->sigma_w2;
  h.lam = p->lambda;
  h.alpha = p->alpha;
  h.beta = p->beta_phi;
  h.r_floor = p->r_floor;
  h.qg_p = p->qg_p;
  h.qg_q = p->qg_q;
  h.qg_T = p->qg_T;
  h.qg_sigma = p->qg_sigma;
  h.qg_inv_sp = (float)(1.0 / ((double)p->qg_sigma * (double)p->qg_sigma));
  h.qg_inv_Ts = (float)(1.0 / ((double)p->qg_T * (double)p->qg_sigma));
  h.qg_pmq = p->qg_p - p->qg_q;
  h.qg_lc = (float)(((double)p->qg_p - (double)p->qg_q) * std::log2(1.0 / ((double)p->qg_T * (double)p->qg_sigma)));
  h.qg_qop = p->qg_q / p->qg_p;
  h.qg_pm2 = p->qg_p - 2.0f;
  if (!(h.qg_pmq > 0.0f)) {
    // q = p: the edge weight does not depend on d.  The kernels evaluate
    // v = 2^(pmq log2|d| + lc) without a branch for d = 0, so v is made 0 for
    // every d instead of 1 (a positive pmq far too small to move lc, and lc
    // below the exponent range): the shape is then 1 instead of 1/2, and the
    // prior scale is halved to match (bit for bit: both are powers of two)
    h.qg_pmq = 1e-30f;
    h.qg_lc = -256.0f;
    h.qg_inv_sp *= 0.5f;
  }
  memcpy(h.mom, mom, sizeof mom);
  memcpy(h.minv, minv, sizeof minv);
  s->d = (StreamDesc*)(mem + o_desc);
  s->dptr = (StreamDesc**)(mem + o_dptr);
  s->diag = (double*)(mem + o_diag);
  auto fail = [&](int code) {
    (void)hipFree(mem);
    delete s;
    return code;
  };
  e = hipMemcpy(s->d, &h, sizeof(StreamDesc), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpy(desc)"));
  StreamDesc* dv = s->d;
  e = hipMemcpy(s->dptr, &dv, sizeof(StreamDesc*), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpy(dptr)"));
  // r <- 0, phi <- 0 (Fig. 1) on the caller's stream; scratch zeroed too
  e = launch_fill_zero((float*)mem, (long long)(o_T / 4), st);
  if (e != hipSuccess) return fail(hip_fail(e, "fill_zero"));
  e = launch_fill_zero((float*)(mem + o_part), (long long)((o_desc - o_part) / 4), st);
  if (e != hipSuccess) return fail(hip_fail(e, "fill_zero"));
  e = hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return fail(hip_fail(e, "hipStreamCreate"));
  const char* g = getenv("DDH_SINGLE_GRAPH");
  s->use_graph = (g && g[0] == '1');
  live_add(s);
  *out = s;
  return DDH_OK;
}

int ddh_destroy_stream(ddh_stream_t s) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  live_remove(s);
  set_device_of(s->device);
  (void)hipDeviceSynchronize();
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->cap) (void)hipStreamDestroy(s->cap);
  (void)hipFree(s->mem);
  delete s;
  return DDH_OK;
}

int ddh_get_params(ddh_stream_t s, ddh_params* out) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!out) return DDH_EINVAL;
  *out = s->prm;
  return DDH_OK;
}

int ddh_frame_count(ddh_stream_t s, long long* n) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!n) return DDH_EINVAL;
  *n = s->n;
  return DDH_OK;
}

int ddh_step(ddh_stream_t s, const void* y, void* hip_stream) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!y) return DDH_EINVAL;
  return single_step(s, y, static_cast<hipStream_t>(hip_stream), 1);
}

int ddh_em(ddh_stream_t s, const void* y, void* hip_stream) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!y) return DDH_EINVAL;
  return single_step(s, y, static_cast<hipStream_t>(hip_stream), 0);
}

int ddh_mbir(ddh_stream_t s, const void* y, int iters, int reset_every, void* hip_stream) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!y || iters < 0 || reset_every < 1) return DDH_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const float2* yp = static_cast<const float2*>(y);
  std::vector<Group> g{{s->N, 0, 1, tiles_for(s->N), s->tw, s->h.ctl}};
  for (int it = 0; it < iters; ++it) {
    // a reset is the frame prologue with Eq. (3) and one EM iteration; the
    // other iterations are plain EM
    const int mode = it % reset_every == 0 ? 1 : 0;
    rc = enqueue_frame(s->dptr, g, 1, 1, mode, st, NoTiming{}, &yp, &s->parity);
    if (rc != DDH_OK) return rc;
    s->parity ^= 1;
  }
  if (iters > 0) s->n++;
  return DDH_OK;
}

static int copy_state(ddh_stream_t s, float* out, bool phase, hipStream_t st) {
  const float* src = phase ? s->h.phi[s->parity] : s->h.r[s->parity];
  DDH_CHECK(hipMemcpyAsync(out, src, sizeof(float) * (size_t)s->N * s->N, hipMemcpyDeviceToDevice, st));
  return DDH_OK;
}

int ddh_get_phase(ddh_stream_t s, float* out, void* hip_stream) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!out) return DDH_EINVAL;
  return copy_state(s, out, true, static_cast<hipStream_t>(hip_stream));
}

int ddh_get_reflectance(ddh_stream_t s, float* out, void* hip_stream) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!out) return DDH_EINVAL;
  return copy_state(s, out, false, static_cast<hipStream_t>(hip_stream));
}

int ddh_set_state(ddh_stream_t s, const float* r, const float* phi, long long n, void* hip_stream) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!r || !phi || n < 0) return DDH_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t bytes = sizeof(float) * (size_t)s->N * s->N;
  DDH_CHECK(hipMemcpyAsync(s->h.r[s->parity], r, bytes, hipMemcpyDeviceToDevice, st));
  DDH_CHECK(launch_copy_pupil(s->h.phi[s->parity], phi, s->N, s->h.geo, st));
  DDH_CHECK(launch_fill_zero(reinterpret_cast<float*>(s->h.ctl), CTL_WORDS, st));  // work-list words
  s->n = n;
  return DDH_OK;
}

int ddh_status(ddh_stream_t s, void* hip_stream) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  float flag = 0.f;
  unsigned gave_up = 0;
  DDH_CHECK(hipMemcpyAsync(&flag, s->h.scal + SC_FLAG, sizeof(float), hipMemcpyDeviceToHost, st));
  DDH_CHECK(hipMemcpyAsync(&gave_up, s->h.ctl + CTL_GIVEUP, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  DDH_CHECK(hipStreamSynchronize(st));
  if (gave_up) {
    // reported once.  After a give-up an item of an earlier stage can finish
    // after its stream's counters were reset, so all the stream's work-list
    // words are cleared (every launch on st has ended by now)
    DDH_CHECK(launch_fill_zero(reinterpret_cast<float*>(s->h.ctl), CTL_WORDS, st));
    DDH_CHECK(hipStreamSynchronize(st));
    g_last_err = "a wait of the work-list frame kernel gave up; the stream's state is unspecified";
    return DDH_EDEVICE;
  }
  return flag != 0.f ? DDH_EDATA : DDH_OK;
}

// ------------------------------------------------------------ diagnostics
int ddh_cost(ddh_stream_t s, const void* y, double* U, void* hip_stream) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!y || !U) return DDH_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const float2* yp = static_cast<const float2*>(y);
  hipError_t e = launch_stats(s->dptr, 1, s->N, 0, &yp, &s->parity, nullptr, st);
  if (e != hipSuccess) return hip_fail(e, "stats");
  e = launch_finalize(s->dptr, 1, s->N, 0, st);
  if (e != hipSuccess) return hip_fail(e, "finalize");
  // b into U, work in T (both are scratch between frames)
  e = launch_backproject_cur(s->d, s->N, s->parity, s->tw, s->h.U, s->h.T, st);
  if (e != hipSuccess) return hip_fail(e, "backproject");
  e = launch_cost_terms(s->d, s->parity, s->h.U, s->diag, kDiagParts, st);
  if (e != hipSuccess) return hip_fail(e, "cost_terms");
  std::vector<double> part(kDiagParts);
  float flag = 0.f;
  DDH_CHECK(hipMemcpyAsync(part.data(), s->diag, sizeof(double) * kDiagParts, hipMemcpyDeviceToHost, st));
  DDH_CHECK(hipMemcpyAsync(&flag, s->h.scal + SC_FLAG, sizeof(float), hipMemcpyDeviceToHost, st));
  DDH_CHECK(hipStreamSynchronize(st));
  if (flag != 0.f) return DDH_EDATA;
  double acc = 0.0;
  for (double v : part) acc += v;
  *U = acc;
  return DDH_OK;
}

int ddh_strehl(ddh_stream_t s, const float* phi_true, double* S, void* hip_stream) {
  int rc = check_stream(s);
  if (rc != DDH_OK) return rc;
  if (!phi_true || !S) return DDH_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int N = s->N;
  hipError_t e = launch_strehl_sums(s->d, s->parity, phi_true, s->diag, kDiagParts, st);
  if (e != hipSuccess) return hip_fail(e, "strehl_sums");
  std::vector<double> part(kDiagParts * 3);
  DDH_CHECK(hipMemcpyAsync(part.data(), s->diag, sizeof(double) * kDiagParts * 3, hipMemcpyDeviceToHost, st));
  DDH_CHECK(hipStreamSynchronize(st));
  double rhs[3] = {0, 0, 0};
  for (int b = 0; b < kDiagParts; ++b)
    for (int k = 0; k < 3; ++k) rhs[k] += part[b * 3 + k];
  const double* m = s->h.mom;
  const double a00 = m[0], a01 = m[1], a02 = m[2], a11 = m[3], a12 = m[4], a22 = m[5];
  const double det = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) + a02 * (a01 * a12 - a11 * a02);
  double coef[3] = {0, 0, 0};
  if (det != 0.0) {
    const double s0 = rhs[0], s1 = rhs[1], s2 = rhs[2];
    coef[0] = (s0 * (a11 * a22 - a12 * a12) - a01 * (s1 * a22 - a12 * s2) + a02 * (s1 * a12 - a11 * s2)) / det;
    coef[1] = (a00 * (s1 * a22 - a12 * s2) - s0 * (a01 * a22 - a12 * a02) + a02 * (a01 * s2 - s1 * a02)) / det;
    coef[2] = (a00 * (a11 * s2 - s1 * a12) - a01 * (a01 * s2 - s1 * a02) + s0 * (a01 * a12 - a11 * a02)) / det;
  }
  double* dcoef = s->diag + kDiagParts * 3;
  DDH_CHECK(hipMemcpyAsync(dcoef, coef, sizeof coef, hipMemcpyHostToDevice, st));
  double peak[2];
  for (int pass = 0; pass < 2; ++pass) {
    e = launch_strehl_field(s->d, N, s->parity, pass == 0 ? phi_true : nullptr, dcoef, s->h.U, st);
    if (e != hipSuccess) return hip_fail(e, "strehl_field");
    e = launch_fft2(N, 1, s->h.U, s->h.U, s->h.T, s->tw, 1, st);
    if (e != hipSuccess) return hip_fail(e, "fft2");
    e = launch_max_abs2(s->h.U, N * N, s->diag, kDiagParts, st);
    if (e != hipSuccess) return hip_fail(e, "max_abs2");
    std::vector<double> mx(kDiagParts);
    DDH_CHECK(hipMemcpyAsync(mx.data(), s->diag, sizeof(double) * kDiagParts, hipMemcpyDeviceToHost, st));
    DDH_CHECK(hipStreamSynchronize(st));
    peak[pass] = *std::max_element(mx.begin(), mx.end());
  }
  *S = peak[0] / peak[1];
  return DDH_OK;
}

// ----------------------------------------------------------------- batches
// Batch creation; `over` (may be null) gives the tilings to use instead of
// the process-wide ones (the autotuners time candidates this way without
// installing them).
static int batch_create_impl(const ddh_stream_t* streams, int count, int flags,
                             const std::map<int, TileConfig>* over, ddh_batch_t* out) {
  if (!streams || count <= 0 || !out) return DDH_EINVAL;
  int dev = -1, n_k = -1;
  for (int i = 0; i < count; ++i) {
    int rc = check_stream(streams[i]);
    if (rc != DDH_OK) return rc;
    if (dev < 0) dev = streams[i]->device;
    if (streams[i]->device != dev) return DDH_ESTATE;
    if (n_k < 0) n_k = streams[i]->prm.n_k;
    if (streams[i]->prm.n_k != n_k) return DDH_EINVAL;
    for (int j = 0; j < i; ++j)
      if (streams[j] == streams[i]) return DDH_EINVAL;
  }
  const int nl = (flags >> 8) & 0xff;
  if (nl > 8) return DDH_EINVAL;
  std::vector<int> sizes;  // distinct N, largest first
  for (int i = 0; i < count; ++i)
    if (std::find(sizes.begin(), sizes.end(), streams[i]->N) == sizes.end()) sizes.push_back(streams[i]->N);
  std::sort(sizes.rbegin(), sizes.rend());
  // lane count 0: one lane per distinct N (a uniform batch has one lane)
  const bool by_n = nl == 0;
  const int nlanes = by_n ? (int)sizes.size() : std::min(nl, std::min(count, 8));
  ddh_batch_t b = new ddh_batch_s();
  b->streams.assign(streams, streams + count);
  b->total = count;
  b->n_k = n_k;
  b->flags = flags;
  b->device = dev;
  b->pos.assign(count, -1);
  // assign streams to lanes: largest grids first, each to the lane with the
  // fewest pixels so far (ties to the lowest lane)
  std::vector<int> idx(count);
  for (int i = 0; i < count; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return streams[a]->N > streams[c]->N; });
  std::vector<long long> load(nlanes, 0);
  std::vector<std::vector<int>> members(nlanes);
  for (int i : idx) {
    const int l = by_n ? (int)(std::find(sizes.begin(), sizes.end(), streams[i]->N) - sizes.begin())
                       : (int)(std::min_element(load.begin(), load.end()) - load.begin());
    members[l].push_back(i);
    load[l] += (long long)streams[i]->N * streams[i]->N;
  }
  std::vector<StreamDesc*> order;
  b->lanes.resize(nlanes);
  for (int l = 0; l < nlanes; ++l) {
    Lane& ln = b->lanes[l];
    ln.off = (int)order.size();
    for (int N : {64, 128, 256, 512}) {
      TileConfig tc = tiles_for(N);
      if (over && over->count(N)) tc = over->at(N);
      Group g{N, (int)order.size(), 0, tc, nullptr};
      for (int i : members[l]) {
        if (streams[i]->N != N) continue;
        if (g.count == 0) g.ctl0 = streams[i]->h.ctl;
        b->pos[i] = (int)order.size();
        order.push_back(streams[i]->d);
        g.count++;
        g.tw = streams[i]->tw;
      }
      if (g.count) {
        b->groups.push_back(g);  // the timed path runs every group alone
        // lanes run at once: each work-list launch fills its lane's part of the device
        long long all = 0;
        for (long long v : load) all += v;
        if (nlanes > 1 && all > 0) g.share = std::max(0.05f, (float)((double)load[l] / (double)all));
        ln.groups.push_back(g);
      }
    }
    ln.count = (int)order.size() - ln.off;
  }
  b->yord.assign(count, nullptr);
  b->curord.assign(count, 0);
  b->worklist = (flags & DDH_BATCH_WORKLIST) != 0;
  b->wl.nq = xcd_count(dev);
  b->wl.giveup = (flags & DDH_BATCH_TEST_GIVEUP) ? 1 : 0;
  if (const char* lag = getenv("DDH_WORKLIST_LAG")) b->wl.lag = std::max(1, std::min(64, atoi(lag)));
  b->fuse_stats = fused_stats_for(nlanes, (flags & DDH_BATCH_GRAPH) != 0);
  hipError_t e = hipMalloc(&b->dptrs, sizeof(StreamDesc*) * count);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipMalloc(batch)");
  }
  e = hipMemcpy(b->dptrs, order.data(), sizeof(StreamDesc*) * count, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess && nlanes > 1) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int l = 0; l < nlanes && nlanes > 1 && e == hipSuccess; ++l) {
    e = hipStreamCreateWithFlags(&b->lanes[l].s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->lanes[l].join, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    for (Lane& ln : b->lanes) {
      if (ln.s) (void)hipStreamDestroy(ln.s);
      if (ln.join) (void)hipEventDestroy(ln.join);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    (void)hipFree(b->dptrs);
    delete b;
    return hip_fail(e, "batch setup");
  }
  live_add(b);
  *out = b;
  return DDH_OK;
}

int ddh_batch_create(const ddh_stream_t* streams, int count, int flags, ddh_batch_t* out) {
  return batch_create_impl(streams, count, flags, nullptr, out);
}

// Release a batch; with device_sync == false only the batch's own HIP
// streams are waited for (the caller has synchronised the stream it stepped
// the batch on), so other work on the device is not stalled.
static int batch_release(ddh_batch_t b, bool device_sync) {
  if (!b) return DDH_EINVAL;
  if (!is_live(b)) return DDH_ESTATE;
  live_remove(b);
  set_device_of(b->device);
  if (device_sync) {
    (void)hipDeviceSynchronize();
  } else {
    for (Lane& ln : b->lanes)
      if (ln.s) (void)hipStreamSynchronize(ln.s);
    if (b->cap) (void)hipStreamSynchronize(b->cap);
  }
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (Lane& ln : b->lanes) {
    if (ln.s) (void)hipStreamDestroy(ln.s);
    if (ln.join) (void)hipEventDestroy(ln.join);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipEvent_t ev : b->pool) (void)hipEventDestroy(ev);
  (void)hipFree(b->dptrs);
  delete b;
  return DDH_OK;
}

int ddh_batch_destroy(ddh_batch_t b) { return batch_release(b, true); }

int ddh_batch_set_timing(ddh_batch_t b, int enable) {
  if (!b) return DDH_EINVAL;
  if (!is_live(b)) return DDH_ESTATE;
  b->timing = enable != 0;
  for (int k = 0; k < KK_COUNT; ++k) {
    b->acc_ms[k] = 0;
    b->acc_n[k] = 0;
  }
  b->recs.clear();
  b->pool_used = 0;
  return DDH_OK;
}

// Timing-only events: without the system-scope fence at each record, which
// would write back and invalidate the L2 between the timed kernels and make
// each kernel start with cold caches (its inputs were just written by the
// previous kernel).
static hipError_t timing_event(hipEvent_t* ev) { return hipEventCreateWithFlags(ev, hipEventDisableSystemFence); }

static hipEvent_t pool_event(ddh_batch_t b) {
  if (b->pool_used == b->pool.size()) {
    hipEvent_t ev;
    if (timing_event(&ev) != hipSuccess) return nullptr;
    b->pool.push_back(ev);
  }
  return b->pool[b->pool_used++];
}

static int drain_timing(ddh_batch_t b) {
  for (auto& r : b->recs) {
    DDH_CHECK(hipEventSynchronize(r.b));
    float ms = 0.f;
    DDH_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
    b->acc_ms[r.kind] += ms;
    b->acc_n[r.kind] += 1;
  }
  b->recs.clear();
  b->pool_used = 0;
  return DDH_OK;
}

// Fork the lanes off stream st, enqueue each lane's chain on its own stream,
// join them back into st (capturable: the graph then has parallel branches).
extern "C++" {
template <class OnLaunch>
static int batch_enqueue(ddh_batch_t b, const std::vector<Group>& groups, int count, hipStream_t st, OnLaunch&& around,
                         const float2* const* ys, const int* cs) {
  if (b->worklist)
    return enqueue_frame_worklist(b->dptrs, groups.data(), (int)groups.size(), b->n_k, 1, st, around, b->wl, ys, cs);
  return enqueue_frame(b->dptrs, groups, count, b->n_k, 1, st, around, ys, cs, nullptr, b->fuse_stats);
}
}  // extern "C++"

static int enqueue_lanes(ddh_batch_t b, hipStream_t st) {
  const float2* const* ys = b->capturing ? nullptr : b->yord.data();
  const int* cs = b->curord.data();
  if (b->lanes.size() == 1) return batch_enqueue(b, b->lanes[0].groups, b->lanes[0].count, st, NoTiming{}, ys, cs);
  DDH_CHECK(hipEventRecord(b->fork, st));
  for (Lane& ln : b->lanes) {
    DDH_CHECK(hipStreamWaitEvent(ln.s, b->fork, 0));
    int rc = batch_enqueue(b, ln.groups, ln.count, ln.s, NoTiming{}, ys, cs);
    if (rc != DDH_OK) return rc;
    DDH_CHECK(hipEventRecord(ln.join, ln.s));
  }
  for (Lane& ln : b->lanes) DDH_CHECK(hipStreamWaitEvent(st, ln.join, 0));
  return DDH_OK;
}

int ddh_batch_step(ddh_batch_t b, const void* const* y, void* hip_stream) {
  if (!b || !y) return DDH_EINVAL;
  if (!is_live(b)) return DDH_ESTATE;
  for (int i = 0; i < b->total; ++i) {
    if (!is_live(b->streams[i])) return DDH_ESTATE;
    if (!y[i]) return DDH_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < b->total; ++i) {
    b->yord[b->pos[i]] = static_cast<const float2*>(y[i]);
    b->curord[b->pos[i]] = b->streams[i]->parity;
  }
  if (b->timing && b->recs.size() > 4096) {
    int rc = drain_timing(b);
    if (rc != DDH_OK) return rc;
  }
  auto timed = [&](int kind, auto&& f) -> hipError_t {
    if (!b->timing) return f();
    hipEvent_t a = pool_event(b), c = pool_event(b);
    if (!a || !c) return hipErrorOutOfMemory;
    // the kernels of f record a at the first one's start and c at the last
    // one's end (their own execution, without the dispatch in between)
    LaunchEvents& le = launch_events();
    le = LaunchEvents{a, c, 0};
    hipError_t e = f();
    const int launched = le.launches;
    le = LaunchEvents{};
    if (e != hipSuccess) return e;
    if (launched == 0) {  // nothing launched: an empty interval
      e = hipEventRecord(a, st);
      if (e == hipSuccess) e = hipEventRecord(c, st);
    }
    b->recs.push_back({kind, a, c});
    return e;
  };
  const bool graph = (b->flags & DDH_BATCH_GRAPH) && !b->timing;
  if (b->timing) {
    // per-kernel timing: every lane's launches in sequence on the caller's stream
    int rc = batch_enqueue(b, b->groups, b->total, st, timed, b->yord.data(), b->curord.data());
    if (rc != DDH_OK) return rc;
  } else if (graph) {
    // the replayed graph reads the frame start from the descriptors
    hipError_t e = launch_begin(b->dptrs, b->yord.data(), b->curord.data(), b->total, st);
    if (e != hipSuccess) return hip_fail(e, "launch_begin");
    if (!b->gexec) {
      hipGraph_t g = nullptr;
      DDH_CHECK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      b->capturing = true;
      int rc = enqueue_lanes(b, b->cap);
      b->capturing = false;
      hipError_t ec = hipStreamEndCapture(b->cap, &g);
      if (rc != DDH_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
      ec = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ec != hipSuccess) {
        b->gexec = nullptr;
        return hip_fail(ec, "hipGraphInstantiate");
      }
    }
    DDH_CHECK(hipGraphLaunch(b->gexec, st));
  } else {
    int rc = enqueue_lanes(b, st);
    if (rc != DDH_OK) return rc;
  }
  for (ddh_stream_t s : b->streams) {
    s->parity = (s->parity + b->n_k) & 1;
    s->n++;
  }
  return DDH_OK;
}

// ---------------------------------------------------------------- serving
int ddh_server_create(int max_streams, ddh_server_t* out) {
  if (!out || max_streams < 1 || max_streams > (1 << 20)) return DDH_EINVAL;
  int dev = 0;
  DDH_CHECK(hipGetDevice(&dev));
  ddh_server_t v = new ddh_server_s();
  v->device = dev;
  v->max = max_streams;
  hipError_t e = hipMalloc(&v->list, sizeof(StreamDesc*) * max_streams);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&v->fork, hipEventDisableTiming);
  for (int l = 0; l < 4 && e == hipSuccess; ++l) {
    e = hipStreamCreateWithFlags(&v->lane[l], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&v->join[l], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    for (int l = 0; l < 4; ++l) {
      if (v->lane[l]) (void)hipStreamDestroy(v->lane[l]);
      if (v->join[l]) (void)hipEventDestroy(v->join[l]);
    }
    if (v->fork) (void)hipEventDestroy(v->fork);
    if (v->list) (void)hipFree(v->list);
    delete v;
    return hip_fail(e, "ddh_server_create");
  }
  live_add(v);
  *out = v;
  return DDH_OK;
}

int ddh_server_destroy(ddh_server_t v) {
  if (!v) return DDH_EINVAL;
  if (!is_live(v)) return DDH_ESTATE;
  live_remove(v);
  set_device_of(v->device);
  (void)hipDeviceSynchronize();
  for (int l = 0; l < 4; ++l) {
    (void)hipStreamDestroy(v->lane[l]);
    (void)hipEventDestroy(v->join[l]);
  }
  (void)hipEventDestroy(v->fork);
  (void)hipFree(v->list);
  delete v;
  return DDH_OK;
}

int ddh_server_step(ddh_server_t v, const ddh_stream_t* streams, const void* const* y, int count, void* hip_stream) {
  if (!v || (count > 0 && (!streams || !y))) return DDH_EINVAL;
  if (!is_live(v)) return DDH_ESTATE;
  if (count < 0 || count > v->max) return DDH_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < count; ++i) {
    int rc = check_stream(streams[i]);
    if (rc != DDH_OK) return rc;
    if (streams[i]->device != v->device) return DDH_ESTATE;
    if (!y[i]) return DDH_EINVAL;
    for (int j = 0; j < i; ++j)
      if (streams[j] == streams[i]) return DDH_EINVAL;
  }
  if (v->bound && st != v->st) return DDH_ESTATE;
  if (count == 0) return DDH_OK;
  v->bound = true;
  v->st = st;
  // list order: by n_k, then by N (the per-N kernels take contiguous ranges)
  v->order.resize(count);
  for (int i = 0; i < count; ++i) v->order[i] = i;
  std::stable_sort(v->order.begin(), v->order.end(), [&](int a, int c) {
    if (streams[a]->prm.n_k != streams[c]->prm.n_k) return streams[a]->prm.n_k < streams[c]->prm.n_k;
    return streams[a]->N < streams[c]->N;
  });
  v->ys.resize(count);
  v->curs.resize(count);
  v->ds.resize(count);
  for (int p = 0; p < count; ++p) {
    const int i = v->order[p];
    v->ys[p] = static_cast<const float2*>(y[i]);
    v->curs[p] = streams[i]->parity;
    v->ds[p] = streams[i]->d;
  }
  int p0 = 0;
  while (p0 < count) {
    const int n_k = streams[v->order[p0]]->prm.n_k;
    int p1 = p0;
    std::vector<Group> groups;
    while (p1 < count && streams[v->order[p1]]->prm.n_k == n_k) {
      const int N = streams[v->order[p1]]->N;
      Group g{N, p1 - p0, 0, tiles_for(N), streams[v->order[p1]]->tw, streams[v->order[p1]]->h.ctl};
      while (p1 < count && streams[v->order[p1]]->prm.n_k == n_k && streams[v->order[p1]]->N == N) {
        ++g.count;
        ++p1;
      }
      groups.push_back(g);
    }
    if (groups.size() == 1) {
      int rc = enqueue_frame(v->list + p0, groups, p1 - p0, n_k, 1, st, NoTiming{}, v->ys.data() + p0,
                             v->curs.data() + p0, v->ds.data() + p0, fused_stats_for(1, false));
      if (rc != DDH_OK) return rc;
    } else {  // the N groups (at most 4) on their own lanes, so that their launches overlap
      DDH_CHECK(hipEventRecord(v->fork, st));
      for (size_t l = 0; l < groups.size(); ++l) {
        DDH_CHECK(hipStreamWaitEvent(v->lane[l], v->fork, 0));
        const std::vector<Group> one{groups[l]};
        int rc = enqueue_frame(v->list + p0, one, groups[l].count, n_k, 1, v->lane[l], NoTiming{},
                               v->ys.data() + p0, v->curs.data() + p0, v->ds.data() + p0,
                               fused_stats_for((int)groups.size(), false));
        if (rc != DDH_OK) return rc;
        DDH_CHECK(hipEventRecord(v->join[l], v->lane[l]));
      }
      for (size_t l = 0; l < groups.size(); ++l) DDH_CHECK(hipStreamWaitEvent(st, v->join[l], 0));
    }
    p0 = p1;
  }
  for (int i = 0; i < count; ++i) {
    streams[i]->parity = (streams[i]->parity + streams[i]->prm.n_k) & 1;
    streams[i]->n++;
  }
  return DDH_OK;
}

// One-shot batched frame step: a server per (device, HIP stream), created on
// the first call with that pair and replaced by a larger one when a call
// passes more streams than it holds; kept until the process ends.  Calls on
// one HIP stream run in order, so the server's device list is reused safely.
int ddh_step_batch(const ddh_stream_t* streams, const void* const* y, int count, void* hip_stream) {
  if (count < 0 || (count > 0 && (!streams || !y))) return DDH_EINVAL;
  if (count > (1 << 20)) return DDH_EINVAL;
  for (int i = 0; i < count; ++i) {
    int rc = check_stream(streams[i]);
    if (rc != DDH_OK) return rc;
    if (!y[i]) return DDH_EINVAL;
    for (int j = 0; j < i; ++j)
      if (streams[j] == streams[i]) return DDH_EINVAL;
  }
  if (count == 0) return DDH_OK;
  const int dev = streams[0]->device;
  for (int i = 1; i < count; ++i)
    if (streams[i]->device != dev) return DDH_ESTATE;
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, ddh_server_t> servers;
  ddh_server_t v = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(dev, static_cast<hipStream_t>(hip_stream));
    auto it = servers.find(key);
    if (it != servers.end() && it->second->max < count) {
      // grow: the old list may still be read by this HIP stream's queued work
      int rc = set_device_of(dev);
      if (rc != DDH_OK) return rc;
      DDH_CHECK(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
      ddh_server_destroy(it->second);
      servers.erase(it);
      it = servers.end();
    }
    if (it == servers.end()) {
      int cap = 64;
      while (cap < count) cap *= 2;
      int cur = -1;
      DDH_CHECK(hipGetDevice(&cur));
      int rc = set_device_of(dev);
      if (rc == DDH_OK) rc = ddh_server_create(cap, &v);
      if (cur != dev) (void)hipSetDevice(cur);
      if (rc != DDH_OK) return rc;
      servers[key] = v;
    } else {
      v = it->second;
    }
  }
  return ddh_server_step(v, streams, y, count, hip_stream);
}

// ddh_step_batch without any allocation: the device list of descriptor
// pointers is the file-scope `scratch` array of the streams' device (filled
// by the frame's first launches from their arguments, read by the later
// ones), every group of (n_k, N) runs on the caller's HIP stream, and the
// host side uses fixed-size stack arrays only.
int ddh_step_batch_noalloc(const ddh_stream_t* streams, const void* const* y, int count, void* hip_stream) {
  if (count < 0 || count > kNoAllocMaxStreams) return DDH_EINVAL;
  if (count > 0 && (!streams || !y)) return DDH_EINVAL;
  for (int i = 0; i < count; ++i) {
    int rc = check_stream(streams[i]);
    if (rc != DDH_OK) return rc;
    if (!y[i]) return DDH_EINVAL;
    for (int j = 0; j < i; ++j)
      if (streams[j] == streams[i]) return DDH_EINVAL;
  }
  if (count == 0) return DDH_OK;
  const int dev = streams[0]->device;
  for (int i = 1; i < count; ++i)
    if (streams[i]->device != dev) return DDH_ESTATE;
  StreamDesc** list = scratch_of(dev);  // set when the first stream was created on dev
  if (!list) return DDH_ESTATE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int pos = 0, prev_nk = 0;
  for (;;) {
    // next distinct n_k, ascending
    int nk = 0;
    for (int i = 0; i < count; ++i) {
      const int v = streams[i]->prm.n_k;
      if (v > prev_nk && (nk == 0 || v < nk)) nk = v;
    }
    if (nk == 0) break;
    for (int N : {64, 128, 256, 512}) {
      Group g{N, 0, 0, tiles_for(N), nullptr};
      const float2* ys[FRAME_CHUNK];
      int curs[FRAME_CHUNK];
      StreamDesc* ds[FRAME_CHUNK];
      int m = 0;
      auto flush = [&]() -> int {
        if (m == 0) return DDH_OK;
        const hipError_t e = launch_stats(list + pos + g.count, m, N, 1, ys, curs, ds, st);
        if (e != hipSuccess) return hip_fail(e, "launch_stats");
        g.count += m;
        m = 0;
        return DDH_OK;
      };
      for (int i = 0; i < count; ++i) {
        const ddh_stream_t s = streams[i];
        if (s->prm.n_k != nk || s->N != N) continue;
        ys[m] = static_cast<const float2*>(y[i]);
        curs[m] = s->parity;
        ds[m] = s->d;
        g.tw = s->tw;
        if (++m == FRAME_CHUNK) {
          int rc = flush();
          if (rc != DDH_OK) return rc;
        }
      }
      int rc = flush();
      if (rc != DDH_OK) return rc;
      if (g.count == 0) continue;
      rc = enqueue_iters(list + pos, &g, 1, nk, 1, st, NoTiming{});
      if (rc != DDH_OK) return rc;
      pos += g.count;
    }
    prev_nk = nk;
  }
  for (int i = 0; i < count; ++i) {
    streams[i]->parity = (streams[i]->parity + streams[i]->prm.n_k) & 1;
    streams[i]->n++;
  }
  return DDH_OK;
}

int ddh_batch_stage_times(ddh_batch_t b, double* ms, long long* calls, const char** names, int* n) {
  if (!b || !n) return DDH_EINVAL;
  if (!is_live(b)) return DDH_ESTATE;
  int rc = drain_timing(b);
  if (rc != DDH_OK) return rc;
  const int m = std::min(*n, (int)KK_COUNT);
  for (int k = 0; k < m; ++k) {
    if (ms) ms[k] = b->acc_ms[k];
    if (calls) calls[k] = b->acc_n[k];
    if (names) names[k] = kKindNames[k];
  }
  *n = m;
  return DDH_OK;
}

// ------------------------------------------------------------------- tiles
int ddh_set_tiles(int N, const int* cfg) {
  if (!valid_N(N) || !cfg) return DDH_EINVAL;
  TileConfig t{cfg[0], cfg[1], cfg[2], cfg[3]};
  if (!tiles_ok(N, t)) return DDH_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  tile_cache()[N] = t;
  return DDH_OK;
}

int ddh_get_tiles(int N, int* cfg) {
  if (!valid_N(N) || !cfg) return DDH_EINVAL;
  TileConfig t = tiles_for(N);
  cfg[0] = t.row_lines;
  cfg[1] = t.col_width;
  cfg[2] = t.m_tile_h;
  cfg[3] = t.m_tile_w;
  return DDH_OK;
}

// Tiling for a mix of sizes: the whole batched step of `count` temporary
// streams with sizes Ns (default lanes: one per N) is timed, and each size's
// row, column and M-step tilings are chosen in turn (coordinate descent, sizes
// ascending), a candidate replacing the current one only when the step is
// more than 1 % faster.  Per-kernel timing of one size alone (ddh_autotune)
// misses how the lanes of different sizes share the device.
int ddh_autotune_mix(const int* Ns, int count, int* cfgs, double* step_us) {
  if (!Ns || count < 1 || count > 4096) return DDH_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!valid_N(Ns[i])) return DDH_EINVAL;
  std::vector<int> sizes(Ns, Ns + count);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  const int rows_c[4] = {4, 8, 16, 32}, cols_c[4] = {4, 8, 16, 32};
  const int ms_c[7][2] = {{16, 16}, {16, 32}, {16, 64}, {32, 32}, {32, 64}, {64, 64}, {32, 128}};
  std::vector<ddh_stream_t> ss;
  std::vector<const void*> ys(count);
  float2* ybuf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t ts = nullptr;  // the tuner's own stream: other work on the device is not synchronised with
  std::map<int, TileConfig> start;
  for (int N : sizes) start[N] = tiles_for(N);
  auto install = [&](const std::map<int, TileConfig>& m) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : m) tile_cache()[kv.first] = kv.second;
  };
  auto cleanup = [&]() {
    if (ts) (void)hipStreamSynchronize(ts);
    for (ddh_stream_t s : ss) ddh_destroy_stream(s);
    if (ybuf) (void)hipFree(ybuf);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ts) (void)hipStreamDestroy(ts);
  };
  size_t px_total = 0;
  for (int i = 0; i < count; ++i) px_total += (size_t)Ns[i] * Ns[i];
  hipError_t e = hipStreamCreateWithFlags(&ts, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "autotune stream");
  e = hipMalloc(&ybuf, sizeof(float2) * px_total);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "hipMalloc(autotune)");
  }
  e = launch_synth_frames(ybuf, (long long)px_total, 54321u, ts);
  if (e == hipSuccess) e = timing_event(&e0);
  if (e == hipSuccess) e = timing_event(&e1);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "autotune setup");
  }
  int rc = DDH_OK;
  size_t off = 0;
  for (int i = 0; i < count && rc == DDH_OK; ++i) {
    ddh_params p;
    ddh_default_params(Ns[i], &p);
    ddh_stream_t s = nullptr;
    rc = ddh_init_stream(&p, nullptr, ts, &s);
    if (rc == DDH_OK) ss.push_back(s);
    ys[i] = ybuf + off;
    off += (size_t)Ns[i] * Ns[i];
  }
  // microseconds per batched step with the tilings `tiles` (given to the
  // timing batch only; the process-wide tilings are not touched): best of two
  // runs of 10 steps after 2 warm-up steps, on a freshly created batch
  auto time_step = [&](const std::map<int, TileConfig>& tiles, double* out) -> int {
    double best = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
      ddh_batch_t b = nullptr;
      int r = batch_create_impl(ss.data(), count, 0, &tiles, &b);
      if (r != DDH_OK) return r;
      for (int f = 0; f < 2 && r == DDH_OK; ++f) r = ddh_batch_step(b, ys.data(), ts);
      hipError_t he = hipEventRecord(e0, ts);
      for (int f = 0; f < 10 && r == DDH_OK && he == hipSuccess; ++f) r = ddh_batch_step(b, ys.data(), ts);
      if (he == hipSuccess) he = hipEventRecord(e1, ts);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      (void)hipStreamSynchronize(ts);
      batch_release(b, false);
      if (r != DDH_OK) return r;
      if (he != hipSuccess) return hip_fail(he, "autotune timing");
      best = std::min(best, 1e3 * (double)ms / 10.0);
    }
    *out = best;
    return DDH_OK;
  };
  std::map<int, TileConfig> cur = start;
  double t_best = 0.0;
  if (rc == DDH_OK) rc = time_step(cur, &t_best);
  for (int N : sizes) {
    for (int dim = 0; dim < 3 && rc == DDH_OK; ++dim) {
      std::vector<TileConfig> cands;
      const TileConfig c0 = cur[N];
      if (dim == 0)
        for (int v : rows_c) cands.push_back({v, c0.col_width, c0.m_tile_h, c0.m_tile_w});
      else if (dim == 1)
        for (int v : cols_c) cands.push_back({c0.row_lines, v, c0.m_tile_h, c0.m_tile_w});
      else
        for (const auto& m : ms_c) cands.push_back({c0.row_lines, c0.col_width, m[0], m[1]});
      for (const TileConfig& c : cands) {
        if (!tiles_ok(N, c) || (c.row_lines == c0.row_lines && c.col_width == c0.col_width &&
                                c.m_tile_h == c0.m_tile_h && c.m_tile_w == c0.m_tile_w))
          continue;
        std::map<int, TileConfig> trial = cur;
        trial[N] = c;
        double t = 0.0;
        rc = time_step(trial, &t);
        if (rc != DDH_OK) break;
        if (t < 0.99 * t_best) {
          t_best = t;
          cur = trial;
        }
      }
    }
  }
  cleanup();
  if (rc != DDH_OK) return rc;  // nothing was installed
  install(cur);
  if (cfgs) {
    int k = 0;
    for (int N : sizes) {
      const TileConfig& c = cur[N];
      cfgs[k++] = c.row_lines;
      cfgs[k++] = c.col_width;
      cfgs[k++] = c.m_tile_h;
      cfgs[k++] = c.m_tile_w;
    }
  }
  if (step_us) *step_us = t_best;
  return DDH_OK;
}

int ddh_autotune(int N, int count, int* cfg, double* us) {
  if (!valid_N(N) || count < 1 || count > 4096) return DDH_EINVAL;
  const int rows_c[4] = {4, 8, 16, 32}, cols_c[4] = {4, 8, 16, 32};
  const int ms_c[8][2] = {{16, 16}, {16, 32}, {16, 64}, {32, 32}, {32, 64}, {64, 64}, {32, 128}, {0, 0}};
  std::vector<int> rows, cols;
  std::vector<std::pair<int, int>> mss;
  const TileConfig base = tiles_for(N);
  for (int v : rows_c)
    if (tiles_ok(N, {v, base.col_width, base.m_tile_h, base.m_tile_w})) rows.push_back(v);
  for (int v : cols_c)
    if (tiles_ok(N, {base.row_lines, v, base.m_tile_h, base.m_tile_w})) cols.push_back(v);
  for (auto& m : ms_c)
    if (tiles_ok(N, {base.row_lines, base.col_width, m[0], m[1]})) mss.push_back({m[0], m[1]});
  if (rows.empty() || cols.empty() || mss.empty()) return DDH_EINVAL;
  ddh_params p;
  ddh_default_params(N, &p);
  std::vector<ddh_stream_t> ss;
  float2* ybuf = nullptr;
  hipStream_t ts = nullptr;  // the tuner's own stream (other work is not synchronised with)
  int rc = DDH_OK;
  auto cleanup = [&]() {
    if (ts) (void)hipStreamSynchronize(ts);
    for (ddh_stream_t s : ss) ddh_destroy_stream(s);
    if (ybuf) (void)hipFree(ybuf);
    if (ts) (void)hipStreamDestroy(ts);
  };
  const size_t px = (size_t)N * N;
  hipError_t e = hipStreamCreateWithFlags(&ts, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "autotune stream");
  e = hipMalloc(&ybuf, sizeof(float2) * px * count);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "hipMalloc(autotune)");
  }
  e = launch_synth_frames(ybuf, (long long)(px * count), 12345u, ts);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "synth_frames");
  }
  for (int i = 0; i < count && rc == DDH_OK; ++i) {
    ddh_stream_t s = nullptr;
    rc = ddh_init_stream(&p, nullptr, ts, &s);
    if (rc == DDH_OK) ss.push_back(s);
  }
  if (rc != DDH_OK) {
    cleanup();
    return rc;
  }
  std::vector<const void*> ys(count);
  for (int i = 0; i < count; ++i) ys[i] = ybuf + px * i;
  const int ncand = (int)std::max({rows.size(), cols.size(), mss.size()});
  std::vector<double> t_rows(rows.size(), 1e30), t_cols(cols.size(), 1e30), t_ms(mss.size(), 1e30);
  for (int c = 0; c < ncand && rc == DDH_OK; ++c) {
    const int ir = std::min(c, (int)rows.size() - 1), ic = std::min(c, (int)cols.size() - 1),
              im = std::min(c, (int)mss.size() - 1);
    // the candidate goes to the timing batch only, not to the process-wide tilings
    const std::map<int, TileConfig> cand{{N, TileConfig{rows[ir], cols[ic], mss[im].first, mss[im].second}}};
    ddh_batch_t b = nullptr;
    rc = batch_create_impl(ss.data(), count, 0, &cand, &b);
    if (rc != DDH_OK) break;
    for (int f = 0; f < 2 && rc == DDH_OK; ++f) rc = ddh_batch_step(b, ys.data(), ts);
    if (rc == DDH_OK) rc = ddh_batch_set_timing(b, 1);
    for (int f = 0; f < 5 && rc == DDH_OK; ++f) rc = ddh_batch_step(b, ys.data(), ts);
    double ms[KK_COUNT];
    long long calls[KK_COUNT];
    int n = KK_COUNT;
    if (rc == DDH_OK) rc = ddh_batch_stage_times(b, ms, calls, nullptr, &n);
    (void)hipStreamSynchronize(ts);
    batch_release(b, false);
    if (rc != DDH_OK) break;
    auto avg = [&](int kk) { return calls[kk] ? 1e3 * ms[kk] / calls[kk] : 1e30; };
    t_rows[ir] = std::min(t_rows[ir], avg(KK_ROW1) + avg(KK_ROW2));
    t_cols[ic] = std::min(t_cols[ic], avg(KK_COL));
    t_ms[im] = std::min(t_ms[im], avg(KK_MSTEP));
  }
  const int br = (int)(std::min_element(t_rows.begin(), t_rows.end()) - t_rows.begin());
  const int bc = (int)(std::min_element(t_cols.begin(), t_cols.end()) - t_cols.begin());
  const int bm = (int)(std::min_element(t_ms.begin(), t_ms.end()) - t_ms.begin());
  const TileConfig best{rows[br], cols[bc], mss[bm].first, mss[bm].second};
  cleanup();
  if (rc != DDH_OK) return rc;  // nothing was installed
  {
    std::lock_guard<std::mutex> lk(g_mu);
    tile_cache()[N] = best;
  }
  if (cfg) {
    cfg[0] = best.row_lines;
    cfg[1] = best.col_width;
    cfg[2] = best.m_tile_h;
    cfg[3] = best.m_tile_w;
  }
  if (us) {
    us[0] = t_rows[br];  // row-ifft + row-fft
    us[1] = t_cols[bc];
    us[2] = 0.0;
    us[3] = t_ms[bm];
  }
  return DDH_OK;
}

// ------------------------------------------------------------------- FFT
int ddh_fft2(int N, int count, const void* in, void* out, void* work, int inverse, void* hip_stream) {
  if (!valid_N(N) || count <= 0 || !in || !out || !work) return DDH_EINVAL;
  if (inverse != 0 && inverse != 1) return DDH_EINVAL;
  int dev = 0;
  DDH_CHECK(hipGetDevice(&dev));
  float2* tw = nullptr;
  int rc = ensure_twiddles(dev, &tw);
  if (rc != DDH_OK) return rc;
  hipError_t e = launch_fft2(N, count, static_cast<const float2*>(in), static_cast<float2*>(out),
                             static_cast<float2*>(work), tw + twiddle_offset(N), inverse,
                             static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "launch_fft2");
  return DDH_OK;
}


// ------------------------------------------------------- differentiation
// Inverse of the pupil's plane-fit moment matrix (symmetric: 00 01 02 11 12
// 22), computed once per (N, diameter^2) and kept.
static std::array<double, 6> pupil_moment_inverse(int N, float d2) {
  static std::mutex mu;
  static std::map<std::pair<int, float>, std::array<double, 6>> cache;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(N, d2);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  double m[6] = {0, 0, 0, 0, 0, 0};
  const double c = 0.5 * (N - 1);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const int di = 2 * i - N + 1, dj = 2 * j - N + 1;
      if ((float)(di * di + dj * dj) > d2) continue;
      const double a = i - c, e = j - c;
      m[0] += 1, m[1] += a, m[2] += e, m[3] += a * a, m[4] += a * e, m[5] += e * e;
    }
  const double a00 = m[0], a01 = m[1], a02 = m[2], a11 = m[3], a12 = m[4], a22 = m[5];
  const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
  const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
  const double det = a00 * c00 + a01 * c01 + a02 * c02;
  std::array<double, 6> inv{};
  if (det != 0.0) inv = {c00 / det, c01 / det, c02 / det, c11 / det, c12 / det, c22 / det};
  cache[key] = inv;
  return inv;
}

int ddh_unrolled_grad_batch(const ddh_params* p, int count, int K, const void* const* y, const float* const* phi0,
                            const float* const* phi_true, int ckpt, float* const* d_phi0, ddh_grad_out* out,
                            void* hip_stream) {
  if (!p || !y || !phi0 || !phi_true || !d_phi0 || !out || count < 1 || K < 1 || ckpt < 1) return DDH_EINVAL;
  const int N = p[0].N;
  for (int b = 0; b < count; ++b) {
    const int rc = validate(&p[b]);
    if (rc != DDH_OK) return rc;
    if (p[b].n_k != 1 || !(p[b].qg_p == 2.0f) || p[b].N != N) return DDH_EINVAL;
    if (!phi0[b] || !phi_true[b] || !d_phi0[b]) return DDH_EINVAL;
    for (int k = 0; k < K; ++k)
      if (!y[(size_t)b * K + k]) return DDH_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  DDH_CHECK(hipGetDevice(&dev));
  float2* tw_all = nullptr;
  int rc = ensure_twiddles(dev, &tw_all);
  if (rc != DDH_OK) return rc;
  const int B = count;
  const size_t px = (size_t)N * N, bpx = (size_t)B * px;
  if (bpx > (size_t)INT32_MAX) return DDH_EINVAL;  // pixel indices of a batch are 32-bit
  const int nrec = g_records(N);
  // per-stream constants and the inverse of each pupil's moment matrix (plane fit)
  std::vector<GradPrm> prm(B);
  std::vector<double> minv(6 * (size_t)B);
  for (int b = 0; b < B; ++b) {
    const ddh_params& q = p[b];
    GradPrm& P = prm[b];
    P.N = N;
    P.d2 = q.pupil_diameter * q.pupil_diameter;
    P.lam = q.lambda;
    P.alpha = q.alpha;
    P.fl = q.r_floor;
    P.s2 = q.sigma_w2;
    P.inv_sp = (float)(1.0 / ((double)q.qg_sigma * (double)q.qg_sigma));
    P.pmq = q.qg_p - q.qg_q;
    P.lc = (float)(((double)q.qg_p - (double)q.qg_q) * std::log2(1.0 / ((double)q.qg_T * (double)q.qg_sigma)));
    P.qop = q.qg_q / q.qg_p;
    P.beta = q.beta_phi;
    P.sig_r = q.qg_sigma;
    const std::array<double, 6> inv = pupil_moment_inverse(N, P.d2);
    for (int k = 0; k < 6; ++k) minv[6 * (size_t)b + k] = inv[k];
  }
  // frame tables, frame-major: ytab[k * B + b]
  std::vector<const void*> ytab((size_t)K * B);
  for (int b = 0; b < B; ++b)
    for (int k = 0; k < K; ++k) ytab[(size_t)k * B + b] = y[(size_t)b * K + k];
  // ---- workspace: checkpoints, one segment of frame stashes, adjoint arrays, scalars
  const int nseg = (K + ckpt - 1) / ckpt;
  const int per_frame_f = 4 + 5 + 4;  // phip s kap tth | rs[0..4] | ps[1..4]
  const int per_frame_c = 5;          // yh v b mu z
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t o_ck = take(2 * (size_t)nseg * bpx * 4);
  const size_t o_st = take((size_t)ckpt * (per_frame_f * bpx * 4 + per_frame_c * bpx * 8));
  const size_t o_work = take(bpx * 8);
  const size_t o_r0 = take(bpx * 4);
  const size_t o_in = take(2 * bpx * 4);  // phi0 and phi_true of every stream, batched
  const size_t o_bf = take(12 * bpx * 4);
  const size_t o_bc = take(2 * bpx * 8);
  const size_t o_part = take((size_t)B * nrec * 6 * 8);
  const size_t o_prm = take(sizeof(GradPrm) * B);
  const size_t o_minv = take(sizeof(double) * 6 * B);
  const size_t o_loss = take(sizeof(GradLoss) * B);
  const size_t o_flag = take(sizeof(int) * B);
  const size_t o_ytab = take(sizeof(void*) * (size_t)K * B);
  // the device's workspace, kept between calls and grown when too small;
  // calls on one device take turns on it (each ends synchronised)
  static std::mutex ws_mu[kMaxDev];
  static char* ws_mem[kMaxDev] = {nullptr};
  static size_t ws_cap[kMaxDev] = {0};
  if (dev < 0 || dev >= kMaxDev) return DDH_EDEVICE;
  std::lock_guard<std::mutex> ws_lock(ws_mu[dev]);
  if (ws_cap[dev] < off) {
    if (ws_mem[dev]) {
      (void)hipFree(ws_mem[dev]);
      ws_mem[dev] = nullptr;
      ws_cap[dev] = 0;
    }
    hipError_t ea = hipMalloc(&ws_mem[dev], off);
    if (ea != hipSuccess) {
      ws_mem[dev] = nullptr;
      return hip_fail(ea, "hipMalloc(grad)");
    }
    ws_cap[dev] = off;
  }
  char* mem = ws_mem[dev];
  hipError_t e = hipSuccess;
  auto fail = [&](int code) {
    (void)hipStreamSynchronize(st);
    return code;
  };
  GradDev dv{};
  dv.prm = (const GradPrm*)(mem + o_prm);
  dv.minv = (const double*)(mem + o_minv);
  dv.loss = (GradLoss*)(mem + o_loss);
  dv.flag = (int*)(mem + o_flag);
  dv.part = (double*)(mem + o_part);
  const float2* const* dytab = (const float2* const*)(mem + o_ytab);
  if (hipMemcpyAsync(mem + o_prm, prm.data(), sizeof(GradPrm) * B, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(mem + o_minv, minv.data(), sizeof(double) * 6 * B, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(mem + o_ytab, ytab.data(), sizeof(void*) * ytab.size(), hipMemcpyHostToDevice, st) !=
          hipSuccess)
    return fail(DDH_EDEVICE);
  float* ck = (float*)(mem + o_ck);
  auto ck_r = [&](int sgi) { return ck + (size_t)(2 * sgi) * bpx; };
  auto ck_p = [&](int sgi) { return ck + (size_t)(2 * sgi + 1) * bpx; };
  std::vector<GradFwd> slot(ckpt);
  {
    char* q = mem + o_st;
    for (int t = 0; t < ckpt; ++t) {
      GradFwd& a = slot[t];
      float* fb = (float*)q;
      a.phip = fb, a.s = fb + bpx, a.kap = fb + 2 * bpx, a.tth = fb + 3 * bpx;
      for (int c = 0; c < 5; ++c) a.rs[c] = fb + (4 + c) * bpx;
      a.ps[0] = nullptr;
      for (int c = 1; c < 5; ++c) a.ps[c] = fb + (8 + c) * bpx;
      float2* cb = (float2*)(q + per_frame_f * bpx * 4);
      a.yh = cb, a.v = cb + bpx, a.b = cb + 2 * bpx, a.mu = cb + 3 * bpx, a.z = cb + 4 * bpx;
      a.work = (float2*)(mem + o_work);
      a.tw = tw_all + twiddle_offset(N);
      q += per_frame_f * bpx * 4 + per_frame_c * bpx * 8;
    }
  }
  float* rzero = (float*)(mem + o_r0);
  float* pin = (float*)(mem + o_in);
  float* ptrue = pin + bpx;
  GradBwd g{};
  {
    float* f = (float*)(mem + o_bf);
    float** fp[12] = {&g.rbar, &g.pbar, &g.pb2, &g.em, &g.kbar, &g.tbar, &g.sbar, &g.Abar, &g.Bbar,
                      &g.gs2, &g.gsr, &g.gbeta};
    for (int q = 0; q < 12; ++q) *fp[q] = f + q * bpx;
    float2* c = (float2*)(mem + o_bc);
    g.zbar = c, g.vbar = c + bpx;
  }
  if (launch_fill_zero(rzero, (long long)bpx, st) != hipSuccess ||
      launch_fill_zero((float*)(mem + o_bf), 12 * (long long)bpx, st) != hipSuccess ||
      launch_fill_zero((float*)dv.flag, B, st) != hipSuccess)
    return fail(DDH_EDEVICE);
  for (int b = 0; b < B; ++b)
    if (launch_copy(pin + b * px, phi0[b], (long long)px, st) != hipSuccess ||
        launch_copy(ptrue + b * px, phi_true[b], (long long)px, st) != hipSuccess)
      return fail(DDH_EDEVICE);
  // one frame forward into slot t from (r_in, phi_in)
  auto frame = [&](int k, int t, const float* r_in, const float* phi_in) -> bool {
    GradFwd& a = slot[t];
    a.y = dytab + (size_t)k * B;
    a.r_in = r_in;
    a.phi_in = phi_in;
    return g_launch_forward(a, dv, N, B, st) == hipSuccess;
  };
  // ---- forward with checkpoints
  const float* r_cur = rzero;
  const float* p_cur = pin;
  for (int k = 0; k < K; ++k) {
    if (k % ckpt == 0) {
      if (launch_copy(ck_r(k / ckpt), r_cur, (long long)bpx, st) != hipSuccess ||
          launch_copy(ck_p(k / ckpt), p_cur, (long long)bpx, st) != hipSuccess)
        return fail(DDH_EDEVICE);
      r_cur = ck_r(k / ckpt);
      p_cur = ck_p(k / ckpt);
    }
    const int t = k % ckpt;
    if (!frame(k, t, r_cur, p_cur)) return fail(DDH_EDEVICE);
    r_cur = slot[t].rs[4];
    p_cur = slot[t].ps[4];
  }
  // ---- loss on the last phase and its adjoint
  if (g_launch_loss(p_cur, ptrue, dv, N, B, g.pbar, st) != hipSuccess) return fail(DDH_EDEVICE);
  // ---- backward, segment by segment (recomputing each segment's stashes)
  for (int sgi = nseg - 1; sgi >= 0; --sgi) {
    const int k0 = sgi * ckpt, k1 = std::min(K, k0 + ckpt);
    const float* rr = ck_r(sgi);
    const float* pp = ck_p(sgi);
    for (int k = k0; k < k1; ++k) {
      if (!frame(k, k - k0, rr, pp)) return fail(DDH_EDEVICE);
      rr = slot[k - k0].rs[4];
      pp = slot[k - k0].ps[4];
    }
    for (int k = k1 - 1; k >= k0; --k)
      if (g_launch_backward(slot[k - k0], g, dv, N, B, st) != hipSuccess) return fail(DDH_EDEVICE);
  }
  // ---- outputs
  if (g_launch_totals(g, dv, N, B, st) != hipSuccess) return fail(DDH_EDEVICE);
  for (int b = 0; b < B; ++b)
    if (launch_copy(d_phi0[b], g.pbar + b * px, (long long)px, st) != hipSuccess) return fail(DDH_EDEVICE);
  std::vector<GradLoss> lo(B);
  std::vector<double> rec(3 * (size_t)B * nrec);
  std::vector<int> flag(B);
  if (hipMemcpyAsync(lo.data(), dv.loss, sizeof(GradLoss) * B, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(rec.data(), dv.part, sizeof(double) * rec.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(flag.data(), dv.flag, sizeof(int) * B, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(DDH_EDEVICE);
  // the totals' records in record order (the same for every batch composition)
  std::vector<double> tot(3 * (size_t)B, 0.0);
  for (int b = 0; b < B; ++b)
    for (int r = 0; r < nrec; ++r)
      for (int q = 0; q < 3; ++q) tot[3 * b + q] += rec[((size_t)b * nrec + r) * 3 + q];
  int res = DDH_OK;
  for (int b = 0; b < B; ++b) {
    out[b].loss = lo[b].loss;
    out[b].d_sigma_w = 2.0 * std::sqrt((double)p[b].sigma_w2) * tot[3 * b];
    out[b].d_sigma_r = tot[3 * b + 1];
    out[b].d_beta = tot[3 * b + 2];
    if (flag[b]) res = DDH_EDATA;
  }
  return fail(res);
}

int ddh_unrolled_grad(const ddh_params* p, int K, const void* const* y, const float* phi0, const float* phi_true,
                      int ckpt, float* d_phi0, ddh_grad_out* out, void* hip_stream) {
  return ddh_unrolled_grad_batch(p, 1, K, y, &phi0, &phi_true, ckpt, &d_phi0, out, hip_stream);
}

}  // extern "C"
