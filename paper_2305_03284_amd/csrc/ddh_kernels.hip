// HIP kernels of the Dynamic DH-MBIR per-frame EM step for gfx950 (MI355X).
//
// Per frame and per stream (N x N grid, complex64 data, FP32 arithmetic):
//   k_stats     y -> per-row records of mean / centred power (Eq. (4) Normalize)
//               phi -> per-row records of the least-squares plane (RemoveTipTilt)
//   k_finalize  records -> mean, scale, plane coefficients, reject flag
//   k_row1      rows:    a exp(-j phi') (y - mean) scale, inverse 1-D DFT   (A_phi^H, first half);
//               at a frame's first EM iteration every block combines the records itself
//   k_row1s     k_stats and the first k_row1 of a frame as one launch (the blocks of
//               a stream publish their row records and wait for each other)
//   k_col       columns: inverse 1-D DFT -> b, Eq. (3) init, E-step -> mu,
//               forward 1-D DFT of mu                                   (A_phi^H second half, F first half)
//   k_row2      rows:    forward 1-D DFT -> z = F mu, per-pupil-pixel phase data term (kappa, theta~)
//   k_mstep     halo-tiled 4-colour sweep: r M-step (QGGMRF surrogate, cubic) and phi M-step (GMRF)
// The 2-D DFTs are unitary (scale 1/N per 2-D transform) with the exp(-2 pi i k n/N)
// kernel for the forward direction.  No MFMA: nothing here is a dense contraction.
#include "ddh_internal.h"
#include <hip/hip_ext.h>
#include <cfloat>
#include <cmath>
#include <type_traits>

namespace ddh {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// sin and cos of x via v_sin_f32 / v_cos_f32 on x / (2 pi) reduced to
// [-1/2, 1/2) revolutions (absolute error about 1e-6 for |x| below ~100 rad).
__device__ __forceinline__ void fsincos(float x, float* sn, float* cs) {
  float rev = x * 0.15915494309189534f;
  rev -= rintf(rev);
  *sn = __builtin_amdgcn_sinf(rev);
  *cs = __builtin_amdgcn_cosf(rev);
}

// cos(2 pi q / 16) and sin(2 pi q / 16): the 16th roots of unity used by the
// in-register DFTs, folded at compile time.
__device__ __forceinline__ constexpr float cos16(int q) {
  return q == 0 ? 1.0f : q == 1 ? 0.92387953251128674f : q == 2 ? 0.70710678118654752f
       : q == 3 ? 0.38268343236508977f : q == 4 ? 0.0f : q == 5 ? -0.38268343236508977f
       : q == 6 ? -0.70710678118654752f : q == 7 ? -0.92387953251128674f : -1.0f;
}
__device__ __forceinline__ constexpr float sin16(int q) {  // q in [0, 8)
  return q == 0 ? 0.0f : q == 1 ? 0.38268343236508977f : q == 2 ? 0.70710678118654752f
       : q == 3 ? 0.92387953251128674f : q == 4 ? 1.0f : q == 5 ? 0.92387953251128674f
       : q == 6 ? 0.70710678118654752f : 0.38268343236508977f;
}

// ---------------------------------------------------------------------------
// In-register DFT of size R (R = 1, 2, 4, 8, 16), natural order in and out:
//   X[q] = sum_r x[r] exp(DIR * 2 pi i r q / R)   (DIR = -1 forward, +1 inverse)
// Radix-2 decimation in time: X[q] = E[q] + w^q O[q], X[q + R/2] = E[q] - w^q O[q].
// ---------------------------------------------------------------------------
template <int R, int DIR>
struct RegDFT {
  static __device__ __forceinline__ void run(float2* x) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    RegDFT<R / 2, DIR>::run(e);
    RegDFT<R / 2, DIR>::run(o);
#pragma unroll
    for (int q = 0; q < R / 2; ++q) {
      constexpr int step = 16 / R;
      float2 t;
      if (q == 0) {
        t = o[q];
      } else if (4 * q == R) {  // w^q = DIR * i
        t = DIR > 0 ? make_float2(-o[q].y, o[q].x) : make_float2(o[q].y, -o[q].x);
      } else {
        const float c = cos16(q * step);
        const float s = DIR > 0 ? sin16(q * step) : -sin16(q * step);
        t = make_float2(o[q].x * c - o[q].y * s, o[q].x * s + o[q].y * c);
      }
      x[q] = cadd(e[q], t);
      x[q + R / 2] = csub(e[q], t);
    }
  }
};
template <int DIR>
struct RegDFT<1, DIR> {
  static __device__ __forceinline__ void run(float2*) {}
};

// ---------------------------------------------------------------------------
// Stockham autosort FFT of one line of length N held by T = N/E threads, each
// with E values in registers.  Stage with radix R after earlier radices of
// product NS: butterfly j (j < N/R) reads elements j + r N/R, multiplies
// element r by w_N^(r (j mod NS) N/(NS R)), does a radix-R DFT and writes
// element (j / NS) NS R + (j mod NS) + r NS.  Thread t owns butterflies
// j = t + b T, b < E/R, register v[b R + r].
// ---------------------------------------------------------------------------
template <int... Rs>
struct RadixList {};

template <int N>
struct Plan;
template <>
struct Plan<64> {
  static constexpr int E = 8;
  using Inv = RadixList<8, 8>;
  using Fwd = RadixList<8, 8>;
  static constexpr int R0_INV = 8, RL_INV = 8, R0_FWD = 8, RL_FWD = 8;
};
template <>
struct Plan<128> {
  static constexpr int E = 16;
  using Inv = RadixList<16, 8>;
  using Fwd = RadixList<8, 16>;
  static constexpr int R0_INV = 16, RL_INV = 8, R0_FWD = 8, RL_FWD = 16;
};
template <>
struct Plan<256> {
  static constexpr int E = 16;
  using Inv = RadixList<16, 16>;
  using Fwd = RadixList<16, 16>;
  static constexpr int R0_INV = 16, RL_INV = 16, R0_FWD = 16, RL_FWD = 16;
};
template <>
struct Plan<512> {
  static constexpr int E = 16;
  using Inv = RadixList<16, 16, 2>;
  using Fwd = RadixList<2, 16, 16>;
  static constexpr int R0_INV = 16, RL_INV = 2, R0_FWD = 2, RL_FWD = 16;
};

// element index held in register i by thread t for the first stage of radix R0
template <int N, int E, int R0>
__device__ __forceinline__ int pos_first(int i, int t) {
  constexpr int T = N / E;
  return t + (i / R0) * T + (i % R0) * (N / R0);
}
// element index held in register i by thread t after the last stage of radix RL
template <int N, int E, int RL>
__device__ __forceinline__ int pos_last(int i, int t) {
  constexpr int T = N / E;
  return t + (i / RL) * T + (i % RL) * (N / RL);
}

// LDS index maps: element n of the line this thread works on.
template <int N>
struct RowLds {  // lines are rows; pad one element every 16 against bank conflicts
  static constexpr int STRIDE = N + N / 16;
  float2* base;
  __device__ __forceinline__ float2& operator()(int n) const { return base[n + (n >> 4)]; }
};
template <int W>
struct ColLds {  // lines are columns of a W-wide strip stored row-major with one pad element
  static constexpr int STRIDE = W + 1;
  float2* base;  // already offset by the column within the strip
  __device__ __forceinline__ float2& operator()(int n) const { return base[n * STRIDE]; }
};

template <int N, int E, int DIR, int R, int NS>
__device__ __forceinline__ void stage_compute(float2 (&v)[E], int t, const float2* __restrict__ tw) {
  constexpr int T = N / E;
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    if constexpr (NS > 1) {
      const int j = t + b * T;
      const int k = j & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * k * (N / (NS * R))];
        if (DIR > 0) w.y = -w.y;
        v[b * R + r] = cmul(v[b * R + r], w);
      }
    }
    RegDFT<R, DIR>::run(&v[b * R]);
  }
}

template <int N, int E, int R, int NS, class L>
__device__ __forceinline__ void stage_store(const float2 (&v)[E], int t, const L& lds) {
  constexpr int T = N / E;
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    const int j = t + b * T;
    const int d0 = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
    for (int r = 0; r < R; ++r) lds(d0 + r * NS) = v[b * R + r];
  }
}

template <int N, int E, int R, class L>
__device__ __forceinline__ void stage_load(float2 (&v)[E], int t, const L& lds) {
  constexpr int T = N / E;
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    const int j = t + b * T;
#pragma unroll
    for (int r = 0; r < R; ++r) v[b * R + r] = lds(j + r * (N / R));
  }
}

template <int N, int E, int DIR, int NS, class L, int R, int... Rest>
struct StockhamRun {
  static __device__ __forceinline__ void run(float2 (&v)[E], int t, const L& lds, const float2* tw) {
    stage_compute<N, E, DIR, R, NS>(v, t, tw);
    if constexpr (sizeof...(Rest) > 0) {
      constexpr int R2 = first_of<Rest...>();
      stage_store<N, E, R, NS>(v, t, lds);
      __syncthreads();
      stage_load<N, E, R2>(v, t, lds);
      __syncthreads();
      StockhamRun<N, E, DIR, NS * R, L, Rest...>::run(v, t, lds, tw);
    }
  }
  template <int A, int... B>
  static constexpr int first_of() { return A; }
};

template <int N, int E, int DIR, class L, int... Rs>
__device__ __forceinline__ void line_fft_impl(float2 (&v)[E], int t, const L& lds, const float2* tw,
                                              RadixList<Rs...>) {
  StockhamRun<N, E, DIR, 1, L, Rs...>::run(v, t, lds, tw);
}

// Inverse (DIR=+1) uses Plan::Inv, forward (DIR=-1) Plan::Fwd.  Unnormalised.
template <int N, int DIR, class L>
__device__ __forceinline__ void line_fft(float2 (&v)[Plan<N>::E], int t, const L& lds, const float2* tw) {
  if constexpr (DIR > 0)
    line_fft_impl<N, Plan<N>::E, DIR>(v, t, lds, tw, typename Plan<N>::Inv{});
  else
    line_fft_impl<N, Plan<N>::E, DIR>(v, t, lds, tw, typename Plan<N>::Fwd{});
}

template <int N, int DIR>
__device__ __forceinline__ int first_pos(int i, int t) {
  if constexpr (DIR > 0) return pos_first<N, Plan<N>::E, Plan<N>::R0_INV>(i, t);
  else return pos_first<N, Plan<N>::E, Plan<N>::R0_FWD>(i, t);
}
template <int N, int DIR>
__device__ __forceinline__ int last_pos(int i, int t) {
  if constexpr (DIR > 0) return pos_last<N, Plan<N>::E, Plan<N>::RL_INV>(i, t);
  else return pos_last<N, Plan<N>::E, Plan<N>::RL_FWD>(i, t);
}

// ---------------------------------------------------------------------------
// Global-memory views.  The descriptors hold generic pointers; memory reached
// through a generic pointer is accessed with flat instructions, which also
// count against the LDS/scalar wait counter, so every LDS wait would stall
// behind outstanding HBM loads.  All these buffers live in global memory: the
// kernels read their descriptor and the buffers through address-space-1
// views.
// ---------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <class T>
using gptr = T*;  // the host pass only parses kernel bodies
#endif
template <class T>
__device__ __forceinline__ gptr<T> glb(T* p) {
  return (gptr<T>)p;
}
template <class T>
__device__ __forceinline__ auto& desc_ref(T* p) {
  return *glb(p);
}

// ---------------------------------------------------------------------------
// Arithmetic that more than one kernel evaluates for the same pixel (Eq. (3),
// the E-step statistics, the M-step pixel updates) is written with explicit
// FMAs and compiled without contraction, so every kernel and every tiling
// rounds it identically.
// ---------------------------------------------------------------------------
#define DDH_EXACT_FP _Pragma("clang fp contract(off)")

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
// (|2i - N + 1| < 2^23: the squares use the full-rate 24-bit multiplier)
__device__ __forceinline__ bool in_pupil(int i, int j, int N, float d2) {
  const int di = 2 * i - N + 1, dj = 2 * j - N + 1;
  return (float)(__mul24(di, di) + __mul24(dj, dj)) <= d2;
}

// Per-pixel aperture geometry byte of a stream (D_a of the Forward Model):
// bit 4 = the pixel is in the aperture, bits 0-3 = prior weight of its
// aperture neighbours in twelfths (2 per edge, 1 per diagonal neighbour);
// zero off the aperture.  Built on the host from the circle or the mask.
constexpr unsigned GEO_IN = 16u;
__device__ __forceinline__ bool geo_in(unsigned g) { return (g & GEO_IN) != 0u; }

// least-squares plane c0 + c1 (i - c) + c2 (j - c), c = (N-1)/2 (RemoveTipTilt)
__device__ __forceinline__ float plane_val(float c0, float c1, float c2, int i, int j, int N) {
  DDH_EXACT_FP
  const float cc = 0.5f * (float)(N - 1);
  return __builtin_fmaf(c2, (float)j - cc, __builtin_fmaf(c1, (float)i - cc, c0));
}

// Eq. (3) initialisation and E-step statistics, shared by k_col and k_mstep so
// that both evaluate exactly the same FP32 operations.
__device__ __forceinline__ float rinit_of(float rp, float bb, float lam, float alpha, float floor_) {
  DDH_EXACT_FP
  return fmaxf(__builtin_fmaf(1.0f - lam, rp, (lam * alpha) * bb), floor_);
}
__device__ __forceinline__ float wiener_of(float r, float s2) {
  DDH_EXACT_FP
  return r * __builtin_amdgcn_rcpf(r + s2);
}
__device__ __forceinline__ float second_moment(float w, float bb, float s2) {
  DDH_EXACT_FP
  // s = C + |mu|^2 = s2 w + w^2 |b|^2
  return __builtin_fmaf(s2, w, (w * w) * bb);
}

// ---------------------------------------------------------------------------
// block reductions (fixed-shape trees: deterministic)
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_sum(float (&x)[NV], float* red /* >= NV*16 */) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x[k] += __shfl_xor(x[k], off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * 16 + wv] = x[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += red[k * 16 + w];
    x[k] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Block -> (item, stream) of a (items, streams) grid.  Workgroups are
// dispatched round-robin over the 8 XCDs in linear order; when the streams
// split evenly, every block of a stream has the same linear index mod 8 and
// so goes to one XCD (streams [x S/8, (x+1) S/8) share the blocks of index
// x mod 8, the same grouping as the M-step's), so that what one kernel of a
// stream writes, the next reads through the same L2 (which XCD that is
// depends on where the dispatch starts).
// ---------------------------------------------------------------------------
struct XcdBlock {
  int item, strm;
};
__device__ __forceinline__ XcdBlock xcd_block() {
  const int I = gridDim.x, S = gridDim.y;
  if (S % 8 != 0) return {(int)blockIdx.x, (int)blockIdx.y};
  const int L = blockIdx.x + blockIdx.y * I;
  const int k = L / 8;
  return {k % I, (L % 8) * (S / 8) + k / I};
}

// ---------------------------------------------------------------------------
// Cross-workgroup synchronisation helpers (work-list kernel, fused first row
// pass).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned xcc_id() {
  // hwreg(HW_REG_XCC_ID, 0, 4): the XCD the wave runs on
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
}
// Invalidate this CU's vector L1 (lines another CU of the XCD may have
// rewritten since they were cached here); the L2 is the XCD's coherence point.
__device__ __forceinline__ void l1_invalidate() { asm volatile("buffer_inv sc0" ::: "memory"); }
// lgkmcnt(0): this wave's LDS stores have completed.  Issued after the store
// of the next ticket, which the loop-top barrier publishes: on that loop's
// back edge the compiler has been seen to place no LDS wait before the
// barrier, and another wave could then read the previous ticket.
__device__ __forceinline__ void lds_stores_done() { __builtin_amdgcn_s_waitcnt(0xC07F); }
__device__ __forceinline__ unsigned ctl_load(gptr<unsigned> p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ctl_add(gptr<unsigned> p, unsigned v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Frame start arguments: this frame's y and current state buffer per stream
// of a launch (at most 64 streams per launch).
// ---------------------------------------------------------------------------
constexpr int FRAME_ARGS_MAX = 64;
struct FrameArgs {
  const float2* y[FRAME_ARGS_MAX];
  int cur[FRAME_ARGS_MAX];
  StreamDesc* d[FRAME_ARGS_MAX];  // descriptors, when the launch's device list is filled here
};
// k_begin: store the frame arguments in the descriptors (used before a
// replayed graph, whose kernels read them there).  grid 1, block 64
__global__ void k_begin(StreamDesc* const* dptrs, FrameArgs a, int count) {
  const int i = threadIdx.x;
  if (i < count) {
    const auto d = glb(dptrs[i]);
    d->y = a.y[i];
    d->cur = a.cur[i];
  }
}

// ---------------------------------------------------------------------------
// Normalize (Eq. 4) and RemoveTipTilt statistics, one record per grid row
// (PART_STRIDE floats): the sum of y over the row, the power of y about the
// row's own mean, and the sums of phi and of (j - c) phi over the row's pupil
// pixels.  The row's T = N/E threads each hold E of its values, at the
// positions the first row transform loads (first_pos), sum them in a fixed
// order and then across the T lanes by an xor butterfly (every lane ends with
// the same bits), so the stats kernel, the work list's stats items and the
// first row pass form each row's record bit for bit alike.
// ---------------------------------------------------------------------------
template <int T>
__device__ __forceinline__ float row_sum(float x) {
#pragma unroll
  for (int off = T / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
// yv, phv, gv: the thread's y, phi and aperture bytes; phi counts on the
// pupil only, and not at all without the tip/tilt plane (with_phi = 0);
// t: the thread's lane within the row.
template <int N>
__device__ __forceinline__ void row_record(const float2 (&yv)[Plan<N>::E], const float (&phv)[Plan<N>::E],
                                           const unsigned (&gv)[Plan<N>::E], int with_phi, int t, float (&rec)[5]) {
  constexpr int E = Plan<N>::E, T = N / E;
  constexpr float c = 0.5f * (float)(N - 1);
  float sr = 0.f, si = 0.f;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    sr += yv[i].x;
    si += yv[i].y;
  }
  sr = row_sum<T>(sr);
  si = row_sum<T>(si);
  const float mr = sr * (1.0f / (float)N), mi = si * (1.0f / (float)N);
  float m2 = 0.f, p0 = 0.f, p1 = 0.f;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const float dr = yv[i].x - mr, di = yv[i].y - mi;
    m2 += dr * dr + di * di;
    const float pm = (with_phi && geo_in(gv[i])) ? phv[i] : 0.0f;
    p0 += pm;
    p1 += ((float)first_pos<N, +1>(i, t) - c) * pm;
  }
  rec[0] = sr;
  rec[1] = si;
  rec[2] = row_sum<T>(m2);
  rec[3] = row_sum<T>(p0);
  rec[4] = row_sum<T>(p1);
}
// rows per stats block (256 threads) and stats blocks per stream
template <int N>
struct StatsGeom {
  static constexpr int T = N / Plan<N>::E, RPB = 256 / T, BLOCKS = N / RPB;
};

// Body of one stats block (item: rows [item RPB, (item + 1) RPB)) of one
// stream: y is the stream's frame and cur its current state buffer; writes the
// rows' records.
template <int N>
__device__ __forceinline__ void stats_body(const StreamDesc& D, const float2* y, int cur, int item, int with_phi,
                                           int tid) {
  constexpr int E = Plan<N>::E, T = N / E;
  const int line = tid / T, t = tid - line * T;
  const int row = item * StatsGeom<N>::RPB + line;
  const auto yr = glb(y) + row * N;
  const auto phi = glb(D.phi[cur]) + row * N;
  // descriptor fields are read once, here: read inside the loops they would
  // be re-read after every store (which may alias the descriptor) and each
  // re-read waits for every memory operation in flight
  const auto geo = glb(D.geo) + row * N;
  const auto out = glb(D.part) + row * PART_STRIDE;
  // every global read is issued up front; phi is loaded at every pixel
  // (branch-free: a load under a per-pixel branch makes the compiler wait for
  // all loads in flight at each join) and masked to the pupil afterwards
  float2 yv[E];
  float phv[E];
  unsigned gv[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int n = first_pos<N, +1>(i, t);
    yv[i] = yr[n];
    phv[i] = phi[n];
    gv[i] = geo[n];
  }
  float rec[5];
  row_record<N>(yv, phv, gv, with_phi, t, rec);
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < 5; ++q) out[q] = rec[q];
  }
}

// use_args: 0 frame start from the descriptor; 1 from the arguments; 2 from
// the arguments, and the descriptor pointers too, which block 0 of each
// stream also stores in the device list dptrs for the later kernels.
template <int N>
__global__ __launch_bounds__(256) void k_stats(StreamDesc** dptrs, int with_phi, FrameArgs a, int use_args) {
  const XcdBlock xb = xcd_block();
  StreamDesc* const dp = use_args == 2 ? a.d[xb.strm] : dptrs[xb.strm];
  const auto& D = desc_ref(dp);
  // frame start: from the arguments (block 0 stores them in the descriptor
  // for the later kernels; no block of this launch reads them there) or from
  // the descriptor
  const float2* y = use_args ? a.y[xb.strm] : D.y;
  const int cur = use_args ? a.cur[xb.strm] : D.cur;
  stats_body<N>(D, y, cur, xb.item, with_phi, threadIdx.x);
  // after the body's descriptor reads (a store that may alias the
  // descriptor would make later reads of it wait for all memory in flight)
  if (use_args && xb.item == 0 && threadIdx.x == 0) {
    const auto d = glb(dp);
    d->y = a.y[xb.strm];
    d->cur = cur;
    if (use_args == 2) glb(dptrs)[xb.strm] = dp;
  }
}

// ---------------------------------------------------------------------------
// Combine the row records of one stream (fixed order, FP64) into mean, scale,
// plane coefficients and the reject flag: out[SC_*].  The block first stages
// the records in LDS (one round of global loads); the first wave then
// combines them, lane l taking rows l, l + 64, ...  The centred power is the
// rows' own centred powers plus N times the spread of the row means.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
// Stage the N row records of a stream into LDS, st[q * N + row] (5 N
// floats), with the nthr threads of the block.  ATOMIC: the records are read
// with device-coherent loads (they were written by other workgroups of the
// same launch).
template <int N, bool ATOMIC, class Desc>
__device__ __forceinline__ void stage_records(const Desc& D, float* st, int tid, int nthr) {
  const auto part = glb(D.part);
  for (int row = tid; row < N; row += nthr) {
    const auto rec = part + row * PART_STRIDE;
    float v[5];
    if constexpr (ATOMIC) {
#pragma unroll
      for (int q = 0; q < 5; ++q) v[q] = __hip_atomic_load(rec + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const float4 a = *reinterpret_cast<gptr<const float4>>(rec);
      v[0] = a.x;
      v[1] = a.y;
      v[2] = a.z;
      v[3] = a.w;
      v[4] = rec[4];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) st[q * N + row] = v[q];
  }
}
template <int N, class Desc>
__device__ __forceinline__ void combine_stats(const Desc& D, int with_phi, const float* st, float* out) {
  const int lane = threadIdx.x & 63;
  // a 32-thread block (the smallest row tiling) has each thread take lanes l
  // and l + 32 of the 64-lane tree, so that every tiling sums alike
  const bool half = blockDim.x < 64;
  constexpr int R = N / 64;  // rows per lane (N >= 64)
  // sum over the 64 lanes: first lane l with lane l ^ 32, then a butterfly
  auto tree = [&](double a0, double a1) {
    double x = half ? a0 + a1 : a0 + __shfl_xor(a0, 32, 64);
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
  };
  const double c = 0.5 * (double)(N - 1);
  double acc[2][6];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[h][q] = 0.0;
    if (h == 1 && !half) continue;
#pragma unroll 2
    for (int k = 0; k < R; ++k) {
      const int row = lane + 32 * h + 64 * k;
      acc[h][0] += st[row];
      acc[h][1] += st[N + row];
      acc[h][2] += st[2 * N + row];
      const float v3 = st[3 * N + row];
      acc[h][3] += v3;
      acc[h][4] += ((double)row - c) * (double)v3;
      acc[h][5] += st[4 * N + row];
    }
  }
  const double npx = (double)N * (double)N;
  const double mr = tree(acc[0][0], acc[1][0]) / npx, mi = tree(acc[0][1], acc[1][1]) / npx;
  // second pass over the row sums
  double dd[2] = {0.0, 0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h == 1 && !half) continue;
#pragma unroll 2
    for (int k = 0; k < R; ++k) {
      const int row = lane + 32 * h + 64 * k;
      const double er = (double)st[row] / (double)N - mr, ei = (double)st[N + row] / (double)N - mi;
      dd[h] += er * er + ei * ei;
    }
  }
  const double m2 = tree(acc[0][2], acc[1][2]) + (double)N * tree(dd[0], dd[1]);
  const double s0 = tree(acc[0][3], acc[1][3]), s1 = tree(acc[0][4], acc[1][4]), s2 = tree(acc[0][5], acc[1][5]);
  if (lane != 0) return;
  const bool ok = (m2 > 0.0) && isfinite(m2) && isfinite(mr) && isfinite(mi);
  out[SC_MU_RE] = (float)mr;
  out[SC_MU_IM] = (float)mi;
  out[SC_SCALE] = ok ? (float)sqrt(npx / m2) : 0.0f;
  out[SC_FLAG] = ok ? 0.0f : 1.0f;
  double c0 = 0, c1 = 0, c2 = 0;
  if (with_phi) {
    // least-squares plane c0 + c1 di + c2 dj over the pupil: the normal
    // equations' inverse matrix is precomputed per stream
    const auto& m = D.minv;
    c0 = m[0] * s0 + m[1] * s1 + m[2] * s2;
    c1 = m[1] * s0 + m[3] * s1 + m[4] * s2;
    c2 = m[2] * s0 + m[4] * s1 + m[5] * s2;
  }
  out[SC_C0] = (float)c0;
  out[SC_C1] = (float)c1;
  out[SC_C2] = (float)c2;
}

// k_finalize: standalone combine (diagnostic path).  grid (streams), block 64
template <int N>
__global__ __launch_bounds__(64) void k_finalize(StreamDesc* const* dptrs, int with_phi) {
  __shared__ float st[5 * N];
  const auto& D = desc_ref(dptrs[blockIdx.x]);
  stage_records<N, false>(D, st, threadIdx.x, 64);
  __syncthreads();
  combine_stats<N>(D, with_phi, st, glb(D.scal));
}

// ---------------------------------------------------------------------------
// k_row1: first half of A_phi^H yhat.  Row i: v = a exp(-j phi') (y - mu) scale,
// inverse 1-D DFT along the row (unnormalised) -> T.
// grid (N/LPW, streams), block LPW * N/E
// ---------------------------------------------------------------------------
// Body of one row1 block (item = LPW rows) of one stream with frame yf and
// current state buffer cur.  STAGE_TW: stage the twiddles into s_tw here
// (otherwise the caller has).  lds holds LPW * RowLds<N>::STRIDE entries.
// FUSE: this block also forms its rows' statistics records (the first EM
// iteration of a frame, fin), publishes them, and waits (bounded by
// spin_limit polls; a wait that gives up sets the stream's give-up word)
// until all N rows of its stream have been published before the combine;
// ctl: the stream's control words.  local: every block of the stream runs on
// this XCD, so the records go through its L2 (plain stores, completed before
// the count; the CU's L1 invalidated after the wait); otherwise they are
// written and read with device-coherent accesses.
template <int N, int LPW, bool STAGE_TW, bool FUSE = false>
__device__ __forceinline__ void row1_body(const StreamDesc& D, const float2* yf, int cur, int item,
                                          const float2* __restrict__ tw, int k, int use_plane, int fin, int with_phi,
                                          float2* lds, float2* s_tw, float* scs, int tid,
                                          gptr<unsigned> ctl = nullptr, unsigned spin_limit = 0, bool local = false) {
  constexpr int E = Plan<N>::E, T = N / E;
  const int line = tid / T, t = tid - line * T;
  const int row = item * LPW + line;
  const float* phi = glb(D.phi[(cur + k) & 1]) + row * N;
  const float2* y = glb(yf) + row * N;
  const auto geo = glb(D.geo) + row * N;  // read before any store (see k_stats)
  // global reads first (they depend on nothing computed here): the row of y,
  // phi and the aperture bytes, and the twiddle table into LDS
  float2 yv[E];
  float phv[E];
  unsigned gv[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int n = first_pos<N, +1>(i, t);
    yv[i] = y[n];
    phv[i] = phi[n];
    gv[i] = geo[n];
  }
  if (STAGE_TW)
    for (int i = tid; i < N; i += LPW * T) s_tw[i] = tw[i];
  float sc[SC_COUNT];
  if (fin) {
    if constexpr (FUSE) {
      float rec[5];
      row_record<N>(yv, phv, gv, with_phi, t, rec);
      if (t == 0) {
        const auto out = glb(D.part) + row * PART_STRIDE;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          if (local)
            out[q] = rec[q];
          else
            __hip_atomic_store(out + q, rec[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's records are stored
      __syncthreads();
      if (tid == 0) {
        ctl_add(ctl + CTL_ROWS, (unsigned)LPW);
        unsigned polls = 0;
        while (ctl_load(ctl + CTL_ROWS) < (unsigned)N) {
          if (++polls > spin_limit) {
            __hip_atomic_store(ctl + CTL_GIVEUP, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (local) l1_invalidate();
      }
      __syncthreads();
    }
    // first EM iteration of a frame: every block combines the row records
    // itself (identical arithmetic in all blocks); block 0 publishes them.
    // The records are staged in the row transform's LDS buffer, which is
    // free until the transform (5 N floats <= LPW (N + pad) float2).
    static_assert(5 * N <= 2 * LPW * RowLds<N>::STRIDE, "records do not fit the row buffer");
    float* const stg = reinterpret_cast<float*>(lds);
    if (FUSE && !local)
      stage_records<N, true>(D, stg, tid, LPW * T);
    else
      stage_records<N, false>(D, stg, tid, LPW * T);
    __syncthreads();
    if (tid < 64) combine_stats<N>(D, with_phi, stg, scs);
    __syncthreads();
    if constexpr (FUSE) {
      // the last of the stream's blocks past its wait clears the counters
      if (tid == 0 && ctl_add(ctl + CTL_ROWS_DONE, 1u) + 1 == (unsigned)(N / LPW)) {
        __hip_atomic_store(ctl + CTL_ROWS, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(ctl + CTL_ROWS_DONE, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(ctl + CTL_XCC, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (item == 0 && tid < SC_COUNT) glb(D.scal)[tid] = scs[tid];
#pragma unroll
    for (int q = 0; q < SC_COUNT; ++q) sc[q] = scs[q];
  } else {
#pragma unroll
    for (int q = 0; q < SC_COUNT; ++q) sc[q] = glb(D.scal)[q];
  }
  if (sc[SC_FLAG] != 0.0f) return;
  const float2 mu = make_float2(sc[SC_MU_RE], sc[SC_MU_IM]);
  const float scale = sc[SC_SCALE];
  const float c0 = sc[SC_C0], c1 = sc[SC_C1], c2 = sc[SC_C2];
  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int n = first_pos<N, +1>(i, t);
    if (geo_in(gv[i])) {
      const float p = use_plane ? phv[i] - plane_val(c0, c1, c2, row, n, N) : phv[i];
      float sn, cs;
      fsincos(p, &sn, &cs);
      const float2 yh = make_float2((yv[i].x - mu.x) * scale, (yv[i].y - mu.y) * scale);
      v[i] = cmul(yh, make_float2(cs, -sn));
    } else {
      v[i] = make_float2(0.f, 0.f);
    }
  }
  RowLds<N> L{lds + line * RowLds<N>::STRIDE};
  line_fft<N, +1>(v, t, L, s_tw);
  float2* out = glb(D.T) + row * N;
#pragma unroll
  for (int i = 0; i < E; ++i) out[last_pos<N, +1>(i, t)] = v[i];
}

template <int N, int LPW>
__global__ __launch_bounds__(LPW*(N / Plan<N>::E)) void k_row1(StreamDesc* const* dptrs, const float2* __restrict__ tw,
                                                             int k, int use_plane, int fin, int with_phi) {
  __shared__ float2 lds[LPW * RowLds<N>::STRIDE];
  __shared__ float2 s_tw[N];
  __shared__ float scs[SC_COUNT];
  const XcdBlock xb = xcd_block();
  const auto& D = desc_ref(dptrs[xb.strm]);
  row1_body<N, LPW, true>(D, D.y, D.cur, xb.item, tw, k, use_plane, fin, with_phi, lds, s_tw, scs, threadIdx.x);
}

// ---------------------------------------------------------------------------
// k_row1s: the first row pass of a frame's first EM iteration with the
// Normalize and RemoveTipTilt statistics formed in the same launch (no
// separate stats launch).  Each block forms its rows' records, publishes them
// (through the XCD's L2 when every block of its stream runs on one XCD,
// device-coherent otherwise; see row1_body) and waits until its stream's N
// rows are all published, then combines them like k_row1.  Blocks map to (row block,
// stream) as in the other frame kernels (a stream's blocks consecutive on one
// XCD), and the dispatcher starts blocks in increasing order, so when a
// block waits, every earlier block has started and a stream's other blocks
// are among the next to start once earlier streams' blocks end: no deadlock.
// Waits are bounded all the same: one that gives up sets the stream's give-up
// word.  Four waves per SIMD (no spill at N <= 256): the row data stay live
// through the wait, and at three waves per SIMD a 64-stream batch needed a
// second, partial generation of blocks (37 against 29 us at 64 x N = 256).
// grid (N/LPW, streams), block LPW * N/E
// ---------------------------------------------------------------------------
template <int N, int LPW>
__global__ __launch_bounds__(LPW*(N / Plan<N>::E)) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_row1s(StreamDesc** dptrs, FrameArgs a, int use_args,
                                                              const float2* __restrict__ tw, int with_phi,
                                                              unsigned spin_limit, int nq) {
  __shared__ float2 lds[LPW * RowLds<N>::STRIDE];
  __shared__ float2 s_tw[N];
  __shared__ float scs[SC_COUNT];
  const XcdBlock xb = xcd_block();
  StreamDesc* const dp = use_args == 2 ? a.d[xb.strm] : dptrs[xb.strm];
  const auto& D = desc_ref(dp);
  const float2* y = use_args ? a.y[xb.strm] : D.y;
  const int cur = use_args ? a.cur[xb.strm] : D.cur;
  // Workgroups go to the 8 XCDs round-robin in linear order (from whichever
  // XCD the dispatch starts at), so xcd_block's grouping by linear index mod
  // 8 puts every block of a stream on one XCD when 8 divides the streams and
  // the device has 8 XCDs.  The protocol relies on that, so each block checks
  // it: the first block of the stream to arrive records its XCC_ID, and a
  // block on another XCD marks the stream's frame as failed.
  const bool local = nq == 8 && gridDim.y % 8 == 0;
  if (local && threadIdx.x == 0) {
    const unsigned me = xcc_id() + 1u;  // 0: not yet recorded
    unsigned seen = 0u;
    if (!__hip_atomic_compare_exchange_strong(glb(D.ctl) + CTL_XCC, &seen, me, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT) &&
        seen != me)
      __hip_atomic_store(glb(D.ctl) + CTL_GIVEUP, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  row1_body<N, LPW, true, true>(D, y, cur, xb.item, tw, 0, with_phi, 1, with_phi, lds, s_tw, scs, threadIdx.x,
                                glb(D.ctl), spin_limit, local);
  // after the body's descriptor reads: the frame start for the later kernels
  if (use_args && xb.item == 0 && threadIdx.x == 0) {
    const auto d = glb(dp);
    d->y = y;
    d->cur = cur;
    if (use_args == 2) glb(dptrs)[xb.strm] = dp;
  }
}

// ---------------------------------------------------------------------------
// k_col: column strip of W columns.  Inverse 1-D DFT down each column and the
// 1/N scale give b = A_phi^H yhat; then per pixel the Eq. (3) initialisation
// (first EM iteration of a frame), the E-step mu = r/(r+s2) b, |b|^2 -> bb,
// and the forward 1-D DFT of mu down the column (unnormalised) -> U.
// grid (N/W, streams), block W * N/E
// ---------------------------------------------------------------------------
// Body of one column-pass block (item = W columns) of one stream with
// current state buffer cur; lds holds N * ColLds<W>::STRIDE entries.
template <int N, int W, bool STAGE_TW>
__device__ __forceinline__ void col_body(const StreamDesc& D, int cur, int item, const float2* __restrict__ tw, int k,
                                         int do_rinit, int mat, float2* lds, float2* s_tw, int tid) {
  constexpr int E = Plan<N>::E;
  const int w = tid % W, t = tid / W;
  const int col = item * W + w;
  float2 v[E];
  float rpv[E];
  const float* rin = glb(D.r[(cur + k) & 1]);
  float* rmat = glb(D.r[((cur + k) & 1) ^ 1]);
  // output pointers and constants are read before any store (see k_stats)
  float* bbo = glb(D.bb);
  float2* uo = glb(D.U);
  const float s2 = D.sigma2, lam = D.lam, alpha = D.alpha, fl = D.r_floor;
  // global reads first: the column, this thread's r values, the twiddles
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = glb(D.T)[first_pos<N, +1>(i, t) * N + col];
#pragma unroll
  for (int i = 0; i < E; ++i) rpv[i] = rin[last_pos<N, +1>(i, t) * N + col];
  if (STAGE_TW)
    for (int i = tid; i < N; i += W * (N / E)) s_tw[i] = tw[i];
  if (glb(D.scal)[SC_FLAG] != 0.0f) return;
  ColLds<W> L{lds + w};
  line_fft<N, +1>(v, t, L, s_tw);
  const float invN = 1.0f / (float)N;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int n = last_pos<N, +1>(i, t);
    const float2 b = cscale(v[i], invN);
    const float bb = b.x * b.x + b.y * b.y;
    const float rp = rpv[i];
    const float ri = do_rinit ? rinit_of(rp, bb, lam, alpha, fl) : rp;
    const float wgt = wiener_of(ri, s2);
    bbo[n * N + col] = bb;
    if (mat) rmat[n * N + col] = ri;  // the whole-image colour passes update this copy in place
    v[i] = cscale(b, wgt);
  }
  __syncthreads();
  line_fft<N, -1>(v, t, L, s_tw);
#pragma unroll
  for (int i = 0; i < E; ++i) uo[last_pos<N, -1>(i, t) * N + col] = v[i];
}

template <int N, int W>
__global__ __launch_bounds__(W*(N / Plan<N>::E)) void k_col(StreamDesc* const* dptrs, const float2* __restrict__ tw,
                                                          int k, int do_rinit, int mat) {
  __shared__ float2 lds[N * ColLds<W>::STRIDE];
  __shared__ float2 s_tw[N];
  const XcdBlock xb = xcd_block();
  const auto& D = desc_ref(dptrs[xb.strm]);
  col_body<N, W, true>(D, D.cur, xb.item, tw, k, do_rinit, mat, lds, s_tw, threadIdx.x);
}

// ---------------------------------------------------------------------------
// atan2 in (-pi, pi]: reduction to a = min(|x|,|y|)/max(|x|,|y|) in [0, 1],
// atan(a) = a + a u Q(u), u = a^2, with a degree-7 Q fitted here (Lawson-
// weighted least squares towards the minimax of the absolute error on
// [0, 1]; FP32 evaluation error below 7e-8 absolute and 1e-7 relative),
// then the octant and quadrant reflections.  atan2(0, 0) = 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fatan2(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float a = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const float u = a * a;
  float q = 2.622134222e-03f;
  q = __builtin_fmaf(q, u, -1.513207969e-02f);
  q = __builtin_fmaf(q, u, 4.112108693e-02f);
  q = __builtin_fmaf(q, u, -7.366637325e-02f);
  q = __builtin_fmaf(q, u, 1.057389778e-01f);
  q = __builtin_fmaf(q, u, -1.418596587e-01f);
  q = __builtin_fmaf(q, u, 1.999039534e-01f);
  q = __builtin_fmaf(q, u, -3.333298699e-01f);
  float r = __builtin_fmaf(a * u, q, a);
  r = ay > ax ? 1.57079632679489662f - r : r;
  r = x < 0.0f ? 3.14159265358979324f - r : r;
  return copysignf(r, y);
}

// ---------------------------------------------------------------------------
// k_row2: forward 1-D DFT along rows of U and the 1/N scale give z = F mu.
// Per pupil pixel, the phase data term -c cos(phi - theta),
// c = (2/s2)|yhat||z|, theta = arg(yhat conj z), is majorised at
// x0 = wrap(phi' - theta) by (kappa/2)(phi - theta~)^2 with kappa = c sinc(x0),
// theta~ = phi' - x0.  Writes (kappa, theta~) into T on the pupil (T keeps
// the first row pass's values elsewhere).
// ---------------------------------------------------------------------------
// Body of one row2 block (item = LPW rows) of one stream with frame yf and
// current state buffer cur.
template <int N, int LPW, bool STAGE_TW>
__device__ __forceinline__ void row2_body(const StreamDesc& D, const float2* yf, int cur, int item,
                                          const float2* __restrict__ tw, int k, int use_plane, int mat, float2* lds,
                                          float2* s_tw, int tid) {
  constexpr int E = Plan<N>::E, T = N / E;
  const float* sc = glb(D.scal);
  const int line = tid / T, t = tid - line * T;
  const int row = item * LPW + line;
  if (STAGE_TW)
    for (int i = tid; i < N; i += LPW * T) s_tw[i] = tw[i];
  float2 v[E];
  const float2* u = glb(D.U) + row * N;
  const float* phi = glb(D.phi[(cur + k) & 1]) + row * N;
  const float2* y = glb(yf) + row * N;
  // descriptor fields are read before any store (see k_stats)
  const auto geo = glb(D.geo) + row * N;
  const float c2s = 2.0f / D.sigma2;
  float2* out = glb(D.T) + row * N;
  float* pmat = glb(D.phi[((cur + k) & 1) ^ 1]) + row * N;
  // every global read is issued up front: the aperture bytes at this
  // thread's output positions (first: the loads below wait for them), the
  // row, and y and phi at the output positions that lie in the pupil
  float2 yv[E];
  float phv[E];
  unsigned gv[E];
#pragma unroll
  for (int i = 0; i < E; ++i) gv[i] = geo[last_pos<N, -1>(i, t)];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = u[first_pos<N, -1>(i, t)];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int m = last_pos<N, -1>(i, t);
    yv[i] = make_float2(0.f, 0.f);
    phv[i] = 0.f;
    if (geo_in(gv[i])) {
      yv[i] = y[m];
      phv[i] = phi[m];
    }
  }
  if (sc[SC_FLAG] != 0.0f) return;
  RowLds<N> L{lds + line * RowLds<N>::STRIDE};
  line_fft<N, -1>(v, t, L, s_tw);
  const float invN = 1.0f / (float)N;
  const float2 mu = make_float2(sc[SC_MU_RE], sc[SC_MU_IM]);
  const float scale = sc[SC_SCALE];
  const float c0 = sc[SC_C0], c1 = sc[SC_C1], c2 = sc[SC_C2];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int m = last_pos<N, -1>(i, t);
    // (kappa, theta~) only on the pupil: their readers (the phi update of
    // the M-step) use them nowhere else
    if (geo_in(gv[i])) {
      const float2 z = cscale(v[i], invN);
      const float2 yh = make_float2((yv[i].x - mu.x) * scale, (yv[i].y - mu.y) * scale);
      const float p = use_plane ? phv[i] - plane_val(c0, c1, c2, row, m, N) : phv[i];
      // w = exp(j p) conj(yhat) z: |w| = |yhat||z| and arg w = p - theta, so
      // x0 = arg w lies in [-pi, pi] already (kappa is zero at +-pi) and
      // c sin(x0) = (2/s2) Im w.
      float sn, cs;
      fsincos(p, &sn, &cs);
      const float qr = yh.x * z.x + yh.y * z.y, qi = yh.x * z.y - yh.y * z.x;  // conj(yhat) z
      const float wr = cs * qr - sn * qi, wi = sn * qr + cs * qi;
      const float x0 = fatan2(wi, wr);
      // kappa = c sinc(x0) = (2/s2) |w| sin(x0)/x0 = (2/s2) Im(w)/x0 (x0 = 0: w real, |w| = Re w)
      const float ka = x0 != 0.0f ? c2s * wi * __builtin_amdgcn_rcpf(x0) : c2s * wr;
      out[m] = make_float2(ka, p - x0);
      if (mat) pmat[m] = p;  // the colour passes update this copy in place
    }
  }
}

template <int N, int LPW>
__global__ __launch_bounds__(LPW*(N / Plan<N>::E)) void k_row2(StreamDesc* const* dptrs, const float2* __restrict__ tw,
                                                             int k, int use_plane, int mat) {
  __shared__ float2 lds[LPW * RowLds<N>::STRIDE];
  __shared__ float2 s_tw[N];
  const XcdBlock xb = xcd_block();
  const auto& D = desc_ref(dptrs[xb.strm]);
  row2_body<N, LPW, true>(D, D.y, D.cur, xb.item, tw, k, use_plane, mat, lds, s_tw, threadIdx.x);
}

// ---------------------------------------------------------------------------
// k_frame: the stats, row1, column and row2 stages of `count` streams of one
// N as one persistent work list.  Each workgroup repeatedly claims the next
// ticket of its XCD's queue and runs that item with the same block body as
// the eager kernel of its stage, so every result is bit for bit the eager
// path's.
//
// Work list.  Stream s is dealt to queue s % nq.  A queue's items are
// numbered slot by slot: at slot j the stats items of the queue's stream j,
// the row1 items of its stream j - lag, the column items of j - 2 lag and
// the row2 items of j - 3 lag, those streams that exist (without a stats
// stage, k > 0, the other stages move up one place).  An item waits until
// every item of the previous stage of its stream has completed; those carry
// smaller numbers of the same queue.  A workgroup claims its next number
// while it runs its current item; the smallest unfinished item is then always
// some workgroup's current item (a workgroup's claimed-ahead item is larger
// than its current one), and every item it waits on is smaller, hence
// finished: the list cannot deadlock.  Waits are bounded by spin_limit polls;
// a wait that gives up sets the stream's give-up word and the item runs
// anyway, so every workgroup ends (giveup != 0 forces this, for tests).
//
// Coherence.  A workgroup claims from the queue of the XCD it runs on (the
// hardware XCC_ID register), so every item of a stream runs on one XCD, whose
// L2 all its CUs share: synchronisation is at XCD scope, as for a workgroup
// split over CUs.  Release: each wave's stores have completed at the L2
// (vmcnt(0)) before the barrier after which the completion count is
// incremented there.  Acquire: the waiting wave reads the count at the L2
// and then invalidates its CU's L1 before the barrier that lets the item's
// waves read, so no line cached on this CU before the producers wrote it is
// read.  (Agent-scope fences, which write back and invalidate the L2 at every
// item, are not needed for this and cost about twice the step time.)  Frame
// arguments reach every stage from the kernel arguments, so no stage reads a
// descriptor field that this launch writes.
//
// Every queue is served only if the dispatcher places workgroups on every
// XCD (it deals them out round-robin; the grid is a multiple of nq).  The
// last workgroup to finish checks that every queue's tickets were all
// claimed and otherwise sets the give-up word of that queue's streams, so
// such a frame is reported, not silently left undone.
// The last workgroup to finish resets the queue tickets, and the last row2
// item of a stream its stage counters, so the next launch starts from zero.
// grid: persistent, a multiple of nq; block 256 (LPW, W chosen so that each
// stage's block is 256 threads).
// ---------------------------------------------------------------------------
template <int N>
struct FrameTiles {  // rows per row item and columns per column item at 256 threads
  static constexpr int T = N / Plan<N>::E;
  static constexpr int LPW = 256 / T, W = 256 / T;
  static constexpr int ROWL = LPW * RowLds<N>::STRIDE, COLL = N * ColLds<W>::STRIDE;
  static constexpr int LDS = ROWL > COLL ? ROWL : COLL;
};


template <int N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_frame(StreamDesc** dptrs, int count, FrameArgs a, int use_args,
                                               const float2* __restrict__ tw, int k, int mode, unsigned* ctl0,
                                               int nq, int lag, unsigned spin_limit, int giveup, int mat) {
  using FT = FrameTiles<N>;
  constexpr int LPW = FT::LPW, W = FT::W;
  __shared__ float2 lds[FT::LDS];
  __shared__ float2 s_tw[N];
  __shared__ float scs[SC_COUNT];
  __shared__ int s_ticket;
  const int fin = k == 0, first = (mode && k == 0) ? 1 : 0;
  const int nA = fin ? StatsGeom<N>::BLOCKS : 0, nB = N / LPW, nC = N / W, nD = N / LPW;
  const int s0 = fin ? 0 : 1;  // first stage present
  const int q = (int)(xcc_id() % (unsigned)nq);
  const int Sq = q < count ? (count - q + nq - 1) / nq : 0;
  const int need[4] = {nA, nB, nC, nD};
  const int tickets = Sq * (nA + nB + nC + nD);  // only real items are numbered
  for (int i = threadIdx.x; i < N; i += 256) s_tw[i] = tw[i];
  if (threadIdx.x == 0) {
    s_ticket = (int)atomicAdd(ctl0 + CTL_TICKETS + q, 1u);
    lds_stores_done();
  }
  int next = 0;  // thread 0: the ticket claimed ahead for the next item
  for (;;) {
    __syncthreads();  // s_ticket is written, and the previous item is done with the LDS
    const int t = s_ticket;
    if (t >= tickets) break;
    // claim the next item now: the atomic's round trip overlaps this item
    if (threadIdx.x == 0) next = (int)atomicAdd(ctl0 + CTL_TICKETS + q, 1u);
    // ticket -> (stage, queue position of the stream, item): walk the slots;
    // at slot j the queue's streams j, j - lag, j - 2 lag, j - 3 lag (those
    // in range) contribute the items of stages s0, s0 + 1, ... in that order
    int stage = s0, jq = 0, item = 0;
    {
      int rem = t;
      for (int j = 0;; ++j) {
        bool found = false;
        for (int st = s0; st < 4; ++st) {
          const int i = j - (st - s0) * lag;
          if (i < 0 || i >= Sq) continue;
          if (rem < need[st]) {
            stage = st;
            jq = i;
            item = rem;
            found = true;
            break;
          }
          rem -= need[st];
        }
        if (found) break;
      }
    }
    const int strm = jq * nq + q;
    // the thread index, opaque to the compiler in each item: otherwise every
    // stage's per-thread index arithmetic is hoisted out of the loop and all
    // of it stays live at once
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    StreamDesc* const dp = use_args == 2 ? a.d[strm] : dptrs[strm];
    const auto& D = desc_ref(dp);
    const float2* y = use_args ? a.y[strm] : D.y;
    const int cur = use_args ? a.cur[strm] : D.cur;
    const auto ctl = glb(D.ctl);  // global, not flat, atomics
    // ---- wait for the previous stage of this stream
    if (stage > s0) {
      if (threadIdx.x == 0) {
        unsigned polls = 0;
        while (giveup || ctl_load(ctl + CTL_STAGE + stage - 1) < (unsigned)need[stage - 1]) {
          if (giveup || ++polls > spin_limit) {
            __hip_atomic_store(ctl + CTL_GIVEUP, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        // acquire within the XCD: this CU's L1 is invalidated, so the loads
        // below miss to the L2 that the producers' stores have reached
        l1_invalidate();
      }
      __syncthreads();
    }
    // ---- the item (block bodies of the eager kernels)
    if (stage == 0) {
      stats_body<N>(D, y, cur, item, mode, tid);
      if (use_args && item == 0 && threadIdx.x == 0) {
        // the later launches of the frame (M-step, diagnostics) read these
        const auto d = glb(dp);
        d->y = y;
        d->cur = cur;
        if (use_args == 2) glb(dptrs)[strm] = dp;
      }
    } else if (stage == 1) {
      row1_body<N, LPW, false>(D, y, cur, item, tw, k, first, fin, mode, lds, s_tw, scs, tid);
    } else if (stage == 2) {
      col_body<N, W, false>(D, cur, item, tw, k, first, mat, lds, s_tw, tid);
    } else {
      row2_body<N, LPW, false>(D, y, cur, item, tw, k, first, mat, lds, s_tw, tid);
    }
    // ---- completion (release within the XCD): every wave's stores have
    // reached the L2 (vmcnt(0)) before the barrier, and the count follows it
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned done = ctl_add(ctl + CTL_STAGE + stage, 1u);
      if (stage == 3 && done + 1 == (unsigned)nD) {
        for (int g = 0; g < 4; ++g) __hip_atomic_store(ctl + CTL_STAGE + g, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      s_ticket = next;
      lds_stores_done();
    }
  }
  if (threadIdx.x == 0 && atomicAdd(ctl0 + CTL_FINISHED, 1u) + 1 == gridDim.x) {
    // a queue that no workgroup served (the dispatcher put none on its XCD)
    // left its streams' items undone: their give-up words say so
    for (int g = 0; g < nq && g < count; ++g) {
      const int sq = (count - g + nq - 1) / nq;
      // read with an atomic: the counter was updated on another XCD
      if (atomicAdd(ctl0 + CTL_TICKETS + g, 0u) < (unsigned)(sq * (nA + nB + nC + nD)))
        for (int j = 0; j < sq; ++j) {
          const int strm = j * nq + g;
          StreamDesc* const dp = use_args == 2 ? a.d[strm] : dptrs[strm];
          __hip_atomic_store(glb(desc_ref(dp).ctl) + CTL_GIVEUP, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    for (int g = 0; g < CTL_MAX_QUEUES; ++g)
      __hip_atomic_store(ctl0 + CTL_TICKETS + g, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(ctl0 + CTL_FINISHED, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Fast single-instruction math (v_rcp_f32, v_exp_f32, v_log_f32, v_sqrt_f32,
// v_cos_f32: about 1 ulp on normal inputs).  Every cubic root found with them
// is polished by Newton steps on the cubic itself, so their error does not
// reach the result beyond a few ulp.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fcbrt(float x) {  // real cube root
  DDH_EXACT_FP
  const float m = fexp2(flog2(fabsf(x)) * (1.0f / 3.0f));
  return copysignf(m, x);
}
__device__ __forceinline__ float fcos_rev(float rev) { return __builtin_amdgcn_cosf(rev); }  // cos(2 pi rev)

// ---------------------------------------------------------------------------
// r M-step pixel solve: global minimiser on (0, inf) of
//   h(rho) = log rho + s/rho + (A/2) rho^2 - B rho
// via the stationarity cubic A rho^3 - B rho^2 + rho - s = 0 (all real roots
// are positive for s > 0, A > 0, B >= 0).  One real root: Cardano; three:
// trigonometric form; each root polished by guarded Newton steps (one for the
// Cardano root, whose FP32 error is within a few ulp after one step; two for
// the trigonometric roots).  With three
// roots the middle one is a local maximum of h; the outer two are compared by
// h(rho1) - h(rho3) written as one difference; ties take the smaller root.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float cubic_f(float A, float B, float s, float x) {
  DDH_EXACT_FP
  return __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(A, x, -B), x, 1.0f), x, -s);
}
// Guarded Newton steps on the cubic; A3 = 3A and B2 = 2B are the derivative's
// coefficients, formed once per pixel by the caller.
template <int IT>
__device__ __forceinline__ float polish(float A, float B, float A3, float B2, float s, float x) {
  DDH_EXACT_FP
  float f = cubic_f(A, B, s, x);
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const float fp = __builtin_fmaf(__builtin_fmaf(A3, x, -B2), x, 1.0f);
    const float xn = __builtin_fmaf(-f, frcp(fp), x);
    const float fn = cubic_f(A, B, s, xn);
    const bool take = (xn > 0.0f) && (fabsf(fn) < fabsf(f));
    x = take ? xn : x;
    f = take ? fn : f;
  }
  return x;
}
// Depressed form: rho = t + b3 with b3 = B/(3A), c = 1/A, gives
// t^3 + p t + q = 0, p = c - 3 b3^2, q = c (b3 - s) - 2 b3^3, and the
// discriminant q^2/4 + p^3/27 (>= 0: one real root).
__device__ __forceinline__ float solve_r(float s, float A, float B) {
  DDH_EXACT_FP
  if (!(A > 0.0f)) return s;
  const float c = frcp(A);
  const float b3 = (B * c) * (1.0f / 3.0f);
  const float p = __builtin_fmaf(-3.0f * b3, b3, c);
  const float b3sq = b3 * b3;
  const float q = __builtin_fmaf(c, b3 - s, (-2.0f * b3sq) * b3);
  const float disc = __builtin_fmaf(0.25f * q, q, (p * (1.0f / 27.0f)) * (p * p));
  const float A3 = 3.0f * A, B2 = 2.0f * B;
  if (disc >= 0.0f || p >= 0.0f) {
    const float sq = fsqrt(fmaxf(disc, 0.0f));
    const float u = fcbrt(__builtin_fmaf(-0.5f, q, -copysignf(sq, q)));
    const float t = (u != 0.0f) ? __builtin_fmaf(-p, frcp(3.0f * u), u) : 0.0f;
    float x = t + b3;
    if (!(x > 0.0f) || !isfinite(x)) x = s;
    return polish<1>(A, B, A3, B2, s, x);
  }
  // three real roots: t_k = 2 m cos(th - k/3 rev), m = sqrt(-p/3),
  // th = acos(arg)/3 in [0, 1/6] rev; k = 0 gives the largest root and
  // k = 2 the smallest (the middle one is a local maximum of h)
  const float m = fsqrt(-p * (1.0f / 3.0f));
  float arg = (1.5f * q * frcp(p)) * fsqrt(-3.0f * frcp(p));
  arg = fminf(1.0f, fmaxf(-1.0f, arg));
  const float th = acosf(arg) * (1.0f / (6.0f * 3.14159265358979323846f));
  float hi = __builtin_fmaf(2.0f * m, fcos_rev(th), b3);
  float lo = __builtin_fmaf(2.0f * m, fcos_rev(th - (2.0f / 3.0f)), b3);
  if (!(lo > 0.0f)) lo = fminf(s, hi);
  lo = polish<2>(A, B, A3, B2, s, lo);
  hi = polish<2>(A, B, A3, B2, s, hi);
  // h(lo) - h(hi) as one difference
  const float dh = 0.69314718055994531f * flog2(lo * frcp(hi)) + s * (hi - lo) * frcp(lo * hi) +
                   (lo - hi) * (0.5f * A * (lo + hi) - B);
  return dh <= 0.0f ? lo : hi;
}

// rho'(d)/d of the QGGMRF prior for p = 2:
//   (1/sig^2) (1 + (q/2) v) / (1 + v)^2,  v = |d/(T sig)|^(2-q)
// evaluated as u (q/2 + (1 - q/2) u) with u = 1/(1 + v) and
// log2 v = (2-q) log2|d| + lc, lc = (2-q) log2(1/(T sig)).  q = 2 (the
// quadratic prior, v = 1 for every d) arrives as pmq = 1e-30 and lc = -256,
// which give v = 0 for every d, d = 0 included, with inv_sp halved.  inv_sp
// is folded into the neighbour weights by the caller.
__device__ __forceinline__ float qg_shape(float d, float lc, float pmq, float qop) {
  DDH_EXACT_FP
  const float v = fexp2(__builtin_fmaf(pmq, flog2(fabsf(d)), lc));
  const float u = frcp(1.0f + v);
  return u * __builtin_fmaf(1.0f - qop, u, qop);
}

// ---------------------------------------------------------------------------
// Per-pixel M-step arithmetic shared by the halo-tiled kernel and the
// whole-image colour passes, written with explicit FMAs so that both produce
// bit-identical results.  Neighbour order: up, down, left, right, up-left,
// up-right, down-left, down-right (edges weight 1/6, diagonals 1/12).
// ---------------------------------------------------------------------------
// neighbour-existence mask bits of a pixel at the grid border
enum : int { NB_UP = 1, NB_DN = 2, NB_LF = 4, NB_RT = 8, NB_ALL = 15 };
__device__ __forceinline__ int nb_mask(int gi, int gj, int N) {
  return (gi > 0 ? NB_UP : 0) | (gi < N - 1 ? NB_DN : 0) | (gj > 0 ? NB_LF : 0) | (gj < N - 1 ? NB_RT : 0);
}
// r update of one pixel from its 8 neighbours, with the edge and diagonal
// prior weights wE = inv_sp/6 and wD = inv_sp/12.  CHECK: some neighbours may
// be off the grid (mask bits clear); their weight is zero and their staged
// value is finite.
template <bool CHECK>
__device__ __forceinline__ float r_pixel_w(float rp, float s, const float (&rq)[8], int mask, float wE, float wD,
                                           float lc, float pmq, float qop, float fl) {
  DDH_EXACT_FP
  float Ae = 0.f, Be = 0.f, Ad = 0.f, Bd = 0.f;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float sh = qg_shape(rp - rq[e], lc, pmq, qop);
    if (CHECK) {
      constexpr int need[8] = {NB_UP, NB_DN, NB_LF, NB_RT, NB_UP | NB_LF, NB_UP | NB_RT, NB_DN | NB_LF, NB_DN | NB_RT};
      sh = ((mask & need[e]) == need[e]) ? sh : 0.f;
    }
    if (e == 0 || e == 4) {  // first term of each sum (shapes are >= +0)
      (e == 0 ? Ae : Ad) = sh;
      (e == 0 ? Be : Bd) = sh * rq[e];
    } else if (e < 4) {
      Ae += sh;
      Be = __builtin_fmaf(sh, rq[e], Be);
    } else {
      Ad += sh;
      Bd = __builtin_fmaf(sh, rq[e], Bd);
    }
  }
  const float A = __builtin_fmaf(wE, Ae, wD * Ad), B = __builtin_fmaf(wE, Be, wD * Bd);
  return fmaxf(solve_r(s, A, B), fl);
}

// the same with the weights formed from inv_sp = 1/sigma^p
template <bool CHECK>
__device__ __forceinline__ float r_pixel(float rp, float s, const float (&rq)[8], int mask, float inv_sp,
                                         float lc, float pmq, float qop, float fl) {
  return r_pixel_w<CHECK>(rp, s, rq, mask, inv_sp * (1.0f / 6.0f), inv_sp * (1.0f / 12.0f), lc, pmq, qop, fl);
}
// phi update of one pupil pixel; pq holds the neighbours' phases (zero off
// the pupil and off the grid), P the prior weight of the pupil neighbours
__device__ __forceinline__ float phi_pixel(const float (&pq)[8], float P, float ka, float tt, float beta2,
                                           float cur) {
  DDH_EXACT_FP
  const float se = (pq[0] + pq[1]) + (pq[2] + pq[3]);
  const float sd = (pq[4] + pq[5]) + (pq[6] + pq[7]);
  const float Ph = __builtin_fmaf(1.0f / 6.0f, se, (1.0f / 12.0f) * sd);
  const float den = __builtin_fmaf(beta2, P, ka);
  return den > 0.0f ? __builtin_fmaf(ka, tt, beta2 * Ph) * frcp(den) : cur;
}
// prior weight of the pupil neighbours of a pupil pixel, as twelfths:
// 2 per edge neighbour and 1 per diagonal neighbour inside the pupil
__device__ __forceinline__ int pupil_nbr_12(int gi, int gj, int N, float d2) {
  const int nb[8][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {-1, 1}, {1, -1}, {1, 1}};
  int n12 = 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ii = gi + nb[e][0], jj = gj + nb[e][1];
    if (ii >= 0 && ii < N && jj >= 0 && jj < N && in_pupil(ii, jj, N, d2)) n12 += e < 4 ? 2 : 1;
  }
  return n12;
}
__device__ __forceinline__ float pupil_weight_of(int n12) { return (float)n12 * (1.0f / 12.0f); }

constexpr int MS_THREADS = 256;

// compile-time loop: f(std::integral_constant<int, I>) for I in [I0, I1)
template <int I0, int I1, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I0 < I1) {
    f(std::integral_constant<int, I0>{});
    static_for<I0 + 1, I1>(f);
  }
}

// Geometry of the halo-tiled sweep: region RH x RW = (TH + 8) x (TW + 8);
// pass c updates the colour-c pixels of rows/cols [c+1, R-c-1).  Tile origins
// are even, so local parities equal global ones and everything is static.
template <int TH, int TW>
struct MsGeom {
  static constexpr int RH = TH + 8, RW = TW + 8, RP = RH * RW;
  static constexpr int li0(int c) { return (((c + 1) & 1) == (c & 1)) ? c + 1 : c + 2; }
  static constexpr int lj0(int c) { return (((c + 1) & 1) == (c >> 1)) ? c + 1 : c + 2; }
  static constexpr int nu(int c) { return (RH - c - 1 - li0(c) + 1) / 2; }
  static constexpr int nv(int c) { return (RW - c - 1 - lj0(c) + 1) / 2; }
  static constexpr int n(int c) { return nu(c) * nv(c); }
  // block size: one round per pass when the first (largest) pass fits in 1024 threads
  static constexpr int BT = ((n(0) + 63) / 64) * 64 <= 1024 ? ((n(0) + 63) / 64) * 64 : MS_THREADS;
  static constexpr int rounds(int c) { return (n(c) + BT - 1) / BT; }
  static constexpr int slot0(int c) { return c == 0 ? 0 : slot0(c - 1) + rounds(c - 1); }
  static constexpr int SLOTS = rounds(0) + rounds(1) + rounds(2) + rounds(3);
};

// ---------------------------------------------------------------------------
// k_mstep: one 4-colour sweep of the r and phi M-steps on a TH x TW output
// tile.  The tile and a 4-pixel halo of r and phi are staged in LDS; pass c
// updates the colour-c pixels of the region shrunk by c+1, so the inner tile
// sees exactly the values a whole-grid sweep produces.  All global reads of
// a block are issued before the first wait.  r is staged after the Eq. (3)
// initialisation; s = E|g|^2 is formed only at the pixels a thread updates
// (no neighbour needs it); each thread keeps the per-pixel constants of those
// pixels (LDS offset, border mask, s, pupil-neighbour weight, kappa, theta~)
// in registers.  Colour(i, j) = (i mod 2) + 2 (j mod 2).  Reads state buffer
// in = (cur + k) & 1, writes in ^ 1.  grid (tiles, streams), block BT (the
// first pass's pixel count rounded up to whole waves); blocks are remapped
// so that neighbouring tiles of a stream run on the same XCD (shared L2 for
// the halo).
// ---------------------------------------------------------------------------
template <int N, int TH, int TW>
__global__ __launch_bounds__((MsGeom<TH, TW>::BT)) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_mstep(StreamDesc* const* dptrs, int k, int use_plane,
                                                                                                        int do_rinit) {
  using G = MsGeom<TH, TW>;
  constexpr int BT = G::BT;
  constexpr int RW = G::RW, RP = G::RP, SLOTS = G::SLOTS;
  constexpr int TPC = N / TW, TPR = N / TH;
  constexpr int TILES = TPC * TPR;
  constexpr int offs[8] = {-RW, RW, -1, 1, -RW - 1, -RW + 1, RW - 1, RW + 1};
  __shared__ __align__(16) float sR[RP], sP[RP];
  const int total = TILES * gridDim.y;
  const int L = blockIdx.x + blockIdx.y * TILES;
  const int logical = (total % 8 == 0) ? (L % 8) * (total / 8) + (L / 8) : L;
  const int g = logical / TILES, tile = logical - g * TILES;
  const auto& D = desc_ref(dptrs[g]);
  const int ti = tile / TPC, tj = tile - ti * TPC;
  const int gi0 = ti * TH - 4, gj0 = tj * TW - 4;
  const int in = (D.cur + k) & 1;
  // global (address space 1) pointers throughout: through generic pointers
  // the compiler emits flat loads, which also count against the LDS wait
  // counter
  const auto rin = glb(D.r[in]);
  const auto pin = glb(D.phi[in]);
  const auto rout = glb(D.r[in ^ 1]);
  const auto pout = glb(D.phi[in ^ 1]);
  const auto sc = glb(D.scal);
  const float s2 = D.sigma2, lam = D.lam, alpha = D.alpha, fl = D.r_floor, beta2 = 2.0f * D.beta;
  // ---- every global read is issued up front: r, |b|^2 and phi of the
  // region in 4-pixel vectors with their aperture bytes (the halo is 4 wide
  // and tile origins are multiples of 4, so a vector is wholly on or off the
  // grid), and |b|^2 and (kappa, theta~) of the pixels this thread updates.
  // phi is zero off the pupil in every state buffer, so it is read
  // unconditionally.  Tiles away from the grid border have every neighbour
  // and read their whole region without bounds tests.
  constexpr int RW4 = RW / 4, RP4 = G::RH * RW4;
  constexpr int SR = (RP4 + BT - 1) / BT;
  const auto rin4 = reinterpret_cast<gptr<const float4>>(rin);
  const auto pin4 = reinterpret_cast<gptr<const float4>>(pin);
  const auto bb4 = reinterpret_cast<gptr<const float4>>(glb(D.bb));
  const auto rout4 = reinterpret_cast<gptr<float4>>(rout);
  const auto pout4 = reinterpret_cast<gptr<float4>>(pout);
  const auto ktp = glb(D.T);
  const auto bbp = glb(D.bb);
  const auto geop = glb(D.geo);
  const auto geo4 = reinterpret_cast<gptr<const unsigned>>(geop);
  const bool border = ti == 0 || ti == TPR - 1 || tj == 0 || tj == TPC - 1;
  float4 gr[SR], gb[SR], gph[SR];
  unsigned gw[SR];  // aperture bytes of the 4 pixels of the vector
  auto load_region = [&](auto brd) {
    constexpr bool BRD = decltype(brd)::value;
#pragma unroll
    for (int q = 0; q < SR; ++q) {
      const int idx = threadIdx.x + q * BT;
      const int li = idx / RW4, gi = gi0 + li, gj = gj0 + 4 * (idx - li * RW4);
      // every thread of a round that ends inside the region has a vector
      const bool in_region = (q + 1) * BT <= RP4 || idx < RP4;
      if (in_region && (!BRD || (gi >= 0 && gi < N && gj >= 0 && gj < N))) {
        const unsigned v = (unsigned)(gi * N + gj) / 4u;
        gr[q] = rin4[v];
        gb[q] = bb4[v];
        gph[q] = pin4[v];
        gw[q] = geo4[v];
      } else if (BRD) {
        // off the grid (a vector beyond the region is never staged)
        gr[q] = gb[q] = gph[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        gw[q] = 0u;
      }
    }
  };
  if (border)
    load_region(std::true_type{});
  else
    load_region(std::false_type{});
  // per own pixel, one packed word: LDS offset (bits 0-15), neighbour mask
  // (16-19), pupil-neighbour weight in twelfths (20-23), in-pupil flag (24);
  // -1 when the pixel is off the grid or beyond this pass.  Then |b|^2, kappa
  // and theta~.  The pupil bits come from the stream's per-pixel geometry bytes,
  // and (kappa, theta~) is read at every own pixel (used only on the pupil;
  // elsewhere T holds other values); the loads are unconditional (a slot
  // without a pixel reads pixel 0) and the bytes are merged once every load
  // has arrived.
  int opk[SLOTS], ogeo[SLOTS];
  float okap[SLOTS], ott[SLOTS], os[SLOTS];
  static_for<0, 4>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
#pragma unroll
    for (int rd = 0; rd < G::rounds(c); ++rd) {
      const int slot = G::slot0(c) + rd;
      const int idx = threadIdx.x + rd * BT;
      const int u = idx / G::nv(c);
      const int li = G::li0(c) + 2 * u, lj = G::lj0(c) + 2 * (idx - u * G::nv(c));
      const int gi = gi0 + li, gj = gj0 + lj;
      const bool own = idx < G::n(c) && (!border || (gi >= 0 && gi < N && gj >= 0 && gj < N));
      const unsigned gp = own ? (unsigned)(gi * N + gj) : 0u;
      const float2 kt = ktp[gp];
      okap[slot] = kt.x;
      ott[slot] = kt.y;
      os[slot] = bbp[gp];  // |b|^2 here; s = E|g|^2 once r is staged
      ogeo[slot] = geop[gp];
      opk[slot] = own ? (li * RW + lj) | ((border ? nb_mask(gi, gj, N) : NB_ALL) << 16) : -1;
    }
  });
  if (sc[SC_FLAG] != 0.0f) {  // rejected frame: carry the state over unchanged
    for (int idx = threadIdx.x; idx < TH * (TW / 4); idx += BT) {
      const int li = idx / (TW / 4);
      const int v = ((ti * TH + li) * N + tj * TW) / 4 + (idx - li * (TW / 4));
      rout4[v] = rin4[v];
      pout4[v] = pin4[v];
    }
    return;
  }
  const float c0 = sc[SC_C0], c1 = sc[SC_C1], c2 = sc[SC_C2];
  // ---- stage the region: r after the Eq. (3) initialisation and phi' (phi
  // less the tip/tilt plane on the pupil; zero off the pupil and off the grid)
#pragma unroll
  for (int q = 0; q < SR; ++q) {
    const int idx = threadIdx.x + q * BT;
    if (idx < RP4) {
      const int li = idx / RW4, c4 = idx - li * RW4;
      const int gi = gi0 + li, gj = gj0 + 4 * c4;
      const float rv[4] = {gr[q].x, gr[q].y, gr[q].z, gr[q].w};
      const float bv[4] = {gb[q].x, gb[q].y, gb[q].z, gb[q].w};
      const float pv[4] = {gph[q].x, gph[q].y, gph[q].z, gph[q].w};
      float r[4], p[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // off the grid r stays 0 (rv = bv = 0; the weight of such a neighbour is 0)
        r[e] = do_rinit ? rinit_of(rv[e], bv[e], lam, alpha, fl) : rv[e];
        // phi' without a per-pixel branch: formed everywhere, kept on the pupil
        const float pe = use_plane ? pv[e] - plane_val(c0, c1, c2, gi, gj + e, N) : pv[e];
        p[e] = geo_in(gw[q] >> (8 * e)) ? pe : 0.f;
      }
      if (border && !(gi >= 0 && gi < N && gj >= 0 && gj < N)) r[0] = r[1] = r[2] = r[3] = 0.f;
      const int o4 = li * RW4 + c4;
      reinterpret_cast<float4*>(sR)[o4] = make_float4(r[0], r[1], r[2], r[3]);
      reinterpret_cast<float4*>(sP)[o4] = make_float4(p[0], p[1], p[2], p[3]);
    }
  }
  __syncthreads();
  // s = E|g|^2 of the pixels this thread updates, from their staged r
#pragma unroll
  for (int slot = 0; slot < SLOTS; ++slot) {
    opk[slot] = opk[slot] >= 0 ? opk[slot] | ((ogeo[slot] & 31) << 20) : -1;
    os[slot] = opk[slot] >= 0 ? second_moment(wiener_of(sR[opk[slot] & 0xffff], s2), os[slot], s2) : 0.f;
  }
  const float inv_sp = D.qg_inv_sp, lc = D.qg_lc, pmq = D.qg_pmq, qop = D.qg_qop;
  const float wE = inv_sp * (1.0f / 6.0f), wD = inv_sp * (1.0f / 12.0f);
  // ---- the four colour passes (same-colour pixels are never neighbours, so
  // each pass updates its pixels in place).  The neighbour-mask test is
  // compiled only into the path of the tiles at the grid border, a
  // block-uniform branch.
  auto passes = [&](auto check) {
    constexpr bool CHECK = decltype(check)::value;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int rd = 0; rd < G::rounds(c); ++rd) {
        const int slot = G::slot0(c) + rd;
        const int pk = opk[slot];
        if (pk >= 0) {
          const int o = pk & 0xffff;
          float rq[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) rq[e] = sR[o + offs[e]];
          const float rn = r_pixel_w<CHECK>(sR[o], os[slot], rq, (pk >> 16) & NB_ALL, wE, wD, lc, pmq, qop, fl);
          if (pk & (1 << 24)) {
            float pq[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) pq[e] = sP[o + offs[e]];
            sP[o] = phi_pixel(pq, pupil_weight_of((pk >> 20) & 15), okap[slot], ott[slot], beta2, sP[o]);
          }
          sR[o] = rn;
        }
      }
      __syncthreads();
    }
  };
  if (border)
    passes(std::true_type{});
  else
    passes(std::false_type{});
  // ---- the inner tile back to the output buffers, 4-pixel vectors
  for (int idx = threadIdx.x; idx < TH * (TW / 4); idx += BT) {
    const int li = idx / (TW / 4), c4 = idx - li * (TW / 4);
    const int o4 = (4 + li) * RW4 + 1 + c4;
    const int v = ((ti * TH + li) * N + tj * TW) / 4 + c4;
    rout4[v] = reinterpret_cast<const float4*>(sR)[o4];
    pout4[v] = reinterpret_cast<const float4*>(sP)[o4];
  }
}

// ---------------------------------------------------------------------------
// k_mpass: one colour pass of the r and phi M-steps over whole images, one
// thread per colour-C pixel.  The column pass has written r after the Eq. (3)
// initialisation, and the second row pass phi', into the output state
// buffers; pass C updates its pixels there in place (pixels of one colour are
// never neighbours), reading the current neighbours through the caches.
// grid (N*N/4/256, streams), block 256.
// ---------------------------------------------------------------------------
template <int N, int C>
__global__ __launch_bounds__(256) void k_mpass(StreamDesc* const* dptrs, int k) {
  const auto& D = desc_ref(dptrs[blockIdx.y]);
  constexpr int H = N / 2;
  const int q = blockIdx.x * 256 + threadIdx.x;  // < N*N/4
  const int u = q / H, v = q - (q / H) * H;
  const int gi = 2 * u + (C & 1), gj = 2 * v + (C >> 1);
  const int p = gi * N + gj;
  const int in = (D.cur + k) & 1;
  float* rw = glb(D.r[in ^ 1]);
  float* pw = glb(D.phi[in ^ 1]);
  const bool up = gi > 0, dn = gi < N - 1, lf = gj > 0, rt = gj < N - 1;
  // global reads first
  const float rp = rw[p];
  const float bb = glb(D.bb)[p];
  float rq[8];
  rq[0] = up ? rw[p - N] : 0.f;
  rq[1] = dn ? rw[p + N] : 0.f;
  rq[2] = lf ? rw[p - 1] : 0.f;
  rq[3] = rt ? rw[p + 1] : 0.f;
  rq[4] = (up && lf) ? rw[p - N - 1] : 0.f;
  rq[5] = (up && rt) ? rw[p - N + 1] : 0.f;
  rq[6] = (dn && lf) ? rw[p + N - 1] : 0.f;
  rq[7] = (dn && rt) ? rw[p + N + 1] : 0.f;
  const unsigned gp = glb(D.geo)[p];
  const bool pup = geo_in(gp);
  float pq[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float2 kt = make_float2(0.f, 0.f);
  if (pup) {
    // off-pupil phases are zero in the buffer, so only the grid edge is masked
    pq[0] = up ? pw[p - N] : 0.f;
    pq[1] = dn ? pw[p + N] : 0.f;
    pq[2] = lf ? pw[p - 1] : 0.f;
    pq[3] = rt ? pw[p + 1] : 0.f;
    pq[4] = (up && lf) ? pw[p - N - 1] : 0.f;
    pq[5] = (up && rt) ? pw[p - N + 1] : 0.f;
    pq[6] = (dn && lf) ? pw[p + N - 1] : 0.f;
    pq[7] = (dn && rt) ? pw[p + N + 1] : 0.f;
    kt = glb(D.T)[p];
  }
  if (glb(D.scal)[SC_FLAG] != 0.0f) {  // rejected frame: carry the state over unchanged
    rw[p] = glb(D.r[in])[p];
    pw[p] = glb(D.phi[in])[p];
    return;
  }
  // ---- r update
  const float s2 = D.sigma2;
  const float s = second_moment(wiener_of(rp, s2), bb, s2);
  rw[p] = r_pixel<true>(rp, s, rq, nb_mask(gi, gj, N), D.qg_inv_sp, D.qg_lc, D.qg_pmq, D.qg_qop, D.r_floor);
  // ---- phi update
  if (pup) {
    pw[p] = phi_pixel(pq, pupil_weight_of((int)(gp & 15u)), kt.x, kt.y, 2.0f * D.beta, pw[p]);
  }
}

// ---------------------------------------------------------------------------
// Plain batched unitary 2-D DFT (used by ddh_fft2 and the diagnostics).
// ---------------------------------------------------------------------------
template <int N, int LPW, int DIR>
__global__ __launch_bounds__(LPW*(N / Plan<N>::E)) void k_row_plain(const float2* __restrict__ in, float2* __restrict__ out,
                                                                  const float2* __restrict__ tw) {
  constexpr int E = Plan<N>::E, T = N / E;
  __shared__ float2 lds[LPW * RowLds<N>::STRIDE];
  const int line = threadIdx.x / T, t = threadIdx.x - line * T;
  const long long row = (long long)blockIdx.y * N + blockIdx.x * LPW + line;
  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = in[row * N + first_pos<N, DIR>(i, t)];
  RowLds<N> L{lds + line * RowLds<N>::STRIDE};
  line_fft<N, DIR>(v, t, L, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) out[row * N + last_pos<N, DIR>(i, t)] = v[i];
}

template <int N, int W, int DIR>
__global__ __launch_bounds__(W*(N / Plan<N>::E)) void k_col_plain(const float2* __restrict__ in, float2* __restrict__ out,
                                                                const float2* __restrict__ tw) {
  constexpr int E = Plan<N>::E;
  __shared__ float2 lds[N * ColLds<W>::STRIDE];
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const long long img = (long long)blockIdx.y * N * N;
  const int col = blockIdx.x * W + w;
  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = in[img + (long long)first_pos<N, DIR>(i, t) * N + col];
  ColLds<W> L{lds + w};
  line_fft<N, DIR>(v, t, L, tw);
  const float invN = 1.0f / (float)N;
#pragma unroll
  for (int i = 0; i < E; ++i) out[img + (long long)last_pos<N, DIR>(i, t) * N + col] = cscale(v[i], invN);
}

// ---------------------------------------------------------------------------
// Diagnostics (FP64 reductions)
// ---------------------------------------------------------------------------
template <class Desc>
__device__ __forceinline__ double qg_rho_d(double d, const Desc& D) {
  const double ad = fabs(d);
  const double p = D.qg_p, q = D.qg_q, T = D.qg_T, sg = D.qg_sigma;
  return pow(ad, p) / (p * pow(sg, p)) / (1.0 + pow(ad / (T * sg), p - q));
}

template <int NV>
__device__ __forceinline__ void block_sum_d(double (&x)[NV], double* red) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x[k] += __shfl_xor(x[k], off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * 16 + wv] = x[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[k * 16 + w];
    x[k] = s;
  }
  __syncthreads();
}

// per-pixel terms of the monitored cost; b = A_phi^H yhat for the current phi.
__global__ __launch_bounds__(256) void k_cost_terms(const StreamDesc* dp, int parity, const float2* b, double* partials) {
  const auto& D = desc_ref(dp);
  __shared__ double red[16];
  const int N = D.N;
  const float* r = glb(D.r[parity]);
  const float* phi = glb(D.phi[parity]);
  const double s2 = D.sigma2;
  double acc[1] = {0.0};
  const int total = N * N;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const int i = idx / N, j = idx - i * N;
    const double ri = r[idx];
    const double bx = b[idx].x, by = b[idx].y;
    acc[0] += (bx * bx + by * by) / (ri + s2) + log(ri + s2);
    const int offs[4][2] = {{0, 1}, {1, 0}, {1, 1}, {1, -1}};
    const double bw[4] = {1.0 / 6.0, 1.0 / 6.0, 1.0 / 12.0, 1.0 / 12.0};
    const bool pi_ = geo_in(glb(D.geo)[idx]);
    for (int q = 0; q < 4; ++q) {
      const int ii = i + offs[q][0], jj = j + offs[q][1];
      if (ii < 0 || ii >= N || jj < 0 || jj >= N) continue;
      const int o = ii * N + jj;
      acc[0] += bw[q] * qg_rho_d(ri - (double)r[o], D);
      if (pi_ && geo_in(glb(D.geo)[o])) {
        const double dph = (double)phi[idx] - (double)phi[o];
        acc[0] += (double)D.beta * bw[q] * dph * dph;
      }
    }
  }
  block_sum_d<1>(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// psi = phi - phi_true on the pupil: plane-fit sums (FP64 partials).
__global__ __launch_bounds__(256) void k_strehl_sums(const StreamDesc* dp, int parity, const float* phi_true,
                                                     double* partials) {
  const auto& D = desc_ref(dp);
  __shared__ double red[3 * 16];
  const int N = D.N;
  const float* phi = glb(D.phi[parity]);
  const double c = 0.5 * (N - 1);
  double acc[3] = {0, 0, 0};
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N * N; idx += gridDim.x * blockDim.x) {
    const int i = idx / N, j = idx - i * N;
    if (!geo_in(glb(D.geo)[idx])) continue;
    const double psi = (double)phi[idx] - (double)phi_true[idx];
    acc[0] += psi;
    acc[1] += (i - c) * psi;
    acc[2] += (j - c) * psi;
  }
  block_sum_d<3>(acc, red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 3 + 0] = acc[0];
    partials[blockIdx.x * 3 + 1] = acc[1];
    partials[blockIdx.x * 3 + 2] = acc[2];
  }
}

// field = a exp(j (psi - plane)); with phi_true == nullptr the field is a itself.
__global__ __launch_bounds__(256) void k_strehl_field(const StreamDesc* dp, int parity, const float* phi_true,
                                                      const double* coef, float2* field) {
  const auto& D = desc_ref(dp);
  const int N = D.N;
  const float* phi = glb(D.phi[parity]);
  const double c = 0.5 * (N - 1);
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N * N; idx += gridDim.x * blockDim.x) {
    const int i = idx / N, j = idx - i * N;
    float2 f = make_float2(0.f, 0.f);
    if (geo_in(glb(D.geo)[idx])) {
      if (phi_true) {
        const double psi = (double)phi[idx] - (double)phi_true[idx] - (coef[0] + coef[1] * (i - c) + coef[2] * (j - c));
        double sn, cs;
        sincos(psi, &sn, &cs);
        f = make_float2((float)cs, (float)sn);
      } else {
        f = make_float2(1.f, 0.f);
      }
    }
    field[idx] = f;
  }
}

__global__ __launch_bounds__(256) void k_max_abs2(const float2* x, int n, double* partials) {
  __shared__ double red[16];
  double m = 0.0;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
    const double a = (double)x[idx].x * x[idx].x + (double)x[idx].y * x[idx].y;
    m = a > m ? a : m;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mm = red[w] > mm ? red[w] : mm;
    partials[blockIdx.x] = mm;
  }
}

// b = A_phi^H yhat for the current phi of one stream (no plane): row pass into
// `work`, then plain inverse column pass into b.
template <int N, int LPW>
__global__ __launch_bounds__(LPW*(N / Plan<N>::E)) void k_row1_cur(const StreamDesc* dp, int parity,
                                                                 const float2* __restrict__ tw, float2* work) {
  constexpr int E = Plan<N>::E, T = N / E;
  __shared__ float2 lds[LPW * RowLds<N>::STRIDE];
  const auto& D = desc_ref(dp);
  const float* sc = glb(D.scal);
  const int line = threadIdx.x / T, t = threadIdx.x - line * T;
  const int row = blockIdx.x * LPW + line;
  const float2 mu = make_float2(sc[SC_MU_RE], sc[SC_MU_IM]);
  const float scale = sc[SC_SCALE];
  const float* phi = glb(D.phi[parity]) + row * N;
  const float2* y = glb(D.y) + row * N;
  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int n = first_pos<N, +1>(i, t);
    if (geo_in(glb(D.geo)[row * N + n])) {
      float sn, cs;
      sincosf(phi[n], &sn, &cs);
      const float2 yv = y[n];
      const float2 yh = make_float2((yv.x - mu.x) * scale, (yv.y - mu.y) * scale);
      v[i] = cmul(yh, make_float2(cs, -sn));
    } else {
      v[i] = make_float2(0.f, 0.f);
    }
  }
  RowLds<N> L{lds + line * RowLds<N>::STRIDE};
  line_fft<N, +1>(v, t, L, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) work[row * N + last_pos<N, +1>(i, t)] = v[i];
}

// Deterministic pseudo-random complex frames for the autotuner (splitmix
// hash of the element index; values uniform in [-1, 1) per component).
__device__ __forceinline__ unsigned int mix32(unsigned int x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__global__ void k_synth_frames(float2* y, long long n, unsigned int seed) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const unsigned int h1 = mix32((unsigned int)i * 2u + seed), h2 = mix32((unsigned int)i * 2u + 1u + seed);
    y[i] = make_float2((float)(h1 >> 8) * (2.0f / 16777216.0f) - 1.0f, (float)(h2 >> 8) * (2.0f / 16777216.0f) - 1.0f);
  }
}
hipError_t launch_synth_frames(float2* y, long long n, unsigned int seed, hipStream_t st) {
  hipLaunchKernelGGL(k_synth_frames, dim3(1024), dim3(256), 0, st, y, n, seed);
  return hipGetLastError();
}

__global__ void k_fill_zero(float* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}
// phi with the off-pupil values set to zero (the state invariant)
__global__ void k_copy_pupil(float* dst, const float* src, int N, const unsigned char* geo) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N * N; i += gridDim.x * blockDim.x)
    dst[i] = geo_in(geo[i]) ? src[i] : 0.0f;
}
hipError_t launch_copy_pupil(float* dst, const float* src, int N, const unsigned char* geo, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_pupil, dim3((N * N + 255) / 256), dim3(256), 0, st, dst, src, N, geo);
  return hipGetLastError();
}

__global__ void k_copy(float* dst, const float* src, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// launch wrappers: runtime dispatch on N and on the tile configuration
// ---------------------------------------------------------------------------
LaunchEvents& launch_events() {
  static thread_local LaunchEvents ev;
  return ev;
}
// A frame-kernel launch: through hipExtLaunchKernelGGL when timing events are
// pending (the kernel itself records the first launch's start and every
// launch's end), else a plain launch.
#define DDH_LAUNCH(K, G, B, SH, ST, ...)                                                      \
  do {                                                                                         \
    LaunchEvents& le_ = launch_events();                                                       \
    if (le_.stop) {                                                                            \
      hipExtLaunchKernelGGL(K, G, B, SH, ST, le_.launches == 0 ? le_.start : nullptr, le_.stop, 0, \
                            __VA_ARGS__);                                                      \
      ++le_.launches;                                                                          \
    } else {                                                                                   \
      hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                                        \
    }                                                                                          \
  } while (0)

#define DDH_DISPATCH_N(N, MACRO) \
  switch (N) {                   \
    case 64: MACRO(64); break;   \
    case 128: MACRO(128); break; \
    case 256: MACRO(256); break; \
    case 512: MACRO(512); break; \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_begin(StreamDesc* const* dptrs, const float2* const* ys, const int* curs, int count,
                        hipStream_t st) {
  for (int off = 0; off < count; off += FRAME_ARGS_MAX) {
    FrameArgs a{};
    const int n = count - off < FRAME_ARGS_MAX ? count - off : FRAME_ARGS_MAX;
    for (int i = 0; i < n; ++i) {
      a.y[i] = ys[off + i];
      a.cur[i] = curs[off + i];
    }
    DDH_LAUNCH(k_begin, dim3(1), dim3(64), 0, st, dptrs + off, a, n);
  }
  return hipGetLastError();
}

hipError_t launch_stats(StreamDesc* const* dptrs, int count, int N, int with_phi, const float2* const* ys,
                        const int* curs, StreamDesc* const* ds, hipStream_t st) {
  StreamDesc** list = const_cast<StreamDesc**>(dptrs);
  for (int off = 0; off < count; off += FRAME_ARGS_MAX) {
    FrameArgs a{};
    const int n = count - off < FRAME_ARGS_MAX ? count - off : FRAME_ARGS_MAX;
    if (ys)
      for (int i = 0; i < n; ++i) {
        a.y[i] = ys[off + i];
        a.cur[i] = curs[off + i];
        a.d[i] = ds ? ds[off + i] : nullptr;
      }
    const int mode = ys ? (ds ? 2 : 1) : 0;
#define DDH_X(NN)                                                                                  \
  DDH_LAUNCH(k_stats<NN>, dim3(StatsGeom<NN>::BLOCKS, n), dim3(256), 0, st, list + off, \
                     with_phi, a, mode);                                                            \
  break;
    switch (N) {
      case 64: DDH_X(64)
      case 128: DDH_X(128)
      case 256: DDH_X(256)
      case 512: DDH_X(512)
      default: return hipErrorInvalidValue;
    }
#undef DDH_X
  }
  return hipGetLastError();
}

hipError_t launch_finalize(StreamDesc* const* dptrs, int count, int N, int with_phi, hipStream_t st) {
#define DDH_X(NN)                                                                     \
  DDH_LAUNCH(k_finalize<NN>, dim3(count), dim3(64), 0, st, dptrs, with_phi); \
  return hipGetLastError()
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}


template <int N>
static hipError_t row1_n(StreamDesc* const* d, int count, const float2* tw, int k, int use_plane, int fin,
                         int with_phi, int lpw, hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
#define DDH_R1(L)                                                                                      \
  case L:                                                                                              \
    DDH_LAUNCH((k_row1<N, L>), dim3(N / L, count), dim3(L * T), 0, st, d, tw, k, use_plane, fin, \
                       with_phi);                                                                       \
    break;
  switch (lpw) {
    DDH_R1(4) DDH_R1(8) DDH_R1(16) DDH_R1(32)
    default: return hipErrorInvalidValue;
  }
#undef DDH_R1
  return hipGetLastError();
}
template <int N>
static hipError_t row2_n(StreamDesc* const* d, int count, const float2* tw, int k, int use_plane, int mat, int lpw,
                         hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
#define DDH_R2(L)                                                                                          \
  case L:                                                                                                  \
    DDH_LAUNCH((k_row2<N, L>), dim3(N / L, count), dim3(L * T), 0, st, d, tw, k, use_plane, mat); \
    break;
  switch (lpw) {
    DDH_R2(4) DDH_R2(8) DDH_R2(16) DDH_R2(32)
    default: return hipErrorInvalidValue;
  }
#undef DDH_R2
  return hipGetLastError();
}
template <int N>
static hipError_t col_n(StreamDesc* const* d, int count, const float2* tw, int k, int do_rinit, int mat, int w,
                        hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
#define DDH_C(W)                                                                                         \
  case W:                                                                                                \
    DDH_LAUNCH((k_col<N, W>), dim3(N / W, count), dim3(W * T), 0, st, d, tw, k, do_rinit, mat); \
    break;
  switch (w) {
    DDH_C(4) DDH_C(8) DDH_C(16) DDH_C(32)
    default: return hipErrorInvalidValue;
  }
#undef DDH_C
  return hipGetLastError();
}
template <int N>
static hipError_t mstep_n(StreamDesc* const* d, int count, int k, int use_plane, int do_rinit, int th, int tw,
                          hipStream_t st) {
  if (th == 0) {  // four whole-image colour passes
    const dim3 grid((N * N / 4) / 256, count);
    DDH_LAUNCH((k_mpass<N, 0>), grid, dim3(256), 0, st, d, k);
    DDH_LAUNCH((k_mpass<N, 1>), grid, dim3(256), 0, st, d, k);
    DDH_LAUNCH((k_mpass<N, 2>), grid, dim3(256), 0, st, d, k);
    DDH_LAUNCH((k_mpass<N, 3>), grid, dim3(256), 0, st, d, k);
    return hipGetLastError();
  }
#define DDH_M(TH, TW)                                                                                          \
  if (th == TH && tw == TW) {                                                                                  \
    if constexpr (N % TH == 0 && N % TW == 0) {                                                                \
      DDH_LAUNCH((k_mstep<N, TH, TW>), dim3((N / TH) * (N / TW), count), dim3((MsGeom<TH, TW>::BT)), 0, st, \
                         d, k, use_plane, do_rinit);                                                           \
      return hipGetLastError();                                                                                \
    }                                                                                                          \
  }
  DDH_M(16, 16) DDH_M(16, 32) DDH_M(16, 64) DDH_M(32, 32) DDH_M(32, 64) DDH_M(64, 64) DDH_M(32, 128)
#undef DDH_M
  return hipErrorInvalidValue;
}

static bool lpw_ok(int N, int lpw) {
  const int T = N / (N == 64 ? 8 : 16);
  return lpw * T <= 1024 && N % lpw == 0;
}
static bool w_ok(int N, int w) {
  const int T = N / (N == 64 ? 8 : 16);
  return w * T <= 1024 && N % w == 0;
}

hipError_t launch_row1(StreamDesc* const* d, int count, int N, const float2* tw, int k, int use_plane, int fin,
                       int with_phi, const TileConfig& tc, hipStream_t st) {
  if (!lpw_ok(N, tc.row_lines)) return hipErrorInvalidValue;
#define DDH_X(NN) return row1_n<NN>(d, count, tw, k, use_plane, fin, with_phi, tc.row_lines, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}
template <int N>
static hipError_t row1s_n(StreamDesc** list, int n, const FrameArgs& a, int use_args, const float2* tw, int with_phi,
                          unsigned spin_limit, int nq, int lpw, hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
#define DDH_R1S(L)                                                                                           \
  case L:                                                                                                    \
    DDH_LAUNCH((k_row1s<N, L>), dim3(N / L, n), dim3(L * T), 0, st, list, a, use_args, tw, with_phi, \
                       spin_limit, nq);                                                                      \
    break;
  switch (lpw) {
    DDH_R1S(4) DDH_R1S(8) DDH_R1S(16) DDH_R1S(32)
    default: return hipErrorInvalidValue;
  }
#undef DDH_R1S
  return hipGetLastError();
}
hipError_t launch_row1s(StreamDesc* const* dptrs, int count, int N, const float2* tw, int with_phi,
                        const float2* const* ys, const int* curs, StreamDesc* const* ds, unsigned spin_limit,
                        int nq, const TileConfig& tc, hipStream_t st) {
  if (!lpw_ok(N, tc.row_lines)) return hipErrorInvalidValue;
  StreamDesc** list = const_cast<StreamDesc**>(dptrs);
  for (int off = 0; off < count; off += FRAME_ARGS_MAX) {
    FrameArgs a{};
    const int n = count - off < FRAME_ARGS_MAX ? count - off : FRAME_ARGS_MAX;
    if (ys)
      for (int i = 0; i < n; ++i) {
        a.y[i] = ys[off + i];
        a.cur[i] = curs[off + i];
        a.d[i] = ds ? ds[off + i] : nullptr;
      }
    const int use_args = ys ? (ds ? 2 : 1) : 0;
    hipError_t e = hipSuccess;
#define DDH_X(NN) e = row1s_n<NN>(list + off, n, a, use_args, tw, with_phi, spin_limit, nq, tc.row_lines, st)
    switch (N) {
      case 64: DDH_X(64); break;
      case 128: DDH_X(128); break;
      case 256: DDH_X(256); break;
      case 512: DDH_X(512); break;
      default: return hipErrorInvalidValue;
    }
#undef DDH_X
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}
hipError_t launch_col(StreamDesc* const* d, int count, int N, const float2* tw, int k, int do_rinit,
                      const TileConfig& tc, hipStream_t st) {
  if (!w_ok(N, tc.col_width)) return hipErrorInvalidValue;
#define DDH_X(NN) return col_n<NN>(d, count, tw, k, do_rinit, tc.m_tile_h == 0, tc.col_width, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}
hipError_t launch_row2(StreamDesc* const* d, int count, int N, const float2* tw, int k, int use_plane,
                       const TileConfig& tc, hipStream_t st) {
  if (!lpw_ok(N, tc.row_lines)) return hipErrorInvalidValue;
#define DDH_X(NN) return row2_n<NN>(d, count, tw, k, use_plane, tc.m_tile_h == 0, tc.row_lines, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}
hipError_t launch_mstep(StreamDesc* const* d, int count, int N, int k, int use_plane, int do_rinit,
                        const TileConfig& tc, hipStream_t st) {
#define DDH_X(NN) return mstep_n<NN>(d, count, k, use_plane, do_rinit, tc.m_tile_h, tc.m_tile_w, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}

hipError_t launch_frame(StreamDesc* const* dptrs, int count, int N, const float2* tw, int k, int mode,
                        const float2* const* ys, const int* curs, StreamDesc* const* ds, unsigned* ctl0, int nq,
                        int lag, unsigned spin_limit, int giveup, int whole_image, float share, hipStream_t st) {
  if (nq < 1 || nq > CTL_MAX_QUEUES || lag < 1 || !(share > 0.0f) || share > 1.0f) return hipErrorInvalidValue;
  StreamDesc** list = const_cast<StreamDesc**>(dptrs);
  // persistent grid: 3 workgroups of 256 threads per CU (the column stage's
  // registers allow 3 waves per SIMD) times the launch's share of the device,
  // a multiple of nq, no more than items
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  for (int off = 0; off < count; off += FRAME_ARGS_MAX) {
    FrameArgs a{};
    const int n = count - off < FRAME_ARGS_MAX ? count - off : FRAME_ARGS_MAX;
    if (ys)
      for (int i = 0; i < n; ++i) {
        a.y[i] = ys[off + i];
        a.cur[i] = curs[off + i];
        a.d[i] = ds ? ds[off + i] : nullptr;
      }
    const int use_args = ys ? (ds ? 2 : 1) : 0;
    const int per_stream = 4 * N;  // upper bound of the items of one stream
    int grid = (int)(3.0f * (float)cus * share + 0.5f);
    if (grid < nq) grid = nq;
    if (grid > n * per_stream) grid = n * per_stream;
    grid = ((grid + nq - 1) / nq) * nq;
    unsigned* c0 = ctl0;
#define DDH_F(NN)                                                                                           \
  DDH_LAUNCH(k_frame<NN>, dim3(grid), dim3(256), 0, st, list + off, n, a, use_args, tw, k, mode, c0, nq, \
                     lag, spin_limit, giveup, whole_image);                                                   \
  break;
    switch (N) {
      case 64: DDH_F(64)
      case 128: DDH_F(128)
      case 256: DDH_F(256)
      case 512: DDH_F(512)
      default: return hipErrorInvalidValue;
    }
#undef DDH_F
  }
  return hipGetLastError();
}

template <int N>
static hipError_t fft2_n(int count, const float2* in, float2* out, float2* work, const float2* tw, int inverse,
                         hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
  constexpr int LPW = 256 / T > N ? N : 256 / T;
  constexpr int W = LPW;
  if (inverse) {
    hipLaunchKernelGGL((k_row_plain<N, LPW, +1>), dim3(N / LPW, count), dim3(LPW * T), 0, st, in, work, tw);
    hipLaunchKernelGGL((k_col_plain<N, W, +1>), dim3(N / W, count), dim3(W * T), 0, st, work, out, tw);
  } else {
    hipLaunchKernelGGL((k_row_plain<N, LPW, -1>), dim3(N / LPW, count), dim3(LPW * T), 0, st, in, work, tw);
    hipLaunchKernelGGL((k_col_plain<N, W, -1>), dim3(N / W, count), dim3(W * T), 0, st, work, out, tw);
  }
  return hipGetLastError();
}

hipError_t launch_fft2(int N, int count, const float2* in, float2* out, float2* work, const float2* tw, int inverse,
                       hipStream_t st) {
#define DDH_X(NN) return fft2_n<NN>(count, in, out, work, tw, inverse, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}

hipError_t launch_cost_terms(const StreamDesc* d, int parity, const float2* b, double* partials, int nparts,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_cost_terms, dim3(nparts), dim3(256), 0, st, d, parity, b, partials);
  return hipGetLastError();
}
hipError_t launch_strehl_sums(const StreamDesc* d, int parity, const float* phi_true, double* partials, int nparts,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_strehl_sums, dim3(nparts), dim3(256), 0, st, d, parity, phi_true, partials);
  return hipGetLastError();
}
hipError_t launch_strehl_field(const StreamDesc* d, int N, int parity, const float* phi_true, const double* coef,
                               float2* field, hipStream_t st) {
  const int nb = (N * N + 255) / 256;
  hipLaunchKernelGGL(k_strehl_field, dim3(nb < 1024 ? nb : 1024), dim3(256), 0, st, d, parity, phi_true, coef, field);
  return hipGetLastError();
}
hipError_t launch_max_abs2(const float2* x, int n, double* partials, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(k_max_abs2, dim3(nparts), dim3(256), 0, st, x, n, partials);
  return hipGetLastError();
}
template <int N>
static hipError_t bp_cur_n(const StreamDesc* d, int parity, const float2* tw, float2* b, float2* work, hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
  constexpr int LPW = 256 / T > N ? N : 256 / T;
  hipLaunchKernelGGL((k_row1_cur<N, LPW>), dim3(N / LPW), dim3(LPW * T), 0, st, d, parity, tw, work);
  hipLaunchKernelGGL((k_col_plain<N, LPW, +1>), dim3(N / LPW, 1), dim3(LPW * T), 0, st, work, b, tw);
  return hipGetLastError();
}
hipError_t launch_backproject_cur(const StreamDesc* d, int N, int parity, const float2* tw, float2* b, float2* work,
                                  hipStream_t st) {
#define DDH_X(NN) return bp_cur_n<NN>(d, parity, tw, b, work, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}
hipError_t launch_fill_zero(float* p, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_zero, dim3(512), dim3(256), 0, st, p, n);
  return hipGetLastError();
}
hipError_t launch_copy(float* dst, const float* src, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(512), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}


// ===========================================================================
// Unrolled frames with a hand-written adjoint (gradient of a loss on the last
// frame's phase with respect to the initial phase, sigma_w, the QGGMRF scale
// sigma_r and the phase-prior weight beta).  Plain whole-image kernels, one
// thread per pixel, no fusion: they keep every intermediate the adjoint needs.
// The forward uses the same per-pixel helpers as the fast path (the colour
// passes are those of k_mpass).  One launch covers a batch of streams of one
// N: blockIdx.y is the stream, every array is the streams' N x N row-major
// images back to back, and each stream's constants and per-frame scalars sit
// in device arrays indexed by the stream.  The scalar reductions (Normalize,
// the tip/tilt plane, the loss) are FP64 block partials combined on the device.
// ===========================================================================


__device__ __forceinline__ bool g_pix(int& i, int& j, int N) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  i = p / N;
  j = p - i * N;
  return p < N * N;
}
// one thread per 2 x 2 quad (one pixel of each colour): quad (qi, qj) holds
// pixels (2qi + a, 2qj + b); its colour-C pixel is a = C & 1, b = C >> 1
__device__ __forceinline__ bool g_quad(int& qi, int& qj, int N) {
  const int q = blockIdx.x * 256 + threadIdx.x, h = N >> 1;
  qi = q / h;
  qj = q - qi * h;
  return q < h * h;
}
// index of pixel (i, j) of this block's stream in a batched array
__device__ __forceinline__ int g_at(int i, int j, int N) { return ((int)blockIdx.y * N + i) * N + j; }
// Reductions (Normalize, the tip/tilt planes, the loss, the scalar
// gradients): 16 pixels per thread and G_RED_PIX per block, each block
// writing one record of NV FP64 sums; the kernel that needs the result sums
// its stream's records (at most 64, N <= 512) in its first wavefront.
constexpr int G_RED_PIX = 4096;
__host__ __device__ constexpr int g_nred(int N) { return (N * N) / G_RED_PIX; }
template <int NV>
__device__ __forceinline__ void g_block_record(double (&x)[NV], double* part) {
  __shared__ double red[NV][4];
#pragma unroll
  for (int k = 0; k < NV; ++k) x[k] = wave_sum_d(x[k]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wv] = x[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k)
      part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NV + k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
}
// the stream's totals, in every lane of the calling wavefront
template <int NV>
__device__ __forceinline__ void g_wave_totals(const double* part, int nred, double (&t)[NV]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double v = lane < nred ? part[((size_t)blockIdx.y * nred + lane) * NV + k] : 0.0;
    t[k] = wave_sum_d(v);
  }
}
__device__ __forceinline__ int g_red_pix(int e) { return blockIdx.x * G_RED_PIX + e * 256 + threadIdx.x; }

// frame statistics: sums of Re y, Im y, |y|^2 and the plane-fit sums over the
// pupil of the incoming phase: sum phi, sum (i-c) phi, sum (j-c) phi
__global__ __launch_bounds__(256) void k_g_stats(const float2* const* ys, const float* phi, const GradPrm* Pd,
                                                 double* part) {
  const int N = Pd[blockIdx.y].N;
  const float d2 = Pd[blockIdx.y].d2;
  const auto y = glb(ys[blockIdx.y]);  // global, not flat, loads
  const auto ph = glb(phi) + (size_t)blockIdx.y * N * N;
  float2 v[16];
  float f[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    v[e] = y[g_red_pix(e)];
    f[e] = ph[g_red_pix(e)];
  }
  const double c = 0.5 * (N - 1);
  double x[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int pix = g_red_pix(e), i = pix / N, j = pix - i * N;
    x[0] += v[e].x;
    x[1] += v[e].y;
    x[2] += (double)v[e].x * v[e].x + (double)v[e].y * v[e].y;
    if (in_pupil(i, j, N, d2)) {
      x[3] += f[e];
      x[4] += (i - c) * f[e];
      x[5] += (j - c) * f[e];
    }
  }
  g_block_record<6>(x, part);
}
// plane-fit sums over the pupil of f (the phase adjoint before the tip/tilt
// projection)
__global__ __launch_bounds__(256) void k_g_psum(const float* f, const GradPrm* Pd, double* part) {
  const int N = Pd[blockIdx.y].N;
  const float d2 = Pd[blockIdx.y].d2;
  const float* fs = f + (size_t)blockIdx.y * N * N;
  float v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = fs[g_red_pix(e)];
  const double c = 0.5 * (N - 1);
  double x[3] = {0, 0, 0};
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int pix = g_red_pix(e), i = pix / N, j = pix - i * N;
    if (in_pupil(i, j, N, d2)) {
      x[0] += v[e];
      x[1] += (i - c) * v[e];
      x[2] += (j - c) * v[e];
    }
  }
  g_block_record<3>(x, part);
}
// piston-removed phase error sums over the pupil: sum d, sum d^2, count, d = phi - phi_true
__global__ __launch_bounds__(256) void k_g_dsum(const float* phi, const float* ptrue, const GradPrm* Pd,
                                                double* part) {
  const int N = Pd[blockIdx.y].N;
  const float d2 = Pd[blockIdx.y].d2;
  const size_t o = (size_t)blockIdx.y * N * N;
  float a[16], t[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    a[e] = phi[o + g_red_pix(e)];
    t[e] = ptrue[o + g_red_pix(e)];
  }
  double x[3] = {0, 0, 0};
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int pix = g_red_pix(e), i = pix / N, j = pix - i * N;
    if (in_pupil(i, j, N, d2)) {
      const double d = (double)a[e] - t[e];
      x[0] += d;
      x[1] += d * d;
      x[2] += 1.0;
    }
  }
  g_block_record<3>(x, part);
}
// sums over the whole image of the three per-pixel gradient accumulators
__global__ __launch_bounds__(256) void k_g_tsum(const float* a0, const float* a1, const float* a2, int N,
                                                double* part) {
  const size_t o = (size_t)blockIdx.y * N * N;
  double x[3] = {0, 0, 0};
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const size_t q = o + g_red_pix(e);
    x[0] += a0[q];
    x[1] += a1[q];
    x[2] += a2[q];
  }
  g_block_record<3>(x, part);
}
// the least-squares plane of a stream from its plane-fit totals
__device__ __forceinline__ void g_plane(const double* minv, const double (&t)[3], float* c) {
  const double* M = minv + 6 * blockIdx.y;
  c[0] = (float)(M[0] * t[0] + M[1] * t[1] + M[2] * t[2]);
  c[1] = (float)(M[1] * t[0] + M[3] * t[1] + M[4] * t[2]);
  c[2] = (float)(M[2] * t[0] + M[4] * t[1] + M[5] * t[2]);
}

// frame prologue: Normalize (Eq. 4) and the plane from the stats records
// (first wavefront; flag bit 1 if y is constant), then per pixel yhat, phi'
// (plane removed, zero off the pupil), v = a exp(-j phi') yhat
__global__ __launch_bounds__(256) void k_g_prologue(const float2* const* ys, const float* phi, const GradPrm* Pd,
                                                    const double* minv, const double* part, int* flag, float2* yh,
                                                    float* phip, float2* v) {
  const GradPrm P = Pd[blockIdx.y];
  __shared__ float sc[6];
  if (threadIdx.x < 64) {
    double t[6];
    g_wave_totals<6>(part, g_nred(P.N), t);
    if (threadIdx.x == 0) {
      const double px = (double)P.N * P.N, mr = t[0] / px, mi = t[1] / px;
      const double m2 = t[2] - px * (mr * mr + mi * mi);
      const bool ok = m2 > 0.0 && m2 < HUGE_VAL;
      sc[0] = (float)mr;
      sc[1] = (float)mi;
      sc[2] = ok ? (float)sqrt(px / m2) : 0.0f;
      const double tp[3] = {t[3], t[4], t[5]};
      g_plane(minv, tp, sc + 3);
      if (!ok && blockIdx.x == 0) flag[blockIdx.y] = flag[blockIdx.y] | 1;
    }
  }
  __syncthreads();
  int i, j;
  if (!g_pix(i, j, P.N)) return;
  const int p = g_at(i, j, P.N);
  const float2 yy = ys[blockIdx.y][i * P.N + j];
  const float2 h = make_float2((yy.x - sc[0]) * sc[2], (yy.y - sc[1]) * sc[2]);
  yh[p] = h;
  float ph = 0.f;
  float2 vv = make_float2(0.f, 0.f);
  if (in_pupil(i, j, P.N, P.d2)) {
    ph = phi[p] - plane_val(sc[3], sc[4], sc[5], i, j, P.N);
    float sn, cs;
    fsincos(ph, &sn, &cs);
    vv = cmul(h, make_float2(cs, -sn));
  }
  phip[p] = ph;
  v[p] = vv;
}
// Eq. (3) and the E-step at one pixel: r0, mu, s from b and the previous r
__device__ __forceinline__ float2 g_estep_px(float2 bv, float rprev, const GradPrm& P, float& r0, float& s) {
  const float bb = bv.x * bv.x + bv.y * bv.y;
  const float r = rinit_of(rprev, bb, P.lam, P.alpha, P.fl);
  const float w = wiener_of(r, P.s2);
  r0 = r;
  s = second_moment(w, bb, P.s2);
  return make_float2(w * bv.x, w * bv.y);
}
// Column pass of the frame's two DFTs with the E-step between them, as the
// fast path's column kernel: work holds the row-transformed v; the inverse
// column DFT gives b, the E-step mu (b, r0, mu and s are kept for the
// adjoint), the forward column DFT of mu goes back into work (scaled by 1/N),
// whose forward row DFT is z.  grid (N / W, streams), in place.
template <int N, int W>
__global__ __launch_bounds__(W*(N / Plan<N>::E)) void k_g_col_fwd(float2* work, const float* rprev, const GradPrm* Pd,
                                                                float2* b, float* r0, float2* mu, float* s,
                                                                const float2* __restrict__ tw) {
  constexpr int E = Plan<N>::E;
  __shared__ float2 lds[N * ColLds<W>::STRIDE];
  const GradPrm P = Pd[blockIdx.y];
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const int img = blockIdx.y * N * N;
  const int col = blockIdx.x * W + w;
  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = work[img + first_pos<N, +1>(i, t) * N + col];
  ColLds<W> L{lds + w};
  line_fft<N, +1>(v, t, L, tw);
  const float invN = 1.0f / (float)N;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int p = img + last_pos<N, +1>(i, t) * N + col;
    const float2 bv = cscale(v[i], invN);
    float rr, ss;
    const float2 m = g_estep_px(bv, rprev[p], P, rr, ss);
    b[p] = bv;
    r0[p] = rr;
    s[p] = ss;
    mu[p] = m;
    v[i] = m;
  }
  __syncthreads();
  line_fft<N, -1>(v, t, L, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) work[img + last_pos<N, -1>(i, t) * N + col] = cscale(v[i], invN);
}
// phase data term: kappa, theta~ on the pupil (as the fast path's second row pass)
__device__ __forceinline__ void g_data_u(float2 h, float ph, float2 z, float& ur, float& ui) {
  float sn, cs;
  fsincos(ph, &sn, &cs);
  const float qr = h.x * z.x + h.y * z.y, qi = h.x * z.y - h.y * z.x;  // conj(yhat) z
  ur = cs * qr - sn * qi;
  ui = sn * qr + cs * qi;
}
__global__ __launch_bounds__(256) void k_g_data(const float2* yh, const float* phip, const float2* z, const GradPrm* Pd,
                                                float* kap, float* tth) {
  const GradPrm P = Pd[blockIdx.y];
  int i, j;
  if (!g_pix(i, j, P.N)) return;
  const int p = g_at(i, j, P.N);
  float ka = 0.f, tt = 0.f;
  if (in_pupil(i, j, P.N, P.d2)) {
    float ur, ui;
    g_data_u(yh[p], phip[p], z[p], ur, ui);
    const float x0 = fatan2(ui, ur);
    const float c2s = 2.0f / P.s2;
    ka = x0 != 0.0f ? c2s * ui * __builtin_amdgcn_rcpf(x0) : c2s * ur;
    tt = phip[p] - x0;
  }
  kap[p] = ka;
  tth[p] = tt;
}
// colour pass C of the r M-step, out of place (rin -> rout): one thread per
// quad updates its colour-C pixel and copies the other three
template <int C>
__device__ __forceinline__ void g_rpass_body(const float* rin, const float* s, const GradPrm* Pd, float* rout) {
  const GradPrm P = Pd[blockIdx.y];
  int qi, qj;
  if (!g_quad(qi, qj, P.N)) return;
  const int N = P.N;
  const int p00 = g_at(2 * qi, 2 * qj, N);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (q != C) rout[p00 + (q & 1) * N + (q >> 1)] = rin[p00 + (q & 1) * N + (q >> 1)];
  const int i = 2 * qi + (C & 1), j = 2 * qj + (C >> 1), p = p00 + (C & 1) * N + (C >> 1);
  const bool up = i > 0, dn = i < N - 1, lf = j > 0, rt = j < N - 1;
  float rq[8];
  rq[0] = up ? rin[p - N] : 0.f;
  rq[1] = dn ? rin[p + N] : 0.f;
  rq[2] = lf ? rin[p - 1] : 0.f;
  rq[3] = rt ? rin[p + 1] : 0.f;
  rq[4] = (up && lf) ? rin[p - N - 1] : 0.f;
  rq[5] = (up && rt) ? rin[p - N + 1] : 0.f;
  rq[6] = (dn && lf) ? rin[p + N - 1] : 0.f;
  rq[7] = (dn && rt) ? rin[p + N + 1] : 0.f;
  rout[p] = r_pixel<true>(rin[p], s[p], rq, nb_mask(i, j, N), P.inv_sp, P.lc, P.pmq, P.qop, P.fl);
}
// colour pass C of the phi M-step, out of place, one thread per quad
template <int C>
__device__ __forceinline__ void g_ppass_body(const float* pin, const float* kap, const float* tth,
                                                 const GradPrm* Pd, float* pout) {
  const GradPrm P = Pd[blockIdx.y];
  int qi, qj;
  if (!g_quad(qi, qj, P.N)) return;
  const int N = P.N;
  const int p00 = g_at(2 * qi, 2 * qj, N);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (q != C) pout[p00 + (q & 1) * N + (q >> 1)] = pin[p00 + (q & 1) * N + (q >> 1)];
  const int i = 2 * qi + (C & 1), j = 2 * qj + (C >> 1), p = p00 + (C & 1) * N + (C >> 1);
  if (!in_pupil(i, j, N, P.d2)) {
    pout[p] = pin[p];
    return;
  }
  const bool up = i > 0, dn = i < N - 1, lf = j > 0, rt = j < N - 1;
  float pq[8];
  pq[0] = up ? pin[p - N] : 0.f;
  pq[1] = dn ? pin[p + N] : 0.f;
  pq[2] = lf ? pin[p - 1] : 0.f;
  pq[3] = rt ? pin[p + 1] : 0.f;
  pq[4] = (up && lf) ? pin[p - N - 1] : 0.f;
  pq[5] = (up && rt) ? pin[p - N + 1] : 0.f;
  pq[6] = (dn && lf) ? pin[p + N - 1] : 0.f;
  pq[7] = (dn && rt) ? pin[p + N + 1] : 0.f;
  pout[p] = phi_pixel(pq, pupil_weight_of(pupil_nbr_12(i, j, N, P.d2)), kap[p], tth[p], 2.0f * P.beta, pin[p]);
}

// ---------------------------------------------------------------- adjoint
// loss: L = sqrt(mean(d - mean d)^2) over the pupil; dL/dphi = (d - mean d)/(n L).
// The first wavefront combines the dsum records; block 0 stores the loss
// (flag bit 2 if it is zero)
__global__ __launch_bounds__(256) void k_g_loss_bar(const float* phi, const float* ptrue, const GradPrm* Pd,
                                                    const double* part, GradLoss* Lo, int* flag, float* pbar) {
  const GradPrm P = Pd[blockIdx.y];
  __shared__ float sc[2];
  if (threadIdx.x < 64) {
    double t[3];
    g_wave_totals<3>(part, g_nred(P.N), t);
    if (threadIdx.x == 0) {
      const double n = t[2], dmean = t[0] / n, var = t[1] / n - dmean * dmean;
      const double L = sqrt(var > 0.0 ? var : 0.0);
      sc[0] = (float)dmean;
      sc[1] = L > 0.0 ? (float)(1.0 / (n * L)) : 0.0f;
      if (blockIdx.x == 0) {
        Lo[blockIdx.y].dmean = sc[0];
        Lo[blockIdx.y].inv_nL = sc[1];
        Lo[blockIdx.y].loss = L;
        if (!(L > 0.0)) flag[blockIdx.y] = flag[blockIdx.y] | 2;
      }
    }
  }
  __syncthreads();
  int i, j;
  if (!g_pix(i, j, P.N)) return;
  const int p = g_at(i, j, P.N);
  pbar[p] = in_pupil(i, j, P.N, P.d2) ? (phi[p] - ptrue[p] - sc[0]) * sc[1] : 0.f;
}
// phi pass C reversed, part a: the colour-C pupil pixels hand their adjoint to
// kappa, theta~, beta and (as em = pbar 2 beta / den) to their neighbours.
// One thread per quad; kbar and tbar are assigned (every pixel is of exactly
// one colour, so the four passes write each once).
template <int C>
__device__ __forceinline__ void g_pback_a_body(const float* pin, const float* pout, const float* kap,
                                                   const float* tth, const GradPrm* Pd, float* pbar, float* em,
                                                   float* kbar, float* tbar, float* gbeta) {
  const GradPrm P = Pd[blockIdx.y];
  int qi, qj;
  if (!g_quad(qi, qj, P.N)) return;
  const int N = P.N;
  const int p00 = g_at(2 * qi, 2 * qj, N);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (q != C) em[p00 + (q & 1) * N + (q >> 1)] = 0.f;
  const int i = 2 * qi + (C & 1), j = 2 * qj + (C >> 1), p = p00 + (C & 1) * N + (C >> 1);
  float emv = 0.f, kb = 0.f, tb = 0.f;
  if (in_pupil(i, j, N, P.d2)) {
    const int nb[8][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {-1, 1}, {1, -1}, {1, 1}};
    float Ph = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ii = i + nb[e][0], jj = j + nb[e][1];
      if (ii >= 0 && ii < N && jj >= 0 && jj < N) Ph += (e < 4 ? 1.0f / 6.0f : 1.0f / 12.0f) * pin[g_at(ii, jj, N)];
    }
    const float Pw = pupil_weight_of(pupil_nbr_12(i, j, N, P.d2));
    const float ka = kap[p], beta2 = 2.0f * P.beta;
    const float den = ka + beta2 * Pw;
    if (den > 0.0f) {  // otherwise the pixel kept its value: its adjoint passes through
      const float g = pbar[p], inv = 1.0f / den, out = pout[p];
      emv = g * beta2 * inv;
      kb = g * (tth[p] - out) * inv;
      tb = g * ka * inv;
      gbeta[p] += g * 2.0f * (Ph - Pw * out) * inv;
      pbar[p] = 0.f;
    }
  }
  em[p] = emv;
  kbar[p] = kb;
  tbar[p] = tb;
}
// data term reversed: (kbar, tbar) -> phi' (pb2 = pbar + ...), z (zbar), s2
__global__ __launch_bounds__(256) void k_g_data_bar(const float2* yh, const float* phip, const float2* z,
                                                    const float* kap, const float* kbar, const float* tbar,
                                                    const float* pbar, const GradPrm* Pd, float* pb2, float2* zbar,
                                                    float* gs2) {
  const GradPrm P = Pd[blockIdx.y];
  int i, j;
  if (!g_pix(i, j, P.N)) return;
  const int p = g_at(i, j, P.N);
  zbar[p] = make_float2(0.f, 0.f);
  pb2[p] = pbar[p];  // pb2 starts as the phase adjoint left by the passes
  if (!in_pupil(i, j, P.N, P.d2)) return;
  float ur, ui;
  g_data_u(yh[p], phip[p], z[p], ur, ui);
  const float x0 = fatan2(ui, ur);
  const float mag = sqrtf(ur * ur + ui * ui);
  const float c2s = 2.0f / P.s2;
  float sc, dsc;  // sinc(x0) and its derivative
  if (fabsf(x0) > 1e-3f) {
    float sn, cs;
    sincosf(x0, &sn, &cs);
    sc = sn / x0;
    dsc = (x0 * cs - sn) / (x0 * x0);
  } else {
    sc = 1.0f - x0 * x0 * (1.0f / 6.0f);
    dsc = -x0 * (1.0f / 3.0f);
  }
  const float kb = kbar[p], tb = tbar[p];
  const float xb = kb * c2s * mag * dsc - tb;  // adjoint of x0
  const float mb = kb * c2s * sc;              // adjoint of |u|
  gs2[p] += -kb * kap[p] / P.s2;
  pb2[p] += tb + xb;
  // u = gz z with gz = exp(j phi') conj(yhat): dx0 = Im(gz dz / u), d|u| = Re(conj(u) gz dz)/|u|
  if (mag > 0.0f) {
    float sn, cs;
    fsincos(phip[p], &sn, &cs);
    const float2 h = yh[p];
    const float2 gz = make_float2(cs * h.x + sn * h.y, sn * h.x - cs * h.y);  // exp(j phi') conj(yhat)
    const float inv2 = 1.0f / (mag * mag);
    // j conj(gz / u) = j conj(gz) u / |u|^2 ; u conj(gz) / |u|
    const float2 cgzu = make_float2(gz.x * ur + gz.y * ui, gz.x * ui - gz.y * ur);  // conj(gz) u
    zbar[p] = make_float2(xb * (-cgzu.y) * inv2 + mb * cgzu.x / mag, xb * cgzu.x * inv2 + mb * cgzu.y / mag);
  }
}
// QGGMRF edge shape and its derivative in d (zero at d = 0, where it is unbounded)
__device__ __forceinline__ void g_shape(float d, const GradPrm& P, float& sh, float& dsh, float& dsh_dsig) {
  const float ad = fabsf(d);
  const float v = P.pmq > 0.0f ? (ad > 0.0f ? exp2f(__builtin_fmaf(P.pmq, log2f(ad), P.lc)) : 0.0f) : 1.0f;
  const float u = 1.0f / (1.0f + v);
  sh = u * __builtin_fmaf(1.0f - P.qop, u, P.qop);
  const float dsh_dv = (P.qop - 2.0f - P.qop * v) * u * u * u;
  dsh = (P.pmq > 0.0f && ad > 0.0f) ? dsh_dv * P.pmq * v / d : 0.0f;
  dsh_dsig = P.pmq > 0.0f ? dsh_dv * (-P.pmq * v / P.sig_r) : 0.0f;
}
// r pass C reversed, part a: colour-C pixels turn their adjoint into (Abar,
// Bbar, sbar), their own old value's adjoint and the sigma_r gradient.  One
// thread per quad; Abar and Bbar are written at colour-C pixels only (part b
// reads nothing else) and sbar is assigned (each pixel once over the passes).
template <int C>
__device__ __forceinline__ void g_rback_a_body(const float* rin, const float* rout, const float* s,
                                                   const GradPrm* Pd, float* rbar, float* sbar, float* Abar,
                                                   float* Bbar, float* gsr) {
  const GradPrm P = Pd[blockIdx.y];
  int qi, qj;
  if (!g_quad(qi, qj, P.N)) return;
  const int N = P.N;
  const int i = 2 * qi + (C & 1), j = 2 * qj + (C >> 1), p = g_at(i, j, N);
  const int nb[8][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {-1, 1}, {1, -1}, {1, 1}};
  const float ri = rin[p];
  float A = 0.f, B = 0.f;
  float sh[8], dsh[8], dss[8], rq[8], W[8];
  bool ok[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ii = i + nb[e][0], jj = j + nb[e][1];
    ok[e] = ii >= 0 && ii < N && jj >= 0 && jj < N;
    rq[e] = ok[e] ? rin[g_at(ii, jj, N)] : 0.f;
    W[e] = ok[e] ? P.inv_sp * (e < 4 ? 1.0f / 6.0f : 1.0f / 12.0f) : 0.f;
    g_shape(ri - rq[e], P, sh[e], dsh[e], dss[e]);
    A += W[e] * sh[e];
    B += W[e] * sh[e] * rq[e];
  }
  const float g = rbar[p];
  const float rho = rout[p];
  float ab = 0.f, bb = 0.f, sb = 0.f, own = 0.f;
  if (rho > P.fl) {         // floored: no dependence on the inputs
    if (!(A > 0.0f)) {      // no prior: rho = s
      sb = g;
    } else {
      const float fp = (3.0f * A * rho - 2.0f * B) * rho + 1.0f;
      if (fp != 0.0f) {
        const float inv = 1.0f / fp;
        ab = -g * rho * rho * rho * inv;
        bb = g * rho * rho * inv;
        sb = g * inv;
        float gs = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (!ok[e]) continue;
          const float shb = W[e] * (ab + bb * rq[e]);  // adjoint of sh_e
          own += shb * dsh[e];
          // d(W sh)/d sigma_r = -2 W sh / sigma_r + W dsh/dsigma
          gs += (ab + bb * rq[e]) * (-2.0f * W[e] * sh[e] / P.sig_r + W[e] * dss[e]);
        }
        gsr[p] += gs;
      }
    }
  }
  Abar[p] = ab;
  Bbar[p] = bb;
  sbar[p] = sb;
  rbar[p] = own;
}
// E-step and Eq. (3) reversed at one pixel: (mubar, sbar, r0bar) -> bbar
// (returned), rbar of the previous state (assigned), s2 (accumulated)
__device__ __forceinline__ float2 g_estep_bar_px(float2 bv, float2 mb, float rprev, float r, float sb, const GradPrm& P,
                                                 float& rbar, float& gs2) {
  const float bb = bv.x * bv.x + bv.y * bv.y;
  const float den = r + P.s2, w = r / den;
  const float wb = (mb.x * bv.x + mb.y * bv.y) + sb * (P.s2 + 2.0f * w * bb);
  float2 gb = make_float2(w * mb.x + 2.0f * sb * w * w * bv.x, w * mb.y + 2.0f * sb * w * w * bv.y);
  const float g2 = sb * w - wb * r / (den * den);
  const float r0b = rbar + wb * P.s2 / (den * den);
  const float x = (1.0f - P.lam) * rprev + P.lam * P.alpha * bb;
  float rp = 0.f;
  if (x > P.fl) {
    rp = (1.0f - P.lam) * r0b;
    gb.x += 2.0f * P.lam * P.alpha * r0b * bv.x;
    gb.y += 2.0f * P.lam * P.alpha * r0b * bv.y;
  }
  rbar = rp;
  gs2 += g2;
  return gb;
}
// Column pass of the adjoint's two DFTs with the E-step adjoint between
// them: work holds the row-transformed zbar; the inverse column DFT gives
// mubar = F^H zbar, the E-step adjoint bbar, whose forward column DFT goes
// back into work (scaled by 1/N); its forward row DFT is vbar = F bbar.
// grid (N / W, streams), in place.
template <int N, int W>
__global__ __launch_bounds__(W*(N / Plan<N>::E)) void k_g_col_bwd(float2* work, const float* rprev, const float2* b,
                                                                const float* r0, const float* sbar,
                                                                const GradPrm* Pd, float* rbar, float* gs2,
                                                                const float2* __restrict__ tw) {
  constexpr int E = Plan<N>::E;
  __shared__ float2 lds[N * ColLds<W>::STRIDE];
  const GradPrm P = Pd[blockIdx.y];
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const int img = blockIdx.y * N * N;
  const int col = blockIdx.x * W + w;
  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = work[img + first_pos<N, +1>(i, t) * N + col];
  ColLds<W> L{lds + w};
  line_fft<N, +1>(v, t, L, tw);
  const float invN = 1.0f / (float)N;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int p = img + last_pos<N, +1>(i, t) * N + col;
    float rb = rbar[p], g2 = gs2[p];
    v[i] = g_estep_bar_px(b[p], cscale(v[i], invN), rprev[p], r0[p], sbar[p], P, rb, g2);
    rbar[p] = rb;
    gs2[p] = g2;
  }
  __syncthreads();
  line_fft<N, -1>(v, t, L, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) work[img + last_pos<N, -1>(i, t) * N + col] = cscale(v[i], invN);
}
// back-projection reversed: phi' adjoint += Im(conj(vbar) v), v = a exp(-j phi') yhat
__global__ __launch_bounds__(256) void k_g_bp_bar(const float2* vbar, const float2* yh, const float* phip,
                                                  const GradPrm* Pd, float* pb2) {
  const GradPrm P = Pd[blockIdx.y];
  int i, j;
  if (!g_pix(i, j, P.N)) return;
  const int p = g_at(i, j, P.N);
  if (!in_pupil(i, j, P.N, P.d2)) return;
  float sn, cs;
  fsincos(phip[p], &sn, &cs);
  const float2 v = cmul(yh[p], make_float2(cs, -sn)), vb = vbar[p];
  pb2[p] += vb.x * v.y - vb.y * v.x;
}
// tip/tilt removal reversed: pbar = pupil ? pb2 - plane(pb2) : 0, the plane
// from the psum records (first wavefront)
__global__ __launch_bounds__(256) void k_g_plane_bar(const float* pb2, const GradPrm* Pd, const double* minv,
                                                     const double* part, float* pbar) {
  const GradPrm P = Pd[blockIdx.y];
  __shared__ float sc[3];
  if (threadIdx.x < 64) {
    double t[3];
    g_wave_totals<3>(part, g_nred(P.N), t);
    if (threadIdx.x == 0) g_plane(minv, t, sc);
  }
  __syncthreads();
  int i, j;
  if (!g_pix(i, j, P.N)) return;
  const int p = g_at(i, j, P.N);
  pbar[p] = in_pupil(i, j, P.N, P.d2) ? pb2[p] - plane_val(sc[0], sc[1], sc[2], i, j, P.N) : 0.f;
}

// The r and phi sweeps are independent of each other (the phi passes read
// only kappa and theta~, fixed for the sweep), so pass C of both runs in one
// launch, forward and reversed.
template <int C>
__global__ __launch_bounds__(256) void k_g_pass(const float* rin, const float* s, const float* pin, const float* kap,
                                                const float* tth, const GradPrm* Pd, float* rout, float* pout) {
  g_rpass_body<C>(rin, s, Pd, rout);
  g_ppass_body<C>(pin, kap, tth, Pd, pout);
}
template <int C>
__global__ __launch_bounds__(256) void k_g_back_a(const float* pin, const float* pout, const float* kap,
                                                  const float* tth, const float* rin, const float* rout,
                                                  const float* s, const GradPrm* Pd, float* pbar, float* em,
                                                  float* kbar, float* tbar, float* gbeta, float* rbar, float* sbar,
                                                  float* Abar, float* Bbar, float* gsr) {
  g_pback_a_body<C>(pin, pout, kap, tth, Pd, pbar, em, kbar, tbar, gbeta);
  g_rback_a_body<C>(rin, rout, s, Pd, rbar, sbar, Abar, Bbar, gsr);
}
// Both parts b in one pass, one thread per 2 x 2 quad: each of the quad's
// three pixels not of colour C gathers from exactly its colour-C neighbours
// (2 vertical, 2 horizontal or 4 diagonal ones, known at compile time), in
// neighbour order (up, down, left, right, then the diagonals).  Neighbours
// of the other colours take no part: their em is zero in this pass and their
// Abar, Bbar belong to other passes.
__host__ __device__ constexpr int g_nb_di(int e) { return e == 0 || e == 4 || e == 5 ? -1 : (e == 1 || e == 6 || e == 7 ? 1 : 0); }
__host__ __device__ constexpr int g_nb_dj(int e) { return e == 2 || e == 4 || e == 6 ? -1 : (e == 3 || e == 5 || e == 7 ? 1 : 0); }
template <int C>
__global__ __launch_bounds__(256) void k_g_back_b(const float* em, const float* rin, const float* Abar,
                                                  const float* Bbar, const GradPrm* Pd, float* pbar, float* rbar) {
  const GradPrm P = Pd[blockIdx.y];
  int qi, qj;
  if (!g_quad(qi, qj, P.N)) return;
  const int N = P.N;
  static_for<0, 4>([&](auto qq) {
    constexpr int q = decltype(qq)::value;
    if constexpr (q != C) {
      constexpr int a = q & 1, b = q >> 1;
      const int i = 2 * qi + a, j = 2 * qj + b, p = g_at(i, j, N);
      const bool inp = in_pupil(i, j, N, P.d2);
      const float rj = rin[p];
      float accp = 0.f, accr = 0.f;
      static_for<0, 8>([&](auto ee) {
        constexpr int e = decltype(ee)::value;
        constexpr int di = g_nb_di(e), dj = g_nb_dj(e);
        if constexpr (((a + di) & 1) + 2 * ((b + dj) & 1) == C) {
          const int ii = i + di, jj = j + dj;
          if (ii >= 0 && ii < N && jj >= 0 && jj < N) {
            const int qn = g_at(ii, jj, N);
            if (inp) accp += (e < 4 ? 1.0f / 6.0f : 1.0f / 12.0f) * em[qn];
            const float ab = Abar[qn], bb = Bbar[qn];
            if (!(ab == 0.0f && bb == 0.0f)) {
              float sh, dsh, dss;
              g_shape(rin[qn] - rj, P, sh, dsh, dss);
              const float W = P.inv_sp * (e < 4 ? 1.0f / 6.0f : 1.0f / 12.0f);
              accr += bb * W * sh - W * (ab + bb * rj) * dsh;
            }
          }
        }
      });
      if (inp) pbar[p] += accp;
      rbar[p] += accr;
    }
  });
}

#define DDH_G_GRID(N, B) dim3(((N) * (N) + 255) / 256, (B)), dim3(256), 0, st
#define DDH_G_QGRID(N, B) dim3(((N) * (N) / 4 + 255) / 256, (B)), dim3(256), 0, st
#define DDH_G_RGRID(N, B) dim3(g_nred(N), (B)), dim3(256), 0, st

// the frame's DFT pair with the E-step (forward) or its adjoint (backward)
// between the column passes: row pass, fused column pass, row pass
template <int N>
static hipError_t g_dfts_fwd_n(const GradFwd& a, const GradDev& d, int B, hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
  constexpr int L = 256 / T > N ? N : 256 / T;
  hipLaunchKernelGGL((k_row_plain<N, L, +1>), dim3(N / L, B), dim3(L * T), 0, st, a.v, a.work, a.tw);
  hipLaunchKernelGGL((k_g_col_fwd<N, L>), dim3(N / L, B), dim3(L * T), 0, st, a.work, a.r_in, d.prm, a.b, a.rs[0],
                     a.mu, a.s, a.tw);
  hipLaunchKernelGGL((k_row_plain<N, L, -1>), dim3(N / L, B), dim3(L * T), 0, st, a.work, a.z, a.tw);
  return hipGetLastError();
}
template <int N>
static hipError_t g_dfts_bwd_n(const GradFwd& a, const GradBwd& g, const GradDev& d, int B, hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
  constexpr int L = 256 / T > N ? N : 256 / T;
  hipLaunchKernelGGL((k_row_plain<N, L, +1>), dim3(N / L, B), dim3(L * T), 0, st, g.zbar, a.work, a.tw);
  hipLaunchKernelGGL((k_g_col_bwd<N, L>), dim3(N / L, B), dim3(L * T), 0, st, a.work, a.r_in, a.b, a.rs[0], g.sbar,
                     d.prm, g.rbar, g.gs2, a.tw);
  hipLaunchKernelGGL((k_row_plain<N, L, -1>), dim3(N / L, B), dim3(L * T), 0, st, a.work, g.vbar, a.tw);
  return hipGetLastError();
}
static hipError_t g_launch_dfts_fwd(const GradFwd& a, const GradDev& d, int N, int B, hipStream_t st) {
#define DDH_X(NN) return g_dfts_fwd_n<NN>(a, d, B, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}
static hipError_t g_launch_dfts_bwd(const GradFwd& a, const GradBwd& g, const GradDev& d, int N, int B,
                                    hipStream_t st) {
#define DDH_X(NN) return g_dfts_bwd_n<NN>(a, g, d, B, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}

hipError_t g_launch_forward(const GradFwd& a, const GradDev& d, int N, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_g_stats, DDH_G_RGRID(N, B), a.y, a.phi_in, d.prm, d.part);
  hipLaunchKernelGGL(k_g_prologue, DDH_G_GRID(N, B), a.y, a.phi_in, d.prm, d.minv, d.part, d.flag, a.yh, a.phip, a.v);
  hipError_t e = g_launch_dfts_fwd(a, d, N, B, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_g_data, DDH_G_GRID(N, B), a.yh, a.phip, a.z, d.prm, a.kap, a.tth);
  hipLaunchKernelGGL(k_g_pass<0>, DDH_G_QGRID(N, B), a.rs[0], a.s, a.phip, a.kap, a.tth, d.prm, a.rs[1], a.ps[1]);
  hipLaunchKernelGGL(k_g_pass<1>, DDH_G_QGRID(N, B), a.rs[1], a.s, a.ps[1], a.kap, a.tth, d.prm, a.rs[2], a.ps[2]);
  hipLaunchKernelGGL(k_g_pass<2>, DDH_G_QGRID(N, B), a.rs[2], a.s, a.ps[2], a.kap, a.tth, d.prm, a.rs[3], a.ps[3]);
  hipLaunchKernelGGL(k_g_pass<3>, DDH_G_QGRID(N, B), a.rs[3], a.s, a.ps[3], a.kap, a.tth, d.prm, a.rs[4], a.ps[4]);
  return hipGetLastError();
}
hipError_t g_launch_loss(const float* phi, const float* ptrue, const GradDev& d, int N, int B, float* pbar,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_g_dsum, DDH_G_RGRID(N, B), phi, ptrue, d.prm, d.part);
  hipLaunchKernelGGL(k_g_loss_bar, DDH_G_GRID(N, B), phi, ptrue, d.prm, d.part, d.loss, d.flag, pbar);
  return hipGetLastError();
}
// frame reversed: pbar (adjoint of the frame's output phase) becomes the
// adjoint of its input phase, rbar likewise for r; gs2, gsr, gbeta accumulate
hipError_t g_launch_backward(const GradFwd& a, const GradBwd& g, const GradDev& d, int N, int B, hipStream_t st) {
  // kbar, tbar (phi passes) and sbar (r passes) are assigned at every pixel
  // by the four passes, so they need no clearing
  // both sweeps reversed, pass by pass (ps[c], rs[c] = inputs of pass c, ps[0] = phi')
  const float* ps0 = a.phip;
#define DDH_BK(C)                                                                                                 \
  hipLaunchKernelGGL(k_g_back_a<C>, DDH_G_QGRID(N, B), C == 0 ? ps0 : a.ps[C], a.ps[C + 1], a.kap, a.tth, a.rs[C], \
                     a.rs[C + 1], a.s, d.prm, g.pbar, g.em, g.kbar, g.tbar, g.gbeta, g.rbar, g.sbar, g.Abar,      \
                     g.Bbar, g.gsr);                                                                             \
  hipLaunchKernelGGL(k_g_back_b<C>, DDH_G_QGRID(N, B), g.em, a.rs[C], g.Abar, g.Bbar, d.prm, g.pbar, g.rbar);
  DDH_BK(3) DDH_BK(2) DDH_BK(1) DDH_BK(0)
#undef DDH_BK
  hipLaunchKernelGGL(k_g_data_bar, DDH_G_GRID(N, B), a.yh, a.phip, a.z, a.kap, g.kbar, g.tbar, g.pbar, d.prm, g.pb2,
                     g.zbar, g.gs2);
  // z = F mu -> mubar = F^H zbar; E-step reversed; b = F^H v -> vbar = F bbar
  hipError_t e = g_launch_dfts_bwd(a, g, d, N, B, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_g_bp_bar, DDH_G_GRID(N, B), g.vbar, a.yh, a.phip, d.prm, g.pb2);
  // tip/tilt removal reversed: the plane of pb2 over the pupil, subtracted
  hipLaunchKernelGGL(k_g_psum, DDH_G_RGRID(N, B), g.pb2, d.prm, d.part);
  hipLaunchKernelGGL(k_g_plane_bar, DDH_G_GRID(N, B), g.pb2, d.prm, d.minv, d.part, g.pbar);
  return hipGetLastError();
}
// sums of gs2, gsr, gbeta: records part[(b * g_nred(N) + blk) * 3 + q], summed by the caller
hipError_t g_launch_totals(const GradBwd& g, const GradDev& d, int N, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_g_tsum, DDH_G_RGRID(N, B), g.gs2, g.gsr, g.gbeta, N, d.part);
  return hipGetLastError();
}
int g_records(int N) { return g_nred(N); }
#undef DDH_G_GRID
#undef DDH_G_QGRID
#undef DDH_G_RGRID

}  // namespace ddh
