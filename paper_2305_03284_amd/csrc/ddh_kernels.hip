// HIP kernels of the Dynamic DH-MBIR per-frame EM step for gfx950 (MI355X).
//
// Per frame and per stream (N x N grid, complex64 data, FP32 arithmetic):
//   k_stats     y -> block partials of mean / centred power (Eq. (4) Normalize)
//               phi -> block partials of the least-squares plane (RemoveTipTilt)
//   k_finalize  partials -> mean, scale, plane coefficients, reject flag
//   k_row1      rows:    a exp(-j phi') (y - mean) scale, inverse 1-D DFT   (A_phi^H, first half)
//   k_col       columns: inverse 1-D DFT -> b, Eq. (3) init, E-step -> mu,
//               forward 1-D DFT of mu                                   (A_phi^H second half, F first half)
//   k_row2      rows:    forward 1-D DFT -> z = F mu, per-pupil-pixel phase data term (kappa, theta~)
//   k_mstep     halo-tiled 4-colour sweep: r M-step (QGGMRF surrogate, cubic) and phi M-step (GMRF)
// The 2-D DFTs are unitary (scale 1/N per 2-D transform) with the exp(-2 pi i k n/N)
// kernel for the forward direction.  No MFMA: nothing here is a dense contraction.
#include "ddh_internal.h"
#include <cfloat>
#include <cmath>

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
// geometry
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool in_pupil(int i, int j, int N, float d2) {
  const int di = 2 * i - N + 1, dj = 2 * j - N + 1;
  return (float)(di * di + dj * dj) <= d2;
}
__device__ __forceinline__ float plane_at(const float* sc, int i, int j, int N) {
  const float c = 0.5f * (float)(N - 1);
  return sc[SC_C0] + sc[SC_C1] * ((float)i - c) + sc[SC_C2] * ((float)j - c);
}

// Eq. (3) initialisation and E-step statistics, shared by k_col and k_mstep so
// that both evaluate exactly the same FP32 operations.
__device__ __forceinline__ float rinit_of(float rp, float bb, float lam, float alpha, float floor_) {
  return fmaxf(__builtin_fmaf(1.0f - lam, rp, (lam * alpha) * bb), floor_);
}
__device__ __forceinline__ float wiener_of(float r, float s2) { return r / (r + s2); }
__device__ __forceinline__ float second_moment(float w, float bb, float s2) {
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
// k_set_y: store this step's frame pointers into the stream descriptors
// ---------------------------------------------------------------------------
struct YArgs {
  const float2* p[64];
};
__global__ void k_set_y(StreamDesc* const* dptrs, YArgs a, int count) {
  const int i = threadIdx.x;
  if (i < count) dptrs[i]->y = a.p[i];
}

// ---------------------------------------------------------------------------
// k_stats: per 4096-pixel block, mean and centred power of y (two passes over
// registers), and the plane-fit sums of phi over the pupil.
// grid (N*N/4096, streams), block 256
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stats(StreamDesc* const* dptrs, int with_phi) {
  const StreamDesc& D = *dptrs[blockIdx.y];
  __shared__ float red[6 * 16];
  const int N = D.N;
  const int base = blockIdx.x * STATS_PIX_PER_BLOCK;
  float2 v[16];
  float s[2] = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = D.y[base + k * 256 + threadIdx.x];
    s[0] += v[k].x;
    s[1] += v[k].y;
  }
  block_sum<2>(s, red);
  const float mr = s[0] * (1.0f / STATS_PIX_PER_BLOCK), mi = s[1] * (1.0f / STATS_PIX_PER_BLOCK);
  float m2[1] = {0.f};
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float dr = v[k].x - mr, di = v[k].y - mi;
    m2[0] += dr * dr + di * di;
  }
  block_sum<1>(m2, red);
  float ps[3] = {0.f, 0.f, 0.f};
  if (with_phi) {
    const float* phi = D.phi[D.cur];
    const float c = 0.5f * (float)(N - 1);
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
      const int idx = base + k * 256 + threadIdx.x;
      const int i = idx / N, j = idx - (idx / N) * N;
      if (in_pupil(i, j, N, D.pupil_d2)) {
        const float p = phi[idx];
        ps[0] += p;
        ps[1] += ((float)i - c) * p;
        ps[2] += ((float)j - c) * p;
      }
    }
    block_sum<3>(ps, red);
  }
  if (threadIdx.x == 0) {
    float* out = D.part + blockIdx.x * PART_STRIDE;
    out[0] = mr;
    out[1] = mi;
    out[2] = m2[0];
    out[3] = ps[0];
    out[4] = ps[1];
    out[5] = ps[2];
  }
}

// ---------------------------------------------------------------------------
// k_finalize: combine the block partials (fixed order, FP64 combine of a few
// dozen values) into mean, scale, plane and the reject flag.  grid (streams)
// ---------------------------------------------------------------------------
__global__ void k_finalize(StreamDesc* const* dptrs, int with_phi) {
  if (threadIdx.x != 0) return;
  const StreamDesc& D = *dptrs[blockIdx.x];
  const int N = D.N;
  const int nb = (N * N) / STATS_PIX_PER_BLOCK;
  double mr = 0, mi = 0;
  for (int b = 0; b < nb; ++b) {
    mr += D.part[b * PART_STRIDE + 0];
    mi += D.part[b * PART_STRIDE + 1];
  }
  mr /= nb;
  mi /= nb;
  double m2 = 0, between = 0, s0 = 0, s1 = 0, s2 = 0;
  for (int b = 0; b < nb; ++b) {
    const float* p = D.part + b * PART_STRIDE;
    m2 += p[2];
    const double dr = p[0] - mr, di = p[1] - mi;
    between += dr * dr + di * di;
    s0 += p[3];
    s1 += p[4];
    s2 += p[5];
  }
  m2 += (double)STATS_PIX_PER_BLOCK * between;
  const bool ok = (m2 > 0.0) && isfinite(m2) && isfinite(mr) && isfinite(mi);
  float* sc = D.scal;
  sc[SC_MU_RE] = (float)mr;
  sc[SC_MU_IM] = (float)mi;
  sc[SC_SCALE] = ok ? (float)sqrt((double)N * (double)N / m2) : 0.0f;
  sc[SC_FLAG] = ok ? 0.0f : 1.0f;
  double c0 = 0, c1 = 0, c2 = 0;
  if (with_phi) {
    // normal equations of the plane c0 + c1 di + c2 dj over the pupil (Cramer)
    const double* m = D.mom;
    const double a00 = m[0], a01 = m[1], a02 = m[2], a11 = m[3], a12 = m[4], a22 = m[5];
    const double det = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) + a02 * (a01 * a12 - a11 * a02);
    if (det != 0.0) {
      c0 = (s0 * (a11 * a22 - a12 * a12) - a01 * (s1 * a22 - a12 * s2) + a02 * (s1 * a12 - a11 * s2)) / det;
      c1 = (a00 * (s1 * a22 - a12 * s2) - s0 * (a01 * a22 - a12 * a02) + a02 * (a01 * s2 - s1 * a02)) / det;
      c2 = (a00 * (a11 * s2 - s1 * a12) - a01 * (a01 * s2 - s1 * a02) + s0 * (a01 * a12 - a11 * a02)) / det;
    }
  }
  sc[SC_C0] = (float)c0;
  sc[SC_C1] = (float)c1;
  sc[SC_C2] = (float)c2;
}

// k_flip: after a frame of n_k EM iterations the current state buffer index advances by n_k.
__global__ void k_flip(StreamDesc* const* dptrs, int count, int nk) {
  const int i = threadIdx.x + blockIdx.x * blockDim.x;
  if (i < count) dptrs[i]->cur = (dptrs[i]->cur + nk) & 1;
}

// ---------------------------------------------------------------------------
// k_row1: first half of A_phi^H yhat.  Row i: v = a exp(-j phi') (y - mu) scale,
// inverse 1-D DFT along the row (unnormalised) -> T.
// grid (N/LPW, streams), block LPW * N/E
// ---------------------------------------------------------------------------
template <int N, int LPW>
__global__ __launch_bounds__(LPW*(N / Plan<N>::E)) void k_row1(StreamDesc* const* dptrs, const float2* __restrict__ tw,
                                                             int k, int use_plane) {
  constexpr int E = Plan<N>::E, T = N / E;
  __shared__ float2 lds[LPW * RowLds<N>::STRIDE];
  const StreamDesc& D = *dptrs[blockIdx.y];
  const float* sc = D.scal;
  if (sc[SC_FLAG] != 0.0f) return;
  const int line = threadIdx.x / T, t = threadIdx.x - line * T;
  const int row = blockIdx.x * LPW + line;
  const float2 mu = make_float2(sc[SC_MU_RE], sc[SC_MU_IM]);
  const float scale = sc[SC_SCALE];
  const float* phi = D.phi[(D.cur + k) & 1] + row * N;
  const float2* y = D.y + row * N;
  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int n = first_pos<N, +1>(i, t);
    const float2 yv = y[n];
    const float ph = phi[n];
    if (in_pupil(row, n, N, D.pupil_d2)) {
      const float p = use_plane ? ph - plane_at(sc, row, n, N) : ph;
      float sn, cs;
      sincosf(p, &sn, &cs);
      const float2 yh = make_float2((yv.x - mu.x) * scale, (yv.y - mu.y) * scale);
      v[i] = cmul(yh, make_float2(cs, -sn));
    } else {
      v[i] = make_float2(0.f, 0.f);
    }
  }
  RowLds<N> L{lds + line * RowLds<N>::STRIDE};
  line_fft<N, +1>(v, t, L, tw);
  float2* out = D.T + row * N;
#pragma unroll
  for (int i = 0; i < E; ++i) out[last_pos<N, +1>(i, t)] = v[i];
}

// ---------------------------------------------------------------------------
// k_col: column strip of W columns.  Inverse 1-D DFT down each column and the
// 1/N scale give b = A_phi^H yhat; then per pixel the Eq. (3) initialisation
// (first EM iteration of a frame), the E-step mu = r/(r+s2) b, |b|^2 -> bb,
// and the forward 1-D DFT of mu down the column (unnormalised) -> U.
// grid (N/W, streams), block W * N/E
// ---------------------------------------------------------------------------
template <int N, int W>
__global__ __launch_bounds__(W*(N / Plan<N>::E)) void k_col(StreamDesc* const* dptrs, const float2* __restrict__ tw,
                                                          int k, int do_rinit) {
  constexpr int E = Plan<N>::E;
  __shared__ float2 lds[N * ColLds<W>::STRIDE];
  const StreamDesc& D = *dptrs[blockIdx.y];
  if (D.scal[SC_FLAG] != 0.0f) return;
  const int w = threadIdx.x % W, t = threadIdx.x / W;
  const int col = blockIdx.x * W + w;
  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = D.T[first_pos<N, +1>(i, t) * N + col];
  ColLds<W> L{lds + w};
  line_fft<N, +1>(v, t, L, tw);
  const float invN = 1.0f / (float)N;
  const float s2 = D.sigma2, lam = D.lam, alpha = D.alpha, fl = D.r_floor;
  const float* rin = D.r[(D.cur + k) & 1];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int n = last_pos<N, +1>(i, t);
    const float2 b = cscale(v[i], invN);
    const float bb = b.x * b.x + b.y * b.y;
    const float rp = rin[n * N + col];
    const float ri = do_rinit ? rinit_of(rp, bb, lam, alpha, fl) : rp;
    const float wgt = wiener_of(ri, s2);
    D.bb[n * N + col] = bb;
    v[i] = cscale(b, wgt);
  }
  __syncthreads();
  line_fft<N, -1>(v, t, L, tw);
#pragma unroll
  for (int i = 0; i < E; ++i) D.U[last_pos<N, -1>(i, t) * N + col] = v[i];
}

// ---------------------------------------------------------------------------
// k_row2: forward 1-D DFT along rows of U and the 1/N scale give z = F mu.
// Per pupil pixel, the phase data term -c cos(phi - theta),
// c = (2/s2)|yhat||z|, theta = arg(yhat conj z), is majorised at
// x0 = wrap(phi' - theta) by (kappa/2)(phi - theta~)^2 with kappa = c sinc(x0),
// theta~ = phi' - x0.  Writes (kappa, theta~) into T (zero off the pupil).
// ---------------------------------------------------------------------------
template <int N, int LPW>
__global__ __launch_bounds__(LPW*(N / Plan<N>::E)) void k_row2(StreamDesc* const* dptrs, const float2* __restrict__ tw,
                                                             int k, int use_plane) {
  constexpr int E = Plan<N>::E, T = N / E;
  __shared__ float2 lds[LPW * RowLds<N>::STRIDE];
  const StreamDesc& D = *dptrs[blockIdx.y];
  const float* sc = D.scal;
  if (sc[SC_FLAG] != 0.0f) return;
  const int line = threadIdx.x / T, t = threadIdx.x - line * T;
  const int row = blockIdx.x * LPW + line;
  float2 v[E];
  const float2* u = D.U + row * N;
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = u[first_pos<N, -1>(i, t)];
  RowLds<N> L{lds + line * RowLds<N>::STRIDE};
  line_fft<N, -1>(v, t, L, tw);
  const float invN = 1.0f / (float)N;
  const float2 mu = make_float2(sc[SC_MU_RE], sc[SC_MU_IM]);
  const float scale = sc[SC_SCALE];
  const float c2s = 2.0f / D.sigma2;
  const float* phi = D.phi[(D.cur + k) & 1] + row * N;
  const float2* y = D.y + row * N;
  float2* out = D.T + row * N;
  constexpr float kPi = 3.14159265358979323846f, k2Pi = 6.28318530717958647692f;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int m = last_pos<N, -1>(i, t);
    float2 res = make_float2(0.f, 0.f);
    if (in_pupil(row, m, N, D.pupil_d2)) {
      const float2 z = cscale(v[i], invN);
      const float2 yv = y[m];
      const float2 yh = make_float2((yv.x - mu.x) * scale, (yv.y - mu.y) * scale);
      const float p = use_plane ? phi[m] - plane_at(sc, row, m, N) : phi[m];
      const float c = c2s * sqrtf(yh.x * yh.x + yh.y * yh.y) * sqrtf(z.x * z.x + z.y * z.y);
      // yhat conj(z)
      const float qr = yh.x * z.x + yh.y * z.y, qi = yh.y * z.x - yh.x * z.y;
      const float theta = atan2f(qi, qr);
      const float x = p - theta;
      float x0 = x - k2Pi * floorf((x + kPi) * (1.0f / k2Pi));
      if (x0 >= kPi) x0 -= k2Pi;
      if (x0 < -kPi) x0 += k2Pi;
      const float sinc = fabsf(x0) > 1e-4f ? sinf(x0) / x0 : 1.0f - x0 * x0 * (1.0f / 6.0f);
      res = make_float2(c * sinc, p - x0);
    }
    out[m] = res;
  }
}

// ---------------------------------------------------------------------------
// r M-step pixel solve: global minimiser on (0, inf) of
//   h(rho) = log rho + s/rho + (A/2) rho^2 - B rho
// via the stationarity cubic A rho^3 - B rho^2 + rho - s = 0 (all real roots
// are positive for s > 0, A > 0, B >= 0).  One real root: Cardano; three:
// trigonometric form; each root polished by guarded Newton steps.  With three
// roots the middle one is a local maximum of h; the outer two are compared by
// h(rho1) - h(rho3) written as one difference; ties take the smaller root.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float cubic_f(float A, float B, float s, float x) {
  return __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(A, x, -B), x, 1.0f), x, -s);
}
__device__ __forceinline__ float polish(float A, float B, float s, float x) {
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const float f = cubic_f(A, B, s, x);
    const float fp = __builtin_fmaf(__builtin_fmaf(3.0f * A, x, -2.0f * B), x, 1.0f);
    if (fp != 0.0f) {
      const float xn = x - f / fp;
      if (xn > 0.0f && fabsf(cubic_f(A, B, s, xn)) < fabsf(f)) x = xn;
    }
  }
  return x;
}
__device__ float solve_r(float s, float A, float B) {
  if (!(A > 0.0f)) return s;
  const float iA = 1.0f / A;
  const float a2 = -B * iA, a1 = iA, a0 = -s * iA;
  const float sh = -a2 * (1.0f / 3.0f);
  const float p = a1 - a2 * a2 * (1.0f / 3.0f);
  const float q = (2.0f / 27.0f) * a2 * a2 * a2 - a2 * a1 * (1.0f / 3.0f) + a0;
  const float disc = 0.25f * q * q + (1.0f / 27.0f) * p * p * p;
  if (disc >= 0.0f || p >= 0.0f) {
    const float sq = sqrtf(fmaxf(disc, 0.0f));
    const float u = cbrtf(-0.5f * q - copysignf(sq, q));
    const float t = (u != 0.0f) ? u - p / (3.0f * u) : 0.0f;
    float x = t + sh;
    if (!(x > 0.0f) || !isfinite(x)) x = s;
    return polish(A, B, s, x);
  }
  const float m = sqrtf(-p * (1.0f / 3.0f));
  float arg = (1.5f * q / p) * sqrtf(-3.0f / p);
  arg = fminf(1.0f, fmaxf(-1.0f, arg));
  const float th = acosf(arg) * (1.0f / 3.0f);
  constexpr float k2Pi3 = 2.09439510239319549231f;
  float x1 = 2.0f * m * cosf(th) + sh;
  float x2 = 2.0f * m * cosf(th - k2Pi3) + sh;
  float x3 = 2.0f * m * cosf(th - 2.0f * k2Pi3) + sh;
  // sort ascending
  float lo = fminf(fminf(x1, x2), x3), hi = fmaxf(fmaxf(x1, x2), x3);
  if (!(lo > 0.0f)) lo = fminf(s, hi);
  lo = polish(A, B, s, lo);
  hi = polish(A, B, s, hi);
  // h(lo) - h(hi)
  const float dh = logf(lo / hi) + s * (hi - lo) / (lo * hi) + (lo - hi) * (0.5f * A * (lo + hi) - B);
  return dh <= 0.0f ? lo : hi;
}

// rho'(d)/d of the QGGMRF prior for p = 2:
//   (1/sig^2) (1 + (q/2) v) / (1 + v)^2,  v = |d/(T sig)|^(2-q)
__device__ __forceinline__ float qg_weight(float d, float inv_sp, float inv_Ts, float pmq, float qop) {
  const float ad = fabsf(d) * inv_Ts;
  const float v = ad > 0.0f ? exp2f(pmq * log2f(ad)) : 0.0f;
  const float den = 1.0f + v;
  return inv_sp * __builtin_fmaf(qop, v, 1.0f) / (den * den);
}

// ---------------------------------------------------------------------------
// k_mstep: one 4-colour sweep of the r and phi M-steps on a TS x TS output
// tile.  The tile and a 4-pixel halo are staged in LDS; pass c updates the
// colour-c pixels of the region shrunk by c+1, so the inner tile sees exactly
// the values a whole-grid sweep produces.  Colour(i, j) = (i mod 2) + 2 (j mod 2).
// Reads state buffer in = (cur + k) & 1, writes in ^ 1.
// grid (tiles, streams), block 256; blocks are remapped so that neighbouring
// tiles of a stream run on the same XCD (shared L2 for the halo).
// ---------------------------------------------------------------------------
template <int N, int TS>
__global__ __launch_bounds__(256) void k_mstep(StreamDesc* const* dptrs, int k, int use_plane, int do_rinit) {
  constexpr int RS = TS + 8;
  constexpr int TPR = N / TS;          // tiles per row
  constexpr int TILES = TPR * TPR;
  __shared__ float sR[RS * RS], sS[RS * RS], sP[RS * RS], sK[RS * RS], sT[RS * RS];
  // XCD-aware remap of the linear block id
  const int total = TILES * gridDim.y;
  const int L = blockIdx.x + blockIdx.y * TILES;
  const int logical = (total % 8 == 0) ? (L % 8) * (total / 8) + (L / 8) : L;
  const int g = logical / TILES, tile = logical - g * TILES;
  const StreamDesc& D = *dptrs[g];
  const int ti = tile / TPR, tj = tile - ti * TPR;
  const int gi0 = ti * TS - 4, gj0 = tj * TS - 4;
  const int in = (D.cur + k) & 1;
  const float* rin = D.r[in];
  const float* pin = D.phi[in];
  float* rout = D.r[in ^ 1];
  float* pout = D.phi[in ^ 1];
  const float* sc = D.scal;
  const float d2 = D.pupil_d2;
  if (sc[SC_FLAG] != 0.0f) {  // rejected frame: carry the state over unchanged
    for (int idx = threadIdx.x; idx < TS * TS; idx += blockDim.x) {
      const int gi = ti * TS + idx / TS, gj = tj * TS + idx % TS;
      rout[gi * N + gj] = rin[gi * N + gj];
      pout[gi * N + gj] = pin[gi * N + gj];
    }
    return;
  }
  const float s2 = D.sigma2, lam = D.lam, alpha = D.alpha, fl = D.r_floor, beta2 = 2.0f * D.beta;
  for (int idx = threadIdx.x; idx < RS * RS; idx += blockDim.x) {
    const int li = idx / RS, lj = idx - li * RS;
    const int gi = gi0 + li, gj = gj0 + lj;
    float r = 0.f, s = 0.f, p = 0.f, ka = 0.f, tt = 0.f;
    if (gi >= 0 && gi < N && gj >= 0 && gj < N) {
      const int pidx = gi * N + gj;
      const float rp = rin[pidx];
      const float bb = D.bb[pidx];
      r = do_rinit ? rinit_of(rp, bb, lam, alpha, fl) : rp;
      s = second_moment(wiener_of(r, s2), bb, s2);
      if (in_pupil(gi, gj, N, d2)) {
        p = use_plane ? pin[pidx] - plane_at(sc, gi, gj, N) : pin[pidx];
        const float2 kt = D.T[pidx];
        ka = kt.x;
        tt = kt.y;
      }
    }
    sR[idx] = r;
    sS[idx] = s;
    sP[idx] = p;
    sK[idx] = ka;
    sT[idx] = tt;
  }
  __syncthreads();
  const float inv_sp = D.qg_inv_sp, inv_Ts = D.qg_inv_Ts, pmq = D.qg_pmq, qop = D.qg_qop;
  constexpr float kE = 1.0f / 6.0f, kD = 1.0f / 12.0f;
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const int lo = c + 1, hi = RS - c - 1;  // region [lo, hi)
    const int pi_ = c & 1, pj_ = c >> 1;     // required parities of gi, gj
    const int li0 = lo + (((gi0 + lo) & 1) != pi_);
    const int lj0 = lo + (((gj0 + lo) & 1) != pj_);
    const int nu = (hi - li0 + 1) >> 1, nv = (hi - lj0 + 1) >> 1;
    for (int idx = threadIdx.x; idx < nu * nv; idx += blockDim.x) {
      const int u = idx / nv;
      const int li = li0 + 2 * u, lj = lj0 + 2 * (idx - u * nv);
      const int gi = gi0 + li, gj = gj0 + lj;
      if (gi < 0 || gi >= N || gj < 0 || gj >= N) continue;
      const int o = li * RS + lj;
      const bool up = gi > 0, dn = gi < N - 1, lf = gj > 0, rt = gj < N - 1;
      // ---- r update
      const float rp = sR[o];
      float A = 0.f, B = 0.f;
#define DDH_RNB(ok, off, bw)                                              \
  if (ok) {                                                               \
    const float rq = sR[o + (off)];                                       \
    const float wq = (bw) * qg_weight(rp - rq, inv_sp, inv_Ts, pmq, qop); \
    A += wq;                                                              \
    B = __builtin_fmaf(wq, rq, B);                                        \
  }
      DDH_RNB(up, -RS, kE)
      DDH_RNB(dn, RS, kE)
      DDH_RNB(lf, -1, kE)
      DDH_RNB(rt, 1, kE)
      DDH_RNB(up && lf, -RS - 1, kD)
      DDH_RNB(up && rt, -RS + 1, kD)
      DDH_RNB(dn && lf, RS - 1, kD)
      DDH_RNB(dn && rt, RS + 1, kD)
#undef DDH_RNB
      sR[o] = fmaxf(solve_r(sS[o], A, B), fl);
      // ---- phi update (pupil pixels only; neighbours must be in the pupil)
      if (in_pupil(gi, gj, N, d2)) {
        float P = 0.f, Ph = 0.f;
#define DDH_PNB(ok, di, dj, off, bw)                     \
  if ((ok) && in_pupil(gi + (di), gj + (dj), N, d2)) { \
    P += (bw);                                         \
    Ph = __builtin_fmaf((bw), sP[o + (off)], Ph);      \
  }
        DDH_PNB(up, -1, 0, -RS, kE)
        DDH_PNB(dn, 1, 0, RS, kE)
        DDH_PNB(lf, 0, -1, -1, kE)
        DDH_PNB(rt, 0, 1, 1, kE)
        DDH_PNB(up && lf, -1, -1, -RS - 1, kD)
        DDH_PNB(up && rt, -1, 1, -RS + 1, kD)
        DDH_PNB(dn && lf, 1, -1, RS - 1, kD)
        DDH_PNB(dn && rt, 1, 1, RS + 1, kD)
#undef DDH_PNB
        const float ka = sK[o];
        const float den = ka + beta2 * P;
        if (den > 0.0f) sP[o] = (ka * sT[o] + beta2 * Ph) / den;
      }
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < TS * TS; idx += blockDim.x) {
    const int li = 4 + idx / TS, lj = 4 + idx % TS;
    const int gi = gi0 + li, gj = gj0 + lj;
    const int o = li * RS + lj;
    rout[gi * N + gj] = sR[o];
    pout[gi * N + gj] = in_pupil(gi, gj, N, d2) ? sP[o] : 0.0f;
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
__device__ __forceinline__ double qg_rho_d(double d, const StreamDesc& D) {
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
  const StreamDesc& D = *dp;
  __shared__ double red[16];
  const int N = D.N;
  const float* r = D.r[parity];
  const float* phi = D.phi[parity];
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
    const bool pi_ = in_pupil(i, j, N, D.pupil_d2);
    for (int q = 0; q < 4; ++q) {
      const int ii = i + offs[q][0], jj = j + offs[q][1];
      if (ii < 0 || ii >= N || jj < 0 || jj >= N) continue;
      const int o = ii * N + jj;
      acc[0] += bw[q] * qg_rho_d(ri - (double)r[o], D);
      if (pi_ && in_pupil(ii, jj, N, D.pupil_d2)) {
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
  const StreamDesc& D = *dp;
  __shared__ double red[3 * 16];
  const int N = D.N;
  const float* phi = D.phi[parity];
  const double c = 0.5 * (N - 1);
  double acc[3] = {0, 0, 0};
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N * N; idx += gridDim.x * blockDim.x) {
    const int i = idx / N, j = idx - i * N;
    if (!in_pupil(i, j, N, D.pupil_d2)) continue;
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
  const StreamDesc& D = *dp;
  const int N = D.N;
  const float* phi = D.phi[parity];
  const double c = 0.5 * (N - 1);
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N * N; idx += gridDim.x * blockDim.x) {
    const int i = idx / N, j = idx - i * N;
    float2 f = make_float2(0.f, 0.f);
    if (in_pupil(i, j, N, D.pupil_d2)) {
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
  const StreamDesc& D = *dp;
  const float* sc = D.scal;
  const int line = threadIdx.x / T, t = threadIdx.x - line * T;
  const int row = blockIdx.x * LPW + line;
  const float2 mu = make_float2(sc[SC_MU_RE], sc[SC_MU_IM]);
  const float scale = sc[SC_SCALE];
  const float* phi = D.phi[parity] + row * N;
  const float2* y = D.y + row * N;
  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int n = first_pos<N, +1>(i, t);
    if (in_pupil(row, n, N, D.pupil_d2)) {
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

__global__ void k_fill_zero(float* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}
__global__ void k_copy(float* dst, const float* src, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// launch wrappers: runtime dispatch on N and on the tile configuration
// ---------------------------------------------------------------------------
#define DDH_DISPATCH_N(N, MACRO) \
  switch (N) {                   \
    case 64: MACRO(64); break;   \
    case 128: MACRO(128); break; \
    case 256: MACRO(256); break; \
    case 512: MACRO(512); break; \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_set_y(StreamDesc* const* dptrs, const float2* const* ys, int count, hipStream_t st) {
  for (int off = 0; off < count; off += 64) {
    YArgs a{};
    const int n = count - off < 64 ? count - off : 64;
    for (int i = 0; i < n; ++i) a.p[i] = ys[off + i];
    hipLaunchKernelGGL(k_set_y, dim3(1), dim3(64), 0, st, dptrs + off, a, n);
  }
  return hipGetLastError();
}

hipError_t launch_stats(StreamDesc* const* dptrs, int count, int N, int with_phi, hipStream_t st) {
  hipLaunchKernelGGL(k_stats, dim3((N * N) / STATS_PIX_PER_BLOCK, count), dim3(256), 0, st, dptrs, with_phi);
  return hipGetLastError();
}

hipError_t launch_finalize(StreamDesc* const* dptrs, int count, int with_phi, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(count), dim3(64), 0, st, dptrs, with_phi);
  return hipGetLastError();
}

hipError_t launch_flip(StreamDesc* const* dptrs, int count, int nk, hipStream_t st) {
  hipLaunchKernelGGL(k_flip, dim3((count + 63) / 64), dim3(64), 0, st, dptrs, count, nk);
  return hipGetLastError();
}

template <int N>
static hipError_t row1_n(StreamDesc* const* d, int count, const float2* tw, int k, int use_plane, int lpw,
                         hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
#define DDH_R1(L)                                                                                     \
  case L:                                                                                             \
    hipLaunchKernelGGL((k_row1<N, L>), dim3(N / L, count), dim3(L * T), 0, st, d, tw, k, use_plane); \
    break;
  switch (lpw) {
    DDH_R1(4) DDH_R1(8) DDH_R1(16) DDH_R1(32)
    default: return hipErrorInvalidValue;
  }
#undef DDH_R1
  return hipGetLastError();
}
template <int N>
static hipError_t row2_n(StreamDesc* const* d, int count, const float2* tw, int k, int use_plane, int lpw,
                         hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
#define DDH_R2(L)                                                                                     \
  case L:                                                                                             \
    hipLaunchKernelGGL((k_row2<N, L>), dim3(N / L, count), dim3(L * T), 0, st, d, tw, k, use_plane); \
    break;
  switch (lpw) {
    DDH_R2(4) DDH_R2(8) DDH_R2(16) DDH_R2(32)
    default: return hipErrorInvalidValue;
  }
#undef DDH_R2
  return hipGetLastError();
}
template <int N>
static hipError_t col_n(StreamDesc* const* d, int count, const float2* tw, int k, int do_rinit, int w,
                        hipStream_t st) {
  constexpr int T = N / Plan<N>::E;
#define DDH_C(W)                                                                                    \
  case W:                                                                                           \
    hipLaunchKernelGGL((k_col<N, W>), dim3(N / W, count), dim3(W * T), 0, st, d, tw, k, do_rinit); \
    break;
  switch (w) {
    DDH_C(4) DDH_C(8) DDH_C(16) DDH_C(32)
    default: return hipErrorInvalidValue;
  }
#undef DDH_C
  return hipGetLastError();
}
template <int N>
static hipError_t mstep_n(StreamDesc* const* d, int count, int k, int use_plane, int do_rinit, int ts,
                          hipStream_t st) {
#define DDH_M(TS)                                                                                          \
  case TS:                                                                                                 \
    if (N % TS) return hipErrorInvalidValue;                                                              \
    hipLaunchKernelGGL((k_mstep<N, TS>), dim3((N / TS) * (N / TS), count), dim3(256), 0, st, d, k,      \
                       use_plane, do_rinit);                                                               \
    break;
  switch (ts) {
    DDH_M(16) DDH_M(32) DDH_M(64)
    default: return hipErrorInvalidValue;
  }
#undef DDH_M
  return hipGetLastError();
}

static bool lpw_ok(int N, int lpw) {
  const int T = N / (N == 64 ? 8 : 16);
  return lpw * T <= 1024 && N % lpw == 0;
}
static bool w_ok(int N, int w) {
  const int T = N / (N == 64 ? 8 : 16);
  return w * T <= 1024 && N % w == 0;
}

hipError_t launch_row1(StreamDesc* const* d, int count, int N, const float2* tw, int k, int use_plane,
                       const TileConfig& tc, hipStream_t st) {
  if (!lpw_ok(N, tc.row_lines)) return hipErrorInvalidValue;
#define DDH_X(NN) return row1_n<NN>(d, count, tw, k, use_plane, tc.row_lines, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}
hipError_t launch_col(StreamDesc* const* d, int count, int N, const float2* tw, int k, int do_rinit,
                      const TileConfig& tc, hipStream_t st) {
  if (!w_ok(N, tc.col_width)) return hipErrorInvalidValue;
#define DDH_X(NN) return col_n<NN>(d, count, tw, k, do_rinit, tc.col_width, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}
hipError_t launch_row2(StreamDesc* const* d, int count, int N, const float2* tw, int k, int use_plane,
                       const TileConfig& tc, hipStream_t st) {
  if (!lpw_ok(N, tc.row_lines)) return hipErrorInvalidValue;
#define DDH_X(NN) return row2_n<NN>(d, count, tw, k, use_plane, tc.row_lines, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
}
hipError_t launch_mstep(StreamDesc* const* d, int count, int N, int k, int use_plane, int do_rinit,
                        const TileConfig& tc, hipStream_t st) {
#define DDH_X(NN) return mstep_n<NN>(d, count, k, use_plane, do_rinit, tc.m_tile, st)
  DDH_DISPATCH_N(N, DDH_X)
#undef DDH_X
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

}  // namespace ddh
