// Internal declarations shared by the kernel and runtime translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ddh {

// Per-stream scalars written by the finalize kernel (float slots).
enum ScalarSlot {
  SC_MU_RE = 0,   // complex mean of y
  SC_MU_IM = 1,
  SC_SCALE = 2,   // sqrt(N^2) / ||y - mean||
  SC_C0 = 3,      // least-squares plane over the pupil: c0 + c1*(i-c) + c2*(j-c)
  SC_C1 = 4,
  SC_C2 = 5,
  SC_FLAG = 6,    // 1 = frame rejected (Normalize undefined)
  SC_COUNT = 8
};

// Stats partials per block: mean_re, mean_im, M2, sum phi, sum (i-c) phi, sum (j-c) phi.
constexpr int PART_STRIDE = 8;

// Device-visible descriptor of one stream; an array of these (grouped by N)
// lives in device memory for every plan.
struct StreamDesc {
  const float2* y;     // current frame (set per step)
  float* r[2];         // ping-pong reflectance state
  float* phi[2];       // ping-pong phase state
  float2* T;           // row-pass output / (kappa, theta~) after the second row pass
  float2* U;           // column-pass output
  float* bb;           // |b|^2 from the column pass
  float* part;         // statistics records, PART_STRIDE floats per grid row
  float* scal;         // SC_COUNT floats
  // the aperture a (D_a), one byte per pixel: prior weight of the aperture
  // neighbours in twelfths (bits 0-3: 2 per edge and 1 per diagonal
  // neighbour inside the aperture) and the in-aperture flag (bit 4); zero
  // off the aperture.  Read-only: for a circular pupil shared by the streams
  // of one device, N and diameter; for an aperture array the stream's own.
  const unsigned char* geo;
  // work-list control words (persistent frame kernel), CTL_WORDS unsigned:
  // queue tickets and the finished-workgroup count (used in the first
  // stream of a launch), this stream's stage counters and its give-up flag
  unsigned* ctl;
  int N;
  int cur;             // index of the current state buffer at the start of a frame
  float sigma2, lam, alpha, beta, r_floor;
  float qg_p, qg_q, qg_T, qg_sigma;
  // precomputed QGGMRF constants
  float qg_inv_sp;     // 1 / sigma^p (halved when q = p, see qg_pmq)
  float qg_inv_Ts;     // 1 / (T sigma)
  float qg_pmq;        // p - q; 1e-30 when q = p (with qg_lc = -256)
  float qg_qop;        // q / p
  float qg_pm2;        // p - 2
  float qg_lc;         // (p - q) log2(1 / (T sigma))
  // pupil moments for the plane fit (exact, host-computed):
  // n, sum di, sum dj, sum di^2, sum di dj, sum dj^2 with di = i-c, dj = j-c
  double mom[6];
  // inverse of the symmetric 3x3 moment matrix [[n, Sdi, Sdj], [Sdi, Sdi2, Sdidj],
  // [Sdj, Sdidj, Sdj2]] as (00, 01, 02, 11, 12, 22); zero if singular
  double minv[6];
};

// Work-list control words of a stream (offsets in unsigned words; the
// tickets, the stage counters and the flag sit on different cache lines).
constexpr int CTL_TICKETS = 0;    // [0, 16): one ticket counter per XCD queue
constexpr int CTL_FINISHED = 16;  // workgroups of the launch that have finished
constexpr int CTL_STAGE = 32;     // [32, 36): completed items per stage (stats, row1, col, row2)
constexpr int CTL_ROWS = 40;      // fused first row pass: rows whose statistics records are stored
constexpr int CTL_ROWS_DONE = 41; // fused first row pass: workgroups past their wait
constexpr int CTL_XCC = 42;       // fused first row pass: XCC_ID + 1 of the stream's first block (0: none yet)
constexpr int CTL_GIVEUP = 48;    // nonzero: a wait of this stream gave up
constexpr int CTL_WORDS = 64;
constexpr int CTL_MAX_QUEUES = 16;

// Launch-site configuration (autotuned per N).
struct TileConfig {
  int row_lines;   // lines per workgroup in the row kernels
  int col_width;   // columns per workgroup in the column kernel
  int m_tile_h;    // output tile height of the M-step kernel
  int m_tile_w;    // output tile width of the M-step kernel
};

// Kernel kinds for per-stage timing.
enum KernelKind { KK_STATS = 0, KK_FINAL, KK_ROW1, KK_COL, KK_ROW2, KK_MSTEP, KK_BEGIN, KK_FRAME, KK_ROW1S, KK_COUNT };

// Twiddle tables: exp(-2 pi i m / N) for m < N, for N = 64,128,256,512,
// concatenated at offsets 0, 64, 192, 448 (total 960).
int twiddle_offset(int N);
constexpr int TWIDDLE_TOTAL = 960;

// Timing of frame-kernel launches: while stop is set, the frame-kernel
// launches of this thread record start at the first kernel's own start and
// stop at each kernel's own end (so the last one's end stays), as a profiler
// would time them; launches counts them.  Set around one launch call by a
// batch's timing mode and cleared afterwards.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  int launches = 0;
};
LaunchEvents& launch_events();

// --- launch wrappers (defined in ddh_kernels.hip) ---------------------------
// dptrs: device array of device descriptor pointers for the streams of one
// launch (one grid size N for the per-N kernels).  k: EM iteration index
// within the frame; the state buffer read is (cur + k) & 1.
// Frame start: ys[i] is stream i's frame and curs[i] its current state buffer
// (host-tracked).  launch_begin stores both in the descriptors; launch_stats
// with ys != nullptr stores them itself (the later kernels of the frame read
// them from the descriptors), with ys == nullptr it reads them there.  With
// ds != nullptr (host array of the streams' device descriptor pointers)
// launch_stats also fills the device list dptrs[0..count) for the later
// kernels of the frame.
hipError_t launch_begin(StreamDesc* const* dptrs, const float2* const* ys, const int* curs, int count,
                        hipStream_t st);
hipError_t launch_stats(StreamDesc* const* dptrs, int count, int N, int with_phi, const float2* const* ys,
                        const int* curs, StreamDesc* const* ds, hipStream_t st);
hipError_t launch_finalize(StreamDesc* const* dptrs, int count, int N, int with_phi, hipStream_t st);
hipError_t launch_row1(StreamDesc* const* dptrs, int count, int N, const float2* tw, int k, int use_plane,
                       int fin, int with_phi, const TileConfig& tc, hipStream_t st);
hipError_t launch_col(StreamDesc* const* dptrs, int count, int N, const float2* tw, int k, int do_rinit,
                      const TileConfig& tc, hipStream_t st);
hipError_t launch_row2(StreamDesc* const* dptrs, int count, int N, const float2* tw, int k, int use_plane,
                       const TileConfig& tc, hipStream_t st);
hipError_t launch_mstep(StreamDesc* const* dptrs, int count, int N, int k, int use_plane, int do_rinit,
                        const TileConfig& tc, hipStream_t st);
// Persistent frame kernel: the stats (k == 0), row1, column and row2 stages
// of `count` streams of one N as one work list (same results as the four
// eager launches).  Frame start as for launch_stats (ys == nullptr: from the
// descriptors).  ctl0: control words of the launch (the first stream's);
// nq: XCD queues; lag: slots between consecutive stages of a stream;
// spin_limit: polls before a wait gives up; giveup != 0 makes every wait
// give up at once (failure-path tests).  whole_image: the M-step runs as
// whole-image colour passes (the column and row2 stages then also write the
// passes' working copies of r and phi).  share in (0, 1]: the part of the
// device this launch may fill (its persistent grid is that fraction of three
// workgroups per CU), for launches of several groups that run at once.
hipError_t launch_frame(StreamDesc* const* dptrs, int count, int N, const float2* tw, int k, int mode,
                        const float2* const* ys, const int* curs, StreamDesc* const* ds, unsigned* ctl0, int nq,
                        int lag, unsigned spin_limit, int giveup, int whole_image, float share, hipStream_t st);

// First EM iteration's first row pass of `count` streams of one N with the
// frame's Normalize and RemoveTipTilt statistics formed in the same launch
// (replaces launch_stats + the k = 0 launch_row1; same results).  Frame start
// as for launch_stats.  spin_limit: polls before a block's wait for its
// stream's other rows gives up (the stream's give-up word is then set); nq:
// the device's XCD count.
hipError_t launch_row1s(StreamDesc* const* dptrs, int count, int N, const float2* tw, int with_phi,
                        const float2* const* ys, const int* curs, StreamDesc* const* ds, unsigned spin_limit,
                        int nq, const TileConfig& tc, hipStream_t st);

// Plain batched unitary 2D DFT (no fusion): rows into work, columns into out.
hipError_t launch_fft2(int N, int count, const float2* in, float2* out, float2* work,
                       const float2* tw, int inverse, hipStream_t st);

// Diagnostics (FP64 reductions) on one stream; d is its device descriptor.
hipError_t launch_backproject_cur(const StreamDesc* d, int N, int parity, const float2* tw,
                                  float2* b, float2* work, hipStream_t st);
hipError_t launch_cost_terms(const StreamDesc* d, int parity, const float2* b, double* partials,
                             int nparts, hipStream_t st);
hipError_t launch_strehl_sums(const StreamDesc* d, int parity, const float* phi_true,
                              double* partials, int nparts, hipStream_t st);
hipError_t launch_strehl_field(const StreamDesc* d, int N, int parity, const float* phi_true,
                               const double* coef, float2* field, hipStream_t st);
hipError_t launch_max_abs2(const float2* x, int n, double* partials, int nparts, hipStream_t st);
hipError_t launch_fill_zero(float* p, long long n, hipStream_t st);
hipError_t launch_synth_frames(float2* y, long long n, unsigned int seed, hipStream_t st);
hipError_t launch_copy(float* dst, const float* src, long long n, hipStream_t st);
hipError_t launch_copy_pupil(float* dst, const float* src, int N, const unsigned char* geo, hipStream_t st);

// --- unrolled frames with a hand-written adjoint (ddh_kernels.hip) ---------
// one stream's constants (a device array of these, one per stream of a batch)
struct GradPrm {
  int N;
  float d2, lam, alpha, fl, s2, inv_sp, lc, pmq, qop, beta, sig_r;
};
struct GradLoss {
  float dmean, inv_nL;
  double loss;
};
// device scalars of a batch of B streams of one N
struct GradDev {
  const GradPrm* prm;  // [B]
  const double* minv;  // [B][6] inverse pupil moment matrix (symmetric, upper triangle)
  GradLoss* loss;      // [B]
  int* flag;           // [B] bit 1: a frame could not be normalised; bit 2: zero loss
  double* part;        // [B][g_records(N)][6] FP64 reduction records
};
// one frame's inputs, intermediates and outputs; arrays are B images of N*N
// back to back
struct GradFwd {
  const float2* const* y;  // device table of the B streams' frames
  const float* phi_in;
  const float* r_in;
  float2 *yh, *v, *b, *mu, *z, *work;
  float *phip, *s, *kap, *tth;
  float* rs[5];  // r before colour pass c (rs[0] = Eq. (3) value), rs[4] = output
  float* ps[5];  // phi after colour pass c-1 (ps[4] = output); pass 0 reads phip
  const float2* tw;
};
// adjoint work arrays (B images of N*N); gs2, gsr, gbeta accumulate per pixel
struct GradBwd {
  float *rbar, *pbar, *pb2, *em, *kbar, *tbar, *sbar, *Abar, *Bbar;
  float2 *zbar, *vbar;
  float *gs2, *gsr, *gbeta;
};
hipError_t g_launch_forward(const GradFwd& a, const GradDev& d, int N, int B, hipStream_t st);
hipError_t g_launch_loss(const float* phi, const float* ptrue, const GradDev& d, int N, int B, float* pbar,
                         hipStream_t st);
hipError_t g_launch_backward(const GradFwd& a, const GradBwd& g, const GradDev& d, int N, int B, hipStream_t st);
hipError_t g_launch_totals(const GradBwd& g, const GradDev& d, int N, int B, hipStream_t st);
int g_records(int N);  // reduction records per stream

}  // namespace ddh
