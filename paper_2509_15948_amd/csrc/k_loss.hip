// Fused multi-resolution STFT loss (Sec. 5.1), evaluated in FP64 from the
// FP32 mix (a log-magnitude loss turns FP32 transform noise in quiet Mel
// cells into a bias).  For every resolution N (hop
// N/4, periodic Hann, frames fully inside [skip, L)) the packed stereo frame
// l + i r is transformed once in LDS; the left/right spectra are separated
// with the mirrored bins, mid = l + r and side = l - r are formed from the
// spectra, magnitudes are A-weighted per bin and projected on the Mel
// triangles (banded, no dense product), and the log-l1 and
// spectral-convergence partial sums are reduced in a fixed order.  Target
// Mel spectra are computed once at setup and stay resident.
// The adjoint recomputes each frame, forms dL/dX per bin, packs the two
// channel gradients into one Hermitian-split spectrum, inverse transforms it
// and windows it; a gather kernel overlap-adds the four frames per sample.
#include <algorithm>
#include <cstring>
#include <vector>

#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {

// threads per block of the frame kernels (up to 137 KB of LDS per block)
constexpr int LOSS_NT = 512;


constexpr double LOG_EPS = 1e-7;

// Frames per workgroup of the backward: 1024 complex FP64 points per batch
// (16 KB of LDS, beside the magnitudes and band gradients it keeps), one
// frame from 1024 points up.
template <int N>
constexpr int loss_fpb() { return N >= 1024 ? 1 : 1024 / N; }
// The forward holds 4096 / N frames per workgroup (64 KB of LDS, two
// workgroups per CU): each radix-8 pass then has 512 butterflies, one per
// thread (one 1024- or 2048-point frame left three quarters or half of the
// lanes idle in every pass; 64 pruning trials 10.25 -> 9.24 ms).
template <int N>
constexpr int loss_fpb_fwd() { return N >= 4096 ? 1 : 4096 / N; }

// frames sit in LDS with one spare slot per 8 points: point t of frame fl at
// buf[fl * loss_bs<N>() + lx(t)].  With 16-byte points the first radix-8
// passes otherwise put the 8 lanes of each 128-byte LDS cycle on one bank
// group; with the spare slots they fall on disjoint ones.
constexpr int LOSS_PAD = 3;
template <int N>
constexpr int loss_bs() { return lds_len<N, LOSS_PAD>(); }
__device__ __forceinline__ int lx(int i) { return lds_ix<LOSS_PAD>(i); }

struct LossTabs {
  const double* win;    // [N]
  const double* aw;     // [N/2+1]
  const int* band_lo;   // [nm]
  const int* band_cnt;  // [nm]
  const int* band_off;  // [nm]
  const double* band_w; // [sum cnt]
  const int* bin_band;  // [N/2+1][2], -1 = none
  const double* bin_w;  // [N/2+1][2]
};

struct LossArgs {
  const float* y;       // [2][L] signal
  int64_t L;
  int skip, hop, F, nm;
  double* tgt;          // [F][4][nm]
  double* part;         // [blocks][8]
  float* scratch;       // [F][N][2] (backward)
  const double* stats;  // [4][4] of this resolution (backward)
  LossTabs tb;
  const double2* tw;
};

// The frame kernels run LOSS_NT threads.  Their loops over frame points and
// over (frame, combo, band) items fetch what a batch of iterations reads
// from global memory (signal, window, band tables, target features) before
// the first is used; the arithmetic and its order are those of one
// iteration after another.
template <int N, int FPB>
__device__ __forceinline__ void load_frames(double2* buf, const LossArgs& a, int f0) {
  static_assert(FPB * N % LOSS_NT == 0, "whole passes");
  constexpr int PER = FPB * N / LOSS_NT;
  constexpr int B = PER < 8 ? PER : 8;
  static_assert(PER % B == 0, "whole batches");
#pragma unroll 1
  for (int k0 = 0; k0 < PER; k0 += B) {
    float yl[B], yr[B];
    double wv[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int idx = threadIdx.x + (k0 + k) * LOSS_NT;
      const int fl = idx / N, t = idx % N;
      const int f = f0 + fl;
      const int64_t s = (int64_t)a.skip + (int64_t)f * a.hop + t;
      const bool ok = f < a.F;
      yl[k] = ok ? a.y[s] : 0.f;
      yr[k] = ok ? a.y[a.L + s] : 0.f;
      wv[k] = ok ? a.tb.win[t] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int idx = threadIdx.x + (k0 + k) * LOSS_NT;
      const int fl = idx / N, t = idx % N;
      const double2 z = (f0 + fl < a.F) ? make_double2((double)yl[k] * wv[k], (double)yr[k] * wv[k])
                                        : make_double2(0.0, 0.0);
      buf[fl * loss_bs<N>() + lx(t)] = z;
    }
  }
}

// a (frame, combo, band) item of the Mel stage with what it reads from
// global memory: the band's first bin, weight offset and width, and the
// target feature
struct MelItem {
  int lo, off, cnt;
  double yt;
};
__device__ __forceinline__ MelItem mel_fetch(const LossArgs& a, int b, int64_t tgt_ix, bool want_tgt) {
  return MelItem{a.tb.band_lo[b], a.tb.band_off[b], a.tb.band_cnt[b], want_tgt ? a.tgt[tgt_ix] : 0.0};
}
template <int N>
__device__ __forceinline__ double mel_sum(const double* mag, const LossArgs& a, int fl, int x, const MelItem& m) {
  constexpr int NB = N / 2 + 1;
  const double* mg = mag + (fl * 4 + x) * NB + m.lo;
  const double* wt = a.tb.band_w + m.off;
  double yh = 0.0;
  for (int j = 0; j < m.cnt; ++j) yh = fma(wt[j], mg[j], yh);
  return yh;
}
constexpr int MEL_B = 4;  // Mel items per thread whose loads are in flight together

// packed spectrum z (bin k) and zm (bin N-k) -> left and right spectra
__device__ __forceinline__ void split_pair(double2 z, double2 zm, double2& xl, double2& xr) {
  xl = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
  xr = make_double2(0.5 * (z.y + zm.y), -0.5 * (z.x - zm.x));
}

template <int N>
__device__ __forceinline__ void frame_mags(const double2* buf, double* mag, const LossArgs& a) {
  constexpr int FPB = loss_fpb<N>();
  constexpr int NB = N / 2 + 1;
  for (int idx = threadIdx.x; idx < FPB * NB; idx += blockDim.x) {
    const int fl = idx / NB, k = idx % NB;
    double2 xl, xr;
    split_pair(buf[fl * loss_bs<N>() + lx(k)], buf[fl * loss_bs<N>() + lx((N - k) & (N - 1))], xl, xr);
    const double aw = a.tb.aw[k];
    double* m = mag + (fl * 4) * NB + k;
    m[0] = aw * sqrt(xl.x * xl.x + xl.y * xl.y);
    m[NB] = aw * sqrt(xr.x * xr.x + xr.y * xr.y);
    const double mr = xl.x + xr.x, mi = xl.y + xr.y, sr = xl.x - xr.x, si = xl.y - xr.y;
    m[2 * NB] = aw * sqrt(mr * mr + mi * mi);
    m[3 * NB] = aw * sqrt(sr * sr + si * si);
  }
}

// The same magnitudes written over the spectrum itself (the forward needs
// the spectrum no further): every thread first takes its bins' values into
// registers, the block synchronises, then the magnitudes go to mag, which
// aliases buf (FPB (N + 2) complex values hold FPB * 4 * (N/2 + 1) doubles).
template <int N, int FPB>
__device__ __forceinline__ void frame_mags_inplace(double2* buf, const LossArgs& a) {
  constexpr int NB = N / 2 + 1;
  constexpr int Q = (FPB * NB + LOSS_NT - 1) / LOSS_NT;
  double m4[Q][4];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int idx = threadIdx.x + q * LOSS_NT;
    if (idx >= FPB * NB) break;
    const int fl = idx / NB, k = idx % NB;
    double2 xl, xr;
    split_pair(buf[fl * loss_bs<N>() + lx(k)], buf[fl * loss_bs<N>() + lx((N - k) & (N - 1))], xl, xr);
    const double aw = a.tb.aw[k];
    m4[q][0] = aw * sqrt(xl.x * xl.x + xl.y * xl.y);
    m4[q][1] = aw * sqrt(xr.x * xr.x + xr.y * xr.y);
    const double mr = xl.x + xr.x, mi = xl.y + xr.y, sr = xl.x - xr.x, si = xl.y - xr.y;
    m4[q][2] = aw * sqrt(mr * mr + mi * mi);
    m4[q][3] = aw * sqrt(sr * sr + si * si);
  }
  __syncthreads();
  double* mag = reinterpret_cast<double*>(buf);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int idx = threadIdx.x + q * LOSS_NT;
    if (idx >= FPB * NB) break;
    const int fl = idx / NB, k = idx % NB;
    double* m = mag + (fl * 4) * NB + k;
#pragma unroll
    for (int x = 0; x < 4; ++x) m[x * NB] = m4[q][x];
  }
}

// LDS of one frame workgroup, in bytes: forward = spectra (the magnitudes
// are written over them), twiddles, block-sum slots; backward = spectra,
// twiddles, magnitudes, dL/dYh per (frame, combo, band)
template <int N>
constexpr int loss_fwd_lds() {
  return loss_fpb_fwd<N>() * loss_bs<N>() * 16 + (int)sizeof(TwTab<N, double2>) + LOSS_NT / 64 * 8;
}
template <int N>
constexpr int loss_bwd_lds() {
  return loss_fpb<N>() * loss_bs<N>() * 16 + (int)sizeof(TwTab<N, double2>) + loss_fpb<N>() * 4 * (N / 2 + 1) * 8 +
         loss_fpb<N>() * 4 * 128 * 8;
}
constexpr int cmax(int x, int y) { return x > y ? x : y; }
// the largest over the sizes 256 .. NMAX
template <int NMAX, bool FWD>
constexpr int loss_lds_max() {
  const int here = FWD ? loss_fwd_lds<NMAX>() : loss_bwd_lds<NMAX>();
  if constexpr (NMAX <= 256) return here;
  else return cmax(here, loss_lds_max<NMAX / 2, FWD>());
}

// MODE 0: target features (write tgt, partial sum Y^2); MODE 1: loss partials.
// blk: the workgroup's index within its resolution; smem: loss_fwd_lds<N>()
// bytes of LDS (16-byte aligned)
template <int N, int MODE>
__device__ __forceinline__ void loss_fwd_body(const LossArgs& a, int blk, double2* smem) {
  constexpr int FPB = loss_fpb_fwd<N>();
  double2* buf = smem;   // spectra, then the magnitudes over them
  static_assert(loss_bs<N>() >= N + 2, "the magnitudes fit over the padded frames");
  TwTab<N, double2>& tt = *reinterpret_cast<TwTab<N, double2>*>(smem + FPB * loss_bs<N>());
  double* red = reinterpret_cast<double*>(reinterpret_cast<char*>(&tt) + sizeof(TwTab<N, double2>));
  tw_fill<N>(tt, a.tw, (const double2*)nullptr);
  const double* mag = reinterpret_cast<const double*>(buf);
  const int f0 = blk * FPB;
  load_frames<N, FPB>(buf, a, f0);
  __syncthreads();
  fft_lds<N, FPB, loss_bs<N>(), LOSS_NT, -1, LOSS_PAD>(buf, tt);
  frame_mags_inplace<N, FPB>(buf, a);
  __syncthreads();
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int items = FPB * 4 * a.nm;
#pragma unroll 1
  for (int it0 = threadIdx.x; it0 < items; it0 += MEL_B * LOSS_NT) {
    MelItem mi[MEL_B];
#pragma unroll
    for (int k = 0; k < MEL_B; ++k) {
      const int it = it0 + k * LOSS_NT;
      const int fl = it / (4 * a.nm), x = (it / a.nm) % 4, b = it % a.nm;
      const int f = f0 + fl;
      if (it < items && f < a.F) mi[k] = mel_fetch(a, b, ((int64_t)f * 4 + x) * a.nm + b, MODE == 1);
    }
#pragma unroll
    for (int k = 0; k < MEL_B; ++k) {
      const int it = it0 + k * LOSS_NT;
      const int fl = it / (4 * a.nm), x = (it / a.nm) % 4, b = it % a.nm;
      const int f = f0 + fl;
      if (it >= items || f >= a.F) continue;
      const double yh = mel_sum<N>(mag, a, fl, x, mi[k]);
      if (MODE == 0) {
        a.tgt[((int64_t)f * 4 + x) * a.nm + b] = yh;
        acc[x] += yh * yh;
      } else {
        const double yt = mi[k].yt;
        acc[x] += fabs(log(yt + LOG_EPS) - log(yh + LOG_EPS));
        const double dd = yt - yh;
        acc[4 + x] += dd * dd;
      }
    }
  }
  for (int k = 0; k < 8; ++k) {
    const double s = block_sum<LOSS_NT>(acc[k], red);
    if (threadIdx.x == 0) a.part[(int64_t)blk * 8 + k] = s;
  }
}

// stats[x][0] = sum Y^2 (MODE 0), [1] = sum (Y - Yh)^2, [2] = sum|dlog| / cells
// (fixed order: strided per thread, then a tree)
// One block per resolution.  stats[x][0] = sum Y^2 (MODE 0), [1] = sum
// (Y - Yh)^2, [2] = sum |dlog| / cells.  tgt: the target's statistics of the
// resolution (setup), copied into a separate record (pruning trials) so that
// it is complete on its own.
struct ReduceArgs {
  const double* part[8];
  int nblocks[8];
  int cells[8];
  double* stats[8];
  const double* tgt[8];
  int mode;
};

__global__ __launch_bounds__(MG_BLOCK) void k_loss_reduce(ReduceArgs ra) {
  __shared__ double red[MG_BLOCK];
  const int i = blockIdx.x;
  const double* part = ra.part[i];
  double* stats = ra.stats[i];
  const double* tgt = ra.tgt[i];
  const int nblocks = ra.nblocks[i], mode = ra.mode;
  if (mode == 1 && tgt != stats && threadIdx.x < 4) stats[threadIdx.x * 4 + 0] = tgt[threadIdx.x * 4 + 0];
  // one pass over the partial rows (each thread: blocks t, t + MG_BLOCK, ...
  // in order, all eight sums at once), then the eight block sums
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += MG_BLOCK) {
    const double* pb = part + (int64_t)b * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] += pb[q];
  }
  for (int q = 0; q < 8; ++q) {
    const double s = block_sum<MG_BLOCK>(acc[q], red);
    if (threadIdx.x == 0) {
      const int x = q % 4;
      if (mode == 0) {
        if (q < 4) stats[x * 4 + 0] = s;
      } else if (q < 4) {
        stats[x * 4 + 2] = s / (double)ra.cells[i];
      } else {
        stats[x * 4 + 1] = s;
      }
    }
  }
}

// per frame: dL/dy for the frame's samples (windowed), to scratch [F][N][2];
// blk and smem (loss_bwd_lds<N>() bytes) as in the forward
template <int N>
__device__ __forceinline__ void loss_bwd_body(const LossArgs& a, int blk, double2* smem) {
  constexpr int FPB = loss_fpb<N>();
  constexpr int NB = N / 2 + 1;
  double2* buf = smem;
  TwTab<N, double2>& tt = *reinterpret_cast<TwTab<N, double2>*>(smem + FPB * loss_bs<N>());
  double* mag = reinterpret_cast<double*>(reinterpret_cast<char*>(&tt) + sizeof(TwTab<N, double2>));
  double* dyh = mag + FPB * 4 * NB;
  tw_fill<N>(tt, a.tw, (const double2*)nullptr);
  const int f0 = blk * FPB;
  load_frames<N, FPB>(buf, a, f0);
  __syncthreads();
  fft_lds<N, FPB, loss_bs<N>(), LOSS_NT, -1, LOSS_PAD>(buf, tt);
  frame_mags<N>(buf, mag, a);
  __syncthreads();
  // dL/dYh per (frame, combo, band); every combo carries weight 1/4 in L_a
  const double cells = (double)a.F * (double)a.nm;
  double kl[4], ksc[4];
  for (int x = 0; x < 4; ++x) {
    const double Y2 = a.stats[x * 4 + 0], D2 = a.stats[x * 4 + 1];
    const double D = sqrt(D2);
    kl[x] = 0.25 / cells;
    ksc[x] = D > 0.0 ? 0.25 / (D * (sqrt(Y2) + 1e-12)) : 0.0;
  }
  const int items = FPB * 4 * a.nm;
#pragma unroll 1
  for (int it0 = threadIdx.x; it0 < items; it0 += MEL_B * LOSS_NT) {
    MelItem mi[MEL_B];
#pragma unroll
    for (int k = 0; k < MEL_B; ++k) {
      const int it = it0 + k * LOSS_NT;
      const int fl = it / (4 * a.nm), x = (it / a.nm) % 4, b = it % a.nm;
      const int f = f0 + fl;
      if (it < items && f < a.F) mi[k] = mel_fetch(a, b, ((int64_t)f * 4 + x) * a.nm + b, true);
    }
#pragma unroll
    for (int k = 0; k < MEL_B; ++k) {
      const int it = it0 + k * LOSS_NT;
      if (it >= items) break;
      const int fl = it / (4 * a.nm), x = (it / a.nm) % 4, b = it % a.nm;
      const int f = f0 + fl;
      double g = 0.0;
      if (f < a.F) {
        const double yh = mel_sum<N>(mag, a, fl, x, mi[k]);
        const double yt = mi[k].yt;
        const double dl = log(yh + LOG_EPS) - log(yt + LOG_EPS);
        const double sg = dl > 0.0 ? 1.0 : (dl < 0.0 ? -1.0 : 0.0);
        g = kl[x] * sg / (yh + LOG_EPS) + ksc[x] * (yh - yt);
      }
      dyh[(fl * 4 + x) * 128 + b] = g;
    }
  }
  __syncthreads();
  // per bin pair (k, N-k): dL/dX for l and r, packed Hermitian spectrum
  for (int idx = threadIdx.x; idx < FPB * NB; idx += LOSS_NT) {
    const int fl = idx / NB, k = idx % NB;
    const int km = (N - k) & (N - 1);
    double2 xl, xr;
    split_pair(buf[fl * loss_bs<N>() + lx(k)], buf[fl * loss_bs<N>() + lx(km)], xl, xr);
    const double2 X[4] = {xl, xr, c_add(xl, xr), c_sub(xl, xr)};
    double2 dX[4];
    const double aw = a.tb.aw[k];
    for (int x = 0; x < 4; ++x) {
      double dm = 0.0;
      for (int s = 0; s < 2; ++s) {
        const int b = a.tb.bin_band[2 * k + s];
        if (b >= 0) dm += a.tb.bin_w[2 * k + s] * dyh[(fl * 4 + x) * 128 + b];
      }
      dm *= aw;
      const double mg = sqrt(X[x].x * X[x].x + X[x].y * X[x].y);
      dX[x] = mg > 0.0 ? c_scale(X[x], dm / mg) : make_double2(0.0, 0.0);
    }
    const double2 gl = c_add(c_add(dX[0], dX[2]), dX[3]);
    const double2 gr = c_sub(c_add(dX[1], dX[2]), dX[3]);
    double2* fr = buf + fl * loss_bs<N>();
    if (k == 0 || k == N / 2) {
      fr[lx(k)] = make_double2(gl.x, gr.x);
    } else {
      // P[k] = (gl + i gr)/2, P[N-k] = (conj(gl) + i conj(gr))/2
      fr[lx(k)] = make_double2(0.5 * (gl.x - gr.y), 0.5 * (gl.y + gr.x));
      fr[lx(km)] = make_double2(0.5 * (gl.x + gr.y), 0.5 * (-gl.y + gr.x));
    }
  }
  __syncthreads();
  fft_lds<N, FPB, loss_bs<N>(), LOSS_NT, +1, LOSS_PAD>(buf, tt);
  for (int idx = threadIdx.x; idx < FPB * N; idx += LOSS_NT) {
    const int fl = idx / N, t = idx % N;
    const int f = f0 + fl;
    if (f >= a.F) continue;
    const double wv = a.tb.win[t];
    const double2 v = buf[fl * loss_bs<N>() + lx(t)];
    float* o = a.scratch + ((int64_t)f * N + t) * 2;
    o[0] = (float)(v.x * wv);
    o[1] = (float)(v.y * wv);
  }
}

struct GatherRes {
  const float* scratch;
  int N, hop, F;
};

struct GatherArgs {
  GatherRes r[8];
  int nres;
  int skip;
  int64_t L;
  float* out;  // [2][L]
};

__global__ __launch_bounds__(MG_BLOCK) void k_loss_gather(GatherArgs a) {
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < a.L; n += (int64_t)gridDim.x * blockDim.x) {
    float sl = 0.f, sr = 0.f;
    const int64_t m = n - a.skip;
    if (m >= 0) {
      for (int i = 0; i < a.nres; ++i) {
        const GatherRes& R = a.r[i];
        int64_t fh = m / R.hop;
        for (int64_t f = fh - 3; f <= fh; ++f) {
          if (f < 0 || f >= R.F) continue;
          const int64_t t = m - f * R.hop;
          if (t < 0 || t >= R.N) continue;
          const float* s = R.scratch + (f * R.N + t) * 2;
          sl += s[0];
          sr += s[1];
        }
      }
    }
    a.out[n] = sl;
    a.out[a.L + n] = sr;
  }
}

// Several resolutions in one launch: workgroup b belongs to resolution i
// when first[i] <= b < first[i + 1] and runs the frame body of that size.
// One grid for all of them needs no second stream (no fork and join on the
// caller's queue) and lets the short transforms fill the long ones' tail.
struct LossMulti {
  LossArgs a[8];
  int first[9];
  int nfft[8];
  int nres;
};

__device__ __forceinline__ int multi_res(const LossMulti& m, int& blk) {
  int i = 0;
  while (i + 1 < m.nres && (int)blockIdx.x >= m.first[i + 1]) ++i;
  blk = (int)blockIdx.x - m.first[i];
  return i;
}

template <int NMAX, int MODE>
__global__ __launch_bounds__(LOSS_NT) void k_loss_fwd_multi(LossMulti m) {
  __shared__ double2 smem[loss_lds_max<NMAX, true>() / 16 + 1];
  int blk;
  const int i = multi_res(m, blk);
  switch (m.nfft[i]) {
#define MG_FB(NN)                                                \
  case NN:                                                       \
    if constexpr (NN <= NMAX) loss_fwd_body<NN, MODE>(m.a[i], blk, smem); \
    break;
    MG_FB(256) MG_FB(512) MG_FB(1024) MG_FB(2048) MG_FB(4096)
#undef MG_FB
  }
}

template <int NMAX>
__global__ __launch_bounds__(LOSS_NT) void k_loss_bwd_multi(LossMulti m) {
  __shared__ double2 smem[loss_lds_max<NMAX, false>() / 16 + 1];
  int blk;
  const int i = multi_res(m, blk);
  switch (m.nfft[i]) {
#define MG_BB(NN)                                                \
  case NN:                                                       \
    if constexpr (NN <= NMAX) loss_bwd_body<NN>(m.a[i], blk, smem); \
    break;
    MG_BB(256) MG_BB(512) MG_BB(1024) MG_BB(2048) MG_BB(4096)
#undef MG_BB
  }
}

// ---------------------------------------------------------------- host
static LossTabs tabs_of(const Ctx& c, const LossRes& r) {
  const mg_graph* g = c.g;
  LossTabs t;
  const char* b = c.base + r.tab_off;
  const int N = r.nfft, NB = N / 2 + 1, nm = g->cfg.n_mels;
  size_t o = 0;
  t.win = (const double*)(b + o);
  o += N * 8;
  t.aw = (const double*)(b + o);
  o += NB * 8;
  t.band_lo = (const int*)(b + o);
  o += nm * 4;
  t.band_cnt = (const int*)(b + o);
  o += nm * 4;
  t.band_off = (const int*)(b + o);
  o += nm * 4;
  t.bin_band = (const int*)(b + o);
  o += 2 * NB * 4;
  o = (o + 7) / 8 * 8;
  t.bin_w = (const double*)(b + o);
  o += 2 * NB * 8;
  t.band_w = (const double*)(b + o);
  return t;
}

// host: build the table blob of one resolution (layout of tabs_of)
size_t loss_table_bytes(int N, int nm, int fs, std::vector<char>* blob) {
  const int NB = N / 2 + 1;
  const double pi = 3.14159265358979323846;
  auto hz2mel = [](double f) { return 2595.0 * log10(1.0 + f / 700.0); };
  auto mel2hz = [](double m) { return 700.0 * (pow(10.0, m / 2595.0) - 1.0); };
  std::vector<double> pts(nm + 2);
  const double mmax = hz2mel(fs / 2.0);
  for (int i = 0; i < nm + 2; ++i) pts[i] = mel2hz(mmax * i / (nm + 1));
  std::vector<int> lo(nm), cnt(nm), off(nm), bb(2 * NB, -1);
  std::vector<double> bw, binw(2 * NB, 0.0);
  for (int b = 0; b < nm; ++b) {
    int first = -1, last = -1;
    std::vector<float> ws;
    for (int k = 0; k < NB; ++k) {
      const double f = (double)k * fs / N;
      const double up = (f - pts[b]) / (pts[b + 1] - pts[b]);
      const double dn = (pts[b + 2] - f) / (pts[b + 2] - pts[b + 1]);
      const double w = std::max(0.0, std::min(up, dn));
      if (w > 0.0) {
        if (first < 0) first = k;
        last = k;
      }
    }
    if (first < 0) {
      first = 0;
      last = -1;
    }
    lo[b] = first;
    cnt[b] = last - first + 1;
    off[b] = (int)bw.size();
    for (int k = first; k <= last; ++k) {
      const double f = (double)k * fs / N;
      const double up = (f - pts[b]) / (pts[b + 1] - pts[b]);
      const double dn = (pts[b + 2] - f) / (pts[b + 2] - pts[b + 1]);
      const double w = std::max(0.0, std::min(up, dn));
      bw.push_back(w);
      if (w > 0.0) {
        const int s = (bb[2 * k] < 0) ? 0 : 1;
        bb[2 * k + s] = b;
        binw[2 * k + s] = w;
      }
    }
  }
  auto ra = [](double x) {
    const double x2 = x * x;
    return (12194.0 * 12194.0 * x2 * x2) /
           ((x2 + 20.6 * 20.6) * sqrt((x2 + 107.7 * 107.7) * (x2 + 737.9 * 737.9)) * (x2 + 12194.0 * 12194.0));
  };
  const double r1k = ra(1000.0);
  size_t o_int = (size_t)N * 8 + NB * 8 + 3 * nm * 4 + 2 * NB * 4;
  size_t o_binw = (o_int + 7) / 8 * 8;
  size_t bytes = o_binw + 2 * NB * 8 + bw.size() * 8;
  if (blob) {
    blob->assign(bytes, 0);
    char* p = blob->data();
    size_t o = 0;
    for (int t = 0; t < N; ++t) ((double*)(p + o))[t] = 0.5 - 0.5 * cos(2.0 * pi * t / N);
    o += N * 8;
    for (int k = 0; k < NB; ++k) ((double*)(p + o))[k] = ra((double)k * fs / N) / r1k;
    o += NB * 8;
    memcpy(p + o, lo.data(), nm * 4);
    o += nm * 4;
    memcpy(p + o, cnt.data(), nm * 4);
    o += nm * 4;
    memcpy(p + o, off.data(), nm * 4);
    o += nm * 4;
    memcpy(p + o, bb.data(), 2 * NB * 4);
    o = o_binw;
    memcpy(p + o, binw.data(), 2 * NB * 8);
    o += 2 * NB * 8;
    if (!bw.empty()) memcpy(p + o, bw.data(), bw.size() * 8);
  }
  return bytes;
}

static LossArgs loss_args(const Ctx& c, int i, const float* y) {
  const mg_graph* g = c.g;
  const LossRes& r = g->lres[i];
  LossArgs a;
  a.y = y;
  a.L = c.L;
  a.skip = g->cfg.loss_skip;
  a.hop = r.hop;
  a.F = r.frames;
  a.nm = g->cfg.n_mels;
  a.tgt = (double*)(c.base + r.tgt_off);
  a.part = (double*)(c.base + r.part_off);
  a.scratch = (float*)(c.base + g->ws.ls_part) + 0;  // set per resolution below
  a.stats = (const double*)(c.base + g->ws.ls_stats) + i * 16;
  a.tb = tabs_of(c, r);
  a.tw = wsp<double2>(c, g->ws.twd);
  return a;
}

// The resolutions up to 2048 points share one launch (the 4096-point body
// needs more registers and LDS, which would halve the short ones' occupancy);
// larger ones get a launch of their own on the side stream, forked from and
// joined back to the caller's stream, so that the two groups overlap.
constexpr int LOSS_SPLIT_N = 2048;
constexpr int EV_LOSS_FORK = 62, EV_LOSS_JOIN = 63;

// when the resolutions form two groups: the context of the second one (the
// side stream after a fork) in cs; false when everything stays on c's stream
static bool loss_fork(const Ctx& c, Ctx& cs) {
  const mg_graph* g = c.g;
  bool lo = false, hi = false;
  for (const LossRes& r : g->lres) (r.nfft <= LOSS_SPLIT_N ? lo : hi) = true;
  cs = c;
  if (!lo || !hi || !g->side || g->sev.size() < 64) return false;
  cs.st = g->side;
  hipEventRecord(g->sev[EV_LOSS_FORK], c.st);
  hipStreamWaitEvent(g->side, g->sev[EV_LOSS_FORK], 0);
  return true;
}

static void loss_join(const Ctx& c) {
  const mg_graph* g = c.g;
  hipEventRecord(g->sev[EV_LOSS_JOIN], g->side);
  hipStreamWaitEvent(c.st, g->sev[EV_LOSS_JOIN], 0);
}

template <int NMAX, int MODE>
static void fwd_multi(const Ctx& c, const LossMulti& m) {
  MG_LAUNCH(c, (k_loss_fwd_multi<NMAX, MODE>), dim3(m.first[m.nres]), dim3(LOSS_NT), 0, c.st, m);
}
template <int NMAX>
static void bwd_multi(const Ctx& c, const LossMulti& m) {
  MG_LAUNCH(c, k_loss_bwd_multi<NMAX>, dim3(m.first[m.nres]), dim3(LOSS_NT), 0, c.st, m);
}

#define MG_LOSS_SWITCH(N_, CALL)   \
  switch (N_) {                    \
    case 256: CALL(256); break;    \
    case 512: CALL(512); break;    \
    case 1024: CALL(1024); break;  \
    case 2048: CALL(2048); break;  \
    case 4096: CALL(4096); break;  \
  }

// launch groups: every resolution in [lo, hi] points, with its args from
// args_of(i); fills the group's grid layout and returns its largest size
template <typename F>
static int loss_group(const mg_graph* g, int lo, int hi, bool fwd, LossMulti& m, F args_of) {
  m.nres = 0;
  m.first[0] = 0;
  int nmax = 0;
  for (size_t i = 0; i < g->lres.size(); ++i) {
    const LossRes& r = g->lres[i];
    if (r.nfft < lo || r.nfft > hi) continue;
    const int FPB = fwd ? loss_frames_per_block_fwd(r.nfft) : loss_frames_per_block(r.nfft);
    const int k = m.nres++;
    m.a[k] = args_of((int)i);
    m.nfft[k] = r.nfft;
    m.first[k + 1] = m.first[k] + (r.frames + FPB - 1) / FPB;
    nmax = std::max(nmax, r.nfft);
  }
  return nmax;
}

static void run_loss_fwd(const Ctx& c, const float* y, int mode, double* stats_out) {
  const mg_graph* g = c.g;
  double* stats = stats_out ? stats_out : wsp<double>(c, g->ws.ls_stats);
  ReduceArgs ra;
  ra.mode = mode;
  for (size_t i = 0; i < g->lres.size(); ++i) {
    const LossRes& r = g->lres[i];
    const int FPB = loss_frames_per_block_fwd(r.nfft);
    ra.part[i] = (double*)(c.base + r.part_off);
    ra.nblocks[i] = (r.frames + FPB - 1) / FPB;
    ra.cells[i] = r.frames * g->cfg.n_mels;
    ra.stats[i] = stats + i * 16;
    ra.tgt[i] = wsp<double>(c, g->ws.ls_stats) + i * 16;
  }
  const int groups[2][2] = {{0, LOSS_SPLIT_N}, {LOSS_SPLIT_N + 1, 1 << 30}};
  Ctx cs;
  const bool forked = loss_fork(c, cs);
  for (int k = 0; k < 2; ++k) {
    const Ctx& cc = (k == 1) ? cs : c;
    LossMulti m;
    const int nmax = loss_group(g, groups[k][0], groups[k][1], true, m, [&](int i) { return loss_args(c, i, y); });
    if (m.nres == 0) continue;
#define MG_F0(NN) fwd_multi<NN, 0>(cc, m)
#define MG_F1(NN) fwd_multi<NN, 1>(cc, m)
    if (mode == 0) {
      MG_LOSS_SWITCH(nmax, MG_F0)
    } else {
      MG_LOSS_SWITCH(nmax, MG_F1)
    }
#undef MG_F0
#undef MG_F1
  }
  if (forked) loss_join(c);
  MG_LAUNCH(c, k_loss_reduce, dim3((unsigned)g->lres.size()), dim3(MG_BLOCK), 0, c.st, ra);
}

void loss_setup(const Ctx& c, const float* target) {
  const mg_graph* g = c.g;
  for (size_t i = 0; i < g->lres.size(); ++i) {
    std::vector<char> blob;
    loss_table_bytes(g->lres[i].nfft, g->cfg.n_mels, g->cfg.sample_rate, &blob);
    hipMemcpyAsync(c.base + g->lres[i].tab_off, blob.data(), blob.size(), hipMemcpyHostToDevice, c.st);
    hipStreamSynchronize(c.st);
  }
  loss_target(c, target);
}

void loss_target(const Ctx& c, const float* target) {
  launch_zero(c.base + c.g->ws.ls_stats, 8 * sizeof(double) * 16, c.st);
  run_loss_fwd(c, target, 0, nullptr);
}

void loss_forward(const Ctx& c, const float* yhat, double* stats) {
  ProfScope ps(c, "loss", 8.0 * c.L);
  run_loss_fwd(c, yhat, 1, stats);
}

void loss_backward(const Ctx& c, const float* yhat, float* dyhat) {
  const mg_graph* g = c.g;
  ProfScope ps(c, "loss", 16.0 * c.L);
  GatherArgs ga;
  ga.nres = (int)g->lres.size();
  ga.skip = g->cfg.loss_skip;
  ga.L = c.L;
  ga.out = dyhat;
  // per-resolution dL/dy frames, one after another in the scratch area
  std::vector<float*> scratch(g->lres.size());
  size_t off = g->ws.ls_part;
  for (size_t i = 0; i < g->lres.size(); ++i) {
    const LossRes& r = g->lres[i];
    scratch[i] = (float*)(c.base + off);
    ga.r[i].scratch = scratch[i];
    ga.r[i].N = r.nfft;
    ga.r[i].hop = r.hop;
    ga.r[i].F = r.frames;
    off += (((size_t)r.frames * r.nfft * 2 * 4) + 255) / 256 * 256;
  }
  const int groups[2][2] = {{0, LOSS_SPLIT_N}, {LOSS_SPLIT_N + 1, 1 << 30}};
  Ctx cs;
  const bool forked = loss_fork(c, cs);
  for (int k = 0; k < 2; ++k) {
    const Ctx& cc = (k == 1) ? cs : c;
    LossMulti m;
    const int nmax = loss_group(g, groups[k][0], groups[k][1], false, m, [&](int i) {
      LossArgs a = loss_args(c, i, yhat);
      a.scratch = scratch[i];
      return a;
    });
    if (m.nres == 0) continue;
#define MG_B(NN) bwd_multi<NN>(cc, m)
    MG_LOSS_SWITCH(nmax, MG_B)
#undef MG_B
  }
  if (forked) loss_join(c);
  int64_t blocks = (c.L + MG_BLOCK - 1) / MG_BLOCK;
  if (blocks > 2048) blocks = 2048;
  MG_LAUNCH(c, k_loss_gather, dim3((unsigned)blocks), dim3(MG_BLOCK), 0, c.st, ga);
}

}  // namespace mg
