// FIR synthesis of the FIR processors and the adjoints back to their raw
// parameters.
//  * equalizer (Sec. 3.3): h[n] = cos^2(pi n/N) (H0 + 2 sum_k H_k cos(2 pi k n/N)) / N,
//    H_k = exp(p_k), n = -(N-1)/2..(N-1)/2; angles reduced exactly as (k n mod N)
//  * multitap delay (Sec. 3.7): per channel and tap an integer delay from the
//    angle of z and a zero-phase FIR c_m built like the equalizer; the z
//    gradient is the straight-through surrogate with the normalised update rule
//  * reverb (Sec. 3.4): masked STFT of fixed noise -> least-squares ISTFT ->
//    mid/side to left/right; mask exp(H0 + g0 + m d) with the per-frame decay
//    d = -softplus(H_delta + beta)
// These are small next to the convolutions; they use FP64 accumulation.
#include <cstring>
#include <vector>

#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {

// ---------------------------------------------------------------- equalizer
// Both directions are cosine sums of about a thousand terms per output.  Each
// output is split over FIR_SPLIT threads of one block; a thread
// walks its part of the sum with an FP64 rotation e^{i theta} started from an
// exactly reduced angle, so no table is read and the drift stays at the FP64
// rounding level.  The parts are added in a fixed order.
constexpr int FIR_SPLIT = 16;
constexpr int FIR_PER_BLOCK = MG_BLOCK / FIR_SPLIT;   // outputs per block

// exp(i 2 pi (a mod N) / N) in FP64
__device__ __forceinline__ double2 unit_root(int64_t a, int N) {
  const int64_t r = ((a % N) + N) % N;
  double s, c;
  sincospi(2.0 * (double)r / (double)N, &s, &c);
  return make_double2(c, s);
}

// h[n] = v[n] (H0 + 2 sum_{k=1}^{K-1} H_k cos(2 pi k n / N)) / N, v = cos^2(pi n / N);
// grid (ceil(N / FIR_PER_BLOCK), nodes)
__global__ __launch_bounds__(MG_BLOCK) void k_eq_synth(const NodeDesc* __restrict__ desc,
                                                        const float* __restrict__ theta, int N,
                                                        float* __restrict__ h_out) {
  __shared__ double H[4096];
  __shared__ double part[FIR_SPLIT][FIR_PER_BLOCK];
  const NodeDesc d = desc[blockIdx.y];
  const int K = (N + 1) / 2;
  const float* p = theta + d.theta_off;
  for (int k = threadIdx.x; k < K; k += MG_BLOCK) H[k] = exp((double)p[k]);
  __syncthreads();
  const int lane = threadIdx.x % FIR_PER_BLOCK, c = threadIdx.x / FIR_PER_BLOCK;
  const int i = blockIdx.x * FIR_PER_BLOCK + lane;
  const int half = (N - 1) / 2;
  const int n = i - half;
  const int Q = (K - 1 + FIR_SPLIT - 1) / FIR_SPLIT;
  const int k0 = 1 + c * Q, k1 = min(K, k0 + Q);
  double acc = 0.0;
  if (i < N && k0 < k1) {
    double2 w = unit_root((int64_t)k0 * n, N);
    const double2 step = unit_root(n, N);
    for (int k = k0; k < k1; ++k) {
      acc = fma(H[k], w.x, acc);
      w = c_mul(w, step);
    }
  }
  part[c][lane] = acc;
  __syncthreads();
  if (c != 0 || i >= N) return;
  double s = 0.0;
  for (int q = 0; q < FIR_SPLIT; ++q) s += part[q][lane];
  const double h0 = (H[0] + 2.0 * s) / (double)N;
  const double2 r = unit_root(n, N);
  const double v = 0.5 * (1.0 + r.x);  // cos^2(pi n / N)
  h_out[(int64_t)d.aux * N + i] = (float)(v * h0);
}

// dL/dp_k = H_k (c_k / N) sum_n v[n] dh[n] cos(2 pi k n / N), c_0 = 1, c_k = 2;
// grid (ceil(K / FIR_PER_BLOCK), nodes)
__global__ __launch_bounds__(MG_BLOCK) void k_eq_adjoint(const NodeDesc* __restrict__ desc,
                                                          const float* __restrict__ theta, int N,
                                                          const float* __restrict__ dh,
                                                          float* __restrict__ grad_theta) {
  __shared__ double gv[4096];
  __shared__ double part[FIR_SPLIT][FIR_PER_BLOCK];
  const NodeDesc d = desc[blockIdx.y];
  const int K = (N + 1) / 2;
  const int half = (N - 1) / 2;
  for (int i = threadIdx.x; i < N; i += MG_BLOCK) {
    const double2 r = unit_root(i - half, N);
    gv[i] = 0.5 * (1.0 + r.x) * (double)dh[(int64_t)d.aux * N + i];
  }
  __syncthreads();
  const int lane = threadIdx.x % FIR_PER_BLOCK, c = threadIdx.x / FIR_PER_BLOCK;
  const int k = blockIdx.x * FIR_PER_BLOCK + lane;
  const int Q = (N + FIR_SPLIT - 1) / FIR_SPLIT;
  const int i0 = c * Q, i1 = min(N, i0 + Q);
  double acc = 0.0;
  if (k < K && i0 < i1) {
    double2 w = unit_root((int64_t)k * (i0 - half), N);
    const double2 step = unit_root(k, N);
    for (int i = i0; i < i1; ++i) {
      acc = fma(gv[i], w.x, acc);
      w = c_mul(w, step);
    }
  }
  part[c][lane] = acc;
  __syncthreads();
  if (c != 0 || k >= K) return;
  double s = 0.0;
  for (int q = 0; q < FIR_SPLIT; ++q) s += part[q][lane];
  const double ck = (k == 0) ? 1.0 : 2.0;
  const float* p = theta + d.theta_off;
  grad_theta[d.theta_off + k] = (float)(exp((double)p[k]) * ck / (double)N * s);
}

// ---------------------------------------------------------------- multitap delay
// Per node table: [2][M] integer delays (stored as float) then [2][M][taps]
// coefficients.  grid (nodes), block 256.
__global__ __launch_bounds__(MG_BLOCK) void k_delay_synth(const NodeDesc* __restrict__ desc,
                                                           const float* __restrict__ theta,
                                                           const float* __restrict__ cosT, int M, int D, int taps,
                                                           float* __restrict__ tab) {
  const NodeDesc d = desc[blockIdx.x];
  const int Kc = (taps + 1) / 2;
  const int half = (taps - 1) / 2;
  const float* p = theta + d.theta_off;
  float* t = tab + (int64_t)d.aux * 2 * M * (1 + taps);
  const int stride = 2 + Kc;
  for (int cm = threadIdx.x; cm < 2 * M; cm += MG_BLOCK) {
    const int m = cm % M;
    const double zr = p[cm * stride], zi = p[cm * stride + 1];
    const double phi = atan2(zi, zr);
    long long r = (long long)floor(-phi * (double)D / (2.0 * 3.14159265358979323846) + 0.5);
    r %= D;
    if (r < 0) r += D;
    t[cm] = (float)((long long)m * D + r);
  }
  for (int e = threadIdx.x; e < 2 * M * taps; e += MG_BLOCK) {
    const int cm = e / taps, i = e % taps;
    const float* lm = p + cm * stride + 2;
    const int n = i - half;
    const int nn = ((n % taps) + taps) % taps;
    double acc = 0.0;
    int idx = 0;
    for (int k = 1; k < Kc; ++k) {
      idx += nn;
      if (idx >= taps) idx -= taps;
      acc += exp((double)lm[k]) * (double)cosT[idx];
    }
    const double h0 = (exp((double)lm[0]) + 2.0 * acc) / (double)taps;
    const double v = 0.5 * (1.0 + (double)cosT[nn]);
    t[2 * M + e] = (float)(v * h0);
  }
}

// Dense compact delay FIR h[c][x] for lags x - half (x < dl_len): the sum over
// taps m of c_m[x - d_m] where that index is inside the tap's FIR; the taps
// are added in order m = 0..M-1.  grid (ceil(dl_len / 256), 2, nodes)
__global__ __launch_bounds__(MG_BLOCK) void k_delay_compact(const NodeDesc* __restrict__ desc,
                                                             const float* __restrict__ tab, int M, int taps,
                                                             int64_t dl_len, float* __restrict__ h) {
  const NodeDesc d = desc[blockIdx.z];
  const int c = blockIdx.y;
  const int64_t x = (int64_t)blockIdx.x * MG_BLOCK + threadIdx.x;
  if (x >= dl_len) return;
  const float* t = tab + (int64_t)d.aux * 2 * M * (1 + taps);
  float a = 0.0f;
  for (int m = 0; m < M; ++m) {
    const int64_t k = x - (int64_t)t[c * M + m];
    if (k >= 0 && k < taps) a += t[2 * M + (c * M + m) * taps + k];
  }
  h[((int64_t)d.aux * 2 + c) * dl_len + x] = a;
}

// P(a) = sum_{k=1}^{D-1} k a^{k-1}, closed form away from a = 1, Horner near it
__device__ inline void poly_P(double ar, double ai, int D, double zDr, double zDi, double zD1r, double zD1i,
                              double wr, double wi, double& pr, double& pi) {
  // a = z w^q; a^D = z^D; a^{D-1} = z^{D-1} w^{-q}
  const double br = 1.0 - ar, bi = -ai;
  const double bb = br * br + bi * bi;
  if (bb > 1e-12) {
    // numerator 1 - D a^{D-1} + (D-1) a^D
    const double a1r = zD1r * wr + zD1i * wi, a1i = zD1i * wr - zD1r * wi;  // z^{D-1} conj(w^q)
    const double nr = 1.0 - D * a1r + (D - 1) * zDr;
    const double ni = -D * a1i + (D - 1) * zDi;
    // divide by (1 - a)^2
    const double sr = br * br - bi * bi, si = 2.0 * br * bi;
    const double ss = sr * sr + si * si;
    pr = (nr * sr + ni * si) / ss;
    pi = (ni * sr - nr * si) / ss;
  } else {
    double accr = D - 1, acci = 0.0;
    for (int k = D - 2; k >= 1; --k) {
      const double tr = accr * ar - acci * ai + k;
      const double ti = accr * ai + acci * ar;
      accr = tr;
      acci = ti;
    }
    pr = accr;
    pi = acci;
  }
}

// One workgroup per (node, channel, tap, chunk of the delay range): the
// straight-through z gradient as partial sums over its chunk of q,
//   f'(z) = (1/D) sum_q Gc[q] w^q P(z w^q),  Gc[q] = sum_j c_m[j] dh[m D + q + j],
// written to zpart; chunk 0 also forms dL/dc_m (-> log-magnitudes).
// k_delay_zrule then adds the chunks in order and applies the update rule
//   g = conj(f'(z)),  update = g/|g| + gamma (|z| - 1) z/|z|.
constexpr int DL_CHUNKS = 8;

__global__ __launch_bounds__(MG_BLOCK) void k_delay_adjoint(const NodeDesc* __restrict__ desc,
                                                             const float* __restrict__ theta,
                                                             const float* __restrict__ tab,
                                                             const float* __restrict__ cosT, int M, int D,
                                                             int taps, int64_t dl_len,
                                                             const float* __restrict__ dh,
                                                             float* __restrict__ grad_theta,
                                                             double2* __restrict__ zpart) {
  __shared__ double red_r[MG_BLOCK];
  __shared__ double red_i[MG_BLOCK];
  __shared__ float cm[256];
  __shared__ float dc[256];
  const int j = blockIdx.z;
  const int chunk = blockIdx.y;
  const NodeDesc d = desc[j];
  const int cmi = blockIdx.x;  // c * M + m
  const int c = cmi / M, m = cmi % M;
  const int Kc = (taps + 1) / 2;
  const int half = (taps - 1) / 2;
  const int stride = 2 + Kc;
  const float* t = tab + (int64_t)d.aux * 2 * M * (1 + taps);
  const int dm = (int)t[cmi];
  const float* dhc = dh + (int64_t)d.aux * 2 * dl_len + (int64_t)c * dl_len;
  for (int i = threadIdx.x; i < taps; i += MG_BLOCK) {
    cm[i] = t[2 * M + cmi * taps + i];
    dc[i] = dhc[dm + i];  // compact index of lag dm + (i - half) is dm + i
  }
  __syncthreads();
  const float* p = theta + d.theta_off + (int64_t)cmi * stride;
  float* gp = grad_theta + d.theta_off + (int64_t)cmi * stride;
  if (chunk == 0) {
    // log-magnitudes of c_m
    for (int k = threadIdx.x; k < Kc; k += MG_BLOCK) {
      double acc = 0.0;
      for (int i = 0; i < taps; ++i) {
        const int n = i - half;
        const int nn = ((n % taps) + taps) % taps;
        const int idx = (int)(((int64_t)k * nn) % taps);
        acc += 0.5 * (1.0 + (double)cosT[nn]) * (double)dc[i] * (double)cosT[idx];
      }
      const double ck = (k == 0) ? 1.0 : 2.0;
      gp[2 + k] = (float)(exp((double)p[2 + k]) * ck / (double)taps * acc);
    }
  }
  // z surrogate gradient over this chunk of q
  const double zr = p[0], zi = p[1];
  const double lz = 0.5 * log(zr * zr + zi * zi), az = atan2(zi, zr);
  const double mD = exp(D * lz), mD1 = exp((D - 1) * lz);
  const double zDr = mD * cos(D * az), zDi = mD * sin(D * az);
  const double zD1r = mD1 * cos((D - 1) * az), zD1i = mD1 * sin((D - 1) * az);
  const int Qc = (D + DL_CHUNKS - 1) / DL_CHUNKS;
  const int q0 = chunk * Qc, q1 = min(D, q0 + Qc);
  double sr = 0.0, si = 0.0;
  for (int q = q0 + threadIdx.x; q < q1; q += MG_BLOCK) {
    double gc = 0.0;
    const int64_t base = (int64_t)m * D + q;
    for (int i = 0; i < taps; ++i) gc += (double)cm[i] * (double)dhc[base + i];
    double wr, wi;
    sincospi(2.0 * (double)q / (double)D, &wi, &wr);
    const double ar = zr * wr - zi * wi, ai = zr * wi + zi * wr;
    double pr, pi;
    poly_P(ar, ai, D, zDr, zDi, zD1r, zD1i, wr, wi, pr, pi);
    // w^q P
    const double tr = wr * pr - wi * pi, ti = wr * pi + wi * pr;
    sr += gc * tr;
    si += gc * ti;
  }
  red_r[threadIdx.x] = sr;
  red_i[threadIdx.x] = si;
  __syncthreads();
  for (int st = MG_BLOCK / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      red_r[threadIdx.x] += red_r[threadIdx.x + st];
      red_i[threadIdx.x] += red_i[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) zpart[((int64_t)d.aux * 2 * M + cmi) * DL_CHUNKS + chunk] = make_double2(red_r[0], red_i[0]);
}

// grid (nodes), one thread per (channel, tap)
__global__ void k_delay_zrule(const NodeDesc* __restrict__ desc, const float* __restrict__ theta, int M, int D,
                              int taps, const double2* __restrict__ zpart, float* __restrict__ grad_theta,
                              float gamma) {
  const NodeDesc d = desc[blockIdx.x];
  const int cmi = threadIdx.x;
  if (cmi >= 2 * M) return;
  const int stride = 2 + (taps + 1) / 2;
  const float* p = theta + d.theta_off + (int64_t)cmi * stride;
  float* gp = grad_theta + d.theta_off + (int64_t)cmi * stride;
  double fr = 0.0, fi = 0.0;
  for (int ch = 0; ch < DL_CHUNKS; ++ch) {
    const double2 v = zpart[((int64_t)d.aux * 2 * M + cmi) * DL_CHUNKS + ch];
    fr += v.x;
    fi += v.y;
  }
  fr /= D;
  fi /= D;
  const double zr = p[0], zi = p[1];
  const double gr = fr, gi = -fi;  // conj(f')
  const double ag = sqrt(gr * gr + gi * gi);
  const double amz = sqrt(zr * zr + zi * zi);
  double ur = 0.0, ui = 0.0;
  if (ag > 0.0) {
    ur = gr / ag;
    ui = gi / ag;
  }
  if (amz > 0.0) {
    ur += (double)gamma * (amz - 1.0) * zr / amz;
    ui += (double)gamma * (amz - 1.0) * zi / amz;
  }
  gp[0] = (float)ur;
  gp[1] = (float)ui;
}

// ---------------------------------------------------------------- reverb
// The reverb's STFT frames are 384 = 3 * 4 * 4 * 4 * 2 points: a mixed-radix
// Stockham FFT in LDS (table tw384[m] = exp(-2 pi i m / 384), FP64-rounded),
// with two real frames packed into one complex transform.
constexpr int RV_N = 384;
constexpr int RV_FPB = 16;            // frames per workgroup (8 packed transforms)
constexpr int RV_SEQ = RV_FPB / 2;

// exp(DIR 2 pi i e / 384) from the LDS copy of the table
template <int DIR>
__device__ __forceinline__ float2 rv_tw(const float2* tw, int e) {
  float2 w = tw[e];
  if (DIR > 0) w.y = -w.y;
  return w;
}

// copy the 384-entry table into LDS (the caller synchronises)
__device__ __forceinline__ void rv_tw_fill(float2* tws, const float2* __restrict__ tw) {
  for (int i = threadIdx.x; i < RV_N; i += MG_BLOCK) tws[i] = tw[i];
}

template <int R, int DIR>
__device__ __forceinline__ void rv_pass(float2* buf, const float2* tw, int Ns) {
  constexpr int Q = RV_N / R;
  constexpr int NB = RV_SEQ * Q;
  constexpr int PER = NB / MG_BLOCK;
  static_assert(NB % MG_BLOCK == 0, "even split");
  float2 v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int g = tid + q * MG_BLOCK;
    const int b = g / Q, j = g % Q;
#pragma unroll
    for (int r = 0; r < R; ++r) v[q][r] = buf[b * RV_N + j + r * Q];
  }
  __syncthreads();
  const int stride = RV_N / (Ns * R);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int g = tid + q * MG_BLOCK;
    const int b = g / Q, j = g % Q;
    const int k = j % Ns;
#pragma unroll
    for (int r = 1; r < R; ++r) v[q][r] = c_mul(v[q][r], rv_tw<DIR>(tw, r * k * stride));
    float2 y[R];
    if (R == 2) {
      y[0] = c_add(v[q][0], v[q][1]);
      y[1] = c_sub(v[q][0], v[q][1]);
    } else if (R == 3) {
      const float s3 = 0.86602540378443864676f * (DIR < 0 ? -1.0f : 1.0f);
      const float2 t1 = c_add(v[q][1], v[q][2]);
      const float2 t2 = make_float2(v[q][0].x - 0.5f * t1.x, v[q][0].y - 0.5f * t1.y);
      const float2 d = c_sub(v[q][1], v[q][2]);
      const float2 t3 = make_float2(-s3 * d.y, s3 * d.x);  // i * s3 * (a1 - a2)
      y[0] = c_add(v[q][0], t1);
      y[1] = c_add(t2, t3);
      y[2] = c_sub(t2, t3);
    } else {
      const float2 t0 = c_add(v[q][0], v[q][2]), t1 = c_sub(v[q][0], v[q][2]);
      const float2 t2 = c_add(v[q][1], v[q][3]), t3 = c_rot<DIR>(c_sub(v[q][1], v[q][3]));
      y[0] = c_add(t0, t2);
      y[1] = c_add(t1, t3);
      y[2] = c_sub(t0, t2);
      y[3] = c_sub(t1, t3);
    }
    const int idx = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[b * RV_N + idx + r * Ns] = y[r];
  }
  __syncthreads();
}

// RV_SEQ unnormalised 384-point transforms in LDS (caller syncs after filling)
template <int DIR>
__device__ __forceinline__ void rv_fft(float2* buf, const float2* tw) {
  rv_pass<3, DIR>(buf, tw, 1);
  rv_pass<4, DIR>(buf, tw, 3);
  rv_pass<4, DIR>(buf, tw, 12);
  rv_pass<4, DIR>(buf, tw, 48);
  rv_pass<2, DIR>(buf, tw, 192);
}

// noise STFT (setup): U[row][x][m][k] = sum_t w[t] noise_x[m hop - nfft/2 + t] e^{-2 pi i k t / nfft}
// grid (ceil(nf / 16), 2, rows)
__global__ __launch_bounds__(MG_BLOCK) void k_rv_noise_stft(const float* __restrict__ noise, int Lr, int nf,
                                                             const float2* __restrict__ tw,
                                                             const float* __restrict__ win,
                                                             float2* __restrict__ Uout) {
  __shared__ float2 buf[RV_SEQ * RV_N];
  __shared__ float2 tws[RV_N];
  rv_tw_fill(tws, tw);
  const int m0 = blockIdx.x * RV_FPB, x = blockIdx.y, row = blockIdx.z;
  const float* nz = noise + ((int64_t)row * 2 + x) * Lr;
  for (int i = threadIdx.x; i < RV_SEQ * RV_N; i += MG_BLOCK) {
    const int p = i / RV_N, t = i % RV_N;
    float v[2];
    for (int h = 0; h < 2; ++h) {
      const int m = m0 + 2 * p + h;
      const int64_t n = (int64_t)m * 192 - 192 + t;
      v[h] = (m < nf && n >= 0 && n < Lr) ? win[t] * nz[n] : 0.0f;
    }
    buf[i] = make_float2(v[0], v[1]);
  }
  __syncthreads();
  rv_fft<-1>(buf, tws);
  for (int i = threadIdx.x; i < RV_SEQ * 192; i += MG_BLOCK) {
    const int p = i / 192, k = i % 192;
    const float2 z = buf[p * RV_N + k], zm = buf[p * RV_N + ((RV_N - k) % RV_N)];
    const float2 a = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
    const float2 b = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
    for (int h = 0; h < 2; ++h) {
      const int m = m0 + 2 * p + h;
      if (m < nf) Uout[(((int64_t)row * 2 + x) * nf + m) * 192 + k] = h ? b : a;
    }
  }
}

// frames: fr[row][x][m][t] = w[t] (1/384) sum_{k<192} c_k Re(U M e^{+2 pi i k t/384}),
// M = exp(H0 + g0 + m d), d = -softplus(Hd + beta).  grid (ceil(nf / 16), 2, nodes)
__global__ __launch_bounds__(MG_BLOCK) void k_rv_frames(const NodeDesc* __restrict__ desc,
                                                         const float* __restrict__ theta,
                                                         const float2* __restrict__ Unz, int nf,
                                                         const float2* __restrict__ tw,
                                                         const float* __restrict__ win, float gbias, float beta,
                                                         float* __restrict__ frames) {
  __shared__ float2 buf[RV_SEQ * RV_N];
  __shared__ float2 tws[RV_N];
  rv_tw_fill(tws, tw);
  __shared__ float h0[192], dk[192];
  const int m0 = blockIdx.x * RV_FPB, x = blockIdx.y;
  const NodeDesc d = desc[blockIdx.z];
  const float* p = theta + d.theta_off + x * 384;  // [H0 (192), Hd (192)]
  for (int k = threadIdx.x; k < 192; k += MG_BLOCK) {
    h0[k] = p[k] + gbias;
    dk[k] = (float)(-log1p(exp((double)p[192 + k] + (double)beta)));
  }
  __syncthreads();
  const float2* U = Unz + ((int64_t)d.aux * 2 + x) * nf * 192;
  // Hermitian spectra of frame pairs: Z = A + i B
  for (int i = threadIdx.x; i < RV_SEQ * RV_N; i += MG_BLOCK) {
    const int pr = i / RV_N, k = i % RV_N;
    float2 s[2];
    for (int h = 0; h < 2; ++h) {
      const int m = m0 + 2 * pr + h;
      float2 v = make_float2(0.f, 0.f);
      if (m < nf && k != 192) {
        const int kk = k < 192 ? k : RV_N - k;
        const float mk = expf(h0[kk] + (float)m * dk[kk]);
        const float2 u = U[(int64_t)m * 192 + kk];
        v = make_float2(u.x * mk, u.y * mk);
        if (kk == 0) v.y = 0.f;
        if (k > 192) v.y = -v.y;
      }
      s[h] = v;
    }
    buf[i] = make_float2(s[0].x - s[1].y, s[0].y + s[1].x);
  }
  __syncthreads();
  rv_fft<+1>(buf, tws);
  for (int i = threadIdx.x; i < RV_SEQ * RV_N; i += MG_BLOCK) {
    const int pr = i / RV_N, t = i % RV_N;
    const float2 z = buf[i];
    const float wt = win[t] * (1.0f / RV_N);
    for (int h = 0; h < 2; ++h) {
      const int m = m0 + 2 * pr + h;
      if (m < nf) frames[(((int64_t)d.aux * 2 + x) * nf + m) * RV_N + t] = (h ? z.y : z.x) * wt;
    }
  }
}

// overlap-add + LS normalisation + mid/side -> left/right; grid (ceil(Lr/256), nodes)
__global__ __launch_bounds__(MG_BLOCK) void k_rv_ola(const NodeDesc* __restrict__ desc,
                                                      const float* __restrict__ frames, int nf, int Lr,
                                                      const float* __restrict__ wsum, float* __restrict__ h) {
  const NodeDesc d = desc[blockIdx.y];
  const int n = blockIdx.x * MG_BLOCK + threadIdx.x;
  if (n >= Lr) return;
  const int q = n / 192, r = n % 192;
  float hx[2];
  for (int x = 0; x < 2; ++x) {
    const float* f = frames + ((int64_t)d.aux * 2 + x) * nf * 384;
    hx[x] = (f[(int64_t)q * 384 + r + 192] + f[(int64_t)(q + 1) * 384 + r]) / wsum[r];
  }
  float* o = h + (int64_t)d.aux * 2 * Lr;
  o[n] = hx[0] + hx[1];
  o[Lr + n] = hx[0] - hx[1];
}

// adjoint per frame: dMM[k] = dM[k] M[k] with dM = Re(dH conj(U)),
// dH[k] = (c_k / 384) DFT(w dh / wsum)[k].  grid (ceil(nf / 16), 2, nodes)
__global__ __launch_bounds__(MG_BLOCK) void k_rv_adj_frames(const NodeDesc* __restrict__ desc,
                                                             const float* __restrict__ theta,
                                                             const float2* __restrict__ Unz, int nf, int Lr,
                                                             const float2* __restrict__ tw,
                                                             const float* __restrict__ win,
                                                             const float* __restrict__ wsum, float gbias,
                                                             float beta, const float* __restrict__ dh,
                                                             float* __restrict__ dMout) {
  __shared__ float2 buf[RV_SEQ * RV_N];
  __shared__ float2 tws[RV_N];
  rv_tw_fill(tws, tw);
  __shared__ float h0[192], dk[192];
  const int m0 = blockIdx.x * RV_FPB, x = blockIdx.y;
  const NodeDesc d = desc[blockIdx.z];
  const float* p = theta + d.theta_off + x * 384;
  for (int k = threadIdx.x; k < 192; k += MG_BLOCK) {
    h0[k] = p[k] + gbias;
    dk[k] = (float)(-log1p(exp((double)p[192 + k] + (double)beta)));
  }
  const float* dhn = dh + (int64_t)d.aux * 2 * Lr;
  for (int i = threadIdx.x; i < RV_SEQ * RV_N; i += MG_BLOCK) {
    const int pr = i / RV_N, t = i % RV_N;
    float v[2];
    for (int h = 0; h < 2; ++h) {
      const int m = m0 + 2 * pr + h;
      const int64_t n = (int64_t)m * 192 - 192 + t;
      float a = 0.f;
      if (m < nf && n >= 0 && n < Lr) {
        const float gx = x == 0 ? dhn[n] + dhn[Lr + n] : dhn[n] - dhn[Lr + n];
        a = win[t] * gx / wsum[t % 192];
      }
      v[h] = a;
    }
    buf[i] = make_float2(v[0], v[1]);
  }
  __syncthreads();
  rv_fft<-1>(buf, tws);
  const float2* U = Unz + ((int64_t)d.aux * 2 + x) * nf * 192;
  float* o = dMout + ((int64_t)d.aux * 2 + x) * nf * 192;
  for (int i = threadIdx.x; i < RV_SEQ * 192; i += MG_BLOCK) {
    const int pr = i / 192, k = i % 192;
    const float2 z = buf[pr * RV_N + k], zm = buf[pr * RV_N + ((RV_N - k) % RV_N)];
    const float2 Da = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
    const float2 Db = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
    const float ck = (k == 0 ? 1.0f : 2.0f) / RV_N;
    for (int h = 0; h < 2; ++h) {
      const int m = m0 + 2 * pr + h;
      if (m >= nf) continue;
      const float2 D = h ? Db : Da;
      const float2 u = U[(int64_t)m * 192 + k];
      const float dM = ck * (D.x * u.x + D.y * u.y);
      o[(int64_t)m * 192 + k] = dM * expf(h0[k] + (float)m * dk[k]);
    }
  }
}

// reduce over frames: dH0[k] = sum_m dMM[m][k];
// dtheta_d[k] = -sigmoid(theta_d[k] + beta) sum_m m dMM[m][k].
// grid (192 / 16, 2, nodes), block 256 = 16 bins x 16 frame lanes
__global__ __launch_bounds__(MG_BLOCK) void k_rv_adj_reduce(const NodeDesc* __restrict__ desc, int nf,
                                                             const float* __restrict__ dM,
                                                             const float* __restrict__ theta, float beta,
                                                             float* __restrict__ grad_theta) {
  __shared__ double ra[MG_BLOCK], rb[MG_BLOCK];
  const int x = blockIdx.y;
  const NodeDesc d = desc[blockIdx.z];
  const int kl = threadIdx.x % 16, lane = threadIdx.x / 16;
  const int k = blockIdx.x * 16 + kl;
  const float* src = dM + ((int64_t)d.aux * 2 + x) * nf * 192;
  double a = 0.0, b = 0.0;
  for (int m = lane; m < nf; m += 16) {
    const double v = src[(int64_t)m * 192 + k];
    a += v;
    b += (double)m * v;
  }
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int s = 8; s > 0; s >>= 1) {
    if (lane < s) {
      ra[threadIdx.x] += ra[threadIdx.x + s * 16];
      rb[threadIdx.x] += rb[threadIdx.x + s * 16];
    }
    __syncthreads();
  }
  if (lane == 0) {
    const double sg = 1.0 / (1.0 + exp(-((double)theta[d.theta_off + x * 384 + 192 + k] + (double)beta)));
    grad_theta[d.theta_off + x * 384 + k] = (float)ra[kl];
    grad_theta[d.theta_off + x * 384 + 192 + k] = (float)(-sg * rb[kl]);
  }
}

// ---------------------------------------------------------------- host side
static double reverb_gain_bias(int fs) { return -0.5 * log(0.5 * fs / (6.0 * 6.91)); }
// beta with softplus(beta) = per-frame log decay of a 0.5 s RT60
static double reverb_decay_offset(int fs, int hop) { return log(expm1(6.91 * hop / (0.5 * fs))); }

void fir_setup(const Ctx& c, const float* reverb_noise) {
  const mg_graph* g = c.g;
  const mg_config& cf = g->cfg;
  const double pi = 3.14159265358979323846;
  if (g->type_count[MG_EQ] > 0) {
    std::vector<float> t(cf.eq_taps);
    for (int m = 0; m < cf.eq_taps; ++m) t[m] = (float)cos(2.0 * pi * m / cf.eq_taps);
    hipMemcpyAsync(wsp<float>(c, g->ws.eq_cos), t.data(), t.size() * 4, hipMemcpyHostToDevice, c.st);
    hipStreamSynchronize(c.st);
  }
  if (g->type_count[MG_DELAY] > 0) {
    std::vector<float> t(cf.delay_fir_taps);
    for (int m = 0; m < cf.delay_fir_taps; ++m) t[m] = (float)cos(2.0 * pi * m / cf.delay_fir_taps);
    hipMemcpyAsync(wsp<float>(c, g->ws.dl_cos), t.data(), t.size() * 4, hipMemcpyHostToDevice, c.st);
    hipStreamSynchronize(c.st);
  }
  if (g->type_count[MG_REVERB] > 0) {
    std::vector<float2> cs(384);
    std::vector<float> win(384), ws(192);
    for (int m = 0; m < 384; ++m) {
      cs[m] = make_float2((float)cos(2.0 * pi * m / 384), (float)-sin(2.0 * pi * m / 384));
      win[m] = (float)(0.5 - 0.5 * cos(2.0 * pi * m / 384));
    }
    for (int r = 0; r < 192; ++r) {
      const double a = 0.5 - 0.5 * cos(2.0 * pi * r / 384), b = 0.5 - 0.5 * cos(2.0 * pi * (r + 192) / 384);
      ws[r] = (float)(a * a + b * b);
    }
    hipMemcpyAsync(wsp<float2>(c, g->ws.rv_cs), cs.data(), cs.size() * sizeof(float2), hipMemcpyHostToDevice, c.st);
    hipMemcpyAsync(wsp<float>(c, g->ws.rv_win), win.data(), win.size() * 4, hipMemcpyHostToDevice, c.st);
    hipMemcpyAsync(wsp<float>(c, g->ws.rv_wsum), ws.data(), ws.size() * 4, hipMemcpyHostToDevice, c.st);
    const int nrv = g->type_count[MG_REVERB];
    MG_LAUNCH(c, k_rv_noise_stft, dim3((g->nf_rev + RV_FPB - 1) / RV_FPB, 2, nrv), dim3(MG_BLOCK), 0, c.st,
                       reverb_noise,
                       cf.reverb_length, g->nf_rev, wsp<float2>(c, g->ws.rv_cs), wsp<float>(c, g->ws.rv_win),
                       wsp<float2>(c, g->ws.rv_U));
    hipStreamSynchronize(c.st);
  }
}

void fir_synth(const Ctx& c, int type, int desc_off, int n) {
  const mg_graph* g = c.g;
  const mg_config& cf = g->cfg;
  ProfScope ps(c, "fir", 0.0);
  const NodeDesc* d = c.desc + desc_off;
  if (type == MG_EQ) {
    MG_LAUNCH(c, k_eq_synth, dim3((cf.eq_taps + FIR_PER_BLOCK - 1) / FIR_PER_BLOCK, n), dim3(MG_BLOCK), 0,
              c.st, d, c.theta, cf.eq_taps, wsp<float>(c, g->ws.eq_h));
  } else if (type == MG_DELAY) {
    MG_LAUNCH(c, k_delay_synth, dim3(n), dim3(MG_BLOCK), 0, c.st, d, c.theta, wsp<float>(c, g->ws.dl_cos),
                       cf.delay_taps, cf.delay_range, cf.delay_fir_taps, wsp<float>(c, g->ws.dl_tab));
    MG_LAUNCH(c, k_delay_compact, dim3((unsigned)((g->dl_len + MG_BLOCK - 1) / MG_BLOCK), 2, n), dim3(MG_BLOCK),
                       0, c.st, d, wsp<float>(c, g->ws.dl_tab), cf.delay_taps, cf.delay_fir_taps, g->dl_len,
                       wsp<float>(c, g->ws.dl_h));
  } else if (type == MG_REVERB) {
    const float gb = (float)reverb_gain_bias(cf.sample_rate);
    const float db = (float)reverb_decay_offset(cf.sample_rate, cf.reverb_hop);
    ProfScope pr(c, "reverb_fir", (double)n * 2 * g->nf_rev * (192 * 8 + 384 * 4));
    MG_LAUNCH(c, k_rv_frames, dim3((g->nf_rev + RV_FPB - 1) / RV_FPB, 2, n), dim3(MG_BLOCK), 0, c.st, d,
                       c.theta,
                       wsp<float2>(c, g->ws.rv_U), g->nf_rev, wsp<float2>(c, g->ws.rv_cs),
                       wsp<float>(c, g->ws.rv_win), gb, db, wsp<float>(c, g->ws.rv_fr));
    MG_LAUNCH(c, k_rv_ola, dim3((cf.reverb_length + MG_BLOCK - 1) / MG_BLOCK, n), dim3(MG_BLOCK), 0, c.st, d,
                       wsp<float>(c, g->ws.rv_fr), g->nf_rev, cf.reverb_length, wsp<float>(c, g->ws.rv_wsum),
                       wsp<float>(c, g->ws.rv_h));
  }
}

void fir_adjoint(const Ctx& c, int type, int desc_off, int n, float* grad_theta) {
  const mg_graph* g = c.g;
  const mg_config& cf = g->cfg;
  ProfScope ps(c, "fir", 0.0);
  const NodeDesc* d = c.desc + desc_off;
  if (type == MG_EQ) {
    const int K = (cf.eq_taps + 1) / 2;
    MG_LAUNCH(c, k_eq_adjoint, dim3((K + FIR_PER_BLOCK - 1) / FIR_PER_BLOCK, n), dim3(MG_BLOCK), 0, c.st, d,
                       c.theta, cf.eq_taps, wsp<float>(c, g->ws.eq_dh), grad_theta);
  } else if (type == MG_DELAY) {
    double2* zp = wsp<double2>(c, g->ws.dl_zp);
    MG_LAUNCH(c, k_delay_adjoint, dim3(2 * cf.delay_taps, DL_CHUNKS, n), dim3(MG_BLOCK), 0, c.st, d, c.theta,
                       wsp<float>(c, g->ws.dl_tab), wsp<float>(c, g->ws.dl_cos), cf.delay_taps, cf.delay_range,
                       cf.delay_fir_taps, g->dl_len, wsp<float>(c, g->ws.dl_dh), grad_theta, zp);
    MG_LAUNCH(c, k_delay_zrule, dim3(n), dim3(128), 0, c.st, d, c.theta, cf.delay_taps, cf.delay_range,
                       cf.delay_fir_taps, (const double2*)zp, grad_theta, 0.01f);
  } else if (type == MG_REVERB) {
    const float gb = (float)reverb_gain_bias(cf.sample_rate);
    const float db = (float)reverb_decay_offset(cf.sample_rate, cf.reverb_hop);
    ProfScope pr(c, "reverb_fir", (double)n * 2 * g->nf_rev * (192 * 8 + 384 * 4 + 192 * 4));
    MG_LAUNCH(c, k_rv_adj_frames, dim3((g->nf_rev + RV_FPB - 1) / RV_FPB, 2, n), dim3(MG_BLOCK), 0, c.st, d,
                       c.theta,
                       wsp<float2>(c, g->ws.rv_U), g->nf_rev, cf.reverb_length, wsp<float2>(c, g->ws.rv_cs),
                       wsp<float>(c, g->ws.rv_win), wsp<float>(c, g->ws.rv_wsum), gb, db,
                       wsp<float>(c, g->ws.rv_dh), wsp<float>(c, g->ws.rv_dM));
    MG_LAUNCH(c, k_rv_adj_reduce, dim3(192 / 16, 2, n), dim3(MG_BLOCK), 0, c.st, d, g->nf_rev,
                       wsp<float>(c, g->ws.rv_dM), c.theta, db, grad_theta);
  }
}

}  // namespace mg
