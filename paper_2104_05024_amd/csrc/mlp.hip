// Learned warm start for the GMRES density of the bidomain step (not part of the paper's
// method: Algorithm 1 starts from psi = 0).
//
// The previous solve left A psi^{n-1} = g'^{n-1}, so psi^n - psi^{n-1} = A^{-1}(g'^n - g'^{n-1}),
// with A one half of the identity plus a compact part.  The network approximates this change by
// a local linear map whose coefficients depend on the local geometry only:
//   geometry rows  G(i) = (n(i), h tr W(i))  (static, BF16)
//   change fields  F(i) = ((psi^{n-1} - psi^{n-2})_c / s_d, (g'^n - g'^{n-1})_c / s_g)  (FP32)
//   coefficients   K(i) = net(G(i)),  y_c(i) = sum_f K_{c,f}(i) F_f(i),  psi0 = psi^{n-1} + s_d y.
// Weighting the fields' changes keeps the start as smooth as the fields (a start with
// node-to-node noise slows GMRES down even when its residual is small).  net has three tanh
// layers of width 128; weights and activations are BF16, products accumulate in FP32 on the
// matrix cores (v_mfma_f32_16x16x16_bf16), Adam master weights are FP32.  K depends on the
// static geometry only, so it is evaluated once after training; training is full-batch over
// the recorded steps (one forward and one backward pass of the network per epoch).
//
// MFMA 16x16x16 operand layout (wave of 64 lanes, l = lane): A[i][k] with i = l%16,
// k = 4(l/16)+j; B[k][n] with n = l%16, k = 4(l/16)+j; D[i][n] with n = l%16, i = 4(l/16)+j.
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "solver.h"

namespace kfbi {

constexpr int kIn = 16;     // padded input features
constexpr int kHid = 128;   // hidden width
constexpr int kOut = 16;    // padded outputs (ncomp real)
constexpr int kWgBlocks = 256;   // blocks of the weight-gradient reduction (fixed order)
constexpr int kRowsWG = 64; // rows per workgroup in the row-parallel kernels

struct Mlp {
  int ncomp = 2, dim = 3, nfeat = 0, nf = 4;
  int64_t M = 0;
  int cap = 0, count = 0, head = 0, adam_t = 0;
  bool enabled = true, k_valid = false;
  int since_check = 0, check_every = 8, fallbacks = 0;
  // solve cost (FP64 matvecs + FP32 matvecs / 2) of the last 8 steps started from psi^{n-1}
  // and of the learned starts since the last cost check
  double plain_ring[8] = {0, 0, 0, 0, 0, 0, 0, 0}, learned_cost = 0;
  int plain_n = 0, learned_n = 0;
  // parameters: fp32 master, bf16 copies, gradients and Adam moments
  float *W[4] = {}, *b[4] = {}, *gW[4] = {}, *gb[4] = {}, *mW[4] = {}, *vW[4] = {}, *mb[4] = {}, *vb[4] = {};
  uint16_t *Wb[4] = {};
  int wrows[4] = {kHid, kHid, kHid, kOut}, wcols[4] = {kIn, kHid, kHid, kHid};
  uint16_t *G = nullptr;    // [M][kIn] geometry rows
  float *Fs = nullptr;      // [cap][M][nf] recorded change fields
  float *Ts = nullptr;      // [cap][M][ncomp] recorded targets
  float *F = nullptr;       // [M][nf] change fields of the current step
  // per-pass work
  uint16_t *X = nullptr, *A1 = nullptr, *A2 = nullptr, *A3 = nullptr, *dZ4 = nullptr, *dZ3 = nullptr,
           *dZ2 = nullptr, *dZ1 = nullptr;
  float *Y = nullptr;       // [M][kOut] network output (the coefficients K once trained)
  double *scal = nullptr;   // [0] s_d, [1] s_g, [2..] partial maxima
  float *loss = nullptr;    // [blocks]
  int nloss = 0;
  // per-block weight-gradient partials [kWgBlocks][kHid * kHid] and [kWgBlocks][kHid], summed
  // in a fixed order (training is deterministic: no atomics)
  float *gWp = nullptr, *gbp = nullptr;
};

namespace {

constexpr int kB = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);   // round to nearest even
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
inline uint16_t f2bf_host(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

// |x| maxima: one block finishes the per-block partials (fixed order)
__global__ __launch_bounds__(kB) void k_absmax_finish(const double *__restrict__ part, int nb, double *__restrict__ out) {
  __shared__ double s[kB];
  double m = 0;
  for (int i = threadIdx.x; i < nb; i += kB) m = fmax(m, part[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0] > 0 ? s[0] : 1.0;
}

// |a - b| maxima: per-block partials (k_absmax_finish completes them)
__global__ __launch_bounds__(kB) void k_absmax_diff(const double *__restrict__ a, const double *__restrict__ b,
                                                    int64_t n, double *__restrict__ part) {
  __shared__ double s[kB];
  double m = 0;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    m = fmax(m, fabs(a[i] - b[i]));
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// change fields F[q][2c] = (psi1 - psi2)_c / s_d, F[q][2c + 1] = (gp - gq)_c / s_g   (FP32)
__global__ __launch_bounds__(kB) void k_fields(const double *__restrict__ psi1, const double *__restrict__ psi2,
                                               const double *__restrict__ gp, const double *__restrict__ gq,
                                               const double *__restrict__ scal, int64_t M, int ncomp,
                                               float *__restrict__ F) {
  const int64_t q = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (q >= M) return;
  const double isd = 1.0 / scal[0], isg = 1.0 / scal[1];
  for (int c = 0; c < ncomp; ++c) {
    F[q * 2 * ncomp + 2 * c] = (float)((psi1[c * M + q] - psi2[c * M + q]) * isd);
    F[q * 2 * ncomp + 2 * c + 1] = (float)((gp[c * M + q] - gq[c * M + q]) * isg);
  }
}

// targets T[q][c] = (psi - psi1)_c / s_d
__global__ __launch_bounds__(kB) void k_targets(const double *__restrict__ psi, const double *__restrict__ psi1,
                                                const double *__restrict__ scal, int64_t M, int ncomp,
                                                float *__restrict__ T) {
  const int64_t q = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (q >= M) return;
  const double isd = 1.0 / scal[0];
  for (int c = 0; c < ncomp; ++c) T[q * ncomp + c] = (float)((psi[c * M + q] - psi1[c * M + q]) * isd);
}

// psi0 = psi1 + s_d sum_f K[q][c nf + f] F[q][f]
__global__ __launch_bounds__(kB) void k_predict(const float *__restrict__ K, const float *__restrict__ F,
                                                const double *__restrict__ psi1, const double *__restrict__ scal,
                                                int64_t M, int ncomp, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= M * ncomp) return;
  const int64_t c = i / M, q = i - c * M;
  const int nf = 2 * ncomp;
  double y = 0;
  for (int f = 0; f < nf; ++f) y += (double)K[q * kOut + c * nf + f] * (double)F[q * nf + f];
  out[i] = psi1[i] + scal[0] * y;
}

// Loss gradient with respect to the coefficients over S recorded steps:
// dK[q][c nf + f] = sum_s d_s[q][c] F_s[q][f] / n, d_s = K F_s - T_s, n = M ncomp S (BF16 out),
// and the partial sums of the loss 0.5 sum d^2 / n.
__global__ __launch_bounds__(kB) void k_dk(const float *__restrict__ K, const float *__restrict__ Fs,
                                           const float *__restrict__ Ts, int S, int64_t M, int ncomp,
                                           uint16_t *__restrict__ dZ, float *__restrict__ part) {
  __shared__ float sh[kB];
  const int nf = 2 * ncomp;
  const float inv = 1.0f / ((float)M * (float)ncomp * (float)S);
  float lacc = 0.f;
  for (int64_t q = (int64_t)blockIdx.x * kB + threadIdx.x; q < M; q += (int64_t)gridDim.x * kB) {
    float k[kOut], g[kOut];
#pragma unroll
    for (int o = 0; o < kOut; ++o) {
      k[o] = K[q * kOut + o];
      g[o] = 0.f;
    }
    for (int s = 0; s < S; ++s) {
      const float *F = Fs + ((int64_t)s * M + q) * nf;
      const float *T = Ts + ((int64_t)s * M + q) * ncomp;
      for (int c = 0; c < ncomp; ++c) {
        float y = 0.f;
        for (int f = 0; f < nf; ++f) y += k[c * nf + f] * F[f];
        const float d = y - T[c];
        lacc += 0.5f * d * d;
        for (int f = 0; f < nf; ++f) g[c * nf + f] += d * F[f];
      }
    }
#pragma unroll
    for (int o = 0; o < kOut; ++o) dZ[q * kOut + o] = f2bf(g[o] * inv);
  }
  sh[threadIdx.x] = lacc;
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] * inv;
}

// One dense layer on a wave's 16 rows: out[16 x NOUT] = in[16 x K] W^T + b (then tanh).
// in: LDS rows (stride lds_in), W: [NOUT][K] bf16 global.  Results to LDS (bf16), and to
// global act rows if `gout` is given; or fp32 to Y when LAST.
template <int K, int NOUT, bool LAST>
__device__ __forceinline__ void dense_wave(const uint16_t *in, int lds_in, const uint16_t *__restrict__ W,
                                           const float *__restrict__ bias, uint16_t *outl, int lds_out,
                                           uint16_t *__restrict__ gout, int64_t grow0, int64_t R,
                                           float *__restrict__ Y, int lane) {
  constexpr int NB = NOUT / 16;
  f4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f4{0, 0, 0, 0};
  const int i = lane % 16, kg = 4 * (lane / 16);
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) {
    s4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = (short)in[i * lds_in + k0 + kg + j];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      s4 b;
      const uint16_t *wr = W + (int64_t)(nb * 16 + i) * K + k0 + kg;
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = (short)wr[j];
      acc[nb] = mfma(a, b, acc[nb]);
    }
  }
  const int col = lane % 16;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const float bb = bias[nb * 16 + col];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = kg + j;
      const float z = acc[nb][j] + bb;
      if (LAST) {
        if (grow0 + row < R) Y[(grow0 + row) * kOut + nb * 16 + col] = z;
      } else {
        const uint16_t h = f2bf(tanhf(z));
        outl[row * lds_out + nb * 16 + col] = h;
        if (gout && grow0 + row < R) gout[(grow0 + row) * kHid + nb * 16 + col] = h;
      }
    }
  }
}

// Forward pass over R rows: 64 rows per workgroup, one wave per 16 rows (no cross-wave traffic).
template <bool STORE>
__global__ __launch_bounds__(256) void k_mlp_fwd(const uint16_t *__restrict__ X, int64_t R,
                                                 const uint16_t *__restrict__ W1, const uint16_t *__restrict__ W2,
                                                 const uint16_t *__restrict__ W3, const uint16_t *__restrict__ W4,
                                                 const float *__restrict__ b1, const float *__restrict__ b2,
                                                 const float *__restrict__ b3, const float *__restrict__ b4,
                                                 uint16_t *__restrict__ A1, uint16_t *__restrict__ A2,
                                                 uint16_t *__restrict__ A3, float *__restrict__ Y) {
  constexpr int LP = kHid + 8;   // padded LDS row
  __shared__ uint16_t s_in[kRowsWG * kIn];
  __shared__ uint16_t s_a[kRowsWG * LP], s_b[kRowsWG * LP];
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  const int64_t r0 = (int64_t)blockIdx.x * kRowsWG;
  for (int e = tid; e < kRowsWG * kIn; e += 256) {
    const int64_t r = r0 + e / kIn;
    s_in[e] = r < R ? X[r * kIn + (e % kIn)] : (uint16_t)0;
  }
  __syncthreads();
  const int64_t g0 = r0 + 16 * w;
  dense_wave<kIn, kHid, false>(s_in + 16 * w * kIn, kIn, W1, b1, s_a + 16 * w * LP, LP, STORE ? A1 : nullptr, g0, R,
                               nullptr, lane);
  __syncthreads();
  dense_wave<kHid, kHid, false>(s_a + 16 * w * LP, LP, W2, b2, s_b + 16 * w * LP, LP, STORE ? A2 : nullptr, g0, R,
                                nullptr, lane);
  __syncthreads();
  dense_wave<kHid, kHid, false>(s_b + 16 * w * LP, LP, W3, b3, s_a + 16 * w * LP, LP, STORE ? A3 : nullptr, g0, R,
                                nullptr, lane);
  __syncthreads();
  dense_wave<kHid, kOut, true>(s_a + 16 * w * LP, LP, W4, b4, nullptr, 0, nullptr, g0, R, Y, lane);
}

// Backward through a layer: dZout[r][n] = (sum_o dZin[r][o] W[o][n]) * (1 - A[r][n]^2).
// KIN = width of dZin (out features of the layer), W: [KIN][kHid].
template <int KIN>
__global__ __launch_bounds__(256) void k_bwd_data(const uint16_t *__restrict__ dZin, const uint16_t *__restrict__ W,
                                                  const uint16_t *__restrict__ A, int64_t R,
                                                  uint16_t *__restrict__ dZout) {
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  const int64_t g0 = (int64_t)blockIdx.x * kRowsWG + 16 * w;
  const int i = lane % 16, kg = 4 * (lane / 16);
  constexpr int NB = kHid / 16;
  f4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = f4{0, 0, 0, 0};
#pragma unroll
  for (int k0 = 0; k0 < KIN; k0 += 16) {
    s4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = (g0 + i < R) ? (short)dZin[(g0 + i) * KIN + k0 + kg + j] : (short)0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      s4 b;
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = (short)W[(int64_t)(k0 + kg + j) * kHid + nb * 16 + i];
      acc[nb] = mfma(a, b, acc[nb]);
    }
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t r = g0 + kg + j;
      const int n = nb * 16 + (lane % 16);
      if (r < R) {
        const float a = bf2f(A[r * kHid + n]);
        dZout[r * kHid + n] = f2bf(acc[nb][j] * (1.f - a * a));
      }
    }
}

// Weight-gradient partials of this block's rows: gWp[block][o][c] = sum_r dZ[r][o] Ain[r][c],
// gbp[block][o] = sum_r dZ[r][o].  NO x NC output tiles of 16x16 spread over 4 waves; reduction
// over rows in steps of 16.  k_wgrad_sum adds the blocks' partials in block order.
template <int NO, int NCI>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t *__restrict__ dZ, const uint16_t *__restrict__ Ain,
                                               int64_t R, int64_t rows_per_block, float *__restrict__ gWp,
                                               float *__restrict__ gbp) {
  constexpr int TO = NO / 16, TC = NCI / 16, NT = TO * TC, PW = (NT + 3) / 4;
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  const int i = lane % 16, kg = 4 * (lane / 16);
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block, re = rb + rows_per_block < R ? rb + rows_per_block : R;
  f4 acc[PW];
#pragma unroll
  for (int t = 0; t < PW; ++t) acc[t] = f4{0, 0, 0, 0};
  float bsum = 0.f;
  for (int64_t r0 = rb; r0 < re; r0 += 16) {
#pragma unroll
    for (int t = 0; t < PW; ++t) {
      const int tile = w + 4 * t;
      if (tile >= NT) break;
      const int to = tile / TC, tc = tile % TC;
      s4 a, b;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t r = r0 + kg + j;
        const bool ok = r < re;
        a[j] = ok ? (short)dZ[r * NO + to * 16 + i] : (short)0;
        b[j] = ok ? (short)Ain[r * NCI + tc * 16 + i] : (short)0;
      }
      acc[t] = mfma(a, b, acc[t]);
    }
    if (tid < NO) {
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (r0 + j < re) bsum += bf2f(dZ[(r0 + j) * NO + tid]);
    }
  }
#pragma unroll
  for (int t = 0; t < PW; ++t) {
    const int tile = w + 4 * t;
    if (tile >= NT) break;
    const int to = tile / TC, tc = tile % TC;
    float *gw = gWp + (int64_t)blockIdx.x * NO * NCI;
#pragma unroll
    for (int j = 0; j < 4; ++j) gw[(to * 16 + kg + j) * NCI + tc * 16 + (lane % 16)] = acc[t][j];
  }
  if (tid < NO) gbp[(int64_t)blockIdx.x * NO + tid] = bsum;
}

// gW[e] += sum over blocks b < nblocks of gWp[b][e] (and the biases likewise), in block order.
template <int NO, int NCI>
__global__ __launch_bounds__(kB) void k_wgrad_sum(const float *__restrict__ gWp, const float *__restrict__ gbp,
                                                  int nblocks, float *__restrict__ gW, float *__restrict__ gb) {
  const int e = blockIdx.x * kB + threadIdx.x;
  if (e < NO * NCI) {
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += gWp[(int64_t)b * NO * NCI + e];
    gW[e] += s;
  } else if (e < NO * NCI + NO) {
    const int o = e - NO * NCI;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += gbp[(int64_t)b * NO + o];
    gb[o] += s;
  }
}

// Adam (bias-corrected) on fp32 master weights; refreshes the bf16 copy and clears the gradient.
__global__ __launch_bounds__(kB) void k_adam(float *__restrict__ p, float *__restrict__ g, float *__restrict__ m,
                                             float *__restrict__ v, uint16_t *__restrict__ pb, int64_t n, float lr,
                                             float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float x = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  p[i] = x;
  if (pb) pb[i] = f2bf(x);
  g[i] = 0.f;
}

template <typename T>
T *dalloc(size_t n) {
  T *p = nullptr;
  KFBI_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
  KFBI_HIP(hipMemset(p, 0, std::max<size_t>(n, 1) * sizeof(T)));
  return p;
}

// SplitMix64 (Steele, Lea, Flood 2014) -> uniform doubles in [0, 1)
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

void build_fields(bidomain_s *b, const double *psi1, const double *psi2, hipStream_t st) {
  Mlp &m = *b->mlp;
  Solver &sv = *b->solver;
  const int64_t L = sv.L;
  const int nbm = (int)std::min<int64_t>(256, (L + kB - 1) / kB);
  k_absmax_diff<<<nbm, kB, 0, st>>>(psi1, psi2, L, m.scal + 2);
  k_absmax_finish<<<1, kB, 0, st>>>(m.scal + 2, nbm, m.scal + 0);
  k_absmax_diff<<<nbm, kB, 0, st>>>(sv.gp, b->gp_prev, L, m.scal + 2);
  k_absmax_finish<<<1, kB, 0, st>>>(m.scal + 2, nbm, m.scal + 1);
  k_fields<<<nblk(m.M), kB, 0, st>>>(psi1, psi2, sv.gp, b->gp_prev, m.scal, m.M, m.ncomp, m.F);
  KFBI_HIP(hipGetLastError());
}

void forward(Mlp &m, const uint16_t *X, int64_t R, bool store, hipStream_t st) {
  const unsigned g = (unsigned)((R + kRowsWG - 1) / kRowsWG);
  if (store)
    k_mlp_fwd<true><<<g, 256, 0, st>>>(X, R, m.Wb[0], m.Wb[1], m.Wb[2], m.Wb[3], m.b[0], m.b[1], m.b[2], m.b[3], m.A1,
                                      m.A2, m.A3, m.Y);
  else
    k_mlp_fwd<false><<<g, 256, 0, st>>>(X, R, m.Wb[0], m.Wb[1], m.Wb[2], m.Wb[3], m.b[0], m.b[1], m.b[2], m.b[3],
                                       nullptr, nullptr, nullptr, m.Y);
  KFBI_HIP(hipGetLastError());
}

// Parameter gradients (accumulated into gW, gb) from the output gradient already in dZ4,
// after forward(X, store = true).
void backward_net(Mlp &m, const uint16_t *X, int64_t R, hipStream_t st) {
  const unsigned g = (unsigned)((R + kRowsWG - 1) / kRowsWG);
  k_bwd_data<kOut><<<g, 256, 0, st>>>(m.dZ4, m.Wb[3], m.A3, R, m.dZ3);
  k_bwd_data<kHid><<<g, 256, 0, st>>>(m.dZ3, m.Wb[2], m.A2, R, m.dZ2);
  k_bwd_data<kHid><<<g, 256, 0, st>>>(m.dZ2, m.Wb[1], m.A1, R, m.dZ1);
  // at most kWgBlocks blocks of a multiple of 16 rows each
  const int64_t rpb = std::max<int64_t>(16, ((R + kWgBlocks - 1) / kWgBlocks + 15) / 16 * 16);
  const unsigned gw = (unsigned)((R + rpb - 1) / rpb);
  auto sum_blocks = [&](int no, int nci, int l) {
    const unsigned g = nblk((int64_t)no * nci + no);
    if (no == kOut) k_wgrad_sum<kOut, kHid><<<g, kB, 0, st>>>(m.gWp, m.gbp, (int)gw, m.gW[l], m.gb[l]);
    else if (nci == kIn) k_wgrad_sum<kHid, kIn><<<g, kB, 0, st>>>(m.gWp, m.gbp, (int)gw, m.gW[l], m.gb[l]);
    else k_wgrad_sum<kHid, kHid><<<g, kB, 0, st>>>(m.gWp, m.gbp, (int)gw, m.gW[l], m.gb[l]);
  };
  k_wgrad<kOut, kHid><<<gw, 256, 0, st>>>(m.dZ4, m.A3, R, rpb, m.gWp, m.gbp);
  sum_blocks(kOut, kHid, 3);
  k_wgrad<kHid, kHid><<<gw, 256, 0, st>>>(m.dZ3, m.A2, R, rpb, m.gWp, m.gbp);
  sum_blocks(kHid, kHid, 2);
  k_wgrad<kHid, kHid><<<gw, 256, 0, st>>>(m.dZ2, m.A1, R, rpb, m.gWp, m.gbp);
  sum_blocks(kHid, kHid, 1);
  k_wgrad<kHid, kIn><<<gw, 256, 0, st>>>(m.dZ1, X, R, rpb, m.gWp, m.gbp);
  sum_blocks(kHid, kIn, 0);
  KFBI_HIP(hipGetLastError());
}

void adam(Mlp &m, double lr, hipStream_t st) {
  m.adam_t += 1;
  const float c1 = 1.0f - std::pow(0.9f, (float)m.adam_t), c2 = 1.0f - std::pow(0.999f, (float)m.adam_t);
  for (int l = 0; l < 4; ++l) {
    const int64_t nw = (int64_t)m.wrows[l] * m.wcols[l];
    k_adam<<<nblk(nw), kB, 0, st>>>(m.W[l], m.gW[l], m.mW[l], m.vW[l], m.Wb[l], nw, (float)lr, c1, c2);
    k_adam<<<nblk(m.wrows[l]), kB, 0, st>>>(m.b[l], m.gb[l], m.mb[l], m.vb[l], nullptr, m.wrows[l], (float)lr, c1,
                                            c2);
  }
  KFBI_HIP(hipGetLastError());
}

}  // namespace
}  // namespace kfbi

using namespace kfbi;

void mlp_release(bidomain_s *b) {
  if (!b->mlp) return;
  Mlp &m = *b->mlp;
  for (int l = 0; l < 4; ++l) {
    float **fs[] = {&m.W[l], &m.b[l], &m.gW[l], &m.gb[l], &m.mW[l], &m.vW[l], &m.mb[l], &m.vb[l]};
    for (float **f : fs)
      if (*f) (void)hipFree(*f);
    if (m.Wb[l]) (void)hipFree(m.Wb[l]);
  }
  uint16_t *us[] = {m.G, m.X, m.A1, m.A2, m.A3, m.dZ4, m.dZ3, m.dZ2, m.dZ1};
  for (uint16_t *u : us)
    if (u) (void)hipFree(u);
  float *fs[] = {m.Fs, m.Ts, m.F, m.Y, m.loss, m.gWp, m.gbp};
  for (float *f : fs)
    if (f) (void)hipFree(f);
  if (m.scal) (void)hipFree(m.scal);
  delete b->mlp;
  b->mlp = nullptr;
}

void bidomain_s::mlp_init(int capacity, uint64_t seed) {
  mlp_release(this);
  mlp = new Mlp();
  Mlp &m = *mlp;
  const DevProblem &p = *prob;
  m.ncomp = p.ncomp;
  m.dim = p.dim;
  m.M = p.M;
  m.nfeat = p.dim + 1;
  m.nf = 2 * p.ncomp;
  if (m.nfeat > kIn || m.ncomp * m.nf > kOut) throw std::invalid_argument("network shape");
  m.cap = capacity;
  SplitMix64 rng{seed};
  for (int l = 0; l < 4; ++l) {
    const int r = m.wrows[l], c = m.wcols[l];
    const int fan_in = l == 0 ? m.nfeat : c, fan_out = l == 3 ? m.ncomp * m.nf : r;
    const double bound = 1.0 / std::sqrt((double)fan_in);
    std::vector<float> w((size_t)r * c, 0.f);
    std::vector<uint16_t> wb((size_t)r * c, 0);
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < c; ++j) {
        const double u = rng.uniform();
        // the output layer starts at zero: the untrained network predicts no change
        if (l < 3 && i < fan_out && j < fan_in) w[(size_t)i * c + j] = (float)((2.0 * u - 1.0) * bound);
        wb[(size_t)i * c + j] = f2bf_host(w[(size_t)i * c + j]);
      }
    m.W[l] = dalloc<float>(w.size());
    m.Wb[l] = dalloc<uint16_t>(w.size());
    KFBI_HIP(hipMemcpy(m.W[l], w.data(), w.size() * 4, hipMemcpyHostToDevice));
    KFBI_HIP(hipMemcpy(m.Wb[l], wb.data(), wb.size() * 2, hipMemcpyHostToDevice));
    m.b[l] = dalloc<float>(r);
    m.gW[l] = dalloc<float>(w.size());
    m.gb[l] = dalloc<float>(r);
    m.mW[l] = dalloc<float>(w.size());
    m.vW[l] = dalloc<float>(w.size());
    m.mb[l] = dalloc<float>(r);
    m.vb[l] = dalloc<float>(r);
  }
  m.gWp = dalloc<float>((size_t)kWgBlocks * kHid * kHid);
  m.gbp = dalloc<float>((size_t)kWgBlocks * kHid);
  const int64_t M = m.M;
  m.Fs = dalloc<float>((size_t)m.cap * M * m.nf);
  m.Ts = dalloc<float>((size_t)m.cap * M * m.ncomp);
  m.F = dalloc<float>((size_t)M * m.nf);
  m.G = dalloc<uint16_t>((size_t)M * kIn);
  m.X = dalloc<uint16_t>((size_t)M * kIn);
  m.A1 = dalloc<uint16_t>((size_t)M * kHid);
  m.A2 = dalloc<uint16_t>((size_t)M * kHid);
  m.A3 = dalloc<uint16_t>((size_t)M * kHid);
  m.dZ4 = dalloc<uint16_t>((size_t)M * kOut);
  m.dZ3 = dalloc<uint16_t>((size_t)M * kHid);
  m.dZ2 = dalloc<uint16_t>((size_t)M * kHid);
  m.dZ1 = dalloc<uint16_t>((size_t)M * kHid);
  m.Y = dalloc<float>((size_t)M * kOut);
  m.nloss = 256;
  m.loss = dalloc<float>(m.nloss);
  m.scal = dalloc<double>(2 + 256);
  // static geometry rows: n (d entries), h tr W, zeros
  const HostTables &t = p.ht;
  std::vector<uint16_t> g((size_t)M * kIn, 0);
  for (int64_t q = 0; q < M; ++q) {
    double tr = 0;
    for (int a = 0; a < t.dim; ++a) {
      tr += t.W[(q * t.dim + a) * t.dim + a];
      g[q * kIn + a] = f2bf_host((float)t.nrm[q * t.dim + a]);
    }
    g[q * kIn + t.dim] = f2bf_host((float)(t.h * tr));
  }
  KFBI_HIP(hipMemcpy(m.G, g.data(), g.size() * 2, hipMemcpyHostToDevice));
}

// Record (change fields, target) of the step just solved: psi1 = psi^{n-1}, psi2 = psi^{n-2}, psi = psi^n.
void mlp_record(bidomain_s *b, const double *psi1, const double *psi2, const double *psi, hipStream_t st) {
  Mlp &m = *b->mlp;
  build_fields(b, psi1, psi2, st);
  const int slot = m.head;
  KFBI_HIP(hipMemcpyAsync(m.Fs + (size_t)slot * m.M * m.nf, m.F, m.M * m.nf * sizeof(float),
                          hipMemcpyDeviceToDevice, st));
  k_targets<<<nblk(m.M), kB, 0, st>>>(psi, psi1, m.scal, m.M, m.ncomp, m.Ts + (size_t)slot * m.M * m.ncomp);
  KFBI_HIP(hipGetLastError());
  m.head = (m.head + 1) % m.cap;
  m.count = std::min(m.count + 1, m.cap);
}

// Predicted start density; false if the network is untrained or switched off (fallback to psi^{n-1}).
bool mlp_warm_start(bidomain_s *b, const double *psi1, const double *psi2, double *out, hipStream_t st) {
  Mlp &m = *b->mlp;
  if (!m.enabled || !m.k_valid) return false;
  build_fields(b, psi1, psi2, st);
  k_predict<<<nblk(m.M * m.ncomp), kB, 0, st>>>(m.Y, m.F, psi1, m.scal, m.M, m.ncomp, out);
  KFBI_HIP(hipGetLastError());
  return true;
}

double bidomain_s::mlp_train(int epochs, double lr, hipStream_t st) {
  Mlp &m = *mlp;
  if (m.count == 0) throw std::invalid_argument("no recorded samples");
  std::vector<float> part(m.nloss);
  double last = 0;
  for (int e = 0; e < epochs; ++e) {
    forward(m, m.G, m.M, true, st);
    k_dk<<<m.nloss, kB, 0, st>>>(m.Y, m.Fs, m.Ts, m.count, m.M, m.ncomp, m.dZ4, m.loss);
    KFBI_HIP(hipGetLastError());
    if (e == epochs - 1) {
      KFBI_HIP(hipMemcpyAsync(part.data(), m.loss, m.nloss * sizeof(float), hipMemcpyDeviceToHost, st));
      KFBI_HIP(hipStreamSynchronize(st));
      last = 0;
      for (float v : part) last += v;
    }
    backward_net(m, m.G, m.M, st);
    adam(m, lr, st);
  }
  forward(m, m.G, m.M, false, st);      // coefficients K for inference
  KFBI_HIP(hipStreamSynchronize(st));
  m.k_valid = true;
  m.enabled = true;
  m.since_check = 0;
  m.learned_cost = 0;
  m.learned_n = 0;
  return last;
}

int bidomain_s::mlp_params(float *dst, int64_t *count) {
  Mlp &m = *mlp;
  int64_t n = 0;
  for (int l = 0; l < 4; ++l) n += (int64_t)m.wrows[l] * m.wcols[l] + m.wrows[l];
  if (count) *count = n;
  if (!dst) return KFBI_OK;
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    const int64_t nw = (int64_t)m.wrows[l] * m.wcols[l];
    KFBI_HIP(hipMemcpy(dst + off, m.W[l], nw * 4, hipMemcpyDeviceToHost));
    off += nw;
    KFBI_HIP(hipMemcpy(dst + off, m.b[l], m.wrows[l] * 4, hipMemcpyDeviceToHost));
    off += m.wrows[l];
  }
  return KFBI_OK;
}

// Test hook: network output on host rows X [R][kIn]; with dY [R][kOut] also the parameter
// gradients of sum(dY * output).  The trained coefficients are restored afterwards.
int mlp_eval(bidomain_s *b, const float *X_host, int64_t R, float *Y_host, float *grad_host, const float *dY_host,
             hipStream_t st) {
  Mlp &m = *b->mlp;
  if (R > m.M) throw std::invalid_argument("too many rows");
  std::vector<uint16_t> xb((size_t)R * kIn);
  for (int64_t i = 0; i < R * kIn; ++i) xb[i] = f2bf_host(X_host[i]);
  KFBI_HIP(hipMemcpy(m.X, xb.data(), xb.size() * 2, hipMemcpyHostToDevice));
  forward(m, m.X, R, dY_host != nullptr, st);
  KFBI_HIP(hipStreamSynchronize(st));
  if (Y_host) KFBI_HIP(hipMemcpy(Y_host, m.Y, (size_t)R * kOut * 4, hipMemcpyDeviceToHost));
  if (dY_host) {
    std::vector<uint16_t> db((size_t)R * kOut);
    for (int64_t i = 0; i < R * kOut; ++i) db[i] = f2bf_host(dY_host[i]);
    KFBI_HIP(hipMemcpy(m.dZ4, db.data(), db.size() * 2, hipMemcpyHostToDevice));
    backward_net(m, m.X, R, st);
    KFBI_HIP(hipStreamSynchronize(st));
    int64_t off = 0;
    for (int l = 0; l < 4; ++l) {
      const int64_t nw = (int64_t)m.wrows[l] * m.wcols[l];
      if (grad_host) KFBI_HIP(hipMemcpy(grad_host + off, m.gW[l], nw * 4, hipMemcpyDeviceToHost));
      off += nw;
      if (grad_host) KFBI_HIP(hipMemcpy(grad_host + off, m.gb[l], m.wrows[l] * 4, hipMemcpyDeviceToHost));
      off += m.wrows[l];
      KFBI_HIP(hipMemset(m.gW[l], 0, (size_t)nw * 4));
      KFBI_HIP(hipMemset(m.gb[l], 0, (size_t)m.wrows[l] * 4));
    }
  }
  if (m.k_valid) forward(m, m.G, m.M, false, st);
  KFBI_HIP(hipStreamSynchronize(st));
  return KFBI_OK;
}

void mlp_disable(bidomain_s *b) {
  if (b->mlp) {
    b->mlp->enabled = false;
    b->mlp->fallbacks += 1;
  }
}

// Cost bookkeeping after each solve: every check_every learned solves, compare their mean cost
// with that of the last 8 solves started from psi^{n-1}; switch the learned start off if it is
// not cheaper.
void mlp_note_cost(bidomain_s *b, double cost, bool learned) {
  Mlp &m = *b->mlp;
  if (!learned) {
    m.plain_ring[m.plain_n % 8] = cost;
    m.plain_n += 1;
    return;
  }
  m.learned_cost += cost;
  m.learned_n += 1;
  if (m.learned_n >= m.check_every) {
    const int np = std::min(m.plain_n, 8);
    double pc = 0;
    for (int i = 0; i < np; ++i) pc += m.plain_ring[i];
    if (np > 0 && m.learned_cost / m.learned_n >= pc / np) {
      m.enabled = false;
      m.fallbacks += 1;
    }
    m.learned_cost = 0;
    m.learned_n = 0;
  }
}

bool mlp_should_check(bidomain_s *b) {
  Mlp &m = *b->mlp;
  const bool c = (m.since_check % m.check_every) == 0;
  m.since_check += 1;
  return c;
}
