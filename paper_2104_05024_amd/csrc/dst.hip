// Fast box solver: batched DST-I pencils with LDS-staged tiles (gfx950).
//
// The 5/7-point operator of Sec. 5.2 (eq. FDE) with u = 0 on the box boundary is
// diagonalised by the sine modes of every axis, so one solve is
//   DST-I along x, y (, z) -> divide by the mode eigenvalues -> inverse DST-I,
// the eigenvalue division being a scalar or a closed-form 2x2 solve per mode for the
// coupled pair (the fast solver named at the end of Sec. 5.3).
//
// DST-I of length N = M - 1 (M = 2^m) is computed for two real pencils at once from one
// complex FFT of length M:
//   t_n = sin(pi n/M)(x_n + x_{M-n}) + (x_n - x_{M-n})/2,  t_0 = 0,
//   T = FFT_M(t):  y_{2k} = -Im T_k,  y_{2k+1} = y_{2k-1} + Re T_k,  y_1 = Re T_0 / 2,
// and the two real pencils ride in the real and imaginary parts of t.  The prefix sum
// over the odd outputs is a chunked scan across the lanes that own the pencil pair.
// The FFT is a Stockham radix-16 (then 2/4/8/16) transform in LDS: every thread holds
// exactly 16 complex values per stage.
//
// Passes (3D, fields in the padded [comp][z][y][x] layout with row pitch P = M):
//   x (contiguous rows) -> y (tiles of columns, one z-plane) -> z fused with the mode
//   scaling and the inverse z transform -> y inverse -> x inverse.
// Each pass reads and writes its tile once; y and z passes work in place.
#include <algorithm>
#include <array>
#include <map>
#include <mutex>

#include "device.h"

namespace kfbi {
namespace {

template <typename T>
struct C2 {
  T x, y;
};
template <typename T>
__device__ __forceinline__ C2<T> operator+(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> operator-(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> operator*(T s, C2<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// exp(-2 pi i m / 16)
template <typename T>
__device__ __forceinline__ C2<T> w16(int m) {
  constexpr T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, r2 = (T)0.70710678118654752440;
  switch (m & 15) {
    case 0: return {1, 0};
    case 1: return {c1, -s1};
    case 2: return {r2, -r2};
    case 3: return {s1, -c1};
    case 4: return {0, -1};
    case 5: return {-s1, -c1};
    case 6: return {-r2, -r2};
    case 7: return {-c1, -s1};
    case 8: return {-1, 0};
    case 9: return {-c1, s1};
    case 10: return {-r2, r2};
    case 11: return {-s1, c1};
    case 12: return {0, 1};
    case 13: return {s1, c1};
    case 14: return {r2, r2};
    default: return {c1, s1};
  }
}

template <typename T>
__device__ __forceinline__ void dft4(C2<T> &a, C2<T> &b, C2<T> &c, C2<T> &d) {
  const C2<T> t0 = a + c, t1 = a - c, t2 = b + d, u = b - d;
  const C2<T> t3 = {u.y, -u.x};  // -i (b - d)
  a = t0 + t2;
  b = t1 + t3;
  c = t0 - t2;
  d = t1 - t3;
}

// In-register forward DFT of length R on v[0..R).
template <typename T, int R>
__device__ __forceinline__ void dft(C2<T> *v) {
  if constexpr (R == 2) {
    const C2<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    C2<T> y[2][4];
#pragma unroll
    for (int n2 = 0; n2 < 2; ++n2) {
      y[n2][0] = v[n2];
      y[n2][1] = v[2 + n2];
      y[n2][2] = v[4 + n2];
      y[n2][3] = v[6 + n2];
      dft4(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
    }
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) y[1][k1] = cmul(y[1][k1], w16<T>(2 * k1));
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      v[k1] = y[0][k1] + y[1][k1];
      v[k1 + 4] = y[0][k1] - y[1][k1];
    }
  } else {  // R == 16
    C2<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      y[n2][0] = v[n2];
      y[n2][1] = v[4 + n2];
      y[n2][2] = v[8 + n2];
      y[n2][3] = v[12 + n2];
      dft4(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
    }
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
      for (int k1 = 1; k1 < 4; ++k1) y[n2][k1] = cmul(y[n2][k1], w16<T>(n2 * k1));
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C2<T> a = y[0][k1], b = y[1][k1], c = y[2][k1], d = y[3][k1];
      dft4(a, b, c, d);
      v[k1] = a;
      v[k1 + 4] = b;
      v[k1 + 8] = c;
      v[k1 + 12] = d;
    }
  }
}

#ifndef KFBI_LDS_PAD_SHIFT
#define KFBI_LDS_PAD_SHIFT 4
#endif
#ifndef KFBI_LDS_PAIR_SKEW
#define KFBI_LDS_PAIR_SKEW 1
#endif
__device__ __forceinline__ int pad(int i) { return i + (i >> KFBI_LDS_PAD_SHIFT); }

// Barrier for the LDS exchanges inside one pencil pair.  The M / 16 threads of a pair are
// consecutive and M <= 1024, so a pair never straddles two wavefronts, and one wavefront's LDS
// operations are carried out in program order: a wavefront-scope fence, which only stops the
// compiler from moving LDS accesses across it, is enough.  Exchanges between pairs (the tile
// loads and stores) still need __syncthreads.
__device__ __forceinline__ void pair_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// W: tile-width multiplier picked by the autotuner (1 or 2 times the base pairs per workgroup)
template <typename T, int M, int W = 1>
struct Shape {
  static constexpr int N = M - 1;
  static constexpr int TPP = M / 16;                          // threads per pencil pair
  static_assert(TPP <= 64 && 64 % TPP == 0, "a pencil pair must lie inside one wavefront");
  static constexpr int NP = W * (sizeof(T) == 8 ? 2048 : 4096) / M;  // pencil pairs per workgroup
  static constexpr int NT = NP * TPP;                         // threads per workgroup (W x 128 / 256)
  static constexpr int PADM = M + (M >> KFBI_LDS_PAD_SHIFT) + KFBI_LDS_PAIR_SKEW;                  // padded LDS length of one pair (odd:
                                                              // pairs start on different banks)
};

// One Stockham stage of radix R after Ns points have been combined.
template <typename T, int M, int R, int Ns>
__device__ __forceinline__ void stage(C2<T> *buf, int lane, const C2<T> *__restrict__ tw) {
  constexpr int NB = 16 / R, MR = M / R, TPP = M / 16;
  C2<T> v[16];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + TPP * b;
    const int k = j & (Ns - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      C2<T> x = buf[pad(j + r * MR)];
      if (Ns > 1 && r > 0) x = cmul(x, tw[r * k * (M / (Ns * R))]);
      v[b * R + r] = x;
    }
    dft<T, R>(&v[b * R]);
  }
  pair_sync();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + TPP * b;
    const int k = j & (Ns - 1);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[pad(base + r * Ns)] = v[b * R + r];
  }
  pair_sync();
}

template <typename T, int M, int Ns>
__device__ __forceinline__ void fft_stages(C2<T> *buf, int lane, const C2<T> *tw) {
  constexpr int rem = M / Ns;
  if constexpr (rem > 16) {
    stage<T, M, 16, Ns>(buf, lane, tw);
    fft_stages<T, M, Ns * 16>(buf, lane, tw);
  } else {
    stage<T, M, rem, Ns>(buf, lane, tw);
  }
}

template <typename T>
__device__ __forceinline__ T shfl_up_w(T v, int d, int w) { return __shfl_up(v, d, w); }
template <typename T>
__device__ __forceinline__ T shfl_w(T v, int s, int w) { return __shfl(v, s, w); }

// Mode hook that leaves the values alone.
template <typename T>
struct NoHook {
  __device__ __forceinline__ void operator()(int, C2<T> &) const {}
};

// s_n = sin(pi n / M) at the positions n = 1 + lane + (M/16) i, i < 8, that one thread's
// pre-processing combines, from a table in global memory or LDS.  Kernels load them from
// memory with their tile, so that the pre-processing, which follows a barrier, does not wait
// on memory (the last-axis pass reads them from an LDS copy instead, to hold no registers
// across its forward transform).
template <typename T, int M>
struct Sines {
  T s[8];
  __device__ __forceinline__ Sines(const T *sp, int lane) {
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = sp[1 + lane + (M / 16) * i];
  }
};

// Pre-processing t_n = s_n (x_n + x_{M-n}) + (x_n - x_{M-n})/2: (n, M-n) pairs are owned by one
// thread, so no barrier inside; the hook sees every input value (position m = 1..N) as it is
// read.
template <typename T, int M, typename Hook>
__device__ __forceinline__ void dst_pre(C2<T> *buf, int lane, const Sines<T, M> &sn, const Hook &hook) {
  constexpr int TPP = M / 16;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int n = 1 + lane + TPP * i;
    C2<T> a = buf[pad(n)], b = buf[pad(M - n)];
    hook(n, a);
    hook(M - n, b);
    const T s = sn.s[i];
    const C2<T> sum = s * (a + b), dif = (T)0.5 * (a - b);
    buf[pad(n)] = sum + dif;
    buf[pad(M - n)] = sum - dif;
  }
  if (lane == 0) buf[pad(0)] = {0, 0};
}

// Post-processing of the FFT of a pre-processed pencil pair held in buf (prefix scan over the odd
// outputs): lane owns k in [8 lane, 8 lane + 8), so its outputs are the DST values at positions
// 16 lane + q, q < 16, returned in y[q] (y[0] of lane 0, position 0, is not an output: zero).
template <typename T, int M>
__device__ __forceinline__ void dst_post(const C2<T> *buf, int lane, C2<T> (&y)[16]) {
  constexpr int TPP = M / 16;
  C2<T> ev[8], od[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = 8 * lane + i;
    const C2<T> zk = buf[pad(k)], zm = buf[pad((M - k) & (M - 1))];
    ev[i] = {(T)0.5 * (zm.y - zk.y), (T)0.5 * (zk.x - zm.x)};
    od[i] = {(T)0.5 * (zk.x + zm.x), (T)0.5 * (zk.y + zm.y)};
  }
  const C2<T> e0 = od[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) od[i] = od[i] + od[i - 1];
  const C2<T> tot = od[7];
  C2<T> inc = tot;
#pragma unroll
  for (int off = 1; off < TPP; off <<= 1) {
    const C2<T> u = {shfl_up_w(inc.x, off, TPP), shfl_up_w(inc.y, off, TPP)};
    if (lane >= off) inc = inc + u;
  }
  const C2<T> excl = inc - tot;
  const C2<T> E0 = {shfl_w(e0.x, 0, TPP), shfl_w(e0.y, 0, TPP)};
  const C2<T> half0 = (T)0.5 * E0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    y[2 * i] = (i > 0 || lane > 0) ? ev[i] : C2<T>{T(0), T(0)};
    y[2 * i + 1] = (excl + od[i]) - half0;
  }
}

// The FFT of the pre-processed pencil pair and the post-processing; result at positions 1..N.
// All threads of the workgroup must call it.  BLOCK: end with a workgroup barrier (the caller
// reads other pairs' results next) rather than a pair one.
template <typename T, int M, bool BLOCK = true>
__device__ __forceinline__ void dst_rest(C2<T> *buf, int lane, const C2<T> *__restrict__ tw) {
  fft_stages<T, M, 1>(buf, lane, tw);
  C2<T> y[16];
  dst_post<T, M>(buf, lane, y);
  pair_sync();
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (q > 0 || lane > 0) buf[pad(16 * lane + q)] = y[q];
  if constexpr (BLOCK) __syncthreads();
  else pair_sync();
}

// DST-I (unnormalised: y_k = sum_n x_n sin(pi n k / M)) of one pencil pair held in LDS as
// complex values at positions 1..N; result at the same positions.  All threads of the
// workgroup must call it (it contains barriers).
template <typename T, int M, typename Hook = NoHook<T>>
__device__ __forceinline__ void dst_pair(C2<T> *buf, int lane, const C2<T> *__restrict__ tw,
                                         const Sines<T, M> &sn, const Hook &hook = Hook()) {
  dst_pre<T, M>(buf, lane, sn, hook);
  pair_sync();
  dst_rest<T, M>(buf, lane, tw);
}

template <typename T>
__device__ __forceinline__ T &lane_of(C2<T> &c, int which) {
  return which ? c.y : c.x;
}

// 16-byte vector of T for wide global loads / stores
template <typename T>
struct alignas(16) V16 {
  T v[16 / sizeof(T)];
};

// ---------------------------------------------------------------- pass kernels
//
// Every pass stages its whole tile through registers: all global loads of the tile are in
// flight before the first LDS write, and all LDS reads of the result precede the global
// stores.  Padded fields are accessed with 16-byte vectors; the pad column (x = N) is kept
// at zero so that the y and z passes may carry it along.

// DST along contiguous rows: pairs of consecutive rows of the flattened [comp][..][x] list.
// PIN / POUT: input / output in the padded layout (row pitch M) instead of pitch N.
// One tile (2 NP rows, tile index blk) in the LDS buffer sbuf of NP * PADM values.
template <typename T, int M, bool PIN, bool POUT, int W = 1>
__device__ __forceinline__ void dst_x_tile(const T *__restrict__ in, T *__restrict__ out, int64_t nrows,
                                           const C2<T> *__restrict__ tw, const T *__restrict__ sp, C2<T> *sbuf,
                                           int64_t blk) {
  using Sh = Shape<T, M, W>;
  constexpr int N = Sh::N, NP = Sh::NP, NT = Sh::NT, PADM = Sh::PADM, VW = 16 / sizeof(T);
  constexpr int ROWS = 2 * NP;
  const int tid = threadIdx.x;
  const int64_t r0 = blk * ROWS;
  const Sines<T, M> sn(sp, tid % Sh::TPP);
  if constexpr (M >= 64) {
    // one pencil pair per wave at a time; a lane moves whole complex values (two 8-byte row
    // elements per 16-byte LDS word, unit stride: no LDS bank conflicts)
    constexpr int NWV = NT / 64, PPW = NP / NWV, KS = M / 64;
    constexpr int64_t PI = PIN ? M : N, PO = POUT ? M : N;
    const int wv = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    C2<T> v[PPW][KS];
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp) {
      const int64_t rowa = r0 + 2 * (wv + NWV * pp);
      const bool oka = rowa < nrows, okb = rowa + 1 < nrows;
      const T *ra = in + rowa * PI, *rb = ra + PI;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int n = lane + 64 * k;
        v[pp][k] = {oka && n < N ? ra[n] : T(0), okb && n < N ? rb[n] : T(0)};
      }
    }
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp)
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int n = lane + 64 * k;
        if (n < N) sbuf[(wv + NWV * pp) * PADM + pad(n + 1)] = v[pp][k];
      }
    __syncthreads();
    dst_pair<T, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, tw, sn);
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp) {
      const int rr = wv + NWV * pp;
      const int64_t rowa = r0 + 2 * rr;
      const bool oka = rowa < nrows, okb = rowa + 1 < nrows;
      T *oa = out + rowa * PO, *ob = oa + PO;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int n = lane + 64 * k;   // n = N: the pad column of the padded layout, zero
        if (POUT || n < N) {
          const C2<T> c = n < N ? sbuf[rr * PADM + pad(n + 1)] : C2<T>{T(0), T(0)};
          if (oka) oa[n] = c.x;
          if (okb) ob[n] = c.y;
        }
      }
    }
  } else {
    if constexpr (PIN) {
      constexpr int VPR = M / VW, NV = ROWS * VPR, PER = (NV + NT - 1) / NT;
      V16<T> reg[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int rr = e / VPR, s = e - rr * VPR;
        const int64_t row = r0 + rr;
        if (e < NV && row < nrows)
          reg[i] = *reinterpret_cast<const V16<T> *>(in + row * M + s * VW);
        else
#pragma unroll
          for (int j = 0; j < VW; ++j) reg[i].v[j] = T(0);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        if (e < NV) {
          const int rr = e / VPR, s = e - rr * VPR;
#pragma unroll
          for (int j = 0; j < VW; ++j) {
            const int n = s * VW + j;
            if (n < N) lane_of(sbuf[(rr >> 1) * PADM + pad(n + 1)], rr & 1) = reg[i].v[j];
          }
        }
      }
    } else {
      constexpr int NE = ROWS * N, PER = (NE + NT - 1) / NT;
      T reg[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int rr = e / N, n = e - rr * N;
        const int64_t row = r0 + rr;
        reg[i] = (e < NE && row < nrows) ? in[row * N + n] : T(0);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        if (e < NE) {
          const int rr = e / N, n = e - rr * N;
          lane_of(sbuf[(rr >> 1) * PADM + pad(n + 1)], rr & 1) = reg[i];
        }
      }
    }
    __syncthreads();
    dst_pair<T, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, tw, sn);
    if constexpr (POUT) {
      constexpr int VPR = M / VW, NV = ROWS * VPR, PER = (NV + NT - 1) / NT;
      V16<T> reg[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int rr = e / VPR, s = e - rr * VPR;
#pragma unroll
        for (int j = 0; j < VW; ++j) {
          const int n = s * VW + j;
          reg[i].v[j] = (e < NV && n < N) ? lane_of(sbuf[(rr >> 1) * PADM + pad(n + 1)], rr & 1) : T(0);
        }
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int rr = e / VPR, s = e - rr * VPR;
        const int64_t row = r0 + rr;
        if (e < NV && row < nrows) *reinterpret_cast<V16<T> *>(out + row * M + s * VW) = reg[i];
      }
    } else {
      constexpr int NE = ROWS * N, PER = (NE + NT - 1) / NT;
      T reg[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int rr = e / N, n = e - rr * N;
        reg[i] = e < NE ? lane_of(sbuf[(rr >> 1) * PADM + pad(n + 1)], rr & 1) : T(0);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int rr = e / N, n = e - rr * N;
        const int64_t row = r0 + rr;
        if (e < NE && row < nrows) out[row * N + n] = reg[i];
      }
    }
  }
}

template <typename T, int M, bool PIN, bool POUT, int W = 1>
__global__ __launch_bounds__((Shape<T, M, W>::NT)) void k_dst_x(const T *__restrict__ in, T *__restrict__ out,
                                                             int64_t nrows, const C2<T> *__restrict__ tw,
                                                             const T *__restrict__ sp) {
  using Sh = Shape<T, M, W>;
  __shared__ C2<T> sbuf[Sh::NP * Sh::PADM];
  dst_x_tile<T, M, PIN, POUT, W>(in, out, nrows, tw, sp, sbuf, blockIdx.x);
}

// Row predicates of the strided tile mover: every row; rows in a bit set read once from memory
// (a uniform address: scalar loads; null means every row); rows in a bit set passed as a
// kernel argument.  Bits avoid a memory load per row ahead of the tile's data loads.
struct AllRows {
  __device__ bool operator()(int) const { return true; }
};
template <int NW>
struct BitRowsMem {
  uint64_t w[NW];
  __device__ explicit BitRowsMem(const uint64_t *__restrict__ p) {
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = p ? p[i] : ~uint64_t(0);
  }
  __device__ bool operator()(int r) const {
    uint64_t x = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) x = (r >> 6) == i ? w[i] : x;
    return (x >> (r & 63)) & 1;
  }
};
template <int NW>
struct BitRows {
  const PlaneBits &b;
  __device__ bool operator()(int r) const {
    uint64_t x = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) x = (r >> 6) == i ? b.w[i] : x;
    return (x >> (r & 63)) & 1;
  }
};

// Tile mover for the strided passes: a tile is NR rows (stride RS elements) of TX consecutive
// columns starting at column x0, for NC components (stride CS); element (row r, column xo,
// component c) lives at LDS pair PAIR(xo, c), lane LANE(xo, c), position r + 1.
template <typename T, int M, int TX, int NC, int W = 1>
struct StridedTile {
  using Sh = Shape<T, M, W>;
  static constexpr int N = Sh::N, NT = Sh::NT, PADM = Sh::PADM, VW = 16 / sizeof(T);
  static constexpr bool VEC = (TX % VW == 0) && (TX <= M);
  static constexpr int NE = VEC ? N * NC * (TX / VW) : N * NC * TX;
  static constexpr int PER = (NE + NT - 1) / NT;
  __device__ static int pair_of(int xo, int c) { return NC == 2 ? xo : (xo >> 1); }
  __device__ static int lane_sel(int xo, int c) { return NC == 2 ? c : (xo & 1); }

  // rows: rows r with rows(r) false are known to be zero and are not read.
  // Vector path: NC = 1 pairs adjacent columns, so the elements of a 16-byte vector form whole
  // complex LDS words; NC = 2 loads both components of the same columns in one thread.
  template <typename R = AllRows>
  __device__ static void load(const T *__restrict__ base, int64_t RS, int64_t CS, int x0, C2<T> *sbuf, int tid,
                              const R &rows = R()) {
    if constexpr (VEC) {
      constexpr int VPR = TX / VW, NU = N * VPR, PU = (NU + NT - 1) / NT;
      V16<T> reg[PU][NC];
#pragma unroll
      for (int i = 0; i < PU; ++i) {
        const int e = tid + i * NT;
        const int s = e % VPR, r = e / VPR;
        const bool ok = e < NU && rows(r);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (ok)
            reg[i][c] = *reinterpret_cast<const V16<T> *>(base + c * CS + (int64_t)r * RS + x0 + s * VW);
          else
#pragma unroll
            for (int j = 0; j < VW; ++j) reg[i][c].v[j] = T(0);
        }
      }
#pragma unroll
      for (int i = 0; i < PU; ++i) {
        const int e = tid + i * NT;
        if (e < NU) {
          const int s = e % VPR, r = e / VPR;
          if constexpr (NC == 2) {
#pragma unroll
            for (int j = 0; j < VW; ++j) sbuf[(s * VW + j) * PADM + pad(r + 1)] = {reg[i][0].v[j], reg[i][1].v[j]};
          } else {
#pragma unroll
            for (int j = 0; j < VW / 2; ++j)
              sbuf[(s * (VW / 2) + j) * PADM + pad(r + 1)] = {reg[i][0].v[2 * j], reg[i][0].v[2 * j + 1]};
          }
        }
      }
    } else {
      T reg[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int xo = e % TX, rc = e / TX, c = rc % NC, r = rc / NC;
        reg[i] = (e < NE && x0 + xo < N && rows(r)) ? base[c * CS + (int64_t)r * RS + x0 + xo] : T(0);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        if (e < NE) {
          const int xo = e % TX, rc = e / TX, c = rc % NC, r = rc / NC;
          lane_of(sbuf[pair_of(xo, c) * PADM + pad(r + 1)], lane_sel(xo, c)) = reg[i];
        }
      }
    }
  }

  // load() followed by the DST pre-processing of every pencil pair of the tile (dst_pre), the
  // two fused: a thread loads rows r and N-1-r (positions n and M-n) of its columns and writes
  // t_n and t_{M-n} straight into LDS, which saves one LDS round trip of the tile.  The same
  // arithmetic as load(), barrier, dst_pre.  A barrier must follow before the transform.
  // ANTI (NC = 2): only component 0 is read; component 1 is taken as its negative.  ADD2 (with
  // ANTI): the pair read from base2 (both components, on the rows flagged by rows2) is added.
  template <bool ANTI = false, bool ADD2 = false, typename R = AllRows, typename R2 = AllRows>
  __device__ static void load_pre(const T *__restrict__ base, int64_t RS, int64_t CS, int x0, C2<T> *sbuf, int tid,
                                  const T *__restrict__ sp, const R &rows = R(),
                                  const T *__restrict__ base2 = nullptr, const R2 &rows2 = R2()) {
    static_assert(!ANTI || (NC == 2 && VEC), "an antisymmetric pair is read as two components");
    static_assert(!ADD2 || ANTI, "the second input is added to an antisymmetric pair");
    if constexpr (!VEC) {
      load(base, RS, CS, x0, sbuf, tid, rows);
      __syncthreads();
      dst_pre<T, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, Sines<T, M>(sp, tid % Sh::TPP), NoHook<T>());
    } else {
      constexpr int VPR = TX / VW, NPR = M / 2, NU = NPR * VPR, PU = (NU + NT - 1) / NT;
      V16<T> ra[PU][NC], rb[PU][NC];
      V16<T> sa[ADD2 ? PU : 1][2], sb[ADD2 ? PU : 1][2];
#pragma unroll
      for (int i = 0; i < PU; ++i) {
        const int e = tid + i * NT;
        const int s = e % VPR, p = e / VPR, r0 = p, r1 = N - 1 - p;
        const bool ok0 = e < NU && rows(r0), ok1 = e < NU && rows(r1);
        if constexpr (ADD2) {
          const bool o20 = e < NU && rows2(r0), o21 = e < NU && rows2(r1);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const T *q2 = base2 + c * CS + x0 + s * VW;
            if (o20) sa[i][c] = *reinterpret_cast<const V16<T> *>(q2 + (int64_t)r0 * RS);
            else
#pragma unroll
              for (int j = 0; j < VW; ++j) sa[i][c].v[j] = T(0);
            if (o21) sb[i][c] = *reinterpret_cast<const V16<T> *>(q2 + (int64_t)r1 * RS);
            else
#pragma unroll
              for (int j = 0; j < VW; ++j) sb[i][c].v[j] = T(0);
          }
        }
#pragma unroll
        for (int c = 0; c < (ANTI ? 1 : NC); ++c) {
          const T *q = base + c * CS + x0 + s * VW;
          if (ok0) ra[i][c] = *reinterpret_cast<const V16<T> *>(q + (int64_t)r0 * RS);
          else
#pragma unroll
            for (int j = 0; j < VW; ++j) ra[i][c].v[j] = T(0);
          if (ok1) rb[i][c] = *reinterpret_cast<const V16<T> *>(q + (int64_t)r1 * RS);
          else
#pragma unroll
            for (int j = 0; j < VW; ++j) rb[i][c].v[j] = T(0);
        }
      }
#pragma unroll
      for (int i = 0; i < PU; ++i) {
        const int e = tid + i * NT;
        if (e < NU) {
          const int s = e % VPR, p = e / VPR, n = p + 1;
          const T sn = sp[n];
          constexpr int NW = NC == 2 ? VW : VW / 2;     // complex LDS words per 16-byte vector
#pragma unroll
          for (int j = 0; j < NW; ++j) {
            C2<T> a, b;
            if constexpr (ADD2) {
              a = {ra[i][0].v[j] + sa[i][0].v[j], -ra[i][0].v[j] + sa[i][1].v[j]};
              b = {rb[i][0].v[j] + sb[i][0].v[j], -rb[i][0].v[j] + sb[i][1].v[j]};
            } else if constexpr (ANTI) {
              a = {ra[i][0].v[j], -ra[i][0].v[j]};
              b = {rb[i][0].v[j], -rb[i][0].v[j]};
            } else if constexpr (NC == 2) {
              a = {ra[i][0].v[j], ra[i][1].v[j]};
              b = {rb[i][0].v[j], rb[i][1].v[j]};
            } else {
              a = {ra[i][0].v[2 * j], ra[i][0].v[2 * j + 1]};
              b = {rb[i][0].v[2 * j], rb[i][0].v[2 * j + 1]};
            }
            const C2<T> sum = sn * (a + b), dif = (T)0.5 * (a - b);
            C2<T> *col = sbuf + (s * NW + j) * PADM;
            col[pad(n)] = sum + dif;
            col[pad(M - n)] = sum - dif;
            if (p == 0) col[pad(0)] = {0, 0};
          }
        }
      }
    }
  }

  // rows: only rows r with rows(r) true are written.  DIFF (NC = 2): only the difference
  // component 0 - component 1 is written, into component 0.
  template <bool DIFF = false, typename R = AllRows>
  __device__ static void store(T *__restrict__ base, int64_t RS, int64_t CS, int x0, C2<T> *sbuf, int tid,
                               const R &rows = R()) {
    static_assert(!DIFF || (NC == 2 && VEC), "a difference is stored from a pair of components");
    if constexpr (VEC) {
      constexpr int VPR = TX / VW, NU = N * VPR, PU = (NU + NT - 1) / NT;
      V16<T> reg[PU][NC];
#pragma unroll
      for (int i = 0; i < PU; ++i) {
        const int e = tid + i * NT;
        const int s = e % VPR, r = e / VPR;
        if (e < NU) {
          if constexpr (DIFF) {
#pragma unroll
            for (int j = 0; j < VW; ++j) {
              const C2<T> v = sbuf[(s * VW + j) * PADM + pad(r + 1)];
              reg[i][0].v[j] = x0 + s * VW + j < N ? v.x - v.y : T(0);
            }
          } else if constexpr (NC == 2) {
#pragma unroll
            for (int j = 0; j < VW; ++j) {
              const C2<T> v = sbuf[(s * VW + j) * PADM + pad(r + 1)];
              const bool live = x0 + s * VW + j < N;
              reg[i][0].v[j] = live ? v.x : T(0);
              reg[i][1].v[j] = live ? v.y : T(0);
            }
          } else {
#pragma unroll
            for (int j = 0; j < VW / 2; ++j) {
              const C2<T> v = sbuf[(s * (VW / 2) + j) * PADM + pad(r + 1)];
              reg[i][0].v[2 * j] = x0 + s * VW + 2 * j < N ? v.x : T(0);
              reg[i][0].v[2 * j + 1] = x0 + s * VW + 2 * j + 1 < N ? v.y : T(0);
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < PU; ++i) {
        const int e = tid + i * NT;
        const int s = e % VPR, r = e / VPR;
        if (e < NU && rows(r))
#pragma unroll
          for (int c = 0; c < (DIFF ? 1 : NC); ++c)
            *reinterpret_cast<V16<T> *>(base + c * CS + (int64_t)r * RS + x0 + s * VW) = reg[i][c];
      }
    } else {
      T reg[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int xo = e % TX, rc = e / TX, c = rc % NC, r = rc / NC;
        reg[i] = e < NE ? lane_of(sbuf[pair_of(xo, c) * PADM + pad(r + 1)], lane_sel(xo, c)) : T(0);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int xo = e % TX, rc = e / TX, c = rc % NC, r = rc / NC;
        if (e < NE && x0 + xo < N && rows(r)) base[c * CS + (int64_t)r * RS + x0 + xo] = reg[i];
      }
    }
  }
};

// DST along y (3D): tile = 2 NP consecutive x columns of one (comp, z) plane.  in and out
// may alias.  mask_in / mask_out (optional, [z][16] bit rows, bit y of plane z): rows known to
// be zero on input are not read; only rows flagged on output are written.  planes (optional, [z] bytes): planes
// flagged 0 are skipped altogether (no reads, no writes).
template <typename T, int M, int W = 1>
__global__ __launch_bounds__((Shape<T, M, W>::NT)) void k_dst_y(const T *__restrict__ in, T *__restrict__ out,
                                                               int64_t P, int64_t comp_stride,
                                                               const uint64_t *__restrict__ mask_in,
                                                               const uint64_t *__restrict__ mask_out,
                                                               const uint8_t *__restrict__ planes,
                                                               const C2<T> *__restrict__ tw, const T *__restrict__ sp) {
  using Sh = Shape<T, M, W>;
  using Tl = StridedTile<T, M, 2 * Sh::NP, 1, W>;
  __shared__ C2<T> sbuf[Sh::NP * Sh::PADM];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * 2 * Sh::NP, z = blockIdx.y, c = blockIdx.z;
  const int64_t off = c * comp_stride + (int64_t)z * Sh::N * P;
  if (planes && !planes[z]) return;   // nothing to read or write in this plane (whole workgroup)
  constexpr int NW = (Sh::N + 63) / 64;
  const Sines<T, M> sn(sp, tid % Sh::TPP);
  Tl::load(in + off, P, 0, x0, sbuf, tid, BitRowsMem<NW>(mask_in ? mask_in + (int64_t)z * 16 : nullptr));
  __syncthreads();
  dst_pair<T, M>(sbuf + (tid / Sh::TPP) * Sh::PADM, tid % Sh::TPP, tw, sn);
  Tl::store(out + off, P, 0, x0, sbuf, tid, BitRowsMem<NW>(mask_out ? mask_out + (int64_t)z * 16 : nullptr));
}

using ModeScale = ModeParams;

// Mode solve applied to each value as the inverse transform reads it (position m = mode index
// along the last axis): u^ = f^ / (L + kappa), or the closed-form inverse of the coupled 2x2,
// with the mode sums L = b + dz lambda_m (b: the other axes' part, fixed per pencil).
template <typename T, int NC>
struct ModeHook {
  const T *slam;
  T b0, b1, dz0, dz1, kap, nrm;   // NC = 2: components 0 / 1 of one column; NC = 1: columns a / b
  __device__ __forceinline__ void operator()(int m, C2<T> &v) const {
    const T lz = slam[m - 1];
    if (NC == 2) {
      const T ai = b0 + dz0 * lz, ae = b1 + dz1 * lz;
      const T s = nrm * recip(ai * ae + kap * (ai + ae));
      const T fi = v.x, fe = v.y;
      v.x = s * ((ae + kap) * fi + kap * fe);
      v.y = s * (kap * fi + (ai + kap) * fe);
    } else {
      v.x *= nrm * recip(b0 + dz0 * lz + kap);
      v.y *= nrm * recip(b1 + dz0 * lz + kap);
    }
  }
};

// Last axis (z in 3D, y in 2D), fused: forward DST -> mode solve -> inverse DST, from ain to a
// (which may alias).
// The mode solve is u^ = f^ / (D L + kappa) (one component) or the closed-form inverse of
// [[a_i + kappa, -kappa], [-kappa, a_e + kappa]], a_c = D_c L (coupled pair), with
// L = lambda_kx + lambda_ky (+ lambda_kz) and norm = (2/M)^d for the inverse transforms.
// ncomp = 2: a pencil pair is (comp 0, comp 1) of one column; ncomp = 1: two adjacent columns.
// In 2D, blockIdx.y may index the problems of a batch of equal-size fields at stride pstride,
// each with its own mode parameters msv[problem] (msv = nullptr: one problem, parameters ms).
// ZM (3D): plane-masked forms, kernels of their own so that traces tell them apart.  ZM = 1:
// the bit sets zin / zout name the planes that may be nonzero on input (the others are not
// read) and the planes needed on output (the others are not written); ZM = 2: every plane is
// read, only the planes in zout are written; ZM = 3 (coupled pair): as ZM = 2 for an
// antisymmetric source, component 1 of the input being minus component 0, so that only
// component 0 is read (the input may then hold one component); ZM = 4 (coupled pair): every
// plane read, and only the difference component 0 - component 1 written, into component 0 (the
// final solve of a step whose potentials are not returned needs only Phi_i - Phi_e); ZM = 5
// (coupled pair): as ZM = 4 for an input that is the antisymmetric pair (g, -g) of ain's
// component 0 plus the pair read from ain2 on the planes in zin.
// One tile of the pass: tile number id of total (gx tiles per row of the grid of tiles), LDS
// buffers sbuf (NP * PADM values), slam (M) and ssin (M / 2 + 1).
template <typename T, int M, int NC, int DIM, int W = 1, int ZM = 0>
__device__ __forceinline__ void dst_last_tile(const T *__restrict__ ain, T *__restrict__ a, int64_t P,
                                              int64_t comp_stride, const ModeScale &ms0,
                                              const C2<T> *__restrict__ tw, const T *__restrict__ sp,
                                              const ModeScale *__restrict__ msv, int64_t pstride,
                                              const PlaneBits &zin, const PlaneBits &zout, C2<T> *sbuf, T *slam,
                                              T *ssin, int64_t id, int64_t total, int gx,
                                              const T *__restrict__ ain2 = nullptr) {
  using Sh = Shape<T, M, W>;
  constexpr int N = Sh::N, NP = Sh::NP, NT = Sh::NT, PADM = Sh::PADM;
  constexpr int TX = NC == 2 ? NP : 2 * NP;          // columns per tile
  constexpr int64_t LS = DIM == 3 ? (int64_t)N : 1;  // rows of the last axis step by LS * P
  using Tl = StridedTile<T, M, TX, NC, W>;
  const int tid = threadIdx.x;
  // At W = 1 a tile row of TX columns is half of a 128-byte line; the tile sharing the line is
  // given to the workgroup dispatched 8 later, i.e. on the same XCD (round-robin dispatch), so
  // the second half of the line comes from that XCD's L2 instead of a second HBM fetch.
  if (id < (total & ~int64_t(15))) id = (id & ~int64_t(15)) + 2 * (id & 7) + ((id >> 3) & 1);
  const int bx = (int)(id % gx), by = (int)(id / gx);
  const int x0 = bx * TX, y = DIM == 3 ? by : 0;
  const int64_t boff = DIM == 3 ? (int64_t)y * P : (int64_t)by * pstride;
  T *base = a + boff;
  const ModeScale ms = (DIM == 2 && msv) ? msv[by] : ms0;
  for (int i = tid; i < N; i += NT) slam[i] = (T)ms.lam[i];
  for (int i = tid; i <= M / 2; i += NT) ssin[i] = sp[i];
  constexpr int NW = (N + 63) / 64;
  static_assert(ZM < 3 || (NC == 2 && DIM == 3), "the ZM = 3, 4, 5 z passes are for the coupled 3D pair");
  if constexpr (ZM == 1) Tl::load_pre(ain + boff, LS * P, comp_stride, x0, sbuf, tid, sp, BitRows<NW>{zin});
  else if constexpr (ZM == 3) Tl::template load_pre<true>(ain + boff, LS * P, comp_stride, x0, sbuf, tid, sp);
  else if constexpr (ZM == 5)
    Tl::template load_pre<true, true>(ain + boff, LS * P, comp_stride, x0, sbuf, tid, sp, AllRows{}, ain2 + boff,
                                      BitRows<NW>{zin});
  else Tl::load_pre(ain + boff, LS * P, comp_stride, x0, sbuf, tid, sp);
  __syncthreads();
  const int pr = tid / Sh::TPP, lane = tid % Sh::TPP;
  C2<T> *mine = sbuf + pr * PADM;
  dst_rest<T, M, false>(mine, lane, tw);
  // inverse transform with the mode solve applied as it reads the spectrum
  ModeHook<T, NC> mh;
  mh.slam = slam;
  {
    const T ly = DIM == 3 ? slam[y] : T(0);
    const int last = DIM - 1;
    if (NC == 2) {
      const int x = x0 + pr;
      const T lx = x < N ? slam[x] : T(0);
      mh.b0 = (T)ms.D0[0] * lx + (DIM == 3 ? (T)ms.D0[1] * ly : T(0));
      mh.b1 = (T)ms.D1[0] * lx + (DIM == 3 ? (T)ms.D1[1] * ly : T(0));
      mh.dz0 = (T)ms.D0[last];
      mh.dz1 = (T)ms.D1[last];
    } else {
      const int xa = x0 + 2 * pr, xb = xa + 1;
      const T la = xa < N ? slam[xa] : T(0), lb = xb < N ? slam[xb] : T(0);
      const T yy = DIM == 3 ? (T)ms.D0[1] * ly : T(0);
      mh.b0 = (T)ms.D0[0] * la + yy;
      mh.b1 = (T)ms.D0[0] * lb + yy;
      mh.dz0 = mh.dz1 = (T)ms.D0[last];
    }
  }
  mh.kap = (T)ms.kappa;
  mh.nrm = (T)ms.norm;
  dst_pair<T, M>(mine, lane, tw, Sines<T, M>(ssin, lane), mh);
  if constexpr (ZM == 4 || ZM == 5) Tl::template store<true>(base, LS * P, comp_stride, x0, sbuf, tid);
  else if constexpr (ZM != 0) Tl::store(base, LS * P, comp_stride, x0, sbuf, tid, BitRows<NW>{zout});
  else Tl::store(base, LS * P, comp_stride, x0, sbuf, tid);
}

template <typename T, int M, int NC, int DIM, int W = 1, int ZM = 0>
__global__ __launch_bounds__((Shape<T, M, W>::NT)) void k_dst_last(const T *__restrict__ ain, T *__restrict__ a,
                                                                     int64_t P, int64_t comp_stride,
                                                                  ModeScale ms0, const C2<T> *__restrict__ tw,
                                                                  const T *__restrict__ sp,
                                                                  const ModeScale *__restrict__ msv = nullptr,
                                                                  int64_t pstride = 0, PlaneBits zin = {},
                                                                  PlaneBits zout = {},
                                                                  const T *__restrict__ ain2 = nullptr) {
  using Sh = Shape<T, M, W>;
  __shared__ C2<T> sbuf[Sh::NP * Sh::PADM];
  __shared__ T slam[M];
  __shared__ T ssin[M / 2 + 1];
  dst_last_tile<T, M, NC, DIM, W, ZM>(ain, a, P, comp_stride, ms0, tw, sp, msv, pstride, zin, zout, sbuf, slam, ssin,
                                      blockIdx.x + (int64_t)gridDim.x * blockIdx.y,
                                      (int64_t)gridDim.x * gridDim.y, (int)gridDim.x, ain2);
}

// DST along contiguous rows listed in `rows` (indices into the flattened [comp][..] row list),
// padded layout in and out; used by the sparse passes of the matrix-vector product.
template <typename T, int M>
__global__ __launch_bounds__((Shape<T, M>::NT)) void k_dst_x_rows(const T *__restrict__ in, T *__restrict__ out,
                                                                    const int32_t *__restrict__ rows, int64_t nlist,
                                                                    const C2<T> *__restrict__ tw,
                                                                    const T *__restrict__ sp) {
  using Sh = Shape<T, M>;
  constexpr int N = Sh::N, NP = Sh::NP, NT = Sh::NT, PADM = Sh::PADM, VW = 16 / sizeof(T);
  constexpr int ROWS = 2 * NP, VPR = M / VW, NV = ROWS * VPR, PER = (NV + NT - 1) / NT;
  __shared__ C2<T> sbuf[NP * PADM];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * ROWS;
  // the tile's row indices through uniform (scalar) loads, then picked per thread from
  // registers: no data load waits on a per-thread index load
  int32_t ri[ROWS];
#pragma unroll
  for (int k = 0; k < ROWS; ++k) ri[k] = r0 + k < nlist ? rows[r0 + k] : 0;
  auto row_of = [&](int rr) {
    int32_t v = 0;
#pragma unroll
    for (int k = 0; k < ROWS; ++k) v = rr == k ? ri[k] : v;
    return v;
  };
  const Sines<T, M> sn(sp, tid % Sh::TPP);
  if constexpr (M >= 64) {
    // one pencil pair per wave at a time (pair index uniform in the wave, so its two rows are
    // picked by scalar selects); a lane moves whole complex values: two 8-byte row elements
    // per 16-byte LDS word, unit stride, no bank conflicts
    constexpr int NWV = NT / 64, PPW = NP / NWV, KS = M / 64;
    const int wv = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    C2<T> v[PPW][KS];
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp) {
      const int rr = wv + NWV * pp;
      const bool oka = r0 + 2 * rr < nlist, okb = r0 + 2 * rr + 1 < nlist;
      const T *ra = in + (int64_t)row_of(2 * rr) * M, *rb = in + (int64_t)row_of(2 * rr + 1) * M;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int n = lane + 64 * k;
        v[pp][k] = {oka && n < N ? ra[n] : T(0), okb && n < N ? rb[n] : T(0)};
      }
    }
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp)
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int n = lane + 64 * k;
        if (n < N) sbuf[(wv + NWV * pp) * PADM + pad(n + 1)] = v[pp][k];
      }
    __syncthreads();
    dst_pair<T, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, tw, sn);
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp) {
      const int rr = wv + NWV * pp;
      const bool oka = r0 + 2 * rr < nlist, okb = r0 + 2 * rr + 1 < nlist;
      T *ra = out + (int64_t)row_of(2 * rr) * M, *rb = out + (int64_t)row_of(2 * rr + 1) * M;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int n = lane + 64 * k;   // n = N is the pad column: written as zero
        const C2<T> c = n < N ? sbuf[rr * PADM + pad(n + 1)] : C2<T>{T(0), T(0)};
        if (oka) ra[n] = c.x;
        if (okb) rb[n] = c.y;
      }
    }
  } else {
    V16<T> reg[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      const int rr = e / VPR, s = e - rr * VPR;
      if (e < NV && r0 + rr < nlist)
        reg[i] = *reinterpret_cast<const V16<T> *>(in + (int64_t)row_of(rr) * M + s * VW);
      else
#pragma unroll
        for (int j = 0; j < VW; ++j) reg[i].v[j] = T(0);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      if (e < NV) {
        const int rr = e / VPR, s = e - rr * VPR;
#pragma unroll
        for (int j = 0; j < VW; ++j) {
          const int n = s * VW + j;
          if (n < N) lane_of(sbuf[(rr >> 1) * PADM + pad(n + 1)], rr & 1) = reg[i].v[j];
        }
      }
    }
    __syncthreads();
    dst_pair<T, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, tw, sn);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      const int rr = e / VPR, s = e - rr * VPR;
#pragma unroll
      for (int j = 0; j < VW; ++j) {
        const int n = s * VW + j;
        reg[i].v[j] = (e < NV && n < N) ? lane_of(sbuf[(rr >> 1) * PADM + pad(n + 1)], rr & 1) : T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      const int rr = e / VPR, s = e - rr * VPR;
      if (e < NV && r0 + rr < nlist) *reinterpret_cast<V16<T> *>(out + (int64_t)row_of(rr) * M + s * VW) = reg[i];
    }
  }
}

// ---------------------------------------------------------------- bidomain x passes
//
// The x passes of a coupled bidomain step pair row r of component 0 with row r of component 1
// (instead of two rows of one component), so that the two potentials of a node share one
// complex value in LDS.  The reaction half steps of the splitting are pointwise, so they ride
// in these passes instead of separate sweeps over the box:
//   FHN_FE   source f = (kappa V1, -kappa V1 + beta I) of the forward Euler half step
//            (V1, q1) = FE(V, q), forward DST into work;
//   FHN_SRC  the same source plus the irregular-node correction C psi (rhs, read only on rows
//            flagged in mask, every row when mask is null), forward DST into work;
//   FHN_BE   inverse DST of work, then V <- 2 (u_i - u_e) - V1 and the backward Euler half step
//            from q1, written to V and q.
// V and q keep the step's starting state until FHN_BE: each pass recomputes (V1, q1) from
// them (the same arithmetic, so the same values), which costs less than writing and reading
// back the intermediate state.
// A thread handles whole nodes, so its LDS accesses are unit-stride 16-byte values.  The
// pointwise arithmetic is fhn_fe / fhn_be, which the separate midpoint sweep (k_mid_be, used
// when the potentials are returned) shares.
enum { FHN_FE = 0, FHN_SRC = 1, FHN_BE = 2 };

template <int M, int MODE>
__global__ __launch_bounds__((Shape<double, M>::NT)) void k_dst_x_fhn(FhnArgs a, double *__restrict__ work,
                                                                    const double *__restrict__ rhs,
                                                                    const uint64_t *__restrict__ mask, int64_t rows,
                                                                    int64_t cs, const C2<double> *__restrict__ tw,
                                                                    const double *__restrict__ sp) {
  using Sh = Shape<double, M>;
  using C = C2<double>;
  constexpr int N = Sh::N, NP = Sh::NP, NT = Sh::NT, PADM = Sh::PADM;
  constexpr int NE = NP * N, PER = (NE + NT - 1) / NT;
  __shared__ C sbuf[NP * PADM];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * NP;
  double *__restrict__ V = a.V;
  double *__restrict__ q = a.q;
  const double *__restrict__ stim = a.stim;
  const Sines<double, M> sn(sp, tid % Sh::TPP);
  double va[PER], qa[PER];
  if constexpr (MODE == FHN_BE) {
    C u[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      const int rr = e / N, n = e - rr * N;
      const int64_t row = r0 + rr;
      const bool ok = e < NE && row < rows;
      u[i] = ok ? C{work[row * M + n], work[cs + row * M + n]} : C{0.0, 0.0};
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      const int rr = e / N, n = e - rr * N;
      if (e < NE) sbuf[rr * PADM + pad(n + 1)] = u[i];
    }
  } else {
    double sa[PER], c0[PER], c1[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      const int rr = e / N, n = e - rr * N;
      const int64_t row = r0 + rr;
      const bool ok = e < NE && row < rows;
      va[i] = ok ? V[row * N + n] : 0.0;
      qa[i] = ok ? q[row * N + n] : 0.0;
      sa[i] = ok && stim ? stim[row * N + n] : 0.0;
    }
    // rows of the tile holding irregular nodes, from uniform loads of the bit rows [z][16]
    // (all issued before the first is used: the correction loads wait on them)
    uint64_t rb = ~uint64_t(0);
    if constexpr (MODE == FHN_SRC && NP <= 64) {
      if (mask) {
        constexpr int NB = NP < 16 ? NP : 16;
        rb = 0;
#pragma unroll 1
        for (int k0 = 0; k0 < NP; k0 += NB) {
          uint64_t wd[NB];
          int sh[NB];
#pragma unroll
          for (int k = 0; k < NB; ++k) {
            const int64_t row = r0 + k0 + k < rows ? r0 + k0 + k : rows - 1;
            const int64_t z = row / N, y = row - z * N;
            wd[k] = mask[z * 16 + (y >> 6)];
            sh[k] = (int)(y & 63);
          }
#pragma unroll
          for (int k = 0; k < NB; ++k)
            rb |= ((wd[k] >> sh[k]) & uint64_t(r0 + k0 + k < rows)) << (k0 + k);
        }
      }
    }
    auto flagged = [&](int rr) -> bool {
      if constexpr (NP > 64) return true;
      else return (rb >> rr) & 1;
    };
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      const int rr = e / N, n = e - rr * N;
      if (e < NE) {
        double v = va[i], g = qa[i];
        fhn_fe(v, g, a.dth, a.m);
        sbuf[rr * PADM + pad(n + 1)] = C{a.kappa * v, -a.kappa * v + (stim ? a.beta * sa[i] : 0.0)};
      }
    }
    if constexpr (MODE == FHN_SRC) {
      // the correction, added to the source words this thread wrote (loaded after the source
      // is in LDS, so that both sets of loads are not held in registers at once)
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int rr = e / N, n = e - rr * N;
        const int64_t row = r0 + rr;
        const bool has = e < NE && row < rows && flagged(rr);
        c0[i] = has ? rhs[row * M + n] : 0.0;
        c1[i] = has ? rhs[cs + row * M + n] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        const int rr = e / N, n = e - rr * N;
        if (e < NE && r0 + rr < rows && flagged(rr)) {
          C &w = sbuf[rr * PADM + pad(n + 1)];
          w.x = w.x + c0[i];
          w.y = w.y + c1[i];
        }
      }
    }
  }
  __syncthreads();
  dst_pair<double, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, tw, sn);
  if constexpr (MODE == FHN_BE) {
    // V and q after the transform: fetched ahead of it they would be held across it in
    // registers (a second wave per SIMD would no longer fit)
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      const int rr = e / N, n = e - rr * N;
      const int64_t row = r0 + rr;
      const bool ok = e < NE && row < rows;
      va[i] = ok ? V[row * N + n] : 0.0;
      qa[i] = ok ? q[row * N + n] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      const int rr = e / N, n = e - rr * N;
      const int64_t row = r0 + rr;
      if (e < NE && row < rows) {
        const C u = sbuf[rr * PADM + pad(n + 1)];
        double v1 = va[i], q1 = qa[i], vn, qn;
        fhn_fe(v1, q1, a.dth, a.m);
        fhn_be(2.0 * (u.x - u.y) - v1, q1, a.dth, a.m, vn, qn);
        V[row * N + n] = vn;
        q[row * N + n] = qn;
      }
    }
  } else {
    // whole padded rows of both components; the pad column (x = N) is written as zero
    constexpr int NO = NP * M, PO = (NO + NT - 1) / NT;
#pragma unroll
    for (int i = 0; i < PO; ++i) {
      const int e = tid + i * NT;
      const int rr = e / M, x = e - rr * M;
      const int64_t row = r0 + rr;
      if (e < NO && row < rows) {
        const C v = x < N ? sbuf[rr * PADM + pad(x + 1)] : C{0.0, 0.0};
        work[row * M + x] = v.x;
        work[cs + row * M + x] = v.y;
      }
    }
  }
}

// The forward x pass of the volume solve when the source is antisymmetric (no stimulus current:
// f = (kappa V1, -kappa V1), V1 the forward Euler half step of V): only g = kappa V1 is
// transformed, as one field in component 0 of work (rows of that field paired as in k_dst_x),
// and the z pass takes component 1 as -g.  Half the pencils and half the writes of FHN_FE.
// One pencil pair per wave at a time: a lane forms the values of both rows at one position and
// writes them as one 16-byte LDS word.  M >= 64.
template <int M>
__global__ __launch_bounds__((Shape<double, M>::NT)) void k_dst_x_fe1(FhnArgs a, double *__restrict__ work,
                                                                    int64_t rows, const C2<double> *__restrict__ tw,
                                                                    const double *__restrict__ sp) {
  static_assert(M >= 64, "one pencil pair per wave needs M >= 64");
  using Sh = Shape<double, M>;
  using C = C2<double>;
  constexpr int N = Sh::N, NP = Sh::NP, NT = Sh::NT, PADM = Sh::PADM;
  constexpr int NWV = NT / 64, PPW = NP / NWV, KS = M / 64;
  __shared__ C sbuf[NP * PADM];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 2 * NP;
  const Sines<double, M> sn(sp, tid % Sh::TPP);
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
  const double *__restrict__ V = a.V;
  const double *__restrict__ q = a.q;
  double va[PPW][KS][2], qa[PPW][KS][2];
#pragma unroll
  for (int pp = 0; pp < PPW; ++pp) {
    const int64_t rowa = r0 + 2 * (wv + NWV * pp);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool ok = rowa + h < rows;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int n = lane + 64 * k;
        va[pp][k][h] = ok && n < N ? V[(rowa + h) * N + n] : 0.0;
        qa[pp][k][h] = ok && n < N ? q[(rowa + h) * N + n] : 0.0;
      }
    }
  }
#pragma unroll
  for (int pp = 0; pp < PPW; ++pp)
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int n = lane + 64 * k;
      if (n < N) {
        double v0 = va[pp][k][0], g0 = qa[pp][k][0], v1 = va[pp][k][1], g1 = qa[pp][k][1];
        fhn_fe(v0, g0, a.dth, a.m);
        fhn_fe(v1, g1, a.dth, a.m);
        sbuf[(wv + NWV * pp) * PADM + pad(n + 1)] = C{a.kappa * v0, a.kappa * v1};
      }
    }
  __syncthreads();
  dst_pair<double, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, tw, sn);
#pragma unroll
  for (int pp = 0; pp < PPW; ++pp) {
    const int rr = wv + NWV * pp;
    const int64_t rowa = r0 + 2 * rr;
    const bool oka = rowa < rows, okb = rowa + 1 < rows;
    double *oa = work + rowa * M, *ob = oa + M;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int n = lane + 64 * k;   // n = N: the pad column, written as zero
      const C c = n < N ? sbuf[rr * PADM + pad(n + 1)] : C{0.0, 0.0};
      if (oka) oa[n] = c.x;
      if (okb) ob[n] = c.y;
    }
  }
}

// The inverse x pass of the final solve when its potentials are not returned: only
// d = Phi_i - Phi_e enters the step (V <- 2 d - V1, then backward Euler), and the inverse
// transforms are linear, so the z pass stores d (ZM = 4), the inverse y pass runs over that one
// field, and this pass transforms its rows in pairs (as k_dst_x) before the pointwise update of
// FHN_BE.  Half the pencils and a sixth less traffic than FHN_BE.  M >= 64.
template <int M>
__global__ __launch_bounds__((Shape<double, M>::NT)) void k_dst_x_be1(FhnArgs a, const double *__restrict__ work,
                                                                    int64_t rows, const C2<double> *__restrict__ tw,
                                                                    const double *__restrict__ sp) {
  static_assert(M >= 64, "one pencil pair per wave needs M >= 64");
  using Sh = Shape<double, M>;
  using C = C2<double>;
  constexpr int N = Sh::N, NP = Sh::NP, NT = Sh::NT, PADM = Sh::PADM;
  constexpr int NWV = NT / 64, PPW = NP / NWV, KS = M / 64;
  __shared__ C sbuf[NP * PADM];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 2 * NP;
  const Sines<double, M> sn(sp, tid % Sh::TPP);
  const int wv = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
  double *__restrict__ V = a.V;
  double *__restrict__ q = a.q;
  {
    C d[PPW][KS];
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp) {
      const int64_t rowa = r0 + 2 * (wv + NWV * pp);
      const bool oka = rowa < rows, okb = rowa + 1 < rows;
      const double *ra = work + rowa * M, *rb = ra + M;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int n = lane + 64 * k;
        d[pp][k] = {oka && n < N ? ra[n] : 0.0, okb && n < N ? rb[n] : 0.0};
      }
    }
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp)
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int n = lane + 64 * k;
        if (n < N) sbuf[(wv + NWV * pp) * PADM + pad(n + 1)] = d[pp][k];
      }
  }
  __syncthreads();
  dst_pair<double, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, tw, sn);
  // V and q after the transform (fetched ahead of it they would be held across it), a thread's
  // elements in two chunks whose loads are all issued before the chunk's first store (V and q
  // are read and written through the same pointers, so loads are not moved across stores)
  constexpr int NE = 2 * NP * N, PER = (NE + NT - 1) / NT, CH = PER > 16 ? 16 : PER;
#pragma unroll
  for (int c0 = 0; c0 < PER; c0 += CH) {
    double va[CH], qa[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int e = tid + (c0 + i) * NT;
      const int rr = e / N, n = e - rr * N;
      const int64_t row = r0 + rr;
      const bool ok = c0 + i < PER && e < NE && row < rows;
      va[i] = ok ? V[row * N + n] : 0.0;
      qa[i] = ok ? q[row * N + n] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int e = tid + (c0 + i) * NT;
      const int rr = e / N, n = e - rr * N;
      const int64_t row = r0 + rr;
      if (c0 + i < PER && e < NE && row < rows) {
        const C u = sbuf[(rr >> 1) * PADM + pad(n + 1)];
        double v1 = va[i], q1 = qa[i], vn, qn;
        fhn_fe(v1, q1, a.dth, a.m);
        fhn_be(2.0 * ((rr & 1) ? u.y : u.x) - v1, q1, a.dth, a.m, vn, qn);
        V[row * N + n] = vn;
        q[row * N + n] = qn;
      }
    }
  }
}

// ---------------------------------------------------------------- launchers
//
// Every dense pass exists at two tile widths (W = 1, 2: pencil pairs per workgroup); the
// width per (grid size, precision, pass) is picked by autotune_tiles() from timed launches.

template <typename T>
constexpr int prec_index() { return sizeof(T) == 8 ? 0 : 1; }

// x pass over `rows` contiguous rows (padded in/out unless stated)
template <typename T, int M, int W>
void launch_x(const T *in, bool in_plain, T *out, bool out_plain, int64_t rows, const C2<T> *tw, const T *sp,
              hipStream_t st) {
  using Sh = Shape<T, M, W>;
  const dim3 g((unsigned)((rows + 2 * Sh::NP - 1) / (2 * Sh::NP)));
  if (in_plain) k_dst_x<T, M, false, true, W><<<g, Sh::NT, 0, st>>>(in, out, rows, tw, sp);
  else if (out_plain) k_dst_x<T, M, true, false, W><<<g, Sh::NT, 0, st>>>(in, out, rows, tw, sp);
  else k_dst_x<T, M, true, true, W><<<g, Sh::NT, 0, st>>>(in, out, rows, tw, sp);
  KFBI_HIP(hipGetLastError());
}

template <typename T, int M, int W>
void launch_y(const T *in, T *out, int64_t P, int64_t cs, int ncomp, const uint64_t *mask_in,
              const uint64_t *mask_out, const uint8_t *planes, const C2<T> *tw, const T *sp, hipStream_t st) {
  using Sh = Shape<T, M, W>;
  const dim3 g((Sh::N + 2 * Sh::NP - 1) / (2 * Sh::NP), Sh::N, ncomp);
  k_dst_y<T, M, W><<<g, Sh::NT, 0, st>>>(in, out, P, cs, mask_in, mask_out, planes, tw, sp);
  KFBI_HIP(hipGetLastError());
}

// fused last-axis pass; nprob > 1 only in 2D (batched groups with per-problem msv)
template <typename T, int M, int W>
void launch_last(const T *in, T *a, int dim, int ncomp, int64_t P, int64_t cs, const ModeScale &ms,
                 const C2<T> *tw, const T *sp, const ModeScale *msv, int nprob, int64_t pstride, hipStream_t st,
                 const PlaneBits *zin = nullptr, const PlaneBits *zout = nullptr, int form = 0,
                 const T *in2 = nullptr) {
  using Sh = Shape<T, M, W>;
  const int tx = ncomp == 2 ? Sh::NP : 2 * Sh::NP;
  const dim3 g((Sh::N + tx - 1) / tx, dim == 3 ? Sh::N : nprob, 1);
  // form 3: antisymmetric source (needs zout); form 4: the difference of the pair (no masks);
  // form 5: form 4 for the antisymmetric pair of in plus the pair of in2 on the planes in zin
  if (form == 3 && (dim != 3 || ncomp != 2 || zin || !zout))
    throw std::invalid_argument("the antisymmetric z pass takes the coupled 3D pair and an output plane mask");
  if (form == 4 && (dim != 3 || ncomp != 2 || zin || zout))
    throw std::invalid_argument("the difference z pass takes the coupled 3D pair and no plane masks");
  if (form == 5 && (dim != 3 || ncomp != 2 || !zin || zout || !in2))
    throw std::invalid_argument("the combined z pass takes the coupled 3D pair, a second input and its plane mask");
  if (dim == 3) {
    if (form >= 3) {
      if constexpr (StridedTile<T, M, Sh::NP, 2, W>::VEC) {
        if (form == 3) k_dst_last<T, M, 2, 3, W, 3><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp, nullptr, 0, {}, *zout);
        else if (form == 4) k_dst_last<T, M, 2, 3, W, 4><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp);
        else k_dst_last<T, M, 2, 3, W, 5><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp, nullptr, 0, *zin, {}, in2);
      } else {
        throw std::invalid_argument("the z passes of forms 3 to 5 need tiles of whole 16-byte vectors (M >= 64)");
      }
    } else if (zin && zout) {
      if (ncomp == 2) k_dst_last<T, M, 2, 3, W, 1><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp, nullptr, 0, *zin, *zout);
      else k_dst_last<T, M, 1, 3, W, 1><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp, nullptr, 0, *zin, *zout);
    } else if (zout) {
      if (ncomp == 2) k_dst_last<T, M, 2, 3, W, 2><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp, nullptr, 0, {}, *zout);
      else k_dst_last<T, M, 1, 3, W, 2><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp, nullptr, 0, {}, *zout);
    } else {
      if (zin) throw std::invalid_argument("an input plane mask needs an output plane mask");
      if (ncomp == 2) k_dst_last<T, M, 2, 3, W><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp);
      else k_dst_last<T, M, 1, 3, W><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp);
    }
  } else {
    if (ncomp == 2) k_dst_last<T, M, 2, 2, W><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp, msv, pstride);
    else k_dst_last<T, M, 1, 2, W><<<g, Sh::NT, 0, st>>>(in, a, P, cs, ms, tw, sp, msv, pstride);
  }
  KFBI_HIP(hipGetLastError());
}

template <typename T, int M>
void pass_x(int w, const T *in, bool in_plain, T *out, bool out_plain, int64_t rows, const C2<T> *tw, const T *sp,
            hipStream_t st) {
  if (w == 2) launch_x<T, M, 2>(in, in_plain, out, out_plain, rows, tw, sp, st);
  else launch_x<T, M, 1>(in, in_plain, out, out_plain, rows, tw, sp, st);
}
template <typename T, int M>
void pass_y(int w, const T *in, T *out, int64_t P, int64_t cs, int ncomp, const uint64_t *mi, const uint64_t *mo,
            const C2<T> *tw, const T *sp, hipStream_t st, const uint8_t *planes = nullptr) {
  if (w == 2) launch_y<T, M, 2>(in, out, P, cs, ncomp, mi, mo, planes, tw, sp, st);
  else launch_y<T, M, 1>(in, out, P, cs, ncomp, mi, mo, planes, tw, sp, st);
}
template <typename T, int M>
void pass_last(int w, T *a, int dim, int ncomp, int64_t P, int64_t cs, const ModeScale &ms, const C2<T> *tw,
               const T *sp, const ModeScale *msv, int nprob, int64_t pstride, hipStream_t st,
               const T *in = nullptr, const PlaneBits *zin = nullptr, const PlaneBits *zout = nullptr,
               int form = 0, const T *in2 = nullptr) {
  if (!in) in = a;
  if (w == 2) launch_last<T, M, 2>(in, a, dim, ncomp, P, cs, ms, tw, sp, msv, nprob, pstride, st, zin, zout, form, in2);
  else launch_last<T, M, 1>(in, a, dim, ncomp, P, cs, ms, tw, sp, msv, nprob, pstride, st, zin, zout, form, in2);
}

template <typename T>
ModeScale mode_of(const DevProblem &p) {
  ModeScale m{};
  m.lam = p.lam;
  for (int a = 0; a < 3; ++a) {
    m.D0[a] = p.D[0][a];
    m.D1[a] = p.D[p.ncomp == 2 ? 1 : 0][a];
  }
  m.kappa = p.kappa;
  m.norm = p.lam_scale;
  return m;
}

// skip & 1: work already holds the forward x pass of the source (src unused); skip & 2: stop
// after the inverse y (3D) / last-axis (2D) pass, leaving its output in work.
template <typename T, int M>
void run_box(DevProblem &p, const T *src, bool src_plain, T *dst, bool dst_plain, hipStream_t st, int skip = 0) {
  constexpr int N = M - 1;
  PrecTables<T> &tb = p.tab<T>();
  T *A = tb.work;
  const C2<T> *tw = reinterpret_cast<const C2<T> *>(tb.tw);
  const T *sp = tb.sp;
  const int64_t P = p.P, cs = p.comp_stride;
  const int64_t rows = (int64_t)p.ncomp * (p.dim == 3 ? (int64_t)N * N : N);
  const int *w = p.tile_w[prec_index<T>()];
  const ModeScale ms = mode_of<T>(p);
  auto tic = [&](Timer &t) { t.tic(p.profile, st); };
  auto toc = [&](Timer &t) { t.toc(p.profile, st); };
  if (!(skip & 1)) {
    tic(p.t_dst_x);
    pass_x<T, M>(w[0], src, src_plain, A, false, rows, tw, sp, st);
    toc(p.t_dst_x);
  }
  if (p.dim == 3) {
    tic(p.t_dst_y);
    pass_y<T, M>(w[1], A, A, P, cs, p.ncomp, nullptr, nullptr, tw, sp, st);
    toc(p.t_dst_y);
  }
  tic(p.t_dst_last);
  pass_last<T, M>(w[2], A, p.dim, p.ncomp, P, cs, ms, tw, sp, nullptr, 1, 0, st);
  toc(p.t_dst_last);
  if (p.dim == 3) {
    tic(p.t_dst_y);
    pass_y<T, M>(w[1], A, A, P, cs, p.ncomp, nullptr, nullptr, tw, sp, st);
    toc(p.t_dst_y);
  }
  if (!(skip & 2)) {
    tic(p.t_dst_x);
    pass_x<T, M>(w[0], A, false, dst, dst_plain, rows, tw, sp, st);
    toc(p.t_dst_x);
  }
}

// Box solve whose result is read only at extrapolation-stencil nodes (the volume part of the
// BIE right-hand side): dense forward passes, then the z pass writes and the inverse y and x
// passes transform only the planes and rows that hold stencil nodes.  Result in work; the
// values at every stencil node are identical to the full solve.
// skip_x: work already holds the forward x pass of the source (src unused).
template <typename T, int M>
void run_box_stencils(DevProblem &p, const T *src, hipStream_t st, bool skip_x = false, bool anti = false) {
  constexpr int N = M - 1;
  using Sh = Shape<T, M>;
  PrecTables<T> &tb = p.tab<T>();
  T *A = tb.work;
  const C2<T> *tw = reinterpret_cast<const C2<T> *>(tb.tw);
  const T *sp = tb.sp;
  const int64_t P = p.P, cs = p.comp_stride;
  const int64_t rows = (int64_t)p.ncomp * N * N;
  const int *w = p.tile_w[prec_index<T>()];
  const ModeScale ms = mode_of<T>(p);
  auto tic = [&](Timer &t) { t.tic(p.profile, st); };
  auto toc = [&](Timer &t) { t.toc(p.profile, st); };
  if (!skip_x) {
    tic(p.t_dst_x);
    pass_x<T, M>(w[0], src, false, A, false, rows, tw, sp, st);
    toc(p.t_dst_x);
  }
  if (anti) {
    // antisymmetric source (component 1 = -component 0), its one field in gbuf after the x
    // pass: y forward over it (kept there for the step's final solve), and the z pass reads it
    // as the pair (g, -g) and writes both components' stencil planes into work
    T *G = tb.gbuf;
    if (!G) throw std::logic_error("antisymmetric volume solve without its buffer");
    tic(p.t_dst_y1);
    pass_y<T, M>(w[1], G, G, P, cs, 1, nullptr, nullptr, tw, sp, st);
    toc(p.t_dst_y1);
    tic(p.t_dst_last_anti);
    pass_last<T, M>(w[2], A, 3, p.ncomp, P, cs, ms, tw, sp, nullptr, 1, 0, st, G, nullptr, &p.planes_out_bits, 3);
    toc(p.t_dst_last_anti);
  } else {
    tic(p.t_dst_y);
    pass_y<T, M>(w[1], A, A, P, cs, p.ncomp, nullptr, nullptr, tw, sp, st);
    toc(p.t_dst_y);
    tic(p.t_dst_last_out);
    pass_last<T, M>(w[2], A, 3, p.ncomp, P, cs, ms, tw, sp, nullptr, 1, 0, st, nullptr, nullptr, &p.planes_out_bits);
    toc(p.t_dst_last_out);
  }
  tic(p.t_dst_y_sparse);
  pass_y<T, M>(w[1], A, A, P, cs, p.ncomp, nullptr, p.mask_out, tw, sp, st, p.planes_out);
  toc(p.t_dst_y_sparse);
  const unsigned gout = (unsigned)((p.n_rows_out + 2 * Sh::NP - 1) / (2 * Sh::NP));
  tic(p.t_dst_x_rows);
  if (gout) k_dst_x_rows<T, M><<<gout, Sh::NT, 0, st>>>(A, A, p.rows_out, p.n_rows_out, tw, sp);
  KFBI_HIP(hipGetLastError());
  toc(p.t_dst_x_rows);
}

template <int M, int MODE>
void launch_x_fhn(DevProblem &p, const FhnArgs &a, hipStream_t st) {
  using Sh = Shape<double, M>;
  if (p.ncomp != 2 || p.P != M) throw std::invalid_argument("bidomain x pass: coupled pair in the padded layout");
  const int64_t rows = p.dim == 3 ? p.N * p.N : p.N;
  const unsigned g = (unsigned)((rows + Sh::NP - 1) / Sh::NP);
  const uint64_t *mask = MODE == FHN_SRC && p.dim == 3 && p.sparse ? p.mask_in : nullptr;
  PrecTables<double> &tb = p.f64;
  p.t_dst_x_fhn.tic(p.profile, st);
  k_dst_x_fhn<M, MODE><<<g, Sh::NT, 0, st>>>(a, tb.work, tb.rhs, mask, rows, p.comp_stride,
                                             reinterpret_cast<const C2<double> *>(tb.tw), tb.sp);
  KFBI_HIP(hipGetLastError());
  p.t_dst_x_fhn.toc(p.profile, st);
}

// Without a stimulus current the source (kappa V1, -kappa V1) is antisymmetric: the 3D volume
// solve then transforms the one field kappa V1 forward along x and y (into gbuf, where the
// step's final solve finds it again), and its z pass takes the second component as the
// negative of the first (k_dst_x_fe1, dst_last_tile with ZM = 3).
template <int M>
void launch_x_fe1(DevProblem &p, const FhnArgs &a, hipStream_t st) {
  using Sh = Shape<double, M>;
  if (p.ncomp != 2 || p.P != M || p.dim != 3) throw std::invalid_argument("antisymmetric x pass: coupled 3D pair");
  const int64_t rows = p.N * p.N;
  const unsigned g = (unsigned)((rows + 2 * Sh::NP - 1) / (2 * Sh::NP));
  if (!p.f64.gbuf) throw std::logic_error("antisymmetric x pass without its buffer");
  p.t_dst_x_fe1.tic(p.profile, st);
  k_dst_x_fe1<M><<<g, Sh::NT, 0, st>>>(a, p.f64.gbuf, rows, reinterpret_cast<const C2<double> *>(p.f64.tw),
                                       p.f64.sp);
  KFBI_HIP(hipGetLastError());
  p.t_dst_x_fe1.toc(p.profile, st);
}

template <int M>
void run_bidomain_volume(DevProblem &p, const FhnArgs &a, hipStream_t st) {
  if constexpr (M >= 64) {
    if (p.dim == 3 && p.sparse && !a.stim) {
      launch_x_fe1<M>(p, a, st);
      run_box_stencils<double, M>(p, nullptr, st, true, true);
      return;
    }
  }
  launch_x_fhn<M, FHN_FE>(p, a, st);
  if (p.dim == 3 && p.sparse) run_box_stencils<double, M>(p, nullptr, st, true);
  else run_box<double, M>(p, nullptr, false, p.f64.work, false, st, 1);
}

template <int M>
void run_bidomain_final(DevProblem &p, const FhnArgs &a, bool fuse_be, hipStream_t st) {
  if constexpr (M >= 64) {
    if (p.dim == 3 && fuse_be) {
      // only Phi_i - Phi_e is needed: the z pass stores it, and the inverse y and x passes (the
      // latter with the backward Euler update) run over that one field
      using Sh = Shape<double, M>;
      PrecTables<double> &tb = p.f64;
      double *A = tb.work;
      const C2<double> *tw = reinterpret_cast<const C2<double> *>(tb.tw);
      const int64_t P = p.P, cs = p.comp_stride;
      const int *w = p.tile_w[0];
      if (p.sparse && !a.stim && tb.gbuf) {
        // f + C psi with f = (g, -g) antisymmetric: the volume solve left g's x-y transform in
        // gbuf, so only C psi is transformed, on the rows and planes holding irregular nodes as
        // in the product, and the z pass adds the two as it loads
        double *X = tb.xbuf, *Y = tb.ybuf;
        const unsigned gin = (unsigned)((p.n_rows_in + 2 * Sh::NP - 1) / (2 * Sh::NP));
        p.t_dst_x_rows.tic(p.profile, st);
        if (gin) k_dst_x_rows<double, M><<<gin, Sh::NT, 0, st>>>(tb.rhs, X, p.rows_in, p.n_rows_in, tw, tb.sp);
        KFBI_HIP(hipGetLastError());
        p.t_dst_x_rows.toc(p.profile, st);
        p.t_dst_y_sparse.tic(p.profile, st);
        pass_y<double, M>(w[1], X, Y, P, cs, 2, p.mask_in, nullptr, tw, tb.sp, st, p.planes_in);
        p.t_dst_y_sparse.toc(p.profile, st);
        p.t_dst_last_comb.tic(p.profile, st);
        pass_last<double, M>(w[2], A, 3, 2, P, cs, mode_of<double>(p), tw, tb.sp, nullptr, 1, 0, st, tb.gbuf,
                             &p.planes_in_bits, nullptr, 5, Y);
        p.t_dst_last_comb.toc(p.profile, st);
      } else {
        launch_x_fhn<M, FHN_SRC>(p, a, st);
        p.t_dst_y.tic(p.profile, st);
        pass_y<double, M>(w[1], A, A, P, cs, 2, nullptr, nullptr, tw, tb.sp, st);
        p.t_dst_y.toc(p.profile, st);
        p.t_dst_last_diff.tic(p.profile, st);
        pass_last<double, M>(w[2], A, 3, 2, P, cs, mode_of<double>(p), tw, tb.sp, nullptr, 1, 0, st, nullptr, nullptr,
                             nullptr, 4);
        p.t_dst_last_diff.toc(p.profile, st);
      }
      p.t_dst_y1.tic(p.profile, st);
      pass_y<double, M>(w[1], A, A, P, cs, 1, nullptr, nullptr, tw, tb.sp, st);
      p.t_dst_y1.toc(p.profile, st);
      const int64_t rows = p.N * p.N;
      p.t_dst_x_be1.tic(p.profile, st);
      k_dst_x_be1<M><<<(unsigned)((rows + 2 * Sh::NP - 1) / (2 * Sh::NP)), Sh::NT, 0, st>>>(a, A, rows, tw, tb.sp);
      KFBI_HIP(hipGetLastError());
      p.t_dst_x_be1.toc(p.profile, st);
      return;
    }
  }
  launch_x_fhn<M, FHN_SRC>(p, a, st);
  run_box<double, M>(p, nullptr, false, p.f64.work, false, st, fuse_be ? 3 : 1);
  if (fuse_be) launch_x_fhn<M, FHN_BE>(p, a, st);
}

// Box solve inside the matrix-vector product: the right-hand side is zero outside the rows
// that hold irregular nodes, and only the rows that hold extrapolation-stencil nodes are read
// afterwards.  x forward runs on the first rows only (into a buffer whose other rows stay zero),
// y forward skips reading zero rows and skips whole z planes without such rows (its output
// buffer stays zero there), y inverse writes and x inverse transforms only the second rows,
// skipping whole planes without them.  The values at every stencil node are identical to the
// full solve.
template <typename T, int M>
void run_box_sparse(DevProblem &p, hipStream_t st) {
  using Sh = Shape<T, M>;
  PrecTables<T> &tb = p.tab<T>();
  T *A = tb.work, *X = tb.xbuf;
  const C2<T> *tw = reinterpret_cast<const C2<T> *>(tb.tw);
  const T *sp = tb.sp;
  const int64_t P = p.P, cs = p.comp_stride;
  const int *w = p.tile_w[prec_index<T>()];
  const ModeScale ms = mode_of<T>(p);
  auto tic = [&](Timer &t) { t.tic(p.profile, st); };
  auto toc = [&](Timer &t) { t.toc(p.profile, st); };
  const unsigned gin = (unsigned)((p.n_rows_in + 2 * Sh::NP - 1) / (2 * Sh::NP));
  const unsigned gout = (unsigned)((p.n_rows_out + 2 * Sh::NP - 1) / (2 * Sh::NP));
  tic(p.t_dst_x_rows);
  if (gin) k_dst_x_rows<T, M><<<gin, Sh::NT, 0, st>>>(tb.rhs, X, p.rows_in, p.n_rows_in, tw, sp);
  KFBI_HIP(hipGetLastError());
  toc(p.t_dst_x_rows);
  T *Y = tb.ybuf;
  tic(p.t_dst_y_sparse);
  pass_y<T, M>(w[1], X, Y, P, cs, p.ncomp, p.mask_in, nullptr, tw, sp, st, p.planes_in);
  toc(p.t_dst_y_sparse);
  tic(p.t_dst_last_sparse);
  // planes without rhs rows are zero in Y (not read); only planes with stencil rows are used
  // by the inverse passes (only those are written)
  pass_last<T, M>(w[2], A, 3, p.ncomp, P, cs, ms, tw, sp, nullptr, 1, 0, st, Y, &p.planes_in_bits, &p.planes_out_bits);
  toc(p.t_dst_last_sparse);
  tic(p.t_dst_y_sparse);
  pass_y<T, M>(w[1], A, A, P, cs, p.ncomp, nullptr, p.mask_out, tw, sp, st, p.planes_out);
  toc(p.t_dst_y_sparse);
  tic(p.t_dst_x_rows);
  if (gout) k_dst_x_rows<T, M><<<gout, Sh::NT, 0, st>>>(A, A, p.rows_out, p.n_rows_out, tw, sp);
  KFBI_HIP(hipGetLastError());
  toc(p.t_dst_x_rows);
}

// Grouped 2D box solve of G one-component problems of equal size, stored at stride cs in
// padded layout: one launch per pass for the whole group.
template <typename T, int M>
void run_box_group(int G, const T *src, T *dst, int64_t cs, const ModeParams *msv, const T *tw_, const T *sp,
                   const int *w, hipStream_t st) {
  constexpr int N = M - 1;
  const C2<T> *tw = reinterpret_cast<const C2<T> *>(tw_);
  const int64_t rows = (int64_t)G * N;
  if (cs != (int64_t)N * M) throw std::invalid_argument("group stride");
  pass_x<T, M>(w[0], src, false, dst, false, rows, tw, sp, st);
  pass_last<T, M>(w[2], dst, 2, 1, M, cs, ModeParams{}, tw, sp, msv, G, cs, st);
  pass_x<T, M>(w[0], dst, false, dst, false, rows, tw, sp, st);
}

// ---------------------------------------------------------------- merged 2D group passes
//
// One launch per pass over several size groups: the workgroups of group k are the block range
// [begin_k, begin_{k+1}) and run that group's tile at its own size M (a switch on the uniform
// size).  The workgroup size BASE / 16 is the same at every M, and so is the LDS tile buffer
// up to a few hundred bytes, so one shape serves all sizes.

template <typename T>
struct MultiX {
  struct G {
    const T *in;
    T *out;
    int64_t rows;
    const C2<T> *tw;
    const T *sp;
    int M, begin;
  } g[kMaxMultiGroups];
  int ng;
};

template <typename T>
struct MultiLast {
  struct G {
    T *a;
    int64_t cs;
    const ModeScale *msv;
    const C2<T> *tw;
    const T *sp;
    int M, begin, gx, nprob;
  } g[kMaxMultiGroups];
  int ng;
};

// largest tile buffer over the sizes 64..1024 at width 1 (NP * PADM, in complex values)
template <typename T>
constexpr int multi_sbuf() {
  return std::max({Shape<T, 64>::NP * Shape<T, 64>::PADM, Shape<T, 128>::NP * Shape<T, 128>::PADM,
                   Shape<T, 256>::NP * Shape<T, 256>::PADM, Shape<T, 512>::NP * Shape<T, 512>::PADM,
                   Shape<T, 1024>::NP * Shape<T, 1024>::PADM});
}

template <typename T, typename Mp>
__device__ __forceinline__ int multi_group(const Mp &mp) {
  int k = 0;
#pragma unroll
  for (int j = 1; j < kMaxMultiGroups; ++j)
    if (j < mp.ng && (int)blockIdx.x >= mp.g[j].begin) k = j;
  return k;
}

template <typename T>
__global__ __launch_bounds__((Shape<T, 64>::NT)) void k_dst_x_multi(MultiX<T> mp) {
  static_assert(Shape<T, 64>::NT == Shape<T, 1024>::NT, "one workgroup size for every M");
  __shared__ C2<T> sbuf[multi_sbuf<T>()];
  const int k = multi_group<T>(mp);
  const auto &g = mp.g[k];
  const int64_t b = (int64_t)blockIdx.x - g.begin;
  switch (g.M) {
    case 64: dst_x_tile<T, 64, true, true>(g.in, g.out, g.rows, g.tw, g.sp, sbuf, b); break;
    case 128: dst_x_tile<T, 128, true, true>(g.in, g.out, g.rows, g.tw, g.sp, sbuf, b); break;
    case 256: dst_x_tile<T, 256, true, true>(g.in, g.out, g.rows, g.tw, g.sp, sbuf, b); break;
    case 512: dst_x_tile<T, 512, true, true>(g.in, g.out, g.rows, g.tw, g.sp, sbuf, b); break;
    default: dst_x_tile<T, 1024, true, true>(g.in, g.out, g.rows, g.tw, g.sp, sbuf, b); break;
  }
}

template <typename T>
__global__ __launch_bounds__((Shape<T, 64>::NT)) void k_dst_last_multi(MultiLast<T> mp) {
  __shared__ C2<T> sbuf[multi_sbuf<T>()];
  __shared__ T slam[1024];
  __shared__ T ssin[1024 / 2 + 1];
  const int k = multi_group<T>(mp);
  const auto &g = mp.g[k];
  const int64_t b = (int64_t)blockIdx.x - g.begin, total = (int64_t)g.gx * g.nprob;
  const ModeScale none{};
  const PlaneBits nob{};
  switch (g.M) {
#define KFBI_MULTI_LAST(MM)                                                                                    \
    case MM:                                                                                                   \
      dst_last_tile<T, MM, 1, 2>(g.a, g.a, MM, g.cs, none, g.tw, g.sp, g.msv, g.cs, nob, nob, sbuf, slam, ssin, b, \
                                 total, g.gx);                                                                 \
      break;
    KFBI_MULTI_LAST(64) KFBI_MULTI_LAST(128) KFBI_MULTI_LAST(256) KFBI_MULTI_LAST(512)
    default:
      dst_last_tile<T, 1024, 1, 2>(g.a, g.a, 1024, g.cs, none, g.tw, g.sp, g.msv, g.cs, nob, nob, sbuf, slam, ssin,
                                   b, total, g.gx);
      break;
#undef KFBI_MULTI_LAST
  }
}

template <typename T>
int tile_rows(int M) {   // rows per x-pass tile at width 1
  return 2 * ((sizeof(T) == 8 ? 2048 : 4096) / M);
}

// Timing data: a fixed pseudo-random pattern in [-0.5, 0.5) (all-zero data runs at a higher
// clock than real data under the power limit, which would bias the choice).
template <typename T>
__global__ void k_fill_pattern(T *__restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) a[i] = (T)((((uint32_t)i * 2654435761u) >> 8) & 0xffffu) * (T)(1.0 / 65536.0) - (T)0.5;
}

// One launch of a pass at width w, in place on `a`, timed with events.
template <typename T, int M>
float time_pass(int pass, int w, T *a, int dim, int ncomp, int64_t P, int64_t cs, int64_t rows, const ModeScale &ms,
                const C2<T> *tw, const T *sp, const ModeScale *msv, int nprob, hipEvent_t e0, hipEvent_t e1,
                hipStream_t st) {
  // fresh data for every launch (the unnormalised passes would otherwise grow it without bound)
  const int64_t nfill = dim == 3 ? (int64_t)ncomp * cs : (int64_t)nprob * cs;
  k_fill_pattern<T><<<(unsigned)((nfill + 255) / 256), 256, 0, st>>>(a, nfill);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipEventRecord(e0, st));
  if (pass == 0) pass_x<T, M>(w, a, false, a, false, rows, tw, sp, st);
  else if (pass == 1) pass_y<T, M>(w, a, a, P, cs, ncomp, nullptr, nullptr, tw, sp, st);
  else pass_last<T, M>(w, a, dim, ncomp, P, cs, ms, tw, sp, msv, nprob, cs, st);
  KFBI_HIP(hipEventRecord(e1, st));
  KFBI_HIP(hipEventSynchronize(e1));
  float ms_ = 0;
  KFBI_HIP(hipEventElapsedTime(&ms_, e0, e1));
  return ms_;
}

// Both widths are launched alternately (after warm-up launches that bring the clocks up), so
// that clock and cache drift affect both alike; the median of each decides.
template <typename T, int M>
void tune(int *w, T *a, int dim, int ncomp, int64_t P, int64_t cs, int64_t rows, const ModeScale &ms,
          const C2<T> *tw, const T *sp, const ModeScale *msv, int nprob, hipStream_t st) {
  constexpr int kRounds = 7;
  hipEvent_t e0, e1;
  KFBI_HIP(hipEventCreate(&e0));
  KFBI_HIP(hipEventCreate(&e1));
  for (int pass = 0; pass < 3; ++pass) {
    if (pass == 1 && dim != 3) continue;
    float t[2][kRounds];
    for (int r = -2; r < kRounds; ++r)
      for (int k = 0; k < 2; ++k) {
        const float v = time_pass<T, M>(pass, k + 1, a, dim, ncomp, P, cs, rows, ms, tw, sp, msv, nprob, e0, e1, st);
        if (r >= 0) t[k][r] = v;
      }
    std::sort(t[0], t[0] + kRounds);
    std::sort(t[1], t[1] + kRounds);
    w[pass] = t[1][kRounds / 2] < 0.97f * t[0][kRounds / 2] ? 2 : 1;   // the wider tile must win clearly
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

template <typename T>
void autotune_prec(DevProblem &p, hipStream_t st) {
  PrecTables<T> &tb = p.tab<T>();
  T *A = tb.work;
  const C2<T> *tw = reinterpret_cast<const C2<T> *>(tb.tw);
  const int64_t N = p.N;
  const int64_t rows = (int64_t)p.ncomp * (p.dim == 3 ? N * N : N);
  const ModeScale ms = mode_of<T>(p);
  int *w = p.tile_w[prec_index<T>()];
  switch (p.Mfft) {
#define KFBI_TUNE_CASE(MM) \
    case MM: tune<T, MM>(w, A, p.dim, p.ncomp, p.P, p.comp_stride, rows, ms, tw, tb.sp, nullptr, 1, st); break;
    KFBI_TUNE_CASE(16) KFBI_TUNE_CASE(32) KFBI_TUNE_CASE(64) KFBI_TUNE_CASE(128) KFBI_TUNE_CASE(256)
    KFBI_TUNE_CASE(512) KFBI_TUNE_CASE(1024)
#undef KFBI_TUNE_CASE
    default: throw std::invalid_argument("unsupported grid size");
  }
}

}  // namespace

// Tile widths per (dimension, grid size, components, precision): measured once per process.
void autotune_tiles(DevProblem &p, hipStream_t st) {
  static std::mutex mu;
  static std::map<std::array<int, 4>, std::array<int, 3>> cache;
  for (int prec = 0; prec < 2; ++prec) {
    const std::array<int, 4> key{p.dim, (int)p.Mfft, p.ncomp, prec};
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = cache.find(key);
      if (it != cache.end()) {
        for (int k = 0; k < 3; ++k) p.tile_w[prec][k] = it->second[k];
        continue;
      }
    }
    if (prec == 0) autotune_prec<double>(p, st);
    else autotune_prec<float>(p, st);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = {p.tile_w[prec][0], p.tile_w[prec][1], p.tile_w[prec][2]};
  }
  // the timing launches ran in place on the work buffers: leave them zeroed
  const size_t field = (size_t)p.ncomp * p.comp_stride;
  KFBI_HIP(hipMemsetAsync(p.f64.work, 0, field * sizeof(double), st));
  KFBI_HIP(hipMemsetAsync(p.f32.work, 0, field * sizeof(float), st));
  KFBI_HIP(hipStreamSynchronize(st));
}

// Batched groups: widths of the x and last-axis passes for one group, timed on its buffers.
template <typename T>
void autotune_group(int Mfft, int G, T *a, int64_t cs, const ModeParams *msv, const T *tw_, const T *sp, int *w,
                    hipStream_t st) {
  const C2<T> *tw = reinterpret_cast<const C2<T> *>(tw_);
  const int64_t rows = (int64_t)G * (Mfft - 1);
  switch (Mfft) {
#define KFBI_TUNE_CASE(MM) \
    case MM: tune<T, MM>(w, a, 2, 1, MM, cs, rows, ModeParams{}, tw, sp, msv, G, st); break;
    KFBI_TUNE_CASE(16) KFBI_TUNE_CASE(32) KFBI_TUNE_CASE(64) KFBI_TUNE_CASE(128) KFBI_TUNE_CASE(256)
    KFBI_TUNE_CASE(512) KFBI_TUNE_CASE(1024)
#undef KFBI_TUNE_CASE
    default: throw std::invalid_argument("unsupported grid size");
  }
  KFBI_HIP(hipMemsetAsync(a, 0, (size_t)G * cs * sizeof(T), st));
  KFBI_HIP(hipStreamSynchronize(st));
}
template void autotune_group<double>(int, int, double *, int64_t, const ModeParams *, const double *,
                                     const double *, int *, hipStream_t);
template void autotune_group<float>(int, int, float *, int64_t, const ModeParams *, const float *, const float *,
                                    int *, hipStream_t);

template <typename T>
void box_solve_group(int Mfft, int G, const T *src, T *dst, int64_t cs, const ModeParams *msv, const T *tw,
                     const T *sp, const int *w, hipStream_t st) {
  switch (Mfft) {
    case 16: run_box_group<T, 16>(G, src, dst, cs, msv, tw, sp, w, st); break;
    case 32: run_box_group<T, 32>(G, src, dst, cs, msv, tw, sp, w, st); break;
    case 64: run_box_group<T, 64>(G, src, dst, cs, msv, tw, sp, w, st); break;
    case 128: run_box_group<T, 128>(G, src, dst, cs, msv, tw, sp, w, st); break;
    case 256: run_box_group<T, 256>(G, src, dst, cs, msv, tw, sp, w, st); break;
    case 512: run_box_group<T, 512>(G, src, dst, cs, msv, tw, sp, w, st); break;
    case 1024: run_box_group<T, 1024>(G, src, dst, cs, msv, tw, sp, w, st); break;
    default: throw std::invalid_argument("unsupported grid size");
  }
}
template <typename T>
void box_solve_multi(const MultiGroupDesc *gd, int ng, hipStream_t st) {
  if (ng < 1 || ng > kMaxMultiGroups) throw std::invalid_argument("merged passes take 1 to 8 groups");
  // largest grids first: their long-running tiles start first, the small ones fill in after
  int order[kMaxMultiGroups];
  for (int k = 0; k < ng; ++k) order[k] = k;
  std::sort(order, order + ng, [&](int a, int b) { return gd[a].Mfft > gd[b].Mfft; });
  MultiX<T> x1{}, x2{};
  MultiLast<T> la{};
  int bx = 0, bl = 0;
  for (int j = 0; j < ng; ++j) {
    const MultiGroupDesc &d = gd[order[j]];
    const int M = d.Mfft, N = M - 1;
    if (M < 64 || M > 1024 || (M & (M - 1)) || d.G < 1 || d.cs != (int64_t)N * M)
      throw std::invalid_argument("merged passes: sizes 64..1024, padded groups");
    const int64_t rows = (int64_t)d.G * N;
    const int tr = tile_rows<T>(M), np = tr / 2;
    const C2<T> *tw = reinterpret_cast<const C2<T> *>(d.tw);
    const T *sp = static_cast<const T *>(d.sp);
    T *dst = static_cast<T *>(d.dst);
    x1.g[j] = {static_cast<const T *>(d.src), dst, rows, tw, sp, M, bx};
    x2.g[j] = {dst, dst, rows, tw, sp, M, bx};
    bx += (int)((rows + tr - 1) / tr);
    const int gx = (N + 2 * np - 1) / (2 * np);
    la.g[j] = {dst, d.cs, d.msv, tw, sp, M, bl, gx, d.G};
    bl += gx * d.G;
  }
  x1.ng = x2.ng = la.ng = ng;
  constexpr int NT = Shape<T, 64>::NT;
  k_dst_x_multi<T><<<bx, NT, 0, st>>>(x1);
  KFBI_HIP(hipGetLastError());
  k_dst_last_multi<T><<<bl, NT, 0, st>>>(la);
  KFBI_HIP(hipGetLastError());
  k_dst_x_multi<T><<<bx, NT, 0, st>>>(x2);
  KFBI_HIP(hipGetLastError());
}
template void box_solve_multi<double>(const MultiGroupDesc *, int, hipStream_t);
template void box_solve_multi<float>(const MultiGroupDesc *, int, hipStream_t);

template void box_solve_group<double>(int, int, const double *, double *, int64_t, const ModeParams *,
                                      const double *, const double *, const int *, hipStream_t);
template void box_solve_group<float>(int, int, const float *, float *, int64_t, const ModeParams *, const float *,
                                     const float *, const int *, hipStream_t);

template <typename T>
void box_solve(DevProblem &p, const T *src, bool src_plain, T *dst, bool dst_plain, hipStream_t st) {
  switch (p.Mfft) {
    case 16: run_box<T, 16>(p, src, src_plain, dst, dst_plain, st); break;
    case 32: run_box<T, 32>(p, src, src_plain, dst, dst_plain, st); break;
    case 64: run_box<T, 64>(p, src, src_plain, dst, dst_plain, st); break;
    case 128: run_box<T, 128>(p, src, src_plain, dst, dst_plain, st); break;
    case 256: run_box<T, 256>(p, src, src_plain, dst, dst_plain, st); break;
    case 512: run_box<T, 512>(p, src, src_plain, dst, dst_plain, st); break;
    case 1024: run_box<T, 1024>(p, src, src_plain, dst, dst_plain, st); break;
    default: throw std::invalid_argument("unsupported grid size");
  }
}

template void box_solve<double>(DevProblem &, const double *, bool, double *, bool, hipStream_t);
template void box_solve<float>(DevProblem &, const float *, bool, float *, bool, hipStream_t);

template <typename T>
void box_solve_stencils(DevProblem &p, const T *src, hipStream_t st) {
  if (p.dim != 3 || !p.sparse) {
    box_solve<T>(p, src, false, p.tab<T>().work, false, st);
    return;
  }
  switch (p.Mfft) {
    case 16: run_box_stencils<T, 16>(p, src, st); break;
    case 32: run_box_stencils<T, 32>(p, src, st); break;
    case 64: run_box_stencils<T, 64>(p, src, st); break;
    case 128: run_box_stencils<T, 128>(p, src, st); break;
    case 256: run_box_stencils<T, 256>(p, src, st); break;
    case 512: run_box_stencils<T, 512>(p, src, st); break;
    case 1024: run_box_stencils<T, 1024>(p, src, st); break;
    default: throw std::invalid_argument("unsupported grid size");
  }
}
template void box_solve_stencils<double>(DevProblem &, const double *, hipStream_t);

void bidomain_volume_solve(DevProblem &p, const FhnArgs &a, hipStream_t st) {
  switch (p.Mfft) {
    case 16: run_bidomain_volume<16>(p, a, st); break;
    case 32: run_bidomain_volume<32>(p, a, st); break;
    case 64: run_bidomain_volume<64>(p, a, st); break;
    case 128: run_bidomain_volume<128>(p, a, st); break;
    case 256: run_bidomain_volume<256>(p, a, st); break;
    case 512: run_bidomain_volume<512>(p, a, st); break;
    case 1024: run_bidomain_volume<1024>(p, a, st); break;
    default: throw std::invalid_argument("unsupported grid size");
  }
}

void bidomain_final_solve(DevProblem &p, const FhnArgs &a, bool fuse_be, hipStream_t st) {
  switch (p.Mfft) {
    case 16: run_bidomain_final<16>(p, a, fuse_be, st); break;
    case 32: run_bidomain_final<32>(p, a, fuse_be, st); break;
    case 64: run_bidomain_final<64>(p, a, fuse_be, st); break;
    case 128: run_bidomain_final<128>(p, a, fuse_be, st); break;
    case 256: run_bidomain_final<256>(p, a, fuse_be, st); break;
    case 512: run_bidomain_final<512>(p, a, fuse_be, st); break;
    case 1024: run_bidomain_final<1024>(p, a, fuse_be, st); break;
    default: throw std::invalid_argument("unsupported grid size");
  }
}

template <typename T>
void box_solve_matvec(DevProblem &p, hipStream_t st) {
  if (p.dim != 3 || !p.sparse) {
    box_solve<T>(p, p.tab<T>().rhs, false, p.tab<T>().work, false, st);
    return;
  }
  switch (p.Mfft) {
    case 16: run_box_sparse<T, 16>(p, st); break;
    case 32: run_box_sparse<T, 32>(p, st); break;
    case 64: run_box_sparse<T, 64>(p, st); break;
    case 128: run_box_sparse<T, 128>(p, st); break;
    case 256: run_box_sparse<T, 256>(p, st); break;
    case 512: run_box_sparse<T, 512>(p, st); break;
    case 1024: run_box_sparse<T, 1024>(p, st); break;
    default: throw std::invalid_argument("unsupported grid size");
  }
}
template void box_solve_matvec<double>(DevProblem &, hipStream_t);
template void box_solve_matvec<float>(DevProblem &, hipStream_t);

}  // namespace kfbi
