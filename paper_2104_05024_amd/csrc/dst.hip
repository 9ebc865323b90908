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

__device__ __forceinline__ int pad(int i) { return i + (i >> 3); }

template <int M>
struct Shape {
  static constexpr int N = M - 1;
  static constexpr int TPP = M / 16;       // threads per pencil pair
  static constexpr int NP = 2048 / M;      // pencil pairs per workgroup
  static constexpr int NT = NP * TPP;      // threads per workgroup (128)
  static constexpr int PADM = M + M / 8;   // padded LDS length of one pair
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
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + TPP * b;
    const int k = j & (Ns - 1);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[pad(base + r * Ns)] = v[b * R + r];
  }
  __syncthreads();
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

// DST-I (unnormalised: y_k = sum_n x_n sin(pi n k / M)) of one pencil pair held in LDS as
// complex values at positions 1..N; result at the same positions.  All threads of the
// workgroup must call it (it contains barriers).
template <typename T, int M>
__device__ __forceinline__ void dst_pair(C2<T> *buf, int lane, const C2<T> *__restrict__ tw,
                                         const T *__restrict__ sp) {
  constexpr int TPP = M / 16;
  // pre-processing: (n, M-n) pairs are owned by one thread, so no barrier inside
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int n = 1 + lane + TPP * i;
    const C2<T> a = buf[pad(n)], b = buf[pad(M - n)];
    const T s = sp[n];
    const C2<T> sum = s * (a + b), dif = (T)0.5 * (a - b);
    buf[pad(n)] = sum + dif;
    buf[pad(M - n)] = sum - dif;
  }
  if (lane == 0) buf[pad(0)] = {0, 0};
  __syncthreads();
  fft_stages<T, M, 1>(buf, lane, tw);
  // post-processing: lane owns k in [8 lane, 8 lane + 8)
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
    const C2<T> y = {shfl_up_w(inc.x, off, TPP), shfl_up_w(inc.y, off, TPP)};
    if (lane >= off) inc = inc + y;
  }
  const C2<T> excl = inc - tot;
  const C2<T> E0 = {shfl_w(e0.x, 0, TPP), shfl_w(e0.y, 0, TPP)};
  const C2<T> half0 = (T)0.5 * E0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = 8 * lane + i;
    if (k > 0) buf[pad(2 * k)] = ev[i];
    buf[pad(2 * k + 1)] = (excl + od[i]) - half0;
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T &lane_of(C2<T> &c, int which) {
  return which ? c.y : c.x;
}

// ---------------------------------------------------------------- pass kernels

// DST along contiguous rows: pairs of consecutive rows of the flattened [comp][..][x] list.
template <typename T, int M>
__global__ __launch_bounds__(Shape<M>::NT) void k_dst_x(const T *__restrict__ in, int64_t in_pitch,
                                                          T *__restrict__ out, int64_t out_pitch, int64_t nrows,
                                                          const C2<T> *__restrict__ tw, const T *__restrict__ sp) {
  using Sh = Shape<M>;
  constexpr int N = Sh::N, NP = Sh::NP, NT = Sh::NT, PADM = Sh::PADM;
  __shared__ C2<T> sbuf[NP * PADM];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 2 * NP;
  for (int e = tid; e < 2 * NP * N; e += NT) {
    const int rr = e / N, n = e - rr * N;
    const int64_t row = r0 + rr;
    const T v = row < nrows ? in[row * in_pitch + n] : T(0);
    lane_of(sbuf[(rr >> 1) * PADM + pad(n + 1)], rr & 1) = v;
  }
  __syncthreads();
  dst_pair<T, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, tw, sp);
  for (int e = tid; e < 2 * NP * N; e += NT) {
    const int rr = e / N, n = e - rr * N;
    const int64_t row = r0 + rr;
    if (row < nrows) out[row * out_pitch + n] = lane_of(sbuf[(rr >> 1) * PADM + pad(n + 1)], rr & 1);
  }
}

// DST along y (3D, in place): tile = 2 NP consecutive x columns of one (comp, z) plane.
template <typename T, int M>
__global__ __launch_bounds__(Shape<M>::NT) void k_dst_y(T *__restrict__ a, int64_t P, int64_t comp_stride,
                                                          const C2<T> *__restrict__ tw, const T *__restrict__ sp) {
  using Sh = Shape<M>;
  constexpr int N = Sh::N, NP = Sh::NP, NT = Sh::NT, PADM = Sh::PADM, TX = 2 * NP;
  __shared__ C2<T> sbuf[NP * PADM];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, z = blockIdx.y, c = blockIdx.z;
  T *base = a + c * comp_stride + (int64_t)z * N * P;
  for (int e = tid; e < N * TX; e += NT) {
    const int y = e / TX, xo = e - y * TX, x = x0 + xo;
    lane_of(sbuf[(xo >> 1) * PADM + pad(y + 1)], xo & 1) = x < N ? base[(int64_t)y * P + x] : T(0);
  }
  __syncthreads();
  dst_pair<T, M>(sbuf + (tid / Sh::TPP) * PADM, tid % Sh::TPP, tw, sp);
  for (int e = tid; e < N * TX; e += NT) {
    const int y = e / TX, xo = e - y * TX, x = x0 + xo;
    if (x < N) base[(int64_t)y * P + x] = lane_of(sbuf[(xo >> 1) * PADM + pad(y + 1)], xo & 1);
  }
}

struct ModeScale {
  const double *lam;   // (4/h^2) sin^2(k pi / 2M), k = 1..N
  double D0, D1, kappa, norm;
};

// Last axis (z in 3D, y in 2D), fused: forward DST -> mode solve -> inverse DST, in place.
// ncomp = 2: a pencil pair is (comp 0, comp 1) of one column; ncomp = 1: two adjacent columns.
template <typename T, int M, int NC, int DIM>
__global__ __launch_bounds__(Shape<M>::NT) void k_dst_last(T *__restrict__ a, int64_t P, int64_t comp_stride,
                                                             ModeScale ms, const C2<T> *__restrict__ tw,
                                                             const T *__restrict__ sp) {
  using Sh = Shape<M>;
  constexpr int N = Sh::N, NP = Sh::NP, NT = Sh::NT, PADM = Sh::PADM;
  constexpr int TX = NC == 2 ? NP : 2 * NP;          // columns per tile
  constexpr int64_t LS = DIM == 3 ? (int64_t)N : 1;  // rows of the last axis step by LS * P
  __shared__ C2<T> sbuf[NP * PADM];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, y = DIM == 3 ? (int)blockIdx.y : 0;
  T *base = a + (DIM == 3 ? (int64_t)y * P : 0);
  for (int e = tid; e < N * TX * NC; e += NT) {
    int rest = e;
    const int xo = rest % TX;
    rest /= TX;
    const int c = NC == 2 ? rest % 2 : 0;
    const int zz = NC == 2 ? rest / 2 : rest;
    const int x = x0 + xo;
    const T v = x < N ? base[c * comp_stride + (int64_t)zz * LS * P + x] : T(0);
    if (NC == 2)
      lane_of(sbuf[xo * PADM + pad(zz + 1)], c) = v;
    else
      lane_of(sbuf[(xo >> 1) * PADM + pad(zz + 1)], xo & 1) = v;
  }
  __syncthreads();
  C2<T> *mine = sbuf + (tid / Sh::TPP) * PADM;
  const int lane = tid % Sh::TPP;
  dst_pair<T, M>(mine, lane, tw, sp);
  // mode solve: pair p, position m (= mode index along the last axis)
  for (int e = tid; e < NP * N; e += NT) {
    const int pr = e / N, m = e - pr * N + 1;
    C2<T> &v = sbuf[pr * PADM + pad(m)];
    const double lyz = (DIM == 3 ? ms.lam[y] : 0.0) + ms.lam[m - 1];
    if (NC == 2) {
      const int x = x0 + pr;
      const double L = ms.lam[x < N ? x : 0] + lyz;
      const double ai = ms.D0 * L, ae = ms.D1 * L, k = ms.kappa;
      const double det = ai * ae + k * (ai + ae);
      const double fi = (double)v.x, fe = (double)v.y;
      const double s = ms.norm / det;
      v.x = (T)(s * ((ae + k) * fi + k * fe));
      v.y = (T)(s * (k * fi + (ai + k) * fe));
    } else {
      const int xa = x0 + 2 * pr, xb = xa + 1;
      const double La = ms.lam[xa < N ? xa : 0] + lyz, Lb = ms.lam[xb < N ? xb : 0] + lyz;
      v.x = (T)((double)v.x * ms.norm / (ms.D0 * La + ms.kappa));
      v.y = (T)((double)v.y * ms.norm / (ms.D0 * Lb + ms.kappa));
    }
  }
  __syncthreads();
  dst_pair<T, M>(mine, lane, tw, sp);
  for (int e = tid; e < N * TX * NC; e += NT) {
    int rest = e;
    const int xo = rest % TX;
    rest /= TX;
    const int c = NC == 2 ? rest % 2 : 0;
    const int zz = NC == 2 ? rest / 2 : rest;
    const int x = x0 + xo;
    if (x < N)
      base[c * comp_stride + (int64_t)zz * LS * P + x] =
          NC == 2 ? lane_of(sbuf[xo * PADM + pad(zz + 1)], c) : lane_of(sbuf[(xo >> 1) * PADM + pad(zz + 1)], xo & 1);
  }
}

template <typename T, int M>
void run_box(DevProblem &p, const T *src, bool src_plain, T *dst, bool dst_plain, hipStream_t st) {
  using Sh = Shape<M>;
  constexpr int N = Sh::N;
  PrecTables<T> &tb = p.tab<T>();
  T *A = tb.work;
  const C2<T> *tw = reinterpret_cast<const C2<T> *>(tb.tw);
  const T *sp = tb.sp;
  const int64_t P = p.P, cs = p.comp_stride;
  const int64_t rows = (int64_t)p.ncomp * (p.dim == 3 ? (int64_t)N * N : N);
  const dim3 gx((unsigned)((rows + 2 * Sh::NP - 1) / (2 * Sh::NP)));
  ModeScale ms{p.lam, p.sigma[0], p.ncomp == 2 ? p.sigma[1] : p.sigma[0], p.kappa, p.lam_scale};
  auto tic = [&](Timer &t) {
    if (p.profile) KFBI_HIP(hipEventRecord(t.a, st));
  };
  auto toc = [&](Timer &t) {
    if (p.profile) {
      KFBI_HIP(hipEventRecord(t.b, st));
      KFBI_HIP(hipEventSynchronize(t.b));
      float ms_ = 0;
      KFBI_HIP(hipEventElapsedTime(&ms_, t.a, t.b));
      t.total_ms += ms_;
      t.n += 1;
    }
  };
  tic(p.t_dst_x);
  k_dst_x<T, M><<<gx, Sh::NT, 0, st>>>(src, src_plain ? N : P, A, P, rows, tw, sp);
  KFBI_HIP(hipGetLastError());
  toc(p.t_dst_x);
  const dim3 gy((N + 2 * Sh::NP - 1) / (2 * Sh::NP), N, p.ncomp);
  if (p.dim == 3) {
    tic(p.t_dst_y);
    k_dst_y<T, M><<<gy, Sh::NT, 0, st>>>(A, P, cs, tw, sp);
    KFBI_HIP(hipGetLastError());
    toc(p.t_dst_y);
  }
  const int tx = p.ncomp == 2 ? Sh::NP : 2 * Sh::NP;
  const dim3 gl((N + tx - 1) / tx, p.dim == 3 ? N : 1, 1);
  tic(p.t_dst_last);
  if (p.dim == 3) {
    if (p.ncomp == 2) k_dst_last<T, M, 2, 3><<<gl, Sh::NT, 0, st>>>(A, P, cs, ms, tw, sp);
    else k_dst_last<T, M, 1, 3><<<gl, Sh::NT, 0, st>>>(A, P, cs, ms, tw, sp);
  } else {
    if (p.ncomp == 2) k_dst_last<T, M, 2, 2><<<gl, Sh::NT, 0, st>>>(A, P, cs, ms, tw, sp);
    else k_dst_last<T, M, 1, 2><<<gl, Sh::NT, 0, st>>>(A, P, cs, ms, tw, sp);
  }
  KFBI_HIP(hipGetLastError());
  toc(p.t_dst_last);
  if (p.dim == 3) {
    tic(p.t_dst_y);
    k_dst_y<T, M><<<gy, Sh::NT, 0, st>>>(A, P, cs, tw, sp);
    KFBI_HIP(hipGetLastError());
    toc(p.t_dst_y);
  }
  tic(p.t_dst_x);
  k_dst_x<T, M><<<gx, Sh::NT, 0, st>>>(A, P, dst, dst_plain ? N : P, rows, tw, sp);
  KFBI_HIP(hipGetLastError());
  toc(p.t_dst_x);
}

}  // namespace

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

}  // namespace kfbi
