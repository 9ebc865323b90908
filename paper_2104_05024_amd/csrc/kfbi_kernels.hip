// Interface-side kernels of the KFBI matrix-vector product and the table upload.
//
//  k_jumps_cross : density -> jumps [u_a], [u_aa] at every grid-line intersection
//                  (single-layer interface problem, Sec. 5.1 eq. single; jump relations
//                  from [u] = 0 and [n.D grad u] = psi for isotropic D_c).
//  k_jumps_nodes : density -> [grad u] and [Hess u] at every interface node.
//  k_correct     : right-hand-side correction at irregular grid nodes (Sec. 5.3, eq.
//                  correct): rhs_p = D_c sum_arms s_p/h^2 ([u_a] d + [u_aa] d^2 / 2).
//                  One thread owns one irregular node, so no atomics are needed.
//  k_gather      : n.D grad u+ at every interface node from its 6/10-node quadratic fit,
//                  adding the Taylor-expanded jump to values on the "-" side
//                  (Sec. 5.4, eqs. taylor-i-po, taylor-i-co, ji).
#include <cmath>
#include <stdexcept>

#include "device.h"

namespace kfbi {
namespace {

constexpr int kBlock = 256;

// All stencil sizes are compile-time constants so that every index load of a thread is
// issued before the dependent gathers (the kernels are latency-bound, not bandwidth-bound).
template <typename T, int D, int K>
__device__ __forceinline__ void jumps_cross_at(int64_t c, const T *__restrict__ psi, int64_t M, int64_t nc,
                                               const int32_t *__restrict__ z_idx, const T *__restrict__ z_w0,
                                               const T *__restrict__ z_wga, const T *__restrict__ z_na,
                                               const T *__restrict__ z_cw, int ncomp, T is0, T is1,
                                               T *__restrict__ jz) {
  int32_t j[K];
  T w[K], wg[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    j[k] = z_idx[k * nc + c];
    w[k] = z_w0[k * nc + c];
    wg[k] = z_wga[k * nc + c];
  }
  const T na = z_na[c], cw = z_cw[c];
  for (int comp = 0; comp < ncomp; ++comp) {
    const T *ps = psi + comp * M;
    T v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = ps[j[k]];
    T pz = 0, ga = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      pz += w[k] * v[k];
      ga += wg[k] * v[k];
    }
    const T is = comp == 0 ? is0 : is1;
    const T a = pz * is;
    jz[(2 * comp) * nc + c] = a * na;
    jz[(2 * comp + 1) * nc + c] = a * cw + (T)2 * na * ga * is;
  }
}

template <typename T, int D, int K>
__global__ __launch_bounds__(kBlock) void k_jumps_cross(const T *__restrict__ psi, int64_t M, int64_t nc,
                                                        const int32_t *__restrict__ z_idx,
                                                        const T *__restrict__ z_w0, const T *__restrict__ z_wga,
                                                        const T *__restrict__ z_na, const T *__restrict__ z_cw,
                                                        int ncomp, T is0, T is1, T *__restrict__ jz) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) jumps_cross_at<T, D, K>(c, psi, M, nc, z_idx, z_w0, z_wga, z_na, z_cw, ncomp, is0, is1, jz);
}

// One thread per irregular node; at most 2D arms, loaded predicated and all at once.
template <typename T, int D>
__device__ __forceinline__ void correct_at(int64_t r, const int32_t *__restrict__ irr_pos,
                                           const int32_t *__restrict__ irr_ptr, const int32_t *__restrict__ arm_cross,
                                           const T *__restrict__ arm_d, const T *__restrict__ arm_s,
                                           const T *__restrict__ jz, int64_t nc, int ncomp, T D0, T D1,
                                           T *__restrict__ rhs, int64_t comp_stride, int accumulate) {
  constexpr int MAXA = 2 * D;
  const int32_t b = irr_ptr[r], e = irr_ptr[r + 1];
  const int64_t pos = irr_pos[r];
  int32_t cr[MAXA];
  T d[MAXA], sg[MAXA];
#pragma unroll
  for (int i = 0; i < MAXA; ++i) {
    const bool ok = b + i < e;
    cr[i] = ok ? arm_cross[b + i] : 0;
    d[i] = ok ? arm_d[b + i] : T(0);
    sg[i] = ok ? arm_s[b + i] : T(0);
  }
  for (int comp = 0; comp < ncomp; ++comp) {
    T du[MAXA], duu[MAXA];
#pragma unroll
    for (int i = 0; i < MAXA; ++i) {
      du[i] = jz[(2 * comp) * nc + cr[i]];
      duu[i] = jz[(2 * comp + 1) * nc + cr[i]];
    }
    T acc = 0;
#pragma unroll
    for (int i = 0; i < MAXA; ++i) acc += sg[i] * (du[i] * d[i] + (T)0.5 * duu[i] * d[i] * d[i]);
    T *o = rhs + comp * comp_stride + pos;
    const T val = (comp == 0 ? D0 : D1) * acc;
    if (accumulate)
      *o += val;
    else
      *o = val;
  }
}

template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_correct(int64_t nirr, const int32_t *__restrict__ irr_pos,
                                                    const int32_t *__restrict__ irr_ptr,
                                                    const int32_t *__restrict__ arm_cross,
                                                    const T *__restrict__ arm_d, const T *__restrict__ arm_s,
                                                    const T *__restrict__ jz, int64_t nc, int ncomp, T D0, T D1,
                                                    T *__restrict__ rhs, int64_t comp_stride, int accumulate) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nirr)
    correct_at<T, D>(r, irr_pos, irr_ptr, arm_cross, arm_d, arm_s, jz, nc, ncomp, D0, D1, rhs, comp_stride,
                     accumulate);
}

template <int D>
struct NH {
  static constexpr int v = D == 2 ? 3 : 6;   // symmetric entries: xx yy (zz) xy (xz yz)
};

template <int D>
__device__ __forceinline__ void sym_index(int e, int &a, int &b) {
  if (D == 2) {
    a = e == 1 ? 1 : 0;
    b = e == 0 ? 0 : 1;
  } else {
    a = e < 3 ? e : (e == 5 ? 1 : 0);
    b = e < 3 ? e : (e == 3 ? 1 : 2);
  }
}

template <typename T, int D, int KN>
__device__ __forceinline__ void jumps_nodes_at(int64_t q, const T *__restrict__ psi, int64_t M,
                                               const int32_t *__restrict__ q_idx, const T *__restrict__ q_wg,
                                               const T *__restrict__ q_n, const T *__restrict__ q_wt, int ncomp,
                                               T is0, T is1, T *__restrict__ jq) {
  constexpr int NHv = NH<D>::v, STR = D + NHv;
  int32_t j[KN];
#pragma unroll
  for (int k = 0; k < KN; ++k) j[k] = q_idx[k * M + q];
  T n[D], wt[NHv];
#pragma unroll
  for (int a = 0; a < D; ++a) n[a] = q_n[a * M + q];
#pragma unroll
  for (int e = 0; e < NHv; ++e) wt[e] = q_wt[e * M + q];
  for (int comp = 0; comp < ncomp; ++comp) {
    const T *ps = psi + comp * M;
    const T is = comp == 0 ? is0 : is1;
    T v[KN];
#pragma unroll
    for (int k = 0; k < KN; ++k) v[k] = ps[j[k]];
    T g[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      g[a] = 0;
#pragma unroll
      for (int k = 0; k < KN; ++k) g[a] += q_wg[(k * D + a) * M + q] * v[k];
    }
    const T amp = ps[q] * is;
    T *o = jq + (int64_t)comp * STR * M;
#pragma unroll
    for (int a = 0; a < D; ++a) o[a * M + q] = amp * n[a];
#pragma unroll
    for (int e = 0; e < NHv; ++e) {
      int a, b;
      sym_index<D>(e, a, b);
      o[(D + e) * M + q] = amp * wt[e] + (n[a] * g[b] + g[a] * n[b]) * is;
    }
  }
}

template <typename T, int D, int KN>
__global__ __launch_bounds__(kBlock) void k_jumps_nodes(const T *__restrict__ psi, int64_t M,
                                                        const int32_t *__restrict__ q_idx,
                                                        const T *__restrict__ q_wg, const T *__restrict__ q_n,
                                                        const T *__restrict__ q_wt, int ncomp, T is0, T is1,
                                                        T *__restrict__ jq) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < M) jumps_nodes_at<T, D, KN>(q, psi, M, q_idx, q_wg, q_n, q_wt, ncomp, is0, is1, jq);
}

template <typename T, int D, int S>
__device__ __forceinline__ void gather_at(int64_t q, const T *__restrict__ u, int64_t comp_stride, int64_t M,
                                          const int32_t *__restrict__ st_pos, const T *__restrict__ st_nw,
                                          const T *__restrict__ st_r, const T *__restrict__ jq, int ncomp, T s0,
                                          T s1, int with_jumps, T *__restrict__ out) {
  constexpr int NHv = NH<D>::v, STR = D + NHv;
  int32_t pe[S];
  T nw[S];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    pe[j] = st_pos[j * M + q];
    nw[j] = st_nw[j * M + q];
  }
  for (int comp = 0; comp < ncomp; ++comp) {
    const T *uc = u + comp * comp_stride;
    T val[S];
#pragma unroll
    for (int j = 0; j < S; ++j) val[j] = uc[pe[j] < 0 ? -pe[j] - 1 : pe[j]];
    if (with_jumps) {
      const T *o = jq + (int64_t)comp * STR * M;
      T du[D], H[D][D];
#pragma unroll
      for (int a = 0; a < D; ++a) du[a] = o[a * M + q];
#pragma unroll
      for (int e = 0; e < NHv; ++e) {
        int a, b;
        sym_index<D>(e, a, b);
        H[a][b] = H[b][a] = o[(D + e) * M + q];
      }
#pragma unroll
      for (int j = 0; j < S; ++j) {
        if (pe[j] >= 0) continue;
        T r[D];
#pragma unroll
        for (int a = 0; a < D; ++a) r[a] = st_r[(j * D + a) * M + q];
        T J = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          T hr = 0;
#pragma unroll
          for (int b = 0; b < D; ++b) hr += H[a][b] * r[b];
          J += r[a] * (du[a] + (T)0.5 * hr);
        }
        val[j] += J;
      }
    }
    T acc = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) acc += nw[j] * val[j];
    out[comp * M + q] = (comp == 0 ? s0 : s1) * acc;
  }
}

template <typename T, int D, int S>
__global__ __launch_bounds__(kBlock) void k_gather(const T *__restrict__ u, int64_t comp_stride, int64_t M,
                                                   const int32_t *__restrict__ st_pos,
                                                   const T *__restrict__ st_nw, const T *__restrict__ st_r,
                                                   const T *__restrict__ jq, int ncomp, T s0, T s1, int with_jumps,
                                                   T *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < M) gather_at<T, D, S>(q, u, comp_stride, M, st_pos, st_nw, st_r, jq, ncomp, s0, s1, with_jumps, out);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Problem of a flattened batch item: the largest p with cum[p] <= i (cum[0] = 0 <= i < cum[n]).
__device__ __forceinline__ int batch_problem(const int64_t *__restrict__ cum, int n, int64_t i) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (cum[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Work list of one launch: all crossings of all problems, then all their nodes.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_jumps(const BatchItem<T> *__restrict__ items, BatchCounts c,
                                                        const T *__restrict__ psi) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < c.tot_nc) {
    const int p = batch_problem(c.cum_nc, c.n, i);
    const BatchItem<T> &it = items[p];
    jumps_cross_at<T, 2, 4>(i - c.cum_nc[p], psi + it.ioff, it.M, it.nc, it.z_idx, it.z_w0, it.z_wga, it.z_na,
                            it.z_cw, 1, it.isig, it.isig, it.jz);
    return;
  }
  i -= c.tot_nc;
  if (i >= c.tot_M) return;
  const int p = batch_problem(c.cum_M, c.n, i);
  const BatchItem<T> &it = items[p];
  jumps_nodes_at<T, 2, 5>(i - c.cum_M[p], psi + it.ioff, it.M, it.q_idx, it.q_wg, it.q_n, it.q_wt, 1, it.isig,
                          it.isig, it.jq);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_correct(const BatchItem<T> *__restrict__ items, BatchCounts c,
                                                          int target) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.tot_nirr) return;
  const int p = batch_problem(c.cum_nirr, c.n, i);
  const BatchItem<T> &it = items[p];
  correct_at<T, 2>(i - c.cum_nirr[p], it.irr_pos, it.irr_ptr, it.arm_cross, it.arm_d, it.arm_s, it.jz, it.nc, 1,
                   it.sigma, it.sigma, target ? it.fpad : it.rhs, 0, target);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_gather(const BatchItem<T> *__restrict__ items, BatchCounts c,
                                                         int with_jumps, T *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.tot_M) return;
  const int p = batch_problem(c.cum_M, c.n, i);
  const BatchItem<T> &it = items[p];
  gather_at<T, 2, 6>(i - c.cum_M[p], it.work, 0, it.M, it.st_pos, it.st_nw, it.st_r, it.jq, 1, it.sigma, it.sigma,
                     with_jumps, out + it.ioff);
}

template <typename T>
T *dalloc(size_t n) {
  T *p = nullptr;
  if (n == 0) n = 1;
  KFBI_HIP(hipMalloc(&p, n * sizeof(T)));
  return p;
}
template <typename T>
T *dupload(const std::vector<T> &v) {
  T *p = dalloc<T>(v.size());
  if (!v.empty()) KFBI_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}
template <typename T>
std::vector<T> cast_vec(const std::vector<double> &v) {
  return std::vector<T>(v.begin(), v.end());
}

template <typename T>
void upload_prec(DevProblem &p, PrecTables<T> &tb, const std::vector<double> &z_w0, const std::vector<double> &z_wga,
                 const std::vector<double> &z_na, const std::vector<double> &z_cw, const std::vector<double> &q_wg,
                 const std::vector<double> &q_n, const std::vector<double> &q_wt, const std::vector<double> &arm_d,
                 const std::vector<double> &arm_s, const std::vector<double> &st_nw, const std::vector<double> &st_r,
                 const std::vector<double> &tw, const std::vector<double> &sp) {
  tb.z_w0 = dupload(cast_vec<T>(z_w0));
  tb.z_wga = dupload(cast_vec<T>(z_wga));
  tb.z_na = dupload(cast_vec<T>(z_na));
  tb.z_cw = dupload(cast_vec<T>(z_cw));
  tb.q_wg = dupload(cast_vec<T>(q_wg));
  tb.q_n = dupload(cast_vec<T>(q_n));
  tb.q_wt = dupload(cast_vec<T>(q_wt));
  tb.arm_d = dupload(cast_vec<T>(arm_d));
  tb.arm_s = dupload(cast_vec<T>(arm_s));
  tb.st_nw = dupload(cast_vec<T>(st_nw));
  tb.st_r = dupload(cast_vec<T>(st_r));
  tb.tw = dupload(cast_vec<T>(tw));
  tb.sp = dupload(cast_vec<T>(sp));
  const size_t field = (size_t)p.ncomp * p.comp_stride;
  tb.rhs = dalloc<T>(field);
  tb.work = dalloc<T>(field);
  KFBI_HIP(hipMemset(tb.rhs, 0, field * sizeof(T)));
  KFBI_HIP(hipMemset(tb.work, 0, field * sizeof(T)));
  if (p.dim == 3) {
    tb.xbuf = dalloc<T>(field);
    KFBI_HIP(hipMemset(tb.xbuf, 0, field * sizeof(T)));
    tb.ybuf = dalloc<T>(field);
    KFBI_HIP(hipMemset(tb.ybuf, 0, field * sizeof(T)));
  }
  const int nh = p.dim == 2 ? 3 : 6;
  tb.jz = dalloc<T>((size_t)p.ncomp * 2 * std::max<int64_t>(p.nc, 1));
  tb.jq = dalloc<T>((size_t)p.ncomp * (p.dim + nh) * p.M);
}

template <typename T>
void free_prec(PrecTables<T> &tb) {
  T **all[] = {&tb.z_w0, &tb.z_wga, &tb.z_na, &tb.z_cw, &tb.q_wg, &tb.q_n, &tb.q_wt, &tb.arm_d, &tb.arm_s,
               &tb.st_nw, &tb.st_r, &tb.tw, &tb.sp, &tb.rhs, &tb.work, &tb.xbuf, &tb.ybuf, &tb.jz, &tb.jq};
  for (T **q : all) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
}

}  // namespace

template <typename T>
void launch_jumps(DevProblem &p, const T *psi, hipStream_t st) {
  PrecTables<T> &tb = p.tab<T>();
  const T is0 = (T)(1.0 / p.sigma[0]), is1 = (T)(1.0 / p.sigma[1]);
  if (p.nc > 0) {
    if (p.dim == 2)
      k_jumps_cross<T, 2, 4><<<nblk(p.nc), kBlock, 0, st>>>(psi, p.M, p.nc, p.z_idx, tb.z_w0, tb.z_wga, tb.z_na,
                                                           tb.z_cw, p.ncomp, is0, is1, tb.jz);
    else
      k_jumps_cross<T, 3, kLsqNodes><<<nblk(p.nc), kBlock, 0, st>>>(psi, p.M, p.nc, p.z_idx, tb.z_w0, tb.z_wga,
                                                                   tb.z_na, tb.z_cw, p.ncomp, is0, is1, tb.jz);
    KFBI_HIP(hipGetLastError());
  }
  if (p.dim == 2)
    k_jumps_nodes<T, 2, 5><<<nblk(p.M), kBlock, 0, st>>>(psi, p.M, p.q_idx, tb.q_wg, tb.q_n, tb.q_wt, p.ncomp,
                                                        is0, is1, tb.jq);
  else
    k_jumps_nodes<T, 3, kLsqNodes><<<nblk(p.M), kBlock, 0, st>>>(psi, p.M, p.q_idx, tb.q_wg, tb.q_n, tb.q_wt,
                                                                p.ncomp, is0, is1, tb.jq);
  KFBI_HIP(hipGetLastError());
}

template <typename T>
static void correct_into(DevProblem &p, T *field, int accumulate, hipStream_t st) {
  PrecTables<T> &tb = p.tab<T>();
  if (p.nirr == 0) return;
  if (p.dim == 2)
    k_correct<T, 2><<<nblk(p.nirr), kBlock, 0, st>>>(p.nirr, p.irr_pos, p.irr_ptr, p.arm_cross, tb.arm_d, tb.arm_s,
                                                    tb.jz, p.nc, p.ncomp, (T)p.sigma[0], (T)p.sigma[1], field,
                                                    p.comp_stride, accumulate);
  else
    k_correct<T, 3><<<nblk(p.nirr), kBlock, 0, st>>>(p.nirr, p.irr_pos, p.irr_ptr, p.arm_cross, tb.arm_d, tb.arm_s,
                                                    tb.jz, p.nc, p.ncomp, (T)p.sigma[0], (T)p.sigma[1], field,
                                                    p.comp_stride, accumulate);
  KFBI_HIP(hipGetLastError());
}

template <typename T>
void launch_correct(DevProblem &p, hipStream_t st) {
  correct_into<T>(p, p.tab<T>().rhs, 0, st);
}

template <typename T>
void launch_add_correction(DevProblem &p, T *field_padded, hipStream_t st) {
  correct_into<T>(p, field_padded, 1, st);
}

template <typename T>
void launch_gather(DevProblem &p, const T *u, bool with_jumps, T *out, hipStream_t st) {
  PrecTables<T> &tb = p.tab<T>();
  const T s0 = (T)p.sigma[0], s1 = (T)p.sigma[1];
  if (p.dim == 2)
    k_gather<T, 2, 6><<<nblk(p.M), kBlock, 0, st>>>(u, p.comp_stride, p.M, p.st_pos, tb.st_nw, tb.st_r, tb.jq,
                                                   p.ncomp, s0, s1, with_jumps ? 1 : 0, out);
  else
    k_gather<T, 3, 10><<<nblk(p.M), kBlock, 0, st>>>(u, p.comp_stride, p.M, p.st_pos, tb.st_nw, tb.st_r, tb.jq,
                                                    p.ncomp, s0, s1, with_jumps ? 1 : 0, out);
  KFBI_HIP(hipGetLastError());
}

template <typename T>
void launch_batch_jumps(const BatchItem<T> *items, const BatchCounts &c, const T *psi, hipStream_t st) {
  const int64_t n = c.tot_nc + c.tot_M;
  if (n == 0) return;
  k_batch_jumps<T><<<nblk(n), kBlock, 0, st>>>(items, c, psi);
  KFBI_HIP(hipGetLastError());
}
template <typename T>
void launch_batch_correct(const BatchItem<T> *items, const BatchCounts &c, int target, hipStream_t st) {
  if (c.tot_nirr == 0) return;
  k_batch_correct<T><<<nblk(c.tot_nirr), kBlock, 0, st>>>(items, c, target);
  KFBI_HIP(hipGetLastError());
}
template <typename T>
void launch_batch_gather(const BatchItem<T> *items, const BatchCounts &c, bool with_jumps, T *out, hipStream_t st) {
  if (c.tot_M == 0) return;
  k_batch_gather<T><<<nblk(c.tot_M), kBlock, 0, st>>>(items, c, with_jumps ? 1 : 0, out);
  KFBI_HIP(hipGetLastError());
}
template void launch_batch_jumps<double>(const BatchItem<double> *, const BatchCounts &, const double *, hipStream_t);
template void launch_batch_jumps<float>(const BatchItem<float> *, const BatchCounts &, const float *, hipStream_t);
template void launch_batch_correct<double>(const BatchItem<double> *, const BatchCounts &, int, hipStream_t);
template void launch_batch_correct<float>(const BatchItem<float> *, const BatchCounts &, int, hipStream_t);
template void launch_batch_gather<double>(const BatchItem<double> *, const BatchCounts &, bool, double *,
                                          hipStream_t);
template void launch_batch_gather<float>(const BatchItem<float> *, const BatchCounts &, bool, float *, hipStream_t);

template void launch_jumps<double>(DevProblem &, const double *, hipStream_t);
template void launch_jumps<float>(DevProblem &, const float *, hipStream_t);
template void launch_correct<double>(DevProblem &, hipStream_t);
template void launch_correct<float>(DevProblem &, hipStream_t);
template void launch_add_correction<double>(DevProblem &, double *, hipStream_t);
template void launch_add_correction<float>(DevProblem &, float *, hipStream_t);
template void launch_gather<double>(DevProblem &, const double *, bool, double *, hipStream_t);
template void launch_gather<float>(DevProblem &, const float *, bool, float *, hipStream_t);

void upload_tables(DevProblem &p) {
  const HostTables &t = p.ht;
  const int d = t.dim;
  p.dim = d;
  p.ncomp = t.ncomp;
  p.N = t.N;
  p.M = t.M;
  p.Mfft = t.cells;
  p.P = t.cells;
  p.comp_stride = p.P * (d == 3 ? p.N * p.N : p.N);
  p.nc = t.nc;
  p.nirr = (int64_t)t.irregular.size();
  p.K = t.K;
  p.Kn = t.Kn;
  p.S = t.S;
  p.h = t.h;
  p.kappa = t.kappa;
  p.sigma[0] = t.D[0][0];
  p.sigma[1] = t.ncomp == 2 ? t.D[1][0] : t.D[0][0];
  p.lam_scale = 1.0;
  for (int a = 0; a < d; ++a) p.lam_scale *= 2.0 / (double)t.cells;
  const int64_t N = p.N, M = p.M, nc = p.nc, P = p.P;
  auto padpos = [&](int64_t lin) { return (lin % N) + P * (lin / N); };
  if (padpos(N * (d == 3 ? N * N : N) - 1) >= (int64_t)1 << 31) throw std::invalid_argument("grid too large");

  // crossings (SoA)
  std::vector<int32_t> z_idx(nc * t.K), z_axis(nc);
  std::vector<double> z_w0(nc * t.K), z_wga(nc * t.K), z_na(nc), z_cw(nc);
  for (int64_t c = 0; c < nc; ++c) {
    const int a = (int)t.c_axis[c];
    z_axis[c] = a;
    const double *n = &t.c_n[c * d], *W = &t.c_W[c * d * d];
    double tr = 0;
    for (int b = 0; b < d; ++b) tr += W[b * d + b];
    z_na[c] = n[a];
    z_cw[c] = W[a * d + a] - tr * n[a] * n[a];
    for (int k = 0; k < t.K; ++k) {
      z_idx[k * nc + c] = (int32_t)t.z_idx[c * t.K + k];
      z_w0[k * nc + c] = t.z_w0[c * t.K + k];
      z_wga[k * nc + c] = t.z_wg[(c * t.K + k) * d + a];
    }
  }
  // correction records: CSR over irregular nodes
  std::vector<std::vector<int64_t>> arms_of(t.irregular.size());
  auto rank = [&](int64_t lin) {
    return (int64_t)(std::lower_bound(t.irregular.begin(), t.irregular.end(), lin) - t.irregular.begin());
  };
  for (int64_t c = 0; c < nc; ++c) {
    arms_of[rank(t.c_pin[c])].push_back(2 * c);       // tissue-side node, s = +1
    arms_of[rank(t.c_pout[c])].push_back(2 * c + 1);  // "-"-side node, s = -1
  }
  std::vector<int32_t> irr_pos(t.irregular.size()), irr_ptr(t.irregular.size() + 1, 0), arm_cross;
  std::vector<double> arm_d, arm_s;
  const double ih2 = 1.0 / (t.h * t.h);
  auto coord = [&](int64_t lin, int a) {
    int64_t r = lin;
    for (int b = 0; b < a; ++b) r /= N;
    return t.lo + t.h * (double)(r % N + 1);
  };
  for (size_t r = 0; r < t.irregular.size(); ++r) {
    irr_pos[r] = (int32_t)padpos(t.irregular[r]);
    for (int64_t code : arms_of[r]) {
      const int64_t c = code / 2;
      const bool plus = (code % 2) == 0;
      const int a = (int)t.c_axis[c];
      const int64_t nb = plus ? t.c_pout[c] : t.c_pin[c];
      arm_cross.push_back((int32_t)c);
      arm_d.push_back(coord(nb, a) - t.c_z[c * d + a]);
      arm_s.push_back(plus ? ih2 : -ih2);
    }
    irr_ptr[r + 1] = (int32_t)arm_cross.size();
  }
  p.narm = (int64_t)arm_cross.size();
  // node jumps
  const int nh = d == 2 ? 3 : 6;
  std::vector<int32_t> q_idx(M * t.Kn);
  std::vector<double> q_wg(M * t.Kn * d), q_n(M * d), q_wt(M * nh);
  const int SA[6] = {0, 1, 2, 0, 0, 1}, SB[6] = {0, 1, 2, 1, 2, 2};
  const int SA2[3] = {0, 1, 0}, SB2[3] = {0, 1, 1};
  for (int64_t q = 0; q < M; ++q) {
    const double *n = &t.nrm[q * d], *W = &t.W[q * d * d];
    double tr = 0;
    for (int b = 0; b < d; ++b) tr += W[b * d + b];
    for (int a = 0; a < d; ++a) q_n[a * M + q] = n[a];
    for (int e = 0; e < nh; ++e) {
      const int a = d == 2 ? SA2[e] : SA[e], b = d == 2 ? SB2[e] : SB[e];
      q_wt[e * M + q] = W[a * d + b] - tr * n[a] * n[b];
    }
    for (int k = 0; k < t.Kn; ++k) {
      q_idx[k * M + q] = (int32_t)t.q_idx[q * t.Kn + k];
      for (int a = 0; a < d; ++a) q_wg[(k * d + a) * M + q] = t.q_wg[(q * t.Kn + k) * d + a];
    }
  }
  // gather stencils
  std::vector<int32_t> st_pos(M * t.S);
  std::vector<double> st_nw(M * t.S), st_r(M * t.S * d);
  for (int64_t q = 0; q < M; ++q)
    for (int j = 0; j < t.S; ++j) {
      const int64_t pos = padpos(t.st_lin[q * t.S + j]);
      st_pos[j * M + q] = t.st_chi[q * t.S + j] ? (int32_t)(-pos - 1) : (int32_t)pos;
      double nw = 0;
      for (int a = 0; a < d; ++a) {
        nw += t.nrm[q * d + a] * t.st_wgrad[(q * t.S + j) * d + a];
        st_r[(j * d + a) * M + q] = t.st_r[(q * t.S + j) * d + a];
      }
      st_nw[j * M + q] = nw;
    }
  // DST tables
  const int Mf = p.Mfft;
  std::vector<double> tw(2 * Mf), sp(Mf / 2 + 1), lam(N);
  for (int m = 0; m < Mf; ++m) {
    const double ang = -2.0 * M_PI * (double)m / (double)Mf;
    tw[2 * m] = std::cos(ang);
    tw[2 * m + 1] = std::sin(ang);
  }
  for (int n = 0; n <= Mf / 2; ++n) sp[n] = std::sin(M_PI * (double)n / (double)Mf);
  for (int64_t k = 1; k <= N; ++k) {
    const double s = std::sin((double)k * M_PI / (2.0 * Mf));
    lam[k - 1] = 4.0 / (t.h * t.h) * s * s;
  }
  // tissue mask in the padded layout
  std::vector<int8_t> ins_pad((size_t)p.comp_stride, 0);
  for (int64_t lin = 0; lin < (int64_t)t.inside.size(); ++lin) ins_pad[padpos(lin)] = t.inside[lin];

  // sparse matvec rows: irregular-node rows (right-hand side) and stencil rows (output)
  if (d == 3) {
    std::vector<uint8_t> min_(N * N, 0), mout(N * N, 0);
    for (int64_t lin : t.irregular) min_[lin / N] = 1;
    for (int64_t lin : t.st_lin) mout[lin / N] = 1;
    std::vector<int32_t> rin, rout;
    for (int c = 0; c < t.ncomp; ++c)
      for (int64_t r = 0; r < N * N; ++r) {
        if (min_[r]) rin.push_back((int32_t)(c * N * N + r));
        if (mout[r]) rout.push_back((int32_t)(c * N * N + r));
      }
    p.n_rows_in = (int64_t)rin.size();
    p.n_rows_out = (int64_t)rout.size();
    p.rows_in = dupload(rin);
    p.rows_out = dupload(rout);
    p.mask_in = dupload(min_);
    p.mask_out = dupload(mout);
    std::vector<uint8_t> pin(N, 0), pout(N, 0);
    for (int64_t r = 0; r < N * N; ++r) {
      if (min_[r]) pin[r / N] = 1;
      if (mout[r]) pout[r / N] = 1;
    }
    p.planes_in = dupload(pin);
    p.planes_out = dupload(pout);
  }
  p.z_idx = dupload(z_idx);
  p.z_axis = dupload(z_axis);
  p.q_idx = dupload(q_idx);
  p.irr_pos = dupload(irr_pos);
  p.irr_ptr = dupload(irr_ptr);
  p.arm_cross = dupload(arm_cross);
  p.st_pos = dupload(st_pos);
  p.inside_pad = dupload(ins_pad);
  p.lam = dupload(lam);
  upload_prec<double>(p, p.f64, z_w0, z_wga, z_na, z_cw, q_wg, q_n, q_wt, arm_d, arm_s, st_nw, st_r, tw, sp);
  upload_prec<float>(p, p.f32, z_w0, z_wga, z_na, z_cw, q_wg, q_n, q_wt, arm_d, arm_s, st_nw, st_r, tw, sp);
  p.red = dalloc<double>(4096);
  KFBI_HIP(hipHostMalloc(&p.host_red, 4096 * sizeof(double), hipHostMallocDefault));
  Timer *ts[] = {&p.t_dst_x, &p.t_dst_y, &p.t_dst_last, &p.t_correct, &p.t_gather, &p.t_jumps, &p.t_dst_x_rows,
                 &p.t_dst_y_sparse};
  for (Timer *tm : ts) tm->create();
}

void free_tables(DevProblem &p) {
  int32_t **ip[] = {&p.z_idx, &p.z_axis, &p.q_idx, &p.irr_pos, &p.irr_ptr, &p.arm_cross, &p.st_pos,
                    &p.rows_in, &p.rows_out};
  uint8_t **up[] = {&p.mask_in, &p.mask_out, &p.planes_in, &p.planes_out};
  for (uint8_t **q : up) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  for (int32_t **q : ip) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  if (p.inside_pad) (void)hipFree(p.inside_pad);
  if (p.lam) (void)hipFree(p.lam);
  if (p.red) (void)hipFree(p.red);
  if (p.host_red) (void)hipHostFree(p.host_red);
  p.inside_pad = nullptr;
  p.lam = nullptr;
  p.red = nullptr;
  p.host_red = nullptr;
  free_prec(p.f64);
  free_prec(p.f32);
  Timer *ts[] = {&p.t_dst_x, &p.t_dst_y, &p.t_dst_last, &p.t_correct, &p.t_gather, &p.t_jumps, &p.t_dst_x_rows,
                 &p.t_dst_y_sparse};
  for (Timer *tm : ts) tm->destroy();
}

}  // namespace kfbi
