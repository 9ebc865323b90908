// Interface-side kernels of the KFBI matrix-vector product and the table upload.
//
//  k_jumps_nc     : density -> jumps [u_a], [u_aa] at every grid-line intersection
//                   (single-layer interface problem, Sec. 5.1 eq. single; jump relations
//                   from [u] = 0 and [n.D grad u] = psi for diagonal D_c), and
//                   [grad u], [Hess u] at every interface node, in one launch.
//  k_correct_nc   : right-hand-side correction at irregular grid nodes (Sec. 5.3, eq.
//                   correct): rhs_p = sum_arms s_p D_{c,a}/h^2 ([u_a] d + [u_aa] d^2 / 2).
//                   One thread owns one irregular node, so no atomics are needed.
//  k_gather_coop  : n.D grad u+ at every interface node from its 6/10-node quadratic fit,
//                   adding the Taylor-expanded jump to values on the "-" side
//                   (Sec. 5.4, eqs. taylor-i-po, taylor-i-co, ji).
// The single-problem gather is wavefront-cooperative (a group of lanes per node, one stencil
// point per lane, a DPP butterfly for the sums); the jumps and the correction keep one thread
// per item, as do the batched kernels (each choice measured).
//
// Precision: the density, the transfer and jump weights, the node jumps and the extrapolation
// fits are FP64 in every product.  Only the grid side follows the product's precision T: the
// crossing jumps are stored in T for the correction, which writes the T right-hand side that
// the T box solve transforms, and the gather reads the T grid values into its FP64 fit.
#include <cmath>
#include <type_traits>
#include <stdexcept>

#include "device.h"

namespace kfbi {
namespace {

constexpr int kBlock = 256;

// All stencil sizes are compile-time constants so that every index load of a thread is
// issued before the dependent gathers (the per-item forms are latency-bound).
// The jump relations enter through per-point weights built at setup (linear in the density
// values of the transfer stencil), so these kernels hold no geometry and serve any diagonal D.

// [u_a], [u_aa] at one crossing for every component: two weighted sums of the density values.
template <typename TZ, int K>
__device__ __forceinline__ void jumps_cross_at(int64_t c, const double *__restrict__ psi, int64_t M, int64_t nc,
                                               const int32_t *__restrict__ z_idx, const double *__restrict__ zA,
                                               const double *__restrict__ zB, int ncomp, TZ *__restrict__ jz) {
  int32_t j[K];
#pragma unroll
  for (int k = 0; k < K; ++k) j[k] = z_idx[k * nc + c];
  for (int comp = 0; comp < ncomp; ++comp) {
    const double *ps = psi + comp * M;
    const double *A = zA + (int64_t)comp * K * nc, *B = zB + (int64_t)comp * K * nc;
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = ps[j[k]];
    double ju = 0, juu = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ju += A[k * nc + c] * v[k];
      juu += B[k * nc + c] * v[k];
    }
    jz[(2 * comp) * nc + c] = (TZ)ju;
    jz[(2 * comp + 1) * nc + c] = (TZ)juu;
  }
}

// One irregular node per thread (batched kernels); at most 2D arms, loaded predicated and all at once.
// arm_s[comp][arm] = s_p D_{c,a} / h^2 for the arm's axis a.
template <typename T, int D>
__device__ __forceinline__ void correct_at(int64_t r, const int32_t *__restrict__ irr_pos,
                                           const int32_t *__restrict__ irr_ptr, const int32_t *__restrict__ arm_cross,
                                           const T *__restrict__ arm_d, const T *__restrict__ arm_s, int64_t narm,
                                           const T *__restrict__ jz, int64_t nc, int ncomp, T *__restrict__ rhs,
                                           int64_t comp_stride, int accumulate) {
  constexpr int MAXA = 2 * D;
  const int32_t b = irr_ptr[r], e = irr_ptr[r + 1];
  const int64_t pos = irr_pos[r];
  int32_t cr[MAXA];
  T d[MAXA];
#pragma unroll
  for (int i = 0; i < MAXA; ++i) {
    const bool ok = b + i < e;
    cr[i] = ok ? arm_cross[b + i] : 0;
    d[i] = ok ? arm_d[b + i] : T(0);
  }
  for (int comp = 0; comp < ncomp; ++comp) {
    T du[MAXA], duu[MAXA], sg[MAXA];
#pragma unroll
    for (int i = 0; i < MAXA; ++i) {
      const bool ok = b + i < e;
      du[i] = jz[(2 * comp) * nc + cr[i]];
      duu[i] = jz[(2 * comp + 1) * nc + cr[i]];
      sg[i] = ok ? arm_s[comp * narm + b + i] : T(0);
    }
    T acc = 0;
#pragma unroll
    for (int i = 0; i < MAXA; ++i) acc += sg[i] * (du[i] * d[i] + (T)0.5 * duu[i] * d[i] * d[i]);
    T *o = rhs + comp * comp_stride + pos;
    if (accumulate)
      *o += acc;
    else
      *o = acc;
  }
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

// [grad u] (D entries) and [Hess u] (NH entries) at one node for every component:
// out_j = psi_q qc[j] + sum_f g_f qG[j][f], g = surface gradient of psi from the transfer fit.
template <int D, int KN>
__device__ __forceinline__ void jumps_nodes_at(int64_t q, const double *__restrict__ psi, int64_t M,
                                               const int32_t *__restrict__ q_idx, const double *__restrict__ q_wg,
                                               const double *__restrict__ q_c, const double *__restrict__ q_G,
                                               int ncomp, double *__restrict__ jq) {
  constexpr int J = D + NH<D>::v;
  int32_t j[KN];
#pragma unroll
  for (int k = 0; k < KN; ++k) j[k] = q_idx[k * M + q];
  for (int comp = 0; comp < ncomp; ++comp) {
    const double *ps = psi + comp * M;
    double v[KN];
#pragma unroll
    for (int k = 0; k < KN; ++k) v[k] = ps[j[k]];
    double g[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      g[a] = 0;
#pragma unroll
      for (int k = 0; k < KN; ++k) g[a] += q_wg[(k * D + a) * M + q] * v[k];
    }
    const double pq = ps[q];
    const double *C = q_c + (int64_t)comp * J * M, *G = q_G + (int64_t)comp * J * D * M;
    double *o = jq + (int64_t)comp * J * M;
#pragma unroll
    for (int e = 0; e < J; ++e) {
      double acc = pq * C[e * M + q];
#pragma unroll
      for (int f = 0; f < D; ++f) acc += g[f] * G[(e * D + f) * M + q];
      o[e * M + q] = acc;
    }
  }
}

// n.D_c grad u+ at one node: st_nw[comp][j] = sum_a n_a D_{c,a} (gradient weight of node j)_a.
template <typename TU, int D, int S>
__device__ __forceinline__ void gather_at(int64_t q, const TU *__restrict__ u, int64_t comp_stride, int64_t M,
                                          const int32_t *__restrict__ st_pos, const double *__restrict__ st_nw,
                                          const double *__restrict__ st_r, const double *__restrict__ jq, int ncomp,
                                          int with_jumps, double *__restrict__ out) {
  constexpr int NHv = NH<D>::v, STR = D + NHv;
  int32_t pe[S];
#pragma unroll
  for (int j = 0; j < S; ++j) pe[j] = st_pos[j * M + q];
  for (int comp = 0; comp < ncomp; ++comp) {
    const TU *uc = u + comp * comp_stride;
    double val[S];
#pragma unroll
    for (int j = 0; j < S; ++j) val[j] = (double)uc[pe[j] < 0 ? -pe[j] - 1 : pe[j]];
    if (with_jumps) {
      const double *o = jq + (int64_t)comp * STR * M;
      double du[D], H[D][D];
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
        double r[D];
#pragma unroll
        for (int a = 0; a < D; ++a) r[a] = st_r[(j * D + a) * M + q];
        double Jv = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double hr = 0;
#pragma unroll
          for (int b = 0; b < D; ++b) hr += H[a][b] * r[b];
          Jv += r[a] * (du[a] + 0.5 * hr);
        }
        val[j] += Jv;
      }
    }
    const double *nw = st_nw + (int64_t)comp * S * M;
    double acc = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) acc += nw[j * M + q] * val[j];
    out[comp * M + q] = acc;
  }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------- wavefront-cooperative gather
//
// One thread per node leaves the single-problem gather short of parallelism: 40,960 nodes of a
// 3D problem are 640 wavefronts for 1024 SIMDs, each a chain of dependent loads (stencil index
// -> grid value -> weighted sum).  Here a group of G consecutive lanes (4, 8 or 16, the next
// power of two at or above the stencil size) shares one node: lane k takes stencil point k, and
// the weighted sum is finished by a butterfly across the group.  Tables keep their
// [point][node] layout.  The summation order differs from the one-thread form (a fixed tree
// instead of a left-to-right sum), deterministically.

constexpr int coop_group(int S) { return S <= 4 ? 4 : (S <= 8 ? 8 : 16); }

// Sum over the G lanes of a group (G = 4, 8 or 16, aligned); every lane receives the total.
// A butterfly of DPP moves within a row of 16 lanes: swap neighbours, swap pairs (quad
// permutes 1,0,3,2 and 2,3,0,1), then mirror within half rows and within the row, each step
// pairing every lane with one of the other half of its current block.  VALU moves only, so the
// LDS pipe, which a lane shuffle would use, stays free.  Additions are commutative, so every
// lane holds bitwise the same total.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int2 w = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_update_dpp(0, w.x, CTRL, 0xF, 0xF, false),
                                              __builtin_amdgcn_update_dpp(0, w.y, CTRL, 0xF, 0xF, false)));
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(G == 4 || G == 8 || G == 16, "group of 4, 8 or 16 lanes");
  auto mv = [](T x, auto ctrl) {
    if constexpr (sizeof(T) == 8) return dpp_f64<decltype(ctrl)::value>(x);
    else return dpp_f32<decltype(ctrl)::value>(x);
  };
  v += mv(v, std::integral_constant<int, 0xB1>{});   // quad_perm 1,0,3,2
  v += mv(v, std::integral_constant<int, 0x4E>{});   // quad_perm 2,3,0,1
  if constexpr (G >= 8) v += mv(v, std::integral_constant<int, 0x141>{});   // row_half_mirror
  if constexpr (G >= 16) v += mv(v, std::integral_constant<int, 0x140>{});  // row_mirror
  return v;
}

// [u_a], [u_aa] at crossing c for NC components, one thread per crossing: at 154,210 crossings
// of a 3D problem that is 2.4 wavefronts per SIMD already, and a lane group per crossing (one
// density point per lane, lane-shuffle sums) was measured slower, 28 -> 51 us for the launch.
template <typename TZ, int K, int NC>
__device__ __forceinline__ void jumps_cross_nc(int64_t c, const double *__restrict__ psi, int64_t M, int64_t nc,
                                               const int32_t *__restrict__ z_idx, const double *__restrict__ zA,
                                               const double *__restrict__ zB, TZ *__restrict__ jz) {
  int32_t j[K];
#pragma unroll
  for (int k = 0; k < K; ++k) j[k] = z_idx[k * nc + c];
#pragma unroll
  for (int comp = 0; comp < NC; ++comp) {
    const double *ps = psi + comp * M;
    const double *A = zA + (int64_t)comp * K * nc, *B = zB + (int64_t)comp * K * nc;
    double ju = 0, juu = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double v = ps[j[k]];
      ju += A[k * nc + c] * v;
      juu += B[k * nc + c] * v;
    }
    jz[(2 * comp) * nc + c] = (TZ)ju;
    jz[(2 * comp + 1) * nc + c] = (TZ)juu;
  }
}

// Both jump sets in one launch (they are independent): blocks [0, nbc) take the crossings,
// the others the interface nodes, one thread per item with the components unrolled.  A lane
// group per node (one transfer point per lane, then butterflies over the group) was measured
// slower: with the tables in [point][node] order each load of a group touches a separate line
// per point, where a thread per node reads whole lines.
template <typename TZ, int D, int K, int KN, int NC>
__global__ __launch_bounds__(kBlock) void k_jumps_nc(const double *__restrict__ psi, int64_t M, int64_t nc,
                                                     int64_t nbc, const int32_t *__restrict__ z_idx,
                                                     const double *__restrict__ zA, const double *__restrict__ zB,
                                                     const int32_t *__restrict__ q_idx, const double *__restrict__ q_wg,
                                                     const double *__restrict__ q_c, const double *__restrict__ q_G,
                                                     TZ *__restrict__ jz, double *__restrict__ jq) {
  if ((int64_t)blockIdx.x < nbc) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c < nc) jumps_cross_nc<TZ, K, NC>(c, psi, M, nc, z_idx, zA, zB, jz);
  } else {
    const int64_t q = ((int64_t)blockIdx.x - nbc) * kBlock + threadIdx.x;
    if (q < M) jumps_nodes_at<D, KN>(q, psi, M, q_idx, q_wg, q_c, q_G, NC, jq);
  }
}

// n.D_c grad u+ at node q, lane k < S taking stencil point k (its value, its jump term on the
// "-" side, its flux weight).
template <typename TU, int D, int S, int NC, int G>
__device__ __forceinline__ void gather_coop(int64_t q, int k, const TU *__restrict__ u, int64_t comp_stride,
                                            int64_t M, const int32_t *__restrict__ st_pos,
                                            const double *__restrict__ st_nw, const double *__restrict__ st_r,
                                            const double *__restrict__ jq, int with_jumps,
                                            double *__restrict__ out) {
  constexpr int NHv = NH<D>::v, STR = D + NHv;
  const bool act = k < S;
  const int32_t pe = act ? st_pos[k * M + q] : 0;
  const int64_t pu = pe < 0 ? -(int64_t)pe - 1 : pe;
  const bool minus = act && pe < 0 && with_jumps;
  double val[NC], nw[NC], r[D];
#pragma unroll
  for (int comp = 0; comp < NC; ++comp) {
    val[comp] = act ? (double)u[comp * comp_stride + pu] : 0.0;
    nw[comp] = act ? st_nw[((int64_t)comp * S + k) * M + q] : 0.0;
  }
  if (minus) {
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = st_r[(k * D + a) * M + q];
#pragma unroll
    for (int comp = 0; comp < NC; ++comp) {
      const double *o = jq + (int64_t)comp * STR * M;
      double du[D], H[D][D];
#pragma unroll
      for (int a = 0; a < D; ++a) du[a] = o[a * M + q];
#pragma unroll
      for (int e = 0; e < NHv; ++e) {
        int a, b;
        sym_index<D>(e, a, b);
        H[a][b] = H[b][a] = o[(D + e) * M + q];
      }
      double Jv = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double hr = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) hr += H[a][b] * r[b];
        Jv += r[a] * (du[a] + 0.5 * hr);
      }
      val[comp] += Jv;
    }
  }
#pragma unroll
  for (int comp = 0; comp < NC; ++comp) {
    const double acc = group_sum<G>(nw[comp] * val[comp]);
    if (k == comp) out[comp * M + q] = acc;
  }
}

template <typename TU, int D, int S, int NC>
__global__ __launch_bounds__(kBlock) void k_gather_coop(const TU *__restrict__ u, int64_t comp_stride, int64_t M,
                                                        const int32_t *__restrict__ st_pos,
                                                        const double *__restrict__ st_nw,
                                                        const double *__restrict__ st_r,
                                                        const double *__restrict__ jq, int with_jumps,
                                                        double *__restrict__ out) {
  constexpr int G = coop_group(S);
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t q = t / G;
  if (q < M) gather_coop<TU, D, S, NC, G>(q, (int)(t % G), u, comp_stride, M, st_pos, st_nw, st_r, jq, with_jumps,
                                          out);
}

// Correction at irregular node r, one thread per node with the components unrolled (a lane
// per arm was measured slower: at most six arms give little to share).
template <typename T, int D, int NC>
__global__ __launch_bounds__(kBlock) void k_correct_nc(int64_t nirr, const int32_t *__restrict__ irr_pos,
                                                       const int32_t *__restrict__ irr_ptr,
                                                       const int32_t *__restrict__ arm_cross,
                                                       const T *__restrict__ arm_d, const T *__restrict__ arm_s,
                                                       int64_t narm, const T *__restrict__ jz, int64_t nc,
                                                       T *__restrict__ rhs, int64_t comp_stride, int accumulate) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nirr)
    correct_at<T, D>(r, irr_pos, irr_ptr, arm_cross, arm_d, arm_s, narm, jz, nc, NC, rhs, comp_stride, accumulate);
}

inline unsigned nblk_g(int64_t n, int G) { return (unsigned)((n * G + kBlock - 1) / kBlock); }

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
                                                        const double *__restrict__ psi) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < c.tot_nc) {
    const int p = batch_problem(c.cum_nc, c.n, i);
    const BatchItem<T> &it = items[p];
    jumps_cross_at<T, 4>(i - c.cum_nc[p], psi + it.ioff, it.M, it.nc, it.z_idx, it.z_A, it.z_B, 1, it.jz);
    return;
  }
  i -= c.tot_nc;
  if (i >= c.tot_M) return;
  const int p = batch_problem(c.cum_M, c.n, i);
  const BatchItem<T> &it = items[p];
  jumps_nodes_at<2, 5>(i - c.cum_M[p], psi + it.ioff, it.M, it.q_idx, it.q_wg, it.q_c, it.q_G, 1, it.jq);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_correct(const BatchItem<T> *__restrict__ items, BatchCounts c,
                                                          int target) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.tot_nirr) return;
  const int p = batch_problem(c.cum_nirr, c.n, i);
  const BatchItem<T> &it = items[p];
  correct_at<T, 2>(i - c.cum_nirr[p], it.irr_pos, it.irr_ptr, it.arm_cross, it.arm_d, it.arm_s, it.narm, it.jz,
                   it.nc, 1, target ? it.fpad : it.rhs, 0, target);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_gather(const BatchItem<T> *__restrict__ items, BatchCounts c,
                                                         int with_jumps, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.tot_M) return;
  const int p = batch_problem(c.cum_M, c.n, i);
  const BatchItem<T> &it = items[p];
  gather_at<T, 2, 6>(i - c.cum_M[p], it.work, 0, it.M, it.st_pos, it.st_nw, it.st_r, it.jq, 1, with_jumps,
                     out + it.ioff);
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

// Numeric tables in FP64 (as built on the host) and their device copies in one precision.
struct NumTables {
  std::vector<double> z_A, z_B, q_wg, q_c, q_G, arm_d, arm_s, st_nw, st_r, tw, sp;
};

// The density-side tables (transfer and jump weights, extrapolation fits) and the node jumps
// exist in FP64 only; every precision keeps its correction weights, DST tables, fields and
// crossing jumps.
template <typename T>
void upload_prec(DevProblem &p, PrecTables<T> &tb, const NumTables &h) {
  const bool fits = sizeof(T) == sizeof(double);
  if (fits) {
    tb.z_A = dupload(cast_vec<T>(h.z_A));
    tb.z_B = dupload(cast_vec<T>(h.z_B));
    tb.q_wg = dupload(cast_vec<T>(h.q_wg));
    tb.q_c = dupload(cast_vec<T>(h.q_c));
    tb.q_G = dupload(cast_vec<T>(h.q_G));
    tb.st_nw = dupload(cast_vec<T>(h.st_nw));
    tb.st_r = dupload(cast_vec<T>(h.st_r));
  }
  tb.arm_d = dupload(cast_vec<T>(h.arm_d));
  tb.arm_s = dupload(cast_vec<T>(h.arm_s));
  tb.tw = dupload(cast_vec<T>(h.tw));
  tb.sp = dupload(cast_vec<T>(h.sp));
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
    if (fits && p.ncomp == 2) {
      tb.gbuf = dalloc<T>((size_t)p.comp_stride);
      KFBI_HIP(hipMemset(tb.gbuf, 0, (size_t)p.comp_stride * sizeof(T)));
    }
  }
  const int nh = p.dim == 2 ? 3 : 6;
  tb.jz = dalloc<T>((size_t)p.ncomp * 2 * std::max<int64_t>(p.nc, 1));
  if (fits) tb.jq = dalloc<T>((size_t)p.ncomp * (p.dim + nh) * p.M);
}

template <typename T>
void free_prec(PrecTables<T> &tb) {
  T **all[] = {&tb.z_A, &tb.z_B, &tb.q_wg, &tb.q_c, &tb.q_G, &tb.arm_d, &tb.arm_s, &tb.st_nw, &tb.st_r,
               &tb.tw, &tb.sp, &tb.rhs, &tb.work, &tb.xbuf, &tb.ybuf, &tb.gbuf, &tb.jz, &tb.jq};
  for (T **q : all) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
}

}  // namespace

template <typename T, int D, int K, int KN, int NC>
static void jumps_nc(DevProblem &p, const double *psi, hipStream_t st) {
  const PrecTables<double> &tb = p.f64;
  const int64_t nbc = p.nc > 0 ? nblk(p.nc) : 0;
  const unsigned g = (unsigned)(nbc + nblk(p.M));
  k_jumps_nc<T, D, K, KN, NC><<<g, kBlock, 0, st>>>(psi, p.M, p.nc, nbc, p.z_idx, tb.z_A, tb.z_B, p.q_idx, tb.q_wg,
                                                    tb.q_c, tb.q_G, p.tab<T>().jz, tb.jq);
}

template <typename T>
void launch_jumps(DevProblem &p, const double *psi, hipStream_t st) {
  if (p.dim == 2) {
    if (p.ncomp == 2) jumps_nc<T, 2, 4, 5, 2>(p, psi, st);
    else jumps_nc<T, 2, 4, 5, 1>(p, psi, st);
  } else {
    if (p.ncomp == 2) jumps_nc<T, 3, kLsqNodes, kLsqNodes, 2>(p, psi, st);
    else jumps_nc<T, 3, kLsqNodes, kLsqNodes, 1>(p, psi, st);
  }
  KFBI_HIP(hipGetLastError());
}

template <typename T, int D, int NC>
static void correct_nc(DevProblem &p, T *field, int accumulate, hipStream_t st) {
  PrecTables<T> &tb = p.tab<T>();
  k_correct_nc<T, D, NC><<<nblk(p.nirr), kBlock, 0, st>>>(
      p.nirr, p.irr_pos, p.irr_ptr, p.arm_cross, tb.arm_d, tb.arm_s, p.narm, tb.jz, p.nc, field, p.comp_stride,
      accumulate);
}

template <typename T>
static void correct_into(DevProblem &p, T *field, int accumulate, hipStream_t st) {
  if (p.nirr == 0) return;
  if (p.dim == 2) {
    if (p.ncomp == 2) correct_nc<T, 2, 2>(p, field, accumulate, st);
    else correct_nc<T, 2, 1>(p, field, accumulate, st);
  } else {
    if (p.ncomp == 2) correct_nc<T, 3, 2>(p, field, accumulate, st);
    else correct_nc<T, 3, 1>(p, field, accumulate, st);
  }
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

template <typename T, int D, int S, int NC>
static void gather_coop_launch(DevProblem &p, const T *u, bool with_jumps, double *out, hipStream_t st) {
  const PrecTables<double> &tb = p.f64;
  k_gather_coop<T, D, S, NC><<<nblk_g(p.M, coop_group(S)), kBlock, 0, st>>>(
      u, p.comp_stride, p.M, p.st_pos, tb.st_nw, tb.st_r, tb.jq, with_jumps ? 1 : 0, out);
}

template <typename T>
void launch_gather(DevProblem &p, const T *u, bool with_jumps, double *out, hipStream_t st) {
  if (p.dim == 2) {
    if (p.ncomp == 2) gather_coop_launch<T, 2, 6, 2>(p, u, with_jumps, out, st);
    else gather_coop_launch<T, 2, 6, 1>(p, u, with_jumps, out, st);
  } else {
    if (p.ncomp == 2) gather_coop_launch<T, 3, 10, 2>(p, u, with_jumps, out, st);
    else gather_coop_launch<T, 3, 10, 1>(p, u, with_jumps, out, st);
  }
  KFBI_HIP(hipGetLastError());
}

template <typename T>
void launch_batch_jumps(const BatchItem<T> *items, const BatchCounts &c, const double *psi, hipStream_t st) {
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
void launch_batch_gather(const BatchItem<T> *items, const BatchCounts &c, bool with_jumps, double *out,
                         hipStream_t st) {
  if (c.tot_M == 0) return;
  k_batch_gather<T><<<nblk(c.tot_M), kBlock, 0, st>>>(items, c, with_jumps ? 1 : 0, out);
  KFBI_HIP(hipGetLastError());
}
template void launch_batch_jumps<double>(const BatchItem<double> *, const BatchCounts &, const double *, hipStream_t);
template void launch_batch_jumps<float>(const BatchItem<float> *, const BatchCounts &, const double *, hipStream_t);
template void launch_batch_correct<double>(const BatchItem<double> *, const BatchCounts &, int, hipStream_t);
template void launch_batch_correct<float>(const BatchItem<float> *, const BatchCounts &, int, hipStream_t);
template void launch_batch_gather<double>(const BatchItem<double> *, const BatchCounts &, bool, double *,
                                          hipStream_t);
template void launch_batch_gather<float>(const BatchItem<float> *, const BatchCounts &, bool, double *, hipStream_t);

template void launch_jumps<double>(DevProblem &, const double *, hipStream_t);
template void launch_jumps<float>(DevProblem &, const double *, hipStream_t);
template void launch_correct<double>(DevProblem &, hipStream_t);
template void launch_correct<float>(DevProblem &, hipStream_t);
template void launch_add_correction<double>(DevProblem &, double *, hipStream_t);
template void launch_add_correction<float>(DevProblem &, float *, hipStream_t);
template void launch_gather<double>(DevProblem &, const double *, bool, double *, hipStream_t);
template void launch_gather<float>(DevProblem &, const float *, bool, double *, hipStream_t);

// Jump-relation coefficients of one component at a point with normal n and shape operator W
// (diagonal conductivity Dv): with a = psi / (n.D n),
//   [grad u] = a n,
//   [Hess u] = a W + n b^T + b n^T + c n n^T,  b = (g - 2 a W D n) / (n.D n),
//   c = (-a tr(D W) - 2 b.D n) / (n.D n),
// written as [Hess u]_ab = psi alpha_ab + sum_f g_f beta_ab,f (g = surface gradient of psi).
struct JumpCoef {
  int d;
  double nDn, n[3], Dn[3], WDn[3], W[9], trDW, WDnDn;
  JumpCoef(int d_, const double *nrm, const double *Wm, const double *Dv) : d(d_) {
    nDn = 0;
    for (int a = 0; a < d; ++a) {
      n[a] = nrm[a];
      Dn[a] = Dv[a] * nrm[a];
      nDn += n[a] * Dn[a];
    }
    trDW = 0;
    WDnDn = 0;
    for (int a = 0; a < d; ++a) {
      WDn[a] = 0;
      for (int b = 0; b < d; ++b) {
        W[a * d + b] = Wm[a * d + b];
        WDn[a] += Wm[a * d + b] * Dn[b];
      }
      trDW += Dv[a] * Wm[a * d + a];
    }
    for (int a = 0; a < d; ++a) WDnDn += WDn[a] * Dn[a];
  }
  double grad(int a) const { return n[a] / nDn; }
  double alpha(int a, int b) const {
    return (W[a * d + b] - 2.0 * (n[a] * WDn[b] + WDn[a] * n[b]) / nDn - trDW * n[a] * n[b] / nDn +
            4.0 * WDnDn * n[a] * n[b] / (nDn * nDn)) / nDn;
  }
  double beta(int a, int b, int f) const {
    return ((a == f ? n[b] : 0.0) + (b == f ? n[a] : 0.0)) / nDn - 2.0 * Dn[f] * n[a] * n[b] / (nDn * nDn);
  }
};

void upload_tables(DevProblem &p) {
  const HostTables &t = p.ht;
  const int d = t.dim, nc_ = t.ncomp;
  p.dim = d;
  p.ncomp = nc_;
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
  for (int c = 0; c < 2; ++c)
    for (int a = 0; a < 3; ++a) p.D[c][a] = t.D[c < nc_ ? c : 0][a < d ? a : 0];
  p.lam_scale = 1.0;
  for (int a = 0; a < d; ++a) p.lam_scale *= 2.0 / (double)t.cells;
  const int64_t N = p.N, M = p.M, nc = p.nc, P = p.P, K = t.K, Kn = t.Kn, S = t.S;
  auto padpos = [&](int64_t lin) { return (lin % N) + P * (lin / N); };
  if (padpos(N * (d == 3 ? N * N : N) - 1) >= (int64_t)1 << 31) throw std::invalid_argument("grid too large");
  NumTables h;

  // crossings: [u_a] and [u_aa] (a = the arm's axis) as weights on the transfer stencil
  std::vector<int32_t> z_idx(nc * K), z_axis(nc);
  h.z_A.assign((size_t)nc_ * K * nc, 0.0);
  h.z_B.assign((size_t)nc_ * K * nc, 0.0);
  for (int64_t c = 0; c < nc; ++c) {
    const int a = (int)t.c_axis[c];
    z_axis[c] = a;
    for (int k = 0; k < K; ++k) z_idx[k * nc + c] = (int32_t)t.z_idx[c * K + k];
    for (int comp = 0; comp < nc_; ++comp) {
      const JumpCoef jc(d, &t.c_n[c * d], &t.c_W[c * d * d], t.D[comp]);
      const double al = jc.alpha(a, a);
      for (int k = 0; k < K; ++k) {
        const double w0 = t.z_w0[c * K + k];
        double bk = w0 * al;
        for (int f = 0; f < d; ++f) bk += t.z_wg[(c * K + k) * d + f] * jc.beta(a, a, f);
        h.z_A[((size_t)comp * K + k) * nc + c] = w0 * jc.grad(a);
        h.z_B[((size_t)comp * K + k) * nc + c] = bk;
      }
    }
  }
  // correction records: CSR over irregular nodes; arm_s[comp][arm] = s D_{comp,a} / h^2
  std::vector<std::vector<int64_t>> arms_of(t.irregular.size());
  auto rank = [&](int64_t lin) {
    return (int64_t)(std::lower_bound(t.irregular.begin(), t.irregular.end(), lin) - t.irregular.begin());
  };
  for (int64_t c = 0; c < nc; ++c) {
    arms_of[rank(t.c_pin[c])].push_back(2 * c);       // tissue-side node, s = +1
    arms_of[rank(t.c_pout[c])].push_back(2 * c + 1);  // "-"-side node, s = -1
  }
  std::vector<int32_t> irr_pos(t.irregular.size()), irr_ptr(t.irregular.size() + 1, 0), arm_cross;
  std::vector<int> arm_axis;
  std::vector<double> arm_sign;
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
      h.arm_d.push_back(coord(nb, a) - t.c_z[c * d + a]);
      arm_axis.push_back(a);
      arm_sign.push_back(plus ? ih2 : -ih2);
    }
    irr_ptr[r + 1] = (int32_t)arm_cross.size();
  }
  p.narm = (int64_t)arm_cross.size();
  h.arm_s.assign((size_t)nc_ * std::max<int64_t>(p.narm, 1), 0.0);
  for (int comp = 0; comp < nc_; ++comp)
    for (int64_t i = 0; i < p.narm; ++i) h.arm_s[comp * p.narm + i] = arm_sign[i] * t.D[comp][arm_axis[i]];
  // node jumps: [grad u] and [Hess u] from psi at the node and the surface gradient g
  const int nh = d == 2 ? 3 : 6, J = d + nh;
  const int SA[6] = {0, 1, 2, 0, 0, 1}, SB[6] = {0, 1, 2, 1, 2, 2};
  const int SA2[3] = {0, 1, 0}, SB2[3] = {0, 1, 1};
  std::vector<int32_t> q_idx(M * Kn);
  h.q_wg.assign((size_t)M * Kn * d, 0.0);
  h.q_c.assign((size_t)nc_ * J * M, 0.0);
  h.q_G.assign((size_t)nc_ * J * d * M, 0.0);
  for (int64_t q = 0; q < M; ++q) {
    for (int k = 0; k < Kn; ++k) {
      q_idx[k * M + q] = (int32_t)t.q_idx[q * Kn + k];
      for (int a = 0; a < d; ++a) h.q_wg[(k * d + a) * M + q] = t.q_wg[(q * Kn + k) * d + a];
    }
    for (int comp = 0; comp < nc_; ++comp) {
      const JumpCoef jc(d, &t.nrm[q * d], &t.W[q * d * d], t.D[comp]);
      double *C = &h.q_c[(size_t)comp * J * M], *G = &h.q_G[(size_t)comp * J * d * M];
      for (int a = 0; a < d; ++a) C[a * M + q] = jc.grad(a);
      for (int e = 0; e < nh; ++e) {
        const int a = d == 2 ? SA2[e] : SA[e], b = d == 2 ? SB2[e] : SB[e];
        C[(d + e) * M + q] = jc.alpha(a, b);
        for (int f = 0; f < d; ++f) G[((d + e) * d + f) * M + q] = jc.beta(a, b, f);
      }
    }
  }
  // gather stencils: st_nw[comp][j] = n . D_comp (gradient weights of stencil node j)
  std::vector<int32_t> st_pos(M * S);
  h.st_nw.assign((size_t)nc_ * S * M, 0.0);
  h.st_r.assign((size_t)M * S * d, 0.0);
  for (int64_t q = 0; q < M; ++q)
    for (int j = 0; j < S; ++j) {
      const int64_t pos = padpos(t.st_lin[q * S + j]);
      st_pos[j * M + q] = t.st_chi[q * S + j] ? (int32_t)(-pos - 1) : (int32_t)pos;
      for (int a = 0; a < d; ++a) h.st_r[(j * d + a) * M + q] = t.st_r[(q * S + j) * d + a];
      for (int comp = 0; comp < nc_; ++comp) {
        double nw = 0;
        for (int a = 0; a < d; ++a) nw += t.nrm[q * d + a] * t.D[comp][a] * t.st_wgrad[(q * S + j) * d + a];
        h.st_nw[((size_t)comp * S + j) * M + q] = nw;
      }
    }
  // DST tables
  const int Mf = p.Mfft;
  h.tw.resize(2 * Mf);
  h.sp.resize(Mf / 2 + 1);
  std::vector<double> lam(N);
  for (int m = 0; m < Mf; ++m) {
    const double ang = -2.0 * M_PI * (double)m / (double)Mf;
    h.tw[2 * m] = std::cos(ang);
    h.tw[2 * m + 1] = std::sin(ang);
  }
  for (int n = 0; n <= Mf / 2; ++n) h.sp[n] = std::sin(M_PI * (double)n / (double)Mf);
  for (int64_t k = 1; k <= N; ++k) {
    const double sn = std::sin((double)k * M_PI / (2.0 * Mf));
    lam[k - 1] = 4.0 / (t.h * t.h) * sn * sn;
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
    std::vector<uint64_t> bin((size_t)N * 16, 0), bout((size_t)N * 16, 0);
    for (int64_t r = 0; r < N * N; ++r) {
      const int64_t z = r / N, y = r % N;
      if (min_[r]) bin[(size_t)z * 16 + (y >> 6)] |= uint64_t(1) << (y & 63);
      if (mout[r]) bout[(size_t)z * 16 + (y >> 6)] |= uint64_t(1) << (y & 63);
    }
    p.mask_in = dupload(bin);
    p.mask_out = dupload(bout);
    std::vector<uint8_t> pin(N, 0), pout(N, 0);
    for (int64_t r = 0; r < N * N; ++r) {
      if (min_[r]) pin[r / N] = 1;
      if (mout[r]) pout[r / N] = 1;
    }
    p.planes_in = dupload(pin);
    p.planes_out = dupload(pout);
    p.planes_in_bits = PlaneBits{};
    p.planes_out_bits = PlaneBits{};
    for (int64_t z = 0; z < N; ++z) {
      if (pin[z]) p.planes_in_bits.w[z >> 6] |= uint64_t(1) << (z & 63);
      if (pout[z]) p.planes_out_bits.w[z >> 6] |= uint64_t(1) << (z & 63);
    }
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
  upload_prec<double>(p, p.f64, h);
  upload_prec<float>(p, p.f32, h);
  p.red = dalloc<double>(4096);
  KFBI_HIP(hipHostMalloc(&p.host_red, 4096 * sizeof(double), hipHostMallocDefault));
  Timer *ts[] = {&p.t_dst_x, &p.t_dst_y, &p.t_dst_last, &p.t_correct, &p.t_gather, &p.t_jumps, &p.t_dst_x_rows,
                 &p.t_dst_y_sparse, &p.t_dst_last_sparse, &p.t_dst_last_out, &p.t_dst_x_fhn, &p.t_dst_x_fe1,
                 &p.t_dst_y1, &p.t_dst_last_anti, &p.t_dst_last_diff, &p.t_dst_x_be1, &p.t_dst_last_comb};
  for (Timer *tm : ts) tm->create();
}

void free_tables(DevProblem &p) {
  int32_t **ip[] = {&p.z_idx, &p.z_axis, &p.q_idx, &p.irr_pos, &p.irr_ptr, &p.arm_cross, &p.st_pos,
                    &p.rows_in, &p.rows_out};
  uint8_t **up[] = {&p.planes_in, &p.planes_out};
  for (uint8_t **q : up) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  uint64_t **bp[] = {&p.mask_in, &p.mask_out};
  for (uint64_t **q : bp) {
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
                 &p.t_dst_y_sparse, &p.t_dst_last_sparse, &p.t_dst_last_out, &p.t_dst_x_fhn, &p.t_dst_x_fe1,
                 &p.t_dst_y1, &p.t_dst_last_anti, &p.t_dst_last_diff, &p.t_dst_x_be1, &p.t_dst_last_comb};
  for (Timer *tm : ts) tm->destroy();
}

}  // namespace kfbi
