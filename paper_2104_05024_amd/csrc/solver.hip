// GMRES / Richardson on the KFBI operator, the Neumann solve of Algorithm 1, and the
// Strang-split bidomain step (Secs. 3-6).  Krylov vectors, Arnoldi (classical Gram-Schmidt
// with one re-orthogonalisation), Givens rotations and the least-squares update are FP64;
// only the matrix-vector product may run in FP32 (inner solve of the refinement scheme).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "solver.h"

namespace kfbi {
namespace {

constexpr int kB = 256;
inline unsigned nblk(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

template <typename T>
T *dalloc(size_t n) {
  T *p = nullptr;
  KFBI_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
  return p;
}

// partial dot products: block (bx, k) reduces sum_i a_k[i] b[i] over its grid-stride slice;
// with jlim, only vectors k <= *jlim take part (the Arnoldi step replayed from a graph)
__global__ __launch_bounds__(kB) void k_multidot(const double *__restrict__ A, int64_t lda,
                                                 const double *__restrict__ b, int64_t n,
                                                 double *__restrict__ partials,
                                                 const int *__restrict__ jlim = nullptr) {
  __shared__ double s[kB];
  const int k = blockIdx.y;
  if (jlim && k > *jlim) return;
  const double *a = A + (int64_t)k * lda;
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) acc += a[i] * b[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kB / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[(int64_t)k * gridDim.x + blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kB) void k_finish(const double *__restrict__ partials, int nb,
                                               double *__restrict__ out, const int *__restrict__ jlim = nullptr) {
  __shared__ double s[kB];
  const int k = blockIdx.x;
  if (jlim && k > *jlim) return;
  double acc = 0;
  for (int i = threadIdx.x; i < nb; i += kB) acc += partials[(int64_t)k * nb + i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kB / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = s[0];
}

// w -= sum_k h[k] V_k   (sign = -1)   or   x += sum_k h[k] V_k   (sign = +1)
__global__ __launch_bounds__(kB) void k_combine(double *__restrict__ w, const double *__restrict__ V, int64_t ldv,
                                                const double *__restrict__ h, int K, double sign, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  double acc = 0;
  for (int k = 0; k < K; ++k) acc += h[k] * V[(int64_t)k * ldv + i];
  w[i] += sign * acc;
}

// Sum of the nb block partials of row k by one wave: lane-strided sums, then a butterfly (every
// lane ends with the same value).
__device__ __forceinline__ double wave_sum_partials(const double *__restrict__ partials, int nb, int k) {
  const int lane = threadIdx.x & 63;
  double acc = 0;
  for (int i = lane; i < nb; i += 64) acc += partials[(int64_t)k * nb + i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  return acc;
}

// One classical Gram-Schmidt pass after k_multidot: every block sums the partials into
// h_k (k < K; the sums are identical in every block), then w -= sum_k h_k V_k; block 0 stores h
// for the Hessenberg column.  K = *jdev + 1 when jdev is given (the captured step).  With
// npart (the last pass), each block also stores the sum of its updated w_i^2 in npart[block]:
// the partials of ||w||^2, one element per thread as k_multidot has them when its grid covers
// the vector.
__global__ __launch_bounds__(kB) void k_cgs_combine(double *__restrict__ w, const double *__restrict__ V, int64_t ldv,
                                                    const double *__restrict__ partials, int nb,
                                                    double *__restrict__ hout, const int *__restrict__ jdev, int K,
                                                    int64_t n, double *__restrict__ npart) {
  __shared__ double hs[Solver::kMaxRestart + 1];
  __shared__ double sq[kB];
  if (jdev) K = *jdev + 1;
  for (int k = threadIdx.x >> 6; k < K; k += kB / 64) {
    const double s = wave_sum_partials(partials, nb, k);
    if ((threadIdx.x & 63) == 0) hs[k] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < K; k += kB) hout[k] = hs[k];
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  double wi = 0;
  if (i < n) {
    double acc = 0;
    for (int k = 0; k < K; ++k) acc += hs[k] * V[(int64_t)k * ldv + i];
    wi = w[i] - acc;
    w[i] = wi;
  }
  if (!npart) return;
  sq[threadIdx.x] = wi * wi;
  __syncthreads();
  for (int off = kB / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sq[threadIdx.x] += sq[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) npart[blockIdx.x] = sq[0];
}

// The norm after k_multidot of w with itself: V_{j+1} = w / ||w|| (j = *jdev when given, else
// jh), also into vnext when given (the next step's input); block 0 stores ||w||^2.  w may be
// V_{j+1} itself.
__global__ __launch_bounds__(kB) void k_normalize(double *V, int64_t ldv, const double *w,
                                                  const double *__restrict__ partials, int nb,
                                                  double *__restrict__ hout, const int *__restrict__ jdev, int jh,
                                                  double *__restrict__ vnext, int64_t n) {
  __shared__ double s0;
  if (threadIdx.x < 64) {
    const double s = wave_sum_partials(partials, nb, 0);
    if (threadIdx.x == 0) s0 = s;
  }
  __syncthreads();
  const double nrm2 = s0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *hout = nrm2;
  const int j = jdev ? *jdev : jh;
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const double sc = nrm2 > 0 ? 1.0 / sqrt(nrm2) : 0.0;
  const double v = w[i] * sc;
  V[(int64_t)(j + 1) * ldv + i] = v;
  if (vnext) vnext[i] = v;
}

// j <- j + 1 (when given), and the step counter: seq <- seq + 1, also stored to the host's copy
__global__ void k_inc_j(int *j, int *seq, int *seq_host) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (j) *j += 1;
    const int s = *seq + 1;
    *seq = s;
    __threadfence_system();
    __hip_atomic_store(seq_host, s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ __launch_bounds__(kB) void k_axpby(double *__restrict__ z, double a, const double *__restrict__ x,
                                              double b, const double *__restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  z[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ __launch_bounds__(kB) void k_fill(double *__restrict__ z, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) z[i] = v;
}

// out = psi - c z with the coefficient c = <z, psi> read from device memory (out may be psi)
__global__ __launch_bounds__(kB) void k_remove_along(double *out, const double *psi,
                                                     const double *__restrict__ z, const double *__restrict__ c,
                                                     int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) out[i] = psi[i] - c[0] * z[i];
}

// Starting residual of psi^{n-1} without a product: (g'^n - g'^{n-1}) + (g'^{n-1} - A psi^{n-1}).
// It holds only if the caller's psi^{n-1} (hist1) is still the density the previous solve
// returned (psi_last, the context's own copy): any node that differs sets *bad.
__global__ __launch_bounds__(kB) void k_recycled_resid(double *__restrict__ r, const double *__restrict__ gp,
                                                       const double *__restrict__ gp_prev,
                                                       const double *__restrict__ d_prev,
                                                       const double *__restrict__ hist1,
                                                       const double *__restrict__ psi_last, int *__restrict__ bad,
                                                       int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  bool differs = false;
  if (i < n) {
    r[i] = (gp[i] - gp_prev[i]) + d_prev[i];
    differs = hist1[i] != psi_last[i];
  }
  if (__any(differs) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

// End of a bidomain step: g'^{n-1} <- g'^n, the density history shifts by one step, the context
// keeps its own copy of the new density, and the mismatch flag of the next recycled residual is
// cleared.
__global__ __launch_bounds__(kB) void k_end_step(double *__restrict__ gp_prev, const double *__restrict__ gp,
                                                 double *__restrict__ hist2, double *__restrict__ hist1,
                                                 double *__restrict__ psi_last, const double *__restrict__ psi,
                                                 int *__restrict__ bad, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i == 0) *bad = 0;
  if (i >= n) return;
  const double v = psi[i];
  gp_prev[i] = gp[i];
  hist2[i] = hist1[i];
  hist1[i] = v;
  psi_last[i] = v;
}

template <typename A, typename B>
__global__ __launch_bounds__(kB) void k_cast(const A *__restrict__ x, B *__restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) y[i] = (B)x[i];
}

// plain [comp][N^d] -> padded [comp][..][P]
__global__ __launch_bounds__(kB) void k_to_padded(const double *__restrict__ f, double *__restrict__ fp,
                                                  int64_t nplain, int64_t N, int64_t P, int64_t cs, int ncomp) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= nplain * ncomp) return;
  const int64_t c = i / nplain, lin = i - c * nplain;
  fp[c * cs + (lin % N) + P * (lin / N)] = f[i];
}


__global__ __launch_bounds__(kB) void k_masked_sum(const double *__restrict__ u, const int8_t *__restrict__ mask,
                                                   int64_t n, double *__restrict__ partials) {
  __shared__ double s[kB];
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    if (mask[i]) acc += u[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kB / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// ---------------------------------------------------------------- FitzHugh-Nagumo kernels

// Midpoint update V <- 2 (u_i - u_e) - V1 and step 3 (backward Euler over dt/2) when the
// potentials are also returned: writes them in the gauge of the given mean.  (Without them the
// inverse x pass of the final box solve does this work.)  V and q still hold the step's
// starting state; (V1, q1) is their forward Euler half step, recomputed as the x passes do.
__global__ __launch_bounds__(kB) void k_mid_be(const double *__restrict__ u, double *__restrict__ V,
                                               double *__restrict__ q, double *__restrict__ phi,
                                               const double *__restrict__ mean, int64_t n, int64_t N, int64_t P,
                                               int64_t cs, double dth, FhnCoef m) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int64_t pos = (i % N) + P * (i / N);
  const double ui = u[pos], ue = u[cs + pos];
  double v1 = V[i], q1 = q[i], vn, qn;
  fhn_fe(v1, q1, dth, m);   // V and q hold the step's starting state (see the x passes)
  fhn_be(2.0 * (ui - ue) - v1, q1, dth, m, vn, qn);
  V[i] = vn;
  q[i] = qn;
  if (phi) {
    const double s = mean ? mean[0] : 0.0;
    phi[i] = ui - s;
    phi[n + i] = ue - s;
  }
}

}  // namespace

void Solver::init(DevProblem &p) {
  L = (int64_t)p.ncomp * p.M;
  nb = (int)std::min<int64_t>(512, std::max<int64_t>(1, (L + kB - 1) / kB));
  V = dalloc<double>((size_t)(kMaxRestart + 1) * L);
  r = dalloc<double>(L);
  w = dalloc<double>(L);
  t = dalloc<double>(L);
  gp = dalloc<double>(L);
  d = dalloc<double>(L);
  fpad = dalloc<double>((size_t)p.ncomp * p.comp_stride);
  KFBI_HIP(hipMemset(fpad, 0, (size_t)p.ncomp * p.comp_stride * sizeof(double)));
  partials = dalloc<double>((size_t)(kMaxRestart + 2) * 512);
  npart = dalloc<double>((size_t)nblk(L));
  hdev = dalloc<double>(3 * (kMaxRestart + 2));
  ydev = dalloc<double>(kMaxRestart + 2);
  KFBI_HIP(hipHostMalloc(&hhost, 3 * (kMaxRestart + 2) * sizeof(double), hipHostMallocDefault));
  KFBI_HIP(hipHostMalloc(&ypin, 2 * (kMaxRestart + 2) * sizeof(double), hipHostMallocDefault));
  vin = dalloc<double>(L);
  wv = dalloc<double>(L);
  if (p.ncomp == 2) {
    nullz = dalloc<double>(L);
    nully = dalloc<double>(L);
    nullp = dalloc<double>(L);
    nullc = dalloc<double>(1);
  }
  null_ready = false;
  jdev = dalloc<int>(1);
  KFBI_HIP(hipHostMalloc(&jhost, sizeof(int), hipHostMallocDefault));
  seqdev = dalloc<int>(1);
  KFBI_HIP(hipMemset(seqdev, 0, sizeof(int)));
  KFBI_HIP(hipHostMalloc(&seqhost, sizeof(int), hipHostMallocDefault));
  *seqhost = 0;
  seq_next = 0;
  KFBI_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  n_inside = 0;
  for (int8_t v : p.ht.inside) n_inside += v;
  inside_plain = dalloc<int8_t>(p.ht.inside.size());
  KFBI_HIP(hipMemcpy(inside_plain, p.ht.inside.data(), p.ht.inside.size(), hipMemcpyHostToDevice));
}

void Solver::release() {
  for (int k = 0; k < 2; ++k)
    if (graph[k]) {
      (void)hipGraphExecDestroy(graph[k]);
      graph[k] = nullptr;
    }
  if (cap) (void)hipStreamDestroy(cap);
  cap = nullptr;
  if (jdev) (void)hipFree(jdev);
  if (jhost) (void)hipHostFree(jhost);
  jdev = nullptr;
  jhost = nullptr;
  if (seqdev) (void)hipFree(seqdev);
  if (seqhost) (void)hipHostFree(seqhost);
  seqdev = nullptr;
  seqhost = nullptr;
  double **dp[] = {&V,    &r,    &w,  &t,   &gp,    &d,     &fpad,  &partials, &npart,
                   &hdev, &ydev, &vin, &wv, &nullz, &nully, &nullp, &nullc};
  for (double **q : dp) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  if (inside_plain) (void)hipFree(inside_plain);
  if (hhost) (void)hipHostFree(hhost);
  if (ypin) (void)hipHostFree(ypin);
  ypin = nullptr;
  inside_plain = nullptr;
  hhost = nullptr;
}

template <typename T>
void Solver::apply(DevProblem &p, const double *psi, double *out, hipStream_t st) {
  PrecTables<T> &tb = p.tab<T>();
  p.t_jumps.tic(p.profile, st);
  launch_jumps<T>(p, psi, st);
  p.t_jumps.toc(p.profile, st);
  p.t_correct.tic(p.profile, st);
  launch_correct<T>(p, st);
  p.t_correct.toc(p.profile, st);
  box_solve_matvec<T>(p, st);
  p.t_gather.tic(p.profile, st);
  launch_gather<T>(p, tb.work, true, out, st);
  p.t_gather.toc(p.profile, st);
}
template void Solver::apply<double>(DevProblem &, const double *, double *, hipStream_t);
template void Solver::apply<float>(DevProblem &, const double *, double *, hipStream_t);

void Solver::apply_vec(DevProblem &p, int prec, const double *x, double *y, hipStream_t st) {
  if (prec == 0) apply<double>(p, x, y, st);
  else apply<float>(p, x, y, st);
}

void Solver::apply_f32(DevProblem &p, const float *psi, float *out, hipStream_t st) {
  k_cast<float, double><<<nblk(L), kB, 0, st>>>(psi, t, L);
  apply<float>(p, t, w, st);
  k_cast<double, float><<<nblk(L), kB, 0, st>>>(w, out, L);
  KFBI_HIP(hipGetLastError());
}

double Solver::residual_norm(const double *b, const double *Ax, hipStream_t st) {
  k_axpby<<<nblk(L), kB, 0, st>>>(d, 1.0, b, -1.0, Ax, L);
  KFBI_HIP(hipGetLastError());
  return std::sqrt(dot(d, d, st));
}

double Solver::dot(const double *a, const double *b, hipStream_t st) {
  k_multidot<<<dim3(nb, 1), kB, 0, st>>>(a, L, b, L, partials);
  k_finish<<<1, kB, 0, st>>>(partials, nb, hdev);
  KFBI_HIP(hipMemcpyAsync(hhost, hdev, sizeof(double), hipMemcpyDeviceToHost, st));
  host_wait(st);
  return hhost[0];
}

// One Arnoldi step with j read from device memory (so one captured graph serves every j):
// w = A v for v = V_j (held in vin), two classical Gram-Schmidt passes against V_0..V_j, the
// norm, V_{j+1} (also into vin), the Hessenberg column to pinned host memory, j <- j + 1.
void Solver::arnoldi_step(DevProblem &p, int prec, int m, hipStream_t st) {
  apply_vec(p, prec, vin, wv, st);
  for (int pass = 0; pass < 2; ++pass) {
    k_multidot<<<dim3(nb, m), kB, 0, st>>>(V, L, wv, L, partials, jdev);
    k_cgs_combine<<<nblk(L), kB, 0, st>>>(wv, V, L, partials, nb, hdev + pass * (kMaxRestart + 2), jdev, 0, L,
                                          pass == 1 ? npart : nullptr);
  }
  k_normalize<<<nblk(L), kB, 0, st>>>(V, L, wv, npart, (int)nblk(L), hdev + 2 * (kMaxRestart + 2), jdev, 0, vin,
                                      L);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipMemcpyAsync(hhost, hdev, 3 * (kMaxRestart + 2) * sizeof(double), hipMemcpyDeviceToHost, st));
  k_inc_j<<<1, 1, 0, st>>>(jdev, seqdev, seqhost);
  KFBI_HIP(hipGetLastError());
}

void Solver::host_wait(hipStream_t st) {
  k_inc_j<<<1, 1, 0, st>>>(nullptr, seqdev, seqhost);
  KFBI_HIP(hipGetLastError());
  wait_step(st);
}

int poll_step_counter(const int *seq_host, int expect, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  for (int spins = 0;; ++spins) {
    if (__atomic_load_n(seq_host, __ATOMIC_ACQUIRE) == expect) return expect;
    if ((spins & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) break;
  }
  KFBI_HIP(hipStreamSynchronize(st));
  return __atomic_load_n(seq_host, __ATOMIC_ACQUIRE);
}

// Waits for the step just replayed (its Hessenberg column copy precedes the counter store).
void Solver::wait_step(hipStream_t st) { seq_next = poll_step_counter(seqhost, seq_next + 1, st); }

// Replays the captured Arnoldi step (captured on first use on the solver's own stream).
void Solver::run_step(DevProblem &p, int prec, int m, hipStream_t st) {
  if (!graph[prec] || graph_m[prec] != m) {
    if (graph[prec]) (void)hipGraphExecDestroy(graph[prec]);
    graph[prec] = nullptr;
    hipGraph_t g = nullptr;
    KFBI_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    try {
      arnoldi_step(p, prec, m, cap);
    } catch (...) {
      (void)hipStreamEndCapture(cap, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    KFBI_HIP(hipStreamEndCapture(cap, &g));
    const hipError_t e = hipGraphInstantiate(&graph[prec], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    KFBI_HIP(e);
    graph_m[prec] = m;
  }
  KFBI_HIP(hipGraphLaunch(graph[prec], st));
}

int Solver::gmres(DevProblem &p, const double *b, double bnorm, double *x, bool x_zero, double tol_abs, int restart,
                  int maxit, const GmresArgs &a, GmresStats &s, hipStream_t st) {
  const int m = std::max(1, std::min(restart, kMaxRestart));
  s = GmresStats{};
  if (bnorm == 0.0) {
    // b = 0: the solution is 0 and so is its residual, which callers read from r
    k_axpby<<<nblk(L), kB, 0, st>>>(x, 0.0, b, 0.0, nullptr, L);
    k_axpby<<<nblk(L), kB, 0, st>>>(r, 1.0, b, 0.0, nullptr, L);
    KFBI_HIP(hipGetLastError());
    return KFBI_OK;
  }
  auto count = [&](int prec) {
    if (prec) ++s.mv32;
    else ++s.mv64;
  };
  // the product of a restart residual: FP64 in a relaxed solve, else the solve's own precision
  const int prec_res = a.relax ? 0 : a.prec;
  // r = b - A x
  if (x_zero) {
    KFBI_HIP(hipMemcpyAsync(r, b, L * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else if (a.r0) {
    KFBI_HIP(hipMemcpyAsync(r, a.r0, L * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else {
    apply_vec(p, prec_res, x, t, st);
    count(prec_res);
    k_axpby<<<nblk(L), kB, 0, st>>>(r, 1.0, b, -1.0, t, L);
  }
  double beta = std::sqrt(dot(r, r, st));
  s.beta0 = beta;
  std::vector<double> H((size_t)(m + 1) * m), Hc((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), z(m + 1);
  while (beta > tol_abs && s.its < maxit) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(Hc.begin(), Hc.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    const double beta_cycle = beta;
    k_axpby<<<nblk(L), kB, 0, st>>>(V, 1.0 / beta, r, 0.0, nullptr, L);
    int jend = 0;
    bool breakdown = false, any32 = false;
    const bool graphed = use_graph && !p.profile;
    if (graphed) {
      *jhost = 0;
      KFBI_HIP(hipMemcpyAsync(jdev, jhost, sizeof(int), hipMemcpyHostToDevice, st));
      KFBI_HIP(hipMemcpyAsync(vin, V, L * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    double target = tol_abs;
    for (int j = 0; j < m; ++j) {
      // relaxed: FP32 products once the current (Givens) residual is below sw_abs
      const int pj = a.relax ? (std::fabs(g[j]) <= a.sw_abs ? 1 : 0) : a.prec;
      any32 = any32 || pj == 1;
      if (graphed) {
        run_step(p, pj, m, st);
      } else {
        const double *vj = V + (int64_t)j * L;
        double *vn = V + (int64_t)(j + 1) * L;
        apply_vec(p, pj, vj, vn, st);
        // classical Gram-Schmidt, twice; then the norm
        for (int pass = 0; pass < 2; ++pass) {
          k_multidot<<<dim3(nb, j + 1), kB, 0, st>>>(V, L, vn, L, partials);
          k_cgs_combine<<<nblk(L), kB, 0, st>>>(vn, V, L, partials, nb, hdev + pass * (kMaxRestart + 2), nullptr,
                                                j + 1, L, pass == 1 ? npart : nullptr);
        }
        k_normalize<<<nblk(L), kB, 0, st>>>(V, L, vn, npart, (int)nblk(L), hdev + 2 * (kMaxRestart + 2), nullptr, j,
                                            nullptr, L);
        KFBI_HIP(hipGetLastError());
        KFBI_HIP(hipMemcpyAsync(hhost, hdev, 3 * (kMaxRestart + 2) * sizeof(double), hipMemcpyDeviceToHost, st));
      }
      count(pj);
      ++s.its;
      if (graphed) wait_step(st);
      else KFBI_HIP(hipStreamSynchronize(st));
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hhost[i] + hhost[(kMaxRestart + 2) + i];
      const double hn = std::sqrt(std::max(0.0, hhost[2 * (kMaxRestart + 2)]));
      H[(size_t)(j + 1) * m + j] = hn;
      for (int i = 0; i <= j + 1; ++i) Hc[(size_t)i * m + j] = H[(size_t)i * m + j];   // before rotations
      for (int i = 0; i < j; ++i) {
        const double av = H[(size_t)i * m + j], cv = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * av + sn[i] * cv;
        H[(size_t)(i + 1) * m + j] = -sn[i] * av + cs[i] * cv;
      }
      const double av = H[(size_t)j * m + j], cv = H[(size_t)(j + 1) * m + j];
      const double den = std::hypot(av, cv);
      cs[j] = den > 0 ? av / den : 1.0;
      sn[j] = den > 0 ? cv / den : 0.0;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      jend = j + 1;
      // relaxed solve: after FP32 products the computed residual differs from the true one by
      // the products' errors weighted with the solution's coefficients; converging it to a
      // quarter of the tolerance leaves that gap room before the FP64 certificate
      target = any32 && a.relax ? 0.25 * tol_abs : tol_abs;
      if (std::fabs(g[j + 1]) <= target || s.its >= maxit) break;
      if (hn == 0.0) {
        breakdown = true;
        break;
      }
    }
    for (int i = jend - 1; i >= 0; --i) {
      double acc = g[i];
      for (int k = i + 1; k < jend; ++k) acc -= H[(size_t)i * m + k] * y[k];
      y[i] = acc / H[(size_t)i * m + i];
    }
    // x += V y
    std::copy(y.begin(), y.begin() + jend, ypin);
    KFBI_HIP(hipMemcpyAsync(ydev, ypin, jend * sizeof(double), hipMemcpyHostToDevice, st));
    k_combine<<<nblk(L), kB, 0, st>>>(x, V, L, ydev, jend, 1.0, L);
    KFBI_HIP(hipGetLastError());
    const bool converged = std::fabs(g[jend]) <= target && !breakdown;
    if (converged && !(any32 && a.relax)) {
      // the residual vector follows from the Arnoldi relation without a product,
      //   b - A x = V_{j+1} (beta e_1 - Hbar y):
      // exact to rounding when every product was FP64; for an FP32-operator solve (the inner
      // solve of iterative refinement) it is the residual of that operator, which the caller
      // does not use: it takes the FP64 residual itself.  Checking it with an FP32 product
      // instead would restart without end once the solution's norm makes the product's
      // rounding exceed the tolerance (a large near-null component of the coupled pair).
      for (int i = 0; i <= jend; ++i) {
        double acc = i == 0 ? beta_cycle : 0.0;
        for (int k = 0; k < jend; ++k) acc -= Hc[(size_t)i * m + k] * y[k];
        z[i] = acc;
      }
      std::copy(z.begin(), z.begin() + jend + 1, ypin + (kMaxRestart + 2));
      KFBI_HIP(hipMemcpyAsync(ydev, ypin + (kMaxRestart + 2), (jend + 1) * sizeof(double), hipMemcpyHostToDevice,
                              st));
      k_axpby<<<nblk(L), kB, 0, st>>>(r, 0.0, r, 0.0, nullptr, L);
      k_combine<<<nblk(L), kB, 0, st>>>(r, V, L, ydev, jend + 1, 1.0, L);
      KFBI_HIP(hipGetLastError());
      beta = std::fabs(g[jend]);
      host_wait(st);
      break;
    }
    // the true residual: the FP64 certificate of a relaxed solve, else a restart
    const int pr = any32 && a.relax ? 0 : prec_res;
    apply_vec(p, pr, x, t, st);
    count(pr);
    if (a.relax && any32) ++s.certs;
    k_axpby<<<nblk(L), kB, 0, st>>>(r, 1.0, b, -1.0, t, L);
    beta = std::sqrt(dot(r, r, st));
  }
  s.resid = beta;
  return beta <= tol_abs ? KFBI_OK : KFBI_ENOCONV;
}

// ||v|| or, with nz (unit), ||v - <nz, v> nz|| (formed, not by subtracting squares); uses w
double Solver::norm_without(const double *v, const double *nz, hipStream_t st) {
  if (!nz) return std::sqrt(dot(v, v, st));
  const double c = dot(nz, v, st);
  k_axpby<<<nblk(L), kB, 0, st>>>(w, 1.0, v, -c, nz, L);
  KFBI_HIP(hipGetLastError());
  return std::sqrt(dot(w, w, st));
}

int Solver::richardson(DevProblem &p, const double *b, double bnorm, double *x, double gamma, double tol_abs,
                       int maxit, int &its, int &matvecs, double &resid, hipStream_t st, double *r0,
                       const double *nz) {
  its = 0;
  for (;;) {
    apply_vec(p, 0, x, t, st);
    ++matvecs;
    k_axpby<<<nblk(L), kB, 0, st>>>(r, 1.0, b, -1.0, t, L);
    resid = norm_without(r, nz, st);
    if (r0 && its == 0) *r0 = resid;
    if (resid <= tol_abs || its >= maxit) break;
    k_axpby<<<nblk(L), kB, 0, st>>>(x, 1.0, x, 2.0 * gamma, r, L);
    ++its;
  }
  (void)bnorm;
  return resid <= tol_abs ? KFBI_OK : KFBI_ENOCONV;
}

void Solver::bie_rhs(DevProblem &p, const double *g, hipStream_t st, const FhnArgs *fa) {
  // u_V is needed only at the extrapolation stencils of the interface nodes
  if (fa) bidomain_volume_solve(p, *fa, st);
  else box_solve_stencils<double>(p, fpad, st);
  launch_gather<double>(p, p.f64.work, false, t, st);
  if (g)
    k_axpby<<<nblk(L), kB, 0, st>>>(gp, 1.0, g, -1.0, t, L);
  else
    k_axpby<<<nblk(L), kB, 0, st>>>(gp, -1.0, t, 0.0, nullptr, L);
  KFBI_HIP(hipGetLastError());
}

int Solver::solve_density(DevProblem &p, double *psi, const kfbi_solve_opts &o, bool x0, kfbi_solve_info &info,
                          hipStream_t st, const double *r0, const int *r0_bad) {
  const double gn = std::sqrt(dot(gp, gp, st));
  if (r0 && r0_bad && *r0_bad) r0 = nullptr;   // read after the wait above: r0 does not belong to psi
  info.gp_norm = gn;
  double ref = gn;   // the norm the residual is measured against
  double tol_abs = o.tol * gn;
  int rc = KFBI_OK;
  double res = 0, res0 = gn;
  if (!x0) KFBI_HIP(hipMemsetAsync(psi, 0, L * sizeof(double), st));
  if (o.method == 1) {
    // the coupled pair: residual and right-hand side measured without their component along
    // the null density (the part of g' that no density can match), the iterates unchanged
    const double *nz = p.ncomp == 2 && null_ready ? nullz : nullptr;
    if (nz) {
      ref = norm_without(gp, nz, st);
      tol_abs = o.tol * ref;
      res0 = ref;
    }
    int its = 0, mv = 0;
    rc = richardson(p, gp, ref, psi, o.gamma, tol_abs, o.max_iters, its, mv, res, st, &res0, nz);
    info.iters = its;
    info.matvecs_fp64 = mv;
    last_resid = r;
  } else if (o.precision == 0 || o.precision == 2) {
    // precision 2: one GMRES whose products turn FP32 once the residual is below inner_tol ||g'||,
    // with an FP64 product of the result as its certificate
    GmresArgs a;
    a.relax = o.precision == 2;
    a.sw_abs = o.inner_tol * gn;
    a.r0 = r0;
    GmresStats gs;
    rc = gmres(p, gp, gn, psi, !x0, tol_abs, o.restart, o.max_iters, a, gs, st);
    info.iters = gs.its;
    info.outer = gs.certs;
    info.matvecs_fp64 = gs.mv64;
    info.matvecs_fp32 = gs.mv32;
    res = gs.resid;
    res0 = gs.beta0;
    last_resid = r;
  } else {
    // iterative refinement: FP64 residual, FP32-operator GMRES on the correction
    int total = 0, mv64 = 0, mv32 = 0, outer = 0;
    bool have_x = x0;
    for (;;) {
      if (have_x && outer == 0 && r0) {
        KFBI_HIP(hipMemcpyAsync(d, r0, L * sizeof(double), hipMemcpyDeviceToDevice, st));
      } else if (have_x) {
        apply_vec(p, 0, psi, t, st);
        ++mv64;
        k_axpby<<<nblk(L), kB, 0, st>>>(d, 1.0, gp, -1.0, t, L);
      } else {
        KFBI_HIP(hipMemcpyAsync(d, gp, L * sizeof(double), hipMemcpyDeviceToDevice, st));
      }
      res = std::sqrt(dot(d, d, st));
      if (outer == 0) res0 = res;
      if (res <= tol_abs || outer >= o.max_outer || total >= o.max_iters) break;
      KFBI_HIP(hipMemsetAsync(w, 0, L * sizeof(double), st));
      const double tin = std::max(o.inner_tol * res, 0.5 * tol_abs);
      GmresArgs a;
      a.prec = 1;
      GmresStats gs;
      gmres(p, d, res, w, true, tin, o.restart, o.max_iters - total, a, gs, st);
      total += gs.its;
      mv32 += gs.mv32;
      k_axpby<<<nblk(L), kB, 0, st>>>(psi, 1.0, psi, 1.0, w, L);
      have_x = true;
      ++outer;
    }
    last_resid = d;
    info.iters = total;
    info.outer = outer;
    info.matvecs_fp64 = mv64;
    info.matvecs_fp32 = mv32;
    rc = res <= tol_abs ? KFBI_OK : KFBI_ENOCONV;
  }
  info.rel_resid = ref > 0 ? res / ref : 0.0;
  info.start_resid = ref > 0 ? res0 / ref : 0.0;
  info.true_resid = -1.0;
  if (o.true_resid) {
    // a check: the FP64 residual of the returned density by an explicit product (not counted);
    // d may be last_resid, which it then overwrites with the same vector
    apply_vec(p, 0, psi, t, st);
    double tr = residual_norm(gp, t, st);   // leaves gp - A psi in d
    // measured as the solve measured it: the simple iteration on the coupled pair without the
    // component along the null density
    if (o.method == 1 && p.ncomp == 2 && null_ready) tr = norm_without(d, nullz, st);
    info.true_resid = ref > 0 ? tr / ref : 0.0;
  }
  return rc;
}

void Solver::null_init(DevProblem &p, hipStream_t st) {
  if (p.ncomp != 2 || null_ready) return;
  // inverse iteration from the constant density: z <- A^{-1} z / |A^{-1} z|, each step one FP64
  // GMRES solve to 1e-12, until successive unit iterates agree to 1e-10 up to sign
  k_fill<<<nblk(L), kB, 0, st>>>(nullz, 1.0 / std::sqrt((double)L), L);
  KFBI_HIP(hipGetLastError());
  GmresArgs a;
  for (int it = 0; it < 6; ++it) {
    GmresStats gs;
    k_fill<<<nblk(L), kB, 0, st>>>(nully, 0.0, L);   // gmres adds its update to x
    (void)gmres(p, nullz, 1.0, nully, true, 1e-12, 50, 500, a, gs, st);
    const double ny = std::sqrt(dot(nully, nully, st));
    if (!(ny > 0)) break;
    const double sc = dot(nully, nullz, st) < 0 ? -1.0 / ny : 1.0 / ny;
    k_axpby<<<nblk(L), kB, 0, st>>>(nullp, sc, nully, -1.0, nullz, L);
    const double dn = std::sqrt(dot(nullp, nullp, st));
    k_axpby<<<nblk(L), kB, 0, st>>>(nullz, sc, nully, 0.0, nullptr, L);
    KFBI_HIP(hipGetLastError());
    if (dn < 1e-10) break;
  }
  null_ready = true;
}

void Solver::reconstruct(DevProblem &p, const double *psi, hipStream_t st, const FhnArgs *fa, bool fuse_be) {
  if (p.ncomp == 2) {
    // the coupled pair: the density without its component along the null density
    if (!null_ready) throw std::logic_error("reconstruct: null density not initialised");
    k_multidot<<<dim3(nb, 1), kB, 0, st>>>(nullz, L, psi, L, partials);
    k_finish<<<1, kB, 0, st>>>(partials, nb, nullc);
    k_remove_along<<<nblk(L), kB, 0, st>>>(nullp, psi, nullz, nullc, L);
    KFBI_HIP(hipGetLastError());
    psi = nullp;
  }
  launch_jumps<double>(p, psi, st);
  if (fa) {
    launch_correct<double>(p, st);
    bidomain_final_solve(p, *fa, fuse_be, st);
    return;
  }
  launch_add_correction<double>(p, fpad, st);
  box_solve<double>(p, fpad, false, p.f64.work, false, st);
}

double Solver::gauge_mean(DevProblem &p, hipStream_t st) {
  // mean over tissue nodes of comp 1 in the padded work field (mask in padded layout)
  k_masked_sum<<<nb, kB, 0, st>>>(p.f64.work + p.comp_stride, p.inside_pad, p.comp_stride, partials);
  k_finish<<<1, kB, 0, st>>>(partials, nb, hdev);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipMemcpyAsync(hhost, hdev, sizeof(double), hipMemcpyDeviceToHost, st));
  host_wait(st);
  return n_inside > 0 ? hhost[0] / (double)n_inside : 0.0;
}

namespace {
__global__ __launch_bounds__(kB) void k_from_padded(const double *__restrict__ fp, double *__restrict__ f,
                                                    int64_t nplain, int64_t N, int64_t P, int64_t cs, int ncomp,
                                                    double shift) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= nplain * ncomp) return;
  const int64_t c = i / nplain, lin = i - c * nplain;
  f[i] = fp[c * cs + (lin % N) + P * (lin / N)] - shift;
}
}  // namespace

int Solver::solve_neumann(DevProblem &p, const double *g, const double *f, double *u, double *psi,
                          const kfbi_solve_opts &o, kfbi_solve_info &info, hipStream_t st) {
  if (o.restart < 1 || o.max_iters < 0 || !(o.tol > 0)) throw std::invalid_argument("solve options");
  null_init(p, st);
  const int64_t nplain = (int64_t)p.ht.inside.size();
  k_to_padded<<<nblk(nplain * p.ncomp), kB, 0, st>>>(f, fpad, nplain, p.N, p.P, p.comp_stride, p.ncomp);
  KFBI_HIP(hipGetLastError());
  bie_rhs(p, g, st);
  const int rc = solve_density(p, psi, o, o.x0 != 0, info, st);
  reconstruct(p, psi, st);
  const double shift = p.ncomp == 2 ? gauge_mean(p, st) : 0.0;
  k_from_padded<<<nblk(nplain * p.ncomp), kB, 0, st>>>(p.f64.work, u, nplain, p.N, p.P, p.comp_stride, p.ncomp,
                                                       shift);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipStreamSynchronize(st));
  return rc;
}

}  // namespace kfbi

using namespace kfbi;

void bidomain_s::init() {
  const int64_t L = solver->L;
  KFBI_HIP(hipMalloc(&psi0, L * sizeof(double)));
  KFBI_HIP(hipMalloc(&r0v, L * sizeof(double)));
  KFBI_HIP(hipMalloc(&gp_prev, L * sizeof(double)));
  KFBI_HIP(hipMemset(gp_prev, 0, L * sizeof(double)));
  KFBI_HIP(hipMalloc(&d_prev, L * sizeof(double)));
  KFBI_HIP(hipMemset(d_prev, 0, L * sizeof(double)));
  KFBI_HIP(hipMalloc(&psi_last, L * sizeof(double)));
  KFBI_HIP(hipMemset(psi_last, 0, L * sizeof(double)));
  KFBI_HIP(hipMalloc(&zdir, L * sizeof(double)));
  KFBI_HIP(hipMalloc(&r0_bad_dev, sizeof(int)));
  KFBI_HIP(hipMemset(r0_bad_dev, 0, sizeof(int)));
  KFBI_HIP(hipHostMalloc(&r0_bad_host, sizeof(int), hipHostMallocDefault));
  *r0_bad_host = 0;
  if (params.warm_start == 3 || params.warm_start == 4) {
    KFBI_HIP(hipMalloc(&proj_psi, (size_t)kProj * L * sizeof(double)));
    KFBI_HIP(hipMalloc(&proj_b, (size_t)kProj * L * sizeof(double)));
  }
}

// Start of least residual over span{psi_j}: c = argmin ||g' - B c|| from the normal equations
// (Gram matrix kept up to date as solutions are recorded, a tiny diagonal shift against
// near-collinear columns); psi0 = sum c_j psi_j and its residual g' - sum c_j b_j follow
// without a product.  Any c gives a consistent pair, so the shift affects only the quality.
void bidomain_s::proj_start(double *out_psi, double *out_r, hipStream_t st) {
  Solver &sv = *solver;
  const int64_t L = sv.L;
  const int k = proj_n;
  k_multidot<<<dim3(sv.nb, k), kB, 0, st>>>(proj_b, L, sv.gp, L, sv.partials);
  k_finish<<<k, kB, 0, st>>>(sv.partials, sv.nb, sv.hdev);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipMemcpyAsync(sv.hhost, sv.hdev, k * sizeof(double), hipMemcpyDeviceToHost, st));
  sv.host_wait(st);
  double A[kProj][kProj + 1];
  double dmax = 0;
  for (int i = 0; i < k; ++i) dmax = std::max(dmax, proj_G[i][i]);
  for (int i = 0; i < k; ++i) {
    for (int j = 0; j < k; ++j) A[i][j] = proj_G[i][j] + (i == j ? 1e-13 * dmax : 0.0);
    A[i][k] = sv.hhost[i];
  }
  for (int c = 0; c < k; ++c) {   // Gaussian elimination with partial pivoting
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    for (int j = 0; j <= k; ++j) std::swap(A[c][j], A[piv][j]);
    if (A[c][c] == 0.0) continue;
    for (int r = c + 1; r < k; ++r) {
      const double f = A[r][c] / A[c][c];
      for (int j = c; j <= k; ++j) A[r][j] -= f * A[c][j];
    }
  }
  std::vector<double> cvec(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double acc = A[i][k];
    for (int j = i + 1; j < k; ++j) acc -= A[i][j] * cvec[j];
    cvec[i] = A[i][i] != 0.0 ? acc / A[i][i] : 0.0;
  }
  std::copy(cvec.begin(), cvec.begin() + k, sv.ypin);
  KFBI_HIP(hipMemcpyAsync(sv.ydev, sv.ypin, k * sizeof(double), hipMemcpyHostToDevice, st));
  k_axpby<<<nblk(L), kB, 0, st>>>(out_psi, 0.0, out_psi, 0.0, nullptr, L);
  k_combine<<<nblk(L), kB, 0, st>>>(out_psi, proj_psi, L, sv.ydev, k, 1.0, L);
  KFBI_HIP(hipMemcpyAsync(out_r, sv.gp, L * sizeof(double), hipMemcpyDeviceToDevice, st));
  k_combine<<<nblk(L), kB, 0, st>>>(out_r, proj_b, L, sv.ydev, k, -1.0, L);
  KFBI_HIP(hipGetLastError());
}

// Record the solution just computed: psi and b = g' - (final residual), and the new Gram row.
void bidomain_s::proj_record(const double *psi, hipStream_t st) {
  Solver &sv = *solver;
  const int64_t L = sv.L;
  const int slot = proj_head;
  double *bs = proj_b + (int64_t)slot * L;
  KFBI_HIP(hipMemcpyAsync(proj_psi + (int64_t)slot * L, psi, L * sizeof(double), hipMemcpyDeviceToDevice, st));
  k_axpby<<<nblk(L), kB, 0, st>>>(bs, 1.0, sv.gp, -1.0, sv.last_resid, L);
  proj_head = (proj_head + 1) % kProj;
  proj_n = std::min(proj_n + 1, kProj);
  k_multidot<<<dim3(sv.nb, proj_n), kB, 0, st>>>(proj_b, L, bs, L, sv.partials);
  k_finish<<<proj_n, kB, 0, st>>>(sv.partials, sv.nb, sv.hdev);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipMemcpyAsync(sv.hhost, sv.hdev, proj_n * sizeof(double), hipMemcpyDeviceToHost, st));
  sv.host_wait(st);
  for (int i = 0; i < proj_n; ++i) proj_G[slot][i] = proj_G[i][slot] = sv.hhost[i];
}

void bidomain_s::reset() {
  have_prev = false;
  hist_last = nullptr;
  proj_n = 0;
  proj_head = 0;
  steps_done = 0;
}

void bidomain_s::release() {
  double *ps[] = {psi0, r0v, gp_prev, d_prev, psi_last, zdir, proj_psi, proj_b};
  for (double *q : ps)
    if (q) (void)hipFree(q);
  psi0 = r0v = gp_prev = d_prev = psi_last = zdir = proj_psi = proj_b = nullptr;
  if (r0_bad_dev) (void)hipFree(r0_bad_dev);
  if (r0_bad_host) (void)hipHostFree(r0_bad_host);
  r0_bad_dev = nullptr;
  r0_bad_host = nullptr;
  extern void mlp_release(bidomain_s *);
  mlp_release(this);
}

extern bool mlp_warm_start(bidomain_s *b, const double *psi1, const double *psi2, double *out, hipStream_t st);
extern bool mlp_should_check(bidomain_s *b);
extern void mlp_disable(bidomain_s *b);
extern void mlp_record(bidomain_s *b, const double *psi1, const double *psi2, const double *psi, hipStream_t st);
extern void mlp_note_cost(bidomain_s *b, double cost, bool learned);

int bidomain_s::step(bidomain_state &s, double dt, kfbi_solve_info &info, hipStream_t st) {
  DevProblem &p = *prob;
  Solver &sv = *solver;
  const int64_t n = (int64_t)p.ht.inside.size(), L = sv.L;
  const double dth = 0.5 * dt;
  const FhnCoef m{params.Cm,  params.H,           params.theta,       params.alpha,
                  params.zeta, params.newton_tol, params.newton_maxit, 1.0 / params.Cm,
                  1.0 / (1.0 + dth * params.zeta)};
  const FhnArgs fa{s.V, s.q, s.I_stim, dth, p.kappa, params.beta, m};
  // step 1 (reaction over dt/2, forward Euler) is computed where its result is used: in the x
  // passes of the box solves of step 2 (diffusion, backward Euler over dt/2 for
  // w = (V^{n+1} + V^n)/2, a Neumann BVP); V and q change only at the end of the step
  // the recycled residual is usable only on the history array of the previous step (and, checked
  // on the device, only if its newest density is still the one that step returned)
  const bool prev_ok = have_prev && s.psi_hist == hist_last;
  have_prev = false;   // set again when this step completes
  sv.null_init(p, st);   // once: before any of the step's vectors are formed
  sv.bie_rhs(p, nullptr, st, &fa);
  double *hist1 = s.psi_hist, *hist2 = s.psi_hist + L;
  kfbi_solve_opts o = params.solve;
  bool x0 = true;
  bool have_r0 = false;
  const int *r0_flag = nullptr;   // set while r0v holds the recycled residual, not yet validated
  info.warm_start_used = 0;
  int extra32 = 0, extra64 = 0;
  if (params.warm_start == 2) {
    x0 = false;
  } else {
    // start from psi^{n-1}: its residual is known without a product,
    //   g'^n - A psi^{n-1} = g'^n - g'^{n-1} + (g'^{n-1} - A psi^{n-1}),
    // the last term being the final FP64 residual of the previous solve
    KFBI_HIP(hipMemcpyAsync(psi0, hist1, L * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (prev_ok) {
      k_recycled_resid<<<nblk(L), kB, 0, st>>>(r0v, sv.gp, gp_prev, d_prev, hist1, psi_last, r0_bad_dev, L);
      KFBI_HIP(hipGetLastError());
      KFBI_HIP(hipMemcpyAsync(r0_bad_host, r0_bad_dev, sizeof(int), hipMemcpyDeviceToHost, st));
      have_r0 = true;
      r0_flag = r0_bad_host;
    }
    if ((params.warm_start == 3 || params.warm_start == 4) && proj_n >= 2) {
      // least-residual start over the recorded solutions (its residual is exact whatever the
      // caller's history holds); kept only if that residual is below psi^{n-1}'s, or taken
      // when psi^{n-1}'s residual is unknown or invalid
      proj_start(sv.w, sv.d, st);
      const double rp = sv.dot(sv.d, sv.d, st);
      const bool r0_valid = have_r0 && !*r0_bad_host;   // read after the waits above
      const double rh = r0_valid ? sv.dot(r0v, r0v, st) : 0.0;
      if (!r0_valid || rp < rh) {
        KFBI_HIP(hipMemcpyAsync(psi0, sv.w, L * sizeof(double), hipMemcpyDeviceToDevice, st));
        KFBI_HIP(hipMemcpyAsync(r0v, sv.d, L * sizeof(double), hipMemcpyDeviceToDevice, st));
        info.warm_start_used = 1;
        have_r0 = true;
      }
      r0_flag = nullptr;   // r0v now holds a validated or an exact residual
    } else if (params.warm_start == 1 && mlp && steps_done >= 2 && mlp_warm_start(this, hist1, hist2, sv.w, st)) {
      if (have_r0) {
        // predicted start psi^{n-1} + D: residual r0 - A D, taken only if smaller than
        // psi^{n-1}'s (checked at every use: it costs nothing more).  A D is applied in the
        // precision of the inner solves: FP32 rounding noise in the starting residual would
        // slow an FP64 GMRES that must resolve it, while iterative refinement absorbs it.
        k_axpby<<<nblk(L), kB, 0, st>>>(sv.w, 1.0, sv.w, -1.0, hist1, L);
        const int pd = o.precision != 0 && o.method == 0 ? 1 : 0;
        sv.apply_vec(p, pd, sv.w, sv.t, st);
        if (pd) extra32 = 1;
        else extra64 = 1;
        k_axpby<<<nblk(L), kB, 0, st>>>(sv.d, 1.0, r0v, -1.0, sv.t, L);
        const double rh = sv.dot(r0v, r0v, st), rp = sv.dot(sv.d, sv.d, st);
        if (*r0_bad_host) {
          have_r0 = false;   // psi^{n-1} is not the previous solution: no recycled residual
        } else if (rp < rh) {
          k_axpby<<<nblk(L), kB, 0, st>>>(psi0, 1.0, hist1, 1.0, sv.w, L);
          KFBI_HIP(hipMemcpyAsync(r0v, sv.d, L * sizeof(double), hipMemcpyDeviceToDevice, st));
          info.warm_start_used = 1;
        } else {
          mlp_disable(this);
        }
        r0_flag = nullptr;
      } else if (mlp_should_check(this)) {
        // no recycled residual (first steps): compare FP32 residuals of both starts
        sv.apply_vec(p, 1, sv.w, sv.t, st);
        const double rp = sv.residual_norm(sv.gp, sv.t, st);
        sv.apply_vec(p, 1, hist1, sv.t, st);
        const double rh = sv.residual_norm(sv.gp, sv.t, st);
        extra32 = 2;
        if (rp < rh) {
          KFBI_HIP(hipMemcpyAsync(psi0, sv.w, L * sizeof(double), hipMemcpyDeviceToDevice, st));
          info.warm_start_used = 1;
        } else {
          mlp_disable(this);
        }
      } else {
        KFBI_HIP(hipMemcpyAsync(psi0, sv.w, L * sizeof(double), hipMemcpyDeviceToDevice, st));
        info.warm_start_used = 1;
      }
    }
  }
  // warm_start 4: one minimal-residual step from the projection start along the network's
  // predicted correction d = prediction - start: psi0 += a d, r0 -= a A d with
  // a = <A d, r0> / |A d|^2.  It costs one FP64 product and cannot increase the residual; the cost
  // check below switches it off when the solves it starts are not cheaper than those without it.
  // (Taking d as GMRES's first search direction instead saves that product, but drops the
  // residual itself from the search space: a poor prediction then slows GMRES down.)
  bool learned_dir = false;
  if (params.warm_start == 4 && mlp && steps_done >= 2 && o.method == 0 && have_r0 && !r0_flag &&
      mlp_warm_start(this, hist1, hist2, zdir, st)) {
    k_axpby<<<nblk(L), kB, 0, st>>>(zdir, 1.0, zdir, -1.0, psi0, L);
    if (p.ncomp == 2 && sv.null_ready) {
      // without its component along the null density: the network also predicts the density's
      // step-dependent null component, which A hardly sees, and the step would scale it freely
      k_multidot<<<dim3(sv.nb, 1), kB, 0, st>>>(sv.nullz, L, zdir, L, sv.partials);
      k_finish<<<1, kB, 0, st>>>(sv.partials, sv.nb, sv.nullc);
      k_remove_along<<<nblk(L), kB, 0, st>>>(zdir, zdir, sv.nullz, sv.nullc, L);
    }
    KFBI_HIP(hipGetLastError());
    sv.apply_vec(p, 0, zdir, sv.t, st);
    ++extra64;
    learned_dir = true;   // its product is charged to the learned steps either way
    info.warm_start_used |= 4;
    const double tt = sv.dot(sv.t, sv.t, st), tr = sv.dot(sv.t, r0v, st), rr = sv.dot(r0v, r0v, st);
    // taken only if it cuts the residual at least tenfold (|r0 - a A d|^2 = |r0|^2 - tr^2 / tt):
    // less is worth less than the GMRES iteration its product costs, and a rough correction can
    // make the residual harder for GMRES even where it makes it smaller
    if (tt > 0 && rr - tr * tr / tt <= 0.01 * rr) {
      const double a = tr / tt;
      k_axpby<<<nblk(L), kB, 0, st>>>(psi0, 1.0, psi0, a, zdir, L);
      k_axpby<<<nblk(L), kB, 0, st>>>(r0v, 1.0, r0v, -a, sv.t, L);
      KFBI_HIP(hipGetLastError());
      info.warm_start_used |= 2;
    }
  }
  const int rc = sv.solve_density(p, psi0, o, x0, info, st, have_r0 ? r0v : nullptr, r0_flag);
  info.matvecs_fp32 += extra32;
  info.matvecs_fp64 += extra64;
  KFBI_HIP(hipMemcpyAsync(d_prev, sv.last_resid, L * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (params.warm_start == 3 || params.warm_start == 4) proj_record(psi0, st);
  // u = S(f + C psi); the midpoint update and step 3 (reaction over dt/2, backward Euler) ride
  // in its inverse x pass unless the potentials are returned as well
  sv.reconstruct(p, psi0, st, &fa, s.phi == nullptr);
  if (s.phi) {
    const double mu = sv.gauge_mean(p, st);
    sv.hhost[0] = mu;
    KFBI_HIP(hipMemcpyAsync(sv.ydev, sv.hhost, sizeof(double), hipMemcpyHostToDevice, st));
    k_mid_be<<<nblk(n), kB, 0, st>>>(p.f64.work, s.V, s.q, s.phi, sv.ydev, n, p.N, p.P, p.comp_stride, dth, m);
    KFBI_HIP(hipGetLastError());
  }
  // record (features, target) once two earlier densities and g'^{n-1} exist
  if (mlp && steps_done >= 2) {
    mlp_record(this, hist1, hist2, psi0, st);
    if (params.warm_start == 1) mlp_note_cost(this, info.matvecs_fp64 + 0.5 * info.matvecs_fp32, info.warm_start_used);
    if (params.warm_start == 4) mlp_note_cost(this, info.matvecs_fp64 + 0.5 * info.matvecs_fp32, learned_dir);
  }
  ++steps_done;
  k_end_step<<<nblk(L), kB, 0, st>>>(gp_prev, sv.gp, hist2, hist1, psi_last, psi0, r0_bad_dev, L);
  KFBI_HIP(hipGetLastError());
  sv.host_wait(st);
  have_prev = true;
  hist_last = s.psi_hist;
  return rc;
}
