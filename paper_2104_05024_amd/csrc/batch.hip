// Batched two-dimensional Neumann problems (many interfaces of uneven grid sizes at once).
//
// Every problem keeps its own setup tables; the batch adds
//   * size groups: problems with the same grid size share padded field buffers (stride
//     N * M), so each DST pass of a group is one launch (blockIdx.y = problem for the fused
//     last-axis pass, with per-problem mode parameters);
//   * work lists: the jump, correction and gather kernels of all problems run as one launch
//     each over the concatenated items, the problem found by a binary search over prefix sums;
//   * GMRES(m) for all problems in lockstep on concatenated vectors [problem][M_p]: per-problem
//     dot products, Gram-Schmidt (two passes), norms and basis updates are segment kernels;
//     the Givens least-squares updates run on the host, one synchronisation per iteration.
//     One Arnoldi step (copy of v_j, the batched product, both Gram-Schmidt passes, the norm,
//     v_{j+1}, the copy of the new Hessenberg column to pinned host memory and j <- j + 1)
//     reads j from device memory, so a single hipGraph serves every iteration; it is
//     captured on first use and replayed.
//   * mixed precision as for one problem: FP64 residuals and refinement, FP32-operator inner
//     GMRES with per-problem tolerances.
#include <algorithm>
#include <cmath>
#include <memory>
#include <stdexcept>
#include <vector>

#include "batch.h"

namespace kfbi {
namespace {

constexpr int kB = 256;
inline unsigned nb(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

template <typename T>
T *balloc(size_t n) {
  T *p = nullptr;
  KFBI_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
  KFBI_HIP(hipMemset(p, 0, std::max<size_t>(n, 1) * sizeof(T)));
  return p;
}

// out[y * np + p] = <A_y, w> over segment p, for y <= *jlim (all y if jlim is null)
__global__ __launch_bounds__(kB) void k_seg_dot(const double *__restrict__ A, int64_t lda,
                                                const int *__restrict__ jlim, const double *__restrict__ w,
                                                const int64_t *__restrict__ off, int np, double *__restrict__ out) {
  const int p = blockIdx.x, y = blockIdx.y;
  if (jlim && y > *jlim) return;
  __shared__ double sh[kB];
  const int64_t b = off[p], e = off[p + 1];
  const double *a = A + (int64_t)y * lda;
  double s = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += kB) s += a[i] * w[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)y * np + p] = sh[0];
}

// w -= sum_{i <= j} h[i][pid] V_i
__global__ __launch_bounds__(kB) void k_seg_combine(double *__restrict__ w, const double *__restrict__ V,
                                                    int64_t L, const int *__restrict__ jdev,
                                                    const double *__restrict__ h, const int16_t *__restrict__ pid,
                                                    int np) {
  const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e >= L) return;
  const int j = *jdev, p = pid[e];
  double acc = w[e];
  for (int i = 0; i <= j; ++i) acc -= h[(int64_t)i * np + p] * V[(int64_t)i * L + e];
  w[e] = acc;
}

// V_{j+1} = w / sqrt(nn[pid]) (zero where the norm vanishes)
__global__ __launch_bounds__(kB) void k_seg_next(const double *__restrict__ w, const double *__restrict__ nn,
                                                 const int16_t *__restrict__ pid, double *__restrict__ V, int64_t L,
                                                 const int *__restrict__ jdev) {
  const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e >= L) return;
  const double n2 = nn[pid[e]];
  V[(int64_t)(*jdev + 1) * L + e] = n2 > 0 ? w[e] / sqrt(n2) : 0.0;
}

__global__ __launch_bounds__(kB) void k_take(const double *__restrict__ V, int64_t L, const int *__restrict__ jdev,
                                             double *__restrict__ v) {
  const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e < L) v[e] = V[(int64_t)(*jdev) * L + e];
}

// j <- j + 1 (when given), and the step counter: seq <- seq + 1, also stored to the host's copy
__global__ void k_inc(int *j, int *seq, int *seq_host) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (j) *j += 1;
    const int s = *seq + 1;
    *seq = s;
    __threadfence_system();
    __hip_atomic_store(seq_host, s, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// V_0 = r * s[pid] (s = 1/beta, or 0 for problems that are done)
__global__ __launch_bounds__(kB) void k_seg_scale(const double *__restrict__ r, const double *__restrict__ s,
                                                  const int16_t *__restrict__ pid, double *__restrict__ out,
                                                  int64_t L) {
  const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e < L) out[e] = r[e] * s[pid[e]];
}

// x += sum_{i < jmax} y[i][pid] V_i
__global__ __launch_bounds__(kB) void k_seg_update(double *__restrict__ x, const double *__restrict__ V, int64_t L,
                                                   const double *__restrict__ y, const int16_t *__restrict__ pid,
                                                   int np, int jmax) {
  const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e >= L) return;
  const int p = pid[e];
  double acc = x[e];
  for (int i = 0; i < jmax; ++i) acc += y[(int64_t)i * np + p] * V[(int64_t)i * L + e];
  x[e] = acc;
}

__global__ __launch_bounds__(kB) void k_axpby(double *__restrict__ z, double a, const double *__restrict__ x,
                                              double b, const double *__restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) z[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

template <typename A, typename B>
__global__ __launch_bounds__(kB) void k_cast(const A *__restrict__ a, B *__restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) b[i] = (B)a[i];
}

// zero the segments of problems whose mask entry is 0
__global__ __launch_bounds__(kB) void k_seg_mask(double *__restrict__ v, const int16_t *__restrict__ pid,
                                                 const double *__restrict__ keep, int64_t L) {
  const int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (e < L && keep[pid[e]] == 0.0) v[e] = 0.0;
}

__device__ __forceinline__ int find_seg(const int64_t *__restrict__ cum, int n, int64_t i) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (cum[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// caller layout (concatenated [problem][N_p^2]) <-> padded group buffers
__global__ __launch_bounds__(kB) void k_pack(double *__restrict__ plain, const int64_t *__restrict__ gcum,
                                             const PackItem *__restrict__ it, int n, int64_t tot, int which,
                                             int to_padded) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= tot) return;
  const int p = find_seg(gcum, n, i);
  const PackItem &q = it[p];
  const int64_t lin = i - gcum[p];
  double *pad = which == 0 ? q.fpad : q.work;
  const int64_t pos = (lin % q.N) + q.P * (lin / q.N);
  if (to_padded)
    pad[pos] = plain[i];
  else
    plain[i] = pad[pos];
}

}  // namespace

void Batch::init(int n, const kfbi_interface *ifaces, const kfbi_grid *grids, const kfbi_coeffs *coeffs) {
  if (n < 1 || n > 32767) throw std::invalid_argument("batch size");
  np = n;
  probs.resize(n);
  for (int i = 0; i < n; ++i) {
    if (ifaces[i].dim != 2 || grids[i].dim != 2 || coeffs[i].ncomp != 1)
      throw std::invalid_argument("batched problems are two-dimensional with one component");
    const int c = grids[i].cells;
    if (c < 16 || c > 1024 || (c & (c - 1)) != 0) throw std::invalid_argument("cells must be 2^k in [16, 1024]");
    probs[i] = std::make_unique<DevProblem>();
    build_host_tables(ifaces[i], grids[i], coeffs[i], probs[i]->ht);
  }
  for (int i = 0; i < n; ++i) {
    KFBI_HIP(hipGetDevice(&probs[i]->dev));
    upload_tables(*probs[i]);
    probs[i]->on_device = true;
  }
  // size groups
  std::vector<int> sizes;
  for (auto &p : probs) sizes.push_back((int)p->Mfft);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  group_of.assign(n, 0);
  slot_of.assign(n, 0);
  for (int s : sizes) {
    Group g;
    g.Mfft = s;
    g.N = s - 1;
    g.cs = (int64_t)g.N * s;
    for (int i = 0; i < n; ++i)
      if (probs[i]->Mfft == s) {
        group_of[i] = (int)groups.size();
        slot_of[i] = (int)g.members.size();
        g.members.push_back(i);
      }
    const size_t fs = (size_t)g.members.size() * g.cs;
    g.rhs64 = balloc<double>(fs);
    g.fpad64 = balloc<double>(fs);
    g.work64 = balloc<double>(fs);
    g.rhs32 = balloc<float>(fs);
    g.fpad32 = balloc<float>(fs);
    g.work32 = balloc<float>(fs);
    std::vector<ModeParams> ms;
    for (int i : g.members) {
      const DevProblem &p = *probs[i];
      ModeParams m{};
      m.lam = p.lam;
      for (int a = 0; a < 3; ++a) m.D0[a] = m.D1[a] = p.D[0][a];
      m.kappa = p.kappa;
      m.norm = p.lam_scale;
      ms.push_back(m);
    }
    g.msv = balloc<ModeParams>(ms.size());
    KFBI_HIP(hipMemcpy(g.msv, ms.data(), ms.size() * sizeof(ModeParams), hipMemcpyHostToDevice));
    groups.push_back(g);
  }
  // concatenated interface vectors and work lists
  off.assign(n + 1, 0);
  goff.assign(n + 1, 0);
  std::vector<int64_t> cnc(n + 1, 0), cirr(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const DevProblem &p = *probs[i];
    off[i + 1] = off[i] + p.M;
    goff[i + 1] = goff[i] + p.N * p.N;
    cnc[i + 1] = cnc[i] + p.nc;
    cirr[i + 1] = cirr[i] + p.nirr;
  }
  L = off[n];
  if (L == 0) throw std::invalid_argument("no interface nodes");
  std::vector<int16_t> pidh(L);
  for (int i = 0; i < n; ++i)
    for (int64_t e = off[i]; e < off[i + 1]; ++e) pidh[e] = (int16_t)i;
  pid = balloc<int16_t>(L);
  KFBI_HIP(hipMemcpy(pid, pidh.data(), L * sizeof(int16_t), hipMemcpyHostToDevice));
  off_dev = balloc<int64_t>(n + 1);
  KFBI_HIP(hipMemcpy(off_dev, off.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  goff_dev = balloc<int64_t>(n + 1);
  KFBI_HIP(hipMemcpy(goff_dev, goff.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  cum_nc = balloc<int64_t>(n + 1);
  cum_irr = balloc<int64_t>(n + 1);
  KFBI_HIP(hipMemcpy(cum_nc, cnc.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  KFBI_HIP(hipMemcpy(cum_irr, cirr.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  counts.cum_nc = cum_nc;
  counts.cum_M = off_dev;
  counts.cum_nirr = cum_irr;
  counts.n = n;
  counts.tot_nc = cnc[n];
  counts.tot_M = L;
  counts.tot_nirr = cirr[n];
  std::vector<BatchItem<double>> i64(n);
  std::vector<BatchItem<float>> i32(n);
  std::vector<PackItem> pk(n);
  // fits (transfer, jump and extrapolation weights, node jumps) from the FP64 tables in both precisions
  auto fill = [&](auto &it, auto &tb, auto *rhs, auto *fpad, auto *work, const DevProblem &p, int i) {
    const PrecTables<double> &t64 = p.f64;
    it.z_idx = p.z_idx;
    it.z_A = t64.z_A;
    it.z_B = t64.z_B;
    it.irr_pos = p.irr_pos;
    it.irr_ptr = p.irr_ptr;
    it.arm_cross = p.arm_cross;
    it.arm_d = tb.arm_d;
    it.arm_s = tb.arm_s;
    it.narm = p.narm;
    it.q_idx = p.q_idx;
    it.q_wg = t64.q_wg;
    it.q_c = t64.q_c;
    it.q_G = t64.q_G;
    it.st_pos = p.st_pos;
    it.st_nw = t64.st_nw;
    it.st_r = t64.st_r;
    it.jz = tb.jz;
    it.jq = t64.jq;
    it.rhs = rhs;
    it.fpad = fpad;
    it.work = work;
    it.M = p.M;
    it.nc = p.nc;
    it.nirr = p.nirr;
    it.ioff = off[i];
  };
  for (int i = 0; i < n; ++i) {
    const DevProblem &p = *probs[i];
    const Group &g = groups[group_of[i]];
    const int64_t o = (int64_t)slot_of[i] * g.cs;
    fill(i64[i], probs[i]->f64, g.rhs64 + o, g.fpad64 + o, g.work64 + o, p, i);
    fill(i32[i], probs[i]->f32, g.rhs32 + o, g.fpad32 + o, g.work32 + o, p, i);
    pk[i] = PackItem{g.fpad64 + o, g.work64 + o, p.N, (int64_t)g.Mfft};
  }
  items64 = balloc<BatchItem<double>>(n);
  items32 = balloc<BatchItem<float>>(n);
  packs = balloc<PackItem>(n);
  KFBI_HIP(hipMemcpy(items64, i64.data(), n * sizeof(BatchItem<double>), hipMemcpyHostToDevice));
  KFBI_HIP(hipMemcpy(items32, i32.data(), n * sizeof(BatchItem<float>), hipMemcpyHostToDevice));
  KFBI_HIP(hipMemcpy(packs, pk.data(), n * sizeof(PackItem), hipMemcpyHostToDevice));
  // Krylov workspace
  V = balloc<double>((size_t)(kMaxRestart + 1) * L);
  vin = balloc<double>(L);
  w = balloc<double>(L);
  r = balloc<double>(L);
  d = balloc<double>(L);
  t = balloc<double>(L);
  gp = balloc<double>(L);
  x = balloc<double>(L);
  dx = balloc<double>(L);
  hcols = balloc<double>((size_t)3 * (kMaxRestart + 1) * n);
  KFBI_HIP(hipHostMalloc(&hhost, (size_t)3 * (kMaxRestart + 1) * n * sizeof(double), hipHostMallocDefault));
  KFBI_HIP(hipHostMalloc(&jhost, sizeof(int), hipHostMallocDefault));
  KFBI_HIP(hipHostMalloc(&seqhost, sizeof(int), hipHostMallocDefault));
  *seqhost = 0;
  seq_next = 0;
  ydev = balloc<double>((size_t)kMaxRestart * n);
  sdev = balloc<double>(n);
  nrm = balloc<double>(n);
  jdev = balloc<int>(1);
  seqdev = balloc<int>(1);
  KFBI_HIP(hipMemset(seqdev, 0, sizeof(int)));
  KFBI_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  // tile widths of every size group, timed on the group's own buffers
  for (Group &g : groups) {
    const DevProblem &p0 = *probs[g.members[0]];
    const int G = (int)g.members.size();
    autotune_group<double>(g.Mfft, G, g.work64, g.cs, g.msv, p0.f64.tw, p0.f64.sp, g.tile_w[0], cap);
    autotune_group<float>(g.Mfft, G, g.work32, g.cs, g.msv, p0.f32.tw, p0.f32.sp, g.tile_w[1], cap);
  }
}

void Batch::release() {
  for (int k = 0; k < 2; ++k)
    if (graph[k]) {
      (void)hipGraphExecDestroy(graph[k]);
      graph[k] = nullptr;
    }
  for (Group &g : groups) {
    void *ps[] = {g.rhs64, g.fpad64, g.work64, g.rhs32, g.fpad32, g.work32, g.msv};
    for (void *q : ps)
      if (q) (void)hipFree(q);
  }
  groups.clear();
  void *ps[] = {pid, off_dev, goff_dev, cum_nc, cum_irr, items64, items32, packs, V, vin, w, r, d, t, gp, x, dx,
                hcols, ydev, sdev, nrm, jdev, seqdev};
  for (void *q : ps)
    if (q) (void)hipFree(q);
  if (cap) (void)hipStreamDestroy(cap);
  cap = nullptr;
  if (hhost) (void)hipHostFree(hhost);
  if (jhost) (void)hipHostFree(jhost);
  if (seqhost) (void)hipHostFree(seqhost);
  seqhost = nullptr;
  hhost = nullptr;
  jhost = nullptr;
  for (auto &p : probs)
    if (p && p->on_device) free_tables(*p);
  probs.clear();
}

bool Batch::mergeable() const {
  if (groups.empty() || (int)groups.size() > kMaxMultiGroups) return false;
  for (const Group &g : groups)
    if (g.Mfft < 64 || g.Mfft > 1024) return false;
  return true;
}

void Batch::drop_graphs() {
  for (int k = 0; k < 2; ++k)
    if (graph[k]) {
      (void)hipGraphExecDestroy(graph[k]);
      graph[k] = nullptr;
      graph_m[k] = 0;
    }
}

template <typename T>
void Batch::box_all(bool from_fpad, hipStream_t st) {
  auto src_of = [&](const Group &g) -> const T * {
    if constexpr (sizeof(T) == 8) return from_fpad ? g.fpad64 : g.rhs64;
    else return from_fpad ? g.fpad32 : g.rhs32;
  };
  if (merged && mergeable()) {
    MultiGroupDesc d[kMaxMultiGroups];
    int k = 0;
    for (const Group &g : groups) {
      const PrecTables<T> &tb = const_cast<DevProblem &>(*probs[g.members[0]]).tab<T>();
      d[k++] = MultiGroupDesc{g.Mfft, (int)g.members.size(), g.cs, src_of(g), g.work<T>(), g.msv, tb.tw, tb.sp};
    }
    box_solve_multi<T>(d, k, st);
    return;
  }
  for (const Group &g : groups) {
    const PrecTables<T> &tb = const_cast<DevProblem &>(*probs[g.members[0]]).tab<T>();
    box_solve_group<T>(g.Mfft, (int)g.members.size(), src_of(g), g.work<T>(), g.cs, g.msv, tb.tw, tb.sp,
                       g.tile_w[sizeof(T) == 8 ? 0 : 1], st);
  }
}

template <typename T>
void Batch::matvec(const double *in, double *out, hipStream_t st) {
  launch_batch_jumps<T>(items<T>(), counts, in, st);
  launch_batch_correct<T>(items<T>(), counts, 0, st);
  box_all<T>(false, st);
  launch_batch_gather<T>(items<T>(), counts, true, out, st);
}
template void Batch::matvec<double>(const double *, double *, hipStream_t);
template void Batch::matvec<float>(const double *, double *, hipStream_t);

void Batch::apply_vec(int prec, const double *in, double *out, hipStream_t st) {
  if (prec == 0) matvec<double>(in, out, st);
  else matvec<float>(in, out, st);
}

void Batch::apply_f32(const float *in, float *out, hipStream_t st) {
  k_cast<float, double><<<nb(L), kB, 0, st>>>(in, t, L);
  matvec<float>(t, w, st);
  k_cast<double, float><<<nb(L), kB, 0, st>>>(w, out, L);
  KFBI_HIP(hipGetLastError());
}

// per-problem squared norms of v into nrm (device) and hhost[0..np) (host)
void Batch::seg_norms(const double *v, std::vector<double> &out, hipStream_t st) {
  k_seg_dot<<<dim3(np, 1), kB, 0, st>>>(v, 0, nullptr, v, off_dev, np, nrm);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipMemcpyAsync(hhost, nrm, np * sizeof(double), hipMemcpyDeviceToHost, st));
  host_wait(st);
  out.resize(np);
  for (int p = 0; p < np; ++p) out[p] = std::sqrt(std::max(0.0, hhost[p]));
}

void Batch::arnoldi_step(int prec, int m, hipStream_t st) {
  const int ld = kMaxRestart + 1;
  k_take<<<nb(L), kB, 0, st>>>(V, L, jdev, vin);
  apply_vec(prec, vin, w, st);
  for (int pass = 0; pass < 2; ++pass) {
    double *h = hcols + (size_t)pass * ld * np;
    k_seg_dot<<<dim3(np, m), kB, 0, st>>>(V, L, jdev, w, off_dev, np, h);
    k_seg_combine<<<nb(L), kB, 0, st>>>(w, V, L, jdev, h, pid, np);
  }
  double *hn = hcols + (size_t)2 * ld * np;
  k_seg_dot<<<dim3(np, 1), kB, 0, st>>>(w, 0, nullptr, w, off_dev, np, hn);
  k_seg_next<<<nb(L), kB, 0, st>>>(w, hn, pid, V, L, jdev);
  KFBI_HIP(hipGetLastError());
  KFBI_HIP(hipMemcpyAsync(hhost, hcols, (size_t)3 * ld * np * sizeof(double), hipMemcpyDeviceToHost, st));
  k_inc<<<1, 1, 0, st>>>(jdev, seqdev, seqhost);
  KFBI_HIP(hipGetLastError());
}

void Batch::host_wait(hipStream_t st) {
  k_inc<<<1, 1, 0, st>>>(nullptr, seqdev, seqhost);
  KFBI_HIP(hipGetLastError());
  seq_next = poll_step_counter(seqhost, seq_next + 1, st);
}

void Batch::run_step(int prec, int m, hipStream_t st) {
  if (!use_graph) {
    arnoldi_step(prec, m, st);
    return;
  }
  if (!graph[prec] || graph_m[prec] != m) {
    if (graph[prec]) (void)hipGraphExecDestroy(graph[prec]);
    graph[prec] = nullptr;
    // captured on the batch's own stream, replayed on the caller's
    hipGraph_t g = nullptr;
    KFBI_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    try {
      arnoldi_step(prec, m, cap);
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

// GMRES(m) on A x = b for every problem at once; tol[p] absolute; x updated in place.
void Batch::gmres(int prec, const double *b, double *xv, bool x_zero, const std::vector<double> &tol, int restart,
                  int maxit, std::vector<int> &its, int &matvecs, std::vector<double> &res, hipStream_t st) {
  const int m = std::max(1, std::min(restart, kMaxRestart));
  const int ld = kMaxRestart + 1;
  its.assign(np, 0);
  if (x_zero) {
    KFBI_HIP(hipMemcpyAsync(r, b, L * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else {
    apply_vec(prec, xv, t, st);
    ++matvecs;
    k_axpby<<<nb(L), kB, 0, st>>>(r, 1.0, b, -1.0, t, L);
  }
  std::vector<double> beta;
  seg_norms(r, beta, st);
  std::vector<char> active(np);
  for (int p = 0; p < np; ++p) active[p] = beta[p] > tol[p];
  std::vector<double> H((size_t)np * (m + 1) * m), cs((size_t)np * m), sn((size_t)np * m), g((size_t)np * (m + 1));
  std::vector<int> jend(np);
  std::vector<char> done(np);
  std::vector<double> s(np), yh((size_t)m * np);
  int total = 0;
  while (total < maxit && std::any_of(active.begin(), active.end(), [](char a) { return a; })) {
    for (int p = 0; p < np; ++p) {
      s[p] = active[p] ? 1.0 / beta[p] : 0.0;
      done[p] = !active[p];
      jend[p] = 0;
      std::fill(&g[(size_t)p * (m + 1)], &g[(size_t)p * (m + 1)] + m + 1, 0.0);
      g[(size_t)p * (m + 1)] = active[p] ? beta[p] : 0.0;
    }
    KFBI_HIP(hipMemcpyAsync(sdev, s.data(), np * sizeof(double), hipMemcpyHostToDevice, st));
    k_seg_scale<<<nb(L), kB, 0, st>>>(r, sdev, pid, V, L);
    KFBI_HIP(hipGetLastError());
    *jhost = 0;
    KFBI_HIP(hipMemcpyAsync(jdev, jhost, sizeof(int), hipMemcpyHostToDevice, st));
    for (int j = 0; j < m && total < maxit; ++j) {
      run_step(prec, m, st);
      ++matvecs;
      ++total;
      seq_next = poll_step_counter(seqhost, seq_next + 1, st);   // the step ends with the counter
      bool all = true;
      for (int p = 0; p < np; ++p) {
        if (done[p]) continue;
        double *Hp = &H[(size_t)p * (m + 1) * m];
        double *gp_ = &g[(size_t)p * (m + 1)];
        double *c_ = &cs[(size_t)p * m], *s_ = &sn[(size_t)p * m];
        for (int i = 0; i <= j; ++i)
          Hp[(size_t)i * m + j] = hhost[(size_t)i * np + p] + hhost[(size_t)ld * np + (size_t)i * np + p];
        Hp[(size_t)(j + 1) * m + j] = std::sqrt(std::max(0.0, hhost[(size_t)2 * ld * np + p]));
        for (int i = 0; i < j; ++i) {
          const double a = Hp[(size_t)i * m + j], c = Hp[(size_t)(i + 1) * m + j];
          Hp[(size_t)i * m + j] = c_[i] * a + s_[i] * c;
          Hp[(size_t)(i + 1) * m + j] = -s_[i] * a + c_[i] * c;
        }
        const double a = Hp[(size_t)j * m + j], c = Hp[(size_t)(j + 1) * m + j];
        const double den = std::hypot(a, c);
        c_[j] = den > 0 ? a / den : 1.0;
        s_[j] = den > 0 ? c / den : 0.0;
        Hp[(size_t)j * m + j] = den;
        Hp[(size_t)(j + 1) * m + j] = 0.0;
        gp_[j + 1] = -s_[j] * gp_[j];
        gp_[j] = c_[j] * gp_[j];
        jend[p] = j + 1;
        its[p] += 1;
        if (std::fabs(gp_[j + 1]) <= tol[p] || den == 0.0) done[p] = 1;
        else all = false;
      }
      if (all) break;
    }
    // least-squares coefficients, x += V y
    int jmax = 0;
    std::fill(yh.begin(), yh.end(), 0.0);
    for (int p = 0; p < np; ++p) {
      if (!active[p]) continue;
      const double *Hp = &H[(size_t)p * (m + 1) * m];
      const double *gp_ = &g[(size_t)p * (m + 1)];
      const int je = jend[p];
      jmax = std::max(jmax, je);
      std::vector<double> y(je);
      for (int i = je - 1; i >= 0; --i) {
        double acc = gp_[i];
        for (int k = i + 1; k < je; ++k) acc -= Hp[(size_t)i * m + k] * y[k];
        y[i] = Hp[(size_t)i * m + i] != 0.0 ? acc / Hp[(size_t)i * m + i] : 0.0;
      }
      for (int i = 0; i < je; ++i) yh[(size_t)i * np + p] = y[i];
    }
    if (jmax > 0) {
      KFBI_HIP(hipMemcpyAsync(ydev, yh.data(), (size_t)jmax * np * sizeof(double), hipMemcpyHostToDevice, st));
      k_seg_update<<<nb(L), kB, 0, st>>>(xv, V, L, ydev, pid, np, jmax);
      KFBI_HIP(hipGetLastError());
    }
    // true residual
    apply_vec(prec, xv, t, st);
    ++matvecs;
    k_axpby<<<nb(L), kB, 0, st>>>(r, 1.0, b, -1.0, t, L);
    seg_norms(r, beta, st);
    for (int p = 0; p < np; ++p) active[p] = active[p] && beta[p] > tol[p];
  }
  res = beta;
}

void Batch::pack(const double *plain, int which, bool to_padded, hipStream_t st) {
  const int64_t tot = goff[np];
  // the caller's array is only read when packing into the padded buffers
  k_pack<<<nb(tot), kB, 0, st>>>(const_cast<double *>(plain), goff_dev, packs, np, tot, which, to_padded ? 1 : 0);
  KFBI_HIP(hipGetLastError());
}

int Batch::solve(const double *g, const double *f, double *u, double *psi, const kfbi_solve_opts &o,
                 kfbi_solve_info *info, hipStream_t st) {
  // volume part: u_V = S f, g' = g - n.D grad u_V+
  pack(f, 0, true, st);
  box_all<double>(true, st);
  launch_batch_gather<double>(items64, counts, false, t, st);
  if (g) k_axpby<<<nb(L), kB, 0, st>>>(gp, 1.0, g, -1.0, t, L);
  else k_axpby<<<nb(L), kB, 0, st>>>(gp, -1.0, t, 0.0, nullptr, L);
  KFBI_HIP(hipGetLastError());
  std::vector<double> gn;
  seg_norms(gp, gn, st);
  std::vector<double> tol_abs(np);
  for (int p = 0; p < np; ++p) tol_abs[p] = o.tol * gn[p];
  if (!o.x0) KFBI_HIP(hipMemsetAsync(psi, 0, L * sizeof(double), st));
  std::vector<int> its(np, 0), outer(np, 0), mv64(np, 0), mv32(np, 0);
  std::vector<double> res(np, 0), res0(np, 0);
  int mv = 0;
  if (o.precision == 0) {
    gmres(0, gp, psi, !o.x0, tol_abs, o.restart, o.max_iters, its, mv, res, st);
    for (int p = 0; p < np; ++p) mv64[p] = mv;
    res0 = gn;
  } else {
    bool have_x = o.x0 != 0;
    int total = 0;
    std::vector<int> inner;
    for (int k = 0;; ++k) {
      if (have_x) {
        apply_vec(0, psi, t, st);
        for (int p = 0; p < np; ++p) mv64[p] += 1;
        k_axpby<<<nb(L), kB, 0, st>>>(d, 1.0, gp, -1.0, t, L);
      } else {
        KFBI_HIP(hipMemcpyAsync(d, gp, L * sizeof(double), hipMemcpyDeviceToDevice, st));
      }
      seg_norms(d, res, st);
      if (k == 0) res0 = res;
      bool all = true;
      std::vector<double> keep(np), tin(np);
      for (int p = 0; p < np; ++p) {
        keep[p] = res[p] > tol_abs[p] ? 1.0 : 0.0;
        if (keep[p] != 0.0) all = false;
        tin[p] = std::max(o.inner_tol * res[p], 0.5 * tol_abs[p]);
      }
      if (all || k >= o.max_outer || total >= o.max_iters) break;
      // problems already converged take no part in this refinement step
      KFBI_HIP(hipMemcpyAsync(sdev, keep.data(), np * sizeof(double), hipMemcpyHostToDevice, st));
      k_seg_mask<<<nb(L), kB, 0, st>>>(d, pid, sdev, L);
      KFBI_HIP(hipMemsetAsync(dx, 0, L * sizeof(double), st));
      int mvi = 0;
      gmres(1, d, dx, true, tin, o.restart, o.max_iters - total, inner, mvi, res, st);
      int mx = 0;
      for (int p = 0; p < np; ++p) {
        its[p] += inner[p];
        mx = std::max(mx, inner[p]);
        if (keep[p] != 0.0) {
          mv32[p] += mvi;
          outer[p] += 1;
        }
      }
      total += mx;
      k_axpby<<<nb(L), kB, 0, st>>>(psi, 1.0, psi, 1.0, dx, L);
      have_x = true;
    }
  }
  // u = S(f + C psi)
  launch_batch_jumps<double>(items64, counts, psi, st);
  launch_batch_correct<double>(items64, counts, 1, st);
  box_all<double>(true, st);
  pack(u, 1, false, st);
  KFBI_HIP(hipStreamSynchronize(st));
  bool ok = true;
  for (int p = 0; p < np; ++p) {
    const bool conv = res[p] <= tol_abs[p];
    ok = ok && conv;
    if (info) {
      kfbi_solve_info &in = info[p];
      in = kfbi_solve_info{};
      in.iters = its[p];
      in.outer = outer[p];
      in.matvecs_fp64 = mv64[p];
      in.matvecs_fp32 = mv32[p];
      in.rel_resid = gn[p] > 0 ? res[p] / gn[p] : 0.0;
      in.gp_norm = gn[p];
      in.start_resid = gn[p] > 0 ? res0[p] / gn[p] : 0.0;
      in.true_resid = -1.0;
    }
  }
  return ok ? KFBI_OK : KFBI_ENOCONV;
}

}  // namespace kfbi
