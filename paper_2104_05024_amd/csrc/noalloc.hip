// A box solve that allocates nothing: kfbi_box_solve_noalloc.
//
// The same DST-I solve as kfbi_box_solve (Sec. 5.2 eq. FDE with u = 0 on the box boundary, end of
// Sec. 5.3) for callers that cannot allocate device memory (code under stream capture, serving
// loops): it needs no problem handle.  Its padded work field and its tables (twiddles, DST sines,
// mode eigenvalues) live in `scratch`, a file-scope device array of kScratchBytes that every GPU
// the library runs on holds until the process ends.  The tables are computed on the device by
// one kernel per call, so the call makes no host-to-device copy either, and the forward x pass
// writes every element of the padded field it later reads (pad columns included), so nothing
// needs clearing.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "device.h"
#include "kfbi.h"

namespace kfbi {
extern thread_local const char *g_last_static;
namespace {

constexpr size_t kScratchBytes = size_t(36) << 20;   // 36 MiB
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// device address of `scratch` per device (the host-side name is not a device address)
void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Looked up once per device, with that device current (each GPU holds its own copy of the
// array at its own address); null if the lookup fails.
void *scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

constexpr size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Tables of run_box for a grid of M cells per axis: tw[m] = exp(-2 pi i m / M) (complex),
// sp[n] = sin(pi n / M) (n = 0..M/2), lam[k-1] = (4/h^2) sin^2(k pi / (2M)) (k = 1..M-1).
template <typename T>
__global__ void k_noalloc_tables(T *__restrict__ tw, T *__restrict__ sp, double *__restrict__ lam, int M, double h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) {
    double s, c;
    sincospi(2.0 * (double)i / (double)M, &s, &c);
    tw[2 * i] = (T)c;
    tw[2 * i + 1] = (T)(-s);
  }
  if (i <= M / 2) sp[i] = (T)sinpi((double)i / (double)M);
  if (i >= 1 && i < M) {
    const double sn = sinpi((double)i / (2.0 * (double)M));
    lam[i - 1] = 4.0 / (h * h) * sn * sn;
  }
}

// Bytes of scratch the layout below needs: the padded field, then the tables, each 256-aligned.
size_t scratch_bytes(const kfbi_grid &g, int ncomp, size_t elem) {
  const size_t M = (size_t)g.cells, N = M - 1;
  const size_t field = align256((size_t)ncomp * M * (g.dim == 3 ? N * N : N) * elem);
  return field + align256(2 * M * elem) + align256((M / 2 + 1) * elem) + align256(N * sizeof(double));
}

template <typename T>
void solve(const kfbi_grid &g, const kfbi_coeffs &co, const T *f, T *u, unsigned char *base, hipStream_t st) {
  const int M = g.cells, d = g.dim;
  const int64_t N = M - 1;
  DevProblem p;
  p.dim = d;
  p.ncomp = co.ncomp;
  p.Mfft = M;
  p.N = N;
  p.P = M;
  p.comp_stride = p.P * (d == 3 ? N * N : N);
  p.h = (g.hi - g.lo) / (double)M;
  p.kappa = co.kappa;
  for (int c = 0; c < 2; ++c)
    for (int a = 0; a < 3; ++a) p.D[c][a] = co.D[c < co.ncomp ? c : 0][a < d ? a : 0];
  p.lam_scale = 1.0;
  for (int a = 0; a < d; ++a) p.lam_scale *= 2.0 / (double)M;
  const size_t field = align256((size_t)p.ncomp * p.comp_stride * sizeof(T));
  const size_t twb = align256((size_t)2 * M * sizeof(T)), spb = align256((size_t)(M / 2 + 1) * sizeof(T));
  PrecTables<T> &tb = p.tab<T>();
  tb.work = reinterpret_cast<T *>(base);
  tb.tw = reinterpret_cast<T *>(base + field);
  tb.sp = reinterpret_cast<T *>(base + field + twb);
  p.lam = reinterpret_cast<double *>(base + field + twb + spb);
  k_noalloc_tables<T><<<(M + 255) / 256, 256, 0, st>>>(tb.tw, tb.sp, p.lam, M, p.h);
  KFBI_HIP(hipGetLastError());
  box_solve<T>(p, f, true, u, true, st);
  // p's device pointers point into scratch: nothing to release
  tb.work = tb.tw = tb.sp = nullptr;
  p.lam = nullptr;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0; }

}  // namespace
}  // namespace kfbi

extern "C" int kfbi_box_solve_noalloc(const kfbi_grid *grid, const kfbi_coeffs *coeffs, const void *f, void *u,
                                      int32_t dtype, void *stream) {
  using namespace kfbi;
  auto bad = [](const char *msg) {
    g_last_static = msg;
    return KFBI_EINVAL;
  };
  try {
    if (!grid || !coeffs || !f || !u) return bad("kfbi_box_solve_noalloc: null argument");
    const kfbi_grid g = *grid;
    const kfbi_coeffs co = *coeffs;
    if (g.dim != 2 && g.dim != 3) return bad("kfbi_box_solve_noalloc: dim must be 2 or 3");
    if (g.cells < 16 || g.cells > 1024 || (g.cells & (g.cells - 1)) != 0)
      return bad("kfbi_box_solve_noalloc: cells must be a power of two in [16, 1024]");
    if (!(std::isfinite(g.lo) && std::isfinite(g.hi) && g.hi > g.lo))
      return bad("kfbi_box_solve_noalloc: the box needs finite lo < hi");
    if (co.ncomp != 1 && co.ncomp != 2) return bad("kfbi_box_solve_noalloc: ncomp must be 1 or 2");
    if (!(std::isfinite(co.kappa) && co.kappa >= 0)) return bad("kfbi_box_solve_noalloc: kappa must be finite and >= 0");
    for (int c = 0; c < co.ncomp; ++c)
      for (int a = 0; a < g.dim; ++a)
        if (!finite_pos(co.D[c][a])) return bad("kfbi_box_solve_noalloc: conductivities must be finite and > 0");
    if (dtype != KFBI_F64 && dtype != KFBI_F32) return bad("kfbi_box_solve_noalloc: dtype must be KFBI_F64 or KFBI_F32");
    if (scratch_bytes(g, co.ncomp, dtype == KFBI_F64 ? sizeof(double) : sizeof(float)) > kScratchBytes)
      return bad("kfbi_box_solve_noalloc: the padded field and tables exceed its 36 MiB scratch");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
      g_last_static = "kfbi_box_solve_noalloc: no usable current device";
      return KFBI_EHIP;
    }
    unsigned char *base = static_cast<unsigned char *>(scratch_on(dev));
    if (!base) {
      g_last_static = "kfbi_box_solve_noalloc: hipGetSymbolAddress of the scratch array failed";
      return KFBI_EHIP;
    }
    hipStream_t st = (hipStream_t)stream;
    if (dtype == KFBI_F64) solve<double>(g, co, (const double *)f, (double *)u, base, st);
    else solve<float>(g, co, (const float *)f, (float *)u, base, st);
    return KFBI_OK;
  } catch (const HipError &) {
    g_last_static = "kfbi_box_solve_noalloc: HIP runtime error";
    return KFBI_EHIP;
  } catch (...) {
    return bad("kfbi_box_solve_noalloc: unexpected error");
  }
}
