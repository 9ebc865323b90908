// C ABI of the KFBI library: setup, the KFBI matrix-vector product, the Neumann solve
// (Algorithm 1 with GMRES, optionally FP32-inner / FP64-refinement), the bidomain step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "device.h"
#include "batch.h"
#include "solver.h"

namespace kfbi {
thread_local std::string g_last_error;
// message of the last error of kfbi_box_solve_noalloc: a string literal (that entry point never
// touches the host heap); null once any other call has failed
thread_local const char *g_last_static = nullptr;
}

using namespace kfbi;

int mlp_eval(bidomain_s *b, const float *X_host, int64_t R, float *Y_host, float *grad_host, const float *dY_host,
             hipStream_t st);

struct kfbi_problem_s {
  DevProblem p;
  Solver solver;
};

struct kfbi_batch_s {
  Batch b;
};

namespace {

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  g_last_static = nullptr;
  return code;
}

template <typename F>
int guard(F &&f) {
  try {
    return f();
  } catch (const GeometryError &e) {
    return fail(KFBI_EGEOM, e.what);
  } catch (const HipError &e) {
    return fail(KFBI_EHIP, std::string(hipGetErrorString(e.code)) + " in " + e.where);
  } catch (const std::bad_alloc &) {
    return fail(KFBI_ENOMEM, "host allocation failed");
  } catch (const std::invalid_argument &e) {
    return fail(KFBI_EINVAL, e.what());
  } catch (const std::exception &e) {
    return fail(KFBI_EINVAL, e.what());
  }
}

}  // namespace

extern "C" {

const char *kfbi_strerror(int code) {
  switch (code) {
    case KFBI_OK: return "ok";
    case KFBI_EINVAL: return "invalid argument";
    case KFBI_EGEOM: return "geometry outside the method's assumptions";
    case KFBI_ENOCONV: return "iteration did not converge";
    case KFBI_EHIP: return "HIP runtime error";
    case KFBI_ENOMEM: return "out of memory";
    case KFBI_ENODEV: return "problem was set up host-only";
    default: return "unknown error";
  }
}

const char *kfbi_last_error(void) { return g_last_static ? g_last_static : g_last_error.c_str(); }

int kfbi_setup(const kfbi_interface *iface, const kfbi_grid *grid, const kfbi_coeffs *coeffs, uint32_t flags,
               kfbi_problem *out) {
  return guard([&]() -> int {
    if (!iface || !grid || !coeffs || !out) return fail(KFBI_EINVAL, "null argument");
    *out = nullptr;
    std::unique_ptr<kfbi_problem_s> h(new kfbi_problem_s());
    build_host_tables(*iface, *grid, *coeffs, h->p.ht);
    if (!(flags & KFBI_SETUP_HOST_ONLY)) {
      const int c = grid->cells;
      if (c < 16 || c > 1024 || (c & (c - 1)) != 0)
        return fail(KFBI_EINVAL, "GPU path needs cells = 2^k in [16, 1024]");
      KFBI_HIP(hipGetDevice(&h->p.dev));
      try {
        upload_tables(h->p);
        h->solver.init(h->p);
        if (!(flags & KFBI_SETUP_NO_AUTOTUNE)) autotune_tiles(h->p, nullptr);
      } catch (...) {
        h->solver.release();
        free_tables(h->p);
        throw;
      }
      h->p.on_device = true;
    }
    *out = h.release();
    return KFBI_OK;
  });
}

void kfbi_destroy(kfbi_problem p) {
  if (!p) return;
  if (p->p.on_device) {
    (void)hipDeviceSynchronize();
    p->solver.release();
    free_tables(p->p);
  }
  delete p;
}

int kfbi_query(kfbi_problem p, int64_t *M, int64_t *N, int64_t *n_crossings, int64_t *n_irregular) {
  if (!p) return fail(KFBI_EINVAL, "null problem");
  if (M) *M = p->p.ht.M;
  if (N) *N = p->p.ht.N;
  if (n_crossings) *n_crossings = p->p.ht.nc;
  if (n_irregular) *n_irregular = (int64_t)p->p.ht.irregular.size();
  return KFBI_OK;
}

int kfbi_table(kfbi_problem p, const char *name, void *dst, int64_t *count, int32_t *elem_bytes) {
  if (!p || !name) return fail(KFBI_EINVAL, "null argument");
  const HostTables &t = p->p.ht;
  const void *src = nullptr;
  int64_t n = 0;
  int32_t eb = 0;
  auto pick_d = [&](const std::vector<double> &v) { src = v.data(); n = (int64_t)v.size(); eb = 8; };
  auto pick_i = [&](const std::vector<int64_t> &v) { src = v.data(); n = (int64_t)v.size(); eb = 8; };
  const std::string s(name);
  if (s == "inside") { src = t.inside.data(); n = (int64_t)t.inside.size(); eb = 1; }
  else if (s == "nodes_X") pick_d(t.X);
  else if (s == "nodes_n") pick_d(t.nrm);
  else if (s == "nodes_W") pick_d(t.W);
  else if (s == "cross_axis") pick_i(t.c_axis);
  else if (s == "cross_surf") pick_i(t.c_surf);
  else if (s == "cross_pin") pick_i(t.c_pin);
  else if (s == "cross_pout") pick_i(t.c_pout);
  else if (s == "cross_z") pick_d(t.c_z);
  else if (s == "cross_n") pick_d(t.c_n);
  else if (s == "cross_W") pick_d(t.c_W);
  else if (s == "cross_t") pick_d(t.c_t);
  else if (s == "z_idx") pick_i(t.z_idx);
  else if (s == "z_w0") pick_d(t.z_w0);
  else if (s == "z_wg") pick_d(t.z_wg);
  else if (s == "q_idx") pick_i(t.q_idx);
  else if (s == "q_wg") pick_d(t.q_wg);
  else if (s == "st_lin") pick_i(t.st_lin);
  else if (s == "st_r") pick_d(t.st_r);
  else if (s == "st_wgrad") pick_d(t.st_wgrad);
  else if (s == "irregular") pick_i(t.irregular);
  else return fail(KFBI_EINVAL, "unknown table " + s);
  if (count) *count = n;
  if (elem_bytes) *elem_bytes = eb;
  if (dst && n) std::memcpy(dst, src, (size_t)n * eb);
  return KFBI_OK;
}

int kfbi_apply(kfbi_problem p, const void *psi, void *out, int32_t dtype, void *stream) {
  return guard([&]() -> int {
    if (!p || !psi || !out) return fail(KFBI_EINVAL, "null argument");
    if (!p->p.on_device) return fail(KFBI_ENODEV, "problem set up host-only");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == KFBI_F64)
      p->solver.apply<double>(p->p, (const double *)psi, (double *)out, st);
    else if (dtype == KFBI_F32)
      p->solver.apply_f32(p->p, (const float *)psi, (float *)out, st);
    else
      return fail(KFBI_EINVAL, "dtype");
    return KFBI_OK;
  });
}

int kfbi_box_solve(kfbi_problem p, const void *f, void *u, int32_t dtype, void *stream) {
  return guard([&]() -> int {
    if (!p || !f || !u) return fail(KFBI_EINVAL, "null argument");
    if (!p->p.on_device) return fail(KFBI_ENODEV, "problem set up host-only");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == KFBI_F64)
      box_solve<double>(p->p, (const double *)f, true, (double *)u, true, st);
    else if (dtype == KFBI_F32)
      box_solve<float>(p->p, (const float *)f, true, (float *)u, true, st);
    else
      return fail(KFBI_EINVAL, "dtype");
    return KFBI_OK;
  });
}

int kfbi_solve_neumann(kfbi_problem p, const double *g, const double *f, double *u, double *psi_inout,
                       const kfbi_solve_opts *opts, kfbi_solve_info *info, void *stream) {
  return guard([&]() -> int {
    if (!p || !f || !u || !psi_inout || !opts) return fail(KFBI_EINVAL, "null argument");
    if (!p->p.on_device) return fail(KFBI_ENODEV, "problem set up host-only");
    kfbi_solve_info inf{};
    const int rc = p->solver.solve_neumann(p->p, g, f, u, psi_inout, *opts, inf, (hipStream_t)stream);
    if (info) *info = inf;
    return rc;
  });
}

int kfbi_get_tiles(kfbi_problem p, int32_t dtype, int32_t widths[3]) {
  if (!p || !widths || (dtype != KFBI_F64 && dtype != KFBI_F32)) return fail(KFBI_EINVAL, "argument");
  for (int k = 0; k < 3; ++k) widths[k] = p->p.tile_w[dtype == KFBI_F64 ? 0 : 1][k];
  return KFBI_OK;
}

int kfbi_use_graph(kfbi_problem p, int32_t enable) {
  if (!p) return fail(KFBI_EINVAL, "argument");
  p->solver.use_graph = enable != 0;
  return KFBI_OK;
}

int bidomain_use_graph(bidomain_ctx b, int32_t enable) {
  if (!b || !b->solver) return fail(KFBI_EINVAL, "argument");
  b->solver->use_graph = enable != 0;
  return KFBI_OK;
}

int bidomain_true_resid(bidomain_ctx b, int32_t enable) {
  if (!b || !b->solver) return fail(KFBI_EINVAL, "argument");
  b->params.solve.true_resid = enable != 0;
  return KFBI_OK;
}

int bidomain_reset(bidomain_ctx b) {
  if (!b || !b->solver) return fail(KFBI_EINVAL, "argument");
  b->reset();
  return KFBI_OK;
}

int kfbi_set_tiles(kfbi_problem p, int32_t dtype, const int32_t widths[3]) {
  if (!p || !widths || (dtype != KFBI_F64 && dtype != KFBI_F32)) return fail(KFBI_EINVAL, "argument");
  for (int k = 0; k < 3; ++k)
    if (widths[k] != 1 && widths[k] != 2) return fail(KFBI_EINVAL, "tile widths are 1 or 2");
  for (int k = 0; k < 3; ++k) p->p.tile_w[dtype == KFBI_F64 ? 0 : 1][k] = widths[k];
  return KFBI_OK;
}

int kfbi_batch_setup(int32_t n, const kfbi_interface *ifaces, const kfbi_grid *grids, const kfbi_coeffs *coeffs,
                     kfbi_batch *out) {
  return guard([&]() -> int {
    if (!ifaces || !grids || !coeffs || !out || n < 1) return fail(KFBI_EINVAL, "argument");
    *out = nullptr;
    std::unique_ptr<kfbi_batch_s> h(new kfbi_batch_s());
    try {
      h->b.init(n, ifaces, grids, coeffs);
    } catch (...) {
      h->b.release();
      throw;
    }
    *out = h.release();
    return KFBI_OK;
  });
}

void kfbi_batch_destroy(kfbi_batch b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  b->b.release();
  delete b;
}

int kfbi_batch_query(kfbi_batch b, int32_t i, int64_t *M, int64_t *N, int64_t *iface_offset, int64_t *grid_offset) {
  if (!b || i < -1 || i >= b->b.np) return fail(KFBI_EINVAL, "argument");
  if (i == -1) {
    if (M) *M = b->b.L;
    if (N) *N = 0;
    if (iface_offset) *iface_offset = b->b.L;
    if (grid_offset) *grid_offset = b->b.goff[b->b.np];
    return KFBI_OK;
  }
  if (M) *M = b->b.probs[i]->M;
  if (N) *N = b->b.probs[i]->N;
  if (iface_offset) *iface_offset = b->b.off[i];
  if (grid_offset) *grid_offset = b->b.goff[i];
  return KFBI_OK;
}

int kfbi_batch_apply(kfbi_batch b, const void *psi, void *out, int32_t dtype, void *stream) {
  return guard([&]() -> int {
    if (!b || !psi || !out) return fail(KFBI_EINVAL, "argument");
    const hipStream_t st = (hipStream_t)stream;
    if (dtype == KFBI_F64) b->b.matvec<double>((const double *)psi, (double *)out, st);
    else if (dtype == KFBI_F32) b->b.apply_f32((const float *)psi, (float *)out, st);
    else return fail(KFBI_EINVAL, "dtype");
    KFBI_HIP(hipStreamSynchronize(st));
    return KFBI_OK;
  });
}

int kfbi_batch_solve_neumann(kfbi_batch b, const double *g, const double *f, double *u, double *psi,
                             const kfbi_solve_opts *opts, kfbi_solve_info *info, void *stream) {
  return guard([&]() -> int {
    if (!b || !f || !u || !psi || !opts) return fail(KFBI_EINVAL, "argument");
    if (opts->method != 0) return fail(KFBI_EINVAL, "batched solves use GMRES");
    if (opts->precision != 0 && opts->precision != 1) return fail(KFBI_EINVAL, "batched solves use precision 0 or 1");
    if (opts->restart < 1 || opts->restart > Batch::kMaxRestart || opts->max_iters < 1 || !(opts->tol > 0))
      return fail(KFBI_EINVAL, "solve options");
    const int rc = b->b.solve(g, f, u, psi, *opts, info, (hipStream_t)stream);
    if (rc == KFBI_ENOCONV) g_last_error = "some problems of the batch did not converge";
    return rc;
  });
}

int kfbi_batch_graph(kfbi_batch b, int32_t enable) {
  if (!b) return fail(KFBI_EINVAL, "argument");
  b->b.use_graph = enable != 0;
  return KFBI_OK;
}

int kfbi_batch_merge(kfbi_batch b, int32_t enable) {
  if (!b) return fail(KFBI_EINVAL, "argument");
  return guard([&]() -> int {
    KFBI_HIP(hipStreamSynchronize(b->b.cap));
    b->b.merged = enable != 0;
    b->b.drop_graphs();
    return KFBI_OK;
  });
}

int kfbi_profile(kfbi_problem p, int32_t enable) {
  if (!p) return fail(KFBI_EINVAL, "null problem");
  return guard([&]() -> int {
    if (!p->p.on_device) return fail(KFBI_ENODEV, "problem set up host-only");
    p->p.profile = enable != 0;
    Timer *ts[] = {&p->p.t_dst_x, &p->p.t_dst_y, &p->p.t_dst_last, &p->p.t_correct, &p->p.t_gather,
                   &p->p.t_jumps, &p->p.t_dst_x_rows, &p->p.t_dst_y_sparse, &p->p.t_dst_last_sparse,
                   &p->p.t_dst_last_out, &p->p.t_dst_x_fhn, &p->p.t_dst_x_fe1, &p->p.t_dst_y1,
                   &p->p.t_dst_last_anti, &p->p.t_dst_last_diff, &p->p.t_dst_x_be1, &p->p.t_dst_last_comb};
    for (Timer *t : ts) t->reset();
    return KFBI_OK;
  });
}

int kfbi_kernel_time(kfbi_problem p, const char *kernel, double *avg_us, int64_t *launches) {
  if (!p || !kernel) return fail(KFBI_EINVAL, "null argument");
  const std::string s(kernel);
  Timer *t = nullptr;
  if (s == "dst_x") t = &p->p.t_dst_x;
  else if (s == "dst_y") t = &p->p.t_dst_y;
  else if (s == "dst_last") t = &p->p.t_dst_last;
  else if (s == "correct") t = &p->p.t_correct;
  else if (s == "gather") t = &p->p.t_gather;
  else if (s == "jumps") t = &p->p.t_jumps;
  else if (s == "dst_x_rows") t = &p->p.t_dst_x_rows;
  else if (s == "dst_y_sparse") t = &p->p.t_dst_y_sparse;
  else if (s == "dst_last_sparse") t = &p->p.t_dst_last_sparse;
  else if (s == "dst_last_out") t = &p->p.t_dst_last_out;
  else if (s == "dst_x_fhn") t = &p->p.t_dst_x_fhn;
  else if (s == "dst_x_fe1") t = &p->p.t_dst_x_fe1;
  else if (s == "dst_y1") t = &p->p.t_dst_y1;
  else if (s == "dst_last_anti") t = &p->p.t_dst_last_anti;
  else if (s == "dst_last_diff") t = &p->p.t_dst_last_diff;
  else if (s == "dst_x_be1") t = &p->p.t_dst_x_be1;
  else if (s == "dst_last_comb") t = &p->p.t_dst_last_comb;
  else return fail(KFBI_EINVAL, "unknown kernel class");
  return guard([&]() -> int {
    if (p->p.on_device) t->harvest();
    if (avg_us) *avg_us = t->n ? 1000.0 * t->total_ms / (double)t->n : 0.0;
    if (launches) *launches = t->n;
    return KFBI_OK;
  });
}

// ------------------------------------------------------------------ bidomain

int bidomain_create(kfbi_problem p, const bidomain_params *params, bidomain_ctx *out) {
  return guard([&]() -> int {
    if (!p || !params || !out) return fail(KFBI_EINVAL, "null argument");
    if (!p->p.on_device) return fail(KFBI_ENODEV, "problem set up host-only");
    if (p->p.ncomp != 2) return fail(KFBI_EINVAL, "bidomain needs the coupled two-component problem");
    if (params->warm_start < 0 || params->warm_start > 4) return fail(KFBI_EINVAL, "warm_start is 0..4");
    if (params->solve.precision < 0 || params->solve.precision > 2) return fail(KFBI_EINVAL, "precision is 0, 1 or 2");
    *out = nullptr;
    std::unique_ptr<bidomain_s> b(new bidomain_s());
    b->prob = &p->p;
    b->solver = &p->solver;
    b->params = *params;
    b->init();
    *out = b.release();
    return KFBI_OK;
  });
}

void bidomain_destroy(bidomain_ctx b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  b->release();
  delete b;
}

int bidomain_step(bidomain_ctx b, bidomain_state *state, double dt, kfbi_solve_info *info, void *stream) {
  return guard([&]() -> int {
    if (!b || !state || !state->V || !state->q || !state->psi_hist) return fail(KFBI_EINVAL, "null argument");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(KFBI_EINVAL, "dt");
    const double kap = 2.0 * b->params.Cm * b->params.beta / dt;
    if (std::fabs(kap - b->prob->kappa) > 1e-12 * kap) return fail(KFBI_EINVAL, "kappa != 2 Cm beta / dt");
    kfbi_solve_info inf{};
    const int rc = b->step(*state, dt, inf, (hipStream_t)stream);
    if (info) *info = inf;
    return rc;
  });
}

int bidomain_mlp_init(bidomain_ctx b, int32_t capacity, uint64_t seed) {
  return guard([&]() -> int {
    if (!b || capacity < 1) return fail(KFBI_EINVAL, "argument");
    b->mlp_init(capacity, seed);
    return KFBI_OK;
  });
}

int bidomain_train(bidomain_ctx b, int32_t epochs, double lr, double *loss_out, void *stream) {
  return guard([&]() -> int {
    if (!b || epochs < 0) return fail(KFBI_EINVAL, "argument");
    if (!b->mlp) return fail(KFBI_EINVAL, "call bidomain_mlp_init first");
    const double l = b->mlp_train(epochs, lr, (hipStream_t)stream);
    if (loss_out) *loss_out = l;
    return KFBI_OK;
  });
}

int bidomain_mlp_eval(bidomain_ctx b, const float *X, int64_t R, float *Y, const float *dY, float *grad,
                      void *stream) {
  return guard([&]() -> int {
    if (!b || !b->mlp || !X || R < 1) return fail(KFBI_EINVAL, "argument");
    return mlp_eval(b, X, R, Y, grad, dY, (hipStream_t)stream);
  });
}

int bidomain_mlp_params(bidomain_ctx b, float *host_dst, int64_t *count) {
  return guard([&]() -> int {
    if (!b || !b->mlp) return fail(KFBI_EINVAL, "no network");
    return b->mlp_params(host_dst, count);
  });
}

}  // extern "C"
