/*
 * kfbi.h -- C ABI of the MI355X kernel-free boundary integral (KFBI) library.
 *
 * Method: A Kernel-free Boundary Integral Method for the Bidomain Equations
 * (Gao, Cai, Henriquez, Ying).  The library solves the Neumann boundary value
 * problem of the bidomain diffusion step (Sec. 3, eqs. pde1, bvp, BC)
 *
 *     -div(D_c grad u_c) + (K u)_c = f_c   in Omega,    n . D_c grad u_c = g_c  on dOmega,
 *
 * K = kappa (one component) or kappa [[1,-1],[-1,1]] (intra/extracellular pair),
 * by the boundary integral equation A psi = g' of Sec. 4 (eq. bie) whose
 * operator A is applied without a Green's function (Sec. 5, Algorithm 1):
 * jump data from psi -> right-hand-side correction at irregular grid nodes ->
 * fast DST-I box solve -> quadratic extrapolation of n.D grad u+ at the
 * interface nodes.  Sign convention: the positive form above; the paper's
 * right-hand side is -f.
 *
 * Conventions for every call
 *  - Return value: KFBI_OK (0) or a negative KFBI_E* code; kfbi_strerror()
 *    gives text and kfbi_last_error() a message for the calling thread.
 *  - Grid arrays hold the (I-1)^d interior nodes of the box [lo,hi]^d with
 *    I = cells intervals per axis, C order [comp][z][y][x] (x fastest), no
 *    padding; u = 0 on the box boundary is implied.
 *  - Interface arrays are [comp][M], nodes in descriptor order (surface 0
 *    first).  Node j of a 2D curve sits at polar angle 2 pi j / M; 3D nodes
 *    follow the spherical Fibonacci lattice z_j = 1 - (2j+1)/M, azimuth
 *    j pi (3 - sqrt 5), mapped radially onto the surface.
 *  - "device" pointers are HIP device allocations owned by the caller; the
 *    library never frees them.  `stream` is a hipStream_t (NULL = default).
 *    Calls are stream-ordered; outputs are valid once the stream has drained.
 *  - A kfbi_problem / bidomain_ctx is not thread-safe; distinct handles are
 *    independent.  All library workspace is allocated in kfbi_setup /
 *    bidomain_create and released by the matching destroy call.
 */
#ifndef KFBI_H
#define KFBI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KFBI_OK = 0,
  KFBI_EINVAL = -1,   /* bad argument: null pointer, dtype, NaN, size out of range      */
  KFBI_EGEOM = -2,    /* geometry: interface within 3h of the box, an arm crossed twice, */
                      /* a rank-deficient extrapolation stencil                           */
  KFBI_ENOCONV = -3,  /* the iteration hit max_iters; outputs hold the last iterate       */
  KFBI_EHIP = -4,     /* HIP runtime error                                                 */
  KFBI_ENOMEM = -5,   /* host or device allocation failed                                  */
  KFBI_ENODEV = -6    /* the call needs a GPU but the problem was set up host-only         */
};

enum { KFBI_F64 = 0, KFBI_F32 = 1 };

#define KFBI_MAX_SURFACES 2
#define KFBI_MAX_TERMS 16

/* Kinds of surface descriptor. */
enum { KFBI_SURF_ANALYTIC = 0, KFBI_SURF_SPLINE = 1, KFBI_SURF_MESH = 2 };

/* One closed surface (curve in 2D).  orient = +1: the tissue Omega is inside it; -1: outside
 * (the inner wall of a shell).  n_nodes interface nodes lie on it (Sec. 6, quasi-uniform nodes).
 *
 * kind = KFBI_SURF_ANALYTIC: star-shaped in polar form r = R(u), u = x/|x|:
 *   R(u) = (sum_i u_i^2/axes_i^2)^(-1/2) * (1 + sum_t coef[t] prod_i u_i^exps[t][i]);
 *   the library places the nodes (2D: equal angles; 3D: spherical Fibonacci lattice).
 * kind = KFBI_SURF_SPLINE (2D only; Sec. 7, the 2D set-up): the boundary is given only by
 *   its nodes, points[2*j + a] (host memory, n_nodes >= 8 points in order along the curve,
 *   either direction); the library interpolates them with the periodic cubic spline in the
 *   node index (C2, closed) and reads normals, curvature and grid-line crossings off it.
 *   axes, coef and exps are ignored; the points are copied during kfbi_setup.
 * kind = KFBI_SURF_MESH (3D only; Sec. 6, local coordinate systems on the triangle grid): a
 *   closed, consistently oriented triangle mesh, vertices points[3*j + a] (the n_nodes nodes)
 *   and triangles tris[3*k + c] (n_tris >= 4, host memory, either orientation; every edge
 *   shared by exactly two triangles).  Normals and shape operators come from quadratic height
 *   functions fitted over each vertex's one-ring; grid-line crossings from the flat triangles,
 *   moved onto the quadratic through each triangle's six boundary points (its vertices and
 *   the three across its edges), which also carries psi and its surface gradient to the
 *   crossing (the one-ring fit does at the vertices).  An open or inconsistently oriented
 *   mesh gives KFBI_EGEOM. */
typedef struct {
  double axes[3];
  int32_t orient;
  int32_t n_terms;
  int64_t n_nodes;
  double coef[KFBI_MAX_TERMS];
  int32_t exps[KFBI_MAX_TERMS][3];
  int32_t kind;            /* KFBI_SURF_*; 0 (analytic) when the struct is zero-initialised */
  int32_t pad_;
  const double *points;    /* spline / mesh: node coordinates [n_nodes][dim], host memory */
  const int32_t *tris;     /* mesh: vertex indices [n_tris][3], host memory */
  int64_t n_tris;
} kfbi_surface;

/* Omega = intersection of the per-surface regions (Sec. 4: Omega inside the box B). */
typedef struct {
  int32_t dim;          /* 2 or 3 */
  int32_t n_surfaces;   /* 1 or 2 */
  kfbi_surface surf[KFBI_MAX_SURFACES];
} kfbi_interface;

/* The box B = [lo,hi]^dim with `cells` intervals per axis (Sec. 5.2); the GPU path
 * requires cells to be a power of two in [16, 1024]. */
typedef struct {
  int32_t dim;
  int32_t cells;
  double lo, hi;
} kfbi_grid;

/* ncomp = 1: -div(D[0] grad u) + kappa u;  ncomp = 2: the coupled pair of eq. bvp.
 * D[c][axis] is the diagonal conductivity of component c along each axis (anisotropic
 * allowed; every entry positive and finite, else KFBI_EINVAL). */
typedef struct {
  int32_t ncomp;
  int32_t pad_;
  double D[2][3];
  double kappa;
} kfbi_coeffs;

typedef struct kfbi_problem_s *kfbi_problem;

#define KFBI_SETUP_HOST_ONLY 1u   /* build the host tables only (no GPU calls) */
#define KFBI_SETUP_NO_AUTOTUNE 2u /* keep the default DST tile widths (no timed launches at setup) */

/* kfbi_setup: build every static table of the method for (interface, grid, coeffs)
 * -- interface nodes, normals, shape operators; grid-node sides; grid-line
 * intersections (Sec. 6 implementation paragraph); density-transfer weights;
 * correction records (Sec. 5.3); extrapolation stencils and weights (Sec. 5.4) --
 * in FP64 on the host, deterministically, then (unless KFBI_SETUP_HOST_ONLY)
 * upload them to the current HIP device and allocate all device workspace.
 * *out receives a handle owned by the library (kfbi_destroy). */
int kfbi_setup(const kfbi_interface *iface, const kfbi_grid *grid, const kfbi_coeffs *coeffs,
               uint32_t flags, kfbi_problem *out);
void kfbi_destroy(kfbi_problem p);

/* Sizes: M interface nodes, N = cells-1 interior nodes per axis, crossings,
 * irregular nodes.  Any pointer may be NULL. */
int kfbi_query(kfbi_problem p, int64_t *M, int64_t *N, int64_t *n_crossings, int64_t *n_irregular);

/* Host copy of a setup table, for inspection and parity tests.  Names:
 * "inside"(i8,N^d) "nodes_X" "nodes_n"(f64,M*d) "nodes_W"(f64,M*d*d)
 * "cross_axis" "cross_surf"(i64) "cross_pin" "cross_pout"(i64, linear interior index)
 * "cross_z" "cross_n"(f64,nc*d) "cross_W"(f64,nc*d*d) "cross_t"(f64,nc: spline parameter of
 * the crossing on a spline curve, index of its triangle on a mesh, NaN elsewhere) "z_idx"(i64,nc*K) "z_w0"(f64,nc*K) "z_wg"(f64,nc*K*d)
 * "q_idx"(i64,M*Kn) "q_wg"(f64,M*Kn*d) "st_lin"(i64,M*S) "st_r" "st_wgrad"(f64,M*S*d)
 * "irregular"(i64).  With dst == NULL only *count (elements) and *elem_bytes are set. */
int kfbi_table(kfbi_problem p, const char *name, void *dst, int64_t *count, int32_t *elem_bytes);

/* kfbi_apply: out = A psi, the KFBI matrix-vector product (Sec. 4 eq. bie left side;
 * Algorithm 1, "boundary integral" block): jumps of the single-layer interface
 * problem from psi (Sec. 5.1 eq. single), right-hand-side correction at irregular
 * nodes (Sec. 5.3 eq. correct), DST-I box solve, and n.D grad u+ at the nodes by
 * jump-corrected quadratic extrapolation (Sec. 5.4).  psi, out: device [ncomp][M]
 * in `dtype`.  KFBI_F64: the whole product in FP64.  KFBI_F32 (the reduced-precision product of
 * the mixed-precision solves): the correction and the box solve run in FP32, while the jumps and
 * the extrapolation fits keep FP64 weights and FP64 sums (psi is widened to FP64 on entry, the
 * result rounded to FP32 on exit). */
int kfbi_apply(kfbi_problem p, const void *psi, void *out, int32_t dtype, void *stream);

/* kfbi_box_solve: u = S f, the fast box solve alone (Sec. 5.2 eq. FDE with u = 0 on the box
 * boundary; end of Sec. 5.3): DST-I along every axis, division by the mode eigenvalues
 * (a closed-form 2x2 solve per mode for the coupled pair), inverse DST-I.  f, u: device
 * [ncomp][N^d] in `dtype`; f and u may alias. */
int kfbi_box_solve(kfbi_problem p, const void *f, void *u, int32_t dtype, void *stream);

typedef struct {
  double tol;           /* stop when ||g' - A psi||_2 <= tol ||g'||_2 (FP64 residual) */
  int32_t restart;      /* GMRES(m) restart length, 1..64 */
  int32_t max_iters;    /* total inner iterations */
  int32_t precision;    /* 0: FP64 throughout; 1: FP32 inner GMRES + FP64 refinement;
                           2: one FP64-Arnoldi GMRES whose products run in FP32 (as kfbi_apply's
                           KFBI_F32) once its residual is below inner_tol ||g'|| and in FP64 before,
                           then an FP64 product of the result checks the residual (the solve goes
                           on from that residual if it misses the tolerance) */
  int32_t x0;           /* 0: start from psi = 0 (Algorithm 1); 1: from psi_inout */
  double inner_tol;     /* precision = 1: relative tolerance of each FP32 inner solve;
                           precision = 2: relative residual below which the products are FP32 */
  int32_t max_outer;    /* precision = 1: maximum FP64 refinement steps */
  int32_t method;       /* 0: GMRES; 1: simple (Richardson) iteration (Sec. 4); for the coupled
                           pair its residual and ||g'|| are measured without their component
                           along the null density (the part of g' no density can match; the
                           iterates are the paper's) */
  double gamma;         /* Richardson parameter, gamma in (0,1) */
  int32_t true_resid;   /* 1: after the solve form g' - A64 psi with an explicit FP64 product and
                           report its relative norm in info.true_resid (a check: one product more) */
  int32_t pad_;
} kfbi_solve_opts;

typedef struct {
  int32_t iters;            /* inner iterations (FP64 or FP32) */
  int32_t outer;            /* FP64 refinement steps (precision = 1); FP64 residual checks (2) */
  int32_t matvecs_fp64;
  int32_t matvecs_fp32;
  double rel_resid;         /* final ||g' - A64 psi|| / ||g'|| */
  double gp_norm;           /* ||g'||_2 */
  int32_t warm_start_used;  /* bidomain_step: bit 0: the learned (1) or projection (3, 4) start was
                               taken; bit 1: the learned step (4) was taken; bit 2: it was tried
                               (its product spent, taken or not) */
  int32_t pad_;
  double start_resid;       /* ||g' - A64 psi0|| / ||g'|| of the start density (1 for a zero start) */
  double true_resid;        /* opts.true_resid = 1: ||g' - A64 psi|| / ||g'|| by an explicit product
                               (measured as the solve measures it), else -1 */
} kfbi_solve_info;

/* kfbi_solve_neumann: solve the Neumann problem above (Algorithm 1 with GMRES):
 *   u_V = box solve of f (f extended over the whole box; Sec. 5.1), g' = g - n.D grad u_V+,
 *   A psi = g' by GMRES (FP64, or FP32-inner with FP64 refinement), u = box solve of f + C psi.
 * For ncomp = 2 the pair is returned in the gauge mean_{Omega nodes}(u_2) = 0, reconstructed
 * from the density without its component along the null density: the insulated tissue fixes
 * both potentials only up to one common constant, so A is singular for the pair; its discrete
 * null vector (the eigenvector of smallest |eigenvalue|) is found once, by inverse iteration, at
 * the first coupled solve or bidomain step.  psi is returned as the solver found it.
 * g: device f64 [ncomp][M] (NULL = homogeneous); f, u: device f64 [ncomp][N^d];
 * psi_inout: device f64 [ncomp][M], initial guess if opts->x0 = 1, solution on return.
 * info may be NULL. Returns KFBI_ENOCONV (outputs filled) if max_iters is hit. */
int kfbi_solve_neumann(kfbi_problem p, const double *g, const double *f, double *u,
                       double *psi_inout, const kfbi_solve_opts *opts, kfbi_solve_info *info,
                       void *stream);

/* kfbi_box_solve_noalloc: the box solve of kfbi_box_solve without a problem handle and without
 * allocating, for callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid it).  grid and coeffs as for kfbi_setup (every D[c][a] of
 * the used components and axes finite and > 0, kappa finite and >= 0); f, u: device
 * [ncomp][N^d] in `dtype` (caller layout, may alias).  Its padded work field and its tables
 * (twiddles, DST sines, mode eigenvalues, computed on the device each call) live in a static
 * device array of 36 MiB per GPU, held until the process ends: grids whose padded field
 * ncomp (cells-1)^(d-1) cells entries plus tables exceed it give KFBI_EINVAL (FP64: a coupled
 * 128^3 or 1024^2 field fits, 256^3 does not).  No hipMalloc/hipFree, no host-to-device copy, no
 * memset; errors set a literal message for kfbi_last_error.  Every call on a GPU shares that
 * GPU's array and leaves its last contents there: calls that overlap on one GPU (two streams or
 * threads at once) race. */
int kfbi_box_solve_noalloc(const kfbi_grid *grid, const kfbi_coeffs *coeffs, const void *f, void *u,
                           int32_t dtype, void *stream);

/* ----------------------------------------------------------------- bidomain */

typedef struct {
  double Cm, beta;                  /* membrane capacitance, surface-to-volume ratio */
  double H, theta, alpha, zeta;     /* FitzHugh-Nagumo (Sec. 7): I_ion = H(q - V(V-theta)(1-V)),
                                       dq/dt = alpha V - zeta q */
  double newton_tol;                /* |F| tolerance of the backward-Euler Newton solve */
  int32_t newton_maxit;
  int32_t warm_start;               /* 0: psi^{n-1}; 1: learned (MLP) start with fallback; 2: zero;
                                       3: least-residual combination of the last 8 solutions
                                       (their images are known without a product);
                                       4: that combination, then one minimal-residual step along
                                       the learned prediction's difference from it (one FP64
                                       product; never increases the residual), with the cost
                                       check of the learned start switching it off */
  kfbi_solve_opts solve;            /* diffusion solve options (tol, precision, ...) */
} bidomain_params;

typedef struct bidomain_s *bidomain_ctx;

/* The coupled problem passed here must have ncomp = 2 (D[0] intracellular, D[1]
 * extracellular, diagonal) and kappa = 2 Cm beta / dt for the dt later given to
 * bidomain_step. */
int bidomain_create(kfbi_problem p, const bidomain_params *params, bidomain_ctx *out);
void bidomain_destroy(bidomain_ctx b);

/* State, all device f64, caller-owned: V, q: [N^d] (membrane potential and gate on every
 * box node); phi: [2][N^d] output potentials (Phi_i, Phi_e) of the diffusion solve, may be
 * NULL; psi_hist: [2][2][M] densities of the last two steps (slot 0 = newest), updated;
 * I_stim: [N^d] stimulus current, constant in time (Sec. 3: only space dependent), added to
 * the extracellular source as beta I_stim, or NULL.  A stimulus whose integral over the
 * tissue is not zero has no solution with zero Neumann data (the coupled problem determines
 * the potentials up to a common constant). */
typedef struct {
  double *V, *q, *phi, *psi_hist;
  const double *I_stim;
} bidomain_state;

/* bidomain_step: one Strang step (Sec. 3, eqs. ode1, diffusion, ode2): forward-Euler
 * reaction over dt/2, implicit-midpoint diffusion over dt (backward Euler over dt/2 for
 * w, then V <- 2 w_V - V), backward-Euler reaction over dt/2 solved by Newton.
 * Starting from psi^{n-1} = psi_hist slot 0, the solve takes that density's residual from the
 * previous step of this context without a product (g'^n - g'^{n-1} plus the previous final
 * residual) only while psi_hist is the same array as in that step and its slot 0 still holds,
 * at every node, the density that step returned; otherwise the residual is computed with an
 * FP64 product.  So a caller may reset or rewrite psi_hist, V and q between steps at any time. */
int bidomain_step(bidomain_ctx b, bidomain_state *state, double dt, kfbi_solve_info *info,
                  void *stream);
/* bidomain_reset: start a new simulation on the same context: forgets the recycled residual, the
 * solutions recorded for the projection start (warm_start = 3) and the step count that the
 * learned start waits on (its network is kept). */
int bidomain_reset(bidomain_ctx b);
/* bidomain_true_resid: from the next step on (enable != 0), every solve also forms g' - A64 psi
 * with an explicit FP64 product and reports its relative norm in info.true_resid (a check of the
 * residual the solve reports, at the cost of one product; the same as solve.true_resid = 1). */
int bidomain_true_resid(bidomain_ctx b, int32_t enable);

/* Learned warm start (not in the paper, which starts GMRES from zero).  The change of the
 * density between steps solves A (psi^n - psi^{n-1}) = g'^n - g'^{n-1}; the start is
 *   psi0 = psi^{n-1} + s_d sum_f K_{c,f}(x) F_f(x)
 * with change fields F = ((psi^{n-1} - psi^{n-2}) / s_d, (g'^n - g'^{n-1}) / s_g) per
 * component (s_d, s_g their max norms) and per-node coefficients K = net(n, h tr W) from
 * a small MLP of the static geometry only (3 tanh layers of 128, linear output of 16,
 * BF16 weights and activations on MFMA with FP32 accumulation, FP32 master weights).
 * bidomain_mlp_init allocates the network (output layer zero: the untrained start is
 * psi^{n-1}) and a device ring of `capacity` recorded steps; every bidomain_step from the
 * third on records (F, (psi^n - psi^{n-1}) / s_d).  bidomain_train runs `epochs` full-batch
 * Adam steps (lr, beta = 0.9 / 0.999) on the mean of (K F - target)^2 / 2 over nodes,
 * components and recorded steps, returns the last loss in loss_out and switches the
 * learned start on.  bidomain_step switches back to psi^{n-1} until the next training when
 * either check fails: every 8th use, the FP32 residual of the prediction must be below that of
 * psi^{n-1}; after every 8 uses, their mean solve cost (FP64 matvecs + FP32 matvecs / 2) must
 * be below the mean cost of the last 8 solves started from psi^{n-1}. */
int bidomain_mlp_init(bidomain_ctx b, int32_t capacity, uint64_t seed);
int bidomain_train(bidomain_ctx b, int32_t epochs, double lr, double *loss_out, void *stream);
/* FP32 master parameters: per layer W [out][in] row-major then b; layer shapes
 * [128][16], [128][128], [128][128], [16][128] (inputs beyond dim + 1 are zero padding).
 * host_dst NULL: only *count is set. */
int bidomain_mlp_params(bidomain_ctx b, float *host_dst, int64_t *count);
/* Test hook: run the network on R <= M host input rows X ([R][16] f32, rounded to BF16 on
 * upload) and return its outputs Y ([R][16] f32).  With dY ([R][16] f32) non-NULL also
 * back-propagate dY and return in grad the gradients of sum(dY * Y) with respect to the
 * parameters (order and count of bidomain_mlp_params).  The weights are left unchanged. */
int bidomain_mlp_eval(bidomain_ctx b, const float *X, int64_t R, float *Y, const float *dY, float *grad,
                      void *stream);

/* ----------------------------------------------------------------- batched 2D problems */

/* A batch of independent two-dimensional one-component Neumann problems (the scalar form
 * of the interface problem, Sec. 2 and 4) with uneven grid sizes (cells = 2^k in [16, 1024])
 * and shapes, solved together: the problems share each DST pass launch (kfbi_batch_merge); the
 * jump, correction and gather kernels of all problems run as one launch each over a work
 * list; GMRES runs in lockstep for all problems with one Arnoldi step captured once as a
 * hipGraph and replayed.  Concatenated layouts: interface arrays [problem][M_p] (offsets from
 * kfbi_batch_query), grid arrays [problem][N_p^2] in the caller layout (x fastest). */
typedef struct kfbi_batch_s *kfbi_batch;

int kfbi_batch_setup(int32_t n, const kfbi_interface *ifaces, const kfbi_grid *grids, const kfbi_coeffs *coeffs,
                     kfbi_batch *out);
void kfbi_batch_destroy(kfbi_batch b);
/* problem i: nodes M, grid unknowns per axis N, offsets into the concatenated interface and
 * grid arrays; i = -1 returns the totals in iface_offset / grid_offset. */
int kfbi_batch_query(kfbi_batch b, int32_t i, int64_t *M, int64_t *N, int64_t *iface_offset,
                     int64_t *grid_offset);
/* A psi for every problem (device, concatenated, KFBI_F64 or KFBI_F32 with the same split of
 * precisions as kfbi_apply). */
int kfbi_batch_apply(kfbi_batch b, const void *psi, void *out, int32_t dtype, void *stream);
/* Every problem's Neumann solve (FP64 device arrays, concatenated; g may be NULL for zero
 * Neumann data); opts as for kfbi_solve_neumann (method 0 only), the tolerance relative to
 * each problem's own ||g'||; info: one record per problem.  KFBI_ENOCONV if any problem did
 * not converge (all outputs are still written). */
int kfbi_batch_solve_neumann(kfbi_batch b, const double *g, const double *f, double *u, double *psi,
                             const kfbi_solve_opts *opts, kfbi_solve_info *info, void *stream);
/* enable != 0 (default): replay the captured Arnoldi step; 0: launch its kernels directly. */
int kfbi_batch_graph(kfbi_batch b, int32_t enable);
/* enable != 0 (default): when every grid size of the batch is 64..1024 cells, each DST pass of
 * the box solves is one launch over all size groups together (the tiles of small grids run
 * beside those of large ones); 0: one launch per size group and pass, at the tile widths timed
 * for that group.  Results are identical.  Waits for the batch's capture stream; the captured
 * Arnoldi steps are captured again at their next use. */
int kfbi_batch_merge(kfbi_batch b, int32_t enable);

/* ----------------------------------------------------------------- utilities */

const char *kfbi_strerror(int code);
const char *kfbi_last_error(void);

/* Timing of the kernel launches on the problem's stream since profiling was enabled, measured
 * with HIP events around each launch: average microseconds and launch count for the named
 * kernel class ("dst_x", "dst_y", "dst_last" (dense passes), "dst_x_rows", "dst_y_sparse",
 * "dst_last_sparse" (row- and plane-masked passes of the matrix-vector product), "dst_last_out"
 * (the z pass of the volume solve whose result is read only at the interface stencils: every
 * plane read, stencil planes written), "dst_x_fhn" (the x passes of a bidomain step's box solves
 * that also carry its reaction half steps), "dst_x_fe1", "dst_y1", "dst_last_anti" (the volume
 * solve of a step without stimulus current, whose source is antisymmetric: the forward x and y
 * passes over the one field kappa V1, and the z pass that reads it as the pair (g, -g)),
 * "dst_last_diff", "dst_x_be1" (the final solve of a step whose potentials are not returned:
 * the z pass that stores only Phi_i - Phi_e, and the inverse x pass with the backward Euler
 * update over that one field; its inverse y pass counts under "dst_y1"), "dst_last_comb" (that
 * z pass when the step also has no stimulus current: it adds the transform of C psi, taken
 * through the masked row and plane passes, to the volume solve's transform of kappa V1 as it
 * loads), "correct", "gather", "jumps").
 * Returns KFBI_EINVAL if the name is unknown. */
int kfbi_kernel_time(kfbi_problem p, const char *kernel, double *avg_us, int64_t *launches);
/* DST tile widths (1 or 2: multiples of the base pencil pairs per workgroup) of the x, y and
 * last-axis passes for dtype KFBI_F64 / KFBI_F32, as chosen by the autotuner at setup (each
 * dense pass timed at both widths on the problem's own buffers); kfbi_set_tiles overrides them.
 * Results do not depend on the widths (each pencil is transformed the same way). */
int kfbi_get_tiles(kfbi_problem p, int32_t dtype, int32_t widths[3]);
/* GMRES iterations of kfbi_solve_neumann / bidomain_step replay one captured Arnoldi step
 * (a hipGraph holding the product, both Gram-Schmidt passes, the norm and the next basis
 * vector) unless disabled here or while kfbi_profile is on; results are identical. */
int kfbi_use_graph(kfbi_problem p, int32_t enable);
int bidomain_use_graph(bidomain_ctx b, int32_t enable);
int kfbi_set_tiles(kfbi_problem p, int32_t dtype, const int32_t widths[3]);
int kfbi_profile(kfbi_problem p, int32_t enable);

#ifdef __cplusplus
}
#endif
#endif /* KFBI_H */
