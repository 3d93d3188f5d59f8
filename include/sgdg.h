/*
 * sgdg.h -- C ABI of libsgdg: the sparse-grid time-discontinuous Galerkin
 * streamline-diffusion method for phase-space transport, on AMD MI355X (gfx950).
 *
 * Problem (Sect. 1, (eq:transport)/(eq:inflow)):
 *     d_t u + beta(x,v) . grad_(x,v) u + sigma(x,v) u = f   in (0,T) x Omega_x x Omega_v,
 *     u(0) = u0,   u = g on the inflow boundary {beta . n < 0}.
 * Discretisation (Sect. 2): nested P1 spaces V_l on each box (2^l cells per
 * axis, Kuhn simplices), the sparse space V_L = sum over |l|_1 = L + lmin of
 * V^x_{lx} (x) V^v_{lv}, discontinuous polynomials of degree r in time, and the
 * streamline-diffusion weak form (eq:weak_form_j) on each time strip.
 *
 * Data layout (every vector argument, host or device):
 *   a sparse-grid function of one strip is stored by its spanning-set
 *   coefficients (eq:spanningset): one block per upper-diagonal component
 *   grid (lx, lv), lx + lv = level_max + level_min, blocks in increasing lx;
 *   each block is a row-major [R][n_x][n_v] array, R = r + 1 time slices
 *   (Legendre basis on the strip), v index fastest.  Inside a domain, nodes
 *   are numbered in C order over the axis indices (last axis fastest).
 *   A batch of B vectors is [B][n_dof], contiguous.
 *   "Nodal" arrays (data sampled at grid nodes) use the same per-grid
 *   [n_x][n_v] blocks, upper-diagonal grids first, then the lower-diagonal
 *   grids (lx + lv = level_max + level_min - 1, increasing lx).
 *
 * Ownership: sgdg_grid and sgdg_ops are created by the library and released
 * with the matching *_destroy.  Host arrays passed in are copied during the
 * call.  Device buffers (suffix _dev) are owned by the caller, must hold the
 * stated number of elements of the stated type and stay valid until the
 * stream has executed the call; the library never frees them.  Internal
 * workspace (Krylov bases, scan arrays) belongs to the sgdg_ops handle.
 *
 * Errors: every entry point returns an sgdg_status; no exception crosses the
 * ABI.  Arguments are validated before any device work is queued
 * (SGDG_E_ARG).  sgdg_last_error() returns a thread-local message for the last
 * failing call on the calling thread.
 *
 * Streams: apply / combine / precondition / rhs are queued on the given
 * stream and return without synchronising.  solve_strip synchronises the
 * stream before it returns its statistics.  An sgdg_ops handle must not be
 * used from two threads at once, nor on two streams concurrently.
 */
#ifndef SGDG_H
#define SGDG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SGDG_OK = 0,
  SGDG_E_ARG = -1,        /* invalid argument or shape */
  SGDG_E_ALLOC = -2,      /* device or host allocation failed */
  SGDG_E_HIP = -3,        /* a HIP runtime call failed */
  SGDG_E_NOCONV = -4,     /* iteration limit reached before the tolerance */
  SGDG_E_BREAKDOWN = -5,  /* Krylov breakdown before the tolerance */
  SGDG_E_NAN = -6,        /* NaN/Inf in a residual norm */
  SGDG_E_STATE = -7       /* handle not in a usable state */
} sgdg_status;

typedef enum { SGDG_F64 = 0, SGDG_F32 = 1 } sgdg_dtype;

/* Message of the last failing call on this thread (never NULL). */
const char* sgdg_last_error(void);

/* ---------------------------------------------------------------- layout -- */

/* One box domain, Omega^(1) (x) or Omega^(2) (v), Sect. 2.  dim in 1..3;
 * all axes share the periodic flag. */
typedef struct {
  int dim;
  double lo[3], hi[3];
  int periodic;
} sgdg_domain;

typedef struct sgdg_grid_s* sgdg_grid;

/* Builds the component-grid layout of V_L, (eq:sg_space) with level numbering
 * level_min..level_max on both domains (paper level 1 <-> level_min).
 * time_degree r in 0..2.  Fails with SGDG_E_ARG on dims that differ, dim
 * outside 1..3, level_min > level_max, level_max > 12, lo >= hi. */
sgdg_status sgdg_build_sparse_grid(const sgdg_domain* x, const sgdg_domain* v, int level_min,
                                   int level_max, int time_degree, sgdg_grid* out);

/* Component grids of one diagonal: which = 0 upper (the spanning set), 1 lower
 * (combination technique).  Every output pointer may be NULL; arrays must hold
 * n_comp entries (query n_comp first with the others NULL).  offset[i] is the
 * start of grid i in a one-slice nodal array of that diagonal; n_dof is
 * R * sum(nx*nv) for the upper diagonal and sum(nx*nv) for the lower one. */
sgdg_status sgdg_grid_info(sgdg_grid g, int which, int* n_comp, int64_t* n_dof, int* lx, int* lv,
                           int64_t* nx, int64_t* nv, int64_t* offset);
void sgdg_grid_destroy(sgdg_grid g);

/* ----------------------------------------------------------- coefficients -- */

/* scale * prod_i xf[i](x) * prod_j vf[j](v), each factor a P1 field given by
 * its values at the nodes of the finest level of its domain (host arrays,
 * copied).  This is the separable form of Sect. 4.2. */
typedef struct {
  double scale;
  int n_xf;
  const double* const* xf;
  int n_vf;
  const double* const* vf;
} sgdg_separable;

/* beta[c], c = 0..2*dim-1 (x components, then v components), NULL for a zero
 * component; sigma = sum of n_sigma separable terms.  dt is the strip length,
 * delta the streamline-diffusion parameter (delta > 0, delta < 1/sigma). */
typedef struct {
  const sgdg_separable* beta[6];
  int n_sigma;
  const sgdg_separable* sigma;
  double dt;
  double delta;
} sgdg_problem;

typedef struct sgdg_ops_s* sgdg_ops;

/* Assembles every factor matrix of the strip operator (eq:matrices) on the
 * finest level of each domain by exact integration, restricts it to all
 * coarser levels with the embedding matrices (Sect. 4.2,
 * X_{l,l'} = E_{L,l}^T X_{L,L} E_{L,l'}), builds the Kronecker term lists and
 * uploads everything to the current HIP device.  The inflow weight on a face
 * with normal velocity s*a(x)*b(v) is split exactly into (s a)^+ b^- + (s a)^- b^+
 * (each factor the P1 interpolant of the kinked nodal values); such a face
 * needs beta's component to be one separable term (it is by construction).
 * The grid must outlive the ops handle. */
sgdg_status sgdg_assemble_1d_factors(sgdg_grid g, const sgdg_problem* p, sgdg_ops* out);
/* Coefficients that depend on time (Sect. 4.2, the block formula with an
 * m-point time quadrature): beta and sigma given at the points tau[mu] of the
 * strip's reference interval [-1, 1] (t = t_{j-1} + dt (tau + 1) / 2), as
 * at[mu] (same structure at every point), with weights weight[mu] summing to
 * 2.  Each point contributes the spatial factors of its coefficients times the
 * time matrices w_mu eta_s'(tau_mu) eta_s(tau_mu) and their derivative forms;
 * the operator is the strip's (build one per strip).  dt and delta are taken
 * from at[0] and must agree at every point. */
typedef struct {
  int m;                    /* quadrature points, 1..8 */
  const double* tau;        /* [m] points in [-1, 1] */
  const double* weight;     /* [m] weights on [-1, 1] */
  const sgdg_problem* at;   /* [m] coefficients at each point */
} sgdg_problem_t;

/* As sgdg_assemble_1d_factors for time-dependent coefficients.  SGDG_E_ARG on
 * m outside 1..8, points outside [-1, 1], weights not summing to 2, or
 * dt / delta differing between points. */
sgdg_status sgdg_assemble_factors_t(sgdg_grid g, const sgdg_problem_t* p, sgdg_ops* out);
void sgdg_ops_destroy(sgdg_ops o);

/* -------------------------------------------------------------- operators -- */

typedef enum {
  SGDG_OP_FULL = 0,      /* A^(delta) of (eq:Adelta), all blocks A_{l,l'}; R -> R slices */
  SGDG_OP_BLOCKDIAG = 1, /* only the diagonal blocks A_{l,l} (the grid problems (eq:Adeltall)) */
  SGDG_OP_MASS = 2,      /* (phi', phi) over the spanning set, one slice -> one slice */
  SGDG_OP_DATA_F = 3,    /* f |-> int (f, w + delta(d_t w + d_beta w)), R -> R */
  SGDG_OP_DATA_G = 4     /* g |-> int over the inflow boundary of |beta.n| g w, R -> R */
} sgdg_opkind;

/* y_dev = Op u_dev for a batch of vectors (Sect. 4.2, blockwise application
 * [A u]_l = sum_l' A_{l,l'} u_l').  u_dev, y_dev: device arrays of batch *
 * n_in / batch * n_out elements of type t (n_in = n_out = n_dof, or n_dof/R for
 * SGDG_OP_MASS).  u_dev and y_dev must not overlap.  batch >= 1. */
sgdg_status sgdg_apply_operator(sgdg_ops o, int kind, const void* u_dev, void* y_dev, sgdg_dtype t,
                                int batch, hipStream_t s);

/* Combination formula: spanning coefficients of sum_upper f_l - sum_lower f_l
 * from nodal values on both diagonals (Algorithm 1's combination step; exact
 * for interpolation, Sect. 4.3).  nodal_dev: device FP64 [nslices][all upper
 * nodes + all lower nodes]; coef_dev: device FP64 [grid][nslices][n_x][n_v]. */
sgdg_status sgdg_combine(sgdg_ops o, const double* nodal_dev, double* coef_dev, int nslices,
                         hipStream_t s);

/* ------------------------------------------------------- preconditioners -- */

/* A trained per-grid correction network standing in for the combination
 * technique (see "learned preconditioner" below). */
typedef struct sgdg_net_s* sgdg_net;

typedef struct {
  int kind;             /* 0 = combination technique (Algorithm 1's body); 1 = learned network,
                           falling back to the combination technique */
  double inner_rtol;    /* relative residual of each grid problem (eq:Adeltall) */
  int inner_maxit;      /* iteration cap per grid problem */
  int inner_restart;    /* GMRES restart length of the grid problems */
  int mass_sweeps;      /* mass inverses of the grid-problem preconditioner (Sect. 4.3): 0 = diagonals of
                           M^x and M^v; k = 1..64: k Chebyshev-Jacobi steps per mass factor (a fixed
                           polynomial in D^-1 M, eigenvalues in [1/2, 1 + d/2]); -1 (d = 1 only): exact
                           tridiagonal solves per grid line.  -2 (periodic x only, at most 1024 nodes per
                           x-axis): instead the x-transport preconditioner, an extension beyond Sect. 4.3:
                           the terms of A_{l,l} with translation-invariant x-factors (mass, derivatives,
                           stiffness without x-field weights) and mass v-factors, the v-factors lumped to
                           their row sums, inverted exactly mode by mode after a discrete Fourier
                           transform over x (for every v-node an R x R system per mode) */
  sgdg_net net;         /* kind 1: the trained network of this problem */
  int fallback_iters;   /* kind 1: if over any fallback_iters consecutive FGMRES iterations (default 10) ... */
  double fallback_drop; /* ... the residual estimate drops by less than this factor (default 10), the
                           remaining iterations use kind 0 */
} sgdg_precond_opts;

/* z_dev = P_CT r_dev for `batch` independent vectors ([batch][n_dof], 1..4096).
 * Restricts the residual to the lower diagonal, solves every grid problem
 * A_{l,l} dU_l = r_l by GMRES right-preconditioned with the inverse of
 * (Tt + delta Ct + Gt) (x) M^x (x) M^v (Sect. 4.3; see mass_sweeps), and
 * combines.  The grid problems of all vectors iterate in the same launches.
 * r_dev and z_dev hold batch * n_dof elements of the dtype t: F64 runs
 * everything in FP64, F32 runs the grid problems in FP32.  Grid problems
 * that reach inner_maxit are left at their best iterate (not an error);
 * SGDG_E_NAN if a grid problem's residual is not finite. */
sgdg_status sgdg_precondition(sgdg_ops o, const void* r_dev, void* z_dev, sgdg_dtype t, int batch,
                              const sgdg_precond_opts* po, hipStream_t s);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.
 * y_dev = Op u_dev exactly as sgdg_apply_operator (same arguments, same
 * kernels and launch configuration, same results), but every work array of
 * the call (the cross-grid scan arrays and the staged v-stage values) is
 * carved from one fixed library-owned device array of
 * SGDG_NOALLOC_SCRATCH_BYTES per device, taken at the first call on a device
 * and held until the process ends.  The call allocates nothing and times
 * nothing.
 * Requirements and errors: the current device must be the handle's device
 * (SGDG_E_ARG otherwise); the handle's launch tables for this kind and dtype
 * must exist -- the first sgdg_apply_operator call with that kind and dtype
 * builds them, and tuning or sgdg_set_launch rebuilds them -- else
 * SGDG_E_STATE; a call needing more scratch than the array holds (about
 * (n_xgroups + 4 n_groups 2^-d) n_dof elements per vector, e.g. 0.13 GB for
 * one FP64 vector of the 4D problem at level 7) fails with SGDG_E_ARG and a
 * message giving the bytes it needs.
 * Sharing: every call on one device uses the same array, and it keeps the
 * last call's contents (nothing in it needs to start at zero).  Calls that
 * overlap on one device -- two streams, two threads, two handles -- race on
 * it and give wrong results: order them on one stream. */
#define SGDG_NOALLOC_SCRATCH_BYTES (256u << 20)
sgdg_status sgdg_apply_operator_noalloc(sgdg_ops o, int kind, const void* u_dev, void* y_dev, sgdg_dtype t,
                                        int batch, hipStream_t s);

/* --------------------------------------------------------- strip solves -- */

/* Right-hand side b_j of (eq:weak_form_j) into b_dev (FP64, n_dof):
 *   jump term (U_{j-1}^-, w_{j-1}^+) from u_prev_dev (FP64, prev_slices slices
 *   per grid, the previous strip's solution, or prev_slices = 1 for U_0^-),
 *   plus the data functionals of f and g given as nodal values at the r+2
 *   Gauss-Legendre points of the strip: f_nodal_dev / g_nodal_dev are device
 *   FP64 [r+2][all upper nodes + all lower nodes] or NULL (zero data).  The data
 *   are projected onto P^r in time and interpolated on the sparse grid before
 *   the functionals are applied, so b lies in the range of A^(delta). */
sgdg_status sgdg_rhs(sgdg_ops o, const double* u_prev_dev, int prev_slices, const double* f_nodal_dev,
                     const double* g_nodal_dev, double* b_dev, hipStream_t s);

typedef struct {
  double rtol;          /* stop when ||b - A u||_2 <= rtol ||b||_2 (FP64) */
  int restart;          /* FGMRES restart length (<= 64) */
  int maxit;            /* total FGMRES iterations */
  int mixed_precision;  /* 1: FP64 refinement around an FP32 inner FGMRES (FP32 applies + FP32 CT) */
  double inner_outer_rtol; /* mixed precision: tolerance of each FP32 correction solve */
  sgdg_precond_opts pc;
  int use_graph;          /* 1: replay each grid-problem GMRES cycle from a captured hipGraph */
} sgdg_solve_opts;

typedef struct {
  int outer_iters;        /* FGMRES iterations (summed over refinement steps) */
  int refinement_steps;   /* mixed precision only */
  int inner_iters_total;  /* grid-problem GMRES iterations summed over all calls */
  double rel_residual;    /* final ||b - A u|| / ||b|| in FP64 */
  double seconds;         /* wall time of the call */
  int fallback_used;      /* learned preconditioner: 1 if the solve switched to the combination technique */
  int pc_applications;    /* preconditioner applications (learned + combination technique) */
} sgdg_solve_stats;

/* Solves A^(delta) u = b for one strip by flexible GMRES right-preconditioned
 * with the combination technique (FP64 Arnoldi; in mixed precision FP64
 * iterative refinement around FP32 corrections).  b_dev: FP64 n_dof; u_dev:
 * FP64 n_dof, used as the initial guess and overwritten.  Returns SGDG_E_NOCONV
 * (with u_dev holding the last iterate and st filled) if maxit is reached,
 * SGDG_E_NAN if a residual norm is not finite.  Synchronises s. */
sgdg_status sgdg_solve_strip(sgdg_ops o, const double* b_dev, double* u_dev, const sgdg_solve_opts* so,
                             sgdg_solve_stats* st, hipStream_t s);

/* ------------------------------------------------------ batched problems -- */

/* A batch of independent strip problems (same dimension and time degree,
 * any levels and coefficients), solved in lockstep: every device launch
 * covers all problems (work tables map blocks to problem, grid and tile), so
 * uneven component grids and uneven problems share launches.  Batch vectors
 * are the concatenation of the problems' vectors in the order given. */
typedef struct sgdg_batch_s* sgdg_batch;

/* ops: n handles (n >= 1) that must outlive the batch.  SGDG_E_ARG if they
 * differ in dimension or time degree or live on different devices. */
sgdg_status sgdg_batch_create(const sgdg_ops* ops, int n, sgdg_batch* out);
/* offsets[i] = start of problem i in a batch vector, offsets[n] = total (n+1 entries). */
sgdg_status sgdg_batch_layout(sgdg_batch b, int64_t* offsets);
/* y = A^(delta) u for every problem (FP64 or FP32), one scan sequence and one
 * tiled launch for the whole batch. */
sgdg_status sgdg_batch_apply(sgdg_batch b, const void* u_dev, void* y_dev, sgdg_dtype t, hipStream_t s);
/* Solves every problem's strip system in lockstep (FGMRES with the batched
 * combination-technique preconditioner, or the problems' networks for
 * pc.kind = 1, see sgdg_batch_set_networks; mixed precision as in
 * sgdg_solve_strip).  st receives the totals and the largest relative
 * residual.  SGDG_E_NOCONV if any problem misses the tolerance. */
sgdg_status sgdg_batch_solve(sgdg_batch b, const double* b_dev, double* u_dev, const sgdg_solve_opts* so,
                             sgdg_solve_stats* st, hipStream_t s);
/* Learned preconditioner for a batch: nets[i] (created with sgdg_net_create
 * on problem i's handle, see below) stands in for the combination technique
 * on problem i's slice of every batch vector.  A batch solve with pc.kind = 1
 * then applies every problem's network (pc.net is not used), with the
 * combination technique of the whole batch as the fallback, switched when the
 * largest residual estimate over the problems fails the fallback rule.
 * n = 0 removes them.  The networks must outlive their use by the batch.
 * SGDG_E_ARG unless n is 0 or the batch size and every network belongs to the
 * problem at its position. */
sgdg_status sgdg_batch_set_networks(sgdg_batch b, const sgdg_net* nets, int n);
void sgdg_batch_destroy(sgdg_batch b);

/* ------------------------------------------------ learned preconditioner -- */

/* The combination technique maps the residual of every upper grid l to a
 * correction on the same grid (the lower partner (lx-1, lv) solves for the
 * x-restriction of r_l; Algorithm 1's body).  The learned form replaces this
 * per-grid map by a network N_l of its own per upper grid:
 *     z_l = s_l * rms(r_l) * N_l(r_l / rms(r_l)),  rms(r) = ||r||_2 / sqrt(#entries),
 * where N_l has 4 layers, each a 3x3 convolution over the x-plane followed by
 * a 3x3 convolution over the v-plane (32 channels, biases, ReLU after layers
 * 1-3; periodic padding along periodic domains, zeros otherwise), acting on
 * the grid's coefficients with the time slices as channels.  Weights and
 * activations are bfloat16 with FP32 accumulation (matrix cores); master
 * weights and the Adam state are FP32.  The network is trained on pairs
 * (r, P_CT r) that the solver records.  Only for d = 2 (4D phase space).
 *
 * Parameters: for each upper grid (in order), for each of the 8 convolutions
 * (layer-major, x-plane then v-plane): W[9][32][32] (tap (a,b) -> 3(a+1)+(b+1),
 * output channel, input channel) then the bias[32]; FP32. */
typedef struct {
  int steps;            /* Adam steps */
  int batch;            /* samples per step */
  double lr;            /* Adam learning rate (beta1 0.9, beta2 0.999, eps 1e-8) */
  uint64_t seed;        /* seed of the combination coefficients */
  int mix;              /* 1: each sample is a random N(0,1/K) combination of the K stored pairs
                           (valid because P_CT is linear); 0: the stored pairs in turn */
} sgdg_train_opts;

typedef struct {
  double loss_first;    /* mean of the first min(10, steps) step losses */
  double loss_last;     /* mean of the last min(10, steps) step losses */
  double seconds;
  int steps;
} sgdg_train_stats;

/* Creates the networks of o's upper grids, weights drawn from seed (scaled
 * normal, zero biases, padding channels zero), output scales 1.  Device memory
 * is owned by the handle.  SGDG_E_ARG unless d = 2. */
sgdg_status sgdg_net_create(sgdg_ops o, uint64_t seed, sgdg_net* out);
/* Number of FP32 parameters (grids x 8 x 9248) and of grids. */
sgdg_status sgdg_net_shape(sgdg_net n, int64_t* n_params, int* n_grids);
/* Host copies of the parameters (layout above) and the per-grid output scales. */
sgdg_status sgdg_net_get_params(sgdg_net n, float* params, double* scales);
sgdg_status sgdg_net_set_params(sgdg_net n, const float* params, const double* scales);
/* Appends count pairs (r_i, z_i = P r_i), FP64 device vectors of n_dof each,
 * contiguous, to the training store (converted to FP32).  SGDG_E_ARG beyond capacity. */
sgdg_status sgdg_net_add_pairs(sgdg_net n, const double* r_dev, const double* z_dev, int count, hipStream_t s);
/* capacity > 0: every combination-technique application inside solves of the
 * network's problem appends its (r, z) pair until the store holds capacity
 * pairs; 0 stops recording.  Resets nothing already stored. */
sgdg_status sgdg_net_record(sgdg_net n, int capacity);
sgdg_status sgdg_net_pair_count(sgdg_net n, int* count);
/* Sets the output scales s_l from the stored pairs (mean of rms(z_l)/rms(r_l))
 * and runs Adam on the mean squared error of the normalised outputs. */
sgdg_status sgdg_net_train(sgdg_net n, const sgdg_train_opts* to, sgdg_train_stats* st, hipStream_t s);
/* z_dev = P_learned r_dev (FP64 n_dof vectors). */
sgdg_status sgdg_net_apply(sgdg_net n, const double* r_dev, double* z_dev, hipStream_t s);
/* Raw network on the concatenated grid tensors: x_dev, y_dev FP32 [points][R]
 * channels-last (points of grid l in the order x * n_v + v, grids in order;
 * points = n_dof / R).  No normalisation, no scale. */
sgdg_status sgdg_net_forward(sgdg_net n, const float* x_dev, float* y_dev, hipStream_t s);
/* Gradient of sum(y * dy) for y = forward(x): grad_dev FP32 [n_params] (layout above). */
sgdg_status sgdg_net_backward(sgdg_net n, const float* x_dev, const float* dy_dev, float* grad_dev, hipStream_t s);
void sgdg_net_destroy(sgdg_net n);

/* ------------------------------------------------ Vlasov-Poisson coupling -- */

/* The nonlinear Vlasov-Poisson system of Sect. 5.3 for electrons in a
 * neutralising background:
 *     d_t f + v . grad_x f - E . grad_v f = 0,
 *     -Laplace_x phi = 1 - rho,  rho(x) = int f(x, v) dv,  E = -grad_x phi,
 * solved strip by strip with the fixed point of Sect. 5.3 (eq:E_f, eq:poisson):
 * the transport with the field of the previous iterate, then the density of
 * the new iterate at the strip's midpoint (the midpoint rule: the field is
 * constant over the strip), then the field.  Discretisation of the field: P1
 * elements on the finest x-lattice, K phi = M (1 - rho) with phi of mean zero,
 * and E_i the L2 projection of -d_i phi (M E_i = -D_i phi).  The x-domain must
 * be periodic, d = 1 or 2.  Fields are FP64 device arrays [d][n_fine], n_fine
 * the nodes of the finest x-lattice (C order). */
typedef struct sgdg_vp_s* sgdg_vp;

typedef struct {
  double fp_tol;          /* stop when max|E^(k+1) - E^(k)| + ||f^(k+1) - f^(k)||_L2 (midpoint) < fp_tol */
  int max_fp;             /* fixed-point iterations per strip */
  sgdg_solve_opts solve;  /* the transport solve of each iteration (pc.kind must be 0) */
} sgdg_vp_opts;

typedef struct {
  int fp_iters;           /* fixed-point iterations taken */
  int outer_iters;        /* FGMRES iterations over all transport solves */
  int inner_iters;        /* grid-problem GMRES iterations over all transport solves */
  double dE, df;          /* the last iteration's field and density changes */
  double energy;          /* electric energy 1/2 int |E|^2 of the returned field */
  double rel_residual;    /* relative residual of the last transport solve */
  double seconds;         /* wall time of the call */
  double assemble_seconds; /* host assembly of the transport operators (one per iteration) */
} sgdg_vp_stats;

/* Creates the coupling on the layout g (which must outlive it): dt is the
 * strip length, delta the streamline-diffusion parameter of the transport.
 * Host assembly of the finest-level field matrices and upload; SGDG_E_ARG
 * unless x is periodic and d <= 2. */
sgdg_status sgdg_vp_create(sgdg_grid g, double dt, double delta, sgdg_vp* out);
/* n_fine (nodes of the finest x-lattice) and d; either may be NULL. */
sgdg_status sgdg_vp_info(sgdg_vp p, int64_t* n_fine, int* d);
/* rho_dev (FP64 n_fine) = int f dv on the finest x-lattice, f_dev a sparse-grid
 * function (spanning coefficients) with nslices slices: the number of time
 * slices, evaluated at reference time tau in [-1, 1] of the strip (1 = the
 * strip's end), or 1 (a one-slice function such as U_0).  Queued on s. */
sgdg_status sgdg_vp_density(sgdg_vp p, const double* f_dev, int nslices, double tau, double* rho_dev,
                            hipStream_t s);
/* E_dev (FP64 [d][n_fine]) = the field of the density rho_dev (conjugate
 * gradients in one workgroup, relative tolerance 1e-14); *energy (if not NULL,
 * which synchronises s) = 1/2 int |E|^2. */
sgdg_status sgdg_vp_field(sgdg_vp p, const double* rho_dev, double* E_dev, double* energy, hipStream_t s);
/* One strip of the fixed point: f_prev_dev the previous strip's solution
 * (prev_slices slices) or U_0 (1 slice), E0_dev the field to start from (that
 * of f_prev's end); returns the strip solution in f_dev (FP64 n_dof) and the
 * last field in E_dev.  Each iteration assembles the transport operator of
 * its field on the host.  SGDG_E_NOCONV (results and stats filled) if max_fp
 * iterations do not reach fp_tol.  Synchronises s. */
sgdg_status sgdg_vp_strip(sgdg_vp p, const double* f_prev_dev, int prev_slices, const double* E0_dev, double* f_dev,
                          double* E_dev, const sgdg_vp_opts* o, sgdg_vp_stats* st, hipStream_t s);
void sgdg_vp_destroy(sgdg_vp p);

/* ------------------------------------------------------------- autotuner -- */

/* Launch configuration of the operator application.  variant 0: split
 * application (v-stage, upper-partner and x-stage passes) with
 * vectors_per_thread vectors per thread, and block_map 1 to give each of the
 * chip's 8 XCDs one contiguous range of blocks (0: the hardware's round-robin
 * order); variant 2: the same with the x-stage on LDS tiles (tiles for 1 or 2
 * vectors per thread; with 4 the x-stage runs per point); variant 1: fused
 * box tiles with x-boxes of xbox nodes per axis. */
typedef struct {
  int variant;
  int vectors_per_thread;
  int xbox;
  int block_map;
  double ms;        /* measured time of one full application with this configuration */
  int from_cache;   /* 1 if taken from the tuning cache without measuring */
  int scan_chunks;  /* blocks sharing the factor groups of a level-scan item (tuned for batches of
                       at most 4 vectors, else 1); in sgdg_set_launch 0 keeps the current value */
} sgdg_tune_result;

/* Environment, read when a handle's (or batch's) application state is first
 * created; the tuner and sgdg_set_launch override the launch settings:
 *   SGDG_APPLY_VARIANT  split | fused | split_tiled: initial variant (split)
 *   SGDG_SPLIT_BC       1, 2 or 4: initial vectors per thread (2; 1 for d = 3)
 *   SGDG_SPLIT_XCD      1: initial block map XCD-contiguous (0)
 *   SGDG_SPLIT_ORDER    1: split items ordered v-block first (0: x-node first)
 *   SGDG_SCAN_CHUNKS    n >= 1: blocks sharing the factor groups of a scan item (1);
 *                       0: chosen per launch from the launch's item count
 *   SGDG_TUNE_CACHE     path of the tuning cache (see sgdg_tune) */

/* Times every candidate configuration of the full operator application for
 * `batch` vectors of dtype t on stream s (reps timed applications each, after
 * one warm-up), keeps the fastest for this handle, and records it in the
 * tuning cache, a text file keyed by dimension, slices, dtype, batch and the
 * levels of every grid: $SGDG_TUNE_CACHE, else $HOME/.cache/sgdg_tune.txt.
 * A cached entry is used without measuring unless force is 1.  Allocates and
 * frees two work vectors; synchronises s. */
sgdg_status sgdg_tune(sgdg_ops o, sgdg_dtype t, int batch, int reps, int force, sgdg_tune_result* out,
                      hipStream_t s);
/* The same for a multi-problem batch (one vector per problem). */
sgdg_status sgdg_batch_tune(sgdg_batch b, sgdg_dtype t, int reps, int force, sgdg_tune_result* out, hipStream_t s);
/* Sets the launch configuration directly (variants 0 and 2:
 * vectors_per_thread in {1, 2, 4}, 1 for d = 3, block_map 0 or 1; variant 1:
 * xbox >= 1, shrunk to the LDS budget).  SGDG_E_ARG on other values.  ms and from_cache are
 * ignored. */
sgdg_status sgdg_set_launch(sgdg_ops o, const sgdg_tune_result* cfg);

/* ------------------------------------------------------------ diagnostics -- */

/* Event timing of the operator kernels (for roofline reports).  mode 1 resets
 * the counters and records a HIP event pair on the call's stream around every
 * subsequent launch group of the operator kernels; mode 0 stops recording. */
sgdg_status sgdg_profile(sgdg_ops o, int mode);
/* Accumulated time (ms) and launch-group count of one kernel class since the
 * last reset: slot 0 = level scans of the partner sums (all steps of one
 * application, k_scan2), 1 = box-tiled accumulation (k_fused), 2 = grid-problem
 * GMRES cycles of the preconditioner, 3 = v-stage (k_vstage), 4 =
 * upper-partner pass (k_ustage), 5 = x-stage (k_xstage).  Waits for the
 * recorded events. */
sgdg_status sgdg_profile_read(sgdg_ops o, int slot, double* ms, int64_t* launches);
/* Shape of one operator: Kronecker terms, distinct v- and x-factors, stencil
 * sizes of the two domains and the time slices in/out. */
sgdg_status sgdg_op_info(sgdg_ops o, int kind, int* nterms, int* nvg, int* nxg, int* Sx, int* Sv, int* Rin,
                         int* Rout);
/* Host-only: where the X-factors of operator `kind` can contribute on x-level
 * lx (Sect. 4.2's factors are sparse; face masses live on their face alone).
 * counts (6 entries, caller-owned) = { x-nodes of the level;
 * (node, X-group) pairs whose staged W^m is read by the x-stencil of a row
 * where the group's factor has a nonzero (the v-stage computes exactly
 * these); the Kronecker terms of those pairs; (node, X-group) pairs whose
 * factor row has a nonzero (the x-stage applies exactly these); (node,
 * X-group) pairs where the upper-partner array Qt^m can be nonzero; the terms
 * of those pairs }.  Groups beyond the 64th count everywhere.  SGDG_E_ARG for
 * a null handle or array, an unknown kind or a level outside the hierarchy. */
sgdg_status sgdg_op_support(sgdg_ops o, int kind, int lx, int64_t* counts);

/* Diagnostic: the grid-problem preconditioner alone, out = (Tt + delta Ct +
 * Gt)^-1 (x) M^x^-1 (x) M^v^-1 in (mass inverses as selected by `sweeps`, see
 * mass_sweeps) on the grid-problem layout: every upper grid, then every
 * lower grid, each an [R][n_x][n_v] block; in_dev and out_dev hold that many
 * elements of dtype t and must not overlap.  Queued on s. */
sgdg_status sgdg_debug_grid_precond(sgdg_ops o, int sweeps, const void* in_dev, void* out_dev, sgdg_dtype t,
                                    hipStream_t s);

/* Number of captured grid-problem GMRES graphs that the next graph solve of
 * o's own batch can replay.  A graph holds the device addresses it was
 * captured with, so every (re)allocation of a work buffer or table (a larger
 * batch, a tuning run, a rebuilt table) empties the cache on the next graph
 * solve; this returns 0 once such a change has happened.  SGDG_E_ARG on a null
 * argument. */
sgdg_status sgdg_graph_cache_size(sgdg_ops o, int* count);

/* Host-only: the learned preconditioner's fallback rule applied to a recorded
 * sequence of n FGMRES iterations.  call[i] numbers the FGMRES call of
 * iteration i (mixed precision runs one call per refinement step; the history
 * restarts with each call), rel0[i] is that call's relative residual at entry
 * and est[i] the residual estimate after the iteration, both relative to the
 * call's right-hand side.  *switch_at = index of the iteration after which the
 * solve switches to the combination technique (no drop by `drop` over `iters`
 * consecutive iterations of one call), or -1.  Touches no device. */
sgdg_status sgdg_debug_fallback(int iters, double drop, int n, const int* call, const double* rel0,
                                const double* est, int* switch_at);

/* Host-only: dense block (row_grid, col_grid) of the operator `kind` (FULL,
 * MASS, DATA_F or DATA_G; not BLOCKDIAG) assembled from the host factor
 * tables, for small grids.  Grids are indices on the upper diagonal.  out:
 * host array of (Rout*nx*nv) x (Rin*nx'*nv') doubles, row-major, rows in the
 * [s][kx][kv] order of the row grid.  Touches no device.  Fails with
 * SGDG_E_ARG on bad indices. */
sgdg_status sgdg_debug_dense_block(const sgdg_domain* x, const sgdg_domain* v, int level_min, int level_max,
                                   int time_degree, const sgdg_problem* p, int kind, int row_grid,
                                   int col_grid, double* out);

#ifdef __cplusplus
}
#endif

#endif /* SGDG_H */
