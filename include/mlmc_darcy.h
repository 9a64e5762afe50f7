/*
 * mlmc_darcy.h -- C ABI of the MI355X (gfx950) library for multilevel Monte
 * Carlo estimation of Darcy flow in randomly layered media.
 *
 * Method: Park & Teckentrup, "Improved Multilevel Monte Carlo Methods for
 * Finite Volume Discretisations of Darcy Flow in Randomly Layered Media"
 * (arXiv 1506.04694).  For each sample omega the library
 *   1. samples the layered permeability k(x, omega) at the cell centres
 *      (Section 2, Examples 1 and 2, eq. (2.3); layer shapes of Section 3.4;
 *      circulant embedding of Section 3.4),
 *   2. assembles the cell-centred finite volume system eq. (3.3) with
 *      harmonic-mean faces (Sections 3.1 and 3.4) for Model Problem 2,
 *      eq. (3.11),
 *   3. solves it with a multigrid-preconditioned conjugate gradient method
 *      stopped on ||r_m|| / ||r_0|| (Section 3.5),
 *   4. evaluates the outflow M^(2) through x1 = 1 (Section 3.4), and
 *   5. reduces the samples into the MLMC estimator eq. (3.6)/(3.7) or the
 *      Coarse Grid Variates estimator eq. (4.1)/(4.2) (Section 4.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Grids are uniform m^d boxes on (0,1)^d, h = 1/m; cell (i, j) has centre
 *   ((i + 1/2) h, (j + 1/2) h); i runs along x1 (the flow direction).
 *   A per-sample field is stored row-major [j][i] (x1 fastest), and batches
 *   are sample-major: element (s, j, i) sits at s*m*m + j*m + i.
 * - Only d = 2 is implemented; other values return MLMC_EINVAL.
 * - Every pointer argument named as "device" is device memory owned by the
 *   caller, sized as documented, on the context's device.  Input and output
 *   buffers must not overlap.  Host pointers are marked "host".
 * - Calls enqueue work on the context's stream and return without waiting,
 *   except where documented (mlmc_ce_min_embedding, mlmc_solve's convergence
 *   polling, mlmc_level_run).  Device errors may surface at a later call.
 * - No call throws; every call returns an mlmc_status and, on failure,
 *   leaves a message for mlmc_last_error.
 * - Sample s of a batch is Monte Carlo sample number first_sample + s.  Its
 *   random numbers are a pure function of (seed, level, sample number), so
 *   results do not depend on how samples are batched.
 */
#ifndef MLMC_DARCY_H
#define MLMC_DARCY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mlmc_status {
  MLMC_OK = 0,
  MLMC_EINVAL = 1,   /* invalid argument or unsupported configuration        */
  MLMC_ENOMEM = 2,   /* device allocation failed                              */
  MLMC_EDEVICE = 3,  /* HIP runtime error                                     */
  MLMC_EBUSY = 4,    /* resource limit reached; retry later                   */
  MLMC_ENOCONV = 5,  /* at least one sample did not converge (mlmc_level_run) */
  MLMC_EEMBED = 6    /* circulant embedding has negative eigenvalues          */
} mlmc_status;

/* Per-sample solver outcome written to the status[] array of mlmc_solve. */
enum {
  MLMC_SAMPLE_OK = 0,        /* relative residual below tol                    */
  MLMC_SAMPLE_NOCONV = 1,    /* maxit iterations without reaching tol          */
  MLMC_SAMPLE_BREAKDOWN = 2  /* non-finite value or non-positive p^T A p       */
};

/* Layer geometry (Section 2: random partition independent of k; Section 3.4). */
enum {
  MLMC_IFACE_HORIZONTAL = 0,       /* x2 = y0, y0 ~ U(y_lo, y_hi); 2 layers            */
  MLMC_IFACE_PIECEWISE_LINEAR = 1, /* n_nodes equispaced nodes x = q/(n_nodes-1),
                                      heights ~ U(y_lo, y_hi); 2 layers               */
  MLMC_IFACE_PAPER_TWO_LINES = 2,  /* Section 3.4: lines (0,y1)-(1,y2), (0,y3)-(1,y4),
                                      y1~U(.8,.9) y2~U(.6,.7) y3~U(.2,.3) y4~U(.4,.5);
                                      3 layers                                        */
  MLMC_IFACE_TILTED_PLANE = 3,     /* x2 = a + (b-a) x1 + c (x3 - 1/2), a, b ~ U(y_lo,
                                      y_hi), c ~ U(-0.1, 0.1); 2 layers; in 2-D the
                                      line from (0,a) to (1,b)                        */
  MLMC_IFACE_NONE = 4              /* one layer (stationary field)                    */
};

/* Boundary value problem and quantity of interest (Section 3.4). */
enum {
  MLMC_PROBLEM_OUTFLOW = 0,      /* Model Problem 2: p = 1 on x1 = 0, p = 0 on x1 = 1,
                                    no flow elsewhere, f = 0; QoI = outflow M^(2)
                                    through x1 = 1                                   */
  MLMC_PROBLEM_MEAN_PRESSURE = 1 /* Model Problem 1: f = 1, p = 0 on the whole
                                    boundary; QoI = M^(1), the mean pressure over
                                    D* = [1/2 - 1/16, 1/2 + 1/16]^d (the paper fixes
                                    neither the point nor D*)                       */
};

/* Per-layer law (Section 2). */
enum {
  MLMC_FIELD_PIECEWISE_CONSTANT = 0, /* Example 1: k_l = exp(mu_l + sqrt(sigma2_l) z_l) */
  MLMC_FIELD_CORRELATED = 1          /* Example 2: k = exp(mu_l + g_l(x)), g_l Gaussian
                                        with covariance eq. (2.3) of the layer's own
                                        sigma2, lambda (all layers share r and n_ce),
                                        sampled by circulant embedding; independent
                                        across layers                                  */
};

/*
 * Random layered permeability model.  Layer 0 is the bottom layer; a cell
 * centre exactly on an interface belongs to the upper layer.
 * Random streams (Philox4x32-10, key = seed, counter = (block, sample number,
 * level, tag)): tag 0 geometry uniforms (uniform q = word q%4 of block q/4),
 * tag 1 layer constants (normals z0..z3 of block 0 by Box-Muller), tag 2
 * circulant-embedding noise of embedding sample p at tag 2 + p (noise point
 * (k2, k1) takes (z0, z1) of block (k2/2)*n_ce + k1 for even k2 and (z2, z3)
 * of that block for odd k2).  Layers share an embedding sample only when their
 * (sigma2, lambda) agree: layer l, in order, takes the imaginary part of the
 * first earlier sample with its covariance whose imaginary part is free, else
 * the real part of a new sample (two layers of one covariance: real part ->
 * layer 0, imaginary part -> layer 1).  In 3-D the noise lines along x1 are
 * numbered row = k3 n_ce + k2 and take the same rule with row in place of k2.
 */
typedef struct mlmc_model {
  int32_t dim;            /* 2 or 3                                             */
  int32_t interface_kind; /* MLMC_IFACE_*                                       */
  int32_t n_nodes;        /* nodes of a piecewise-linear interface (2..8)       */
  int32_t n_layers;       /* layers actually used (1..3)                        */
  int32_t field_kind;     /* MLMC_FIELD_*                                       */
  int32_t norm_r;         /* 1 or 2: the l_r norm of eq. (2.3)                  */
  int32_t n_ce;           /* circulant-embedding points per direction for the grid
                             being sampled (>= 2m, factors 2, 3, 5 only, <= 4096) */
  int32_t problem;        /* MLMC_PROBLEM_*: boundary value problem and QoI of the
                             level runs and the server                         */
  double y_lo, y_hi;      /* range of interface heights                         */
  double mu[4];           /* layer means of log k                               */
  double sigma2[4];       /* layer variances of log k                           */
  double lambda[4];       /* correlation lengths (correlated layers)            */
  uint64_t seed;
} mlmc_model;

/* Storage precision of the multigrid preconditioner (the outer CG, its
 * residuals, dot products and the coarsest solve are always FP64). */
enum {
  MLMC_PREC_FP64 = 0,  /* hierarchy in FP64, FP64 arithmetic                        */
  MLMC_PREC_FP32 = 1,  /* hierarchy in FP32, FP32 arithmetic, flexible outer CG      */
  MLMC_PREC_BF16 = 2   /* hierarchy in bfloat16, FP32 arithmetic, flexible outer CG  */
};

/* Multigrid-preconditioned CG options (Section 3.5 uses ||r_m||/||r_0|| < 1e-10). */
typedef struct mlmc_solver_opts {
  double tol;           /* relative residual tolerance in the 2-norm; x0 = 0        */
  double omega;         /* scaling of the coarse-grid correction (default 1.9)      */
  int32_t maxit;        /* iteration cap (default 200)                              */
  int32_t nu1, nu2;     /* red-black Gauss-Seidel sweeps before / after (default 1) */
  int32_t coarse_max;   /* coarsen while the grid is even and larger than this
                           (default 4); the coarsest grid (<= 8 x 8) is solved by
                           dense Cholesky                                           */
  int32_t check_every;  /* iterations between host checks of the active count      */
  int32_t variant;      /* 0: fused LDS-tiled cycle kernels, and for 64 x 64 FP64
                           the whole solve of a sample in one workgroup (needs
                           nu1 = nu2 = 1, else falls back to 1); 1: one launch
                           per sweep / step (3-D: also on the small levels the
                           in-LDS cycle takes otherwise); 2: the tiled kernels on
                           every grid */
  int32_t precision;    /* MLMC_PREC_*; reduced precision needs variant 0, nu = 1;
                           64 x 64 solves (variant 0) run on chip in FP64 at
                           every setting                                      */
  int32_t cycle_max;    /* variant 0: levels of at most this size (2..32, 0 = 32) run
                           in one workgroup per sample                              */
  int32_t gamma;        /* coarse-grid visits on the gamma_levels finest levels:
                           1 V-cycle, 2 W-cycle (default 2); a second visit
                           re-smooths the level before restricting again        */
  int32_t gamma_levels; /* number of finest levels taking gamma visits, the
                           coarser ones take one (default 2; 0 = every level)  */
  int32_t graph;        /* 1: after the first host check, run the 2-D fused
                           iteration as replays of a captured HIP graph of
                           check_every iterations (even check_every; cached per
                           context and configuration; bitwise the same results;
                           not while a kernel is being profiled); default 0 */
  int32_t initial_guess; /* 1: p holds an initial guess on entry (2-D solves; the
                            on-chip 64 x 64 path and the 3-D solver start from
                            zero).  The stopping rule is ||r||/||b|| < tol either
                            way (||b|| = ||r_0|| for the zero guess); default 0 */
  int32_t tile_shape;   /* tile kernels of the 2-D multigrid: 0 the default tile
                           shapes, 1 an alternative set (other tile sizes and
                           workgroup sizes) for the autotuner to try; the same
                           arithmetic per cell (the r^T z partial sums add the
                           tiles in another order); default 0                 */
} mlmc_solver_opts;

/* Per-level sums of the estimator (host struct; accumulates across calls). */
typedef struct mlmc_level_sums {
  int64_t n;            /* samples added                                            */
  int64_t n_failed;     /* samples whose fine or coarse solve did not reach tol     */
  double sum_y;         /* sum of Y = Q_f - Q_c  (Q_c = 0 on level 0)               */
  double sum_y2;        /* sum of Y^2                                               */
  double sum_qf;        /* sum of Q_f                                               */
  double sum_qc;        /* sum of Q_c                                               */
  int64_t iters_fine;   /* total CG iterations of the fine solves                   */
  int64_t iters_coarse; /* total CG iterations of the coarse solves                 */
} mlmc_level_sums;

typedef struct mlmc_estimate_t {
  double estimate;            /* eq. (3.6): sum over levels of mean Y               */
  double variance;            /* statistical part of eq. (3.7): sum V_l / N_l        */
  double std_error;           /* sqrt(variance)                                     */
} mlmc_estimate_t;

typedef struct mlmc_ctx mlmc_ctx;

/* Create a context on `device`.  `hip_stream` (a hipStream_t, may be NULL for
 * the default stream) is the stream every call enqueues on.  The context owns
 * its workspaces (embedding eigenvalues, multigrid hierarchies, scratch
 * vectors) until mlmc_ctx_destroy.  A context is not thread-safe. */
mlmc_status mlmc_ctx_create(int device, void* hip_stream, mlmc_ctx** out);
mlmc_status mlmc_ctx_destroy(mlmc_ctx* ctx);
mlmc_status mlmc_ctx_set_stream(mlmc_ctx* ctx, void* hip_stream);
/* Message of the last failed call on ctx (never NULL; "" when none). */
const char* mlmc_last_error(const mlmc_ctx* ctx);

/* Fill `opts` with the defaults: tol 1e-13, omega 1.9, maxit 200, nu1 = nu2 = 1,
 * coarse_max 4, check_every 4, variant 0, FP64, cycle_max 32, gamma 2,
 * gamma_levels 2. */
mlmc_status mlmc_solver_opts_default(mlmc_solver_opts* opts);

/* Circulant embedding (Section 3.4, exact sampling of eq. (2.3) on a grid):
 * smallest n_ce >= 2m with prime factors in {2,3,5} whose embedding
 * eigenvalues satisfy min >= -1e-12 max for every layer's covariance.
 * Synchronises the stream.
 * n_ce_out: host. */
mlmc_status mlmc_ce_min_embedding(mlmc_ctx* ctx, const mlmc_model* model, int m, int* n_ce_out);

/* Sample k at the cell centres of an m^d grid for samples first_sample ..
 * first_sample + batch - 1 of `level` (Section 2, Examples 1-2, Section 3.4).
 *   k        device, [batch][m][m] (d = 2) or [batch][m][m][m] (d = 3,
 *            k[s][l][j][i] at x = ((i+1/2)h, (j+1/2)h, (l+1/2)h)), written.
 *   k_coarse device, [batch][m/2]^d or NULL.  When given (m even), also
 *            writes the plain MLMC coarse sample of the same omega (eq. (3.6)):
 *            layers re-evaluated at the coarse centres; piecewise constant
 *            layers keep their value; correlated layers take the Gaussian
 *            value of fine cell (2I, 2J) (3-D: (2I, 2J, 2L)).
 * Correlated fields need model->n_ce valid for m (else MLMC_EEMBED; 3-D
 * embeddings are limited to n_ce <= 1024, else MLMC_EINVAL); the embedding
 * eigenvalues are computed once per (d, m, n_ce, sigma2, lambda, r) and cached
 * in the context. */
mlmc_status mlmc_sample_field(mlmc_ctx* ctx, const mlmc_model* model, int m, int level,
                              uint64_t first_sample, int batch, double* k, double* k_coarse);

/* As mlmc_sample_field, for arbitrary sample numbers: batch slot s holds
 * sample number sample_ids[s] (device uint32 [batch]). */
mlmc_status mlmc_sample_field_ids(mlmc_ctx* ctx, const mlmc_model* model, int m, int level,
                                  const uint32_t* sample_ids, int batch, double* k,
                                  double* k_coarse);

/* Coarse Grid Variates sub-samples (Section 4.1, eq. (4.1)): the 2^d coarse
 * samples k^(a)(I, J) = k(2I + a1, 2J + a2), a = a1 + 2 a2 (3-D:
 * k^(a)(I, J, L) = k(2I + a1, 2J + a2, 2L + a3), a = a1 + 2 a2 + 4 a3).
 *   k_fine device [batch][m]^d (m even); k_sub device [batch][2^d][m/2]^d. */
mlmc_status mlmc_cgv_extract(mlmc_ctx* ctx, int dim, int m, int batch,
                             const double* k_fine, double* k_sub);

/* Finite volume system eq. (3.3), harmonic-mean faces, Model Problem 2
 * (p = 1 on x1 = 0, p = 0 on x1 = 1, no flow on the other faces; f = 0).
 * A face between cells P and Q has T = h^(d-2) 2 k_P k_Q / (k_P + k_Q);
 * Dirichlet faces use the half-cell distance: T = 2 k_P h^(d-2).
 * d = 2:
 *   k   device [batch][m][m]            (input, positive)
 *   T   device [batch][2][m][m]: T[s][0][j][i] = transmissibility of the face
 *       x1 = (i+1)h of cell (i,j) (for i = m-1: the outflow boundary face);
 *       T[s][1][j][i] = face x2 = (j+1)h (0 for j = m-1, no flow).
 *   tb  device [batch][2][m]: tb[s][0][j] = face x1 = 0 of cell (0,j) (inflow
 *       boundary); tb[s][1][i] = face x2 = 0 of cell (i,0) (0, no flow).
 *   b   device [batch][m][m]: right-hand side (tb[s][0][j] in column i = 0).
 * d = 3 (cell (i, j, l), c = (l m + j) m + i):
 *   k, b device [batch][m][m][m];
 *   T   device [batch][3][m^3]: T[s][0][c] face x1 = (i+1)h (i = m-1: outflow
 *       boundary), T[s][1][c] face x2 = (j+1)h, T[s][2][c] face x3 = (l+1)h
 *       (0 on x2 = 1 and x3 = 1);
 *   tb  device [batch][3][m^2]: tb[s][0][l m + j] face x1 = 0 (inflow),
 *       tb[s][1][l m + i] face x2 = 0, tb[s][2][j m + i] face x3 = 0 (0).
 * Row P of the system: sum over faces T_f (p_P - p_nb) = b_P, where boundary
 * faces have p_nb = 0 after moving the Dirichlet data to b. */
mlmc_status mlmc_assemble(mlmc_ctx* ctx, int dim, int m, int batch, const double* k,
                          double* T, double* tb, double* b);

/* As mlmc_assemble for either model problem (MLMC_PROBLEM_*).  Model Problem 1
 * (Section 3.4: f = 1, p = 0 on every boundary face): every boundary face is a
 * Dirichlet face with T = 2 k_P h^(d-2) (tb[s][1] and the x2 = 1 (and x3 = 1)
 * faces are no longer 0) and b = f h^d = h^d in every cell.  Same layouts. */
mlmc_status mlmc_assemble_problem(mlmc_ctx* ctx, int problem, int dim, int m, int batch,
                                  const double* k, double* T, double* tb, double* b);

/* Solve A p = b for each sample of the batch (operator as produced by
 * mlmc_assemble) with conjugate gradients preconditioned by one symmetric
 * geometric multigrid cycle (Section 3.5; aggregation coarsening with
 * Galerkin coarse operators, red-black Gauss-Seidel smoothing; W on the
 * opts->gamma_levels finest levels when opts->gamma = 2).
 *   p       device [batch][m]^d, written (initial guess 0).
 * d = 2 needs m = c 2^k with c <= 8; d = 3 needs c <= 4 and an FP64 or FP32
 * hierarchy (bfloat16 is 2-D only)
 * (else MLMC_EINVAL).
 *   status  device int32 [batch], iters device int32 [batch],
 *   relres  device double [batch] = ||b - A p|| / ||b|| recomputed at exit.
 * A sample that fails is reported in status[]; it never stops the batch.
 * Polls a device counter every opts->check_every iterations (stream sync). */
mlmc_status mlmc_solve(mlmc_ctx* ctx, int dim, int m, int batch, const double* T,
                       const double* tb, const double* b, double* p,
                       const mlmc_solver_opts* opts, int32_t* status, int32_t* iters,
                       double* relres);

/* mlmc_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, layouts, results and errors as mlmc_solve (the same kernels run),
 * but every workspace -- residual, search and correction vectors, the
 * multigrid hierarchy, per-sample scalars and partial sums -- is carved from
 * one static 64 MiB device array in the library instead of the context's
 * allocated workspaces.  No hipMalloc, hipFree or allocating library call is
 * made.  Limits and behaviour:
 *   - the solve's workspaces must fit in the 64 MiB array (about 2500 samples
 *     of 64 x 64, 57 of 128 x 128, 14 of 256 x 256 with the FP64 defaults;
 *     3-D: 30 of 32^3); a larger batch is refused with MLMC_EINVAL and a
 *     message naming the workspace that did not fit, before any work is
 *     enqueued;
 *   - opts->graph must be 0 (MLMC_EINVAL otherwise); kernel timing
 *     (mlmc_profile_enable) does not record this call;
 *   - each device holds one copy of the array for the life of the process and
 *     every call on that device uses it: calls that overlap on one device (two
 *     contexts or streams, or threads) race and corrupt each other's results.
 *     Calls on one stream are ordered and safe.  The array keeps the previous
 *     call's contents; nothing in the solve reads a workspace before writing it. */
mlmc_status mlmc_solve_noalloc(mlmc_ctx* ctx, int dim, int m, int batch, const double* T,
                               const double* tb, const double* b, double* p,
                               const mlmc_solver_opts* opts, int32_t* status, int32_t* iters,
                               double* relres);

/* Outflow M^(2) through x1 = 1 (Section 3.4) of the discrete solution:
 * q_out[s] = sum over the cells with i = m-1 of 2 k h^(d-2) p; q_in[s]
 * (optional, may be NULL) = sum over the cells with i = 0 of 2 k h^(d-2)
 * (1 - p) (equal to q_out for the exact solution: local conservation).
 * k, p device [batch][m]^d; q_out, q_in device [batch]. */
mlmc_status mlmc_qoi_outflow(mlmc_ctx* ctx, int dim, int m, int batch, const double* k,
                             const double* p, double* q_out, double* q_in);

/* Model Problem 1's QoI M^(1) (Section 3.4) of the discrete, cell-wise constant
 * pressure: the mean over the box [lo, hi]^d (0 <= lo < hi <= 1),
 *   q[s] = sum over cells P of p_P |P cap [lo, hi]^d| / (hi - lo)^d.
 * p device [batch][m]^d; q device [batch]. */
mlmc_status mlmc_qoi_box_mean(mlmc_ctx* ctx, int dim, int m, int batch, const double* p,
                              double lo, double hi, double* q);

/* One level of the estimator for samples first_sample .. first_sample + n - 1:
 * sample (fine grid m_fine), assemble, solve, QoI; for level >= 1 also the
 * coarse companions on the m_fine/2 grid -- the plain coarse sample of the
 * same omega (eq. (3.6)), or with cgv != 0 the 2^d sub-lattices averaged as in
 * eq. (4.1) -- and Y = Q_f - Q_c (eq. (4.2)); on level 0, Y = Q_f.
 * Adds the level's sums to *sums (host).  q_f, q_c, y: device [n] or NULL.
 * Synchronises the stream before returning.  Returns MLMC_ENOCONV when any
 * solve failed (the sums are still updated, n_failed counts them). */
mlmc_status mlmc_level_run(mlmc_ctx* ctx, const mlmc_model* model, int level, int m_fine,
                           uint64_t first_sample, int n, int cgv,
                           const mlmc_solver_opts* opts, mlmc_level_sums* sums,
                           double* q_f, double* q_c, double* y);

/* As mlmc_level_run for arbitrary sample numbers (device uint32 sample_ids[n]),
 * with optional per-sample outputs: failed (device int32 [n], 1 when the fine or
 * a coarse solve did not reach tol) and iters (device int32 [n], CG iterations
 * of the fine solve).  A sample's results do not depend on the other samples
 * of the call. */
mlmc_status mlmc_level_run_ids(mlmc_ctx* ctx, const mlmc_model* model, int level, int m_fine,
                               const uint32_t* sample_ids, int n, int cgv,
                               const mlmc_solver_opts* opts, mlmc_level_sums* sums, double* q_f,
                               double* q_c, double* y, int32_t* failed, int32_t* iters);

/* Every level of the estimator in one call: level l has n[l] samples starting
 * at first_sample[l] on the m_fine[l] grid (embedding size n_ce[l] for
 * correlated fields; n_ce may be NULL for piecewise constant models) and
 * solver options opts[l].  The levels are independent (eq. (3.6)), so each
 * level's pipeline -- sampling, coarse companions, fine solve, QoI, sums --
 * runs concurrently with the others on a stream of its own (the context keeps
 * one internal context, stream and workspace set per level for later calls),
 * starting after the work already enqueued on the context's stream.  Results
 * are those of mlmc_level_run for each level (same samples, bitwise the same
 * numbers).  All inputs host; sums[n_levels] (host) accumulate.  Synchronises.
 * Kernel timing (mlmc_profile_enable) does not record these launches. */
mlmc_status mlmc_run_levels(mlmc_ctx* ctx, const mlmc_model* model, int n_levels,
                            const int* m_fine, const int* n_ce, const uint64_t* first_sample,
                            const int* n, int cgv, const mlmc_solver_opts* opts,
                            mlmc_level_sums* sums);

/* Estimator eq. (3.6) and the statistical part of eq. (3.7) from per-level
 * sums (host arithmetic only).  levels: host [n_levels]; out: host. */
mlmc_status mlmc_estimate(const mlmc_level_sums* levels, int n_levels, mlmc_estimate_t* out);

/* ---------------------------------------------------------------- choosing L and N_l
 * Section 3.2 splits the mean square error eq. (3.7) evenly between the
 * variance sum_l V_l / N_l and the squared bias (E[Q_L - Q])^2, eps^2 / 2 each,
 * and takes the N_l that reach the variance part at the least cost
 * sum_l N_l C_l (C_l: cost of one sample of Y_l). */

/* N_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k)), the minimiser of
 * the cost under the variance constraint, rounded up.  var, cost (> 0),
 * n_out: host [n_levels].  Host arithmetic only. */
mlmc_status mlmc_optimal_samples(const double* var, const double* cost, int n_levels, double eps,
                                 int64_t* n_out);

/* Rates of the complexity theorem's (M1)-(M3) as least squares slopes of
 * log2 |E[Y_l]|, log2 V[Y_l] and log2 C_l against log2 h_l (h_l = 1/m_l) over
 * the levels l >= 1: |E[Y_l]| ~ h^alpha, V[Y_l] ~ h^beta, C_l ~ h^-gamma.
 * sums, cost, m: host [n_levels] (n_levels >= 3, n >= 2 per level).  Host only. */
mlmc_status mlmc_rates(const mlmc_level_sums* sums, const double* cost, const int* m,
                       int n_levels, double* alpha, double* beta, double* gamma);

#define MLMC_MAX_LEVELS 16

typedef struct mlmc_adaptive_opts {
  double eps;           /* target root mean square error (> 0)                          */
  double alpha;         /* rate of |E[Y_l]| for the bias estimate; 0: fitted over the
                           levels l >= 1 (at least 0.5)                                  */
  int32_t n_initial;    /* samples of a newly added level (>= 2, default 64)            */
  int32_t min_levels;   /* levels to start with (2..max_levels, default 3)              */
  int32_t cgv;          /* 1: Coarse Grid Variates estimator (eq. (4.2))                */
  int32_t reserved;
  int64_t max_samples;  /* cap on the samples of one level (default 2^24)              */
} mlmc_adaptive_opts;

typedef struct mlmc_adaptive_result {
  int32_t n_levels;           /* levels used (L + 1)                                   */
  int32_t converged;          /* 1: variance <= eps^2/2 and bias <= eps/sqrt(2)         */
  double estimate;            /* eq. (3.6)                                             */
  double variance;            /* sum_l V_l / N_l                                       */
  double bias;                /* |E[Y_L]| / (2^alpha - 1)                              */
  double alpha, beta, gamma;  /* alpha used; beta, gamma fitted (NaN below 3 levels)   */
  double seconds;             /* wall time of the level runs                           */
  int64_t n[MLMC_MAX_LEVELS];       /* samples per level                              */
  double mean_y[MLMC_MAX_LEVELS];   /* sample mean of Y_l                             */
  double var_y[MLMC_MAX_LEVELS];    /* unbiased sample variance of Y_l                */
  double cost[MLMC_MAX_LEVELS];     /* seconds per sample of level l                  */
  mlmc_level_sums sums[MLMC_MAX_LEVELS];
} mlmc_adaptive_result;

/* Defaults: eps 1e-2, alpha 0 (fitted), n_initial 64, min_levels 3, cgv 0,
 * max_samples 2^24. */
mlmc_status mlmc_adaptive_opts_default(mlmc_adaptive_opts* opts);

/* MLMC to a root mean square error eps (Section 3.2): start with min_levels
 * levels of n_initial samples; repeatedly run each level's missing samples
 * (mlmc_level_run, new sample numbers after those already taken; at most 4x
 * the level's samples per round), take its cost per sample from its largest
 * call (the per-call overhead does not grow with the samples), and set N_l by
 * mlmc_optimal_samples from the sample variances; once no level lacks samples, estimate the bias of the finest
 * level and add the next level (n_initial samples) while it exceeds
 * eps / sqrt(2) and levels remain.  Level l uses the grid m_levels[l]
 * (m_levels[l] = 2 m_levels[l-1]) and, for correlated fields, n_ce[l] (NULL:
 * model->n_ce).  model, m_levels, n_ce, opts, solver, out: host.
 * max_levels <= MLMC_MAX_LEVELS.  Synchronises. */
mlmc_status mlmc_adaptive(mlmc_ctx* ctx, const mlmc_model* model, int max_levels,
                          const int* m_levels, const int* n_ce, const mlmc_adaptive_opts* opts,
                          const mlmc_solver_opts* solver, mlmc_adaptive_result* out);

/* Kernel timing: when enabled, every launch of the named kernel is bracketed
 * by HIP events on the context's stream; mlmc_profile_read returns the launch
 * count, the summed event time and the algorithmic bytes the library counts
 * for those launches.  kernel_name NULL disables.  Host outputs.
 * The tiled multigrid kernels (k_mg_down, k_mg_mid, k_mg_up) also answer to
 * "<name>@<level>", which times the launches on that level of each solve only
 * (level 0 = the finest grid, the kernel instantiation that works on FP64
 * residuals), and to "<name>@<level>#<cells>", the launches on that level
 * whose batch holds that many cells (batch x m x m; e.g. the 2^24-cell fine
 * solves of a level run apart from its 2^22-cell companions). */
mlmc_status mlmc_profile_enable(mlmc_ctx* ctx, const char* kernel_name);
mlmc_status mlmc_profile_read(mlmc_ctx* ctx, int64_t* launches, double* total_ms,
                              double* algorithmic_bytes);

/* ------------------------------------------------------------------------
 * Request server with continuous batching (serving form of the estimator).
 * A request is one estimator term (eq. (3.6), or eq. (4.2) with CGV): sample
 * number `sample` of `level` on the m_fine grid.  Worker threads each own a
 * context with its own HIP stream and device-resident workspaces; a free
 * worker takes a batch of one (model, level, m_fine) kind -- that kind's
 * oldest waiting requests, up to max_batch, while the estimated device memory
 * of the running batches stays within hbm_budget_bytes (a single request runs
 * whenever nothing else does).  The kind is the one whose oldest request has
 * waited longest in units of the kind's expected service time (estimated from
 * its cells), among the kinds that fit the budget; while short requests wait,
 * at most n_workers - 1 workers serve long kinds (above about 3 ms), unless a
 * long request has waited 50 ms.
 * Requests arriving while others run are admitted as workers and memory free
 * up; batches of different workers overlap on the device.  Results are
 * independent of batching.  Times are seconds on the server's clock
 * (mlmc_serve_now).  All calls are thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct mlmc_server mlmc_server;

typedef struct mlmc_serve_opts {
  int32_t device;
  int32_t n_workers;          /* concurrent batches, 1..16 (default 3)            */
  int32_t max_batch;          /* requests per batch (default 256)                 */
  int32_t cgv;                /* 0: plain coarse companion, 1: CGV                */
  uint64_t hbm_budget_bytes;  /* admission limit for running batches (default 64 GiB) */
  int32_t n_grids;            /* entries in grid_m / grid_n_ce (correlated fields) */
  int32_t grid_m[8];          /* fine grid sizes served ...                       */
  int32_t grid_n_ce[8];       /* ... and their circulant-embedding sizes          */
  int32_t grid_model[8];      /* ... for this model index (0 with one model)      */
  int32_t reserved;
  mlmc_solver_opts solver;
} mlmc_serve_opts;

typedef struct mlmc_request {
  int32_t level;
  int32_t m_fine;
  uint32_t sample;
  int32_t model;       /* index of the model (0 .. n_models - 1)               */
} mlmc_request;

typedef struct mlmc_result {
  uint64_t id;
  int32_t level, m_fine;
  uint32_t sample;
  int32_t failed;      /* 1: a solve missed tol or the batch failed            */
  int32_t iters;       /* CG iterations of the fine solve                      */
  int32_t batch_size;  /* requests in the batch that served it                 */
  int32_t status;      /* MLMC_OK, or the error of the batch                   */
  int32_t model;       /* model index of the request                           */
  double q_f, q_c, y;  /* Q on the fine grid, coarse (companion mean), Y       */
  double t_submit, t_start, t_done;
} mlmc_result;

/* Defaults: device 0, 3 workers, batches up to 256, plain MLMC, 64 GiB budget,
 * mlmc_solver_opts_default. */
mlmc_status mlmc_serve_opts_default(mlmc_serve_opts* opts);
/* Starts the workers for one model (host; copied); opts->solver for every batch.
 * Returns once every worker has warmed up: one level run of up to 16 samples
 * (sample numbers 0xFFFFF000 and up) per served grid, so that each grid's
 * embedding eigenvalues and the worker's workspaces exist before requests
 * arrive.  Workspaces then grow geometrically with the batches served. */
mlmc_status mlmc_serve_start(const mlmc_model* model, const mlmc_serve_opts* opts,
                             mlmc_server** out);
/* Starts the workers for n_models (1..8) models at once, e.g. 2-D and 3-D fields
 * in one request stream.  models: host [n_models] (copied); solvers: host
 * [n_models] solver options per model (copied), or NULL for opts->solver;
 * grid q of opts serves model opts->grid_model[q].  A batch holds requests of
 * one (model, level, m_fine) and runs with that model's solver options.
 * MLMC_EINVAL for a count out of range, a grid of an unknown model or a model
 * whose dim is not 2 or 3. */
mlmc_status mlmc_serve_start_models(const mlmc_model* models, const mlmc_solver_opts* solvers,
                                    int n_models, const mlmc_serve_opts* opts,
                                    mlmc_server** out);
/* Queues a request (host); id (host, may be NULL) receives its identifier.
 * MLMC_EINVAL for an unknown model, a bad level or grid, or a grid with no
 * embedding size for a correlated model. */
mlmc_status mlmc_serve_submit(mlmc_server* srv, const mlmc_request* req, uint64_t* id);
/* Moves up to max finished results into out (host); *n_out = number moved;
 * *pending (may be NULL) = requests queued or finished and not yet polled. */
mlmc_status mlmc_serve_poll(mlmc_server* srv, mlmc_result* out, int max, int* n_out,
                            int64_t* pending);
/* Current time on the server's clock in seconds. */
double mlmc_serve_now(const mlmc_server* srv);
mlmc_status mlmc_serve_stats(mlmc_server* srv, int64_t* batches, int64_t* queued, int* running,
                             uint64_t* in_flight_bytes);
/* Finishes running batches, drops queued requests, frees everything. */
mlmc_status mlmc_serve_stop(mlmc_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* MLMC_DARCY_H */
