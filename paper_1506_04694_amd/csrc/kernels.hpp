// Host-side launch wrappers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <hip/hip_ext.h>

#include "../../include/mlmc_darcy.h"
#include "fft.hpp"

namespace mlmc {

// Kernel timing.  The library's profiled kernels (the tiled multigrid
// kernels, the CG direction, the PCG update, the 3-D half-sweep) are issued
// through launch_k.  When the caller has armed this host thread's event pair
// (the timing wrapper does, for the kernel it profiles), the launch goes out
// with hipExtLaunchKernelGGL, which stamps the two events with the dispatch's
// own start and end, and disarms the pair; otherwise it is a plain launch.
struct ArmedEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
ArmedEvents& armed_events();

template <typename F, typename... Args>
inline void launch_k(F kernel, const dim3& grid, const dim3& block, uint32_t lds, hipStream_t st,
                     Args... args) {
  ArmedEvents& ev = armed_events();
  const hipEvent_t a = ev.start, b = ev.stop;
  ev.start = ev.stop = nullptr;
  hipExtLaunchKernelGGL(kernel, grid, block, lds, st, a, b, 0u, args...);
}

// ------------------------------------------------------------- field.hip
// Sample number of batch slot s: ids[s] when ids != NULL, else first + s.
void launch_sample_params(hipStream_t st, const mlmc_model& mdl, int level, uint64_t first,
                          const uint32_t* ids, int batch, double* params);
void launch_field_pc(hipStream_t st, const mlmc_model& mdl, int m, int batch,
                     const double* params, double* k);
void launch_ce_twiddles(hipStream_t st, int n, double2* tw);
void launch_ce_first_row(hipStream_t st, int n, int m, double sigma2, double lambda, int norm_r,
                         double2* c);
void launch_fft_lines(hipStream_t st, double2* data, int n, int nlines, long long line_stride,
                      long long elem_stride, const double2* tw, const FftPlan& pl);
void launch_ce_minmax(hipStream_t st, const double2* lam, long long count, double* partial,
                      int nblocks);
void launch_ce_sqrt_transpose(hipStream_t st, const double2* lam, int n, double* sqT);
// One circulant-embedding sample ("pair") of a correlated model: the noise
// stream tag it draws from, the layer taking its real part and the layer taking
// its imaginary part (l_im < 0: none), with their means.  Layers share a sample
// only when their covariance parameters agree.
// Sets the context's last-error message (host drivers outside api.hip).
mlmc_status set_error(mlmc_ctx* ctx, mlmc_status code, const char* msg);

struct CePair {
  uint32_t tag;
  int l_re, l_im;
  double mu_re, mu_im;
};
void launch_ce_pass_a(hipStream_t st, const mlmc_model& mdl, const CePair& pr, int level,
                      uint64_t first, const uint32_t* ids, int batch, int m, const double* sqT,
                      const double2* tw, const FftPlan& pl, double2* uT);
void launch_ce_pass_b(hipStream_t st, const mlmc_model& mdl, const CePair& pr, int batch, int m,
                      const double2* uT, const double2* tw, const FftPlan& pl,
                      const double* params, double* k, double* k_coarse);
void launch_cgv_extract(hipStream_t st, int m, int batch, const double* kf, double* ksub);

// ------------------------------------------------------------- fv.hip
void launch_assemble(hipStream_t st, int problem, int m, int batch, const double* k, double* T,
                     double* tb, double* b);
void launch_qoi_box(hipStream_t st, int dim, int m, int batch, double lo, double hi,
                    const double* p, double* q);
void launch_qoi(hipStream_t st, int m, int batch, const double* k, const double* p, double* qout,
                double* qin);
void launch_cgv_average(hipStream_t st, int batch, int ncomp, const double* qcomp, double* qc);
void launch_y_and_fail(hipStream_t st, int n, const double* qf, const double* qc,
                       const int32_t* st_f, const int32_t* st_c, int ncomp, double* y,
                       int32_t* failed);
void launch_level_reduce(hipStream_t st, int n, const double* y, const double* qf,
                         const double* qc, const int32_t* failed, const int32_t* it_f,
                         const int32_t* it_c, int ncomp, double* out6);

// ------------------------------------------------------------- mg_pcg.hip
struct SolverState {          // per-sample scalars, device arrays of length batch
  double* r0sq;
  double* rho;
  double* alpha;
  double* beta;
  int32_t* active;
  int32_t* count;             // one int: active samples after the last convergence check
};

void launch_coarsen(hipStream_t st, int m, int batch, const double* T, const double* tb,
                    double* Tc, double* tbc);
void launch_rbgs(hipStream_t st, int m, int batch, const double* T, const double* tb, double* z,
                 const double* r, const int32_t* active, int color, int zero_init);
void launch_resid_restrict(hipStream_t st, int m, int batch, const double* T, const double* tb,
                           const double* z, const double* r, double* rc,
                           const int32_t* active);
void launch_prolong(hipStream_t st, int m, int batch, const double* zc, double* z, double omega,
                    const int32_t* active);
void launch_dense_factor(hipStream_t st, int m, int batch, const double* T, const double* tb,
                         double* work, double* Ainv);
void launch_dense_apply(hipStream_t st, int m, int batch, const double* Ainv, const double* r,
                        double* z, const int32_t* active);

// ------------------------------------------------------------- mg_fused.hip
constexpr int kTileX = 64;            // fused multigrid tile (cells along x1)
constexpr int kTileY = 16;            // fused multigrid tile (cells along x2)
constexpr int kCoarseCycleMax = 32;   // levels up to this size run in one workgroup per sample
constexpr int kMaxCoarseLevels = 8;

struct CoarseDesc {
  int m[kMaxCoarseLevels];
  const void* T[kMaxCoarseLevels];    // storage type of the hierarchy
  const void* tb[kMaxCoarseLevels];
};

// prec: MLMC_PREC_* storage of the hierarchy (T, tb, z_pre, z and r below the
// finest level).  top: the level is the finest one, whose r and z are FP64.
// With rz_partial != NULL (top only) the up kernel writes r^T z per tile:
// rz_partial[s * mg_rz_parts(m, prec, shape) + tile]; the coarse cycle per
// sample.  shape: mlmc_solver_opts.tile_shape (0 default tiles, 1 alternative).
int mg_rz_parts(int m, int prec, int shape);
size_t prec_bytes(int prec);
void launch_mg_down(hipStream_t st, int prec, int shape, bool top, int m, int batch,
                    const void* T, const void* tb, const void* r, void* z, void* rc,
                    const int32_t* active);
void launch_mg_up(hipStream_t st, int prec, int shape, bool top, int m, int batch, const void* T,
                  const void* tb, const void* r, const void* zpre, void* z, const void* zc,
                  double omega, const int32_t* active, double* rz_partial);
// Second coarse correction of a W-cycle level: z = zpre + omega P zc,
// black-red-black sweeps, z and the restricted residual rc.
void launch_mg_mid(hipStream_t st, int prec, int shape, bool top, int m, int batch, const void* T,
                   const void* tb, const void* r, const void* zpre, void* z, const void* zc,
                   double omega, void* rc, const int32_t* active);
size_t coarse_cycle_lds_bytes(const CoarseDesc& d, int nlev);
// Bit l of wmask: level l of the LDS-held levels takes two coarse visits (W).
void launch_mg_coarse_cycle(hipStream_t st, int prec, bool top, int batch, int nlev,
                            const CoarseDesc& desc, const void* r0, void* z0, const double* Ainv,
                            double omega, unsigned wmask, const int32_t* active,
                            double* rz_partial);
void launch_convert(hipStream_t st, int prec, long long count, const double* x, void* y);
// p_new = z + beta p_old (z when first), q = A p_new, partial[s * tiles + tile] = p_new . q;
// available when cg_direction_fused(m) (fixed tiles; cg_dir_parts(m) partials)
int cg_dir_parts(int m);
bool cg_direction_fused(int m);
void launch_cg_direction(hipStream_t st, int m, int batch, const double* T, const double* tb,
                         const double* z, const double* pold, double* pnew, double* q,
                         const double* beta, int first, double* partial, const int32_t* active);

// only != NULL: initialise just the samples with only[s] != 0
void launch_pcg_init(hipStream_t st, int n, int batch, const double* b, double* x, double* r,
                     double* partial, int bps, const int32_t* only);
void launch_pcg_init_guess(hipStream_t st, int m, int batch, const double* T, const double* tb,
                           const double* b, const double* x, double* r, double* partial,
                           int bps);
void launch_inject(hipStream_t st, int m, int batch, int ncomp, const double* xc, double* x);
void launch_spmv_dot(hipStream_t st, int m, int batch, const double* T, const double* tb,
                     const double* p, double* q, double* partial, int bps,
                     const int32_t* active);
// partial = sum r_new^2; with zold != NULL also partial2 = sum r_new . zold
void launch_axpy_dot(hipStream_t st, int n, int batch, double* x, double* r, const double* p,
                     const double* q, const double* alpha, double* partial, int bps,
                     const int32_t* active, const double* zold, double* partial2);
void launch_dot(hipStream_t st, int n, int batch, const double* a, const double* b,
                double* partial, int bps, const int32_t* active);
void launch_pupdate(hipStream_t st, int n, int batch, double* p, const double* z,
                    const double* beta, int bps, const int32_t* active, int first);
void launch_true_residual(hipStream_t st, int m, int batch, const double* T, const double* tb,
                          const double* b, const double* x, double* partial, int bps);

// restart != 0: only the samples with S.active set (after launch_sc_restart)
void launch_sc_init(hipStream_t st, int batch, const double* partial, int bps, SolverState s,
                    int32_t* status, int32_t* iters, double* relres, int restart);
void launch_sc_restart(hipStream_t st, int batch, SolverState s, int32_t* status, int32_t* iters,
                       int32_t* carried);
void launch_iters_add(hipStream_t st, int batch, int32_t* iters, const int32_t* carried);
// beta = rho_new / rho (standard) or (rho_new - r_new.z_old) / rho (flexible,
// partial2 != NULL: Polak-Ribiere form, for a preconditioner that is not
// exactly symmetric, e.g. one applied in reduced precision)
void launch_sc_rho(hipStream_t st, int batch, const double* partial, int nparts, SolverState s,
                   int32_t* status, int first, const double* partial2, int nparts2);
void launch_sc_alpha(hipStream_t st, int batch, const double* partial, int bps, SolverState s,
                     int32_t* status);
void launch_sc_conv(hipStream_t st, int batch, const double* partial, int bps, SolverState s,
                    int32_t* status, int32_t* iters, double* relres, double tol, int maxit);
void launch_sc_final(hipStream_t st, int batch, const double* partial, int bps, SolverState s,
                     double* relres);

inline int blocks_per_sample(long long n) { return (int)((n + kCellsPerBlock - 1) / kCellsPerBlock); }

// ---- 3-D path (d3.hip): layout T[s][3][m^3], tb[s][3][m^2] (west, south,
// bottom faces), k, b, x [s][m^3] with x1 fastest.
void launch_assemble3(hipStream_t st, int problem, int m, int batch, const double* k, double* T,
                      double* tb, double* b);
size_t qoi3_parts_size(int batch);  // doubles of the partials buffer
void launch_qoi3(hipStream_t st, int m, int batch, const double* k, const double* p, double* part,
                 double* qout, double* qin);
void launch_coarsen3(hipStream_t st, int m, int batch, const double* T, const double* tb,
                     double* Tc, double* tbc);
void launch_dense_factor3(hipStream_t st, int m, int batch, const double* T, const double* tb,
                          double* Ainv);
// Multigrid sweeps of a 3-D hierarchy in FP64 (f32 false) or with the operator,
// z and r stored and computed in float (f32 true); on the finest level (top)
// z and r are the CG's FP64 vectors in either case.  The swept level's T, z
// and r are in colour-split order (cs3.hpp); coarse_split: so are the next
// coarser level's z and r (else natural: the in-LDS or dense coarsest levels).
void launch_rbgs3_p(hipStream_t st, bool f32, bool top, int m, int batch, const void* T,
                    const void* tb, void* z, const void* r, const int32_t* active, int color,
                    int zero_init);
void launch_resid_restrict3_p(hipStream_t st, bool f32, bool top, int m, int batch,
                              const void* T, const void* tb, const void* z, const void* r,
                              void* rc, const int32_t* active, bool coarse_split);
void launch_prolong_black3_p(hipStream_t st, bool f32, bool top, int m, int batch, const void* T,
                             const void* tb, void* z, const void* r, const void* zc,
                             double omega, const int32_t* active, bool coarse_split);
void launch_dense_apply3f(hipStream_t st, int n, int batch, const double* Ainv, const float* r,
                          float* z, const int32_t* active);
// The cycle on levels l0..L of a 3-D hierarchy (desc: their sizes and
// operators, m_l0 <= coarse3_max_side(f32), coarsest <= 4) in LDS, one
// workgroup per sample; wmask bit q: level l0 + q takes two coarse visits.
// r0, z0: the vectors of level l0.
int coarse3_max_side(bool f32);
int coarse3_image_words(int nlev, const int* ms);  // words per sample
void launch_coarse3_image(hipStream_t st, bool f32, int batch, int nlev, const CoarseDesc& desc,
                          void* img);
void launch_coarse3_cycle(hipStream_t st, bool f32, bool top, int batch, int nlev,
                          const CoarseDesc& desc, const void* img, const void* r0, void* z0,
                          const double* Ainv, double omega, unsigned wmask,
                          const int32_t* active);
// q = A p and partial sums of p . q (T natural); p, q in colour-split order
// when split.
void launch_spmv3_dot(hipStream_t st, int m, int batch, const double* T, const double* tb,
                      const double* p, double* q, double* partial, int bps, const int32_t* active,
                      bool split);
// Ts (colour-split order; float when f32, else double) = T (natural, FP64).
void launch_faces_split3(hipStream_t st, bool f32, int m, int batch, const double* T, void* Ts);
// k_pcg_init with r in colour-split order (b natural).
void launch_pcg_init3_split(hipStream_t st, int m, int batch, const double* b, double* x,
                            double* r, double* partial, int bps, const int32_t* only);
// out (natural order) = in (colour-split order).
void launch_from_split3(hipStream_t st, int m, int batch, const double* in, double* out);
void launch_true_residual3(hipStream_t st, int m, int batch, const double* T, const double* tb,
                           const double* b, const double* x, double* partial, int bps);
void launch_field_pc3(hipStream_t st, const mlmc_model& mdl, int m, int batch,
                      const double* params, double* k);
void launch_ce_first_row3(hipStream_t st, int n, int m, double sigma2, double lambda, int norm_r,
                          double2* c);
void launch_ce_sqrt3(hipStream_t st, const double2* lam, int n, double* sq);
void launch_ce3(hipStream_t st, const mlmc_model& mdl, const CePair& pr, int level, uint64_t first,
                const uint32_t* ids, int batch, int m, const double* sq, const double2* tw,
                const FftPlan& pl, const double* params, double2* u1, double2* u2, double* k,
                double* k_coarse);
void launch_cgv_extract3(hipStream_t st, int m, int batch, const double* kf, double* ksub);
// z = A^-1 r for n unknowns per sample (coarsest grid of either dimension).
// Operators of the levels 64, 32, 16, 8 and 4 of a 64 x 64 solve (device).
struct OcHierarchy {
  const double* T[5];
  const double* tb[5];
};
// One workgroup per sample: z = M r for a 64 x 64 level and the four below it
// (wmask bit k: level k of the five takes two coarse visits).
void launch_cycle_onchip64(hipStream_t st, int batch, const OcHierarchy& h, const double* r,
                           double* z, const double* Ainv, double omega, unsigned wmask,
                           const int32_t* active);
// One workgroup per sample: the whole PCG solve of a 64 x 64 system on chip.
void launch_pcg_onchip64(hipStream_t st, int batch, const OcHierarchy& h, const double* b,
                         double* x, const double* Ainv, double tol, int maxit, double omega,
                         int gamma, int gamma_levels, int32_t* status, int32_t* iters,
                         double* relres);

void launch_dense_apply_n(hipStream_t st, int n, int batch, const double* Ainv, const double* r,
                          double* z, const int32_t* active);

}  // namespace mlmc
