// Host side of the C ABI declared in include/mlmc_darcy.h: context, device
// workspaces, the circulant-embedding cache, multigrid-PCG orchestration and
// the per-level estimator driver.  All arithmetic of the method runs in the
// kernels of field.hip, fv.hip and mg_pcg.hip; this file only validates
// arguments, sizes buffers and enqueues launches on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/mlmc_darcy.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace mlmc;

namespace {

struct CeEntry {
  int n = 0;
  FftPlan plan{};
  double2* tw = nullptr;
  double* sqT = nullptr;  // 2-D: sqrt(Lambda / n^2) transposed; 3-D: sqrt(Lambda / n^3)
};

struct Buffer {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// An instantiated graph of `check_every` PCG iterations of one solve
// configuration; `key` holds every value its launches depend on (sizes,
// options, buffer addresses and the workspace generation).
struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
constexpr size_t kGraphCache = 8;

struct ProfEvent {
  hipEvent_t a, b;
  double bytes;  // algorithmic bytes of the launch over the whole batch
  int iter;      // PCG iteration it belongs to (samples still active then do the
                 // work); 0: bytes already final
};

}  // namespace

struct mlmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::map<std::string, Buffer> ws;
  std::map<std::tuple<int, int, int, double, double, int>, CeEntry> ce;  // (dim, m, n, ...)
  void* host_pinned = nullptr;  // small pinned staging buffer
  std::string prof_name;
  double prof_scale = 1.0;  // share of the batch a launch works on (restart passes)
  int prof_iter = 0;        // PCG iteration of the launches being enqueued (0: n/a)
  // a solve ends with the true residual ||b - A x|| / ||b|| in relres; level
  // runs, which keep no residuals, turn it off (relres then holds the CG's
  // recursive residual at its last check)
  bool true_residual = true;
  std::vector<ProfEvent> prof;
  std::vector<hipEvent_t> event_pool;
  uint64_t ws_gen = 0;             // bumped whenever a workspace is (re)allocated
  hipStream_t capture_stream = nullptr;  // private stream graphs are captured on
  std::vector<GraphEntry> graphs;  // PCG iteration graphs, oldest first
  // mlmc_solve_noalloc: while `arena` is set, workspaces are carved from the
  // device's static scratch array (one region per name, 256-byte aligned)
  // instead of being allocated
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  std::map<std::string, std::pair<size_t, size_t>> arena_names;  // name -> (offset, bytes)
  // mlmc_run_levels: one sub-context per level (own stream, own workspaces)
  std::vector<mlmc_ctx*> subs;
  // 3-D level runs: sub-context the coarse companions are solved on
  mlmc_ctx* comp = nullptr;
  bool owns_stream = false;
};

namespace {

mlmc_status fail(mlmc_ctx* ctx, mlmc_status code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(ctx, MLMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)                          \
  do {                                     \
    mlmc_status s_ = (expr);               \
    if (s_ != MLMC_OK) return s_;          \
  } while (0)

#define CHECK_LAUNCH()                                                                 \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, MLMC_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

#define CHECK_LAUNCH_CTX(c)                                                            \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess)                                                              \
      return fail((c), MLMC_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

// Grow-only named device workspace.
mlmc_status ws_get(mlmc_ctx* ctx, const std::string& name, size_t bytes, void** out) {
  if (ctx->arena) {
    auto it = ctx->arena_names.find(name);
    if (it != ctx->arena_names.end()) {
      if (it->second.second < bytes)
        return fail(ctx, MLMC_EINVAL, "workspace '" + name + "' requested twice with a larger size");
      *out = ctx->arena + it->second.first;
      return MLMC_OK;
    }
    const size_t off = (ctx->arena_used + 255) & ~(size_t)255;
    if (off > ctx->arena_bytes || bytes > ctx->arena_bytes - off)
      return fail(ctx, MLMC_EINVAL,
                  "mlmc_solve_noalloc: the solve needs more than the " +
                      std::to_string(ctx->arena_bytes >> 20) +
                      " MiB scratch array (workspace '" + name + "' of " + std::to_string(bytes) +
                      " bytes at offset " + std::to_string(off) +
                      "); use a smaller batch or mlmc_solve");
    ctx->arena_names[name] = {off, bytes};
    ctx->arena_used = off + bytes;
    *out = ctx->arena + off;
    return MLMC_OK;
  }
  Buffer& b = ctx->ws[name];
  if (b.bytes < bytes) {
    // grow by at least half the current size (rounded to 64 KiB / 1 MiB), so
    // batches of slowly rising size reallocate rarely: a free waits for the device
    if (b.bytes > 0) bytes = std::max(bytes, b.bytes + b.bytes / 2);
    const size_t gran = bytes < ((size_t)16 << 20) ? ((size_t)64 << 10) : ((size_t)1 << 20);
    bytes = (bytes + gran - 1) & ~(gran - 1);
    if (b.ptr) {
      HIP_TRY(hipStreamSynchronize(ctx->stream));  // earlier launches may still use it
      HIP_TRY(hipFree(b.ptr));
    }
    b.ptr = nullptr;
    b.bytes = 0;
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, MLMC_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                        " bytes for workspace '" + name + "' failed");
    }
    b.ptr = p;
    b.bytes = bytes;
    ++ctx->ws_gen;
  }
  *out = b.ptr;
  return MLMC_OK;
}

template <class T>
mlmc_status ws(mlmc_ctx* ctx, const std::string& name, size_t count, T** out) {
  void* p = nullptr;
  TRY(ws_get(ctx, name, count * sizeof(T) + 256, &p));
  *out = static_cast<T*>(p);
  return MLMC_OK;
}

hipEvent_t pool_event(mlmc_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Brackets a launch with events when `name` is the profiled kernel.  Launches
// of a multigrid level pass `level`; the profiled name "<name>@<level>" then
// selects that level's launches only (level 0: the finest grid of a solve,
// a kernel instantiation of its own).
thread_local ArmedEvents t_armed;

// Kernels whose launches go through launch_k, timed by their own dispatch
// (the others are bracketed by events recorded on the stream around them).
bool stamped_by_launch(const char* name) {
  for (const char* k : {"k_mg_down", "k_mg_mid", "k_mg_up", "k_cg_direction_t", "k_axpy_dot",
                        "k_rbgs3"})
    if (std::strcmp(name, k) == 0) return true;
  return false;
}

template <class F>
void timed(mlmc_ctx* ctx, const char* name, double bytes, F&& launch, int level = -1,
           long long cells = -1) {
  bool hit = false;
  if (!ctx->prof_name.empty()) {
    // "<name>", "<name>@<level>" or "<name>@<level>#<cells of the launch's batch>"
    std::string p = ctx->prof_name;
    const size_t hash = p.find('#');
    bool grid_ok = true;
    if (hash != std::string::npos) {
      grid_ok = cells >= 0 && std::to_string(cells) == p.substr(hash + 1);
      p = p.substr(0, hash);
    }
    const size_t at = p.find('@');
    hit = grid_ok && (at == std::string::npos
                          ? p == name
                          : (p.compare(0, at, name) == 0 && std::strlen(name) == at &&
                             level >= 0 && std::to_string(level) == p.substr(at + 1)));
  }
  if (hit) {
    ProfEvent pe{pool_event(ctx), pool_event(ctx), bytes * ctx->prof_scale, ctx->prof_iter};
    if (stamped_by_launch(name)) {
      // the kernel's own launch stamps the events with its dispatch's start
      // and end (launch_k)
      armed_events() = ArmedEvents{pe.a, pe.b};
      launch();
      if (armed_events().start != nullptr) {  // not issued through launch_k
        armed_events() = ArmedEvents{};
        ctx->event_pool.push_back(pe.a);
        ctx->event_pool.push_back(pe.b);
        return;
      }
    } else {
      (void)hipEventRecord(pe.a, ctx->stream);
      launch();
      (void)hipEventRecord(pe.b, ctx->stream);
    }
    ctx->prof.push_back(pe);
  } else {
    launch();
  }
}

// Profiled launches of a PCG pass: the work of iteration it is done for the
// samples with iters >= it (converged or failed samples skip their work), so
// each launch's algorithmic bytes are scaled by that share of the batch.
mlmc_status scale_prof_by_active(mlmc_ctx* ctx, size_t prof_begin, const int32_t* iters,
                                 int batch) {
  if (ctx->prof.size() <= prof_begin) return MLMC_OK;
  std::vector<int32_t> hi(batch);
  HIP_TRY(hipMemcpyAsync(hi.data(), iters, batch * sizeof(int32_t), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  std::sort(hi.begin(), hi.end());
  for (size_t e = prof_begin; e < ctx->prof.size(); ++e) {
    ProfEvent& pe = ctx->prof[e];
    if (pe.iter <= 0) continue;
    const long long active = hi.end() - std::lower_bound(hi.begin(), hi.end(), pe.iter);
    pe.bytes *= (double)active / batch;
    pe.iter = 0;
  }
  return MLMC_OK;
}

bool five_smooth(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

// Stage order: the odd radices first.  A Stockham stage with span ns writes
// runs of ns consecutive elements at stride R ns, so a radix-4 stage at ns = 1
// stores with a stride of 8 dwords (8-way LDS bank conflicts on 64 banks),
// while radix 5 or 3 there strides by 10 or 6 dwords (2-way), and the even
// radices come once ns has grown.
FftPlan make_plan(int n) {
  FftPlan pl{};
  pl.n = n;
  int r = n;
  auto push = [&](int R) { pl.radix[pl.nstages++] = R; r /= R; };
  while (r % 5 == 0) push(5);
  while (r % 3 == 0) push(3);
  while (r % 4 == 0) push(4);
  while (r % 2 == 0) push(2);
  // the FP32 reciprocals div_small multiplies by, correctly rounded as the
  // device's FP32 division rounds them
  int ns = 1;
  for (int st = 0; st < pl.nstages; ++st) {
    pl.inv_nb[st] = 1.0f / (float)(n / pl.radix[st]);
    pl.inv_ns[st] = 1.0f / (float)ns;
    ns *= pl.radix[st];
  }
  return pl;
}

mlmc_status check_model(mlmc_ctx* ctx, const mlmc_model* mdl) {
  if (!mdl) return fail(ctx, MLMC_EINVAL, "model is NULL");
  if (mdl->dim != 2 && mdl->dim != 3) return fail(ctx, MLMC_EINVAL, "dim must be 2 or 3");
  const int k = mdl->interface_kind;
  if (k != MLMC_IFACE_HORIZONTAL && k != MLMC_IFACE_PIECEWISE_LINEAR &&
      k != MLMC_IFACE_PAPER_TWO_LINES && k != MLMC_IFACE_TILTED_PLANE && k != MLMC_IFACE_NONE)
    return fail(ctx, MLMC_EINVAL, "unknown interface_kind");
  if (k == MLMC_IFACE_PIECEWISE_LINEAR && (mdl->n_nodes < 2 || mdl->n_nodes > 8))
    return fail(ctx, MLMC_EINVAL, "n_nodes must be in [2, 8]");
  const int need = k == MLMC_IFACE_NONE ? 1 : (k == MLMC_IFACE_PAPER_TWO_LINES ? 3 : 2);
  if (mdl->n_layers != need)
    return fail(ctx, MLMC_EINVAL, "n_layers does not match the interface kind");
  for (int l = 0; l < mdl->n_layers; ++l)
    if (!(mdl->sigma2[l] >= 0.0) || !std::isfinite(mdl->mu[l]))
      return fail(ctx, MLMC_EINVAL, "layer parameters must be finite with sigma2 >= 0");
  if (mdl->field_kind == MLMC_FIELD_CORRELATED) {
    for (int l = 0; l < mdl->n_layers; ++l)
      if (!(mdl->lambda[l] > 0.0)) return fail(ctx, MLMC_EINVAL, "lambda must be positive");
    if (mdl->norm_r != 1 && mdl->norm_r != 2) return fail(ctx, MLMC_EINVAL, "norm_r must be 1 or 2");
  } else if (mdl->field_kind != MLMC_FIELD_PIECEWISE_CONSTANT) {
    return fail(ctx, MLMC_EINVAL, "unknown field_kind");
  }
  if (!(mdl->y_lo <= mdl->y_hi)) return fail(ctx, MLMC_EINVAL, "y_lo > y_hi");
  if (mdl->problem != MLMC_PROBLEM_OUTFLOW && mdl->problem != MLMC_PROBLEM_MEAN_PRESSURE)
    return fail(ctx, MLMC_EINVAL, "unknown problem");
  return MLMC_OK;
}

// Embedding eigenvalues for (m, n, sigma2, lambda, r); computed once, cached.
// With `check_only`, a failing embedding is reported but not cached.
mlmc_status ce_get(mlmc_ctx* ctx, int dim, int m, int n, double sigma2, double lambda, int r,
                   CeEntry** out) {
  auto key = std::make_tuple(dim, m, n, sigma2, lambda, r);
  auto it = ctx->ce.find(key);
  if (it != ctx->ce.end()) {
    *out = &it->second;
    return MLMC_OK;
  }
  if (n < 2 * m || n > kFftMax || !five_smooth(n))
    return fail(ctx, MLMC_EINVAL, "n_ce must satisfy 2m <= n_ce <= 4096 with factors 2, 3, 5");
  if (dim == 3 && n > kFftMax3)
    return fail(ctx, MLMC_EINVAL, "3-D n_ce must be <= " + std::to_string(kFftMax3));
  CeEntry e;
  e.n = n;
  e.plan = make_plan(n);
  const long long npts = dim == 3 ? (long long)n * n * n : (long long)n * n;
  HIP_TRY(hipMalloc(&e.tw, sizeof(double2) * n));
  HIP_TRY(hipMalloc(&e.sqT, sizeof(double) * (size_t)npts));
  double2* c = nullptr;
  TRY(ws(ctx, "ce_setup", (size_t)npts, &c));
  hipStream_t st = ctx->stream;
  launch_ce_twiddles(st, n, e.tw);
  if (dim == 3) {
    // Lambda = FFT3(c): along x1 (lines of n), x2 (per x3 slab) and x3
    launch_ce_first_row3(st, n, m, sigma2, lambda, r, c);
    launch_fft_lines(st, c, n, n * n, n, 1, e.tw, e.plan);
    for (int k3 = 0; k3 < n; ++k3)
      launch_fft_lines(st, c + (long long)k3 * n * n, n, n, 1, n, e.tw, e.plan);
    launch_fft_lines(st, c, n, n * n, 1, (long long)n * n, e.tw, e.plan);
  } else {
    launch_ce_first_row(st, n, m, sigma2, lambda, r, c);
    launch_fft_lines(st, c, n, n, n, 1, e.tw, e.plan);   // along x1 (rows)
    launch_fft_lines(st, c, n, n, 1, n, e.tw, e.plan);   // along x2 (columns)
  }
  const int nb = 256;
  double* part = nullptr;
  TRY(ws(ctx, "ce_minmax", 2 * nb, &part));
  launch_ce_minmax(st, c, npts, part, nb);
  CHECK_LAUNCH();
  std::vector<double> h(2 * nb);
  HIP_TRY(hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double lo = h[0], hi = h[1];
  for (int b = 1; b < nb; ++b) {
    lo = std::fmin(lo, h[2 * b]);
    hi = std::fmax(hi, h[2 * b + 1]);
  }
  if (!(hi > 0.0) || lo < -1e-12 * hi) {
    (void)hipFree(e.tw);
    (void)hipFree(e.sqT);
    char buf[200];
    snprintf(buf, sizeof buf,
             "circulant embedding n_ce = %d for m = %d is not non-negative (min/max = %.3e)", n, m,
             hi > 0 ? lo / hi : 0.0);
    return fail(ctx, MLMC_EEMBED, buf);
  }
  if (dim == 3) launch_ce_sqrt3(st, c, n, e.sqT);
  else launch_ce_sqrt_transpose(st, c, n, e.sqT);
  CHECK_LAUNCH();
  auto res = ctx->ce.emplace(key, e);
  *out = &res.first->second;
  return MLMC_OK;
}

mlmc_status check_opts(mlmc_ctx* ctx, const mlmc_solver_opts* o) {
  if (!o) return fail(ctx, MLMC_EINVAL, "opts is NULL");
  if (!(o->tol > 0.0)) return fail(ctx, MLMC_EINVAL, "tol must be positive");
  if (o->maxit < 1) return fail(ctx, MLMC_EINVAL, "maxit must be >= 1");
  if (o->nu1 < 1 || o->nu1 != o->nu2)
    return fail(ctx, MLMC_EINVAL, "nu1 == nu2 >= 1 is required for a symmetric preconditioner");
  if (o->coarse_max < 1) return fail(ctx, MLMC_EINVAL, "coarse_max must be >= 1");
  if (!(o->omega > 0.0)) return fail(ctx, MLMC_EINVAL, "omega must be positive");
  if (o->precision < MLMC_PREC_FP64 || o->precision > MLMC_PREC_BF16)
    return fail(ctx, MLMC_EINVAL, "unknown precision");
  if (o->cycle_max < 0 || o->cycle_max == 1 || o->cycle_max > kCoarseCycleMax)
    return fail(ctx, MLMC_EINVAL, "cycle_max must be 0 or in [2, 32]");
  if (o->gamma < 1 || o->gamma > 2) return fail(ctx, MLMC_EINVAL, "gamma must be 1 or 2");
  if (o->gamma_levels < 0) return fail(ctx, MLMC_EINVAL, "gamma_levels must be >= 0");
  if (o->graph != 0 && o->graph != 1) return fail(ctx, MLMC_EINVAL, "graph must be 0 or 1");
  if (o->initial_guess != 0 && o->initial_guess != 1)
    return fail(ctx, MLMC_EINVAL, "initial_guess must be 0 or 1");
  if (o->tile_shape != 0 && o->tile_shape != 1)
    return fail(ctx, MLMC_EINVAL, "tile_shape must be 0 or 1");
  if (o->variant < 0 || o->variant > 2) return fail(ctx, MLMC_EINVAL, "variant must be 0, 1 or 2");
  return MLMC_OK;
}

std::string lv(const char* base, int l) { return std::string(base) + std::to_string(l); }

// Algorithmic bytes (FP64) per cell for the launches timed by mlmc_profile_*.
constexpr double kBytesRbgs = 28.0;       // T (16) + own r (4) + other-colour z (4) + own z (4)
constexpr double kBytesRbgsZero = 24.0;   // T (16) + own r (4) + own z write (4)
constexpr double kBytesSpmv = 32.0;       // T (16) + p (8) + q write (8)
constexpr double kBytesAxpy = 48.0;       // x, r, p, q read + x, r write
constexpr double kBytesResRes = 34.0;     // T 16 + z 8 + r 8 + rc write 2
constexpr double kBytesProlong = 18.0;    // z read + write 16 + zc 2

}  // namespace

// ======================================================= scratch of mlmc_solve_noalloc
// The device memory of the allocation-free solve: a file-scope array in the
// code object, one copy per device, held until the process ends.  Host code
// never passes `scratch` itself (its host-side name is not a device address):
// mlmc_ctx_create looks up the array's address on its device once with
// hipGetSymbolAddress and every later use goes through that pointer.
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxScratchDevices = 64;
void* g_scratch_ptr[kMaxScratchDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
// Address of this device's scratch array (the device is current); looked up once.
hipError_t scratch_setup(int device) {
  if (device >= kMaxScratchDevices) return hipSuccess;  // noalloc unavailable there
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch_ptr[device] = ptr;
  return e;
}
}  // namespace

// =================================================================== public ABI
namespace mlmc {
// Error message for the host-side drivers of other source files.
mlmc_status set_error(mlmc_ctx* ctx, mlmc_status code, const char* msg) {
  return fail(ctx, code, msg);
}

// This host thread's event pair for the next launch_k (kernels.hpp).
ArmedEvents& armed_events() { return t_armed; }
}  // namespace mlmc

extern "C" {

mlmc_status mlmc_ctx_create(int device, void* hip_stream, mlmc_ctx** out) {
  mlmc_ctx* ctx = nullptr;
  if (!out) return MLMC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MLMC_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return MLMC_EDEVICE;
  if (scratch_setup(device) != hipSuccess) {
    (void)hipGetLastError();
    return MLMC_EDEVICE;
  }
  ctx = new mlmc_ctx();
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (hipHostMalloc(&ctx->host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return MLMC_ENOMEM;
  }
  *out = ctx;
  return MLMC_OK;
}

mlmc_status mlmc_ctx_destroy(mlmc_ctx* ctx) {
  if (!ctx) return MLMC_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->ws)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  for (auto& kv : ctx->ce) {
    (void)hipFree(kv.second.tw);
    (void)hipFree(kv.second.sqT);
  }
  for (auto& pe : ctx->prof) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  for (auto& g : ctx->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  for (mlmc_ctx* sub : ctx->subs) (void)mlmc_ctx_destroy(sub);
  if (ctx->comp) (void)mlmc_ctx_destroy(ctx->comp);
  if (ctx->owns_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return MLMC_OK;
}

mlmc_status mlmc_ctx_set_stream(mlmc_ctx* ctx, void* hip_stream) {
  if (!ctx) return MLMC_EINVAL;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return MLMC_OK;
}

const char* mlmc_last_error(const mlmc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

mlmc_status mlmc_solver_opts_default(mlmc_solver_opts* o) {
  if (!o) return MLMC_EINVAL;
  std::memset(o, 0, sizeof *o);
  o->tol = 1e-13;
  o->omega = 1.9;
  o->maxit = 200;
  o->nu1 = 1;
  o->nu2 = 1;
  o->coarse_max = 4;
  o->check_every = 4;
  o->gamma = 2;
  o->gamma_levels = 2;
  o->graph = 0;
  o->initial_guess = 0;
  o->tile_shape = 0;
  return MLMC_OK;
}

// Embedding samples of a correlated model: layer l, in order, takes the
// imaginary part of the first earlier sample with its own (sigma2, lambda)
// whose imaginary part is free, else starts a new sample (real part); sample p
// draws its noise from stream tag 2 + p.  Returns the number of samples.
static int ce_pairs(const mlmc_model* mdl, CePair* pr) {
  int np = 0;
  for (int l = 0; l < mdl->n_layers; ++l) {
    int q = 0;
    for (; q < np; ++q)
      if (pr[q].l_im < 0 && mdl->sigma2[pr[q].l_re] == mdl->sigma2[l] &&
          mdl->lambda[pr[q].l_re] == mdl->lambda[l])
        break;
    if (q < np) {
      pr[q].l_im = l;
      pr[q].mu_im = mdl->mu[l];
    } else {
      pr[np] = CePair{kTagNoise + (uint32_t)np, l, -1, mdl->mu[l], 0.0};
      ++np;
    }
  }
  return np;
}

mlmc_status mlmc_ce_min_embedding(mlmc_ctx* ctx, const mlmc_model* model, int m, int* n_ce_out) {
  if (!ctx || !n_ce_out) return MLMC_EINVAL;
  TRY(check_model(ctx, model));
  if (m < 1) return fail(ctx, MLMC_EINVAL, "m must be positive");
  (void)hipSetDevice(ctx->device);
  const int n_max = model->dim == 3 ? kFftMax3 : kFftMax;
  CePair pr[4];
  const int np = ce_pairs(model, pr);
  for (int n = 2 * m; n <= n_max; ++n) {
    if (!five_smooth(n)) continue;
    // the smallest size that embeds every pair's covariance
    mlmc_status s = MLMC_OK;
    for (int q = 0; q < np && s == MLMC_OK; ++q) {
      CeEntry* e = nullptr;
      const int l = pr[q].l_re;
      s = ce_get(ctx, model->dim, m, n, model->sigma2[l], model->lambda[l], model->norm_r, &e);
    }
    if (s == MLMC_OK) {
      *n_ce_out = n;
      ctx->err.clear();
      return MLMC_OK;
    }
    if (s != MLMC_EEMBED) return s;
  }
  return fail(ctx, MLMC_EEMBED,
              "no valid circulant embedding with n_ce <= " + std::to_string(n_max));
}

static mlmc_status sample_field_impl(mlmc_ctx* ctx, const mlmc_model* model, int m, int level,
                                     uint64_t first_sample, const uint32_t* ids, int batch,
                                     double* k, double* k_coarse) {
  if (!ctx) return MLMC_EINVAL;
  TRY(check_model(ctx, model));
  if (m < 1 || batch < 0 || level < 0 || !k) return fail(ctx, MLMC_EINVAL, "bad m/batch/level/k");
  if (k_coarse && (m % 2)) return fail(ctx, MLMC_EINVAL, "k_coarse needs an even m");
  if (!ids && first_sample + (uint64_t)batch > (1ull << 32))
    return fail(ctx, MLMC_EINVAL, "sample numbers must fit in 32 bits");
  if (batch == 0) return MLMC_OK;
  (void)hipSetDevice(ctx->device);
  hipStream_t st = ctx->stream;
  double* params = nullptr;
  TRY(ws(ctx, "params", (size_t)batch * kParamStride, &params));
  launch_sample_params(st, *model, level, first_sample, ids, batch, params);
  if (model->field_kind == MLMC_FIELD_PIECEWISE_CONSTANT) {
    if (model->dim == 3) {
      launch_field_pc3(st, *model, m, batch, params, k);
      if (k_coarse) launch_field_pc3(st, *model, m / 2, batch, params, k_coarse);
    } else {
      launch_field_pc(st, *model, m, batch, params, k);
      if (k_coarse) launch_field_pc(st, *model, m / 2, batch, params, k_coarse);
    }
    CHECK_LAUNCH();
    return MLMC_OK;
  }
  CePair pr[4];
  const int np = ce_pairs(model, pr);
  for (int q = 0; q < np; ++q) {
    CeEntry* e = nullptr;
    const int l = pr[q].l_re;
    TRY(ce_get(ctx, model->dim, m, model->n_ce, model->sigma2[l], model->lambda[l], model->norm_r,
               &e));
    if (model->dim == 3) {
      const int nn = e->n;
      double2 *u1 = nullptr, *u2 = nullptr;
      TRY(ws(ctx, "ce3_u1", (size_t)batch * nn * nn * m, &u1));
      TRY(ws(ctx, "ce3_u2", (size_t)batch * nn * m * m, &u2));
      launch_ce3(st, *model, pr[q], level, first_sample, ids, batch, m, e->sqT, e->tw, e->plan,
                 params, u1, u2, k, k_coarse);
      continue;
    }
    double2* uT = nullptr;
    TRY(ws(ctx, "ce_uT", (size_t)batch * m * e->n, &uT));
    const double cells = (double)batch * m * m;
    const double ratio = (double)e->n / m;
    // bytes of pass B: its reads of uT and its writes of k, which the pairs
    // split between them (every cell is written once over all pairs)
    const double kshare = 1.0 / np;
    timed(ctx, "k_ce_pass_a", cells * (16.0 * ratio + 8.0 * ratio * ratio), [&] {
      launch_ce_pass_a(st, *model, pr[q], level, first_sample, ids, batch, m, e->sqT, e->tw,
                       e->plan, uT);
    });
    timed(ctx, "k_ce_pass_b", cells * (16.0 * ratio + kshare * (8.0 + (k_coarse ? 2.0 : 0.0))),
          [&] {
            launch_ce_pass_b(st, *model, pr[q], batch, m, uT, e->tw, e->plan, params, k,
                             k_coarse);
          });
  }
  CHECK_LAUNCH();
  return MLMC_OK;
}

mlmc_status mlmc_sample_field(mlmc_ctx* ctx, const mlmc_model* model, int m, int level,
                              uint64_t first_sample, int batch, double* k, double* k_coarse) {
  return sample_field_impl(ctx, model, m, level, first_sample, nullptr, batch, k, k_coarse);
}

mlmc_status mlmc_sample_field_ids(mlmc_ctx* ctx, const mlmc_model* model, int m, int level,
                                  const uint32_t* sample_ids, int batch, double* k,
                                  double* k_coarse) {
  if (!sample_ids && batch > 0) return fail(ctx, MLMC_EINVAL, "sample_ids is NULL");
  return sample_field_impl(ctx, model, m, level, 0, sample_ids, batch, k, k_coarse);
}

mlmc_status mlmc_cgv_extract(mlmc_ctx* ctx, int dim, int m, int batch, const double* k_fine,
                             double* k_sub) {
  if (!ctx) return MLMC_EINVAL;
  if (dim != 2 && dim != 3) return fail(ctx, MLMC_EINVAL, "dim must be 2 or 3");
  if (m < 2 || (m % 2) || batch < 0 || !k_fine || !k_sub)
    return fail(ctx, MLMC_EINVAL, "bad arguments to mlmc_cgv_extract");
  if (batch == 0) return MLMC_OK;
  (void)hipSetDevice(ctx->device);
  if (dim == 3) launch_cgv_extract3(ctx->stream, m, batch, k_fine, k_sub);
  else launch_cgv_extract(ctx->stream, m, batch, k_fine, k_sub);
  CHECK_LAUNCH();
  return MLMC_OK;
}

mlmc_status mlmc_assemble_problem(mlmc_ctx* ctx, int problem, int dim, int m, int batch,
                                  const double* k, double* T, double* tb, double* b) {
  if (!ctx) return MLMC_EINVAL;
  if (dim != 2 && dim != 3) return fail(ctx, MLMC_EINVAL, "dim must be 2 or 3");
  if (problem != MLMC_PROBLEM_OUTFLOW && problem != MLMC_PROBLEM_MEAN_PRESSURE)
    return fail(ctx, MLMC_EINVAL, "unknown problem");
  if (m < 1 || batch < 0 || !k || !T || !tb || !b)
    return fail(ctx, MLMC_EINVAL, "bad arguments to mlmc_assemble");
  if (batch == 0) return MLMC_OK;
  (void)hipSetDevice(ctx->device);
  if (dim == 3) {
    launch_assemble3(ctx->stream, problem, m, batch, k, T, tb, b);
    CHECK_LAUNCH();
    return MLMC_OK;
  }
  timed(ctx, "k_assemble", (double)batch * m * m * 40.0,
        [&] { launch_assemble(ctx->stream, problem, m, batch, k, T, tb, b); });
  CHECK_LAUNCH();
  return MLMC_OK;
}

mlmc_status mlmc_assemble(mlmc_ctx* ctx, int dim, int m, int batch, const double* k, double* T,
                          double* tb, double* b) {
  return mlmc_assemble_problem(ctx, MLMC_PROBLEM_OUTFLOW, dim, m, batch, k, T, tb, b);
}

mlmc_status mlmc_qoi_box_mean(mlmc_ctx* ctx, int dim, int m, int batch, const double* p,
                              double lo, double hi, double* q) {
  if (!ctx) return MLMC_EINVAL;
  if (dim != 2 && dim != 3) return fail(ctx, MLMC_EINVAL, "dim must be 2 or 3");
  if (m < 1 || batch < 0 || !p || !q || !(lo >= 0.0) || !(hi <= 1.0) || !(lo < hi))
    return fail(ctx, MLMC_EINVAL, "bad arguments to mlmc_qoi_box_mean");
  if (batch == 0) return MLMC_OK;
  (void)hipSetDevice(ctx->device);
  launch_qoi_box(ctx->stream, dim, m, batch, lo, hi, p, q);
  CHECK_LAUNCH();
  return MLMC_OK;
}

// D* of Model Problem 1 in the level runs: the centred box of side 1/8.
constexpr double kMp1Lo = 0.5 - 1.0 / 16.0, kMp1Hi = 0.5 + 1.0 / 16.0;

// The QoI of the model's problem for a solved batch.
static mlmc_status model_qoi(mlmc_ctx* ctx, const mlmc_model* model, int dim, int m, int batch,
                             const double* k, const double* p, double* q) {
  if (model->problem == MLMC_PROBLEM_MEAN_PRESSURE)
    return mlmc_qoi_box_mean(ctx, dim, m, batch, p, kMp1Lo, kMp1Hi, q);
  return mlmc_qoi_outflow(ctx, dim, m, batch, k, p, q, nullptr);
}

mlmc_status mlmc_qoi_outflow(mlmc_ctx* ctx, int dim, int m, int batch, const double* k,
                             const double* p, double* q_out, double* q_in) {
  if (!ctx) return MLMC_EINVAL;
  if (dim != 2 && dim != 3) return fail(ctx, MLMC_EINVAL, "dim must be 2 or 3");
  if (m < 1 || batch < 0 || !k || !p || !q_out)
    return fail(ctx, MLMC_EINVAL, "bad arguments to mlmc_qoi_outflow");
  if (batch == 0) return MLMC_OK;
  (void)hipSetDevice(ctx->device);
  if (dim == 3) {
    double* part = nullptr;
    TRY(ws(ctx, "qoi3_parts", qoi3_parts_size(batch), &part));
    launch_qoi3(ctx->stream, m, batch, k, p, part, q_out, q_in);
  } else {
    launch_qoi(ctx->stream, m, batch, k, p, q_out, q_in);
  }
  CHECK_LAUNCH();
  return MLMC_OK;
}

// 3-D solve: PCG with the one-launch-per-sweep multigrid cycle (V, or W on the
// opts->gamma_levels finest levels), FP64; same per-sample scalars, convergence
// checks and W breakdown restart as in 2-D.
static mlmc_status solve3_impl(mlmc_ctx* ctx, int m, int batch, const double* T, const double* tb,
                               const double* b, double* p, const mlmc_solver_opts* opts,
                               int32_t* status, int32_t* iters, double* relres) {
  hipStream_t st = ctx->stream;
  if (opts->precision == MLMC_PREC_BF16)
    return fail(ctx, MLMC_EINVAL, "the 3-D multigrid hierarchy is FP64 or FP32");
  // FP32: the hierarchy (operators, z and r below the finest level) in float
  // inside a flexible FP64 CG, as in 2-D; the coarsest inverse stays FP64.
  const bool f32 = opts->precision == MLMC_PREC_FP32;
  std::vector<int> ms{m};
  while (ms.back() % 2 == 0 && ms.back() > opts->coarse_max) ms.push_back(ms.back() / 2);
  const int L = (int)ms.size() - 1;
  if (ms[L] > 4)
    return fail(ctx, MLMC_EINVAL, "coarsest 3-D grid " + std::to_string(ms[L]) +
                                      " > 4: m must be c * 2^k with c <= 4");
  const long long n = (long long)m * m * m;
  const int bps = blocks_per_sample(n);
  double *r, *z, *pv, *q, *partial;
  TRY(ws(ctx, "s3_r", batch * n, &r));
  TRY(ws(ctx, "s3_z", batch * n, &z));
  TRY(ws(ctx, "s3_p", batch * n, &pv));
  TRY(ws(ctx, "s3_q", batch * n, &q));
  TRY(ws(ctx, "s3_partial", (size_t)batch * bps, &partial));
  std::vector<const double*> Tl(L + 1), tbl(L + 1);
  std::vector<double*> zl(L + 1), rl(L + 1);
  Tl[0] = T;
  tbl[0] = tb;
  zl[0] = z;
  rl[0] = r;
  std::vector<double*> Tw(L + 1, nullptr), tbw(L + 1, nullptr);
  for (int l = 1; l <= L; ++l) {
    const long long nl = (long long)ms[l] * ms[l] * ms[l];
    TRY(ws(ctx, lv("s3_T", l), batch * 3 * nl, &Tw[l]));
    TRY(ws(ctx, lv("s3_tb", l), (size_t)batch * 3 * ms[l] * ms[l], &tbw[l]));
    TRY(ws(ctx, lv("s3_zl", l), batch * nl, &zl[l]));
    TRY(ws(ctx, lv("s3_rl", l), batch * nl, &rl[l]));
    Tl[l] = Tw[l];
    tbl[l] = tbw[l];
  }
  const int nc = ms[L] * ms[L] * ms[L];
  double* Ainv = nullptr;
  TRY(ws(ctx, "s3_ainv", (size_t)batch * nc * nc, &Ainv));
  const int nu = opts->nu1;
  // levels from the first one of side <= 8 (FP64) or 16 (FP32) down run in one
  // in-LDS kernel (nu = 1; variant 1 keeps the per-sweep launches on every level)
  int l0 = -1;
  if (nu == 1 && opts->variant != 1)
    for (int l = 0; l < L; ++l)
      if (ms[l] <= coarse3_max_side(f32)) {
        l0 = l;
        break;
      }
  // the levels above the in-LDS (or else the dense coarsest) one are swept per
  // launch and keep their faces, z and r in colour-split order; so does the CG
  // when the finest level is one of them (its x is put back in natural order
  // at the end)
  const int lsplit = l0 >= 0 ? l0 : L;
  auto split = [&](int l) { return l < lsplit; };
  // the operators and vectors the cycle works on, in the hierarchy's type
  // (the faces of a split level: a colour-split copy)
  std::vector<const void*> Th(L + 1), tbh(L + 1);
  std::vector<void*> zh(L + 1), rh(L + 1);
  for (int l = 0; l <= L; ++l) {
    const long long nl = (long long)ms[l] * ms[l] * ms[l];
    const long long fl = (long long)ms[l] * ms[l];
    if (!f32) {
      Th[l] = Tl[l];
      if (split(l)) {
        double* Tcs = nullptr;
        TRY(ws(ctx, lv("s3_Tcs", l), batch * 3 * nl, &Tcs));
        Th[l] = Tcs;
      }
      tbh[l] = tbl[l];
      zh[l] = zl[l];
      rh[l] = rl[l];
      continue;
    }
    void *Tf, *tbf;
    TRY(ws_get(ctx, lv("s3_Tf", l), (size_t)batch * 3 * nl * sizeof(float) + 256, &Tf));
    TRY(ws_get(ctx, lv("s3_tbf", l), (size_t)batch * 3 * fl * sizeof(float) + 256, &tbf));
    Th[l] = Tf;
    tbh[l] = tbf;
    if (l == 0) {
      zh[0] = z;
      rh[0] = r;
    } else {
      TRY(ws_get(ctx, lv("s3_zf", l), (size_t)batch * nl * sizeof(float) + 256, &zh[l]));
      TRY(ws_get(ctx, lv("s3_rf", l), (size_t)batch * nl * sizeof(float) + 256, &rh[l]));
    }
  }
  double* partial2 = nullptr;
  if (f32) TRY(ws(ctx, "s3_partial2", (size_t)batch * bps, &partial2));
  SolverState S;
  TRY(ws(ctx, "s3_r0", batch, &S.r0sq));
  TRY(ws(ctx, "s3_rho", batch, &S.rho));
  TRY(ws(ctx, "s3_alpha", batch, &S.alpha));
  TRY(ws(ctx, "s3_beta", batch, &S.beta));
  TRY(ws(ctx, "s3_active", batch, &S.active));
  TRY(ws(ctx, "s3_count", 1, &S.count));
  int32_t* carried = nullptr;  // iterations of a W pass whose sample restarts with V
  if (opts->gamma == 2) TRY(ws(ctx, "s3_carried", batch, &carried));
  const double omega = opts->omega;
  int cur_gamma = opts->gamma;
  auto visits = [&](int l) {
    return (opts->gamma_levels == 0 || l < opts->gamma_levels) ? cur_gamma : 1;
  };
  CoarseDesc cdesc{};
  void* cimg = nullptr;  // padded operator image of the in-LDS levels
  if (l0 >= 0) {
    for (int q2 = 0; l0 + q2 <= L; ++q2) {
      cdesc.m[q2] = ms[l0 + q2];
      cdesc.T[q2] = Th[l0 + q2];
      cdesc.tb[q2] = tbh[l0 + q2];
    }
    const size_t words = (size_t)coarse3_image_words(L - l0 + 1, cdesc.m);
    TRY(ws_get(ctx, "s3_cimg", (size_t)batch * words * (f32 ? sizeof(float) : sizeof(double)),
               &cimg));
  }
  // every workspace is in hand: the hierarchy's set-up launches
  for (int l = 1; l <= L; ++l)
    launch_coarsen3(st, ms[l - 1], batch, Tl[l - 1], tbl[l - 1], Tw[l], tbw[l]);
  launch_dense_factor3(st, ms[L], batch, Tl[L], tbl[L], Ainv);
  for (int l = 0; l <= L; ++l) {
    const long long nl = (long long)ms[l] * ms[l] * ms[l];
    const long long fl = (long long)ms[l] * ms[l];
    if (split(l)) launch_faces_split3(st, f32, ms[l], batch, Tl[l], const_cast<void*>(Th[l]));
    else if (f32)
      launch_convert(st, MLMC_PREC_FP32, batch * 3 * nl, Tl[l], const_cast<void*>(Th[l]));
    if (f32)
      launch_convert(st, MLMC_PREC_FP32, batch * 3 * fl, tbl[l], const_cast<void*>(tbh[l]));
  }
  if (l0 >= 0) launch_coarse3_image(st, f32, batch, L - l0 + 1, cdesc, cimg);
  CHECK_LAUNCH();
  std::function<void(int)> cycle = [&](int l) {
    if (l == l0) {
      unsigned wmask = 0;
      for (int q2 = 0; l0 + q2 < L; ++q2)
        if (visits(l0 + q2) == 2) wmask |= 1u << q2;
      launch_coarse3_cycle(st, f32, l0 == 0, batch, L - l0 + 1, cdesc, cimg, rh[l0], zh[l0], Ainv,
                           omega, wmask, S.active);
      return;
    }
    if (l == L) {
      if (f32 && L > 0)
        launch_dense_apply3f(st, nc, batch, Ainv, (const float*)rh[L], (float*)zh[L], S.active);
      else launch_dense_apply_n(st, nc, batch, Ainv, rl[L], zl[L], S.active);
      return;
    }
    const int ml = ms[l];
    const bool top = l == 0;
    // algorithmic bytes of a half-sweep per cell: every face once (3 S), r of
    // the swept colour, the other colour's z read and the swept colour's z
    // written (V each, half the cells); from zero no z is read
    const double cells = (double)batch * ml * ml * ml;
    const double sb = f32 ? 4.0 : 8.0, vb = (top || !f32) ? 8.0 : 4.0;
    auto sweep = [&](int color, int zero) {
      timed(ctx, "k_rbgs3", cells * (3.0 * sb + (zero ? 1.0 : 1.5) * vb), [&] {
        launch_rbgs3_p(st, f32, top, ml, batch, Th[l], tbh[l], zh[l], rh[l], S.active, color,
                       zero);
      }, l);
    };
    for (int it = 0; it < nu; ++it) {
      sweep(0, it == 0);
      sweep(1, 0);
    }
    for (int visit = 0; visit < visits(l); ++visit) {
      // a later visit's pre-smoothing starts with the red half-sweep that
      // ended the post-smoothing before it: the red values depend only on the
      // (unchanged) black ones, so it would rewrite them bit for bit, and is
      // skipped
      if (visit > 0)
        for (int it = 0; it < nu; ++it) {
          if (it > 0) sweep(0, 0);
          sweep(1, 0);
        }
      launch_resid_restrict3_p(st, f32, top, ml, batch, Th[l], tbh[l], zh[l], rh[l], rh[l + 1],
                               S.active, split(l + 1));
      cycle(l + 1);
      // the prolongation rides on the first (black) half-sweep of post-smoothing
      launch_prolong_black3_p(st, f32, top, ml, batch, Th[l], tbh[l], zh[l], rh[l], zh[l + 1],
                              omega, S.active, split(l + 1));
      sweep(0, 0);
      for (int it = 1; it < nu; ++it) {
        sweep(1, 0);
        sweep(0, 0);
      }
    }
  };
  auto precond = [&]() {
    cycle(0);
    launch_dot(st, (int)n, batch, r, z, partial, bps, S.active);
  };
  int32_t* hcount = static_cast<int32_t*>(ctx->host_pinned);
  const int check = opts->check_every > 0 ? opts->check_every : 1;
  auto pcg_pass = [&](bool restart) -> mlmc_status {
    if (split(0))
      launch_pcg_init3_split(st, m, batch, b, p, r, partial, bps, restart ? S.active : nullptr);
    else
      launch_pcg_init(st, (int)n, batch, b, p, r, partial, bps, restart ? S.active : nullptr);
    launch_sc_init(st, batch, partial, bps, S, status, iters, relres, restart ? 1 : 0);
    ctx->prof_iter = restart ? 0 : 1;
    precond();
    launch_sc_rho(st, batch, partial, bps, S, status, 1, nullptr, 0);
    launch_pupdate(st, (int)n, batch, pv, z, S.beta, bps, S.active, 1);
    CHECK_LAUNCH();
    for (int it = 1;; ++it) {
      // the operator reads the caller's faces with its cells taken in natural
      // order (the colour-split face copy, read in colour-split order, fetched
      // every face line twice)
      launch_spmv3_dot(st, m, batch, T, tb, pv, q, partial, bps, S.active, split(0));
      launch_sc_alpha(st, batch, partial, bps, S, status);
      // flexible form with a reduced-precision cycle: also r_new . z_old
      launch_axpy_dot(st, (int)n, batch, p, r, pv, q, S.alpha, partial, bps, S.active,
                      f32 ? z : nullptr, partial2);
      launch_sc_conv(st, batch, partial, bps, S, status, iters, relres, opts->tol, opts->maxit);
      CHECK_LAUNCH();
      if (it % check == 0 || it >= opts->maxit) {
        HIP_TRY(hipMemcpyAsync(hcount, S.count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (*hcount == 0) break;
      }
      ctx->prof_iter = restart ? 0 : it + 1;
      precond();
      launch_sc_rho(st, batch, partial, bps, S, status, 0, partial2, f32 ? bps : 0);
      launch_pupdate(st, (int)n, batch, pv, z, S.beta, bps, S.active, 0);
    }
    return MLMC_OK;
  };
  const size_t prof_begin = ctx->prof.size();
  TRY(pcg_pass(false));
  ctx->prof_iter = 0;
  TRY(scale_prof_by_active(ctx, prof_begin, iters, batch));
  if (cur_gamma == 2) {  // V-cycle restart where the W preconditioner broke down
    launch_sc_restart(st, batch, S, status, iters, carried);
    HIP_TRY(hipMemcpyAsync(hcount, S.count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (*hcount > 0) {
      cur_gamma = 1;
      ctx->prof_scale = (double)*hcount / batch;
      const mlmc_status rc = pcg_pass(true);
      ctx->prof_scale = 1.0;
      TRY(rc);
      launch_iters_add(st, batch, iters, carried);
    }
  }
  if (split(0)) {  // x back to natural order, through z
    launch_from_split3(st, m, batch, p, z);
    HIP_TRY(hipMemcpyAsync(p, z, (size_t)batch * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  if (ctx->true_residual) {
    launch_true_residual3(st, m, batch, T, tb, b, p, partial, bps);
    launch_sc_final(st, batch, partial, bps, S, relres);
  }
  CHECK_LAUNCH();
  return MLMC_OK;
}

mlmc_status mlmc_solve(mlmc_ctx* ctx, int dim, int m, int batch, const double* T,
                       const double* tb, const double* b, double* p,
                       const mlmc_solver_opts* opts, int32_t* status, int32_t* iters,
                       double* relres) {
  if (!ctx) return MLMC_EINVAL;
  if (dim != 2 && dim != 3) return fail(ctx, MLMC_EINVAL, "dim must be 2 or 3");
  TRY(check_opts(ctx, opts));
  if (m < 1 || batch < 0 || !T || !tb || !b || !p || !status || !iters || !relres)
    return fail(ctx, MLMC_EINVAL, "bad arguments to mlmc_solve");
  if (batch == 0) return MLMC_OK;
  (void)hipSetDevice(ctx->device);
  if (dim == 3) return solve3_impl(ctx, m, batch, T, tb, b, p, opts, status, iters, relres);
  hipStream_t st = ctx->stream;

  // grid hierarchy: halve while even and above coarse_max
  std::vector<int> ms{m};
  while (ms.back() % 2 == 0 && ms.back() > opts->coarse_max) ms.push_back(ms.back() / 2);
  const int L = (int)ms.size() - 1;
  if (ms[L] > 8)
    return fail(ctx, MLMC_EINVAL, "coarsest grid " + std::to_string(ms[L]) +
                                      " > 8: m must be c * 2^k with c <= 8");
  const long long n = (long long)m * m;
  const int bps = blocks_per_sample(n);
  const int prec = opts->precision;
  const bool fused = (opts->variant == 0 || opts->variant == 2) && opts->nu1 == 1;
  if (prec != MLMC_PREC_FP64 && !fused)
    return fail(ctx, MLMC_EINVAL, "reduced-precision multigrid needs variant 0 and nu1 = nu2 = 1");

  // 64 x 64: the whole solve of a sample in one workgroup (same hierarchy and
  // cycle; the vectors never leave the CU).  It computes in FP64 at every
  // precision setting: a reduced-precision hierarchy would save no memory
  // traffic here, whose only HBM traffic is T, b in and p out.
  if (opts->variant == 0 && opts->nu1 == 1 && m == 64 && L == 4) {
    OcHierarchy h{};
    h.T[0] = T;
    h.tb[0] = tb;
    double* Tw[5] = {};
    double* tbw[5] = {};
    for (int l = 1; l <= L; ++l) {
      const long long nl = (long long)ms[l] * ms[l];
      TRY(ws(ctx, lv("s_T", l), batch * 2 * nl, &Tw[l]));
      TRY(ws(ctx, lv("s_tb", l), (size_t)batch * 2 * ms[l], &tbw[l]));
      h.T[l] = Tw[l];
      h.tb[l] = tbw[l];
    }
    double *work = nullptr, *Ainv = nullptr;
    TRY(ws(ctx, "s_chol", (size_t)batch * 256, &work));
    TRY(ws(ctx, "s_ainv", (size_t)batch * 256, &Ainv));
    // every workspace is in hand before the first launch
    for (int l = 1; l <= L; ++l)
      launch_coarsen(st, ms[l - 1], batch, h.T[l - 1], h.tb[l - 1], Tw[l], tbw[l]);
    launch_dense_factor(st, 4, batch, h.T[L], h.tb[L], work, Ainv);
    // compulsory bytes per sample: T and tb of every level, b, x, the inverse
    const double bytes = (double)batch * (8.0 * (2.0 * 5456 + 2.0 * 124) + 16.0 * n + 8.0 * 256);
    timed(ctx, "k_pcg_onchip64", bytes, [&] {
      launch_pcg_onchip64(st, batch, h, b, p, Ainv, opts->tol, opts->maxit, opts->omega,
                          opts->gamma, opts->gamma_levels, status, iters, relres);
    });
    CHECK_LAUNCH();
    return MLMC_OK;
  }
  const bool flexible = prec != MLMC_PREC_FP64;
  const size_t eb = prec_bytes(prec);

  // FP64 hierarchy (Galerkin coarsening, coarsest inverse) ...
  std::vector<const double*> Tl(L + 1), tbl(L + 1);
  std::vector<double*> zl(L + 1), rl(L + 1);
  Tl[0] = T;
  tbl[0] = tb;
  double *r, *z, *pv, *q, *partial, *partial2 = nullptr;
  TRY(ws(ctx, "s_r", batch * n, &r));
  TRY(ws(ctx, "s_z", batch * n, &z));
  TRY(ws(ctx, "s_p", batch * n, &pv));
  TRY(ws(ctx, "s_q", batch * n, &q));
  const int parts_max =
      std::max({bps, mg_rz_parts(m % 2 == 0 ? m : 2, prec, opts->tile_shape), m % 64 == 0 ? cg_dir_parts(m) : 1});
  TRY(ws(ctx, "s_partial", (size_t)batch * parts_max, &partial));
  if (flexible) TRY(ws(ctx, "s_partial2", (size_t)batch * bps, &partial2));
  zl[0] = z;
  rl[0] = r;
  std::vector<double*> Tw(L + 1, nullptr), tbw(L + 1, nullptr);
  for (int l = 1; l <= L; ++l) {
    const long long nl = (long long)ms[l] * ms[l];
    TRY(ws(ctx, lv("s_T", l), batch * 2 * nl, &Tw[l]));
    TRY(ws(ctx, lv("s_tb", l), (size_t)batch * 2 * ms[l], &tbw[l]));
    if (!fused || prec == MLMC_PREC_FP64) {
      TRY(ws(ctx, lv("s_zl", l), batch * nl, &zl[l]));
      TRY(ws(ctx, lv("s_rl", l), batch * nl, &rl[l]));
    }
    Tl[l] = Tw[l];
    tbl[l] = tbw[l];
  }
  const long long nc = (long long)ms[L] * ms[L];
  double *work = nullptr, *Ainv = nullptr;
  TRY(ws(ctx, "s_chol", batch * nc * nc, &work));
  TRY(ws(ctx, "s_ainv", batch * nc * nc, &Ainv));

  // ... and, for reduced precision, its copy in the storage type.  Vectors of
  // the fused cycle below the finest level (z_l, r_l, z_pre) use that type.
  std::vector<const void*> Ts(L + 1), tbs(L + 1);
  std::vector<void*> zs(L + 1), rs(L + 1), zpre(L + 1, nullptr);
  zs[0] = z;
  rs[0] = r;
  for (int l = 0; l <= L; ++l) {
    const long long nl = (long long)ms[l] * ms[l];
    if (prec == MLMC_PREC_FP64) {
      Ts[l] = Tl[l];
      tbs[l] = tbl[l];
    } else {
      void *Tc, *tbc;
      TRY(ws_get(ctx, lv("s_Tlo", l), batch * 2 * nl * eb + 256, &Tc));
      TRY(ws_get(ctx, lv("s_tblo", l), (size_t)batch * 2 * ms[l] * eb + 256, &tbc));
      Ts[l] = Tc;
      tbs[l] = tbc;
    }
    if (l >= 1) {
      if (prec == MLMC_PREC_FP64) {
        zs[l] = zl[l];
        rs[l] = rl[l];
      } else {
        TRY(ws_get(ctx, lv("s_zlo", l), batch * nl * eb + 256, &zs[l]));
        TRY(ws_get(ctx, lv("s_rlo", l), batch * nl * eb + 256, &rs[l]));
      }
    }
  }

  SolverState S;
  TRY(ws(ctx, "s_r0", batch, &S.r0sq));
  TRY(ws(ctx, "s_rho", batch, &S.rho));
  TRY(ws(ctx, "s_alpha", batch, &S.alpha));
  TRY(ws(ctx, "s_beta", batch, &S.beta));
  TRY(ws(ctx, "s_active", batch, &S.active));
  TRY(ws(ctx, "s_count", 1, &S.count));
  int32_t* carried = nullptr;  // iterations of a W pass whose sample restarts with V
  if (opts->gamma == 2) TRY(ws(ctx, "s_carried", batch, &carried));

  const int nu = opts->nu1;
  const double omega = opts->omega;
  const double cells0 = (double)batch * n;

  // Fused cycle: tiled down/mid/up kernels above level l0, one workgroup per
  // sample for levels l0..L (sizes <= kCoarseCycleMax).
  int l0 = L;
  CoarseDesc cdesc{};
  std::vector<void*> zmid(L + 1, nullptr);  // W-cycle: z after the second visit's pre-smoothing
  // coarse-grid visits of level l (W on the finest levels only, by default)
  int cur_gamma = opts->gamma;
  auto visits = [&](int l) {
    return (opts->gamma_levels == 0 || l < opts->gamma_levels) ? cur_gamma : 1;
  };
  if (fused) {
    l0 = 0;
    const int cmax = opts->cycle_max > 0 ? opts->cycle_max : kCoarseCycleMax;
    while (l0 < L && (ms[l0] > cmax || L - l0 + 1 > kMaxCoarseLevels)) ++l0;
    for (int l = 0; l < l0; ++l) {
      TRY(ws_get(ctx, lv("s_zpre", l), batch * (size_t)ms[l] * ms[l] * eb + 256, &zpre[l]));
      if (visits(l) == 2)
        TRY(ws_get(ctx, lv("s_zmid", l), batch * (size_t)ms[l] * ms[l] * eb + 256, &zmid[l]));
    }
  }
  // CG direction: fused p-update + operator (ping-pong p buffers) when the
  // finest grid takes fixed tiles, else separate p-update and operator kernels
  const bool dir_fused = fused && cg_direction_fused(m);
  double* pbuf[2] = {pv, nullptr};
  if (dir_fused) TRY(ws(ctx, "s_p2", batch * n, &pbuf[1]));
  const int dir_parts = dir_fused ? cg_dir_parts(m) : bps;

  // every workspace is in hand: the hierarchy's set-up launches
  for (int l = 1; l <= L; ++l)
    launch_coarsen(st, ms[l - 1], batch, Tl[l - 1], tbl[l - 1], Tw[l], tbw[l]);
  launch_dense_factor(st, ms[L], batch, Tl[L], tbl[L], work, Ainv);
  if (prec != MLMC_PREC_FP64)
    for (int l = 0; l <= L; ++l) {
      const long long nl = (long long)ms[l] * ms[l];
      launch_convert(st, prec, batch * 2 * nl, Tl[l], const_cast<void*>(Ts[l]));
      launch_convert(st, prec, (long long)batch * 2 * ms[l], tbl[l], const_cast<void*>(tbs[l]));
    }
  CHECK_LAUNCH();
  if (fused) {
    for (int q2 = 0; q2 + l0 <= L; ++q2) {
      cdesc.m[q2] = ms[l0 + q2];
      cdesc.T[q2] = Ts[l0 + q2];
      cdesc.tb[q2] = tbs[l0 + q2];
    }
  }
  const int ncl = L - l0 + 1;
  // algorithmic bytes of the launches (for mlmc_profile_*)
  const double ebd = (double)eb;
  double coarse_bytes = 0.0;
  for (int l = l0; l <= L; ++l) coarse_bytes += 2.0 * ebd * ms[l] * ms[l];
  coarse_bytes = batch * (coarse_bytes + (l0 == 0 ? 16.0 : 2.0 * ebd) * ms[l0] * ms[l0] +
                          8.0 * nc * nc);

  std::function<void(int)> vcycle_unfused = [&](int l) {
    if (l == L) {
      timed(ctx, "k_dense_apply", batch * (8.0 * nc * nc + 16.0 * nc),
            [&] { launch_dense_apply(st, ms[L], batch, Ainv, rl[L], zl[L], S.active); });
      return;
    }
    const int ml = ms[l];
    const double cells = (double)batch * ml * ml;
    for (int it = 0; it < nu; ++it) {
      timed(ctx, "k_rbgs", cells * (it == 0 ? kBytesRbgsZero : kBytesRbgs), [&] {
        launch_rbgs(st, ml, batch, Tl[l], tbl[l], zl[l], rl[l], S.active, 0, it == 0);
      });
      timed(ctx, "k_rbgs", cells * kBytesRbgs, [&] {
        launch_rbgs(st, ml, batch, Tl[l], tbl[l], zl[l], rl[l], S.active, 1, 0);
      });
    }
    for (int visit = 0; visit < visits(l); ++visit) {
      if (visit > 0) {
        for (int it = 0; it < nu; ++it) {
          timed(ctx, "k_rbgs", cells * kBytesRbgs, [&] {
            launch_rbgs(st, ml, batch, Tl[l], tbl[l], zl[l], rl[l], S.active, 0, 0);
          });
          timed(ctx, "k_rbgs", cells * kBytesRbgs, [&] {
            launch_rbgs(st, ml, batch, Tl[l], tbl[l], zl[l], rl[l], S.active, 1, 0);
          });
        }
      }
      timed(ctx, "k_resid_restrict", cells * kBytesResRes, [&] {
        launch_resid_restrict(st, ml, batch, Tl[l], tbl[l], zl[l], rl[l], rl[l + 1], S.active);
      });
      vcycle_unfused(l + 1);
      timed(ctx, "k_prolong", cells * kBytesProlong,
            [&] { launch_prolong(st, ml, batch, zl[l + 1], zl[l], omega, S.active); });
      for (int it = 0; it < nu; ++it) {
        timed(ctx, "k_rbgs", cells * kBytesRbgs, [&] {
          launch_rbgs(st, ml, batch, Tl[l], tbl[l], zl[l], rl[l], S.active, 1, 0);
        });
        timed(ctx, "k_rbgs", cells * kBytesRbgs, [&] {
          launch_rbgs(st, ml, batch, Tl[l], tbl[l], zl[l], rl[l], S.active, 0, 0);
        });
      }
    }
  };
  // z = M r, and the partials of r^T z: rz_parts per sample in `partial`
  int rz_parts = bps;
  if (fused) rz_parts = l0 == 0 ? 1 : mg_rz_parts(ms[0], prec, opts->tile_shape);
  // Fused gamma-cycle: on a tiled level l, the down kernel pre-smooths and
  // restricts; after the first coarse visit the mid kernel adds the correction,
  // post- and pre-smooths and restricts again; the up kernel adds the last
  // correction and post-smooths.  Levels l0..L run in the in-LDS kernel.
  // A 64^2 level below the finest (with 32, 16, 8, 4 under it) runs its whole
  // sub-cycle in one workgroup per sample (FP64, variant 0).
  int l64 = -1;
  OcHierarchy h64{};
  if (fused && opts->variant == 0 && prec == MLMC_PREC_FP64 && L >= 5 && ms[L - 4] == 64 &&
      ms[L] == 4) {
    l64 = L - 4;
    for (int q2 = 0; q2 <= 4; ++q2) {
      h64.T[q2] = Tl[l64 + q2];
      h64.tb[q2] = tbl[l64 + q2];
    }
  }
  std::function<void(int)> fcycle = [&](int l) {
    if (l == l64) {
      unsigned wmask = 0;
      for (int q2 = 0; q2 < 4; ++q2)
        if (visits(l + q2) == 2) wmask |= 1u << q2;
      // T, tb and r read once, z written once per sample (FP64)
      const double bytes = (double)batch * (8.0 * (2.0 * 5456 + 2.0 * 124) + 16.0 * 4096 + 2048.0);
      timed(ctx, "k_cycle_onchip64", bytes, [&] {
        launch_cycle_onchip64(st, batch, h64, static_cast<const double*>(rs[l]),
                              static_cast<double*>(zs[l]), Ainv, omega, wmask, S.active);
      });
      return;
    }
    if (l == l0) {
      unsigned wmask = 0;
      for (int q2 = 0; l0 + q2 < L; ++q2)
        if (visits(l0 + q2) == 2) wmask |= 1u << q2;
      timed(ctx, "k_mg_coarse_cycle", coarse_bytes, [&] {
        launch_mg_coarse_cycle(st, prec, l0 == 0, batch, ncl, cdesc, rs[l0], zs[l0], Ainv, omega,
                               wmask, S.active, l0 == 0 ? partial : nullptr);
      });
      return;
    }
    const double cells = (double)batch * ms[l] * ms[l];
    const double rb = l == 0 ? 8.0 : ebd;  // r (FP64 on the finest level)
    // T 2 words, r, z_pre write, coarse r write (1/4 word)
    timed(ctx, "k_mg_down", cells * (ebd * 3.25 + rb), [&] {
      launch_mg_down(st, prec, opts->tile_shape, l == 0, ms[l], batch, Ts[l], tbs[l], rs[l], zpre[l], rs[l + 1],
                     S.active);
    }, l, (long long)batch * ms[l] * ms[l]);
    fcycle(l + 1);
    const void* zin = zpre[l];
    if (visits(l) == 2) {
      // T 2 words, r, z_pre, coarse z (1/4), z write, coarse r write (1/4)
      timed(ctx, "k_mg_mid", cells * (ebd * 4.5 + rb), [&] {
        launch_mg_mid(st, prec, opts->tile_shape, l == 0, ms[l], batch, Ts[l], tbs[l], rs[l], zpre[l], zmid[l],
                      zs[l + 1], omega, rs[l + 1], S.active);
      }, l, (long long)batch * ms[l] * ms[l]);
      fcycle(l + 1);
      zin = zmid[l];
    }
    // T 2 words, r and z (FP64 on the finest level), z_in, coarse z (1/4 word)
    timed(ctx, "k_mg_up", cells * (ebd * 3.25 + (l == 0 ? 16.0 : 2.0 * ebd)), [&] {
      launch_mg_up(st, prec, opts->tile_shape, l == 0, ms[l], batch, Ts[l], tbs[l], rs[l], zin, zs[l], zs[l + 1],
                   omega, S.active, l == 0 ? partial : nullptr);
    }, l, (long long)batch * ms[l] * ms[l]);
  };
  auto vcycle = [&]() {
    if (!fused) {
      vcycle_unfused(0);
      launch_dot(st, (int)n, batch, r, z, partial, bps, S.active);
      return;
    }
    fcycle(0);
  };

  int32_t* hcount = static_cast<int32_t*>(ctx->host_pinned);
  const int check = opts->check_every > 0 ? opts->check_every : 1;
  // Graph form (opts->graph): after the first host check the iterations run
  // as replays of one captured graph of `check` iterations, a host check after
  // each replay.  The captured launches are those of the eager loop, in the
  // same order and with the same arguments (the ping-pong p buffers repeat
  // with the chunk when `check` is even), so the results are bitwise equal.
  // Not with profiling (its events are per launch) nor on restart passes.
  const bool use_graph = opts->graph != 0 && dir_fused && ctx->prof_name.empty() && check % 2 == 0;
  auto chunk_body = [&](int k0) {
    for (int it = k0 + 1; it <= k0 + check; ++it) {
      vcycle();
      launch_sc_rho(st, batch, partial, rz_parts, S, status, 0, partial2, bps);
      pv = pbuf[it & 1];
      launch_cg_direction(st, m, batch, T, tb, z, pbuf[(it - 1) & 1], pv, q, S.beta, false,
                          partial, S.active);
      launch_sc_alpha(st, batch, partial, dir_parts, S, status);
      launch_axpy_dot(st, (int)n, batch, p, r, pv, q, S.alpha, partial, bps, S.active,
                      flexible ? z : nullptr, partial2);
      launch_sc_conv(st, batch, partial, bps, S, status, iters, relres, opts->tol, opts->maxit);
    }
  };
  auto graph_chunks = [&](int k) -> mlmc_status {
    auto bits = [](double v) {
      uint64_t u;
      std::memcpy(&u, &v, sizeof u);
      return u;
    };
    const std::vector<uint64_t> key = {
        ctx->ws_gen, (uint64_t)m, (uint64_t)batch, (uint64_t)prec, bits(omega), bits(opts->tol),
        (uint64_t)opts->maxit, (uint64_t)cur_gamma, (uint64_t)opts->gamma_levels,
        (uint64_t)check, (uint64_t)opts->cycle_max, (uint64_t)opts->coarse_max,
        (uint64_t)(uintptr_t)T, (uint64_t)(uintptr_t)tb, (uint64_t)(uintptr_t)b,
        (uint64_t)(uintptr_t)p, (uint64_t)(uintptr_t)status, (uint64_t)(uintptr_t)iters,
        (uint64_t)(uintptr_t)relres};
    hipGraphExec_t exec = nullptr;
    for (auto& g : ctx->graphs)
      if (g.key == key) exec = g.exec;
    if (!exec) {
      GraphEntry g;
      g.key = key;
      // capture on the context's own capture stream (the caller's stream may be
      // the null stream, which cannot capture); the launches record, not run
      if (!ctx->capture_stream)
        HIP_TRY(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
      const hipStream_t run_st = st;
      st = ctx->capture_stream;
      const hipError_t be = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
      if (be != hipSuccess) {
        st = run_st;
        return fail(ctx, MLMC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(be));
      }
      chunk_body(k);
      const hipError_t le = hipGetLastError();
      const hipError_t ce = hipStreamEndCapture(st, &g.graph);
      st = run_st;
      if (le != hipSuccess || ce != hipSuccess) {
        if (g.graph) (void)hipGraphDestroy(g.graph);
        return fail(ctx, MLMC_EDEVICE, std::string("graph capture: ") +
                                           hipGetErrorString(le != hipSuccess ? le : ce));
      }
      if (hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g.graph);
        return fail(ctx, MLMC_EDEVICE, "graph instantiation failed");
      }
      if (ctx->graphs.size() >= kGraphCache) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        (void)hipGraphDestroy(ctx->graphs.front().graph);
        ctx->graphs.erase(ctx->graphs.begin());
      }
      ctx->graphs.push_back(g);
      exec = g.exec;
    }
    // every sample stops by maxit (marked not converged), so the count reaches 0
    for (; k < opts->maxit + check; k += check) {
      HIP_TRY(hipGraphLaunch(exec, st));
      HIP_TRY(hipMemcpyAsync(hcount, S.count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (*hcount == 0) break;
    }
    pv = pbuf[(k + check) & 1];
    return MLMC_OK;
  };
  // One PCG pass over the active samples (all of them, or with `restart` the
  // ones marked by launch_sc_restart), x0 = 0.
  auto pcg_pass = [&](bool restart) -> mlmc_status {
    // a restart pass starts its samples from zero
    if (!restart && opts->initial_guess)
      launch_pcg_init_guess(st, m, batch, T, tb, b, p, r, partial, bps);
    else launch_pcg_init(st, (int)n, batch, b, p, r, partial, bps, restart ? S.active : nullptr);
    launch_sc_init(st, batch, partial, bps, S, status, iters, relres, restart ? 1 : 0);
    ctx->prof_iter = restart ? 0 : 1;
    vcycle();
    launch_sc_rho(st, batch, partial, rz_parts, S, status, 1, nullptr, 0);
    if (!dir_fused) launch_pupdate(st, (int)n, batch, pv, z, S.beta, bps, S.active, 1);
    CHECK_LAUNCH();
    for (int it = 1;; ++it) {
      ctx->prof_iter = restart ? 0 : it;
      if (dir_fused) {
        // iteration it writes p into pbuf[it % 2] from pbuf[(it - 1) % 2]
        pv = pbuf[it & 1];
        timed(ctx, "k_cg_direction_t", cells0 * 48.0, [&] {
          launch_cg_direction(st, m, batch, T, tb, z, pbuf[(it - 1) & 1], pv, q, S.beta, it == 1,
                              partial, S.active);
        });
      } else {
        timed(ctx, "k_spmv_dot", cells0 * kBytesSpmv, [&] {
          launch_spmv_dot(st, m, batch, T, tb, pv, q, partial, bps, S.active);
        });
      }
      launch_sc_alpha(st, batch, partial, dir_parts, S, status);
      timed(ctx, "k_axpy_dot", cells0 * (kBytesAxpy + (flexible ? 8.0 : 0.0)), [&] {
        launch_axpy_dot(st, (int)n, batch, p, r, pv, q, S.alpha, partial, bps, S.active,
                        flexible ? z : nullptr, partial2);
      });
      launch_sc_conv(st, batch, partial, bps, S, status, iters, relres, opts->tol, opts->maxit);
      CHECK_LAUNCH();
      if (it % check == 0 || it >= opts->maxit) {
        HIP_TRY(hipMemcpyAsync(hcount, S.count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (*hcount == 0) break;
        if (use_graph && !restart && it % check == 0) return graph_chunks(it);
      }
      ctx->prof_iter = restart ? 0 : it + 1;
      vcycle();
      launch_sc_rho(st, batch, partial, rz_parts, S, status, 0, partial2, bps);
      if (!dir_fused) launch_pupdate(st, (int)n, batch, pv, z, S.beta, bps, S.active, 0);
    }
    return MLMC_OK;
  };
  const size_t prof_begin = ctx->prof.size();
  TRY(pcg_pass(false));
  ctx->prof_iter = 0;
  TRY(scale_prof_by_active(ctx, prof_begin, iters, batch));
  // The W-cycle preconditioner is symmetric but, with over-corrected coarse
  // steps, not positive definite for every operator (two coarse visits act as
  // 2B - BAB, indefinite once B A has an eigenvalue above 2); a sample whose
  // W-preconditioned iteration breaks down (r^T z <= 0) is solved again from
  // x0 = 0 with the V-cycle, positive definite for any omega > 0.  Its
  // iteration count includes both passes.
  if (cur_gamma == 2) {
    launch_sc_restart(st, batch, S, status, iters, carried);
    HIP_TRY(hipMemcpyAsync(hcount, S.count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (*hcount > 0) {
      cur_gamma = 1;
      ctx->prof_scale = (double)*hcount / batch;
      const mlmc_status rc = pcg_pass(true);
      ctx->prof_scale = 1.0;
      TRY(rc);
      launch_iters_add(st, batch, iters, carried);
    }
  }
  if (ctx->true_residual) {
    launch_true_residual(st, m, batch, T, tb, b, p, partial, bps);
    launch_sc_final(st, batch, partial, bps, S, relres);
  }
  CHECK_LAUNCH();
  return MLMC_OK;
}

mlmc_status mlmc_solve_noalloc(mlmc_ctx* ctx, int dim, int m, int batch, const double* T,
                               const double* tb, const double* b, double* p,
                               const mlmc_solver_opts* opts, int32_t* status, int32_t* iters,
                               double* relres) {
  if (!ctx) return MLMC_EINVAL;
  if (opts && opts->graph)
    return fail(ctx, MLMC_EINVAL, "mlmc_solve_noalloc: opts->graph = 1 needs a capture stream "
                                  "and graph objects; use graph = 0");
  void* base = ctx->device < kMaxScratchDevices ? g_scratch_ptr[ctx->device] : nullptr;
  if (!base) return fail(ctx, MLMC_EDEVICE, "mlmc_solve_noalloc: no scratch array on this device");
  ctx->arena = static_cast<char*>(base);
  ctx->arena_bytes = kScratchBytes;
  ctx->arena_used = 0;
  ctx->arena_names.clear();
  std::string prof;
  prof.swap(ctx->prof_name);  // kernel timing would create events: off for this call
  const mlmc_status rc = mlmc_solve(ctx, dim, m, batch, T, tb, b, p, opts, status, iters, relres);
  prof.swap(ctx->prof_name);
  ctx->arena = nullptr;
  ctx->arena_bytes = ctx->arena_used = 0;
  ctx->arena_names.clear();
  return rc;
}

// Turns a context's end-of-solve true residual off for its lifetime (level
// runs keep no residuals) and restores the setting on every return path.
struct NoTrueResidual {
  mlmc_ctx* c;
  bool old;
  explicit NoTrueResidual(mlmc_ctx* cc) : c(cc), old(cc->true_residual) { c->true_residual = false; }
  ~NoTrueResidual() { c->true_residual = old; }
};

static mlmc_status level_run_impl(mlmc_ctx* ctx, const mlmc_model* model, int level, int m_fine,
                                  uint64_t first_sample, const uint32_t* ids, int n, int cgv,
                                  const mlmc_solver_opts* opts, mlmc_level_sums* sums, double* q_f,
                                  double* q_c, double* y, int32_t* failed_out,
                                  int32_t* iters_out) {
  if (!ctx) return MLMC_EINVAL;
  TRY(check_model(ctx, model));
  TRY(check_opts(ctx, opts));
  if (!sums || n < 0 || level < 0 || m_fine < 1)
    return fail(ctx, MLMC_EINVAL, "bad arguments to mlmc_level_run");
  if (level > 0 && (m_fine % 2)) return fail(ctx, MLMC_EINVAL, "level >= 1 needs an even m_fine");
  if (n == 0) return MLMC_OK;
  (void)hipSetDevice(ctx->device);
  const NoTrueResidual no_true_residual(ctx);
  hipStream_t st = ctx->stream;
  const int m = m_fine, mc = m / 2, d = model->dim;
  const long long nf = d == 3 ? (long long)m * m * m : (long long)m * m;
  const long long ncl = d == 3 ? (long long)mc * mc * mc : (long long)mc * mc;
  const long long fface = d == 3 ? (long long)m * m : m;     // boundary faces per side
  const long long cface = d == 3 ? (long long)mc * mc : mc;
  const int ncomp = level == 0 ? 0 : (cgv ? (1 << d) : 1);

  double *k, *T, *tb, *b, *p, *qf, *yv, *relres, *out;
  int32_t *stf, *itf, *failed;
  TRY(ws(ctx, "lr_k", n * nf, &k));
  TRY(ws(ctx, "lr_T", n * d * nf, &T));
  TRY(ws(ctx, "lr_tb", (size_t)n * d * fface, &tb));
  TRY(ws(ctx, "lr_b", n * nf, &b));
  TRY(ws(ctx, "lr_p", n * nf, &p));
  TRY(ws(ctx, "lr_qf", n, &qf));
  TRY(ws(ctx, "lr_y", n, &yv));
  TRY(ws(ctx, "lr_relres", (size_t)n * (ncomp > 0 ? ncomp : 1), &relres));
  TRY(ws(ctx, "lr_stf", n, &stf));
  TRY(ws(ctx, "lr_itf", n, &itf));
  TRY(ws(ctx, "lr_failed", n, &failed));
  TRY(ws(ctx, "lr_out", 8, &out));

  double* kc = nullptr;
  if (ncomp > 0) TRY(ws(ctx, "lr_kc", (size_t)n * ncomp * ncl, &kc));
  TRY(sample_field_impl(ctx, model, m, level, first_sample, ids, n, k,
                        (ncomp == 1) ? kc : nullptr));
  if (ncomp > 1) TRY(mlmc_cgv_extract(ctx, d, m, n, k, kc));

  // In 2-D the companions are solved first and the fine solve starts from the
  // solution of each sample's first companion, injected to the fine cells
  // (about one CG iteration fewer; same stopping rule ||r||/||b|| < tol).  In
  // 3-D the fine solve starts from zero, so the companions (assembly, solve,
  // QoI) run beside it on a sub-context of their own (own stream, workspaces
  // and host thread): the coarse grid's latency-bound launches fill the
  // device while the fine grid's run.  The kernels and their inputs are the
  // same either way, so are the results, bit for bit.
  mlmc_solver_opts zero_guess = *opts;
  zero_guess.initial_guess = 0;
  double* qcv = nullptr;
  double* pc = nullptr;
  int32_t *stc = nullptr, *itc = nullptr;
  const bool beside = d == 3 && ncomp > 0;
  std::thread comp_thread;
  mlmc_status comp_rc = MLMC_OK;
  hipEvent_t comp_start = nullptr, comp_done = nullptr;
  if (ncomp > 0) {
    const int nb = n * ncomp;
    double *Tc, *tbc, *bc, *qcomp, *relres_c;
    TRY(ws(ctx, "lr_Tc", (size_t)nb * d * ncl, &Tc));
    TRY(ws(ctx, "lr_tbc", (size_t)nb * d * cface, &tbc));
    TRY(ws(ctx, "lr_bc", (size_t)nb * ncl, &bc));
    TRY(ws(ctx, "lr_pc", (size_t)nb * ncl, &pc));
    TRY(ws(ctx, "lr_qcomp", nb, &qcomp));
    TRY(ws(ctx, "lr_qc", n, &qcv));
    TRY(ws(ctx, "lr_stc", nb, &stc));
    TRY(ws(ctx, "lr_itc", nb, &itc));
    TRY(ws(ctx, "lr_relres_c", nb, &relres_c));
    auto companions = [=, &zero_guess](mlmc_ctx* cc) -> mlmc_status {
      const NoTrueResidual no_true_residual_c(cc);
      TRY(mlmc_assemble_problem(cc, model->problem, d, mc, nb, kc, Tc, tbc, bc));
      TRY(mlmc_solve(cc, d, mc, nb, Tc, tbc, bc, pc, &zero_guess, stc, itc, relres_c));
      TRY(model_qoi(cc, model, d, mc, nb, kc, pc, qcomp));
      launch_cgv_average(cc->stream, n, ncomp, qcomp, qcv);
      CHECK_LAUNCH_CTX(cc);
      return MLMC_OK;
    };
    if (beside) {
      if (!ctx->comp) {
        hipStream_t cst = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&cst, hipStreamNonBlocking));
        const mlmc_status rc = mlmc_ctx_create(ctx->device, cst, &ctx->comp);
        if (rc != MLMC_OK) {
          (void)hipStreamDestroy(cst);
          return fail(ctx, rc, "could not create the companion context");
        }
        ctx->comp->owns_stream = true;
      }
      mlmc_ctx* cc = ctx->comp;
      comp_start = pool_event(ctx);
      comp_done = pool_event(ctx);
      HIP_TRY(hipEventRecord(comp_start, st));  // k and the companions' k are sampled
      HIP_TRY(hipStreamWaitEvent(cc->stream, comp_start, 0));
      mlmc_status* rc_out = &comp_rc;
      const hipEvent_t done = comp_done;
      comp_thread = std::thread([companions, cc, rc_out, done] {
        (void)hipSetDevice(cc->device);
        mlmc_status rc = companions(cc);
        if (rc == MLMC_OK && hipEventRecord(done, cc->stream) != hipSuccess)
          rc = fail(cc, MLMC_EDEVICE, "hipEventRecord failed");
        *rc_out = rc;
      });
    } else {
      TRY(companions(ctx));
    }
  }
  // joins the companion thread on every path out of here, then returns the
  // events to the pool
  struct Joiner {
    std::thread& t;
    mlmc_ctx* ctx;
    hipEvent_t a, b;
    ~Joiner() {
      if (t.joinable()) t.join();
      if (a) ctx->event_pool.push_back(a);
      if (b) ctx->event_pool.push_back(b);
    }
  } joiner{comp_thread, ctx, comp_start, comp_done};
  TRY(mlmc_assemble_problem(ctx, model->problem, d, m, n, k, T, tb, b));
  mlmc_solver_opts fine = zero_guess;
  if (d == 2 && ncomp > 0) {
    launch_inject(st, m, n, ncomp, pc, p);
    fine.initial_guess = 1;
  }
  TRY(mlmc_solve(ctx, d, m, n, T, tb, b, p, &fine, stf, itf, relres));
  TRY(model_qoi(ctx, model, d, m, n, k, p, qf));
  if (beside) {
    comp_thread.join();
    if (comp_rc != MLMC_OK)
      return fail(ctx, comp_rc, std::string("companion solves: ") + mlmc_last_error(ctx->comp));
    HIP_TRY(hipStreamWaitEvent(st, comp_done, 0));
  }
  launch_y_and_fail(st, n, qf, qcv, stf, stc, ncomp, yv, failed);
  launch_level_reduce(st, n, yv, qf, qcv, failed, itf, itc, ncomp, out);
  if (q_f) HIP_TRY(hipMemcpyAsync(q_f, qf, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  if (q_c) {
    if (qcv) HIP_TRY(hipMemcpyAsync(q_c, qcv, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    else HIP_TRY(hipMemsetAsync(q_c, 0, sizeof(double) * n, st));
  }
  if (y) HIP_TRY(hipMemcpyAsync(y, yv, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  if (failed_out)
    HIP_TRY(hipMemcpyAsync(failed_out, failed, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  if (iters_out)
    HIP_TRY(hipMemcpyAsync(iters_out, itf, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  CHECK_LAUNCH();
  double* h = static_cast<double*>(ctx->host_pinned);
  HIP_TRY(hipMemcpyAsync(h, out, sizeof(double) * 7, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  sums->n += n;
  sums->sum_y += h[0];
  sums->sum_y2 += h[1];
  sums->sum_qf += h[2];
  sums->sum_qc += h[3];
  sums->n_failed += (int64_t)llround(h[4]);
  sums->iters_fine += (int64_t)llround(h[5]);
  sums->iters_coarse += (int64_t)llround(h[6]);
  if (h[4] > 0.5) return fail(ctx, MLMC_ENOCONV, "some solves did not reach the tolerance");
  return MLMC_OK;
}

mlmc_status mlmc_level_run(mlmc_ctx* ctx, const mlmc_model* model, int level, int m_fine,
                           uint64_t first_sample, int n, int cgv, const mlmc_solver_opts* opts,
                           mlmc_level_sums* sums, double* q_f, double* q_c, double* y) {
  return level_run_impl(ctx, model, level, m_fine, first_sample, nullptr, n, cgv, opts, sums, q_f,
                        q_c, y, nullptr, nullptr);
}

mlmc_status mlmc_level_run_ids(mlmc_ctx* ctx, const mlmc_model* model, int level, int m_fine,
                               const uint32_t* sample_ids, int n, int cgv,
                               const mlmc_solver_opts* opts, mlmc_level_sums* sums, double* q_f,
                               double* q_c, double* y, int32_t* failed, int32_t* iters) {
  if (!sample_ids && n > 0) return fail(ctx, MLMC_EINVAL, "sample_ids is NULL");
  return level_run_impl(ctx, model, level, m_fine, 0, sample_ids, n, cgv, opts, sums, q_f, q_c, y,
                        failed, iters);
}

mlmc_status mlmc_run_levels(mlmc_ctx* ctx, const mlmc_model* model, int n_levels,
                            const int* m_fine, const int* n_ce, const uint64_t* first_sample,
                            const int* n, int cgv, const mlmc_solver_opts* opts,
                            mlmc_level_sums* sums) {
  if (!ctx) return MLMC_EINVAL;
  TRY(check_model(ctx, model));
  if (n_levels < 1 || n_levels > 16 || !m_fine || !first_sample || !n || !opts || !sums)
    return fail(ctx, MLMC_EINVAL, "bad arguments to mlmc_run_levels");
  for (int l = 0; l < n_levels; ++l) {
    TRY(check_opts(ctx, &opts[l]));
    if (m_fine[l] < 1 || n[l] < 0 || (l > 0 && m_fine[l] % 2))
      return fail(ctx, MLMC_EINVAL, "bad level size or sample count");
  }
  (void)hipSetDevice(ctx->device);
  // One sub-context per level, each with its own stream and workspaces (kept
  // for later calls), so the levels' pipelines -- sampling, companion solves,
  // fine solve, QoI, reduction -- run concurrently: one level's latency-bound
  // coarse-grid and on-chip launches overlap another's bandwidth-bound
  // fine-grid launches.  Each level runs exactly mlmc_level_run's steps, so its
  // sums are bitwise those of a level run over the same samples.
  while ((int)ctx->subs.size() < n_levels) {
    hipStream_t sst = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&sst, hipStreamNonBlocking));
    mlmc_ctx* sub = nullptr;
    const mlmc_status rc = mlmc_ctx_create(ctx->device, sst, &sub);
    if (rc != MLMC_OK) {
      (void)hipStreamDestroy(sst);
      return fail(ctx, rc, "mlmc_run_levels: could not create a level context");
    }
    sub->owns_stream = true;
    ctx->subs.push_back(sub);
  }
  // the levels start after the work already on the caller's stream
  hipEvent_t start = pool_event(ctx);
  HIP_TRY(hipEventRecord(start, ctx->stream));
  for (int l = 0; l < n_levels; ++l) HIP_TRY(hipStreamWaitEvent(ctx->subs[l]->stream, start, 0));
  std::vector<mlmc_status> rc(n_levels, MLMC_OK);
  std::vector<std::thread> th;
  th.reserve(n_levels);
  for (int l = 0; l < n_levels; ++l) {
    th.emplace_back([&, l] {
      mlmc_model ml = *model;
      if (n_ce) ml.n_ce = n_ce[l];
      rc[l] = level_run_impl(ctx->subs[l], &ml, l, m_fine[l], first_sample[l], nullptr, n[l], cgv,
                             &opts[l], &sums[l], nullptr, nullptr, nullptr, nullptr, nullptr);
    });
  }
  for (auto& t : th) t.join();
  ctx->event_pool.push_back(start);
  // level runs synchronise their streams before returning; report the first
  // error, a non-converged solve only when nothing else failed
  int worst = -1;
  for (int l = 0; l < n_levels; ++l)
    if (rc[l] != MLMC_OK && (worst < 0 || (rc[worst] == MLMC_ENOCONV && rc[l] != MLMC_ENOCONV)))
      worst = l;
  if (worst >= 0)
    return fail(ctx, rc[worst],
                "level " + std::to_string(worst) + ": " + mlmc_last_error(ctx->subs[worst]));
  return MLMC_OK;
}

mlmc_status mlmc_estimate(const mlmc_level_sums* levels, int n_levels, mlmc_estimate_t* out) {
  if (!levels || !out || n_levels < 1) return MLMC_EINVAL;
  double est = 0.0, var = 0.0;
  for (int l = 0; l < n_levels; ++l) {
    const double nn = (double)levels[l].n;
    if (nn < 2) return MLMC_EINVAL;
    const double mean = levels[l].sum_y / nn;
    const double v = (levels[l].sum_y2 - nn * mean * mean) / (nn - 1.0);
    est += mean;
    var += v / nn;
  }
  out->estimate = est;
  out->variance = var;
  out->std_error = std::sqrt(var);
  return MLMC_OK;
}

mlmc_status mlmc_profile_enable(mlmc_ctx* ctx, const char* kernel_name) {
  if (!ctx) return MLMC_EINVAL;
  ctx->prof_name = kernel_name ? kernel_name : "";
  return MLMC_OK;
}

mlmc_status mlmc_profile_read(mlmc_ctx* ctx, int64_t* launches, double* total_ms,
                              double* algorithmic_bytes) {
  if (!ctx || !launches || !total_ms || !algorithmic_bytes) return MLMC_EINVAL;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  double ms = 0.0, bytes = 0.0;
  for (auto& pe : ctx->prof) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, pe.a, pe.b));
    ms += t;
    bytes += pe.bytes;
    ctx->event_pool.push_back(pe.a);
    ctx->event_pool.push_back(pe.b);
  }
  *launches = (int64_t)ctx->prof.size();
  *total_ms = ms;
  *algorithmic_bytes = bytes;
  ctx->prof.clear();
  return MLMC_OK;
}

}  // extern "C"
