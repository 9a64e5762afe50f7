"""Python binding of the MI355X (gfx950) MLMC Darcy-flow library.

A thin ctypes layer over the C ABI of ``include/mlmc_darcy.h``: every
function here has the name of the C entry point it calls and only marshals
arguments (torch tensors -> device pointers, the torch stream -> hipStream_t,
model records -> ``mlmc_model``).  All numerical work runs in the HIP kernels
of ``libmlmc_darcy.so``; there is no fallback.  If the library has not been
built (``python paper_1506_04694_amd/build.py``), importing the binding
raises ImportError.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlmc_darcy.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libmlmc_darcy.so is not built: run `python paper_1506_04694_amd/build.py` "
                      "(or __graft_entry__.build()) before using the GPU path")

_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ constants
MLMC_OK, MLMC_EINVAL, MLMC_ENOMEM, MLMC_EDEVICE, MLMC_EBUSY, MLMC_ENOCONV, MLMC_EEMBED = range(7)
STATUS_NAMES = {0: "MLMC_OK", 1: "MLMC_EINVAL", 2: "MLMC_ENOMEM", 3: "MLMC_EDEVICE",
                4: "MLMC_EBUSY", 5: "MLMC_ENOCONV", 6: "MLMC_EEMBED"}
MLMC_SAMPLE_OK, MLMC_SAMPLE_NOCONV, MLMC_SAMPLE_BREAKDOWN = 0, 1, 2
MLMC_PREC_FP64, MLMC_PREC_FP32, MLMC_PREC_BF16 = 0, 1, 2
MLMC_PROBLEM_OUTFLOW, MLMC_PROBLEM_MEAN_PRESSURE = 0, 1

EXPORTED = ["mlmc_ctx_create", "mlmc_ctx_destroy", "mlmc_ctx_set_stream", "mlmc_last_error",
            "mlmc_solver_opts_default", "mlmc_ce_min_embedding", "mlmc_sample_field",
            "mlmc_cgv_extract", "mlmc_assemble", "mlmc_solve", "mlmc_qoi_outflow",
            "mlmc_level_run", "mlmc_estimate", "mlmc_profile_enable", "mlmc_profile_read",
            "mlmc_sample_field_ids", "mlmc_level_run_ids", "mlmc_serve_opts_default",
            "mlmc_serve_start", "mlmc_serve_submit", "mlmc_serve_poll", "mlmc_serve_now",
            "mlmc_serve_stats", "mlmc_serve_stop", "mlmc_run_levels", "mlmc_serve_start_models",
            "mlmc_assemble_problem", "mlmc_qoi_box_mean", "mlmc_optimal_samples", "mlmc_rates",
            "mlmc_adaptive_opts_default", "mlmc_adaptive", "mlmc_solve_noalloc"]
MLMC_MAX_LEVELS = 16


class mlmc_model(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("interface_kind", ctypes.c_int32),
                ("n_nodes", ctypes.c_int32), ("n_layers", ctypes.c_int32),
                ("field_kind", ctypes.c_int32), ("norm_r", ctypes.c_int32),
                ("n_ce", ctypes.c_int32), ("problem", ctypes.c_int32),
                ("y_lo", ctypes.c_double), ("y_hi", ctypes.c_double),
                ("mu", ctypes.c_double * 4), ("sigma2", ctypes.c_double * 4),
                ("lambda_", ctypes.c_double * 4), ("seed", ctypes.c_uint64)]


class mlmc_solver_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("omega", ctypes.c_double),
                ("maxit", ctypes.c_int32), ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("coarse_max", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("cycle_max", ctypes.c_int32), ("gamma", ctypes.c_int32),
                ("gamma_levels", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("initial_guess", ctypes.c_int32), ("tile_shape", ctypes.c_int32)]


class mlmc_level_sums(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_failed", ctypes.c_int64),
                ("sum_y", ctypes.c_double), ("sum_y2", ctypes.c_double),
                ("sum_qf", ctypes.c_double), ("sum_qc", ctypes.c_double),
                ("iters_fine", ctypes.c_int64), ("iters_coarse", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mlmc_serve_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_workers", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("cgv", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("n_grids", ctypes.c_int32),
                ("grid_m", ctypes.c_int32 * 8), ("grid_n_ce", ctypes.c_int32 * 8),
                ("grid_model", ctypes.c_int32 * 8), ("reserved", ctypes.c_int32),
                ("solver", mlmc_solver_opts)]


class mlmc_request(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("m_fine", ctypes.c_int32),
                ("sample", ctypes.c_uint32), ("model", ctypes.c_int32)]


class mlmc_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("level", ctypes.c_int32), ("m_fine", ctypes.c_int32),
                ("sample", ctypes.c_uint32), ("failed", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("status", ctypes.c_int32), ("model", ctypes.c_int32),
                ("q_f", ctypes.c_double), ("q_c", ctypes.c_double), ("y", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mlmc_estimate_t(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("variance", ctypes.c_double),
                ("std_error", ctypes.c_double)]


class mlmc_adaptive_opts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("alpha", ctypes.c_double),
                ("n_initial", ctypes.c_int32), ("min_levels", ctypes.c_int32),
                ("cgv", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_samples", ctypes.c_int64)]


class mlmc_adaptive_result(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("estimate", ctypes.c_double), ("variance", ctypes.c_double),
                ("bias", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("seconds", ctypes.c_double), ("n", ctypes.c_int64 * MLMC_MAX_LEVELS),
                ("mean_y", ctypes.c_double * MLMC_MAX_LEVELS),
                ("var_y", ctypes.c_double * MLMC_MAX_LEVELS),
                ("cost", ctypes.c_double * MLMC_MAX_LEVELS),
                ("sums", mlmc_level_sums * MLMC_MAX_LEVELS)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_U64 = ctypes.c_uint64
_S = ctypes.c_int  # mlmc_status

_SIGS = {
    "mlmc_ctx_create": (_S, [_I, _P, ctypes.POINTER(_P)]),
    "mlmc_ctx_destroy": (_S, [_P]),
    "mlmc_ctx_set_stream": (_S, [_P, _P]),
    "mlmc_last_error": (ctypes.c_char_p, [_P]),
    "mlmc_solver_opts_default": (_S, [ctypes.POINTER(mlmc_solver_opts)]),
    "mlmc_ce_min_embedding": (_S, [_P, ctypes.POINTER(mlmc_model), _I, ctypes.POINTER(_I)]),
    "mlmc_sample_field": (_S, [_P, ctypes.POINTER(mlmc_model), _I, _I, _U64, _I, _P, _P]),
    "mlmc_cgv_extract": (_S, [_P, _I, _I, _I, _P, _P]),
    "mlmc_assemble": (_S, [_P, _I, _I, _I, _P, _P, _P, _P]),
    "mlmc_solve": (_S, [_P, _I, _I, _I, _P, _P, _P, _P, ctypes.POINTER(mlmc_solver_opts),
                        _P, _P, _P]),
    "mlmc_solve_noalloc": (_S, [_P, _I, _I, _I, _P, _P, _P, _P,
                                ctypes.POINTER(mlmc_solver_opts), _P, _P, _P]),
    "mlmc_qoi_outflow": (_S, [_P, _I, _I, _I, _P, _P, _P, _P]),
    "mlmc_level_run": (_S, [_P, ctypes.POINTER(mlmc_model), _I, _I, _U64, _I, _I,
                            ctypes.POINTER(mlmc_solver_opts), ctypes.POINTER(mlmc_level_sums),
                            _P, _P, _P]),
    "mlmc_estimate": (_S, [ctypes.POINTER(mlmc_level_sums), _I, ctypes.POINTER(mlmc_estimate_t)]),
    "mlmc_profile_enable": (_S, [_P, ctypes.c_char_p]),
    "mlmc_sample_field_ids": (_S, [_P, ctypes.POINTER(mlmc_model), _I, _I, _P, _I, _P, _P]),
    "mlmc_level_run_ids": (_S, [_P, ctypes.POINTER(mlmc_model), _I, _I, _P, _I, _I,
                                ctypes.POINTER(mlmc_solver_opts), ctypes.POINTER(mlmc_level_sums),
                                _P, _P, _P, _P, _P]),
    "mlmc_serve_opts_default": (_S, [ctypes.POINTER(mlmc_serve_opts)]),
    "mlmc_serve_start": (_S, [ctypes.POINTER(mlmc_model), ctypes.POINTER(mlmc_serve_opts),
                              ctypes.POINTER(_P)]),
    "mlmc_serve_start_models": (_S, [ctypes.POINTER(mlmc_model), ctypes.POINTER(mlmc_solver_opts),
                                     _I, ctypes.POINTER(mlmc_serve_opts), ctypes.POINTER(_P)]),
    "mlmc_serve_submit": (_S, [_P, ctypes.POINTER(mlmc_request), ctypes.POINTER(ctypes.c_uint64)]),
    "mlmc_serve_poll": (_S, [_P, ctypes.POINTER(mlmc_result), _I, ctypes.POINTER(_I),
                             ctypes.POINTER(ctypes.c_int64)]),
    "mlmc_serve_now": (ctypes.c_double, [_P]),
    "mlmc_serve_stats": (_S, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_uint64)]),
    "mlmc_serve_stop": (_S, [_P]),
    "mlmc_run_levels": (_S, [_P, ctypes.POINTER(mlmc_model), _I, ctypes.POINTER(_I),
                             ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_uint64),
                             ctypes.POINTER(_I), _I, ctypes.POINTER(mlmc_solver_opts),
                             ctypes.POINTER(mlmc_level_sums)]),
    "mlmc_profile_read": (_S, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double)]),
    "mlmc_assemble_problem": (_S, [_P, _I, _I, _I, _I, _P, _P, _P, _P]),
    "mlmc_qoi_box_mean": (_S, [_P, _I, _I, _I, _P, ctypes.c_double, ctypes.c_double, _P]),
    "mlmc_optimal_samples": (_S, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  _I, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]),
    "mlmc_rates": (_S, [ctypes.POINTER(mlmc_level_sums), ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(_I), _I, ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "mlmc_adaptive_opts_default": (_S, [ctypes.POINTER(mlmc_adaptive_opts)]),
    "mlmc_adaptive": (_S, [_P, ctypes.POINTER(mlmc_model), _I, ctypes.POINTER(_I),
                           ctypes.POINTER(_I), ctypes.POINTER(mlmc_adaptive_opts),
                           ctypes.POINTER(mlmc_solver_opts), ctypes.POINTER(mlmc_adaptive_result)]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class MlmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, code), msg))
        self.code = code


def _check(ctx, code):
    if code != MLMC_OK:
        msg = _lib.mlmc_last_error(ctx).decode() if ctx else ""
        raise MlmcError(code, msg)


def _ptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


def _f64(t, numel, name):
    import torch
    return _ptr(t, torch.float64, numel, name)


def _i32(t, numel, name):
    import torch
    return _ptr(t, torch.int32, numel, name)


def make_model(model, n_ce=0):
    """mlmc_model from any record with the workload fields (see workloads.Model)."""
    mm = mlmc_model()
    mm.dim = int(model.dim)
    mm.interface_kind = int(model.interface_kind)
    mm.n_nodes = int(model.n_nodes)
    mm.n_layers = int(model.n_layers)
    mm.field_kind = int(model.field_kind)
    mm.norm_r = int(model.norm_r)
    mm.n_ce = int(n_ce)
    mm.y_lo = float(model.y_lo)
    mm.y_hi = float(model.y_hi)
    for l in range(4):
        mm.mu[l] = float(model.mu[l])
        mm.sigma2[l] = float(model.sigma2[l])
        mm.lambda_[l] = float(model.lam[l])
    mm.seed = int(model.seed)
    mm.problem = int(getattr(model, "problem", 0))
    return mm


def model_for_grid(model, m):
    """mlmc_model for sampling an m x m grid (picks the model's n_ce for m)."""
    n_ce = model.n_ce.get(m, 0) if getattr(model, "n_ce", None) else 0
    return make_model(model, n_ce)


# ------------------------------------------------------------------ entry points
def mlmc_ctx_create(device=0, stream=None):
    """Returns an opaque context handle bound to `stream` (a torch stream or raw handle)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
    h = ctypes.c_void_p()
    code = _lib.mlmc_ctx_create(int(device), ctypes.c_void_p(raw), ctypes.byref(h))
    if code != MLMC_OK:
        raise MlmcError(code, "mlmc_ctx_create failed on device %d" % device)
    return h


def mlmc_ctx_destroy(ctx):
    _check(ctx, _lib.mlmc_ctx_destroy(ctx))


def mlmc_ctx_set_stream(ctx, stream):
    raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
    _check(ctx, _lib.mlmc_ctx_set_stream(ctx, ctypes.c_void_p(raw)))


def mlmc_last_error(ctx):
    return _lib.mlmc_last_error(ctx).decode()


def mlmc_solver_opts_default(**overrides):
    o = mlmc_solver_opts()
    _check(None, _lib.mlmc_solver_opts_default(ctypes.byref(o)))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def mlmc_ce_min_embedding(ctx, model, m):
    n = ctypes.c_int()
    mm = model if isinstance(model, mlmc_model) else make_model(model)
    _check(ctx, _lib.mlmc_ce_min_embedding(ctx, ctypes.byref(mm), int(m), ctypes.byref(n)))
    return n.value


def mlmc_sample_field(ctx, model, m, level, first_sample, batch, k, k_coarse=None):
    mm = model if isinstance(model, mlmc_model) else model_for_grid(model, m)
    d = int(mm.dim)
    _check(ctx, _lib.mlmc_sample_field(ctx, ctypes.byref(mm), int(m), int(level),
                                       int(first_sample), int(batch),
                                       _f64(k, batch * m ** d, "k"),
                                       _f64(k_coarse, batch * (m // 2) ** d, "k_coarse")))


def mlmc_cgv_extract(ctx, dim, m, batch, k_fine, k_sub):
    d = int(dim)
    _check(ctx, _lib.mlmc_cgv_extract(ctx, d, int(m), int(batch),
                                      _f64(k_fine, batch * m ** d, "k_fine"),
                                      _f64(k_sub, batch * 2 ** d * (m // 2) ** d, "k_sub")))


def mlmc_assemble(ctx, dim, m, batch, k, T, tb, b):
    d = int(dim)
    n = batch * m ** d
    _check(ctx, _lib.mlmc_assemble(ctx, d, int(m), int(batch), _f64(k, n, "k"),
                                   _f64(T, d * n, "T"), _f64(tb, d * batch * m ** (d - 1), "tb"),
                                   _f64(b, n, "b")))


def mlmc_assemble_problem(ctx, problem, dim, m, batch, k, T, tb, b):
    d = int(dim)
    n = batch * m ** d
    _check(ctx, _lib.mlmc_assemble_problem(ctx, int(problem), d, int(m), int(batch),
                                           _f64(k, n, "k"), _f64(T, d * n, "T"),
                                           _f64(tb, d * batch * m ** (d - 1), "tb"),
                                           _f64(b, n, "b")))


def mlmc_qoi_box_mean(ctx, dim, m, batch, p, lo, hi, q):
    d = int(dim)
    _check(ctx, _lib.mlmc_qoi_box_mean(ctx, d, int(m), int(batch), _f64(p, batch * m ** d, "p"),
                                       float(lo), float(hi), _f64(q, batch, "q")))


def mlmc_solve(ctx, dim, m, batch, T, tb, b, p, opts, status, iters, relres):
    d = int(dim)
    n = batch * m ** d
    _check(ctx, _lib.mlmc_solve(ctx, d, int(m), int(batch), _f64(T, d * n, "T"),
                                _f64(tb, d * batch * m ** (d - 1), "tb"), _f64(b, n, "b"),
                                _f64(p, n, "p"), ctypes.byref(opts),
                                _i32(status, batch, "status"), _i32(iters, batch, "iters"),
                                _f64(relres, batch, "relres")))


def mlmc_solve_noalloc(ctx, dim, m, batch, T, tb, b, p, opts, status, iters, relres):
    """mlmc_solve with every workspace in the library's static scratch array."""
    d = int(dim)
    n = batch * m ** d
    _check(ctx, _lib.mlmc_solve_noalloc(ctx, d, int(m), int(batch), _f64(T, d * n, "T"),
                                        _f64(tb, d * batch * m ** (d - 1), "tb"),
                                        _f64(b, n, "b"), _f64(p, n, "p"), ctypes.byref(opts),
                                        _i32(status, batch, "status"),
                                        _i32(iters, batch, "iters"),
                                        _f64(relres, batch, "relres")))


def mlmc_qoi_outflow(ctx, dim, m, batch, k, p, q_out, q_in=None):
    d = int(dim)
    n = batch * m ** d
    _check(ctx, _lib.mlmc_qoi_outflow(ctx, d, int(m), int(batch), _f64(k, n, "k"),
                                      _f64(p, n, "p"), _f64(q_out, batch, "q_out"),
                                      _f64(q_in, batch, "q_in")))


def mlmc_level_run(ctx, model, level, m_fine, first_sample, n, cgv, opts, sums=None,
                   q_f=None, q_c=None, y=None, allow_noconv=False):
    """Runs one estimator level; returns the (accumulated) mlmc_level_sums."""
    mm = model if isinstance(model, mlmc_model) else model_for_grid(model, m_fine)
    if sums is None:
        sums = mlmc_level_sums()
    code = _lib.mlmc_level_run(ctx, ctypes.byref(mm), int(level), int(m_fine), int(first_sample),
                               int(n), int(bool(cgv)), ctypes.byref(opts), ctypes.byref(sums),
                               _f64(q_f, n, "q_f"), _f64(q_c, n, "q_c"), _f64(y, n, "y"))
    if not (allow_noconv and code == MLMC_ENOCONV):
        _check(ctx, code)
    return sums


def mlmc_estimate(levels):
    arr = (mlmc_level_sums * len(levels))(*levels)
    out = mlmc_estimate_t()
    _check(None, _lib.mlmc_estimate(arr, len(levels), ctypes.byref(out)))
    return {"estimate": out.estimate, "variance": out.variance, "std_error": out.std_error}


def mlmc_profile_enable(ctx, kernel_name):
    _check(ctx, _lib.mlmc_profile_enable(ctx, kernel_name.encode() if kernel_name else None))


def mlmc_profile_read(ctx):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(ctx, _lib.mlmc_profile_read(ctx, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return {"launches": n.value, "total_ms": ms.value, "algorithmic_bytes": by.value}


def _u32(t, numel, name):
    import torch
    if t is not None and t.dtype not in (torch.int32, torch.uint32):
        raise ValueError("%s must be int32/uint32" % name)
    return _ptr(t, None, numel, name)


def mlmc_sample_field_ids(ctx, model, m, level, sample_ids, batch, k, k_coarse=None):
    mm = model if isinstance(model, mlmc_model) else model_for_grid(model, m)
    _check(ctx, _lib.mlmc_sample_field_ids(ctx, ctypes.byref(mm), int(m), int(level),
                                           _u32(sample_ids, batch, "sample_ids"), int(batch),
                                           _f64(k, batch * m ** int(mm.dim), "k"),
                                           _f64(k_coarse, batch * (m // 2) ** int(mm.dim), "k_coarse")))


def mlmc_level_run_ids(ctx, model, level, m_fine, sample_ids, n, cgv, opts, sums=None,
                       q_f=None, q_c=None, y=None, failed=None, iters=None, allow_noconv=False):
    mm = model if isinstance(model, mlmc_model) else model_for_grid(model, m_fine)
    if sums is None:
        sums = mlmc_level_sums()
    code = _lib.mlmc_level_run_ids(ctx, ctypes.byref(mm), int(level), int(m_fine),
                                   _u32(sample_ids, n, "sample_ids"), int(n), int(bool(cgv)),
                                   ctypes.byref(opts), ctypes.byref(sums), _f64(q_f, n, "q_f"),
                                   _f64(q_c, n, "q_c"), _f64(y, n, "y"),
                                   _i32(failed, n, "failed"), _i32(iters, n, "iters"))
    if not (allow_noconv and code == MLMC_ENOCONV):
        _check(ctx, code)
    return sums


def mlmc_serve_opts_default(**overrides):
    o = mlmc_serve_opts()
    _check(None, _lib.mlmc_serve_opts_default(ctypes.byref(o)))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def serve_opts_for(model, grids, **overrides):
    """Server options serving the fine grids `grids` of `model` (embedding sizes from model.n_ce)."""
    return serve_opts_for_models([(model, grids)], **overrides)


def serve_opts_for_models(model_grids, **overrides):
    """Server options for several models: model_grids = [(model, grids), ...]; grid entries
    of the q-th pair serve model index q (embedding sizes from model.n_ce)."""
    o = mlmc_serve_opts_default(**overrides)
    q = 0
    for mi, (model, grids) in enumerate(model_grids):
        for m in grids:
            if q >= 8:
                raise ValueError("at most 8 (model, grid) entries")
            o.grid_m[q] = int(m)
            o.grid_n_ce[q] = int(model.n_ce.get(m, 0)) if getattr(model, "n_ce", None) else 0
            o.grid_model[q] = mi
            q += 1
    o.n_grids = q
    return o


def mlmc_serve_start(model, opts):
    mm = model if isinstance(model, mlmc_model) else make_model(model)
    h = ctypes.c_void_p()
    code = _lib.mlmc_serve_start(ctypes.byref(mm), ctypes.byref(opts), ctypes.byref(h))
    if code != MLMC_OK:
        raise MlmcError(code, "mlmc_serve_start failed")
    return h


def mlmc_serve_start_models(models, opts, solvers=None):
    """models: list of workload models or mlmc_model; solvers: list of mlmc_solver_opts
    (one per model) or None for opts.solver."""
    L = len(models)
    arr = (mlmc_model * L)(*[m if isinstance(m, mlmc_model) else make_model(m) for m in models])
    sol = None if solvers is None else (mlmc_solver_opts * L)(*solvers)
    h = ctypes.c_void_p()
    code = _lib.mlmc_serve_start_models(arr, sol, L, ctypes.byref(opts), ctypes.byref(h))
    if code != MLMC_OK:
        raise MlmcError(code, "mlmc_serve_start_models failed")
    return h


def mlmc_serve_submit(srv, level, m_fine, sample, model=0):
    req = mlmc_request(int(level), int(m_fine), int(sample), int(model))
    rid = ctypes.c_uint64()
    code = _lib.mlmc_serve_submit(srv, ctypes.byref(req), ctypes.byref(rid))
    if code != MLMC_OK:
        raise MlmcError(code, "mlmc_serve_submit rejected the request")
    return rid.value


def mlmc_serve_poll(srv, max_results=4096):
    buf = (mlmc_result * max_results)()
    n = ctypes.c_int()
    pend = ctypes.c_int64()
    _check(None, _lib.mlmc_serve_poll(srv, buf, int(max_results), ctypes.byref(n),
                                      ctypes.byref(pend)))
    return [buf[q].as_dict() for q in range(n.value)], pend.value


def mlmc_serve_now(srv):
    return _lib.mlmc_serve_now(srv)


def mlmc_serve_stats(srv):
    b, qd, ru, fl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int(), ctypes.c_uint64()
    _check(None, _lib.mlmc_serve_stats(srv, ctypes.byref(b), ctypes.byref(qd), ctypes.byref(ru),
                                       ctypes.byref(fl)))
    return {"batches": b.value, "queued": qd.value, "running": ru.value,
            "in_flight_bytes": fl.value}


def mlmc_serve_stop(srv):
    _check(None, _lib.mlmc_serve_stop(srv))


def mlmc_run_levels(ctx, model, m_fine, first_sample, n, cgv, opts, sums=None, allow_noconv=False):
    """All levels in one call; opts is one mlmc_solver_opts or a list (one per level).
    Returns the list of mlmc_level_sums."""
    L = len(m_fine)
    if isinstance(opts, mlmc_solver_opts):
        opts = [opts] * L
    mm = make_model(model)
    nce = [int(model.n_ce.get(m, 0)) if getattr(model, "n_ce", None) else 0 for m in m_fine]
    if sums is None:
        sums = [mlmc_level_sums() for _ in range(L)]
    arr_s = (mlmc_level_sums * L)(*sums)
    code = _lib.mlmc_run_levels(ctx, ctypes.byref(mm), L, (ctypes.c_int * L)(*m_fine),
                                (ctypes.c_int * L)(*nce), (ctypes.c_uint64 * L)(*first_sample),
                                (ctypes.c_int * L)(*n), int(bool(cgv)),
                                (mlmc_solver_opts * L)(*opts), arr_s)
    if not (allow_noconv and code == MLMC_ENOCONV):
        _check(ctx, code)
    return [arr_s[q] for q in range(L)]


# ------------------------------------------------------------------ choosing L and N_l
def mlmc_optimal_samples(var, cost, eps):
    """Host arithmetic: N_l for the variance part eps^2/2 at the least cost."""
    L = len(var)
    out = (ctypes.c_int64 * L)()
    code = _lib.mlmc_optimal_samples((ctypes.c_double * L)(*map(float, var)),
                                     (ctypes.c_double * L)(*map(float, cost)), L, float(eps), out)
    _check(None, code)
    return [int(v) for v in out]


def mlmc_rates(sums, cost, m):
    """Host arithmetic: (alpha, beta, gamma) fitted over the levels l >= 1."""
    L = len(sums)
    a, b, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    code = _lib.mlmc_rates((mlmc_level_sums * L)(*sums), (ctypes.c_double * L)(*map(float, cost)),
                           (ctypes.c_int * L)(*m), L, ctypes.byref(a), ctypes.byref(b),
                           ctypes.byref(g))
    _check(None, code)
    return a.value, b.value, g.value


def mlmc_adaptive_opts_default(**kw):
    o = mlmc_adaptive_opts()
    _check(None, _lib.mlmc_adaptive_opts_default(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def mlmc_adaptive(ctx, model, m_levels, opts, solver):
    """MLMC to the root mean square error opts.eps; returns mlmc_adaptive_result."""
    L = len(m_levels)
    mm = make_model(model)
    nce = None
    if getattr(model, "n_ce", None):
        nce = (ctypes.c_int * L)(*[int(model.n_ce.get(m, 0)) for m in m_levels])
    out = mlmc_adaptive_result()
    _check(ctx, _lib.mlmc_adaptive(ctx, ctypes.byref(mm), L, (ctypes.c_int * L)(*m_levels), nce,
                                   ctypes.byref(opts), ctypes.byref(solver), ctypes.byref(out)))
    return out
