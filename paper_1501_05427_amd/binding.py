"""ctypes binding of libulisse_gp.so with the C ABI's names (argument marshalling only).

Device arrays are torch tensors on a ROCm device; every computation runs in the HIP
library.  Conventions of the Python side:
  * X is an (n, d) float32 tensor with unit stride along d (row-major, ldx = X.stride(0));
  * a block of m vectors of length n is an (n, m) tensor with unit stride along n
    (column-major, ld = stride(1)) -- ``colmajor(n, m)`` allocates one; a single vector
    may be a 1-D tensor;
  * psi and g are float64 device tensors; the stream is torch's current stream unless
    one is given.
If the shared library has not been built, every call raises: there is no fallback.
"""
import ctypes
import os
import re
from ctypes import POINTER, Structure, c_char_p, c_double, c_int, c_int32, c_int64, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libulisse_gp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ulisse_gp.h")

GP_OK, GP_EINVAL, GP_ENOMEM, GP_EDEVICE, GP_EUNSUPPORTED = 0, -1, -2, -3, -4
GP_FP32, GP_BF16_SPLIT_V, GP_BF16_SPLIT_KV = 0, 1, 2
ULISSE_NOTCONV, ULISSE_BREAKDOWN, ULISSE_FALLBACK, ULISSE_FP32_RERUN = 1, 2, 4, 8
PROBE_GAUSSIAN, PROBE_RADEMACHER = 0, 1


class gp_data(Structure):
    _fields_ = [("X", c_void_p), ("n", c_int64), ("d", c_int32), ("ldx", c_int64)]


class ulisse_params(Structure):
    _fields_ = [("q", c_double), ("rate", c_double), ("eps", c_double),
                ("eps_relative", c_int32), ("max_iter", c_int32),
                ("two_track_first", c_int32), ("refresh", c_int32),
                ("rng_stream", c_uint64), ("rng_counter", c_uint64), ("prec", c_int)]


class ulisse_sysstat(Structure):
    _fields_ = [("l", c_int32), ("J_a", c_int32), ("J_b", c_int32), ("iters", c_int32),
                ("final_res", c_double), ("flags", c_uint32), ("pad", c_uint32)]


class gp_prior(Structure):
    _fields_ = [("kind", c_int32), ("reserved", c_int32), ("a", c_void_p), ("b", c_void_p)]


class gp_profile_stats(Structure):
    _fields_ = [("kmv_launches", c_int64), ("kmv_ms", c_double), ("dquad_launches", c_int64),
                ("dquad_ms", c_double), ("solves", c_int64), ("kmv_passes", c_int64),
                ("kmv_main_launches", c_int64), ("kmv_main_ms", c_double)]


class gp_precond(Structure):
    _fields_ = [("U", c_void_p), ("ldu", c_int64), ("k", c_int32), ("warm_start", c_int32),
                ("coef", c_void_p), ("c", c_void_p)]


class gp_shift_precond(Structure):
    _fields_ = [("delta", c_double), ("eps_inner", c_double), ("max_inner", c_int32),
                ("prec_inner", c_int)]


class sgld_schedule(Structure):
    _fields_ = [("a", c_double), ("b", c_double), ("gamma", c_double), ("freeze_ratio", c_double),
                ("batch", c_int32), ("probe_period", c_int32), ("n_probes", c_int32),
                ("probe_kind", c_int32)]


class sgld_state(Structure):
    _fields_ = [("t", c_int64), ("frozen", c_int32), ("frozen_at", c_int32), ("eps_frozen", c_double)]


class gp_batch_problem(Structure):
    _fields_ = [("X", gp_data), ("y", c_void_p), ("psi", c_void_p), ("S_warm", c_void_p), ("R", c_void_p),
                ("g", c_void_p), ("stats", c_void_p), ("M_chol", c_void_p), ("prior", gp_prior),
                ("mlp", c_void_p), ("mlp_hidden", c_int32), ("k", c_int32), ("U", c_void_p), ("ldu", c_int64),
                ("coef", c_void_p)]


class gp_batch_stats(Structure):
    _fields_ = [("eager_steps", c_int64), ("graph_steps", c_int64), ("iteration_graphs", c_int64),
                ("captures", c_int64), ("fp32_reruns", c_int64)]


SYSSTAT_BYTES = ctypes.sizeof(ulisse_sysstat)

_lib = None


class LibraryMissing(RuntimeError):
    pass


class GPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def lib():
    """Load the shared library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is missing: build it with `python -m paper_1501_05427_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.gp_last_error.restype = c_char_p
    L.gp_last_error.argtypes = []
    L.gp_create.restype = c_int
    L.gp_create.argtypes = [POINTER(c_void_p), c_int, c_uint64]
    L.gp_destroy.restype = None
    L.gp_destroy.argtypes = [c_void_p]
    L.gp_kmv.restype = c_int
    L.gp_kmv.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_int64, c_int, c_void_p]
    L.gp_kmv_noalloc.restype = c_int
    L.gp_kmv_noalloc.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_int64, c_int, c_void_p]
    L.gp_dkmv.restype = c_int
    L.gp_dkmv.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_int64, c_int64, c_int, c_void_p]
    L.ulisse_solve.restype = c_int
    L.ulisse_solve.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_int32, c_int64, c_void_p,
                               POINTER(ulisse_params), c_void_p, c_void_p, c_void_p, c_void_p]
    L.gp_stoch_grad.restype = c_int
    L.gp_stoch_grad.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                POINTER(ulisse_params), c_void_p, c_void_p, c_void_p, c_void_p]
    L.sgld_step.restype = c_int
    L.sgld_step.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, POINTER(gp_prior), c_void_p,
                            c_double, c_uint64, c_uint64, c_void_p]
    L.gp_draw_probes.restype = c_int
    L.gp_draw_probes.argtypes = [c_void_p, c_int64, c_int32, c_int32, c_uint64, c_uint64, c_void_p, c_int64, c_void_p]
    L.gp_philox.restype = c_int
    L.gp_philox.argtypes = [c_uint64, c_uint64, c_uint64, c_uint64, c_uint64, c_uint64, c_int64, c_void_p, c_void_p]
    L.ulisse_solve_pc.restype = c_int
    L.ulisse_solve_pc.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_int32, c_int64, c_void_p,
                                  POINTER(ulisse_params), POINTER(gp_precond), c_void_p, c_void_p,
                                  c_void_p, c_void_p]
    L.gp_stoch_grad_pc.restype = c_int
    L.gp_stoch_grad_pc.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                   POINTER(ulisse_params), POINTER(gp_precond), c_void_p, c_void_p,
                                   c_void_p, c_void_p]
    L.ulisse_solve_shift_pc.restype = c_int
    L.ulisse_solve_shift_pc.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_int32, c_int64, c_void_p,
                                        POINTER(ulisse_params), POINTER(gp_shift_precond), c_void_p,
                                        c_void_p, c_void_p, c_void_p]
    L.gp_stoch_grad_shift_pc.restype = c_int
    L.gp_stoch_grad_shift_pc.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                         POINTER(ulisse_params), POINTER(gp_shift_precond), c_void_p,
                                         c_void_p, c_void_p, c_void_p]
    L.precond_build_basis.restype = c_int
    L.precond_build_basis.argtypes = [c_void_p, gp_data, c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_void_p]
    L.precond_targets.restype = c_int
    L.precond_targets.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_int32,
                                  c_void_p, c_void_p]
    L.precond_mlp_size.restype = c_int64
    L.precond_mlp_size.argtypes = [c_int32, c_int32, c_int32]
    L.precond_mlp_init.restype = c_int
    L.precond_mlp_init.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int32,
                                   c_uint64, c_void_p]
    L.precond_mlp_train.restype = c_int
    L.precond_mlp_train.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                    c_int32, c_int32, c_int32, ctypes.c_float, c_void_p, c_void_p]
    L.precond_mlp_forward.restype = c_int
    L.precond_mlp_forward.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p,
                                      c_int32, c_void_p]
    L.precond_mlp_grad.restype = c_int
    L.precond_mlp_grad.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int32,
                                   c_void_p, c_void_p, c_void_p]
    L.precond_from_mlp.restype = c_int
    L.precond_from_mlp.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p,
                                   c_void_p, c_void_p]
    L.precond_from_targets.restype = c_int
    L.precond_from_targets.argtypes = [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
    L.precond_warm_start.restype = c_int
    L.precond_warm_start.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_int64, c_void_p, c_void_p, c_void_p]
    L.sgld_run.restype = c_int
    L.sgld_run.argtypes = [c_void_p, gp_data, c_void_p, c_void_p, POINTER(ulisse_params), POINTER(gp_prior),
                           c_void_p, POINTER(sgld_schedule), POINTER(sgld_state), c_int32, c_void_p,
                           c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.gp_profile.restype = c_int
    L.gp_profile.argtypes = [c_void_p, c_int32]
    L.gp_autotune.restype = c_int
    L.gp_autotune.argtypes = [c_void_p, c_int32]
    L.gp_autotune_split.restype = c_int
    L.gp_autotune_split.argtypes = [c_void_p, c_int64, c_int32, c_int32, c_int, POINTER(c_int32)]
    L.gp_pipe_probe.restype = c_int
    L.gp_pipe_probe.argtypes = [c_void_p, c_int32, POINTER(c_double), POINTER(c_double), c_void_p]
    L.gp_tune_set.restype = c_int
    L.gp_tune_set.argtypes = [c_void_p, c_int64, c_int32, c_int32, c_int, c_int32]
    L.gp_tune_get.restype = c_int
    L.gp_tune_get.argtypes = [c_void_p, c_int64, c_int32, c_int32, c_int, POINTER(c_int32), POINTER(c_int32)]
    L.gp_shape_query.restype = c_int
    L.gp_shape_query.argtypes = [c_int64, c_int32, c_int32, c_int, c_int32, POINTER(c_int32), POINTER(c_int32),
                                 POINTER(c_int32), POINTER(c_int64)]
    L.gp_tune_save.restype = c_int
    L.gp_tune_save.argtypes = [c_void_p, ctypes.c_char_p]
    L.gp_tune_load.restype = c_int
    L.gp_tune_load.argtypes = [c_void_p, ctypes.c_char_p]
    L.gp_batch_create.restype = c_int
    L.gp_batch_create.argtypes = [POINTER(c_void_p), c_int, c_uint64, c_int32, POINTER(gp_batch_problem),
                                  c_int32, c_int32, c_int32, POINTER(ulisse_params), c_int32, c_int32, c_int32]
    L.gp_batch_step.restype = c_int
    L.gp_batch_step.argtypes = [c_void_p, c_uint64, c_double, c_void_p]
    L.gp_batch_read_stats.restype = c_int
    L.gp_batch_read_stats.argtypes = [c_void_p, POINTER(gp_batch_stats)]
    L.gp_batch_destroy.restype = None
    L.gp_batch_destroy.argtypes = [c_void_p]
    L.gp_profile_read.restype = c_int
    L.gp_profile_read.argtypes = [c_void_p, POINTER(gp_profile_stats)]
    _lib = L
    return L


def header_functions():
    """Names of the functions declared in include/ulisse_gp.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                                 src, flags=re.M)))


def _check(status):
    if status != GP_OK:
        raise GPError(status, lib().gp_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    return c_void_p(stream)


def _ptr(t):
    return c_void_p(0 if t is None else t.data_ptr())


def _ld(t, n):
    """Leading dimension of a column-major (n, m) tensor or a vector."""
    if t.dim() == 1:
        return n
    if t.shape[1] > 1 and t.stride(0) != 1:
        raise ValueError("blocks of vectors must be column-major: (n, m) with stride (1, ld)")
    return t.stride(1) if t.shape[1] > 1 else max(n, t.stride(1))


def _cols(t):
    return 1 if t.dim() == 1 else t.shape[1]


def colmajor(n, m, dtype=None, device="cuda"):
    import torch
    return torch.zeros((m, n), dtype=dtype or torch.float32, device=device).t()


def _data(X):
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be an (n, d) tensor with unit stride along d")
    return gp_data(X.data_ptr(), X.shape[0], X.shape[1], X.stride(0))


class Handle:
    """gp_create / gp_destroy."""

    def __init__(self, device=0, seed=0):
        self.ptr = c_void_p()
        _check(lib().gp_create(ctypes.byref(self.ptr), int(device), int(seed)))
        self.seed = int(seed)

    def close(self):
        if self.ptr:
            lib().gp_destroy(self.ptr)
            self.ptr = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gp_create(device=0, seed=0):
    return Handle(device, seed)


def gp_destroy(h):
    h.close()


def gp_last_error():
    return lib().gp_last_error().decode()


def gp_kmv(h, X, psi, V, out=None, prec=GP_FP32, stream=None):
    n = X.shape[0]
    m = _cols(V)
    if out is None:
        out = colmajor(n, m, device=V.device) if V.dim() == 2 else V.new_zeros(n)
    _check(lib().gp_kmv(h.ptr, _data(X), _ptr(psi), _ptr(V), m, _ld(V, n), _ptr(out), _ld(out, n),
                        int(prec), _stream(stream)))
    return out


def gp_kmv_noalloc(h, X, psi, V, out, prec=GP_FP32, stream=None):
    """gp_kmv with the library's fixed device scratch: the output must be given."""
    n = X.shape[0]
    m = _cols(V)
    _check(lib().gp_kmv_noalloc(h.ptr, _data(X), _ptr(psi), _ptr(V), m, _ld(V, n), _ptr(out), _ld(out, n),
                                int(prec), _stream(stream)))
    return out


def gp_dkmv(h, X, psi, V, out=None, prec=GP_FP32, stream=None):
    """Returns a (d + 2, m, n) tensor: block j column c = (dK/dpsi_j V)[:, c]."""
    import torch
    n, d = X.shape
    m = _cols(V)
    if out is None:
        out = torch.zeros((d + 2, m, n), dtype=torch.float32, device=V.device)
    _check(lib().gp_dkmv(h.ptr, _data(X), _ptr(psi), _ptr(V), m, _ld(V, n), _ptr(out), out.stride(1),
                         out.stride(0), int(prec), _stream(stream)))
    return out


def make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=1000, two_track_first=0,
                rng_stream=0, rng_counter=0, prec=GP_FP32, refresh=0):
    return ulisse_params(q, rate, eps, eps_relative, max_iter, two_track_first, refresh,
                         rng_stream, rng_counter, prec)


def stats_tensor(m, device="cuda"):
    import torch
    return torch.zeros(m * SYSSTAT_BYTES, dtype=torch.uint8, device=device)


def decode_stats(raw):
    """Device stats buffer -> list of dicts (copies to the host)."""
    b = bytes(raw.cpu().numpy().tobytes())
    out = []
    for k in range(len(b) // SYSSTAT_BYTES):
        s = ulisse_sysstat.from_buffer_copy(b[k * SYSSTAT_BYTES:(k + 1) * SYSSTAT_BYTES])
        out.append(dict(l=s.l, J_a=s.J_a, J_b=s.J_b, iters=s.iters, final_res=s.final_res, flags=s.flags))
    return out


def ulisse_solve(h, X, psi, B, params, S0=None, S_tilde=None, S_cg=None, stats=None, stream=None):
    import torch
    n = X.shape[0]
    m = _cols(B)
    mt = m + (1 if params.two_track_first else 0)
    if S_tilde is None:
        S_tilde = torch.zeros((mt, n), dtype=torch.float64, device=B.device).t()
    if stats is None:
        stats = stats_tensor(m, B.device)
    _check(lib().ulisse_solve(h.ptr, _data(X), _ptr(psi), _ptr(B), m, _ld(B, n), _ptr(S0),
                              ctypes.byref(params), _ptr(S_tilde), _ptr(S_cg), _ptr(stats),
                              _stream(stream)))
    return S_tilde, stats


def gp_stoch_grad(h, X, psi, y, params, R=None, n_probes=None, probe_kind=PROBE_GAUSSIAN,
                  S_warm=None, g=None, stats=None, stream=None):
    import torch
    d = X.shape[1]
    if R is not None:
        n_probes = _cols(R)
    if g is None:
        g = torch.zeros(d + 2, dtype=torch.float64, device=y.device)
    if stats is None:
        stats = stats_tensor(1 + n_probes, y.device)
    _check(lib().gp_stoch_grad(h.ptr, _data(X), _ptr(psi), _ptr(y), _ptr(R), int(n_probes),
                               int(probe_kind), ctypes.byref(params), _ptr(S_warm), _ptr(g),
                               _ptr(stats), _stream(stream)))
    return g, stats


def sgld_step(h, psi, g, eps_t, rng_stream=0, rng_counter=0, prior_kind=0, prior_a=None,
              prior_b=None, M_chol=None, stream=None):
    pr = gp_prior(int(prior_kind), 0, 0 if prior_a is None else prior_a.data_ptr(),
                  0 if prior_b is None else prior_b.data_ptr())
    _check(lib().sgld_step(h.ptr, psi.shape[0], _ptr(psi), _ptr(g), ctypes.byref(pr), _ptr(M_chol),
                           float(eps_t), int(rng_stream), int(rng_counter), _stream(stream)))
    return psi


def gp_draw_probes(h, n, n_probes, probe_kind, rng_stream, rng_counter, R=None, stream=None):
    if R is None:
        R = colmajor(n, n_probes)
    _check(lib().gp_draw_probes(h.ptr, n, n_probes, probe_kind, rng_stream, rng_counter, _ptr(R),
                                _ld(R, n), _stream(stream)))
    return R


def gp_philox(k0, k1, first_block, w1, w2, w3, nblocks, out=None, stream=None):
    import torch
    if out is None:
        out = torch.zeros(4 * nblocks, dtype=torch.int64, device="cuda")
    _check(lib().gp_philox(k0, k1, first_block, w1, w2, w3, nblocks, _ptr(out), _stream(stream)))
    return out


def gp_profile(h, enable):
    _check(lib().gp_profile(h.ptr, int(bool(enable))))


def gp_profile_read(h):
    st = gp_profile_stats()
    _check(lib().gp_profile_read(h.ptr, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in gp_profile_stats._fields_}


def make_schedule(a, b, gamma=1.0, freeze_ratio=0.002, batch=100, probe_period=20, n_probes=4,
                  probe_kind=PROBE_RADEMACHER):
    return sgld_schedule(a, b, gamma, freeze_ratio, batch, probe_period, n_probes, probe_kind)


def new_state(t=0):
    return sgld_state(t, 0, -1, 0.0)


def sgld_run(h, X, psi, y, params, sched, state, T, S_warm, R, prior_kind=0, prior_a=None,
             prior_b=None, M_chol=None, trace=None, eps_trace=None, ratio_trace=None, stream=None):
    """Runs T protocol steps in place on psi, S_warm, R; `state` (sgld_state) advances."""
    pr = gp_prior(int(prior_kind), 0, 0 if prior_a is None else prior_a.data_ptr(),
                  0 if prior_b is None else prior_b.data_ptr())
    _check(lib().sgld_run(h.ptr, _data(X), _ptr(psi), _ptr(y), ctypes.byref(params), ctypes.byref(pr),
                          _ptr(M_chol), ctypes.byref(sched), ctypes.byref(state), int(T), _ptr(S_warm),
                          _ptr(R), _ptr(trace), _ptr(eps_trace), _ptr(ratio_trace), _stream(stream)))
    return state


class Precond:
    """A gp_precond plus references to its device tensors (they must outlive every call
    that uses the descriptor).  U: (n, k) column-major FP32; coef: k + 1 FP64 (h, tau_inv;
    a negative tau_inv selects the plain solver); cvec (optional): k FP64 warm-start
    coefficients, system 0 then starts from U cvec."""

    def __init__(self, U, coef, cvec=None):
        self.U, self.coef, self.cvec = U, coef, cvec
        self.c = gp_precond(U.data_ptr(), _ld(U, U.shape[0]), U.shape[1], 0 if cvec is None else 1,
                            coef.data_ptr(), 0 if cvec is None else cvec.data_ptr())


def make_precond(U, coef, cvec=None):
    return Precond(U, coef, cvec)


def ulisse_solve_pc(h, X, psi, B, params, pc, S0=None, S_tilde=None, S_cg=None, stats=None, stream=None):
    import torch
    n = X.shape[0]
    m = _cols(B)
    mt = m + (1 if params.two_track_first else 0)
    if S_tilde is None:
        S_tilde = torch.zeros((mt, n), dtype=torch.float64, device=B.device).t()
    if stats is None:
        stats = stats_tensor(m, B.device)
    _check(lib().ulisse_solve_pc(h.ptr, _data(X), _ptr(psi), _ptr(B), m, _ld(B, n), _ptr(S0),
                                 ctypes.byref(params), ctypes.byref(pc.c), _ptr(S_tilde), _ptr(S_cg),
                                 _ptr(stats), _stream(stream)))
    return S_tilde, stats


def gp_stoch_grad_pc(h, X, psi, y, params, pc, R=None, n_probes=None, probe_kind=PROBE_GAUSSIAN,
                     S_warm=None, g=None, stats=None, stream=None):
    import torch
    d = X.shape[1]
    if R is not None:
        n_probes = _cols(R)
    if g is None:
        g = torch.zeros(d + 2, dtype=torch.float64, device=y.device)
    if stats is None:
        stats = stats_tensor(1 + n_probes, y.device)
    _check(lib().gp_stoch_grad_pc(h.ptr, _data(X), _ptr(psi), _ptr(y), _ptr(R), int(n_probes),
                                  int(probe_kind), ctypes.byref(params), ctypes.byref(pc.c), _ptr(S_warm),
                                  _ptr(g), _ptr(stats), _stream(stream)))
    return g, stats


def make_shift_precond(delta, eps_inner=0.0, max_inner=10, prec_inner=GP_FP32):
    """J = K + delta I applied by an inner CG (eps_inner relative, at most max_inner steps)."""
    return gp_shift_precond(float(delta), float(eps_inner), int(max_inner), int(prec_inner))


def ulisse_solve_shift_pc(h, X, psi, B, params, sp, S0=None, S_tilde=None, S_cg=None, stats=None,
                          stream=None):
    import torch
    n = X.shape[0]
    m = _cols(B)
    mt = m + (1 if params.two_track_first else 0)
    if S_tilde is None:
        S_tilde = torch.zeros((mt, n), dtype=torch.float64, device=B.device).t()
    if stats is None:
        stats = stats_tensor(m, B.device)
    _check(lib().ulisse_solve_shift_pc(h.ptr, _data(X), _ptr(psi), _ptr(B), m, _ld(B, n), _ptr(S0),
                                       ctypes.byref(params), ctypes.byref(sp), _ptr(S_tilde), _ptr(S_cg),
                                       _ptr(stats), _stream(stream)))
    return S_tilde, stats


def gp_stoch_grad_shift_pc(h, X, psi, y, params, sp, R=None, n_probes=None, probe_kind=PROBE_GAUSSIAN,
                           S_warm=None, g=None, stats=None, stream=None):
    import torch
    d = X.shape[1]
    if R is not None:
        n_probes = _cols(R)
    if g is None:
        g = torch.zeros(d + 2, dtype=torch.float64, device=y.device)
    if stats is None:
        stats = stats_tensor(1 + n_probes, y.device)
    _check(lib().gp_stoch_grad_shift_pc(h.ptr, _data(X), _ptr(psi), _ptr(y), _ptr(R), int(n_probes),
                                        int(probe_kind), ctypes.byref(params), ctypes.byref(sp),
                                        _ptr(S_warm), _ptr(g), _ptr(stats), _stream(stream)))
    return g, stats


# ---------------------------------------------------------------------------------------
# Learned warm start and preconditioner
# ---------------------------------------------------------------------------------------
def mlp_layout(n_in, hidden, n_out):
    """Float offsets of the parameter buffer (the library's layout)."""
    o = {}
    o["W1"] = 0
    o["b1"] = o["W1"] + n_in * hidden
    o["W2"] = o["b1"] + hidden
    o["b2"] = o["W2"] + hidden * hidden
    o["W3"] = o["b2"] + hidden
    o["b3"] = o["W3"] + hidden * n_out
    o["trainable"] = o["b3"] + n_out
    o["in_mu"] = o["trainable"]
    o["in_sd"] = o["in_mu"] + n_in
    o["out_mu"] = o["in_sd"] + n_in
    o["out_sd"] = o["out_mu"] + n_out
    o["total"] = o["out_sd"] + n_out
    return o


def precond_mlp_size(n_in, hidden, n_out):
    return int(lib().precond_mlp_size(n_in, hidden, n_out))


def precond_build_basis(h, X, psi_ref, k, U=None, ritz=None, stream=None):
    import torch
    n = X.shape[0]
    if U is None:
        U = colmajor(n, k)
    if ritz is None:
        ritz = torch.zeros(k, dtype=torch.float64, device=X.device)
    _check(lib().precond_build_basis(h.ptr, _data(X), _ptr(psi_ref), int(k), _ptr(U), _ld(U, n), _ptr(ritz),
                                     _stream(stream)))
    return U, ritz


def precond_targets(h, X, y, U, psis, targets=None, stream=None):
    import torch
    n, k = U.shape
    N = psis.shape[0]
    if targets is None:
        targets = torch.zeros((N, 2 * k + 1), dtype=torch.float32, device=X.device)
    _check(lib().precond_targets(h.ptr, _data(X), _ptr(y), _ptr(U), _ld(U, n), int(k), _ptr(psis), int(N),
                                 _ptr(targets), _stream(stream)))
    return targets


def precond_mlp_init(h, params, n_in, hidden, n_out, psis, targets, seed=0, stream=None):
    _check(lib().precond_mlp_init(h.ptr, _ptr(params), n_in, hidden, n_out, _ptr(psis), _ptr(targets),
                                  psis.shape[0], int(seed), _stream(stream)))


def precond_mlp_train(h, params, adam, n_in, hidden, n_out, psis, targets, steps, first_step=0, lr=1e-3,
                      loss_trace=None, stream=None):
    _check(lib().precond_mlp_train(h.ptr, _ptr(params), _ptr(adam), n_in, hidden, n_out, _ptr(psis),
                                   _ptr(targets), psis.shape[0], int(steps), int(first_step), float(lr),
                                   _ptr(loss_trace), _stream(stream)))


def precond_mlp_forward(h, params, n_in, hidden, n_out, psis, bf16=False, Y=None, stream=None):
    import torch
    B = psis.shape[0]
    if Y is None:
        Y = torch.zeros((B, n_out), dtype=torch.float32, device=psis.device)
    _check(lib().precond_mlp_forward(h.ptr, _ptr(params), n_in, hidden, n_out, _ptr(psis), B, _ptr(Y),
                                     int(bool(bf16)), _stream(stream)))
    return Y


def precond_mlp_grad(h, params, n_in, hidden, n_out, psis, targets, stream=None):
    import torch
    lay = mlp_layout(n_in, hidden, n_out)
    grad = torch.zeros(lay["trainable"], dtype=torch.float32, device=psis.device)
    loss = torch.zeros(1, dtype=torch.float32, device=psis.device)
    _check(lib().precond_mlp_grad(h.ptr, _ptr(params), n_in, hidden, n_out, _ptr(psis), _ptr(targets),
                                  psis.shape[0], _ptr(grad), _ptr(loss), _stream(stream)))
    return loss, grad


def precond_from_mlp(h, params, n_in, hidden, n_out, psi, k, coef=None, c=None, stream=None):
    import torch
    if coef is None:
        coef = torch.zeros(k + 1, dtype=torch.float64, device=psi.device)
    _check(lib().precond_from_mlp(h.ptr, _ptr(params), n_in, hidden, n_out, _ptr(psi), int(k), _ptr(coef),
                                  _ptr(c), _stream(stream)))
    return coef


def precond_from_targets(h, targets, k, coef=None, c=None, stream=None):
    """coef (and c) from one row of precond_targets: the Galerkin preconditioner at that psi."""
    import torch
    if coef is None:
        coef = torch.zeros(k + 1, dtype=torch.float64, device=targets.device)
    _check(lib().precond_from_targets(h.ptr, _ptr(targets), int(k), _ptr(coef), _ptr(c), _stream(stream)))
    return coef


def precond_warm_start(h, U, c, s0, stream=None):
    n, k = U.shape
    _check(lib().precond_warm_start(h.ptr, _ptr(U), _ld(U, n), int(k), int(n), _ptr(c), _ptr(s0),
                                    _stream(stream)))
    return s0


# ---------------------------------------------------------------------------------------
# Autotuner and batched SGLD
# ---------------------------------------------------------------------------------------
def gp_autotune(h, enable):
    _check(lib().gp_autotune(h.ptr, int(enable)))


def gp_autotune_split(h, n, d, m, prec=GP_FP32):
    out = c_int32(0)
    _check(lib().gp_autotune_split(h.ptr, int(n), int(d), int(m), int(prec), ctypes.byref(out)))
    return out.value


PIPE_PROBE_KERNELS = ("valu_fma128", "mfma_f32_x4", "mfma_f32_x4+valu_fma128", "mfma_bf16_x4",
                      "mfma_bf16_x4+valu_fma128", "exp128")


def gp_pipe_probe(h, iters=2000, stream=None):
    """{kernel: (ms, cycles per loop iteration per wave)} for the six probe kernels."""
    ms, cyc = (c_double * 6)(), (c_double * 6)()
    _check(lib().gp_pipe_probe(h.ptr, int(iters), ms, cyc, _stream(stream)))
    return {k: (ms[i], cyc[i]) for i, k in enumerate(PIPE_PROBE_KERNELS)}


SHAPE_SYM = 0  # shape code of the symmetric product; c > 0: split-K for about c workgroups


def gp_tune_set(h, n, d, m, code, prec=GP_FP32):
    """Pin the product shape code of (n, d, m, prec) on h (code -1 removes the pin)."""
    _check(lib().gp_tune_set(h.ptr, int(n), int(d), int(m), int(prec), int(code)))


def gp_tune_get(h, n, d, m, prec=GP_FP32):
    """(code, split) a product of that shape takes now; code -1 = not tuned yet."""
    code, split = c_int32(0), c_int32(0)
    _check(lib().gp_tune_get(h.ptr, int(n), int(d), int(m), int(prec), ctypes.byref(code), ctypes.byref(split)))
    return code.value, split.value


def gp_shape_query(n, d, m, prec=GP_FP32, code=-1):
    """(code, split, mp, partial_floats) of a product's shape, default or of `code`; no
    handle and no device needed."""
    c, sp, mp, pf = c_int32(0), c_int32(0), c_int32(0), c_int64(0)
    _check(lib().gp_shape_query(int(n), int(d), int(m), int(prec), int(code), ctypes.byref(c),
                                ctypes.byref(sp), ctypes.byref(mp), ctypes.byref(pf)))
    return c.value, sp.value, mp.value, pf.value


def gp_tune_save(h, path):
    _check(lib().gp_tune_save(h.ptr, os.fsencode(path)))


def gp_tune_load(h, path):
    _check(lib().gp_tune_load(h.ptr, os.fsencode(path)))


class Batch:
    """B independent SGLD chains over their own GPs, stepped together (gp_batch_*).

    problems: list of dicts with device tensors X (n, d) FP32, y (n,) FP32, psi (d + 2) FP64;
    optional M_chol ((d + 2) x (d + 2) FP64, column-major), prior (kind, a, b).  The batch
    allocates S_warm, R, g and stats per chain and keeps every tensor alive.
    """

    def __init__(self, problems, n_probes, params, seed=0, probe_kind=PROBE_GAUSSIAN, probe_period=20,
                 iters_per_graph=8, autotune=True, streams=8, device=0):
        import torch
        self.keep = []
        descs = (gp_batch_problem * len(problems))()
        self.chains = []
        for i, pr in enumerate(problems):
            X, y, psi = pr["X"], pr["y"], pr["psi"]
            n, d = X.shape
            S_warm = torch.zeros((1 + n_probes, n), dtype=torch.float64, device=X.device).t()
            R = colmajor(n, n_probes, device=X.device)
            g = torch.zeros(d + 2, dtype=torch.float64, device=X.device)
            st = stats_tensor(1 + n_probes, X.device)
            kind, a, b = pr.get("prior", (0, None, None))
            M = pr.get("M_chol")
            chain = {"X": X, "y": y, "psi": psi, "S_warm": S_warm, "R": R, "g": g, "stats": st,
                     "M_chol": M, "a": a, "b": b}
            self.chains.append(chain)
            addr = lambda t: 0 if t is None else t.data_ptr()
            lr = pr.get("learned")
            if lr is not None:
                # keys: mlp (trained parameters), hidden, U (basis, n x k column-major), coef
                # (k + 1 FP64, rewritten every step)
                chain["learned"] = lr
                descs[i] = gp_batch_problem(_data(X), addr(y), addr(psi), addr(S_warm), addr(R), addr(g),
                                            addr(st), addr(M), gp_prior(int(kind), 0, addr(a), addr(b)),
                                            addr(lr["mlp"]), int(lr["hidden"]), lr["U"].shape[1],
                                            addr(lr["U"]), _ld(lr["U"], n), addr(lr["coef"]))
            else:
                descs[i] = gp_batch_problem(_data(X), addr(y), addr(psi), addr(S_warm), addr(R), addr(g),
                                            addr(st), addr(M), gp_prior(int(kind), 0, addr(a), addr(b)))
        self.params = params
        ptr = c_void_p()
        _check(lib().gp_batch_create(ctypes.byref(ptr), device, seed, len(problems), descs, n_probes,
                                     probe_kind, probe_period, ctypes.byref(params), iters_per_graph,
                                     int(bool(autotune)), streams))
        self.ptr = ptr.value

    def step(self, t, eps_t, stream=None):
        _check(lib().gp_batch_step(self.ptr, int(t), float(eps_t), _stream(stream)))

    def stats(self):
        out = gp_batch_stats()
        _check(lib().gp_batch_read_stats(self.ptr, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in gp_batch_stats._fields_}

    def close(self):
        if getattr(self, "ptr", None):
            lib().gp_batch_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
