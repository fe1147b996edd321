"""Thin ctypes binding of ``libadmmdeconv.so`` (declared in include/admm_deconv.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device arrays are torch tensors on the current HIP device (float32,
contiguous); the binding passes their data pointers and the current torch
stream. There is no CPU fallback: if the library is not built, loading it
raises.
"""

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int32, c_uint8, c_uint32, c_void_p, c_char_p

import numpy as np

__all__ = [
    "ADMM_OK", "ADMM_E_INVALID", "ADMM_E_UNSUPPORTED", "ADMM_E_SINGULAR", "ADMM_E_NOMEM",
    "ADMM_E_DEVICE", "ADMM_E_DIVERGED", "ADMM_REG_TV", "ADMM_REG_FRAME", "ADMM_REG_FRAME_SYNTHESIS",
    "ADMM_METHOD_MD", "ADMM_METHOD_CG",
    "ADMM_FLAG_GRAPH",
    "ADMM_FLAG_PROFILE", "admm_plan_kernel_times",
    "AdmmError", "lib", "lib_path", "exported_symbols",
    "admm_deconv_plan", "admm_deconv_solve", "admm_deconv_batch", "admm_deconv_blur",
    "admm_deconv_solve_static", "admm_warmstart_map", "admm_plan_destroy", "admm_last_error", "admm_fft_radices",
    "admm_validate_problem", "admm_fft_schedule", "admm_deconv_plan_with", "admm_plan_schedules",
    "admm_embed_size", "admm_embed_observation",
    "Plan", "make_problem", "alloc_state",
]

ADMM_OK, ADMM_E_INVALID, ADMM_E_UNSUPPORTED, ADMM_E_SINGULAR, ADMM_E_NOMEM, ADMM_E_DEVICE, ADMM_E_DIVERGED = range(7)
ADMM_REG_TV, ADMM_REG_FRAME, ADMM_REG_FRAME_SYNTHESIS = 0, 1, 2
_REGS = {"tv": ADMM_REG_TV, "frame": ADMM_REG_FRAME, "synthesis": ADMM_REG_FRAME_SYNTHESIS}
ADMM_METHOD_MD, ADMM_METHOD_CG = 0, 1
ADMM_FLAG_GRAPH = 1
ADMM_FLAG_PROFILE = 2

_STATUS = {0: "OK", 1: "INVALID", 2: "UNSUPPORTED", 3: "SINGULAR", 4: "NOMEM", 5: "DEVICE", 6: "DIVERGED"}


class AdmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class admm_problem(ctypes.Structure):
    _fields_ = [("H", c_int32), ("W", c_int32), ("ksize", c_int32),
                ("kernel", POINTER(c_float)), ("mask", POINTER(c_uint8)),
                ("reg", c_int32), ("levels", c_int32),
                ("lam", c_double), ("mu1", c_double), ("mu2", c_double), ("method", c_int32)]


class admm_opts(ctypes.Structure):
    _fields_ = [("max_iters", c_int32), ("tol", c_double), ("check_every", c_int32), ("flags", c_uint32),
                ("obj_tol", c_double)]


class admm_info(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("converged", c_int32), ("diverged", c_int32), ("reserved", c_int32),
                ("r_pri", c_double), ("r_dual", c_double), ("objective", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k in ("iters", "converged", "diverged", "r_pri", "r_dual", "objective")}


class admm_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 16), ("launches", c_int32), ("reserved", c_int32), ("total_ms", c_double)]


class admm_tiles(ctypes.Structure):
    _fields_ = [("cols_per_block", c_int32), ("rows_per_block", c_int32), ("row_schedule", c_int32),
                ("col_schedule", c_int32)]


class admm_state(ctypes.Structure):
    _fields_ = [("u1", c_void_p), ("d1", c_void_p), ("ureg", c_void_p), ("dreg", c_void_p)]


_LIB = None


def lib_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "libadmmdeconv.so")


def lib():
    """Load the HIP library (raises if it has not been built).

    torch is imported first: its HIP runtime then provides the library's
    libamdhip64 (same soname), so the process has one HIP runtime and torch's
    device pointers and streams are valid in the library's calls."""
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_1210_2687_amd.build`")
        try:
            import torch  # noqa: F401  (loads the process's HIP runtime)
        except ImportError:
            pass
        L = ctypes.CDLL(path)
        L.admm_deconv_plan.argtypes = [POINTER(admm_problem), c_int32, c_void_p, POINTER(c_void_p)]
        L.admm_deconv_solve.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(admm_state), POINTER(admm_opts),
                                        POINTER(admm_info)]
        L.admm_deconv_batch.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(admm_state),
                                        POINTER(admm_opts), POINTER(admm_info)]
        L.admm_deconv_solve_static.argtypes = [POINTER(admm_problem), c_void_p, c_void_p, POINTER(admm_state),
                                               POINTER(admm_opts), POINTER(admm_info), c_void_p]
        L.admm_deconv_blur.argtypes = [c_void_p, c_int32, c_void_p, c_void_p]
        L.admm_warmstart_map.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, POINTER(admm_state)]
        L.admm_warmstart_dual.argtypes = [c_void_p, c_int32, c_void_p, c_void_p]
        L.admm_plan_destroy.argtypes = [c_void_p]
        L.admm_plan_destroy.restype = None
        L.admm_last_error.restype = c_char_p
        L.admm_fft_radices.argtypes = [c_int32, POINTER(c_int32), c_int32]
        L.admm_validate_problem.argtypes = [POINTER(admm_problem)]
        L.admm_embed_size.argtypes = [c_int32, c_int32, c_int32, POINTER(c_int32), POINTER(c_int32)]
        L.admm_embed_observation.argtypes = [POINTER(c_float), POINTER(c_uint8), c_int32, c_int32, c_int32, c_int32,
                                             c_int32, POINTER(c_float), POINTER(c_uint8)]
        L.admm_plan_kernel_times.argtypes = [c_void_p, POINTER(admm_kernel_time), c_int32]
        L.admm_plan_kernel_times.restype = c_int32
        L.admm_deconv_plan_tuned.argtypes = [POINTER(admm_problem), c_int32, c_void_p, c_char_p, POINTER(c_void_p)]
        L.admm_tune_key.argtypes = [POINTER(admm_problem), c_int32, c_char_p, c_char_p, ctypes.c_size_t]
        L.admm_tune_key.restype = c_int32
        L.admm_tune_cache_lookup.argtypes = [c_char_p, c_char_p, POINTER(c_int32), POINTER(c_int32)]
        L.admm_tune_cache_lookup.restype = c_int32
        L.admm_tune_cache_store.argtypes = [c_char_p, c_char_p, c_int32, c_int32, c_double, c_double]
        L.admm_plan_tiles.argtypes = [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32)]
        L.admm_plan_schedules.argtypes = [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32)]
        L.admm_deconv_plan_with.argtypes = [POINTER(admm_problem), c_int32, c_void_p, POINTER(admm_tiles),
                                            POINTER(c_void_p)]
        L.admm_fft_schedule.argtypes = [c_int32, c_int32, POINTER(c_int32), c_int32]
        L.admm_plan_time_pass.argtypes = [c_void_p, c_char_p, c_int32, POINTER(c_double)]
        vp = c_void_p
        L.admm_conv3x3_pack_weights.argtypes = [vp, c_int32, c_int32, vp, vp, vp]
        L.admm_conv3x3_bf16_fwd.argtypes = [vp, c_int32, c_int32, c_int32, c_int32, vp, vp, c_int32, c_int32,
                                            vp, vp, c_int32, vp]
        L.admm_conv3x3_bf16_wgrad_workspace.argtypes = [c_int32] * 6
        L.admm_conv3x3_bf16_wgrad_workspace.restype = ctypes.c_size_t
        L.admm_conv3x3_bf16_wgrad.argtypes = [vp, vp, c_int32, c_int32, c_int32, c_int32, c_int32, c_int32, vp,
                                              ctypes.c_size_t, vp, vp, c_int32, vp]
        L.admm_adam_step.argtypes = [vp, vp, vp, vp, c_int32, c_float, c_float, c_float, c_float, c_int32, vp]
        L.admm_ws_input.argtypes = [vp, vp, vp, c_int32, c_int32, c_int32, vp, vp]
        L.admm_ws_loss.argtypes = [vp, vp, vp, vp, vp, c_int32, c_int32, c_int32, c_float, vp, vp, vp]
        L.admm_ws_output.argtypes = [vp, vp, vp, c_int32, c_int32, c_int32, vp, vp, vp]
        for f in ("admm_deconv_plan", "admm_deconv_plan_tuned", "admm_tune_cache_store", "admm_plan_tiles",
                  "admm_plan_schedules", "admm_deconv_plan_with", "admm_fft_schedule",
                  "admm_plan_time_pass",
                  "admm_deconv_solve", "admm_deconv_batch", "admm_deconv_blur", "admm_deconv_solve_static",
                  "admm_warmstart_map", "admm_warmstart_dual", "admm_fft_radices", "admm_validate_problem",
                  "admm_conv3x3_pack_weights", "admm_conv3x3_bf16_fwd", "admm_conv3x3_bf16_wgrad",
                  "admm_adam_step", "admm_ws_input", "admm_ws_loss", "admm_ws_output"):
            getattr(L, f).restype = c_int32
        _LIB = L
    return _LIB


def exported_symbols():
    """Names of the C entry points declared in include/admm_deconv.h."""
    return ["admm_deconv_plan", "admm_deconv_solve", "admm_deconv_batch", "admm_deconv_blur",
            "admm_deconv_solve_static",
            "admm_warmstart_map", "admm_warmstart_dual", "admm_plan_destroy", "admm_last_error", "admm_fft_radices",
            "admm_validate_problem", "admm_plan_kernel_times", "admm_deconv_plan_tuned", "admm_tune_key",
            "admm_tune_cache_lookup", "admm_tune_cache_store", "admm_plan_tiles", "admm_plan_time_pass",
            "admm_deconv_plan_with", "admm_plan_schedules", "admm_fft_schedule",
            "admm_embed_size", "admm_embed_observation",
            "admm_conv3x3_pack_weights", "admm_conv3x3_bf16_fwd", "admm_conv3x3_bf16_wgrad_workspace",
            "admm_conv3x3_bf16_wgrad", "admm_adam_step", "admm_ws_input", "admm_ws_loss", "admm_ws_output"]


def admm_last_error():
    return lib().admm_last_error().decode()


def _check(status):
    if status != ADMM_OK:
        raise AdmmError(status, admm_last_error())


def admm_fft_radices(n):
    buf = (c_int32 * 16)()
    k = lib().admm_fft_radices(n, buf, 16)
    return None if k < 0 else list(buf[:k])


def make_problem(kernel, mask, lam, mu1=-1.0, mu2=-1.0, reg=ADMM_REG_TV, levels=0, method=None):
    """Host-side problem description; keeps the host arrays alive with it.
    method: ADMM_METHOD_MD (default, mask decoupling) or ADMM_METHOD_CG (the
    Reeves-Sorel variants TV-CG / FA-CG)."""
    kernel = np.ascontiguousarray(kernel, dtype=np.float32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    p = admm_problem()
    p.H, p.W = mask.shape
    p.ksize = kernel.shape[0]
    p.kernel = kernel.ctypes.data_as(POINTER(c_float))
    p.mask = mask.ctypes.data_as(POINTER(c_uint8))
    p.reg = reg
    p.levels = levels
    p.lam, p.mu1, p.mu2 = float(lam), float(mu1), float(mu2)
    p.method = ADMM_METHOD_MD if method is None else int(method)
    p._keep = (kernel, mask)
    return p


def admm_fft_schedule(n, variant):
    buf = (c_int32 * 16)()
    k = lib().admm_fft_schedule(n, variant, buf, 16)
    return None if k < 0 else list(buf[:k])


def admm_validate_problem(prob):
    return lib().admm_validate_problem(ctypes.byref(prob))


def admm_embed_size(obs_h, obs_w, ksize):
    """(H, W): the smallest 7-smooth unknown domain holding an obs_h x obs_w
    observation blurred by a ksize x ksize kernel."""
    H, W = c_int32(), c_int32()
    _check(lib().admm_embed_size(int(obs_h), int(obs_w), int(ksize), ctypes.byref(H), ctypes.byref(W)))
    return H.value, W.value


def admm_embed_observation(y_obs, ksize, obs_mask=None, shape=None):
    """(y, mask) on the unknown domain ``shape`` (default: admm_embed_size) with
    the observation at rows / columns ksize // 2 onwards."""
    y_obs = np.ascontiguousarray(y_obs, dtype=np.float32)
    oh, ow = y_obs.shape
    H, W = shape if shape is not None else admm_embed_size(oh, ow, ksize)
    y = np.empty((H, W), np.float32)
    m = np.empty((H, W), np.uint8)
    om = None if obs_mask is None else np.ascontiguousarray(obs_mask, dtype=np.uint8)
    _check(lib().admm_embed_observation(y_obs.ctypes.data_as(POINTER(c_float)),
                                        None if om is None else om.ctypes.data_as(POINTER(c_uint8)),
                                        oh, ow, int(ksize), H, W, y.ctypes.data_as(POINTER(c_float)),
                                        m.ctypes.data_as(POINTER(c_uint8))))
    return y, m


def _stream_ptr(stream):
    if stream is not None:
        return c_void_p(stream)
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def admm_deconv_plan(problems, stream=None):
    """Plan a list of problems (see ``make_problem``); returns an opaque handle."""
    arr = (admm_problem * len(problems))(*problems)
    out = c_void_p()
    _check(lib().admm_deconv_plan(arr, len(problems), _stream_ptr(stream), ctypes.byref(out)))
    return out


def admm_deconv_plan_tuned(problems, stream=None, cache_path=None):
    """Plan with tile shapes chosen by the autotuner (optionally cached in a JSON file)."""
    arr = (admm_problem * len(problems))(*problems)
    out = c_void_p()
    cp = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().admm_deconv_plan_tuned(arr, len(problems), _stream_ptr(stream), cp, ctypes.byref(out)))
    return out


def admm_deconv_plan_with(problems, cols_per_block=0, rows_per_block=0, row_schedule=0, col_schedule=0,
                          stream=None):
    """Plan with explicit tile shapes and radix schedule variants."""
    arr = (admm_problem * len(problems))(*problems)
    t = admm_tiles(int(cols_per_block), int(rows_per_block), int(row_schedule), int(col_schedule))
    out = c_void_p()
    _check(lib().admm_deconv_plan_with(arr, len(problems), _stream_ptr(stream), ctypes.byref(t), ctypes.byref(out)))
    return out


def admm_plan_schedules(plan, index):
    r, c = c_int32(), c_int32()
    _check(lib().admm_plan_schedules(plan, index, ctypes.byref(r), ctypes.byref(c)))
    return r.value, c.value


def admm_tune_key(problems, arch):
    arr = (admm_problem * len(problems))(*problems)
    buf = ctypes.create_string_buffer(512)
    n = lib().admm_tune_key(arr, len(problems), arch.encode(), buf, 512)
    if n < 0:
        raise AdmmError(ADMM_E_INVALID, "bad key request")
    return buf.value.decode()


def admm_tune_cache_lookup(path, key):
    """(tc, rows) for key, None if absent; raises on a malformed file."""
    tc, rows = c_int32(), c_int32()
    r = lib().admm_tune_cache_lookup(os.fsencode(path), key.encode(), ctypes.byref(tc), ctypes.byref(rows))
    if r < 0:
        raise AdmmError(ADMM_E_INVALID, f"malformed tuning cache {path}")
    return (tc.value, rows.value) if r == 1 else None


def admm_tune_cache_store(path, key, tc, rows, col_us=0.0, row_us=0.0):
    _check(lib().admm_tune_cache_store(os.fsencode(path), key.encode(), tc, rows, col_us, row_us))


def admm_plan_tiles(plan, index):
    tc, rows = c_int32(), c_int32()
    _check(lib().admm_plan_tiles(plan, index, ctypes.byref(tc), ctypes.byref(rows)))
    return tc.value, rows.value


def admm_plan_time_pass(plan, kernel, reps=50):
    """Average milliseconds of one launch of a pass kernel over `reps` back-to-back launches."""
    out = c_double()
    _check(lib().admm_plan_time_pass(plan, kernel.encode(), int(reps), ctypes.byref(out)))
    return out.value


def admm_plan_destroy(plan):
    lib().admm_plan_destroy(plan)


def _dev(t, n=None):
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError("expected a contiguous float32 tensor on the GPU")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return c_void_p(t.data_ptr())


def _state(st, n, R):
    if st is None:
        return None
    s = admm_state()
    s.u1, s.d1 = _dev(st["u1"], n), _dev(st["d1"], n)
    s.ureg, s.dreg = _dev(st["ureg"], R * n), _dev(st["dreg"], R * n)
    return s


def _opts(max_iters, tol, check_every, graph, profile=False, obj_tol=0.0):
    o = admm_opts()
    o.max_iters, o.tol, o.check_every = int(max_iters), float(tol), int(check_every)
    o.obj_tol = float(obj_tol)
    o.flags = (ADMM_FLAG_GRAPH if graph else 0) | (ADMM_FLAG_PROFILE if profile else 0)
    return o


def admm_deconv_solve(plan, y, x, state=None, max_iters=100, tol=0.0, check_every=10, graph=False,
                      profile=False, nreg=2, obj_tol=0.0):
    n = y.numel()
    info = admm_info()
    st = _state(state, n, nreg)
    _check(lib().admm_deconv_solve(plan, _dev(y), _dev(x, n), ctypes.byref(st) if st else None,
                                   ctypes.byref(_opts(max_iters, tol, check_every, graph, profile, obj_tol)),
                                   ctypes.byref(info)))
    return info.as_dict()


def admm_deconv_solve_static(problem, y, x, state=None, max_iters=100, tol=0.0, check_every=10, nreg=2,
                             stream=None, obj_tol=0.0):
    """Plan and solve one problem (``make_problem``) in the library's static
    device workspace, allocating nothing."""
    n = y.numel()
    info = admm_info()
    st = _state(state, n, nreg)
    _check(lib().admm_deconv_solve_static(ctypes.byref(problem), _dev(y), _dev(x, n),
                                          ctypes.byref(st) if st else None,
                                          ctypes.byref(_opts(max_iters, tol, check_every, False, False, obj_tol)),
                                          ctypes.byref(info), _stream_ptr(stream)))
    return info.as_dict()


def admm_deconv_batch(plan, ys, xs, states=None, max_iters=100, tol=0.0, check_every=10, graph=False,
                      profile=False, nregs=None, raise_on_diverged=True, obj_tol=0.0):
    cnt = len(ys)
    yp = (c_void_p * cnt)(*[_dev(t) for t in ys])
    xp = (c_void_p * cnt)(*[_dev(t, ys[i].numel()) for i, t in enumerate(xs)])
    sts = None
    if states is not None:
        nregs = nregs or [2] * cnt
        sts = (admm_state * cnt)(*[_state(s, ys[i].numel(), nregs[i]) for i, s in enumerate(states)])
    infos = (admm_info * cnt)()
    status = lib().admm_deconv_batch(plan, yp, xp, sts,
                                     ctypes.byref(_opts(max_iters, tol, check_every, graph, profile, obj_tol)),
                                     infos)
    if status != ADMM_OK and not (status == ADMM_E_DIVERGED and not raise_on_diverged):
        _check(status)
    return [i.as_dict() for i in infos]


def admm_plan_kernel_times(plan):
    """{class: (launches, total_ms)} of the last run made with profile=True."""
    buf = (admm_kernel_time * 8)()
    k = lib().admm_plan_kernel_times(plan, buf, 8)
    return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(min(k, 8))}


# ---------------------------------------------------------------- learned warm start
def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def admm_conv3x3_pack_weights(w, cin, cout, wfwd, wbwd=None):
    _check(lib().admm_conv3x3_pack_weights(_ptr(w), cin, cout, _ptr(wfwd), _ptr(wbwd), _stream()))


def admm_conv3x3_bf16_fwd(x, N, H, W, cin, wpacked, bias, cout, relu, gate, y, dil=1):
    _check(lib().admm_conv3x3_bf16_fwd(_ptr(x), N, H, W, cin, _ptr(wpacked), _ptr(bias), cout, int(relu),
                                       _ptr(gate), _ptr(y), int(dil), _stream()))


def admm_conv3x3_bf16_wgrad_workspace(N, H, W, cin, cout, chunk):
    return lib().admm_conv3x3_bf16_wgrad_workspace(N, H, W, cin, cout, chunk)


def admm_conv3x3_bf16_wgrad(x, dy, N, H, W, cin, cout, chunk, workspace, dw, db, dil=1):
    _check(lib().admm_conv3x3_bf16_wgrad(_ptr(x), _ptr(dy), N, H, W, cin, cout, chunk, _ptr(workspace),
                                         workspace.numel() * workspace.element_size(), _ptr(dw), _ptr(db),
                                         int(dil), _stream()))


def admm_adam_step(p, g, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().admm_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), lr, beta1, beta2, eps, int(t),
                                _stream()))


def admm_ws_input(y, mask, emb, N, H, W, x0):
    _check(lib().admm_ws_input(_ptr(y), _ptr(mask), _ptr(emb), N, H, W, _ptr(x0), _stream()))


def admm_ws_loss(out, y, mask, xt, pt, N, H, W, alpha, dout, lpart):
    _check(lib().admm_ws_loss(_ptr(out), _ptr(y), _ptr(mask), _ptr(xt), _ptr(pt), N, H, W, alpha, _ptr(dout),
                              _ptr(lpart), _stream()))


def admm_ws_output(out, y, mask, N, H, W, x0, p0):
    _check(lib().admm_ws_output(_ptr(out), _ptr(y), _ptr(mask), N, H, W, _ptr(x0), _ptr(p0), _stream()))


def admm_deconv_blur(plan, index, x, Ax):
    _check(lib().admm_deconv_blur(plan, int(index), _dev(x), _dev(Ax, x.numel())))


def admm_warmstart_map(plan, index, x0, p0, y, state):
    n = x0.numel()
    st = _state(state, n, 2)
    _check(lib().admm_warmstart_map(plan, int(index), _dev(x0, n), _dev(p0, 2 * n), _dev(y, n),
                                    ctypes.byref(st)))


def admm_warmstart_dual(plan, index, dreg, p0):
    n = p0.numel()
    _check(lib().admm_warmstart_dual(plan, int(index), _dev(dreg, n), _dev(p0, n)))


def alloc_state(H, W, nreg=2, device="cuda"):
    """Zero ADMM state planes (u1, d1: H x W; ureg, dreg: nreg x H x W)."""
    import torch
    z = lambda *s: torch.zeros(*s, dtype=torch.float32, device=device)
    return {"u1": z(H, W), "d1": z(H, W), "ureg": z(nreg, H, W), "dreg": z(nreg, H, W)}


class Plan:
    """Convenience owner of a plan handle built from ``workloads.Problem``-like objects."""

    def __init__(self, problems, stream=None, tune=False, cache_path=None, tiles=None, method=ADMM_METHOD_MD):
        self.problems = list(problems)
        self._cprobs = []
        for p in self.problems:
            reg = _REGS[getattr(p, "reg", "tv")]
            self._cprobs.append(make_problem(p.kernel, p.mask, p.lam, p.mu1, p.mu2, reg, getattr(p, "levels", 0),
                                             method))
        self.nregs = [2 if getattr(p, "reg", "tv") == "tv" else 3 * p.levels + 1 for p in self.problems]
        if tiles is not None:
            self.handle = admm_deconv_plan_with(self._cprobs, stream=stream, **tiles)
        elif tune:
            self.handle = admm_deconv_plan_tuned(self._cprobs, stream, cache_path)
        else:
            self.handle = admm_deconv_plan(self._cprobs, stream)

    def solve(self, y, x, state=None, **kw):
        return admm_deconv_solve(self.handle, y, x, state, nreg=self.nregs[0], **kw)

    def batch(self, ys, xs, states=None, **kw):
        return admm_deconv_batch(self.handle, ys, xs, states, nregs=self.nregs, **kw)

    def blur(self, index, x, Ax):
        admm_deconv_blur(self.handle, index, x, Ax)

    def kernel_times(self):
        return admm_plan_kernel_times(self.handle)

    def tiles(self, index=0):
        return admm_plan_tiles(self.handle, index)

    def schedules(self, index=0):
        return admm_plan_schedules(self.handle, index)

    def time_pass(self, kernel, reps=50):
        return admm_plan_time_pass(self.handle, kernel, reps)

    def warmstart_map(self, index, x0, p0, y, state):
        admm_warmstart_map(self.handle, index, x0, p0, y, state)

    def warmstart_dual(self, index, dreg, p0):
        admm_warmstart_dual(self.handle, index, dreg, p0)

    def close(self):
        if self.handle:
            admm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
