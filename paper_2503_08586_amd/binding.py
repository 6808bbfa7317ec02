"""ctypes binding of the lens likelihood C ABI (include/lens_api.h).

Argument marshalling only: every step of the likelihood runs in the HIP
kernels of liblens_mi355x.so.  The module-level functions carry the C names;
``LensContext`` wraps them for convenience.  torch is imported first so that
its HIP runtime is the one the library binds to; device memory for the
library can come from torch's caching allocator, and the device-buffer entry
point takes torch tensors and streams.

If the library has not been built, ``load()`` raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblens_mi355x.so")
STRIDE = 20
NPARAM = 19

LENS_OK = 0
LENS_PENDING = 1
LENS_EINVAL = -1
LENS_ENOMEM = -2
LENS_ENOENT = -3
LENS_EBUSY = -4
LENS_EAGAIN = -5
LENS_EDEVICE = -6
LENS_ECANCELED = -7
LENS_ETIMEDOUT = -8

LENS_PREC_FP32 = 0
LENS_PREC_F16_SPLIT = 1
LENS_PREC_BF16 = 2
LENS_PREC_BF16_SPLIT3 = 3

LENS_AMP_EXPLICIT = 0
LENS_AMP_NNLS = 1

LENS_MASS_SIE = 0
LENS_MASS_EPL = 1

LENS_LIGHT_BOTH = 0
LENS_LIGHT_LENS = 1
LENS_LIGHT_SOURCE = 2
LENS_LIGHT_DOUBLE = 3

EXPORTED = [
    "lens_init", "lens_shutdown", "lens_load_data", "lens_unload", "lens_get_info",
    "lens_loglike_batch", "lens_loglike_amps", "lens_loglike_batch_device", "lens_loglike_multi",
    "lens_loglike_multi_device", "lens_loglike_batch_device_noalloc",
    "lens_submit", "lens_poll", "lens_wait", "lens_cancel", "lens_get_stats", "lens_reset_stats",
    "lens_model_image", "lens_selftest", "lens_peak_rate", "lens_psf_crop", "lens_strerror", "lens_last_error",
    "lens_ensemble_create", "lens_ensemble_run", "lens_ensemble_run_many", "lens_ensemble_get",
    "lens_ensemble_destroy",
    "lens_philox4x32_10",
]

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class lens_init_opts(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_int64),
        ("max_inflight", ctypes.c_int32),
        ("nonblocking_submit", ctypes.c_int32),
        ("dev_alloc", ALLOC_FN),
        ("dev_free", FREE_FN),
        ("alloc_user", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("autotune", ctypes.c_int32),
    ]


class lens_data_desc(ctypes.Structure):
    _fields_ = [
        ("ny", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("pixel_scale", ctypes.c_double),
        ("supersample", ctypes.c_int32),
        ("psf_size", ctypes.c_int32),
        ("psf", ctypes.POINTER(ctypes.c_double)),
        ("data", ctypes.POINTER(ctypes.c_double)),
        ("sigma", ctypes.POINTER(ctypes.c_double)),
        ("mask", ctypes.POINTER(ctypes.c_uint8)),
        ("precision", ctypes.c_int32),
        ("amplitudes", ctypes.c_int32),
        ("psf_tail", ctypes.c_double),
        ("light_model", ctypes.c_int32),
        ("sersic_n", ctypes.c_double * 4),
        ("mass_model", ctypes.c_int32),
    ]


class lens_info(ctypes.Structure):
    _fields_ = [
        ("ny", ctypes.c_int32), ("nx", ctypes.c_int32), ("supersample", ctypes.c_int32),
        ("psf_size", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("masked_pixels", ctypes.c_int64), ("needed_pixels", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64), ("norm", ctypes.c_double),
        ("strip_rows", ctypes.c_int32), ("threads", ctypes.c_int32), ("lds_bytes", ctypes.c_int64),
        ("blocks_per_cu", ctypes.c_int32), ("psf_used", ctypes.c_int32),
        ("amplitudes", ctypes.c_int32), ("light_model", ctypes.c_int32), ("n_amplitudes", ctypes.c_int32),
        ("mass_model", ctypes.c_int32),
    ]


class lens_ensemble_desc(ctypes.Structure):
    _fields_ = [
        ("walkers", ctypes.c_int32),
        ("stretch", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("lo", ctypes.POINTER(ctypes.c_double)),
        ("hi", ctypes.POINTER(ctypes.c_double)),
        ("init", ctypes.POINTER(ctypes.c_double)),
    ]


class lens_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "requests_submitted", "requests_done", "requests_failed", "requests_canceled",
        "proposals_done", "queued", "inflight", "hbm_budget_bytes", "hbm_used_bytes", "launches",
        "latency_count")] + [(n, ctypes.c_double) for n in ("latency_p50_us", "latency_p99_us", "latency_max_us")] + [
        ("batch_pieces", ctypes.c_int64)]


class LensError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_strerror(status), status, msg))
        self.status = status


_lib = None


def load():
    """Load liblens_mi355x.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblens_mi355x.so is not built; run __graft_entry__.build() "
                           "or python paper_2503_08586_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    sig = {
        "lens_init": ([ctypes.POINTER(lens_init_opts), ctypes.POINTER(vp)], i32),
        "lens_shutdown": ([vp], None),
        "lens_load_data": ([vp, ctypes.POINTER(lens_data_desc), i64p], i32),
        "lens_unload": ([vp, i64], i32),
        "lens_get_info": ([vp, i64, ctypes.POINTER(lens_info)], i32),
        "lens_loglike_batch": ([vp, i64, dp, i64, dp], i32),
        "lens_loglike_amps": ([vp, i64, dp, i64, dp, dp], i32),
        "lens_loglike_batch_device": ([vp, i64, vp, i64, vp, vp], i32),
        "lens_loglike_multi": ([vp, i32, i64p, i64p, dp, dp], i32),
        "lens_loglike_multi_device": ([vp, i32, i64p, i64p, vp, vp, vp], i32),
        "lens_loglike_batch_device_noalloc": ([vp, i64, vp, i64, vp, vp], i32),
        "lens_submit": ([vp, i64, dp, i64, dp, i64p], i32),
        "lens_poll": ([vp, i64], i32),
        "lens_wait": ([vp, i64, i64], i32),
        "lens_cancel": ([vp, i64], i32),
        "lens_get_stats": ([vp, ctypes.POINTER(lens_stats)], i32),
        "lens_reset_stats": ([vp], i32),
        "lens_model_image": ([vp, i64, dp, i32, dp], i32),
        "lens_selftest": ([vp, i32, dp], i32),
        "lens_peak_rate": ([vp, i32, dp], i32),
        "lens_psf_crop": ([dp, i32, ctypes.c_double, ctypes.POINTER(i32)], i32),
        "lens_ensemble_create": ([vp, i64, ctypes.POINTER(lens_ensemble_desc), i64p], i32),
        "lens_ensemble_run": ([vp, i64, i64, i32, dp, dp], i32),
        "lens_ensemble_run_many": ([vp, i32, i64p, i64, i32, ctypes.POINTER(dp), ctypes.POINTER(dp)], i32),
        "lens_ensemble_get": ([vp, i64, dp, dp, i64p, i64p], i32),
        "lens_ensemble_destroy": ([vp, i64], i32),
        "lens_philox4x32_10": ([vp, u32p, u32p, i64, u32p], i32),
        "lens_strerror": ([i32], ctypes.c_char_p),
        "lens_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _strerror(st):
    try:
        return load().lens_strerror(st).decode()
    except Exception:
        return "status"


def _check(ctx, st, ok=(LENS_OK,)):
    if st in ok:
        return st
    msg = load().lens_last_error(ctx).decode() if ctx else ""
    raise LensError(st, msg)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(params) -> np.ndarray:
    p = np.ascontiguousarray(params, dtype=np.float64)
    if p.ndim == 1:
        p = p[None, :]
    if p.shape[1] == NPARAM:
        p = np.concatenate([p, np.zeros((p.shape[0], 1))], axis=1)
    if p.ndim != 2 or p.shape[1] != STRIDE:
        raise ValueError("params must be [n, 19] or [n, 20]")
    return np.ascontiguousarray(p)


# ---------------------------------------------------------------------------
# the C entry points, one Python function each
# ---------------------------------------------------------------------------
class _Hooks:
    """torch caching-allocator hooks handed to lens_init (kept alive with the context)."""

    def __init__(self, device):
        self.device = device

        def _alloc(size, stream, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), self.device, int(stream or 0))
            except Exception:
                return None

        def _free(ptr, stream, user):
            torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


_hooks_by_ctx = {}


def lens_init(device: int = 0, hbm_budget_bytes: int = 0, max_inflight: int = 0,
              nonblocking_submit: bool = False, use_torch_allocator: bool = True,
              stream: Optional[int] = None, autotune: bool = False):
    lib = load()
    o = lens_init_opts()
    o.device = device
    o.hbm_budget_bytes = hbm_budget_bytes
    o.max_inflight = max_inflight
    o.nonblocking_submit = 1 if nonblocking_submit else 0
    hooks = None
    if use_torch_allocator:
        hooks = _Hooks(device)
        o.dev_alloc = hooks.alloc
        o.dev_free = hooks.free
    o.stream = stream
    o.autotune = 1 if autotune else 0
    ctx = ctypes.c_void_p()
    st = lib.lens_init(ctypes.byref(o), ctypes.byref(ctx))
    if st != LENS_OK:
        raise LensError(st, "lens_init failed")
    _hooks_by_ctx[ctx.value] = hooks
    return ctx.value


def lens_shutdown(ctx):
    load().lens_shutdown(ctx)
    _hooks_by_ctx.pop(ctx, None)


def lens_load_data(ctx, ny, nx, pixel_scale, supersample, psf, data, sigma, mask,
                   precision=LENS_PREC_FP32, psf_tail=0.0, amplitudes=0, light_model=0,
                   sersic_n=(1.0, 1.0, 1.0, 1.0), mass_model=0) -> int:
    psf = np.ascontiguousarray(psf, dtype=np.float64)
    data = np.ascontiguousarray(data, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    k = psf.shape[0]
    if psf.shape != (k, k) or data.shape != (ny, nx) or sigma.shape != (ny, nx) or mask.shape != (ny, nx):
        raise ValueError("array shapes do not match ny, nx, psf_size")
    d = lens_data_desc()
    d.ny, d.nx, d.pixel_scale, d.supersample, d.psf_size = ny, nx, pixel_scale, supersample, k
    d.psf, d.data, d.sigma = _dptr(psf), _dptr(data), _dptr(sigma)
    d.mask = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    d.precision = precision
    d.psf_tail = psf_tail
    d.amplitudes = amplitudes
    d.light_model = light_model
    sn = [float(v) for v in sersic_n]
    if len(sn) != 4:
        raise ValueError("sersic_n holds four indices")
    d.sersic_n[:] = sn
    d.mass_model = mass_model
    lid = ctypes.c_int64()
    _check(ctx, load().lens_load_data(ctx, ctypes.byref(d), ctypes.byref(lid)))
    return lid.value


def lens_psf_crop(psf, psf_tail=0.0) -> int:
    """Side of the PSF kernel lens_load_data convolves with after its tail crop (host only)."""
    psf = np.ascontiguousarray(psf, dtype=np.float64)
    k = psf.shape[0]
    out = ctypes.c_int32()
    st = load().lens_psf_crop(_dptr(psf), k, psf_tail, ctypes.byref(out))
    if st != 0:
        raise LensError(st, "lens_psf_crop")
    return out.value


def lens_loglike_amps(ctx, lens_id, params):
    """(lnL [n], amplitudes [n, N]) of every proposal row (host buffers); N is the
    lens's ``n_amplitudes``."""
    p = _params(params)
    info = lens_info()
    _check(ctx, load().lens_get_info(ctx, lens_id, ctypes.byref(info)))
    out = np.empty(p.shape[0], dtype=np.float64)
    amp = np.empty((p.shape[0], info.n_amplitudes), dtype=np.float64)
    _check(ctx, load().lens_loglike_amps(ctx, lens_id, _dptr(p), p.shape[0], _dptr(out), _dptr(amp)))
    return out, amp


def lens_ensemble_create(ctx, lens_id, init, lo, hi, stretch=2.0, seed=0) -> int:
    """A stretch-move ensemble on the device from walkers ``init`` [W, 20] in the box [lo, hi]."""
    w = _params(init)
    lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(STRIDE)
    hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(STRIDE)
    d = lens_ensemble_desc()
    d.walkers = w.shape[0]
    d.stretch = float(stretch)
    d.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    d.lo, d.hi, d.init = _dptr(lo), _dptr(hi), _dptr(w)
    eid = ctypes.c_int64()
    _check(ctx, load().lens_ensemble_create(ctx, lens_id, ctypes.byref(d), ctypes.byref(eid)))
    _ens_sizes[(ctx, eid.value)] = w.shape[0]
    return eid.value


def lens_ensemble_get(ctx, ens):
    """(walkers [W, 20], lnP [W], accepted [W], iterations done)."""
    it = ctypes.c_int64()
    W = _ens_walkers(ctx, ens)
    w = np.empty((W, STRIDE))
    lnp = np.empty(W)
    acc = np.empty(W, dtype=np.int64)
    _check(ctx, load().lens_ensemble_get(ctx, ens, _dptr(w), _dptr(lnp),
                                         acc.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(it)))
    return w, lnp, acc, it.value


_ens_sizes = {}   # (context, ensemble) -> walkers


def _ens_walkers(ctx, ens):
    try:
        return _ens_sizes[(ctx, ens)]
    except KeyError:
        raise LensError(LENS_ENOENT, "unknown ensemble id") from None


def lens_ensemble_run(ctx, ens, iterations, thin=0, chain=False):
    """Advance ``iterations`` iterations on the device; with ``chain`` returns
    (chain [iterations/thin, W, 20], chain_lnp [iterations/thin, W])."""
    if not chain:
        _check(ctx, load().lens_ensemble_run(ctx, ens, int(iterations), int(thin), None, None))
        return None
    thin = max(1, int(thin))
    W = _ens_walkers(ctx, ens)
    ns = int(iterations) // thin
    cw = np.empty((ns, W, STRIDE))
    cl = np.empty((ns, W))
    _check(ctx, load().lens_ensemble_run(ctx, ens, int(iterations), thin, _dptr(cw), _dptr(cl)))
    return cw, cl


def lens_ensemble_run_many(ctx, ens_ids, iterations, thin=0, chain=False):
    """Advance every ensemble of ``ens_ids`` (distinct) by ``iterations``
    iterations together, pooling their proposals into shared launches; with
    ``chain`` returns one (chain [iterations/thin, W, 20], chain_lnp
    [iterations/thin, W]) pair per ensemble."""
    ids = np.ascontiguousarray(np.asarray(ens_ids, dtype=np.int64).reshape(-1))
    ptr = ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if ids.size else None
    if not chain:
        _check(ctx, load().lens_ensemble_run_many(ctx, int(ids.size), ptr, int(iterations), int(thin), None, None))
        return None
    thin = max(1, int(thin))
    ns = int(iterations) // thin
    outs = []
    for e in ids:
        W = _ens_walkers(ctx, int(e))
        outs.append((np.empty((ns, W, STRIDE)), np.empty((ns, W))))
    dp = ctypes.POINTER(ctypes.c_double)
    cw = (dp * max(1, len(outs)))(*[_dptr(a) for a, _ in outs])
    cl = (dp * max(1, len(outs)))(*[_dptr(b) for _, b in outs])
    _check(ctx, load().lens_ensemble_run_many(ctx, int(ids.size), ptr, int(iterations), thin, cw, cl))
    return outs


def lens_ensemble_destroy(ctx, ens):
    _check(ctx, load().lens_ensemble_destroy(ctx, ens))
    _ens_sizes.pop((ctx, ens), None)


def lens_philox4x32_10(ctx, ctr, key, n) -> np.ndarray:
    """Philox4x32-10 words [n, 4] of counters (ctr[0] + i, ctr[1], ctr[2], ctr[3]), computed on the device."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.empty((int(n), 4), dtype=np.uint32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    _check(ctx, load().lens_philox4x32_10(ctx, c.ctypes.data_as(u32p), k.ctypes.data_as(u32p), int(n),
                                          out.ctypes.data_as(u32p)))
    return out


def lens_unload(ctx, lens_id):
    _check(ctx, load().lens_unload(ctx, lens_id))


def lens_get_info(ctx, lens_id) -> dict:
    info = lens_info()
    _check(ctx, load().lens_get_info(ctx, lens_id, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in lens_info._fields_}


def lens_loglike_batch(ctx, lens_id, params) -> np.ndarray:
    p = _params(params)
    out = np.empty(p.shape[0], dtype=np.float64)
    _check(ctx, load().lens_loglike_batch(ctx, lens_id, _dptr(p), p.shape[0], _dptr(out)))
    return out


def lens_loglike_batch_device(ctx, lens_id, params_dev: "torch.Tensor", out_dev: "torch.Tensor",
                              stream: Optional["torch.cuda.Stream"] = None):
    """Device-buffer entry point: params_dev [n, 20] float64 and out_dev [n] float64 on the GPU."""
    if params_dev.dtype != torch.float64 or out_dev.dtype != torch.float64:
        raise TypeError("float64 tensors expected")
    if not (params_dev.is_cuda and out_dev.is_cuda and params_dev.is_contiguous() and out_dev.is_contiguous()):
        raise ValueError("contiguous device tensors expected")
    n = params_dev.shape[0]
    if params_dev.shape != (n, STRIDE) or out_dev.shape != (n,):
        raise ValueError("shapes must be [n, 20] and [n]")
    s = stream if stream is not None else torch.cuda.current_stream(params_dev.device)
    _check(ctx, load().lens_loglike_batch_device(ctx, lens_id, params_dev.data_ptr(), n,
                                                 out_dev.data_ptr(), s.cuda_stream))


def lens_loglike_multi(ctx, lens_ids: Sequence[int], params_list: Sequence[np.ndarray]) -> list:
    ps = [_params(p) for p in params_list]
    counts = np.array([p.shape[0] for p in ps], dtype=np.int64)
    ids = np.array(lens_ids, dtype=np.int64)
    allp = np.ascontiguousarray(np.concatenate(ps, axis=0)) if ps else np.zeros((0, STRIDE))
    out = np.empty(int(counts.sum()), dtype=np.float64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    _check(ctx, load().lens_loglike_multi(ctx, len(ids), ids.ctypes.data_as(i64p), counts.ctypes.data_as(i64p),
                                          _dptr(allp), _dptr(out)))
    return np.split(out, np.cumsum(counts)[:-1])


LENS_NOALLOC_MAX = 32768


def lens_loglike_batch_device_noalloc(ctx, lens_id, params_dev: "torch.Tensor", out_dev: "torch.Tensor",
                                      stream: Optional["torch.cuda.Stream"] = None):
    """The allocation-free device-buffer call: at most LENS_NOALLOC_MAX proposals, prepared
    constants in the library's fixed per-device array (overlapping calls on one GPU race)."""
    if params_dev.dtype != torch.float64 or out_dev.dtype != torch.float64:
        raise TypeError("float64 tensors expected")
    if not (params_dev.is_cuda and out_dev.is_cuda and params_dev.is_contiguous() and out_dev.is_contiguous()):
        raise ValueError("contiguous device tensors expected")
    n = params_dev.shape[0]
    if params_dev.shape != (n, STRIDE) or out_dev.shape != (n,):
        raise ValueError("shapes must be [n, 20] and [n]")
    s = stream if stream is not None else torch.cuda.current_stream(params_dev.device)
    _check(ctx, load().lens_loglike_batch_device_noalloc(ctx, lens_id, params_dev.data_ptr(), n,
                                                         out_dev.data_ptr(), s.cuda_stream))


def lens_loglike_multi_device(ctx, lens_ids: Sequence[int], counts: Sequence[int], params_dev: "torch.Tensor",
                              out_dev: "torch.Tensor", stream: Optional["torch.cuda.Stream"] = None):
    """Many lenses on device buffers: params_dev [sum counts, 20] and out_dev [sum counts]
    float64 on the GPU, lens-major in the order of lens_ids; enqueued on `stream`."""
    if params_dev.dtype != torch.float64 or out_dev.dtype != torch.float64:
        raise TypeError("float64 tensors expected")
    if not (params_dev.is_cuda and out_dev.is_cuda and params_dev.is_contiguous() and out_dev.is_contiguous()):
        raise ValueError("contiguous device tensors expected")
    ids = np.ascontiguousarray(lens_ids, dtype=np.int64)
    cnt = np.ascontiguousarray(counts, dtype=np.int64)
    if ids.shape != cnt.shape or ids.ndim != 1:
        raise ValueError("lens_ids and counts must be 1-d of one length")
    n = int(cnt.sum())
    if params_dev.shape != (n, STRIDE) or out_dev.shape != (n,):
        raise ValueError("shapes must be [sum counts, 20] and [sum counts]")
    s = stream if stream is not None else torch.cuda.current_stream(params_dev.device)
    i64p = ctypes.POINTER(ctypes.c_int64)
    _check(ctx, load().lens_loglike_multi_device(ctx, len(ids), ids.ctypes.data_as(i64p), cnt.ctypes.data_as(i64p),
                                                 params_dev.data_ptr(), out_dev.data_ptr(), s.cuda_stream))


class Request:
    """A submitted serving request: keeps its output buffer alive."""

    def __init__(self, ctx, req_id, out):
        self.ctx, self.id, self.out = ctx, req_id, out


def lens_submit(ctx, lens_id, params) -> Request:
    p = _params(params)
    out = np.empty(p.shape[0], dtype=np.float64)
    rid = ctypes.c_int64()
    _check(ctx, load().lens_submit(ctx, lens_id, _dptr(p), p.shape[0], _dptr(out), ctypes.byref(rid)))
    return Request(ctx, rid.value, out)


def lens_poll(ctx, req: Request) -> int:
    st = load().lens_poll(ctx, req.id)
    return _check(ctx, st, ok=(LENS_OK, LENS_PENDING))


def lens_wait(ctx, req: Request, timeout_us: int = -1) -> int:
    st = load().lens_wait(ctx, req.id, timeout_us)
    return _check(ctx, st, ok=(LENS_OK, LENS_ETIMEDOUT))


def lens_cancel(ctx, req: Request):
    _check(ctx, load().lens_cancel(ctx, req.id))


def lens_reset_stats(ctx):
    _check(ctx, load().lens_reset_stats(ctx))


def lens_get_stats(ctx) -> dict:
    s = lens_stats()
    _check(ctx, load().lens_get_stats(ctx, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in lens_stats._fields_}


def lens_model_image(ctx, lens_id, params1, stage: int, ny: int, nx: int) -> np.ndarray:
    p = _params(params1)[0].copy()
    out = np.empty((ny, nx), dtype=np.float64)
    _check(ctx, load().lens_model_image(ctx, lens_id, _dptr(p), stage, _dptr(out)))
    return out


def lens_selftest(ctx, which: int = 0) -> float:
    r = ctypes.c_double()
    _check(ctx, load().lens_selftest(ctx, which, ctypes.byref(r)))
    return r.value


# instruction kinds of lens_peak_rate (LENS_PEAK_* in include/lens_api.h)
PEAK_OPS = ["fma_f64", "fma_f32", "mul_f64", "add_f64", "exp_f32", "log_f32", "rsq_f32", "rcp_f32",
            "cvt_f64_f32", "ldexp_f64", "frexp_mant_f64", "rndne_f64", "rsq_f64", "mfma_f16", "mfma_bf16",
            "fma_f64_exp_f32", "mfma_f16_fma_f64"]


def lens_peak_rate(ctx, op: int) -> float:
    r = ctypes.c_double()
    _check(ctx, load().lens_peak_rate(ctx, op, ctypes.byref(r)))
    return r.value


def lens_strerror(st: int) -> str:
    return load().lens_strerror(st).decode()


def lens_last_error(ctx) -> str:
    return load().lens_last_error(ctx).decode()


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------
class LensContext:
    """One library context on one GPU."""

    def __init__(self, device: int = 0, **kw):
        self.ctx = lens_init(device=device, **kw)
        self.geom = {}

    def close(self):
        if self.ctx:
            lens_shutdown(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def load(self, spec, precision=LENS_PREC_FP32, data=None, psf_tail=0.0, amplitudes=0, light_model=0,
             sersic_n=(1.0, 1.0, 1.0, 1.0), mass_model=0) -> int:
        """Load a synth.LensSpec (its data, or ``data`` if given)."""
        d = spec.data if data is None else data
        lid = lens_load_data(self.ctx, spec.ny, spec.nx, spec.dpix, spec.s, spec.psf, d, spec.sigma,
                             spec.mask, precision, psf_tail, amplitudes, light_model, sersic_n, mass_model)
        self.geom[lid] = (spec.ny, spec.nx)
        return lid

    def load_raw(self, ny, nx, dpix, s, psf, data, sigma, mask, precision=LENS_PREC_FP32, psf_tail=0.0) -> int:
        lid = lens_load_data(self.ctx, ny, nx, dpix, s, psf, data, sigma, mask, precision, psf_tail)
        self.geom[lid] = (ny, nx)
        return lid

    def unload(self, lid):
        lens_unload(self.ctx, lid)
        self.geom.pop(lid, None)

    def loglike_amps(self, lid, params):
        """(lnL, amplitudes [n, N]) at the solved (LENS_AMP_NNLS) or given amplitudes."""
        return lens_loglike_amps(self.ctx, lid, params)

    def loglike(self, lid, params) -> np.ndarray:
        return lens_loglike_batch(self.ctx, lid, params)

    def loglike_device(self, lid, params_dev, out_dev, stream=None):
        lens_loglike_batch_device(self.ctx, lid, params_dev, out_dev, stream)

    def loglike_multi(self, lids, params_list):
        return lens_loglike_multi(self.ctx, lids, params_list)

    def loglike_multi_device(self, lids, counts, params_dev, out_dev, stream=None):
        return lens_loglike_multi_device(self.ctx, lids, counts, params_dev, out_dev, stream)

    def model_image(self, lid, params1, stage=1) -> np.ndarray:
        ny, nx = self.geom[lid]
        return lens_model_image(self.ctx, lid, params1, stage, ny, nx)

    def info(self, lid) -> dict:
        return lens_get_info(self.ctx, lid)

    def ensemble(self, lid, init, lo, hi, stretch=2.0, seed=0) -> int:
        """A device-resident stretch-move ensemble on lens ``lid`` (walkers ``init`` [W, 20])."""
        return lens_ensemble_create(self.ctx, lid, init, lo, hi, stretch, seed)

    def ensemble_run(self, ens, iterations, thin=0, chain=False):
        return lens_ensemble_run(self.ctx, ens, iterations, thin, chain)

    def ensemble_run_many(self, ens_ids, iterations, thin=0, chain=False):
        return lens_ensemble_run_many(self.ctx, ens_ids, iterations, thin, chain)

    def ensemble_get(self, ens):
        return lens_ensemble_get(self.ctx, ens)

    def ensemble_destroy(self, ens):
        lens_ensemble_destroy(self.ctx, ens)

    def philox(self, ctr, key, n) -> np.ndarray:
        return lens_philox4x32_10(self.ctx, ctr, key, n)

    def submit(self, lid, params) -> Request:
        return lens_submit(self.ctx, lid, params)

    def poll(self, req) -> int:
        return lens_poll(self.ctx, req)

    def wait(self, req, timeout_us=-1) -> int:
        return lens_wait(self.ctx, req, timeout_us)

    def cancel(self, req):
        lens_cancel(self.ctx, req)

    def stats(self) -> dict:
        return lens_get_stats(self.ctx)

    def reset_stats(self):
        lens_reset_stats(self.ctx)

    def selftest(self, which=0) -> float:
        return lens_selftest(self.ctx, which)

    def peak_rate(self, op) -> float:
        """Measured rate of one instruction kind (index or PEAK_OPS name): lane
        operations/s for the vector ALU kinds, FLOP/s for the matrix-core products."""
        if isinstance(op, str):
            op = PEAK_OPS.index(op)
        return lens_peak_rate(self.ctx, op)
