"""Thin Python binding of the C ABI in include/hsp.h (ctypes).

Argument marshalling only: every step of the sampler runs in the HIP
library libhsp.so.  The binding refuses to run when the library is missing.
Device buffers may be torch tensors on the GPU (their data_ptr() is passed);
host buffers are numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsp.so")

HSP_OK, HSP_EINVAL, HSP_ENOMEM, HSP_EHIP, HSP_ENOTPD, HSP_ERANGE, HSP_EPOISONED = 0, -1, -2, -3, -4, -5, -6
HSP_X_F32, HSP_X_BF16 = 0, 1
HSP_STEP_Z, HSP_STEP_LAMBDA, HSP_STEP_TAU, HSP_STEP_BETA, HSP_STEP_NUXI, HSP_STEP_ADVANCE = 1, 2, 4, 8, 16, 32
GAUSS_BIT = 1 << 30

STATUS_NAMES = {0: "HSP_OK", -1: "HSP_EINVAL", -2: "HSP_ENOMEM", -3: "HSP_EHIP", -4: "HSP_ENOTPD",
                -5: "HSP_ERANGE", -6: "HSP_EPOISONED"}

EXPORTS = ["hsp_default_options", "hsp_max_p", "hsp_gram", "hsp_gram_noalloc", "hsp_create", "hsp_sweep", "hsp_sync", "hsp_draws",
           "hsp_destroy", "hsp_last_error", "hsp_get_state", "hsp_set_state", "hsp_step",
           "hsp_get_debug", "hsp_get_gram", "hsp_get_counters", "hsp_set_timing",
           "hsp_get_timing", "hsp_philox", "hsp_set_phase_trace", "hsp_get_phase_trace",
           "hsp_tile_schedule", "hsp_read_ceiling", "hsp_batch_create", "hsp_batch_size",
           "hsp_batch_chain", "hsp_batch_sweep", "hsp_batch_sync", "hsp_batch_set_timing",
           "hsp_batch_get_timing", "hsp_batch_last_error", "hsp_batch_destroy", "hsp_get_plan",
           "hsp_sort_rows", "hsp_batch_get_plan", "hsp_tune_key", "hsp_tune_cache_put", "hsp_tune_cache_get",
           "hsp_batch_set_shape"]


class hsp_options(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("chain_id", C.c_uint32), ("x_type", C.c_int32),
                ("x_on_host", C.c_int32), ("record_lambda", C.c_int32), ("thin", C.c_int64),
                ("max_draws", C.c_int64), ("hip_stream", C.c_void_p), ("debug_store_z", C.c_int32),
                ("use_graph", C.c_int32), ("multi_chain_z", C.c_int32), ("autotune", C.c_int32),
                ("x_stream", C.c_int32), ("stream_rows", C.c_int64)]


class hsp_dataset(C.Structure):
    _fields_ = [("X", C.c_void_p), ("y", C.c_void_p), ("N", C.c_int64), ("p", C.c_int64),
                ("x_type", C.c_int32)]


class HspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libhsp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i64, u64, u32, i32, d = C.c_void_p, C.c_int64, C.c_uint64, C.c_uint32, C.c_int32, C.c_double
    st = C.c_int
    L.hsp_default_options.argtypes = [C.POINTER(hsp_options)]
    L.hsp_default_options.restype = None
    L.hsp_max_p.restype = i64
    L.hsp_create.argtypes = [vp, vp, i64, i64, C.POINTER(hsp_options), C.POINTER(vp)]
    L.hsp_create.restype = st
    L.hsp_gram.argtypes = [vp, i32, i64, i64, i64, vp, vp]; L.hsp_gram.restype = st
    L.hsp_gram_noalloc.argtypes = [vp, i32, i64, i64, i64, vp, vp]; L.hsp_gram_noalloc.restype = st
    L.hsp_sweep.argtypes = [vp, i64]; L.hsp_sweep.restype = st
    L.hsp_sync.argtypes = [vp]; L.hsp_sync.restype = st
    L.hsp_draws.argtypes = [vp, vp, vp, vp, i64, i64, C.POINTER(i64)]; L.hsp_draws.restype = st
    L.hsp_destroy.argtypes = [vp]; L.hsp_destroy.restype = st
    L.hsp_last_error.argtypes = [vp]; L.hsp_last_error.restype = C.c_char_p
    L.hsp_get_state.argtypes = [vp, vp, vp, vp, C.POINTER(d), C.POINTER(d), C.POINTER(u64)]
    L.hsp_get_state.restype = st
    L.hsp_set_state.argtypes = [vp, vp, vp, vp, d, d, u64]; L.hsp_set_state.restype = st
    L.hsp_step.argtypes = [vp, u32]; L.hsp_step.restype = st
    L.hsp_get_debug.argtypes = [vp, vp, vp, vp]; L.hsp_get_debug.restype = st
    L.hsp_get_gram.argtypes = [vp, vp]; L.hsp_get_gram.restype = st
    L.hsp_get_counters.argtypes = [vp, C.POINTER(u64), C.POINTER(u32)]
    L.hsp_get_counters.restype = st
    L.hsp_set_timing.argtypes = [vp, i32]; L.hsp_set_timing.restype = st
    L.hsp_get_timing.argtypes = [vp, C.POINTER(d), C.POINTER(d), C.POINTER(i64)]
    L.hsp_get_timing.restype = st
    L.hsp_philox.argtypes = [u64, vp, i64, vp]; L.hsp_philox.restype = st
    L.hsp_set_phase_trace.argtypes = [vp, i32]; L.hsp_set_phase_trace.restype = st
    L.hsp_get_phase_trace.argtypes = [vp, vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(d)]
    L.hsp_get_phase_trace.restype = st
    L.hsp_tile_schedule.argtypes = [i64, i64, i32, vp, i64, vp, C.POINTER(i64)]
    L.hsp_tile_schedule.restype = st
    L.hsp_read_ceiling.argtypes = [vp, i32, C.POINTER(d), C.POINTER(d)]
    L.hsp_read_ceiling.restype = st
    L.hsp_batch_create.argtypes = [C.POINTER(hsp_dataset), i32, C.POINTER(i32), C.POINTER(hsp_options),
                                   C.POINTER(vp)]
    L.hsp_batch_create.restype = st
    L.hsp_batch_size.argtypes = [vp]; L.hsp_batch_size.restype = i64
    L.hsp_batch_chain.argtypes = [vp, i64, C.POINTER(vp)]; L.hsp_batch_chain.restype = st
    L.hsp_batch_sweep.argtypes = [vp, i64]; L.hsp_batch_sweep.restype = st
    L.hsp_batch_sync.argtypes = [vp]; L.hsp_batch_sync.restype = st
    L.hsp_batch_set_timing.argtypes = [vp, i32]; L.hsp_batch_set_timing.restype = st
    L.hsp_batch_get_timing.argtypes = [vp, C.POINTER(d), C.POINTER(i64)]
    L.hsp_batch_get_timing.restype = st
    L.hsp_batch_last_error.argtypes = [vp]; L.hsp_batch_last_error.restype = C.c_char_p
    L.hsp_batch_destroy.argtypes = [vp]; L.hsp_batch_destroy.restype = st
    pi64 = C.POINTER(i64)
    L.hsp_get_plan.argtypes = [vp, pi64, pi64, pi64, pi64, C.c_char_p, i64]; L.hsp_get_plan.restype = st
    L.hsp_sort_rows.argtypes = [vp]; L.hsp_sort_rows.restype = st
    L.hsp_batch_get_plan.argtypes = [vp, pi64, pi64, pi64, C.c_char_p, i64]
    L.hsp_batch_get_plan.restype = st
    L.hsp_batch_set_shape.argtypes = [vp, C.c_int32, C.c_int32]; L.hsp_batch_set_shape.restype = st
    L.hsp_tune_key.argtypes = [vp, C.c_char_p, i64]; L.hsp_tune_key.restype = st
    L.hsp_tune_cache_put.argtypes = [C.c_char_p, C.c_char_p, C.c_char_p]; L.hsp_tune_cache_put.restype = st
    L.hsp_tune_cache_get.argtypes = [C.c_char_p, C.c_char_p, C.c_char_p, i64]
    L.hsp_tune_cache_get.restype = st
    _lib = L
    return L


def _check(code, state=None):
    if code != HSP_OK:
        msg = load().hsp_last_error(state)
        raise HspError(code, msg.decode() if msg else "")


def _hp(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---- the C entry points under their own names --------------------------------
def hsp_default_options():
    o = hsp_options()
    load().hsp_default_options(C.byref(o))
    return o


def hsp_max_p():
    return load().hsp_max_p()


def hsp_gram(X, x_type, N, p, ld, G, stream=None):
    """G = X^T X (float64) of a device design; X and G are device pointers (int)."""
    _check(load().hsp_gram(X, x_type, N, p, ld, G, stream))


def hsp_gram_noalloc(X, x_type, N, p, ld, G, stream=None):
    """hsp_gram through the library's fixed workspace (no device allocation)."""
    _check(load().hsp_gram_noalloc(X, x_type, N, p, ld, G, stream))


def hsp_create(X, y, N, p, opt=None):
    """X, y: device pointers (int) or, with opt.x_on_host = 1, host pointers."""
    h = C.c_void_p()
    code = load().hsp_create(X, y, N, p, C.byref(opt) if opt is not None else None, C.byref(h))
    _check(code)
    return h


def hsp_sweep(h, n):
    _check(load().hsp_sweep(h, n), h)


def hsp_sync(h):
    _check(load().hsp_sync(h), h)


def hsp_draws(h, first, count, p, lam=False):
    beta = np.zeros((count, p))
    tau = np.zeros(count)
    lamv = np.zeros((count, p)) if lam else None
    n = C.c_int64(0)
    _check(load().hsp_draws(h, _hp(beta), _hp(tau), _hp(lamv), first, count, C.byref(n)), h)
    return (beta, tau, lamv, n.value) if lam else (beta, tau, n.value)


def hsp_destroy(h):
    _check(load().hsp_destroy(h), h)


def hsp_get_state(h, p):
    beta, lam, nu = np.zeros(p), np.zeros(p), np.zeros(p)
    tau, xi, sweep = C.c_double(), C.c_double(), C.c_uint64()
    _check(load().hsp_get_state(h, _hp(beta), _hp(lam), _hp(nu), C.byref(tau), C.byref(xi),
                                C.byref(sweep)), h)
    return dict(beta=beta, lam_m2=lam, nu_m1=nu, tau_m2=tau.value, xi_m1=xi.value,
                sweep=sweep.value)


def hsp_set_state(h, beta, lam_m2, nu_m1, tau_m2, xi_m1, sweep):
    b = np.ascontiguousarray(beta, np.float64)
    l = np.ascontiguousarray(lam_m2, np.float64)
    n = np.ascontiguousarray(nu_m1, np.float64)
    _check(load().hsp_set_state(h, _hp(b), _hp(l), _hp(n), float(tau_m2), float(xi_m1), int(sweep)), h)


def hsp_step(h, which):
    _check(load().hsp_step(h, which), h)


def hsp_get_debug(h, N, p):
    z = np.zeros(N, np.float32)
    att = np.zeros(N, np.int32)
    b = np.zeros(p)
    _check(load().hsp_get_debug(h, _hp(z), _hp(att), _hp(b)), h)
    return z, att, b


def hsp_get_gram(h, p):
    G = np.zeros((p, p))
    _check(load().hsp_get_gram(h, _hp(G)), h)
    return G


def hsp_get_counters(h):
    c, m = C.c_uint64(), C.c_uint32()
    _check(load().hsp_get_counters(h, C.byref(c), C.byref(m)), h)
    return c.value, m.value


def hsp_set_timing(h, enable):
    _check(load().hsp_set_timing(h, int(enable)), h)


def hsp_get_timing(h):
    z, s, n = C.c_double(), C.c_double(), C.c_int64()
    _check(load().hsp_get_timing(h, C.byref(z), C.byref(s), C.byref(n)), h)
    return z.value, s.value, n.value


def hsp_philox(seed, ctr):
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    out = np.zeros_like(ctr)
    _check(load().hsp_philox(seed, _hp(ctr), ctr.shape[0], _hp(out)))
    return out


def hsp_tile_schedule(nt, gp, inverse=None):
    """Task lists of the tiled factorisation: (tasks, list bounds).

    One list for a group of one block; otherwise block 0's chain list and the
    shared queue of the other blocks.  inverse: with the L^-1 tasks (True),
    without (False), or as a lone chain of nt tiles has it (None)."""
    inv = -1 if inverse is None else int(bool(inverse))
    n = C.c_int64()
    st = load().hsp_tile_schedule(nt, gp, inv, None, 0, None, C.byref(n))
    if st not in (HSP_OK, HSP_ERANGE):
        _check(st)
    tasks = np.zeros(max(n.value, 1), np.uint32)
    off = np.zeros(3, np.uint32)
    _check(load().hsp_tile_schedule(nt, gp, inv, _hp(tasks), tasks.size, _hp(off), C.byref(n)))
    return tasks[: n.value], off[: 2 if gp == 1 else 3]


def hsp_read_ceiling(h, iters=10):
    """(ms per pass, bytes per pass) of a plain streaming read of the state's X."""
    ms, nb = C.c_double(), C.c_double()
    _check(load().hsp_read_ceiling(h, iters, C.byref(ms), C.byref(nb)), h)
    return ms.value, nb.value


def _bcheck(code, b=None):
    if code != HSP_OK:
        msg = load().hsp_batch_last_error(b)
        raise HspError(code, msg.decode() if msg else "")


def hsp_batch_create(datasets, chains_per_ds, opt=None):
    """datasets: list of (X pointer, y pointer, N, p, x_type); pointers as for hsp_create."""
    arr = (hsp_dataset * len(datasets))(*[hsp_dataset(X, y, N, p, xt) for X, y, N, p, xt in datasets])
    cnt = (C.c_int32 * len(chains_per_ds))(*chains_per_ds)
    b = C.c_void_p()
    _bcheck(load().hsp_batch_create(arr, len(datasets), cnt, C.byref(opt) if opt is not None else None,
                                    C.byref(b)))
    return b


def hsp_batch_size(b):
    return load().hsp_batch_size(b)


def hsp_batch_chain(b, i):
    h = C.c_void_p()
    _bcheck(load().hsp_batch_chain(b, i, C.byref(h)), b)
    return h


def hsp_batch_sweep(b, n):
    _bcheck(load().hsp_batch_sweep(b, n), b)


def hsp_batch_sync(b):
    _bcheck(load().hsp_batch_sync(b), b)


def hsp_batch_set_timing(b, enable):
    _bcheck(load().hsp_batch_set_timing(b, int(enable)), b)


def hsp_batch_get_timing(b):
    ms, n = C.c_double(), C.c_int64()
    _bcheck(load().hsp_batch_get_timing(b, C.byref(ms), C.byref(n)), b)
    return ms.value, n.value


def hsp_batch_destroy(b):
    _bcheck(load().hsp_batch_destroy(b))


def hsp_set_phase_trace(h, enable):
    _check(load().hsp_set_phase_trace(h, int(enable)), h)


def hsp_get_phase_trace(h):
    gb, sl, tpu = C.c_int64(), C.c_int64(), C.c_double()
    _check(load().hsp_get_phase_trace(h, None, C.byref(gb), C.byref(sl), C.byref(tpu)), h)
    out = np.zeros((gb.value, sl.value), np.uint64)
    _check(load().hsp_get_phase_trace(h, _hp(out), C.byref(gb), C.byref(sl), C.byref(tpu)), h)
    return out, tpu.value


def hsp_get_plan(h):
    """(group_blocks, z_blocks, static_pct, unit, note) of a state's launch plan."""
    v = [C.c_int64() for _ in range(4)]
    note = C.create_string_buffer(256)
    _check(load().hsp_get_plan(h, *[C.byref(x) for x in v], note, 256), h)
    return tuple(x.value for x in v) + (note.value.decode(),)


def hsp_sort_rows(h):
    _check(load().hsp_sort_rows(h), h)


def hsp_batch_get_plan(b):
    """(mc_blocks, bw_pct, packs, note) of a batch's pack shapes."""
    v = [C.c_int64() for _ in range(3)]
    note = C.create_string_buffer(256)
    _check(load().hsp_batch_get_plan(b, *[C.byref(x) for x in v], note, 256))
    return tuple(x.value for x in v) + (note.value.decode(),)


def hsp_batch_set_shape(b, zq_kib, pre_blocks):
    _bcheck(load().hsp_batch_set_shape(b, int(zq_kib), int(pre_blocks)), b)


def hsp_tune_key(h):
    buf = C.create_string_buffer(512)
    _check(load().hsp_tune_key(h, buf, 512), h)
    return buf.value.decode()


def hsp_tune_cache_put(path, key, value):
    _check(load().hsp_tune_cache_put(path.encode(), key.encode(), value.encode()))


def hsp_tune_cache_get(path, key):
    """The cached value of key, or None."""
    buf = C.create_string_buffer(4096)
    code = load().hsp_tune_cache_get(path.encode(), key.encode(), buf, 4096)
    if code == HSP_ERANGE:
        return None
    _check(code)
    return buf.value.decode()


# ---- convenience wrapper --------------------------------------------------------
class Sampler:
    """One Horseshoe Probit chain on the GPU.

    X: (N, p) float32 torch tensor on the GPU, or a numpy array (host copy).
    y: (N,) uint8 tensor / array with values in {0, 1}.
    """

    def __init__(self, X, y, seed=1, chain_id=0, x_type="f32", record_lambda=False, thin=1,
                 max_draws=1024, debug_store_z=False, use_graph=True, stream=None, autotune=False,
                 x_stream=False, stream_rows=0):
        load()
        opt = hsp_default_options()
        opt.autotune = int(autotune)
        opt.x_stream = int(x_stream)
        opt.stream_rows = int(stream_rows)
        opt.seed = seed
        opt.chain_id = chain_id
        opt.x_type = {"f32": HSP_X_F32, "bf16": HSP_X_BF16}[x_type]
        opt.record_lambda = int(record_lambda)
        opt.thin = thin
        opt.max_draws = max_draws
        opt.debug_store_z = int(debug_store_z)
        opt.use_graph = int(use_graph)
        if stream is not None:
            opt.hip_stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        if isinstance(X, np.ndarray):
            X = np.ascontiguousarray(X, np.float32)
            y = np.ascontiguousarray(y, np.uint8)
            opt.x_on_host = 1
            xp, yp = X.ctypes.data, y.ctypes.data
        else:
            if not (X.is_cuda and y.is_cuda):
                raise ValueError("torch inputs must live on the GPU (or pass numpy arrays)")
            X = X.contiguous()
            y = y.contiguous()
            # the library copies X and y on its own stream: finish torch's work first
            import torch
            torch.cuda.synchronize(X.device)
            xp, yp = X.data_ptr(), y.data_ptr()
        self.N, self.p = int(X.shape[0]), int(X.shape[1])
        self.record_lambda = record_lambda
        self.h = hsp_create(xp, yp, self.N, self.p, opt)

    @classmethod
    def _borrowed(cls, h, N, p, record_lambda, keep):
        """A view of a batch's chain (released with the batch)."""
        s = cls.__new__(cls)
        s.h, s.N, s.p, s.record_lambda, s._batch = h, N, p, record_lambda, keep
        return s

    def close(self):
        if getattr(self, "_batch", None) is not None:
            self.h = None  # owned by the batch
            return
        if self.h:
            hsp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n=1):
        hsp_sweep(self.h, n)

    def sync(self):
        hsp_sync(self.h)

    def draws(self, first=0, count=None):
        if count is None:
            _, _, n = hsp_draws(self.h, 0, 0, self.p)
            count = n - first
        return hsp_draws(self.h, first, count, self.p, self.record_lambda)

    def state(self):
        return hsp_get_state(self.h, self.p)

    def set_state(self, beta, lam_m2, nu_m1, tau_m2, xi_m1, sweep):
        hsp_set_state(self.h, beta, lam_m2, nu_m1, tau_m2, xi_m1, sweep)

    def step(self, which):
        hsp_step(self.h, which)

    def debug(self):
        return hsp_get_debug(self.h, self.N, self.p)

    def gram(self):
        return hsp_get_gram(self.h, self.p)

    def counters(self):
        return hsp_get_counters(self.h)

    def set_timing(self, enable):
        hsp_set_timing(self.h, enable)

    def timing(self):
        return hsp_get_timing(self.h)

    def plan(self):
        return hsp_get_plan(self.h)

    def sort_rows(self):
        hsp_sort_rows(self.h)


class Batch:
    """Many independent chains, advanced together by one graph replay per sweep.

    datasets: list of (X, y) or (X, y, x_type) with X, y as for Sampler (all on
    the GPU, or all numpy); chains: chains per dataset (an int for all).
    Chain i (dataset-major) uses chain id chain_id + i.  The chains share
    launches of the sweep kernel (each with its own blocks), so a chain's
    rounding of X^T z can differ from the same chain run alone.
    """

    def __init__(self, datasets, chains=1, seed=1, chain_id=0, record_lambda=False, thin=1,
                 max_draws=1024, debug_store_z=False, stream=None, multi_chain_z=True, autotune=False):
        load()
        opt = hsp_default_options()
        opt.multi_chain_z = int(multi_chain_z)
        opt.autotune = int(autotune)
        opt.seed = seed
        opt.chain_id = chain_id
        opt.debug_store_z = int(debug_store_z)
        opt.record_lambda = int(record_lambda)
        opt.thin = thin
        opt.max_draws = max_draws
        if stream is not None:
            opt.hip_stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        counts = [chains] * len(datasets) if isinstance(chains, int) else list(chains)
        descs, self._keep, shapes = [], [], []
        host = None
        for ds in datasets:
            X, y = ds[0], ds[1]
            xt = {"f32": HSP_X_F32, "bf16": HSP_X_BF16}[ds[2] if len(ds) > 2 else "f32"]
            if isinstance(X, np.ndarray):
                X = np.ascontiguousarray(X, np.float32)
                y = np.ascontiguousarray(y, np.uint8)
                xp, yp, is_host = X.ctypes.data, y.ctypes.data, True
            else:
                if not (X.is_cuda and y.is_cuda):
                    raise ValueError("torch inputs must live on the GPU (or pass numpy arrays)")
                X, y = X.contiguous(), y.contiguous()
                xp, yp, is_host = X.data_ptr(), y.data_ptr(), False
            if host is None:
                host = is_host
            elif host != is_host:
                raise ValueError("all datasets of a batch must be on the host, or all on the GPU")
            self._keep.append((X, y))
            descs.append((xp, yp, int(X.shape[0]), int(X.shape[1]), xt))
            shapes.append((int(X.shape[0]), int(X.shape[1])))
        opt.x_on_host = int(bool(host))
        if not host:
            import torch
            torch.cuda.synchronize()
        self.record_lambda = record_lambda
        self.b = hsp_batch_create(descs, counts, opt)
        self._keep = None  # the library holds its own copies now
        self.shapes = [shapes[d] for d, c in enumerate(counts) for _ in range(c)]
        self.chains = [Sampler._borrowed(hsp_batch_chain(self.b, i), N, p, record_lambda, self)
                       for i, (N, p) in enumerate(self.shapes)]

    def __len__(self):
        return len(self.chains)

    def chain(self, i):
        return self.chains[i]

    def sweep(self, n=1):
        hsp_batch_sweep(self.b, n)

    def sync(self):
        hsp_batch_sync(self.b)

    def set_timing(self, enable):
        hsp_batch_set_timing(self.b, enable)

    def timing(self):
        return hsp_batch_get_timing(self.b)

    def plan(self):
        return hsp_batch_get_plan(self.b)

    def set_shape(self, zq_kib=64, pre_blocks=16):
        """Shared z queue per pack in units of about zq_kib KiB of X (0: off);
        blocks per chain factoring Q beside a multi-chain pass (0: after it)."""
        hsp_batch_set_shape(self.b, zq_kib, pre_blocks)

    def close(self):
        if self.b:
            for c in self.chains:
                c.h = None
            hsp_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
