"""ctypes wrapper of the FP64 CPU oracle (hsp_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may call this; the product path never does.  Argument
marshalling only -- every step of the method is computed in the C code.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

TAG_Z, TAG_LAMBDA, TAG_TAU, TAG_BETA_S, TAG_NU, TAG_XI = 1, 2, 3, 4, 5, 6
X_F32, X_BF16 = 0, 1
BRANCH_ROBERT, BRANCH_GAUSS = 0, 1

_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


class _State(C.Structure):
    _fields_ = [("beta", C.POINTER(C.c_double)), ("lam_m2", C.POINTER(C.c_double)),
                ("nu_m1", C.POINTER(C.c_double)), ("tau_m2", C.c_double),
                ("xi_m1", C.c_double), ("sweep", C.c_uint32)]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        i64, u64, u32, i32, d = C.c_int64, C.c_uint64, C.c_uint32, C.c_int32, C.c_double
        vp = C.c_void_p
        L.orc_set_threads.argtypes = [C.c_int]; L.orc_set_threads.restype = None
        L.orc_max_threads.argtypes = []; L.orc_max_threads.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_uniform.argtypes = [u32]; L.orc_uniform.restype = d
        L.orc_words.argtypes = [u64, u32, u32, u32, u32, u32, _u32p]
        L.orc_tn_draw.argtypes = [d, C.c_int, u64, u32, u32, u32, i32,
                                  C.POINTER(i32), C.POINTER(i32)]
        L.orc_tn_draw.restype = d
        L.orc_gamma_cheng.argtypes = [d, u64, u32, u32, C.POINTER(i32)]
        L.orc_gamma_cheng.restype = d
        L.orc_z_step.argtypes = [vp, C.c_int, _u8p, i64, i64, _dp, u64, u32, u32, _dp, vp, vp]
        L.orc_row_dot.argtypes = [vp, C.c_int, i64, i64, _dp]; L.orc_row_dot.restype = d
        L.orc_xtz.argtypes = [vp, C.c_int, i64, i64, _dp, _dp]
        L.orc_gram.argtypes = [vp, C.c_int, i64, i64, _dp]
        L.orc_gram_entry.argtypes = [vp, C.c_int, i64, i64, i64, i64]
        L.orc_gram_entry.restype = d
        L.orc_lambda_step.argtypes = [i64, _dp, _dp, d, u64, u32, u32, _dp]
        L.orc_lambda_step.restype = i64
        L.orc_tau_step.argtypes = [i64, _dp, _dp, d, u64, u32, u32, C.POINTER(i32)]
        L.orc_tau_step.restype = d
        L.orc_nu_step.argtypes = [i64, _dp, u64, u32, u32, _dp]
        L.orc_xi_step.argtypes = [d, u64, u32, u32]; L.orc_xi_step.restype = d
        L.orc_cholesky_upper.argtypes = [i64, _dp, _dp]; L.orc_cholesky_upper.restype = C.c_int
        L.orc_solve_upper.argtypes = [i64, _dp, _dp, _dp]
        L.orc_solve_upper_t.argtypes = [i64, _dp, _dp, _dp]
        L.orc_beta_step.argtypes = [i64, _dp, _dp, d, _dp, u64, u32, u32, _dp, vp, vp]
        L.orc_beta_step.restype = C.c_int
        L.orc_cold_start.argtypes = [i64, C.POINTER(_State)]
        L.orc_sweep.argtypes = [vp, C.c_int, _u8p, i64, i64, _dp, u64, u32,
                                C.POINTER(_State), vp, vp, C.POINTER(i64)]
        L.orc_sweep.restype = C.c_int
        L.orc_run.argtypes = [vp, C.c_int, _u8p, i64, i64, _dp, u64, u32,
                              C.POINTER(_State), i64, vp, vp, vp]
        L.orc_run.restype = C.c_int
        _lib = L
    return _lib


def _xarg(X):
    """(pointer, xtype, N, p) of a float32 array or a uint16 array of bf16 bits."""
    if X.dtype == np.float32:
        xt = X_F32
    elif X.dtype == np.uint16:
        xt = X_BF16
    else:
        raise TypeError("X must be float32 or uint16 (bfloat16 bits)")
    if X.ndim != 2 or not X.flags["C_CONTIGUOUS"]:
        raise ValueError("X must be a C-contiguous N x p array")
    return X.ctypes.data_as(C.c_void_p), xt, X.shape[0], X.shape[1]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def set_threads(n):
    """Threads of the oracle's N-sized loops (results are identical for any n)."""
    lib().orc_set_threads(int(n))


def max_threads():
    return lib().orc_max_threads()


# ---- random numbers --------------------------------------------------------
def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.ascontiguousarray(ctr, np.uint32),
                            np.ascontiguousarray(key, np.uint32), out)
    return out


def uniform(w):
    return lib().orc_uniform(int(w))


def words(seed, c0, sweep, tag, rnd, chain):
    out = np.zeros(4, np.uint32)
    lib().orc_words(seed, c0, sweep, tag, rnd, chain, out)
    return out


# ---- single draws -----------------------------------------------------------
def tn_draw(eta, y, seed, row, sweep, chain=0, max_attempts=1 << 24):
    a, br = C.c_int32(0), C.c_int32(0)
    z = lib().orc_tn_draw(float(eta), int(y), seed, row, sweep, chain, max_attempts,
                          C.byref(a), C.byref(br))
    return z, a.value, br.value


def gamma_cheng(a, seed, sweep, chain=0):
    m = C.c_int32(0)
    g = lib().orc_gamma_cheng(float(a), seed, sweep, chain, C.byref(m))
    return g, m.value


# ---- conditionals ------------------------------------------------------------
def z_step(X, y, beta, seed, sweep, chain=0):
    px, xt, N, p = _xarg(X)
    z = np.zeros(N)
    att = np.zeros(N, np.int32)
    br = np.zeros(N, np.int32)
    lib().orc_z_step(px, xt, np.ascontiguousarray(y, np.uint8), N, p, _f64(beta), seed,
                     sweep, chain, z, _ptr(att), _ptr(br))
    return z, att, br


def row_dot(X, row, beta):
    px, xt, N, p = _xarg(X)
    return lib().orc_row_dot(px, xt, p, row, _f64(beta))


def xtz(X, z):
    px, xt, N, p = _xarg(X)
    b = np.zeros(p)
    lib().orc_xtz(px, xt, N, p, _f64(z), b)
    return b


def gram(X):
    px, xt, N, p = _xarg(X)
    G = np.zeros((p, p))
    lib().orc_gram(px, xt, N, p, G)
    return G


def gram_fast(X):
    """G = X^T X by a library matmul over the exactly widened float64 X.

    The same definition as gram() (Section 5, beta step i) with numpy's
    summation order instead of the plain row loop; for designs too large for
    the loop to finish in seconds.  Agreement with gram() is pinned in the
    oracle tests.
    """
    if X.dtype == np.uint16:
        Xf = (X.astype(np.uint32) << 16).view(np.float32)
    elif X.dtype == np.float32:
        Xf = X
    else:
        raise TypeError("X must be float32 or uint16 (bfloat16 bits)")
    X64 = Xf.astype(np.float64)
    return X64.T @ X64


def gram_entry(X, j, k):
    px, xt, N, p = _xarg(X)
    return lib().orc_gram_entry(px, xt, N, p, j, k)


def lambda_step(beta, nu_m1, tau_m2, seed, sweep, chain=0):
    beta = _f64(beta)
    lam = np.zeros(beta.size)
    clamps = lib().orc_lambda_step(beta.size, beta, _f64(nu_m1), float(tau_m2), seed, sweep,
                                   chain, lam)
    return lam, clamps


def tau_step(lam_m2, beta, xi_m1, seed, sweep, chain=0):
    beta = _f64(beta)
    m = C.c_int32(0)
    t = lib().orc_tau_step(beta.size, _f64(lam_m2), beta, float(xi_m1), seed, sweep, chain,
                           C.byref(m))
    return t, m.value


def nu_step(lam_m2, seed, sweep, chain=0):
    lam_m2 = _f64(lam_m2)
    nu = np.zeros(lam_m2.size)
    lib().orc_nu_step(lam_m2.size, lam_m2, seed, sweep, chain, nu)
    return nu


def xi_step(tau_m2, seed, sweep, chain=0):
    return lib().orc_xi_step(float(tau_m2), seed, sweep, chain)


def cholesky_upper(Q):
    Q = _f64(Q)
    U = np.zeros_like(Q)
    rc = lib().orc_cholesky_upper(Q.shape[0], Q, U)
    return U, rc


def solve_upper(U, r):
    U = _f64(U)
    x = np.zeros(U.shape[0])
    lib().orc_solve_upper(U.shape[0], U, _f64(r), x)
    return x


def solve_upper_t(U, r):
    U = _f64(U)
    x = np.zeros(U.shape[0])
    lib().orc_solve_upper_t(U.shape[0], U, _f64(r), x)
    return x


def beta_step(G, lam_m2, tau_m2, b, seed, sweep, chain=0):
    G = _f64(G)
    p = G.shape[0]
    beta, mean, noise = np.zeros(p), np.zeros(p), np.zeros(p)
    rc = lib().orc_beta_step(p, G, _f64(lam_m2), float(tau_m2), _f64(b), seed, sweep, chain,
                             beta, _ptr(mean), _ptr(noise))
    return beta, mean, noise, rc


# ---- whole chains ---------------------------------------------------------------
class Chain:
    """Markov state of one oracle chain (beta, lam^-2, nu^-1, tau^-2, xi^-1, sweep)."""

    def __init__(self, p, beta=None, lam_m2=None, nu_m1=None, tau_m2=None, xi_m1=None, sweep=0):
        """The cold start of Section 6.1 (orc_cold_start) unless a state is given."""
        self.p = p
        self.beta, self.lam_m2, self.nu_m1 = np.zeros(p), np.zeros(p), np.zeros(p)
        self.tau_m2 = self.xi_m1 = 0.0
        self.sweep = 0
        st = self._cstate()
        lib().orc_cold_start(p, C.byref(st))
        self._pull(st)
        if beta is not None:
            self.beta = _f64(beta).copy()
        if lam_m2 is not None:
            self.lam_m2 = _f64(lam_m2).copy()
        if nu_m1 is not None:
            self.nu_m1 = _f64(nu_m1).copy()
        if tau_m2 is not None:
            self.tau_m2 = float(tau_m2)
        if xi_m1 is not None:
            self.xi_m1 = float(xi_m1)
        self.sweep = int(sweep)

    def _cstate(self):
        dp = C.POINTER(C.c_double)
        return _State(self.beta.ctypes.data_as(dp), self.lam_m2.ctypes.data_as(dp),
                      self.nu_m1.ctypes.data_as(dp), self.tau_m2, self.xi_m1, self.sweep)

    def _pull(self, st):
        self.tau_m2, self.xi_m1, self.sweep = st.tau_m2, st.xi_m1, st.sweep

    def sweep_once(self, X, y, G, seed, chain=0, want_z=False):
        px, xt, N, p = _xarg(X)
        st = self._cstate()
        z = np.zeros(N) if want_z else None
        b = np.zeros(p) if want_z else None
        clamps = C.c_int64(0)
        rc = lib().orc_sweep(px, xt, np.ascontiguousarray(y, np.uint8), N, p, _f64(G), seed,
                             chain, C.byref(st), _ptr(z), _ptr(b), C.byref(clamps))
        self._pull(st)
        if rc != 0:
            raise RuntimeError(f"oracle sweep failed: Cholesky pivot {rc}")
        return (z, b, clamps.value) if want_z else clamps.value

    def run(self, X, y, G, seed, n, chain=0, record_lambda=False):
        px, xt, N, p = _xarg(X)
        st = self._cstate()
        betas = np.zeros((n, p))
        taus = np.zeros(n)
        lams = np.zeros((n, p)) if record_lambda else None
        rc = lib().orc_run(px, xt, np.ascontiguousarray(y, np.uint8), N, p, _f64(G), seed,
                           chain, C.byref(st), n, _ptr(betas), _ptr(taus), _ptr(lams))
        self._pull(st)
        if rc != 0:
            raise RuntimeError(f"oracle run failed: Cholesky pivot {rc}")
        return (betas, taus, lams) if record_lambda else (betas, taus)
