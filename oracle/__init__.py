"""FP64 CPU oracle of the Anscombe-domain FoE Poisson denoiser.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the GPU library or its binding.
The arithmetic lives in fe_oracle.c (plain double-precision loops written
from the paper's equations); this module only marshals numpy arrays.

All float32 inputs (counts, filters, weights, lambda, tau, gamma) are widened
exactly to double before they reach the C code.
"""
import contextlib
import ctypes
import os

import numpy as np

from .build import LIB, build

QUADRATIC = 1
IDIV = 2

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


_SIGNATURES = None


def _signatures():
    i, d, L = ctypes.c_int, ctypes.c_double, ctypes.c_long
    return {
        "oracle_anscombe": (None, [_dp, _dp, L]),
        "oracle_inverse_anscombe": (None, [_dp, _dp, L]),
        "oracle_inverse_anscombe_scalar": (d, [d]),
        "oracle_extend_symmetric": (None, [_dp, i, i, i, _dp]),
        "oracle_filter": (None, [_dp, i, i, _dp, i, i, _dp]),
        "oracle_filter_adjoint": (None, [_dp, i, i, _dp, i, i, _dp]),
        "oracle_rho": (d, [d]),
        "oracle_rho_prime": (d, [d]),
        "oracle_grad_prior": (None, [_dp, i, i, _dp, _dp, i, i, _dp]),
        "oracle_energy_prior": (d, [_dp, i, i, _dp, _dp, i, i]),
        "oracle_energy_data": (d, [_dp, _dp, L, d, i]),
        "oracle_grad_data": (None, [_dp, _dp, L, d, i, _dp]),
        "oracle_prox_scalar": (d, [d, d, d, d, i]),
        "oracle_prox": (None, [_dp, _dp, L, d, d, i, _dp]),
        "oracle_ipiano_step": (None, [_dp, _dp, _dp, i, i, _dp, _dp, i, i,
                                      d, d, d, i, _dp]),
        "oracle_denoise": (None, [_dp, i, i, _dp, _dp, i, i, d, d, d, i, i,
                                  _dp, _dp]),
        "oracle_energy_grad": (d, [_dp, _dp, i, i, _dp, _dp, i, i, d, i,
                                   _dp]),
        "oracle_power_iteration": (d, [_dp, i, i, _dp, _dp, i, i, i]),
        "oracle_bin3": (None, [_dp, i, i, _dp]),
        "oracle_upsample3": (None, [_dp, i, i, i, i, _dp]),
    }


def _open(path):
    lib = ctypes.CDLL(path)
    for name, (res, args) in _signatures().items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _open(LIB)
    return _lib


@contextlib.contextmanager
def use_library(path):
    """Temporarily route every call to another build of the oracle source
    (the tests use this to show that a planted mistake breaks a pin)."""
    global _lib
    saved = _load()
    _lib = _open(path)
    try:
        yield
    finally:
        _lib = saved


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _f32(x):
    """Widen a parameter exactly as the GPU sees it (float32 -> double)."""
    return float(np.float32(x))


def anscombe(y):
    y, py = _d(y)
    v = np.empty_like(y)
    _load().oracle_anscombe(py, v.ctypes.data_as(_dp), y.size)
    return v


def inverse_anscombe(u):
    u, pu = _d(u)
    x = np.empty_like(u)
    _load().oracle_inverse_anscombe(pu, x.ctypes.data_as(_dp), u.size)
    return x


def inverse_anscombe_scalar(z):
    return _load().oracle_inverse_anscombe_scalar(float(z))


def extend_symmetric(u, r):
    u, pu = _d(u)
    H, W = u.shape
    e = np.empty((H + 2 * r, W + 2 * r))
    _load().oracle_extend_symmetric(pu, H, W, r, e.ctypes.data_as(_dp))
    return e


def _bank(k):
    k = np.asarray(k)
    if k.ndim == 2:
        k = k[None]
    return k.shape[0], k.shape[1], _d(k)


def filter_bank(u, k):
    """z_i = K_i u for every filter; returns [nf, H, W]."""
    u, pu = _d(u)
    H, W = u.shape
    nf, m, (kk, pk) = _bank(k)
    z = np.empty((nf, H, W))
    _load().oracle_filter(pu, H, W, pk, m, nf, z.ctypes.data_as(_dp))
    return z


def filter_adjoint(w, k):
    """sum_i K_i^T w_i for w of shape [nf, H, W] (or [H, W] with one filter)."""
    nf, m, (kk, pk) = _bank(k)
    w = np.asarray(w, np.float64)
    if w.ndim == 2:
        w = w[None]
    w, pw = _d(w)
    H, W = w.shape[1:]
    g = np.empty((H, W))
    _load().oracle_filter_adjoint(pw, H, W, pk, m, nf, g.ctypes.data_as(_dp))
    return g


def rho(z):
    return _load().oracle_rho(float(z))


def rho_prime(z):
    return _load().oracle_rho_prime(float(z))


def grad_prior(u, k, alpha):
    u, pu = _d(u)
    H, W = u.shape
    nf, m, (kk, pk) = _bank(k)
    a, pa = _d(alpha)
    g = np.empty((H, W))
    _load().oracle_grad_prior(pu, H, W, pk, pa, m, nf, g.ctypes.data_as(_dp))
    return g


def energy_prior(u, k, alpha):
    u, pu = _d(u)
    H, W = u.shape
    nf, m, (kk, pk) = _bank(k)
    a, pa = _d(alpha)
    return _load().oracle_energy_prior(pu, H, W, pk, pa, m, nf)


def energy_data(u, v, lam, data_term):
    u, pu = _d(u)
    v, pv = _d(v)
    return _load().oracle_energy_data(pu, pv, u.size, float(lam), int(data_term))


def prox(ut, v, tau, lam, data_term):
    ut, pu = _d(ut)
    v, pv = _d(v)
    out = np.empty_like(ut)
    _load().oracle_prox(pu, pv, ut.size, float(tau), float(lam),
                        int(data_term), out.ctypes.data_as(_dp))
    return out


def prox_scalar(ut, v, tau, lam, data_term):
    return _load().oracle_prox_scalar(float(ut), float(v), float(tau),
                                      float(lam), int(data_term))


def ipiano_step(u, u_prev, v, k, alpha, lam, tau, gamma, data_term):
    u, pu = _d(u)
    up, pup = _d(u_prev)
    v, pv = _d(v)
    H, W = u.shape
    nf, m, (kk, pk) = _bank(k)
    a, pa = _d(alpha)
    out = np.empty_like(u)
    _load().oracle_ipiano_step(pu, pup, pv, H, W, pk, pa, m, nf, float(lam),
                               float(tau), float(gamma), int(data_term),
                               out.ctypes.data_as(_dp))
    return out


def denoise(counts, k, alpha, lam, tau, gamma, iters, data_term, exact=False):
    """Eq. 3.7 end to end.  Unless ``exact``, filters, weights and scalars
    are rounded to float32 first: the values the GPU receives.
    Returns (u_hat, x_hat), both float64 H x W."""
    cast = (lambda a: np.asarray(a, np.float64)) if exact else \
        (lambda a: np.asarray(a, np.float32))
    sc = float if exact else _f32
    y, py = _d(np.asarray(counts, np.float32))
    H, W = y.shape
    nf, m, (kk, pk) = _bank(cast(k))
    a, pa = _d(cast(alpha))
    u = np.empty((H, W))
    x = np.empty((H, W))
    _load().oracle_denoise(py, H, W, pk, pa, m, nf, sc(lam), sc(tau),
                           sc(gamma), int(iters), int(data_term),
                           u.ctypes.data_as(_dp), x.ctypes.data_as(_dp))
    return u, x


def energy_grad(u, v, k, alpha, lam, data_term, want_grad=True):
    u, pu = _d(u)
    v, pv = _d(v)
    H, W = u.shape
    nf, m, (kk, pk) = _bank(k)
    a, pa = _d(alpha)
    g = np.empty((H, W)) if want_grad else None
    e = _load().oracle_energy_grad(pu, pv, H, W, pk, pa, m, nf, float(lam),
                                   int(data_term),
                                   g.ctypes.data_as(_dp) if want_grad else None)
    return e, g


def power_iteration(x0, k, alpha, iters):
    x, px = _d(x0)
    H, W = x.shape
    nf, m, (kk, pk) = _bank(k)
    a, pa = _d(alpha)
    return _load().oracle_power_iteration(px, H, W, pk, pa, m, nf, int(iters))


def set_threads(n):
    """Limit the OpenMP threads the oracle uses (None: library default)."""
    try:
        omp = ctypes.CDLL("libgomp.so.1")
        omp.omp_set_num_threads(int(n))
        return int(n)
    except OSError:
        return None


def bin3(y):
    """Sums of the 3 x 3 blocks of the symmetrically extended image."""
    y, py = _d(y)
    H, W = y.shape
    yb = np.empty(((H + 2) // 3, (W + 2) // 3))
    _load().oracle_bin3(py, H, W, yb.ctypes.data_as(_dp))
    return yb


def upsample3(xb, H, W):
    """Bilinear upscaling of xb / 9 (bin centres at 3i + 1) to H x W."""
    xb, pxb = _d(xb)
    x = np.empty((H, W))
    _load().oracle_upsample3(pxb, xb.shape[0], xb.shape[1], int(H), int(W),
                             x.ctypes.data_as(_dp))
    return x


def denoise_binned(counts, k, alpha, lam, tau, gamma, iters, data_term):
    """The binning variant: bin, denoise the binned counts (eq. 3.7 with the
    binned image's peak deciding the data term), upsample.  The binned
    counts are integers, so they stay exact in float32.  Returns
    (u_hat of the binned image, x_hat at full size)."""
    y = np.asarray(counts, np.float32)
    yb = bin3(y.astype(np.float64)).astype(np.float32)
    ub, xb = denoise(yb, k, alpha, lam, tau, gamma, iters, data_term)
    return ub, upsample3(xb, y.shape[0], y.shape[1])
