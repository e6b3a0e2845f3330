"""Dense brute-force model of the denoiser on tiny images (test helper).

Written independently of the oracle: every filter K_i is materialised as an
N x N matrix, column sources taken from numpy's own half-sample symmetric
padding of an index image (numpy's 'symmetric' mode repeats the edge
sample), K_i^T is the matrix transpose, and the proximal maps are found by a
scalar root solve of their optimality condition u - u~ + tau G'(u) = 0
(eq. 2.9) instead of the closed forms of eq. 3.3 / 3.5.
"""
import numpy as np
from scipy.optimize import brentq

QUADRATIC = 1
IDIV = 2


def dense_filter_matrix(k, H, W):
    """Matrix of u -> (k correlated with the symmetric extension of u)."""
    k = np.asarray(k, np.float64)
    m = k.shape[0]
    r = m // 2
    src = np.pad(np.arange(H * W).reshape(H, W), r, mode="symmetric")
    K = np.zeros((H * W, H * W))
    for y in range(H):
        for x in range(W):
            for a in range(m):
                for b in range(m):
                    K[y * W + x, src[y + a, x + b]] += k[a, b]
    return K


def dense_bank(k, H, W):
    return [dense_filter_matrix(ki, H, W) for ki in np.asarray(k)]


def grad_prior(u, Ks, alpha):
    """sum_i alpha_i K_i^T rho'(K_i u) with rho(z) = log(1 + z^2)."""
    g = np.zeros_like(u)
    for K, a in zip(Ks, alpha):
        z = K @ u
        g += a * (K.T @ (2.0 * z / (1.0 + z * z)))
    return g


def energy_prior(u, Ks, alpha):
    return sum(a * np.sum(np.log1p((K @ u) ** 2)) for K, a in zip(Ks, alpha))


def prox_root(ut, v, tau, lam, data_term):
    """argmin_u 1/2 (u - ut)^2 + tau G(u), from G'(u) by a bracketing solve."""
    tl = tau * lam
    if data_term == QUADRATIC:
        f = lambda u: u - ut + tl * (u - v)
        lo, hi = min(ut, v) - 1.0, max(ut, v) + 1.0
    else:
        f = lambda u: u - ut + tl * (1.0 - v / u)
        lo, hi = 1e-300, max(ut, 0.0) + tl * v + 1.0
        while f(lo) > 0:  # never happens for v > 0; kept as a guard
            lo *= 0.5
    return brentq(f, lo, hi, xtol=1e-15, rtol=8.9e-16, maxiter=500)


def denoise(counts, k, alpha, lam, tau, gamma, iters, data_term):
    y = np.asarray(counts, np.float64)
    H, W = y.shape
    Ks = dense_bank(np.asarray(k, np.float64), H, W)
    alpha = np.asarray(alpha, np.float64)
    v = 2.0 * np.sqrt(y.ravel() + 0.375)
    u, up = v.copy(), v.copy()
    for _ in range(iters):
        ut = u - tau * grad_prior(u, Ks, alpha) + gamma * (u - up)
        un = np.array([prox_root(a, b, tau, lam, data_term) for a, b in zip(ut, v)])
        up, u = u, un
    return u.reshape(H, W)
