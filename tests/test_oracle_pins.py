"""Pins of the FP64 oracle against facts fixed by the paper or by mathematics.

None of these checks re-types the oracle's formula: each compares the oracle
with a printed constant, a library routine, a closed-form property, a dense
brute force or a finite-difference derivative.  ``pins`` holds the measured
discrepancies so that tests/test_oracle_mutants.py can show that planted
mistakes in the oracle source break them.
"""
import json
import os

import numpy as np
import pytest
from scipy.ndimage import correlate
from scipy.stats import poisson

import brute
import oracle
from synth import make_prior, noisy_pair

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _prior(m=5, nf=6, seed=3):
    k, a = make_prior(seed, m, m * m - 1)
    return k[:nf].astype(np.float64), a[:nf].astype(np.float64)


# ----------------------------------------------------------------------------
# measured discrepancies (each returns a non-negative number)
# ----------------------------------------------------------------------------
class pins:
    @staticmethod
    def energy_prior_vs_dense(H=8, W=8, m=5, nf=6):
        """FoE energy (eq. 2.5, rho of eq. 2.6) against the dense matrices."""
        k, a = _prior(m, nf)
        u = np.random.default_rng(9).uniform(0.5, 3.0, (H, W))
        ref = brute.energy_prior(u.ravel(), brute.dense_bank(k, H, W), a)
        return abs(oracle.energy_prior(u, k, a) - ref) / abs(ref)

    @staticmethod
    def energy_quadratic_offset(H=6, W=7, lam=3.0, d=0.25):
        """Quadratic data term (eq. 3.4) at u = v + d: lambda / 2 * N * d^2."""
        v = np.random.default_rng(10).uniform(1.0, 4.0, (H, W))
        return abs(oracle.energy_data(v + d, v, lam, 1) - 0.5 * lam * H * W * d * d)

    @staticmethod
    def idiv_energy_vs_kl(H=6, W=7, lam=2.5):
        """I-divergence data term (eq. 3.6): D(u) - D(v) = lambda times the
        generalised Kullback-Leibler divergence sum v log(v / u) - v + u
        (scipy.special.kl_div), relative to D(u)."""
        from scipy.special import kl_div
        g = np.random.default_rng(12)
        v = oracle.anscombe(g.poisson(2.0, (H, W)).astype(np.float64))
        u = v * g.uniform(0.7, 1.4, v.shape)
        d = oracle.energy_data(u, v, lam, 2) - oracle.energy_data(v, v, lam, 2)
        return abs(d - lam * np.sum(kl_div(v, u))) / abs(oracle.energy_data(u, v, lam, 2))

    @staticmethod
    def power_iteration_vs_eig(H=8, W=8, m=5, nf=6):
        """The step-size bound's lambda_max(sum_i alpha_i K_i^T K_i) from the
        oracle's power iteration against the dense eigenvalue problem."""
        k, a = _prior(m, nf)
        Ks = brute.dense_bank(k, H, W)
        A = sum(ai * K.T @ K for K, ai in zip(Ks, a))
        lam = np.linalg.eigvalsh(A).max()
        x0 = np.random.default_rng(1).standard_normal((H, W))
        return abs(oracle.power_iteration(x0, k, a, 3000) - lam) / lam

    @staticmethod
    def bin3_vs_padded(H=10, W=14):
        """Section 4 binning: 3 x 3 block sums of the symmetric extension to a
        multiple of 3 (numpy's symmetric padding), ragged on both axes."""
        y = np.random.default_rng(H * W).poisson(2.0, (H, W)).astype(np.float64)
        Hb, Wb = (H + 2) // 3, (W + 2) // 3
        e = np.pad(y, ((0, 3 * Hb - H), (0, 3 * Wb - W)), mode="symmetric")
        return np.abs(oracle.bin3(y) - e.reshape(Hb, 3, Wb, 3).sum(axis=(1, 3))).max()

    @staticmethod
    def upsample3_vs_scipy(Hb=5, Wb=7, H=14, W=20):
        """Bilinear upscaling of xb / 9 from the bin centres (3i + 1, 3j + 1),
        coordinates clamped to the outermost centres, against scipy."""
        from scipy.interpolate import RegularGridInterpolator
        xb = np.random.default_rng(13).uniform(0, 50, (Hb, Wb))
        f = RegularGridInterpolator((3 * np.arange(Hb) + 1.0, 3 * np.arange(Wb) + 1.0),
                                    xb / 9.0)
        yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
        pts = np.stack([np.clip(yy, 1, 3 * (Hb - 1) + 1), np.clip(xx, 1, 3 * (Wb - 1) + 1)],
                       -1)
        return np.abs(oracle.upsample3(xb, H, W) - f(pts)).max()

    @staticmethod
    def upsample3_centres():
        """At a bin centre the upscaled value is that bin's estimate / 9."""
        xb = np.random.default_rng(2).uniform(0, 9, (4, 5))
        x = oracle.upsample3(xb, 12, 15)
        return np.abs(x[1::3, 1::3] - xb / 9.0).max()

    @staticmethod
    def anscombe_zero():
        """Section 3.2: a zero count maps to sqrt(3/2)."""
        g = _golden()["anscombe_zero_count"]["value"]
        return abs(oracle.anscombe(np.zeros(1))[0] - g)

    @staticmethod
    def anscombe_variance():
        """Section 2.2: the transform makes Poisson data approximately unit
        variance.  Exact variance from the Poisson law at mean 40."""
        ys = np.arange(0, 400)
        p = poisson.pmf(ys, 40.0)
        f = oracle.anscombe(ys.astype(np.float64))
        mean = np.sum(p * f)
        return abs(np.sum(p * (f - mean) ** 2) - 1.0)

    @staticmethod
    def inverse_zero():
        """I_C(sqrt(3/2)) = 0: the printed coefficients sum to zero there."""
        return abs(oracle.inverse_anscombe_scalar(np.sqrt(1.5)))

    @staticmethod
    def inverse_derivative():
        """The derivative printed with the FoE_A training (Section 3.2)
        equals the numerical derivative of the oracle's I_C."""
        c = _golden()["inverse_anscombe_derivative"]
        s = np.sqrt(1.5)
        worst = 0.0
        for z in np.linspace(1.3, 12.0, 40):
            h = 1e-5 * z
            num = (oracle.inverse_anscombe_scalar(z + h)
                   - oracle.inverse_anscombe_scalar(z - h)) / (2 * h)
            printed = (c["c1"] * z + c["c2"] * s * z ** -2 + c["c3"] * z ** -3
                       + c["c4"] * s * z ** -4)
            worst = max(worst, abs(num - printed) / max(1.0, abs(printed)))
        return worst

    @staticmethod
    def inverse_unbiased():
        """eq. 2.4 approximates the exact unbiased inverse: mapping the exact
        expectation E[f_A(Y)], Y ~ Poisson(x), back through I_C returns x."""
        worst = 0.0
        for x in (0.05, 0.1, 0.2, 0.5, 1, 2, 3, 5, 10, 30, 100):
            ys = np.arange(0, int(x + 40 * np.sqrt(x) + 60))
            e = np.sum(poisson.pmf(ys, x) * oracle.anscombe(ys.astype(np.float64)))
            worst = max(worst, abs(oracle.inverse_anscombe_scalar(e) - x))
        return worst

    @staticmethod
    def inverse_asymptote():
        """For large counts I_C(f_A(y)) - y -> 1/4 (z^2/4 - 1/8 dominates)."""
        y = 1e6
        return abs(oracle.inverse_anscombe_scalar(oracle.anscombe(np.array([y]))[0]) - y - 0.25)

    @staticmethod
    def forward_vs_scipy(H=13, W=17, m=7):
        """K_i u equals scipy.ndimage.correlate with mode='reflect'
        (half-sample symmetric, centred taps)."""
        k, _ = _prior(m, 5)
        u = np.random.default_rng(1).standard_normal((H, W))
        z = oracle.filter_bank(u, k)
        return max(np.abs(z[i] - correlate(u, k[i], mode="reflect")).max()
                   for i in range(k.shape[0]))

    @staticmethod
    def forward_vs_dense(H=8, W=8, m=5):
        k, _ = _prior(m, 4)
        u = np.random.default_rng(2).standard_normal((H, W))
        z = oracle.filter_bank(u, k)
        return max(np.abs(z[i].ravel() - brute.dense_filter_matrix(k[i], H, W) @ u.ravel()).max()
                   for i in range(k.shape[0]))

    @staticmethod
    def adjoint_vs_dense(H=8, W=8, m=5):
        """sum_i K_i^T w_i equals the dense transposes applied to w."""
        k, _ = _prior(m, 4)
        w = np.random.default_rng(3).standard_normal((k.shape[0], H, W))
        g = oracle.filter_adjoint(w, k)
        ref = sum(brute.dense_filter_matrix(k[i], H, W).T @ w[i].ravel()
                  for i in range(k.shape[0]))
        return np.abs(g.ravel() - ref).max()

    @staticmethod
    def adjoint_identity(H=19, W=23, m=7, seed=4):
        """<K u, w> = <u, K^T w>, relative to the size of the terms."""
        k, _ = _prior(m, 6)
        g = np.random.default_rng(seed)
        u = g.standard_normal((H, W))
        w = g.standard_normal((k.shape[0], H, W))
        lhs = np.sum(oracle.filter_bank(u, k) * w)
        rhs = np.sum(u * oracle.filter_adjoint(w, k))
        scale = np.sum(np.abs(oracle.filter_bank(u, k) * w))
        return abs(lhs - rhs) / scale

    @staticmethod
    def constant_kernel(H=11, W=9, m=7):
        """Symmetric padding keeps constants, so K_i c = c * sum(k_i)
        everywhere, border included (zero for zero-mean filters)."""
        k, _ = _prior(m, 6)
        z = oracle.filter_bank(np.full((H, W), 3.7), k)
        return max(np.abs(z[i] - 3.7 * k[i].sum()).max() for i in range(k.shape[0]))

    @staticmethod
    def rho_prime_fd():
        """rho' is the derivative of rho = log(1 + z^2) (eq. 2.6)."""
        worst = 0.0
        for z in np.linspace(-6, 6, 61):
            h = 1e-6
            num = (oracle.rho(z + h) - oracle.rho(z - h)) / (2 * h)
            worst = max(worst, abs(num - oracle.rho_prime(z)))
        return worst

    @staticmethod
    def grad_prior_fd(H=9, W=10, m=5):
        """eq. 3.2 is the gradient of eq. 2.5: directional central differences."""
        k, a = _prior(m, 6)
        g = np.random.default_rng(5)
        u = 2.0 + g.standard_normal((H, W))
        grad = oracle.grad_prior(u, k, a)
        worst = 0.0
        for _ in range(4):
            d = g.standard_normal((H, W))
            h = 1e-5
            num = (oracle.energy_prior(u + h * d, k, a)
                   - oracle.energy_prior(u - h * d, k, a)) / (2 * h)
            worst = max(worst, abs(num - np.sum(grad * d)) / max(1.0, abs(num)))
        return worst

    @staticmethod
    def grad_full_fd(H=7, W=6, m=5):
        """Full energy gradient (prior + both data terms) against finite
        differences, pixel by pixel."""
        k, a = _prior(m, 4)
        g = np.random.default_rng(6)
        u = 2.0 + np.abs(g.standard_normal((H, W)))
        v = 1.5 + np.abs(g.standard_normal((H, W)))
        worst = 0.0
        for dt in (oracle.QUADRATIC, oracle.IDIV):
            _, grad = oracle.energy_grad(u, v, k, a, 3.0, dt)
            for p in range(0, H * W, 5):
                e = np.zeros(H * W)
                e[p] = 1e-6
                e = e.reshape(H, W)
                num = (oracle.energy_grad(u + e, v, k, a, 3.0, dt, False)[0]
                       - oracle.energy_grad(u - e, v, k, a, 3.0, dt, False)[0]) / 2e-6
                worst = max(worst, abs(num - grad.ravel()[p]) / max(1.0, abs(num)))
        return worst

    @staticmethod
    def prox_optimality():
        """eq. 2.9: the prox output satisfies u - u~ + tau G'(u) = 0, and it
        matches a bracketing root solve of that condition."""
        worst = 0.0
        g = np.random.default_rng(7)
        for dt in (oracle.QUADRATIC, oracle.IDIV):
            for _ in range(200):
                ut = g.uniform(-3, 8)
                v = g.uniform(np.sqrt(1.5), 8)
                tau, lam = 10 ** g.uniform(-4, -1), 10 ** g.uniform(-1, 2.5)
                u = oracle.prox_scalar(ut, v, tau, lam, dt)
                gp = lam * (u - v) if dt == oracle.QUADRATIC else lam * (1 - v / u)
                worst = max(worst, abs(u - ut + tau * gp) / max(1.0, abs(ut)))
                worst = max(worst, abs(u - brute.prox_root(ut, v, tau, lam, dt)) / max(1.0, abs(u)))
        return worst

    @staticmethod
    def ipiano_vs_dense(data_term, H=8, W=8, m=5, iters=100):
        """The whole scheme against the dense brute force on an 8 x 8 image."""
        k, a = make_prior(3, m, m * m - 1)
        k, a = k[:8], a[:8]
        y = np.random.default_rng(8).poisson(3.0, (H, W)).astype(np.float32)
        tau, gamma, lam = np.float32(0.004), np.float32(0.8), np.float32(20.0)
        u, _ = oracle.denoise(y, k, a, lam, tau, gamma, iters, data_term)
        ub = brute.denoise(y, k.astype(np.float64), a.astype(np.float64), float(lam),
                           float(tau), float(gamma), iters, data_term)
        return np.abs(u - ub).max()


# ----------------------------------------------------------------------------
# tests
# ----------------------------------------------------------------------------
def test_anscombe_zero_count():
    assert pins.anscombe_zero() < 1e-15


def test_anscombe_stabilises_variance():
    assert pins.anscombe_variance() < 0.02


def test_inverse_vanishes_at_zero_count_level():
    assert pins.inverse_zero() < 1e-14


def test_inverse_matches_printed_derivative():
    assert pins.inverse_derivative() < 1e-8


def test_inverse_is_nearly_unbiased():
    assert pins.inverse_unbiased() < 0.02


def test_inverse_asymptote():
    assert pins.inverse_asymptote() < 1e-3


def test_inverse_clamped_below_range():
    z = np.array([0.0, 0.3, 1.0, 1.2, np.sqrt(1.5) - 1e-12])
    assert np.all(oracle.inverse_anscombe(z) == 0.0)
    zz = np.linspace(np.sqrt(1.5), 20, 500)
    assert np.all(np.diff(oracle.inverse_anscombe(zz)) > 0)


def test_forward_matches_scipy_reflect():
    assert pins.forward_vs_scipy() < 1e-13
    assert pins.forward_vs_scipy(H=3, W=3, m=7) < 1e-13  # H = W = r


def test_forward_matches_dense():
    assert pins.forward_vs_dense() < 1e-13


def test_adjoint_matches_dense_transpose():
    assert pins.adjoint_vs_dense() < 1e-13
    assert pins.adjoint_vs_dense(H=3, W=5, m=7) < 1e-13


@pytest.mark.parametrize("H,W", [(19, 23), (3, 3), (4, 9), (33, 65), (8, 8), (64, 7)])
def test_adjoint_identity(H, W):
    assert pins.adjoint_identity(H, W) < 1e-13


def test_zero_mean_filters_annihilate_constants():
    assert pins.constant_kernel() < 1e-13


def test_rho_prime():
    assert pins.rho_prime_fd() < 1e-8


def test_grad_prior_finite_differences():
    assert pins.grad_prior_fd() < 1e-7


def test_full_gradient_finite_differences():
    assert pins.grad_full_fd() < 1e-6


def test_prox_optimality():
    assert pins.prox_optimality() < 1e-12


def test_idiv_prox_positive():
    for ut in (-50.0, -1.0, 0.0, 1e-8, 3.0):
        assert oracle.prox_scalar(ut, np.sqrt(1.5), 1e-3, 30.0, oracle.IDIV) > 0


@pytest.mark.parametrize("data_term", [1, 2])
def test_ipiano_matches_dense_brute_force(data_term):
    assert pins.ipiano_vs_dense(data_term) < 1e-10


@pytest.mark.parametrize("data_term", [1, 2])
def test_zero_weights_keep_v(data_term):
    """alpha = 0 leaves u = v: v is the prox's fixed point for both terms."""
    k, a = _prior(5, 6)
    y = np.random.default_rng(9).poisson(2.0, (12, 10)).astype(np.float32)
    u, _ = oracle.denoise(y, k, np.zeros_like(a), 10.0, 0.01, 0.8, 30, data_term,
                          exact=True)
    assert np.abs(u - oracle.anscombe(y)).max() < 1e-13


@pytest.mark.parametrize("data_term", [1, 2])
def test_constant_counts_are_fixed(data_term):
    """A constant image is a fixed point: zero-mean filters give K_i v = 0
    only under symmetric boundary handling."""
    k, a = _prior(7, 10)
    k = k - k.mean(axis=(1, 2), keepdims=True)  # zero-mean in double
    y = np.full((9, 13), 4.0, np.float32)
    u, x = oracle.denoise(y, k, a, 10.0, 0.01, 0.8, 20, data_term, exact=True)
    assert np.abs(u - oracle.anscombe(y)).max() < 1e-12


def _lyapunov(data_term, gamma, iters=60):
    """H_n = E(u^n) + gamma / (2 tau) |u^n - u^{n-1}|^2 for tau below
    2 (1 - gamma) / L with L = 2 lambda_max(sum alpha_i K_i^T K_i) from a
    dense eigen-solve (|rho''| <= 2).  Derivation: descent lemma for F,
    strong convexity of the prox objective, and Young's inequality on the
    inertial cross term give
      E(u+) <= E(u) + (L/2 - 1/tau + gamma/(2 tau)) |u+ - u|^2
                    + gamma/(2 tau) |u - u-|^2,
    which is H-monotone when tau <= 2 (1 - gamma) / L."""
    H = W = 8
    k, a = make_prior(5, 5, 24)
    k, a = k[:10].astype(np.float64), a[:10].astype(np.float64)
    Ks = brute.dense_bank(k, H, W)
    M = sum(ai * K.T @ K for K, ai in zip(Ks, a))
    L = 2.0 * np.linalg.eigvalsh(M).max()
    tau = 1.9 * (1 - gamma) / L
    lam = 5.0
    y = np.random.default_rng(10).poisson(2.0, (H, W)).astype(np.float64)
    v = oracle.anscombe(y)
    u_prev, u = v.copy(), v.copy()
    # start from a perturbed point so the first steps are not trivial
    u = v + np.random.default_rng(11).uniform(0, 0.5, (H, W))
    u_prev = u.copy()
    Hs = []
    for _ in range(iters):
        Hs.append(oracle.energy_grad(u, v, k, a, lam, data_term, False)[0]
                  + gamma / (2 * tau) * np.sum((u - u_prev) ** 2))
        u, u_prev = oracle.ipiano_step(u, u_prev, v, k, a, lam, tau, gamma, data_term), u
    return np.array(Hs)


@pytest.mark.parametrize("data_term", [1, 2])
@pytest.mark.parametrize("gamma", [0.0, 0.5, 0.8])
def test_lyapunov_descent(data_term, gamma):
    Hs = _lyapunov(data_term, gamma)
    assert np.all(np.diff(Hs) <= 1e-10 * np.abs(Hs[:-1]))
    assert Hs[-1] < Hs[0]


def test_energy_at_v_without_prior():
    """With alpha = 0 the energy is the data term alone: the quadratic term
    vanishes at u = v, and the I-divergence term (eq. 3.6) differs between
    any u and v by lambda times the generalised Kullback-Leibler divergence
    (scipy.special.kl_div)."""
    y = np.random.default_rng(12).poisson(2.0, (6, 7)).astype(np.float64)
    v = oracle.anscombe(y)
    k, a = _prior(5, 3)
    e_q, _ = oracle.energy_grad(v, v, k, np.zeros(3), 2.5, oracle.QUADRATIC, False)
    assert e_q == 0.0
    assert pins.idiv_energy_vs_kl() < 1e-12


def test_idiv_energy_infinite_off_domain():
    v = np.full((3, 3), 2.0)
    u = v.copy()
    u[1, 1] = 0.0
    k, a = _prior(5, 2)
    assert np.isinf(oracle.energy_grad(u, v, k, a, 1.0, oracle.IDIV, False)[0])


# ---- binning variant -------------------------------------------------------
@pytest.mark.parametrize("H,W", [(9, 12), (10, 11), (7, 8), (31, 17)])
def test_bin3_matches_padded_block_sums(H, W):
    assert pins.bin3_vs_padded(H, W) == 0.0


def test_upsample3_is_bilinear_with_clamped_edges():
    assert pins.upsample3_vs_scipy() < 1e-12


def test_energy_prior_matches_dense():
    assert pins.energy_prior_vs_dense() < 1e-12


def test_quadratic_energy_closed_form():
    assert pins.energy_quadratic_offset() < 1e-12


def test_power_iteration_matches_dense_eigenvalue():
    """The Lipschitz estimate behind tau (reading of Section 2.4)."""
    assert pins.power_iteration_vs_eig() < 1e-8


def test_upsample3_keeps_constants_and_centres():
    xb = np.full((4, 4), 27.0)
    assert np.abs(oracle.upsample3(xb, 12, 11) - 3.0).max() < 1e-14
    assert pins.upsample3_centres() < 1e-14


def test_iterations_are_local():
    """After N iterations u^N at a pixel depends only on v within 2 r N of
    it (forward and adjoint reach r each): the oracle on a crop with that
    margin (or reaching a true border) reproduces the full-image value.
    The GPU test of very large images relies on this."""
    from synth.workloads import prior_for, step_size_for
    k, a = prior_for(5, 24)
    tau, gamma = step_size_for(5, 24)
    _, y = noisy_pair(5, 6, 90, 110, 3.0)
    iters, r = 3, 2
    uf, xf = oracle.denoise(y, k, a, 30.0, tau, gamma, iters, 2)
    marg = 2 * r * iters + 1
    for (py, px) in [(0, 0), (45, 55), (89, 3), (20, 109), (60, 30)]:
        y0, y1 = max(0, py - marg), min(90, py + marg + 1)
        x0, x1 = max(0, px - marg), min(110, px + marg + 1)
        uc, xc = oracle.denoise(y[y0:y1, x0:x1], k, a, 30.0, tau, gamma, iters, 2)
        assert abs(uc[py - y0, px - x0] - uf[py, px]) < 1e-12
    # one pixel less of margin is not enough somewhere
    py, px = 45, 55
    m = marg - 2
    uc, _ = oracle.denoise(y[py - m:py + m + 1, px - m:px + m + 1], k, a, 30.0, tau, gamma,
                           iters, 2)
    assert abs(uc[m, m] - uf[py, px]) > 1e-12
