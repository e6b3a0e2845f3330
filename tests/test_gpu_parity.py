"""Parity of the gfx950 library (through the C ABI) with the FP64 oracle.

Tolerance: the FP32 GPU path must match the FP64 oracle within 1e-4
relative per pixel, |gpu - oracle| <= 1e-4 * max(|oracle|, 1), for both the
Anscombe-domain result u_hat and x_hat = I_C(u_hat).  The floor of 1 keeps
dark pixels, where x_hat is legitimately 0 or tiny, on an absolute 1e-4.
"""
import numpy as np
import pytest

import oracle
from synth import noisy_pair
from synth.workloads import (IDIV, QUADRATIC, fp32_config, oracle_config,
                             prior_for, step_size_for)

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def fe(torch):
    import paper_1609_05722_amd as fe
    fe.library()
    return fe


_PRIORS = {}


def _prior(fe, m, nf):
    key = (m, nf)
    if key not in _PRIORS:
        k, a = prior_for(m, nf)
        _PRIORS[key] = (fe.Prior(k, a), k, a)
    return _PRIORS[key]


def _run(fe, torch, prior, y, lam, tau, gamma, iters, data_term, precision="fp32"):
    c = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    x, u = fe.denoise(c, prior, lam, iters, tau, gamma, data_term=data_term,
                      precision=precision, want_anscombe=True)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64), x.cpu().numpy().astype(np.float64)


def _rel_err(a, ref):
    return np.max(np.abs(a - ref) / np.maximum(np.abs(ref), 1.0))


def _check(fe, torch, m, nf, y, lam, tau, gamma, iters, data_term, tol=TOL):
    prior, k, a = _prior(fe, m, nf)
    print("case H=%d W=%d m=%d nf=%d iters=%d dt=%d" % (y.shape + (m, nf, iters, data_term)),
          flush=True)
    ug, xg = _run(fe, torch, prior, y, lam, tau, gamma, iters, data_term)
    uo, xo = oracle.denoise(y, k, a, lam, tau, gamma, iters, data_term)
    eu, ex = _rel_err(ug, uo), _rel_err(xg, xo)
    assert eu <= tol and ex <= tol, (eu, ex)
    return eu, ex


def test_oracle_size_config(fe, torch):
    """64 x 64 at peak 4, 24 filters of 5 x 5, 100 iterations (I-div)."""
    cfg = oracle_config()
    j = cfg["jobs"][0]
    tau, gamma = step_size_for(5, 24)
    _, y = j.arrays()
    _check(fe, torch, 5, 24, y, j.lam, tau, gamma, j.iterations, j.data_term)


@pytest.mark.parametrize("data_term", [QUADRATIC, IDIV])
@pytest.mark.parametrize("shape", [(8, 8), (37, 53), (3, 3), (5, 200), (130, 67)])
def test_small_shapes(fe, torch, shape, data_term):
    """Several tiles with ragged tails, the H = W = r minimum, thin strips."""
    H, W = shape
    tau, gamma = step_size_for(7, 48)
    x, y = noisy_pair(40 + H, 60 + W, H, W, 3.0)
    _check(fe, torch, 7, 48, y, 50.0, tau, gamma, 30, data_term)


def test_zero_iterations_is_inverse_of_anscombe(fe, torch):
    tau, gamma = step_size_for(7, 48)
    x, y = noisy_pair(5, 6, 33, 47, 2.0)
    prior, k, a = _prior(fe, 7, 48)
    ug, xg = _run(fe, torch, prior, y, 10.0, tau, gamma, 0, IDIV)
    v = oracle.anscombe(y)
    assert _rel_err(ug, v) <= 1e-6
    assert _rel_err(xg, oracle.inverse_anscombe(v)) <= 1e-5


@pytest.mark.parametrize("data_term", [QUADRATIC, IDIV])
def test_zero_weights_keep_v(fe, torch, data_term):
    k, a = prior_for(7, 48)
    prior = fe.Prior(k, np.zeros_like(a))
    tau, gamma = step_size_for(7, 48)
    x, y = noisy_pair(7, 8, 40, 45, 4.0)
    ug, _ = _run(fe, torch, prior, y, 30.0, tau, gamma, 50, data_term)
    assert _rel_err(ug, oracle.anscombe(y)) <= 1e-5


_ORACLE_512 = {}


def _oracle_512(j, k, a, tau, gamma):
    """The oracle's result on one 512 x 512 baseline image, computed once per
    peak and shared by the FP32 and the reduced-precision tests."""
    if j.peak not in _ORACLE_512:
        _, y = j.arrays()
        _ORACLE_512[j.peak] = oracle.denoise(y, k, a, j.lam, tau, gamma, j.iterations,
                                             j.data_term)
    return _ORACLE_512[j.peak]


@pytest.mark.parametrize("peak", [1.0, 2.0, 4.0, 8.0])
def test_full_size_fp32(fe, torch, peak):
    """The four 512 x 512 baseline images (peaks 1, 2, 4: I-div; 8:
    quadratic), 48 filters of 7 x 7, 200 iterations, every pixel of u_hat
    and x_hat against the oracle.  Peaks 1 and 2 take the prox's a < 0
    branch (eq. 3.3 in its cancellation-free form) and the I_C clamp most
    often."""
    cfg = fp32_config()
    j = [jj for jj in cfg["jobs"] if jj.peak == peak][0]
    prior, k, a = _prior(fe, 7, 48)
    tau, gamma = step_size_for(7, 48)
    _, y = j.arrays()
    print("case 512x512 fp32 peak %g dt=%d" % (peak, j.data_term), flush=True)
    ug, xg = _run(fe, torch, prior, y, j.lam, tau, gamma, j.iterations, j.data_term)
    uo, xo = _oracle_512(j, k, a, tau, gamma)
    eu, ex = _rel_err(ug, uo), _rel_err(xg, xo)
    print("  max rel err u %.2e x %.2e" % (eu, ex), flush=True)
    assert eu <= TOL and ex <= TOL, (eu, ex)


def test_batch_equals_alone_and_is_deterministic(fe, torch):
    """Jobs of different sizes, data terms and iteration counts in one call
    give bitwise the same results as each job alone (the launches of the
    later iterations cover only the jobs still running), and repeated runs
    are bitwise equal."""
    prior, k, a = _prior(fe, 7, 48)
    tau, gamma = step_size_for(7, 48)
    shapes = [(64, 64, 1.0, 25), (97, 130, 8.0, 7), (20, 300, 2.0, 40), (256, 256, 4.0, 13)]
    specs, ys = [], []
    for i, (H, W, pk, its) in enumerate(shapes):
        _, y = noisy_pair(300 + i, 400 + i, H, W, pk)
        ys.append(y)
        specs.append(fe.JobSpec(torch.from_numpy(y).cuda(), 40.0, its, tau, gamma,
                                data_term="auto", peak=pk, want_anscombe=True))
    mix = fe.denoise_jobs(prior, specs)
    mix2 = fe.denoise_jobs(prior, specs)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        (x1, u1), = fe.denoise_jobs(prior, [s])
        torch.cuda.synchronize()
        assert torch.equal(u1, mix[i][1]) and torch.equal(x1, mix[i][0])
        assert torch.equal(mix2[i][1], mix[i][1])


def _energy_point(kind, y, v, k, a, data_term):
    """The image at which the energy is evaluated: v plus uniform noise
    (large filter responses), v itself, or the oracle's own iterate after 100
    iterations (smooth regions: small responses, where log(1 + z^2) needs
    its small-argument accuracy).  float32, as the GPU receives it."""
    if kind == "perturbed":
        return (v + np.random.default_rng(3).uniform(-0.3, 0.3, v.shape)).astype(np.float32)
    if kind == "v":
        return v.astype(np.float32)
    tau, gamma = step_size_for(7, 48)
    u, _ = oracle.denoise(y, k, a, 30.0, tau, gamma, 100, data_term)
    return u.astype(np.float32)


def _grad_scale(u32, go, k, a):
    """Scale of the gradient's error: the larger of its two parts, the
    prior's sum_i alpha_i K_i^T rho'(K_i u) and the data term's gradient.
    Near a stationary point the two cancel and grad E itself is small,
    while the rounding of each part stays relative to that part."""
    gp = oracle.grad_prior(u32.astype(np.float64), k.astype(np.float64), a.astype(np.float64))
    return max(np.max(np.abs(gp)), np.max(np.abs(go - gp)), 1e-3)


@pytest.mark.parametrize("point", ["perturbed", "v", "converged"])
@pytest.mark.parametrize("data_term", [QUADRATIC, IDIV])
def test_energy_and_gradient(fe, torch, data_term, point):
    prior, k, a = _prior(fe, 7, 48)
    x, y = noisy_pair(21, 22, 61, 75, 4.0)
    v = oracle.anscombe(y)
    u32 = _energy_point(point, y, v, k, a, data_term)
    e, g = fe.energy_grad(torch.from_numpy(y).cuda(), torch.from_numpy(u32).cuda(),
                          prior, 30.0, data_term)
    eo, go = oracle.energy_grad(u32.astype(np.float64), v, k.astype(np.float64),
                                a.astype(np.float64), np.float32(30.0), data_term)
    g = g.cpu().numpy().astype(np.float64)
    scale = _grad_scale(u32, go, k, a)
    print("energy_grad fp32 %s: energy rel %.2e, grad err %.2e of scale %.3g"
          % (point, abs(e - eo) / abs(eo), np.max(np.abs(g - go)) / scale, scale), flush=True)
    assert abs(e - eo) <= 1e-5 * abs(eo), (e, eo)
    assert np.max(np.abs(g - go)) <= 1e-4 * scale, np.max(np.abs(g - go))
    # energy only (no gradient buffer): the same energy, bitwise
    e2, g2 = fe.energy_grad(torch.from_numpy(y).cuda(), torch.from_numpy(u32).cuda(),
                            prior, 30.0, data_term, want_grad=False)
    assert g2 is None and e2 == e


@pytest.mark.parametrize("m,nf", [(3, 8), (5, 24), (7, 48)])
@pytest.mark.parametrize("shape", [(18, 17), (33, 50), (16, 16), (7, 41), (3, 20), (50, 3),
                                   (97, 130), (130, 59), (61, 117), (200, 70)])
def test_gradient_shapes(fe, torch, m, nf, shape):
    """The gradient on border-dominated and tile-boundary shapes: sizes down
    to r, widths one column past a tile (tiles are 64 - 2r columns wide),
    several tile rows and columns, 16-pixel blocks ending within r of the
    edge; energy and gradient against the oracle."""
    H, W = shape
    if min(H, W) < (m - 1) // 2:
        pytest.skip("below the filter radius")
    prior, k, a = _prior(fe, m, nf)
    x, y = noisy_pair(31 + H, 32 + W, H, W, 2.0)
    v = oracle.anscombe(y)
    u32 = (v + np.random.default_rng(H * W).uniform(-0.3, 0.3, v.shape)).astype(np.float32)
    e, g = fe.energy_grad(torch.from_numpy(y).cuda(), torch.from_numpy(u32).cuda(),
                          prior, 30.0, IDIV)
    eo, go = oracle.energy_grad(u32.astype(np.float64), v, k.astype(np.float64),
                                a.astype(np.float64), np.float32(30.0), IDIV)
    assert abs(e - eo) <= 1e-5 * abs(eo), (e, eo)
    g = g.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(g - go)) <= 1e-4 * _grad_scale(u32, go, k, a), \
        np.max(np.abs(g - go))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_energy_grad_batch_equals_alone(fe, torch, precision):
    """fe_energy_grad_batch over images of different sizes and data terms:
    each gradient bitwise that of fe_energy_grad on the image alone, each
    energy within the rounding of the per-tile FP32 sums (1e-6 relative) of
    it, and FP32 energies within 1e-5 of the oracle's; energy-only and
    gradient-only calls give the same values."""
    prior, k, a = _prior(fe, 7, 48)
    shapes = [(61, 75, 4.0, IDIV), (130, 59, 8.0, QUADRATIC), (8, 300, 1.0, IDIV),
              (200, 128, 2.0, QUADRATIC)]
    items, us = [], []
    for i, (H, W, pk, dt) in enumerate(shapes):
        _, y = noisy_pair(40 + i, 50 + i, H, W, pk)
        v = oracle.anscombe(y)
        u32 = (v + np.random.default_rng(i).uniform(-0.3, 0.3, v.shape)).astype(np.float32)
        us.append((y, v, u32))
        items.append((torch.from_numpy(y).cuda(), torch.from_numpy(u32).cuda(), 30.0, dt))
    es, gs = fe.energy_grad_batch(items, prior, precision=precision)
    e_only, none = fe.energy_grad_batch(items, prior, want_grad=False, precision=precision)
    none2, g_only = fe.energy_grad_batch(items, prior, want_energy=False, precision=precision)
    assert none is None and none2 is None
    torch.cuda.synchronize()
    for i, ((c, u, lam, dt), (y, v, u32)) in enumerate(zip(items, us)):
        e1, g1 = fe.energy_grad(c, u, prior, lam, dt, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(g1, gs[i]) and torch.equal(g1, g_only[i]), shapes[i]
        assert e_only[i] == es[i]
        assert abs(e1 - es[i]) <= 1e-6 * abs(e1), (shapes[i], e1, es[i])
        if precision == "fp32":
            eo, _ = oracle.energy_grad(u32.astype(np.float64), v, k.astype(np.float64),
                                       a.astype(np.float64), np.float32(lam), dt,
                                       want_grad=False)
            assert abs(es[i] - eo) <= 1e-5 * abs(eo), (shapes[i], es[i], eo)


def test_stepping_matches_denoise_and_resumes(fe, torch):
    """fe_begin + fe_advance in pieces + fe_end is bitwise fe_denoise; a
    state copied out after some iterations and restored continues to the
    bitwise same result (checkpoint / resume)."""
    prior, k, a = _prior(fe, 7, 48)
    tau, gamma = step_size_for(7, 48)
    specs = []
    for i, (H, W, pk) in enumerate([(70, 90, 2.0), (128, 64, 8.0)]):
        _, y = noisy_pair(500 + i, 600 + i, H, W, pk)
        specs.append(fe.JobSpec(torch.from_numpy(y).cuda(), 40.0, 37, tau, gamma,
                                data_term="auto", peak=pk, want_anscombe=True))
    ref = fe.denoise_jobs(prior, specs)
    b = fe.Batch(prior, specs)
    b.begin()
    b.advance([10, 10])
    b.advance([0, 27])
    b.advance([27, 0])
    out = b.end()
    torch.cuda.synchronize()
    for (x0, u0), (x1, u1) in zip(ref, out):
        assert torch.equal(u0, u1) and torch.equal(x0, x1)
    # checkpoint after 15 iterations, restore into fresh states, finish
    b2 = fe.Batch(prior, specs)
    b2.begin()
    b2.advance([15, 15])
    torch.cuda.synchronize()
    saved = [s.cpu().clone() for s in b2.states]
    done = [b2.done[i] for i in range(b2.n)]
    b3 = fe.Batch(prior, specs)
    for s_dst, s_src in zip(b3.states, saved):
        s_dst.copy_(s_src.cuda())
    for i in range(b3.n):
        b3.done[i] = done[i]
    b3.advance([22, 22])
    out3 = b3.end()
    torch.cuda.synchronize()
    for (x0, u0), (x1, u1) in zip(ref, out3):
        assert torch.equal(u0, u1) and torch.equal(x0, x1)


def _psnr(xh, x, peak):
    return 10.0 * np.log10(peak ** 2 / np.mean((xh - x) ** 2))


# Reduced-precision contractions (BF16 / FP16 operands, FP32 accumulation):
# reported against the FP64 oracle as max and RMS error of u_hat and the
# PSNR change of x_hat; the bar is |dPSNR| <= 0.05 dB, and the per-pixel
# errors stay within what operand rounding allows (8 and 11 significant
# bits on O(1) filter responses).
_MIXED_TOL = {"bf16": 5e-2, "fp16": 5e-3}


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("peak", [1.0, 8.0])
def test_mixed_precision_error_report(fe, torch, precision, peak):
    prior, k, a = _prior(fe, 7, 48)
    tau, gamma = step_size_for(7, 48)
    from synth.workloads import data_term_for_peak, lambda_for_peak
    x, y = noisy_pair(1, 101, 160, 144, peak)
    lam, dt = lambda_for_peak(peak), data_term_for_peak(peak)
    ug, xg = _run(fe, torch, prior, y, lam, tau, gamma, 200, dt, precision=precision)
    uo, xo = oracle.denoise(y, k, a, lam, tau, gamma, 200, dt)
    err = np.abs(ug - uo)
    dpsnr = _psnr(xg, x, peak) - _psnr(xo, x, peak)
    print("precision %s peak %g: max|du| %.3e rms %.3e dPSNR %+.4f dB"
          % (precision, peak, err.max(), np.sqrt(np.mean(err ** 2)), dpsnr), flush=True)
    assert abs(dpsnr) <= 0.05
    assert err.max() <= _MIXED_TOL[precision]


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("shape", [(8, 8), (3, 3), (3, 1500), (1500, 3), (37, 53), (5, 200)])
def test_reduced_precision_small_shapes(fe, torch, shape, precision):
    """BF16 / FP16 operands on the shapes where every tile touches a border
    (psi masked off the image, ghost rows and columns, partial blocks), both
    data terms in turn, within the reduced-precision bound of the oracle."""
    H, W = shape
    prior, k, a = _prior(fe, 7, 48)
    tau, gamma = step_size_for(7, 48)
    dt = QUADRATIC if (H + W) % 2 else IDIV
    _, y = noisy_pair(70 + H, 90 + W, H, W, 3.0)
    print("case %dx%d %s dt=%d" % (H, W, precision, dt), flush=True)
    ug, _ = _run(fe, torch, prior, y, 50.0, tau, gamma, 30, dt, precision=precision)
    uo, _ = oracle.denoise(y, k, a, 50.0, tau, gamma, 30, dt)
    err = np.abs(ug - uo)
    print("  max|du| %.3e rms %.3e" % (err.max(), np.sqrt(np.mean(err ** 2))), flush=True)
    assert err.max() <= _MIXED_TOL[precision]


@pytest.mark.parametrize("peak", [1.0, 2.0, 4.0, 8.0])
@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_mixed_precision_full_size(fe, torch, precision, peak):
    """The four 512 x 512 baseline images (peaks 1, 2, 4, 8; I-div, I-div,
    I-div, quadratic), 200 iterations, against the FP64 oracle: max and RMS
    error of u_hat and the PSNR change of x_hat, per image and precision."""
    cfg = fp32_config()
    j = [jj for jj in cfg["jobs"] if jj.peak == peak][0]
    prior, k, a = _prior(fe, 7, 48)
    tau, gamma = step_size_for(7, 48)
    x, y = j.arrays()
    ug, xg = _run(fe, torch, prior, y, j.lam, tau, gamma, j.iterations, j.data_term,
                  precision=precision)
    uo, xo = _oracle_512(j, k, a, tau, gamma)
    err = np.abs(ug - uo)
    dpsnr = _psnr(xg, x, j.peak) - _psnr(xo, x, j.peak)
    print("precision %s 512x512 peak %g: max|du| %.3e rms %.3e dPSNR %+.4f dB"
          % (precision, peak, err.max(), np.sqrt(np.mean(err ** 2)), dpsnr), flush=True)
    assert abs(dpsnr) <= 0.05
    assert err.max() <= _MIXED_TOL[precision]


def test_mixed_precision_batch_equals_alone(fe, torch):
    """A reduced-precision job gives bitwise the same result alone and in a
    batch that mixes precisions, sizes and data terms."""
    prior, k, a = _prior(fe, 7, 48)
    tau, gamma = step_size_for(7, 48)
    specs = []
    for i, (H, W, pk, pr) in enumerate([(90, 70, 1.0, "bf16"), (64, 200, 8.0, "fp16"),
                                        (128, 128, 4.0, "fp32"), (33, 47, 2.0, "bf16")]):
        _, y = noisy_pair(700 + i, 800 + i, H, W, pk)
        specs.append(fe.JobSpec(torch.from_numpy(y).cuda(), 40.0, 21, tau, gamma,
                                data_term="auto", peak=pk, precision=pr, want_anscombe=True))
    mix = fe.denoise_jobs(prior, specs)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        (x1, u1), = fe.denoise_jobs(prior, [s])
        torch.cuda.synchronize()
        assert torch.equal(u1, mix[i][1]) and torch.equal(x1, mix[i][0])


@pytest.mark.parametrize("peak", [0.5, 1.0])
@pytest.mark.parametrize("shape", [(96, 120), (101, 77)])
def test_binned_variant(fe, torch, peak, shape):
    """Binning: 3 x 3 sums, the denoiser on the binned counts with the data
    term picked by the binned peak (0.5 -> 4.5: I-div; 1 -> 9: quadratic),
    bilinear upsampling; against the oracle's binned pipeline."""
    from synth.workloads import data_term_for_peak, lambda_for_peak
    prior, k, a = _prior(fe, 7, 48)
    tau, gamma = step_size_for(7, 48)
    H, W = shape
    x, y = noisy_pair(900 + H, 950 + W, H, W, peak)
    lam = lambda_for_peak(9 * peak)
    spec = fe.JobSpec(torch.from_numpy(y).cuda(), lam, 60, tau, gamma, data_term="auto",
                      peak=peak, want_anscombe=True)
    (xg, ubg), = fe.denoise_binned_jobs(prior, [spec])
    torch.cuda.synchronize()
    ub, xo = oracle.denoise_binned(y, k, a, lam, tau, gamma, 60, data_term_for_peak(9 * peak))
    assert _rel_err(ubg.cpu().numpy().astype(np.float64), ub) <= TOL
    assert _rel_err(xg.cpu().numpy().astype(np.float64), xo) <= TOL


# Unit roundoff of the contraction operands.
_UNIT = {"bf16": 2.0 ** -9, "fp16": 2.0 ** -12}


@pytest.mark.parametrize("point", ["perturbed", "v"])
@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("data_term", [QUADRATIC, IDIV])
def test_energy_and_gradient_reduced_precision(fe, torch, precision, data_term, point):
    """Reduced-precision contractions in fe_energy_grad against the FP64
    oracle.  Operands are rounded to a unit roundoff u_r (2^-9 for BF16,
    2^-12 for FP16): u and k in the forward bank, z / (1 + z^2) and
    2 alpha k in the adjoint.  A numpy model of exactly those roundings,
    evaluated in FP64 on these images and on 128 x 128 and 64 x 64 ones,
    gives gradient errors of at most 4.5 u_r of the gradient's scale (the
    larger of its prior and data parts, at most max |grad| there) and energy errors
    of at most 1.7 u_r relative; the bounds are 12 u_r and 4 u_r."""
    prior, k, a = _prior(fe, 7, 48)
    _, y = noisy_pair(23, 24, 53, 66, 2.0)
    v = oracle.anscombe(y)
    u32 = _energy_point(point, y, v, k, a, data_term)
    lam = np.float32(30.0)
    e, g = fe.energy_grad(torch.from_numpy(y).cuda(), torch.from_numpy(u32).cuda(),
                          prior, float(lam), data_term, precision=precision)
    eo, go = oracle.energy_grad(u32.astype(np.float64), v, k.astype(np.float64),
                                a.astype(np.float64), lam, data_term)
    g = g.cpu().numpy().astype(np.float64)
    d = np.max(np.abs(g - go)) / _grad_scale(u32, go, k, a)
    de = abs(e - eo) / abs(eo)
    ur = _UNIT[precision]
    print("energy_grad %s %s: energy rel %.2e (%.2f u_r), grad rel %.2e (%.2f u_r)"
          % (precision, point, de, de / ur, d, d / ur), flush=True)
    assert de <= 4 * ur, (e, eo)
    assert d <= 12 * ur, d


def test_validation_mode_rejects_bad_counts(fe, torch):
    """FE_VALIDATE=1: negative, NaN or infinite counts are rejected before
    any work; valid counts give the same bits as without validation."""
    import os
    prior, k, a = _prior(fe, 7, 48)
    tau, gamma = step_size_for(7, 48)
    _, y = noisy_pair(25, 26, 40, 50, 4.0)
    good = torch.from_numpy(y).cuda()
    ref = fe.denoise(good, prior, 30.0, 10, tau, gamma)
    os.environ["FE_VALIDATE"] = "1"
    try:
        assert torch.equal(fe.denoise(good, prior, 30.0, 10, tau, gamma), ref)
        for bad_value in (-1.0, float("nan"), float("inf")):
            bad = good.clone()
            bad[17, 23] = bad_value
            with pytest.raises(fe.FeError) as err:
                fe.denoise(bad, prior, 30.0, 10, tau, gamma)
            assert err.value.status == fe.FE_ERR_INVALID
            with pytest.raises(fe.FeError):
                fe.energy_grad(bad, good, prior, 30.0, QUADRATIC)
    finally:
        del os.environ["FE_VALIDATE"]
    torch.cuda.synchronize()
