"""Edge cases and full sizes of the gfx950 library against the FP64 oracle.

* degenerate inputs: an empty batch, all-zero counts (v is exactly
  sqrt(3/2), a fixed point), no inertia (gamma = 0), very bright images;
* extreme aspect ratios down to the filter radius;
* the largest serving size (2048 x 2048), every pixel;
* a 4096 x 4096 image on sampled pixels: after N iterations u^N at a pixel
  depends only on v within 2 r N of it, so the oracle run on a crop that
  keeps a margin of 2 r N + 1 around the sample (or reaches a true image
  border) gives that pixel exactly;
* the 256-image uneven batch in one call, as the benchmark launches it: the
  smallest images against the oracle, others bitwise against runs alone.

Tolerance as in test_gpu_parity: |gpu - oracle| <= 1e-4 * max(|oracle|, 1).
"""
import ctypes

import numpy as np
import pytest

import oracle
from synth import noisy_pair
from synth.workloads import (IDIV, QUADRATIC, batch_config, job_counts, lambda_for_peak,
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


@pytest.fixture(scope="module")
def bank(fe):
    k, a = prior_for(7, 48)
    return fe.Prior(k, a), k, a


def _rel_err(a, ref):
    return float(np.max(np.abs(a - ref) / np.maximum(np.abs(ref), 1.0)))


def _gpu(fe, torch, prior, y, lam, iters, data_term, gamma=None, precision="fp32"):
    tau, g0 = step_size_for(7, 48)
    gamma = g0 if gamma is None else gamma
    c = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    x, u = fe.denoise(c, prior, lam, iters, tau, gamma, data_term=data_term,
                      precision=precision, want_anscombe=True)
    torch.cuda.synchronize()
    return u.cpu().numpy().astype(np.float64), x.cpu().numpy().astype(np.float64)


def _check_full(fe, torch, bank, y, lam, iters, data_term, gamma=None):
    prior, k, a = bank
    tau, g0 = step_size_for(7, 48)
    gamma = g0 if gamma is None else gamma
    print("case %dx%d iters=%d dt=%d gamma=%g" % (y.shape + (iters, data_term, gamma)),
          flush=True)
    ug, xg = _gpu(fe, torch, prior, y, lam, iters, data_term, gamma)
    uo, xo = oracle.denoise(y, k, a, lam, tau, gamma, iters, data_term)
    eu, ex = _rel_err(ug, uo), _rel_err(xg, xo)
    assert eu <= TOL and ex <= TOL, (eu, ex)
    return ug, xg


def test_empty_batch(fe, torch, bank):
    prior = bank[0]
    lib = fe.library()
    sz = ctypes.c_size_t()
    assert lib.fe_workspace_size(prior.handle, None, 0, ctypes.byref(sz)) == fe.FE_OK
    assert lib.fe_denoise(prior.handle, None, 0, None, 0, None) == fe.FE_OK
    assert fe.denoise_jobs(prior, []) == []
    torch.cuda.synchronize()


@pytest.mark.parametrize("data_term", [QUADRATIC, IDIV])
def test_all_zero_counts(fe, torch, bank, data_term):
    """y = 0 everywhere: v = 2 sqrt(3/8) = sqrt(3/2) is a fixed point of
    every step (zero-mean filters, the prox keeps v) and I_C(sqrt(3/2)) = 0."""
    y = np.zeros((70, 90), np.float32)
    ug, xg = _check_full(fe, torch, bank, y, 50.0, 30, data_term)
    assert np.abs(ug - np.sqrt(1.5)).max() < 1e-5
    assert np.abs(xg).max() < 1e-5


@pytest.mark.parametrize("data_term", [QUADRATIC, IDIV])
def test_no_inertia(fe, torch, bank, data_term):
    """gamma = 0: plain forward-backward splitting."""
    _, y = noisy_pair(31, 32, 80, 100, 2.0)
    _check_full(fe, torch, bank, y, 40.0, 40, data_term, gamma=0.0)


def test_bright_image(fe, torch, bank):
    """Peak 1e5 (u up to ~630): large filter responses, quadratic term."""
    _, y = noisy_pair(33, 34, 96, 96, 1.0e5)
    _check_full(fe, torch, bank, y, 100.0, 40, QUADRATIC)


@pytest.mark.parametrize("shape", [(3, 1500), (1500, 3), (4, 700), (700, 5)])
def test_extreme_aspect(fe, torch, bank, shape):
    _, y = noisy_pair(35, 36, shape[0], shape[1], 1.0)
    _check_full(fe, torch, bank, y, lambda_for_peak(1.0), 25, IDIV)


def test_largest_serving_size_every_pixel(fe, torch, bank):
    """2048 x 2048 (the serving stream's largest side), peak 0.5, I-div."""
    _, y = noisy_pair(37, 38, 2048, 2048, 0.5)
    _check_full(fe, torch, bank, y, lambda_for_peak(0.5), 12, IDIV)


def _big_counts(n_tiles=4, side=1024):
    """(n_tiles * side)^2 counts assembled from distinct seeded images."""
    rows = []
    for i in range(n_tiles):
        rows.append(np.concatenate([noisy_pair(40 + 8 * i + j, 80 + 8 * i + j, side, side,
                                               2.0 + j)[1] for j in range(n_tiles)], axis=1))
    return np.ascontiguousarray(np.concatenate(rows, axis=0))


def test_large_image_sampled_pixels(fe, torch, bank):
    prior, k, a = bank
    tau, gamma = step_size_for(7, 48)
    iters, r = 4, 3
    y = _big_counts()
    H, W = y.shape
    lam = lambda_for_peak(4.0)
    print("case %dx%d iters=%d sampled" % (H, W, iters), flush=True)
    ug, xg = _gpu(fe, torch, prior, y, lam, iters, QUADRATIC)
    g = np.random.default_rng(7)
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (0, W // 2), (H // 2, 0),
           (H - 1, 1234), (777, W - 1), (1, 1), (H - 2, W - 3)]
    pts += [(int(g.integers(0, H)), int(g.integers(0, W))) for _ in range(30)]
    marg = 2 * r * iters + 1
    for (py, px) in pts:
        y0, y1 = max(0, py - marg), min(H, py + marg + 1)
        x0, x1 = max(0, px - marg), min(W, px + marg + 1)
        uo, xo = oracle.denoise(y[y0:y1, x0:x1], k, a, lam, tau, gamma, iters, QUADRATIC)
        eu = abs(ug[py, px] - uo[py - y0, px - x0]) / max(abs(uo[py - y0, px - x0]), 1.0)
        ex = abs(xg[py, px] - xo[py - y0, px - x0]) / max(abs(xo[py - y0, px - x0]), 1.0)
        assert eu <= TOL and ex <= TOL, ((py, px), eu, ex)


def test_uneven_batch_config(fe, torch, bank):
    """All 256 images of the uneven batch in one fe_denoise call (200
    iterations): the four smallest against the oracle on every pixel, and
    two others bitwise equal to the same job run alone."""
    prior, k, a = bank
    tau, gamma = step_size_for(7, 48)
    cfg = batch_config()
    jobs = cfg["jobs"]
    ys = job_counts(jobs)
    print("uneven batch: %d images, %.1f Mpx" % (len(jobs), sum(y.size for y in ys) / 1e6),
          flush=True)
    specs = [fe.JobSpec(torch.from_numpy(y).cuda(), j.lam, j.iterations, tau, gamma,
                        data_term=j.data_term, peak=j.peak, want_anscombe=True)
             for y, j in zip(ys, jobs)]
    out = fe.denoise_jobs(prior, specs)
    torch.cuda.synchronize()
    order = np.argsort([y.size for y in ys])
    for i in order[:4]:
        j = jobs[i]
        uo, xo = oracle.denoise(ys[i], k, a, j.lam, tau, gamma, j.iterations, j.data_term)
        xg = out[i][0].cpu().numpy().astype(np.float64)
        ug = out[i][1].cpu().numpy().astype(np.float64)
        eu, ex = _rel_err(ug, uo), _rel_err(xg, xo)
        print("image %d %dx%d peak %g: %.2e %.2e" % (i, j.height, j.width, j.peak, eu, ex),
              flush=True)
        assert eu <= TOL and ex <= TOL, (i, eu, ex)
    for i in (order[len(order) // 2], order[-1]):
        (x1, u1), = fe.denoise_jobs(prior, [specs[i]])
        torch.cuda.synchronize()
        assert torch.equal(u1, out[i][1]) and torch.equal(x1, out[i][0])
