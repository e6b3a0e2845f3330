"""The limits of fe_job on the gfx950 library.

* every rule a job description must satisfy is enforced before any device
  work (status FE_ERR_INVALID, a message naming the field), and a valid job
  still runs afterwards;
* the workspace must be present, 256-byte aligned and large enough;
* images of (almost) the largest size a job may have, H * W just below
  2^31 pixels (8.6 GB per plane, byte offsets past 2^32): a square one and
  one only r = 3 rows high.  After N iterations u^N at a pixel depends only
  on v within 2 r N of it, so the oracle on a crop with a margin of
  2 r N + 1 (or reaching the true border) gives sampled pixels exactly.

Tolerance as in test_gpu_parity: |gpu - oracle| <= 1e-4 * max(|oracle|, 1).
"""
import ctypes

import numpy as np
import pytest

import oracle
from synth import noisy_pair
from synth.workloads import IDIV, QUADRATIC, lambda_for_peak, prior_for, step_size_for

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


def _valid_job(fe, c, out):
    tau, gamma = step_size_for(7, 48)
    H, W = c.shape
    return dict(height=H, width=W, counts=c.data_ptr(), out=out.data_ptr(), out_anscombe=None,
                lambda_=lambda_for_peak(2.0), iterations=5, data_term=fe.DATA_AUTO,
                peak=2.0, tau=tau, gamma=gamma, precision=fe.PREC_FP32)


_BAD = [
    ("height below the radius", dict(height=2), "smaller than the filter radius"),
    ("width below the radius", dict(width=2), "smaller than the filter radius"),
    ("zero height", dict(height=0), "smaller than the filter radius"),
    ("2^31 pixels", dict(height=32768, width=65536), "too large"),
    ("46341^2 pixels", dict(height=46341, width=46341), "too large"),
    ("NULL counts", dict(counts=None), "counts is NULL"),
    ("lambda 0", dict(lambda_=0.0), "lambda"),
    ("lambda NaN", dict(lambda_=float("nan")), "lambda"),
    ("lambda inf", dict(lambda_=float("inf")), "lambda"),
    ("tau 0", dict(tau=0.0), "tau"),
    ("tau -1", dict(tau=-1.0), "tau"),
    ("gamma 1", dict(gamma=1.0), "gamma"),
    ("gamma -0.1", dict(gamma=-0.1), "gamma"),
    ("gamma NaN", dict(gamma=float("nan")), "gamma"),
    ("negative iterations", dict(iterations=-1), "negative iteration count"),
    ("data term 7", dict(data_term=7), "unknown data term"),
    ("auto with NaN peak", dict(peak=float("nan")), "peak"),
    ("precision 9", dict(precision=9), "unknown precision"),
]


@pytest.mark.parametrize("name,change,msg", _BAD, ids=[b[0] for b in _BAD])
def test_invalid_job_is_rejected(fe, torch, bank, name, change, msg):
    prior = bank[0]
    lib = fe.library()
    c = torch.full((16, 16), 3.0, device="cuda")
    out = torch.empty_like(c)
    good = _valid_job(fe, c, out)
    bad = dict(good, **change)
    # the bad job second: the whole batch is refused, nothing is enqueued
    jobs = (fe._Job * 2)(fe._Job(**good), fe._Job(**bad))
    sz = ctypes.c_size_t(123)
    assert lib.fe_workspace_size(prior.handle, jobs, 2, ctypes.byref(sz)) == fe.FE_ERR_INVALID
    assert sz.value == 0
    assert msg in lib.fe_last_error().decode()
    assert "job 1" in lib.fe_last_error().decode()
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    out.fill_(-7.0)
    st = lib.fe_denoise(prior.handle, jobs, 2, ws.data_ptr(), ws.numel(), None)
    assert st == fe.FE_ERR_INVALID
    torch.cuda.synchronize()
    assert bool((out == -7.0).all()), "a refused batch must not write any output"
    # the context still serves valid work
    one = (fe._Job * 1)(fe._Job(**good))
    assert lib.fe_workspace_size(prior.handle, one, 1, ctypes.byref(sz)) == fe.FE_OK
    assert lib.fe_denoise(prior.handle, one, 1, ws.data_ptr(), ws.numel(), None) == fe.FE_OK
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all()) and not bool((out == -7.0).any())


def test_workspace_rules(fe, torch, bank):
    prior = bank[0]
    lib = fe.library()
    c = torch.full((40, 50), 2.0, device="cuda")
    out = torch.empty_like(c)
    jobs = (fe._Job * 1)(fe._Job(**_valid_job(fe, c, out)))
    sz = ctypes.c_size_t()
    assert lib.fe_workspace_size(prior.handle, jobs, 1, ctypes.byref(sz)) == fe.FE_OK
    need = sz.value
    assert need >= 2 * 40 * 50 * 4
    ws = torch.empty(need + 1024, dtype=torch.uint8, device="cuda")
    base = ws.data_ptr()
    assert base % 256 == 0
    out.fill_(-7.0)
    cases = [(None, need, "workspace is NULL"), (base + 4, need, "256-byte aligned"),
             (base, need - 1, "workspace too small")]
    for ptr, nbytes, msg in cases:
        assert lib.fe_denoise(prior.handle, jobs, 1, ptr, nbytes, None) == fe.FE_ERR_INVALID
        assert msg in lib.fe_last_error().decode()
    torch.cuda.synchronize()
    assert bool((out == -7.0).all())
    assert lib.fe_denoise(prior.handle, jobs, 1, base, need, None) == fe.FE_OK
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())


# (H, W, period of the repeated seeded tile (rows, cols), peak, data term)
_MAX = [
    (46340, 46340, (2317, 2317), 4.0, QUADRATIC),     # 2,147,395,600 px
    (3, 715827882, (3, 4099), 1.0, IDIV),             # 2,147,483,646 px = 2^31 - 2
]


@pytest.mark.parametrize("H,W,period,peak,data_term", _MAX,
                         ids=["%dx%d" % (m[0], m[1]) for m in _MAX])
def test_largest_images_sampled_pixels(fe, torch, bank, H, W, period, peak, data_term):
    prior, k, a = bank
    tau, gamma = step_size_for(7, 48)
    iters, r = 4, 3
    assert H * W < 2 ** 31
    ph, pw = period
    _, tile = noisy_pair(51, 52, ph, pw, peak)
    tile = np.ascontiguousarray(tile, np.float32)
    lam = lambda_for_peak(peak)
    print("case %dx%d (%.3f G px) iters=%d dt=%d" % (H, W, H * W / 1e9, iters, data_term),
          flush=True)
    # the counts: the seeded tile repeated over the image (built on the device)
    t = torch.from_numpy(tile).cuda()
    c = t.repeat((H + ph - 1) // ph, (W + pw - 1) // pw)
    if c.shape != (H, W):
        c = c[:H, :W].contiguous()
    del t
    torch.cuda.synchronize()
    x, u = fe.denoise(c, prior, lam, iters, tau, gamma, data_term=data_term,
                      want_anscombe=True)
    torch.cuda.synchronize()
    del c
    g = np.random.default_rng(11)
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, W // 2), (H - 1, W // 3),
           (H // 3, W - 1), (min(1, H - 1), 1), (max(H - 2, 0), W - 3)]
    pts += [(int(g.integers(0, H)), int(g.integers(0, W))) for _ in range(24)]
    iy = torch.tensor([p[0] for p in pts], device="cuda")
    ix = torch.tensor([p[1] for p in pts], device="cuda")
    ug = u[iy, ix].cpu().numpy().astype(np.float64)
    xg = x[iy, ix].cpu().numpy().astype(np.float64)
    del x, u
    torch.cuda.empty_cache()
    marg = 2 * r * iters + 1
    for n, (py, px) in enumerate(pts):
        y0, y1 = max(0, py - marg), min(H, py + marg + 1)
        x0, x1 = max(0, px - marg), min(W, px + marg + 1)
        crop = tile[np.ix_(np.arange(y0, y1) % ph, np.arange(x0, x1) % pw)]
        uo, xo = oracle.denoise(crop, k, a, lam, tau, gamma, iters, data_term)
        ro, co = py - y0, px - x0
        eu = abs(ug[n] - uo[ro, co]) / max(abs(uo[ro, co]), 1.0)
        ex = abs(xg[n] - xo[ro, co]) / max(abs(xo[ro, co]), 1.0)
        assert eu <= TOL and ex <= TOL, ((py, px), eu, ex)


@pytest.mark.parametrize("H,W,period,peak,data_term", _MAX,
                         ids=["%dx%d" % (m[0], m[1]) for m in _MAX])
def test_largest_images_energy_and_gradient(fe, torch, bank, H, W, period, peak, data_term):
    """fe_energy_grad at the largest sizes (several launches over the tiles).
    (1) A constant image: every filter response vanishes (zero-mean filters,
    symmetric extension), so E = lambda * N * D(c, v) with D of eq. 3.4 / 3.6
    in closed form, which holds only if every pixel's data energy is counted
    by exactly one tile; the gradient is lambda * grad D everywhere.
    (2) A seeded image repeated with a period: the gradient at sampled pixels
    against the oracle on crops reaching 2r + 1 beyond them (grad E at a pixel
    depends on u within 2r), or to the true border."""
    prior, k, a = bank
    r = 3
    lam = 30.0
    print("energy/gradient case %dx%d (%.3f G px) dt=%d" % (H, W, H * W / 1e9, data_term),
          flush=True)
    # (1) constant counts and image
    cval, uval = 3.0, 3.25
    c = torch.full((H, W), cval, device="cuda")
    u = torch.full((H, W), uval, device="cuda")
    e, g = fe.energy_grad(c, u, prior, lam, data_term)
    torch.cuda.synchronize()
    v = 2.0 * np.sqrt(np.float64(np.float32(cval)) + 0.375)
    uu = np.float64(np.float32(uval))
    d = 0.5 * (uu - v) ** 2 if data_term == QUADRATIC else uu - v * np.log(uu)
    dg = (uu - v) if data_term == QUADRATIC else (1.0 - v / uu)
    e_ref = np.float64(np.float32(lam)) * H * W * d
    # 1e-5: the device rounds v to FP32 (about 1e-6 relative in d for the
    # quadratic term at u - v = -0.42); a tile counted twice or not at all
    # moves E by a whole tile's share, a row of overlap by ~1 %
    assert abs(e - e_ref) <= 1e-5 * abs(e_ref), (e, e_ref)
    gs = g[::max(1, H // 7), ::max(1, W // 7)].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(gs - lam * dg)) <= 1e-4 * max(abs(lam * dg), 1e-3), \
        np.max(np.abs(gs - lam * dg))
    del g
    # (2) the seeded tile repeated over the image
    ph, pw = period
    _, tile = noisy_pair(53, 54, ph, pw, peak)
    tile = np.ascontiguousarray(tile, np.float32)
    ut = (oracle.anscombe(tile) + np.random.default_rng(7).uniform(-0.3, 0.3, tile.shape)
          ).astype(np.float32)
    reps = ((H + ph - 1) // ph, (W + pw - 1) // pw)
    c.copy_(torch.from_numpy(tile).cuda().repeat(*reps)[:H, :W])
    u.copy_(torch.from_numpy(ut).cuda().repeat(*reps)[:H, :W])
    _, g = fe.energy_grad(c, u, prior, lam, data_term, want_energy=False)
    torch.cuda.synchronize()
    del c, u
    rng = np.random.default_rng(12)
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, W // 2), (H - 1, W // 3),
           (H // 3, W - 1), (min(1, H - 1), 1), (max(H - 2, 0), W - 3)]
    pts += [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(24)]
    iy = torch.tensor([p[0] for p in pts], device="cuda")
    ix = torch.tensor([p[1] for p in pts], device="cuda")
    gg = g[iy, ix].cpu().numpy().astype(np.float64)
    del g
    torch.cuda.empty_cache()
    marg = 2 * r + 1
    for n, (py, px) in enumerate(pts):
        y0, y1 = max(0, py - marg), min(H, py + marg + 1)
        x0, x1 = max(0, px - marg), min(W, px + marg + 1)
        rows, cols = np.arange(y0, y1) % ph, np.arange(x0, x1) % pw
        cc, uc = tile[np.ix_(rows, cols)], ut[np.ix_(rows, cols)].astype(np.float64)
        vc = oracle.anscombe(cc)
        _, go = oracle.energy_grad(uc, vc, k.astype(np.float64), a.astype(np.float64),
                                   np.float32(lam), data_term)
        gp = oracle.grad_prior(uc, k.astype(np.float64), a.astype(np.float64))
        scale = max(np.max(np.abs(gp)), np.max(np.abs(go - gp)), 1e-3)
        ro, co = py - y0, px - x0
        assert abs(gg[n] - go[ro, co]) <= 1e-4 * scale, ((py, px), gg[n], go[ro, co])
