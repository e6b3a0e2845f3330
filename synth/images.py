"""Piecewise-smooth synthetic clean images and their Poisson observations.

The observation model is the paper's (Section 2.1, eq. 2.1): every count
y_p is drawn independently from a Poisson law with mean x_p, and a pixel of
mean zero gives a zero count.  The noise level is indexed by the peak, the
maximum of the clean image (Section 2.1).

Recipe for the clean image r in [0, 1] (all draws from one PCG64 stream, in
this order):
  * background level U(0.05, 0.25) plus a linear ramp of amplitude U(0, 0.15)
    along a random direction;
  * U{8..24} shapes, each an ellipse or a rotated rectangle with probability
    1/2: centre uniform over the image, half-extents log-uniform in
    [0.02, 0.25] * min(H, W), angle U[0, pi), level U(0, 1) plus an inner
    linear ramp of amplitude U(0, 0.2); later shapes overwrite earlier ones;
  * low-amplitude texture 0.04 * sum_k sin(2 pi f_k (x cos t_k + y sin t_k)
    + phi_k), k = 1..3, with f_k ~ U(1/48, 1/6) cycles per pixel;
  * clipped to [0, 1].
The clean image is then x = peak * r / max(r).
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def clean_image(seed, height, width, peak):
    """Clean intensity image x (float64, H x W) with max(x) == peak."""
    g = _rng(seed)
    H, W = int(height), int(width)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    r = np.full((H, W), g.uniform(0.05, 0.25))
    th = g.uniform(0.0, 2.0 * np.pi)
    amp = g.uniform(0.0, 0.15)
    proj = (xx * np.cos(th) + yy * np.sin(th))
    span = max(np.ptp(proj), 1.0)
    r += amp * (proj - proj.min()) / span
    n_shapes = int(g.integers(8, 25))
    side = float(min(H, W))
    for _ in range(n_shapes):
        is_ellipse = g.uniform() < 0.5
        cy, cx = g.uniform(0, H), g.uniform(0, W)
        ha = np.exp(g.uniform(np.log(0.02), np.log(0.25))) * side
        hb = np.exp(g.uniform(np.log(0.02), np.log(0.25))) * side
        ang = g.uniform(0.0, np.pi)
        level = g.uniform(0.0, 1.0)
        ramp = g.uniform(0.0, 0.2)
        rdir = g.uniform(0.0, 2.0 * np.pi)
        dy, dx = yy - cy, xx - cx
        u = dx * np.cos(ang) + dy * np.sin(ang)
        v = -dx * np.sin(ang) + dy * np.cos(ang)
        if is_ellipse:
            mask = (u / ha) ** 2 + (v / hb) ** 2 <= 1.0
        else:
            mask = (np.abs(u) <= ha) & (np.abs(v) <= hb)
        inner = level + ramp * ((dx * np.cos(rdir) + dy * np.sin(rdir))
                                / (2.0 * max(ha, hb)) + 0.5)
        r = np.where(mask, inner, r)
    for _ in range(3):
        f = g.uniform(1.0 / 48.0, 1.0 / 6.0)
        t = g.uniform(0.0, np.pi)
        phi = g.uniform(0.0, 2.0 * np.pi)
        r += 0.04 * np.sin(2.0 * np.pi * f * (xx * np.cos(t) + yy * np.sin(t)) + phi)
    r = np.clip(r, 0.0, 1.0)
    mx = r.max()
    if mx <= 0.0:
        r = np.ones_like(r)
        mx = 1.0
    return peak * r / mx


def poisson_counts(seed, x):
    """Poisson counts y ~ P(x) (eq. 2.1), stored as float32 integers."""
    g = _rng(seed)
    return g.poisson(np.asarray(x, np.float64)).astype(np.float32)


def noisy_pair(clean_seed, noise_seed, height, width, peak):
    """(x, y): clean image (float64) and float32 counts."""
    x = clean_image(clean_seed, height, width, peak)
    return x, poisson_counts(noise_seed, x)
