"""Every built filter-bank shape through the C ABI against the FP64 oracle:
filter sides 3, 5 and 7 with 1, 2, 3 and 4 blocks of 16 filters (zero-padded
inside the library), FP32, BF16 and FP16 contractions.  Banks beyond the paper's
DCT construction (more filters than m*m - 1 zero-mean atoms) are seeded
random zero-mean filters; the step size comes from the oracle's power
iteration for each bank."""
import numpy as np
import pytest

import oracle
from synth import make_prior, noisy_pair
from synth.workloads import IDIV, QUADRATIC

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


def _bank(m, nf, seed):
    if nf <= m * m - 1:
        return make_prior(seed, m, nf)
    g = np.random.default_rng(seed)
    k = g.standard_normal((nf, m, m))
    k -= k.mean(axis=(1, 2), keepdims=True)
    k /= np.sqrt((k * k).sum(axis=(1, 2), keepdims=True))
    return k.astype(np.float32), (10.0 ** g.uniform(-1, 1, nf)).astype(np.float32)


def _step(k, a):
    """tau = 1.9 (1 - gamma) / L with L = 2 * 1.05 * lambda_max(sum alpha K^T K)."""
    gamma = 0.8
    x0 = np.random.default_rng(0).standard_normal((48, 48))
    lam_max = oracle.power_iteration(x0, k.astype(np.float64), a.astype(np.float64), 60)
    return np.float32(1.9 * (1 - gamma) / (2 * 1.05 * lam_max)), np.float32(gamma)


@pytest.mark.parametrize("m,nf", [(3, 8), (3, 20), (3, 40), (3, 64), (5, 16), (5, 24),
                                  (5, 40), (5, 64), (7, 16), (7, 20), (7, 48), (7, 64)])
def test_bank_shapes_fp32(fe, torch, m, nf):
    k, a = _bank(m, nf, 300 + 10 * m + nf)
    tau, gamma = _step(k, a)
    prior = fe.Prior(k, a)
    for dt, peak in ((IDIV, 2.0), (QUADRATIC, 8.0)):
        _, y = noisy_pair(31 + nf, 41 + m, 70, 90, peak)
        print("bank %dx%d x %d, data term %d" % (m, m, nf, dt), flush=True)
        x, u = fe.denoise(torch.from_numpy(y).cuda(), prior, 40.0, 20, float(tau),
                          float(gamma), data_term=dt, want_anscombe=True)
        torch.cuda.synchronize()
        uo, xo = oracle.denoise(y, k, a, np.float32(40.0), tau, gamma, 20, dt)
        for g, o in ((u, uo), (x, xo)):
            g = g.cpu().numpy().astype(np.float64)
            assert np.max(np.abs(g - o) / np.maximum(np.abs(o), 1.0)) <= TOL


# Reduced-precision bound on u_hat after 20 iterations: operand rounding to
# 8 (BF16) or 11 (FP16) significant bits on O(1) responses.
_P16_TOL = {"bf16": 5e-2, "fp16": 1e-2}


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("m,nf", [(3, 8), (3, 20), (3, 64), (5, 16), (5, 24), (5, 40),
                                  (7, 20), (7, 48), (7, 64)])
def test_bank_shapes_reduced_precision(fe, torch, m, nf, precision):
    """BF16 / FP16 operands, every filter side with 1 to 4 blocks of 16
    filters: within the reduced-precision bound of the FP64 oracle."""
    k, a = _bank(m, nf, 300 + 10 * m + nf)
    tau, gamma = _step(k, a)
    prior = fe.Prior(k, a)
    _, y = noisy_pair(51 + nf, 61 + m, 70, 90, 2.0)
    x, u = fe.denoise(torch.from_numpy(y).cuda(), prior, 40.0, 20, float(tau), float(gamma),
                      data_term=IDIV, precision=precision, want_anscombe=True)
    torch.cuda.synchronize()
    uo, _ = oracle.denoise(y, k, a, np.float32(40.0), tau, gamma, 20, IDIV)
    err = np.abs(u.cpu().numpy().astype(np.float64) - uo)
    print("bank %dx%d x %d %s: max %.2e rms %.2e" % (m, m, nf, precision, err.max(),
                                                    np.sqrt(np.mean(err ** 2))), flush=True)
    assert err.max() <= _P16_TOL[precision]
