"""The continuous-batching server on the GPU: requests of different sizes,
iteration counts and precisions arrive while others run; each result must
be bitwise the one fe_denoise gives the same job alone."""
import time

import numpy as np
import pytest

from synth import noisy_pair
from synth.workloads import prior_for, step_size_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_05722_amd as fe
    from paper_1609_05722_amd import serving
    k, a = prior_for(7, 48)
    return torch, fe, serving, fe.Prior(k, a)


def _specs(fe, torch, n, seed=0):
    tau, gamma = step_size_for(7, 48)
    g = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        H, W = int(g.integers(8, 200)), int(g.integers(8, 200))
        pk = float(g.choice([0.5, 1.0, 2.0, 4.0, 8.0]))
        prec = ["fp32", "bf16", "fp16"][i % 3]
        _, y = noisy_pair(3000 + i, 4000 + i, H, W, pk)
        specs.append(fe.JobSpec(torch.from_numpy(y).cuda(), 40.0, int(g.integers(0, 45)),
                                tau, gamma, data_term="auto", peak=pk, precision=prec))
    return specs


@pytest.mark.parametrize("budget_mb,per_tick", [(256, 7), (1, 5)])
def test_served_results_equal_alone(env, budget_mb, per_tick):
    torch, fe, serving, prior = env
    specs = _specs(fe, torch, 14)
    srv = serving.Server(prior, budget_mb << 20, iters_per_tick=per_tick, max_active=64)
    arrivals = np.cumsum(np.random.default_rng(1).exponential(0.002, len(specs)))
    comps, outs, wall = serving.run_stream(srv, arrivals, specs, timeout_s=120)
    srv.close()
    torch.cuda.synchronize()
    assert [c["tag"] for c in comps] == list(range(len(specs)))
    for j, s in enumerate(specs):
        (x1, _), = fe.denoise_jobs(prior, [s])
        torch.cuda.synchronize()
        assert torch.equal(outs[j][0], x1), j
        c = comps[j]
        assert c["t_submit"] <= c["t_admit"] + 1e-6 and c["t_admit"] <= c["t_done"] + 1e-3


def test_server_rejects_job_larger_than_budget(env):
    torch, fe, serving, prior = env
    tau, gamma = step_size_for(7, 48)
    srv = serving.Server(prior, 64 << 10, iters_per_tick=5, max_active=4)
    y = torch.zeros((128, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(fe.FeError):
        srv.submit(fe.JobSpec(y, 10.0, 5, tau, gamma, data_term="idiv"), 0)
    srv.close()


def test_server_validation_mode_rejects_bad_request_and_keeps_serving(env):
    """FE_VALIDATE=1: a request with a NaN count is refused at submit; the
    server keeps serving the others, bitwise as alone."""
    import os
    torch, fe, serving, prior = env
    specs = _specs(fe, torch, 4, seed=9)
    os.environ["FE_VALIDATE"] = "1"
    try:
        srv = serving.Server(prior, 256 << 20, iters_per_tick=6, max_active=16)
        bad = specs[0].counts.clone()
        bad[1, 2] = float("nan")
        tau, gamma = step_size_for(7, 48)
        with pytest.raises(fe.FeError):
            srv.submit(fe.JobSpec(bad, 40.0, 10, tau, gamma, data_term="auto", peak=2.0), 99)
        comps, outs, wall = serving.run_stream(srv, np.zeros(len(specs)), specs, timeout_s=120)
        srv.close()
    finally:
        del os.environ["FE_VALIDATE"]
    torch.cuda.synchronize()
    assert sorted(c["tag"] for c in comps) == list(range(len(specs)))
    for j, s in enumerate(specs):
        (x1, _), = fe.denoise_jobs(prior, [s])
        torch.cuda.synchronize()
        assert torch.equal(outs[j][0], x1), j
