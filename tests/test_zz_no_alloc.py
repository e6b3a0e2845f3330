"""fe_advance_noalloc, the allocation-free variant of fe_advance (its job
table lives in the library's static device array), through the C ABI: its
states must be bitwise those of fe_advance on the same jobs, on two calls in
a row, the second with a smaller batch of smaller images (the array keeps
the first call's larger table)."""
import ctypes

import pytest

from synth import noisy_pair
from synth.workloads import prior_for, step_size_for

pytestmark = pytest.mark.gpu


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


def _specs(fe, torch, shapes, seed):
    tau, gamma = step_size_for(7, 48)
    out = []
    for i, (H, W, pk, prec) in enumerate(shapes):
        _, y = noisy_pair(seed + i, seed + 100 + i, H, W, pk)
        out.append(fe.JobSpec(torch.from_numpy(y).cuda(), 40.0, 0, tau, gamma,
                              data_term="auto", peak=pk, precision=prec,
                              want_anscombe=True))
    return out


def _compare(fe, torch, prior, shapes, counts, seed):
    specs = _specs(fe, torch, shapes, seed)
    ref, nal = fe.Batch(prior, specs), fe.Batch(prior, specs)
    for b in (ref, nal):
        b.begin()
    ref.advance(counts)
    nal.advance_noalloc(counts)
    torch.cuda.synchronize()
    for i, (sr, sn) in enumerate(zip(ref.states, nal.states)):
        assert torch.equal(sr, sn), "job %d %s" % (i, shapes[i])
    # a second advance of the same batch continues from the new states
    ref.advance([c + 1 for c in counts])
    nal.advance_noalloc([c + 1 for c in counts])
    for (xr, ur), (xn, un) in zip(ref.end(), nal.end()):
        assert torch.equal(ur, un) and torch.equal(xr, xn)
    torch.cuda.synchronize()


def test_noalloc_matches_advance_twice_then_smaller(fe, torch):
    k, a = prior_for(7, 48)
    prior = fe.Prior(k, a)
    first = [(150, 210, 2.0, "fp32"), (64, 64, 8.0, "bf16"), (200, 70, 1.0, "fp16"),
             (130, 130, 4.0, "fp32"), (37, 53, 8.0, "fp32")]
    print("noalloc: first call, %d jobs" % len(first), flush=True)
    _compare(fe, torch, prior, first, [6, 4, 5, 0, 3], 900)
    second = [(40, 33, 1.0, "fp32"), (20, 24, 8.0, "bf16")]
    print("noalloc: second call, %d smaller jobs" % len(second), flush=True)
    _compare(fe, torch, prior, second, [5, 2], 950)


def test_noalloc_rejects_too_many_jobs(fe, torch):
    k, a = prior_for(5, 24)
    prior = fe.Prior(k, a)
    n = 2049
    spec = _specs(fe, torch, [(8, 8, 4.0, "fp32")], 990)[0]
    arr, keep = fe.make_jobs([spec] * n)
    state = torch.zeros((2, 8, 8), dtype=torch.float32, device="cuda")
    sp = (ctypes.c_void_p * n)(*([state.data_ptr()] * n))
    done = (ctypes.c_int32 * n)()
    cnt = (ctypes.c_int32 * n)(*([1] * n))
    st = fe.library().fe_advance_noalloc(prior.handle, arr, sp, done, cnt, n, None)
    assert st == fe.FE_ERR_INVALID
    assert b"at most 2048" in fe.library().fe_last_error()
    torch.cuda.synchronize()
    assert torch.count_nonzero(state).item() == 0   # nothing was enqueued
