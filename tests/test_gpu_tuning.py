"""The tile-height autotuner and the captured step sequence (HIP graph),
both through the C ABI.  Neither may change a result: tuned, forced and
replayed runs are compared bitwise with plain eager runs."""
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


def _specs(fe, torch, shapes, iters=12):
    tau, gamma = step_size_for(7, 48)
    out = []
    for i, (H, W, pk, prec) in enumerate(shapes):
        _, y = noisy_pair(700 + i, 800 + i, H, W, pk)
        out.append(fe.JobSpec(torch.from_numpy(y).cuda(), 40.0, iters, tau, gamma,
                              data_term="auto", peak=pk, precision=prec,
                              want_anscombe=True))
    return out


SHAPES = [(96, 130, 2.0, "fp32"), (64, 64, 8.0, "bf16"), (200, 70, 1.0, "fp16"),
          (150, 150, 4.0, "fp32")]


def _equal(torch, a, b):
    for (x0, u0), (x1, u1) in zip(a, b):
        assert torch.equal(u0, u1) and torch.equal(x0, x1)


def test_graph_replays_match_eager(fe, torch):
    k, a = prior_for(7, 48)
    prior = fe.Prior(k, a)
    specs = _specs(fe, torch, SHAPES)
    print("graph replay: %d jobs" % len(specs), flush=True)
    eager, g = fe.Batch(prior, specs), fe.Batch(prior, specs)
    for b in (eager, g):
        b.begin()
        b.advance([3, 3, 3, 3])
    counts = [4, 6, 0, 2]
    g.capture(counts)
    try:
        for r in range(4):
            eager.advance(counts)
            g.replay()
            # unrelated eager work and a synchronisation between replays
            junk = torch.randn(1 << 20, device="cuda") * 2.0
            torch.cuda.synchronize()
            del junk
            for se, sg in zip(eager.states, g.states):
                assert torch.equal(se, sg), "replay %d" % r
    finally:
        g.release_graph()
    _equal(torch, eager.end(), g.end())
    torch.cuda.synchronize()


def test_graph_rejects_odd_counts(fe, torch):
    k, a = prior_for(7, 48)
    prior = fe.Prior(k, a)
    b = fe.Batch(prior, _specs(fe, torch, SHAPES[:2]))
    b.begin()
    with pytest.raises(fe.FeError):
        b.capture([3, 2])
    torch.cuda.synchronize()


def test_autotune_and_forced_heights_are_bitwise(fe, torch, tmp_path):
    k, a = prior_for(7, 48)
    specs = _specs(fe, torch, SHAPES)
    ref = fe.denoise_jobs(fe.Prior(k, a), specs)
    torch.cuda.synchronize()
    prior = fe.Prior(k, a)
    fe.Batch(prior, specs).autotune(4)
    _equal(torch, ref, fe.denoise_jobs(prior, specs))
    path = tmp_path / "tune.txt"
    fe._check(fe.library().fe_tuning_save(prior.handle, str(path).encode()))
    lines = [ln for ln in path.read_text().splitlines() if not ln.startswith("#")]
    keys = sorted(ln.split()[2] for ln in lines)
    # one entry per precision group of the batch, keyed by its image sizes
    assert keys == ["p0:96x130,150x150,", "p1:64x64,", "p2:200x70,"], keys
    for ln in lines:
        nw, ty, key = ln.split()
        assert int(nw) in ((8, 12) if key.startswith("p0") else (12,)), ln
    # every variant and height gives the same bits: 8 or 12 waves for FP32;
    # the tallest tiles the LDS allows for 48 filters of 7 x 7: 128 rows for
    # FP32 with 8 waves, 96 with 12, 97 for BF16 / FP16
    for nw32, ty in ((8, 8), (12, 13), (8, 64), (12, 96), (8, 128)):
        forced = tmp_path / ("forced%d_%d.txt" % (nw32, ty))
        shape = {key: (nw32, ty) if key.startswith("p0") else (12, min(ty, 97))
                 for key in keys}
        forced.write_text("".join("%d %d %s\n" % (shape[key] + (key,)) for key in keys))
        p2 = fe.Prior(k, a)
        fe._check(fe.library().fe_tuning_load(p2.handle, str(forced).encode()))
        print("forced FP32 waves %d, tile height %d" % (nw32, ty), flush=True)
        _equal(torch, ref, fe.denoise_jobs(p2, specs))
    torch.cuda.synchronize()


def test_tuning_file_errors(fe, torch, tmp_path):
    k, a = prior_for(7, 48)
    prior = fe.Prior(k, a)
    lib = fe.library()
    assert lib.fe_tuning_load(prior.handle, str(tmp_path / "missing").encode()) == fe.FE_ERR_INVALID
    for bad in ("8 7 p0:64x64,\n", "8 129 p0:64x64,\n", "12 97 p0:64x64,\n",
                "8 64 p1:64x64,\n", "10 64 p0:64x64,\n", "x 64 p0:64x64,\n",
                "64 p0:64x64,\n"):
        f = tmp_path / "bad.txt"
        f.write_text(bad)
        assert lib.fe_tuning_load(prior.handle, str(f).encode()) == fe.FE_ERR_INVALID


def test_tuning_load_is_all_or_nothing(fe, torch, tmp_path):
    """A file with a good line before a bad one changes nothing."""
    k, a = prior_for(7, 48)
    prior = fe.Prior(k, a)
    lib = fe.library()
    f = tmp_path / "mixed.txt"
    f.write_text("12 64 p0:64x64,\n8 999 p0:64x64,\n")
    assert lib.fe_tuning_load(prior.handle, str(f).encode()) == fe.FE_ERR_INVALID
    out = tmp_path / "saved.txt"
    fe._check(lib.fe_tuning_save(prior.handle, str(out).encode()))
    assert [ln for ln in out.read_text().splitlines() if not ln.startswith("#")] == []
    f.write_text("# comment\n12 64 p0:64x64,\n\n8 100 p0:64x64,128x128,\n")
    fe._check(lib.fe_tuning_load(prior.handle, str(f).encode()))
    fe._check(lib.fe_tuning_save(prior.handle, str(out).encode()))
    assert sorted(ln for ln in out.read_text().splitlines() if not ln.startswith("#")) == \
        ["12 64 p0:64x64,", "8 100 p0:64x64,128x128,"]
