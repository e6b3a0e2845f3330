"""The C ABI used from plain C (tests/c_abi_demo.c, built next to libfe.so
by the package build): no Python binding, no PyTorch in that process.  Its
result must match the FP64 oracle like the binding's."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from synth import noisy_pair
from synth.workloads import IDIV, lambda_for_peak, prior_for, step_size_for

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1609_05722_amd", "_build", "c_abi_demo")


def test_plain_c_client_matches_oracle(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.skip("c_abi_demo not built (paper_1609_05722_amd/build.py builds it)")
    H, W, iters = 90, 70, 30
    k, a = prior_for(7, 48)
    tau, gamma = step_size_for(7, 48)
    lam = lambda_for_peak(2.0)
    _, y = noisy_pair(61, 62, H, W, 2.0)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.array([H, W, 7, k.shape[0], iters, IDIV], np.int32).tobytes())
        f.write(np.array([lam, tau, gamma], np.float32).tobytes())
        f.write(np.ascontiguousarray(y, np.float32).tobytes())
        f.write(np.ascontiguousarray(k, np.float32).tobytes())
        f.write(np.ascontiguousarray(a, np.float32).tobytes())
    print("c_abi_demo %dx%d, %d iterations" % (H, W, iters), flush=True)
    r = subprocess.run([EXE, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr
    res = np.fromfile(out, np.float32).astype(np.float64)
    xg, ug = res[:H * W].reshape(H, W), res[H * W:].reshape(H, W)
    uo, xo = oracle.denoise(y, k, a, np.float32(lam), tau, gamma, iters, IDIV)
    for g, o in ((ug, uo), (xg, xo)):
        assert np.max(np.abs(g - o) / np.maximum(np.abs(o), 1.0)) <= 1e-4
