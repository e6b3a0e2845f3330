"""Write configs/params.json: the iteration parameters the paper leaves open.

TEST INFRASTRUCTURE: this script calls only the oracle and the seeded input
generators.  The values it writes are inputs (like the counts), passed as
the same float32 numbers to the GPU library and to the oracle.

  * gamma (iPiano inertia, eq. 2.8): 0.8, a common constant-parameter choice.
  * tau (iPiano step): 1.9 (1 - gamma) / L_hat, where L_hat bounds the
    Lipschitz constant of grad F for F = E_FoE (eq. 3.2).  The Hessian of F
    is sum_i alpha_i K_i^T Gamma_i K_i with rho'' in [-1/4, 2] (Section 2.5),
    so L <= 2 lambda_max(sum_i alpha_i K_i^T K_i); lambda_max comes from a
    power iteration of the oracle and is inflated by 5 %.
  * lambda per peak (data-term weight, eq. 3.7): the paper tunes it per noise
    level without giving values (Section 3.3); here each peak takes the
    value from a fixed grid that maximises the mean PSNR of the oracle's
    output over two seeded 128 x 128 calibration images (seeds disjoint from
    every workload).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from synth import make_prior, noisy_pair  # noqa: E402
from synth.workloads import PARAMS_PATH, QUADRATIC, IDIV  # noqa: E402

GAMMA = 0.8
PRIOR_SEED = 7
SAFETY = 1.05
LAMBDA_GRID = [5, 10, 20, 30, 50, 70, 100, 150, 200, 300, 500]
PEAKS = [0.5, 1, 2, 4, 8, 4.5, 9, 18, 36, 72]


def lipschitz(m, nf, size=128, iters=300):
    k, a = make_prior(PRIOR_SEED, m, nf)
    x0 = np.random.Generator(np.random.PCG64(11)).standard_normal((size, size))
    lam_max = oracle.power_iteration(x0, k.astype(np.float64),
                                     a.astype(np.float64), iters)
    return 2.0 * lam_max * SAFETY, lam_max


def psnr(xhat, x, peak):
    return 10.0 * np.log10(peak ** 2 / np.mean((xhat - x) ** 2))


def calibrate_lambda(tau, iters=200, size=128):
    k, a = make_prior(PRIOR_SEED, 7, 48)
    out = {}
    for peak in PEAKS:
        dt = QUADRATIC if peak >= 5 else IDIV
        pairs = [noisy_pair(900 + j, 950 + j, size, size, peak) for j in range(2)]
        scores = []
        for lam in LAMBDA_GRID:
            s = 0.0
            for x, y in pairs:
                _, xh = oracle.denoise(y, k, a, lam, tau, GAMMA, iters, dt)
                s += psnr(xh, x, peak)
            scores.append(s / len(pairs))
        best = LAMBDA_GRID[int(np.argmax(scores))]
        out[repr(float(peak))] = float(best)
        print("peak %-5s lambda %-5s psnr %s" % (peak, best,
              " ".join("%.2f" % s for s in scores)), flush=True)
    return out


def main():
    t0 = time.time()
    tau, lip = {}, {}
    for m, nf in ((5, 24), (7, 48)):
        L, lm = lipschitz(m, nf)
        key = "%dx%d_%d" % (m, m, nf)
        tau[key] = float(np.float32(1.9 * (1.0 - GAMMA) / L))
        lip[key] = {"lambda_max": lm, "L_hat": L}
        print(key, lip[key], "tau", tau[key], flush=True)
    lam = calibrate_lambda(tau["7x7_48"])
    params = {
        "gamma": GAMMA,
        "prior_seed": PRIOR_SEED,
        "filter_scale": 1.0,
        "tau": tau,
        "lipschitz": lip,
        "lambda_by_peak": lam,
        "lambda_grid": LAMBDA_GRID,
        "written_by": "oracle/calibrate.py",
    }
    os.makedirs(os.path.dirname(PARAMS_PATH), exist_ok=True)
    with open(PARAMS_PATH, "w") as f:
        json.dump(params, f, indent=1, sort_keys=True)
    print("wrote", PARAMS_PATH, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
