"""The workloads the denoiser is exercised on, as seeded job descriptions.

Each job is one noisy image: its size, the seeds of its clean image and of
its Poisson draw, its peak, the iteration count, the data-term weight lambda
and which data term the final scheme (eq. 3.7) selects for that peak
(quadratic for peak >= 5, I-divergence below).  Iteration parameters that
the paper leaves open (the iPiano step tau and inertia gamma, Section 2.4;
lambda per noise level, Section 3.3) are read from ``configs/params.json``.
"""
import json
import os
from dataclasses import dataclass, asdict

import numpy as np

from .images import noisy_pair
from .prior import make_prior

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PARAMS_PATH = os.path.join(_ROOT, "configs", "params.json")

QUADRATIC = 1
IDIV = 2


def load_params(path=PARAMS_PATH):
    with open(path) as f:
        return json.load(f)


def data_term_for_peak(peak):
    """Eq. 3.7: quadratic data term for peak >= 5, I-divergence below."""
    return QUADRATIC if peak >= 5.0 else IDIV


def lambda_for_peak(peak, params=None):
    """Data-term weight for a noise level, from the calibrated table.

    Peaks between table entries take the entry nearest in log(peak)."""
    params = params or load_params()
    table = params["lambda_by_peak"]
    keys = sorted(float(k) for k in table)
    best = min(keys, key=lambda k: abs(np.log(k) - np.log(peak)))
    for k, v in table.items():
        if float(k) == best:
            return float(v)
    raise KeyError(peak)


def step_size_for(m, n_filters, params=None):
    """(tau, gamma) for the prior with m x m filters and n_filters filters."""
    params = params or load_params()
    key = "%dx%d_%d" % (m, m, n_filters)
    return float(params["tau"][key]), float(params["gamma"])


@dataclass
class Job:
    height: int
    width: int
    peak: float
    clean_seed: int
    noise_seed: int
    iterations: int
    lam: float
    data_term: int

    def arrays(self):
        """(clean x float64, counts y float32) for this job."""
        return noisy_pair(self.clean_seed, self.noise_seed, self.height,
                          self.width, self.peak)

    def to_dict(self):
        return asdict(self)


def prior_for(m, n_filters, params=None):
    params = params or load_params()
    return make_prior(int(params["prior_seed"]), m, n_filters,
                      scale=float(params.get("filter_scale", 1.0)))


def _job(h, w, peak, cs, ns, its, params):
    return Job(int(h), int(w), float(peak), int(cs), int(ns), int(its),
               lambda_for_peak(peak, params), data_term_for_peak(peak))


def oracle_config(params=None):
    """One 64 x 64 image at peak 4 (I-divergence branch), 100 iterations;
    prior of 24 zero-mean 5 x 5 filters."""
    params = params or load_params()
    return dict(m=5, n_filters=24,
                jobs=[_job(64, 64, 4.0, 0, 100, 100, params)])


def fp32_config(params=None, size=512, iterations=200):
    """One 512 x 512 clean image at peaks 1, 2, 4, 8 (Poisson seeds 101..104),
    48 zero-mean 7 x 7 filters, 200 iterations."""
    params = params or load_params()
    jobs = [_job(size, size, p, 1, 101 + i, iterations, params)
            for i, p in enumerate((1.0, 2.0, 4.0, 8.0))]
    return dict(m=7, n_filters=48, jobs=jobs)


def _side_pair(g, lo, hi):
    s = np.exp(g.uniform(np.log(lo), np.log(hi)))
    a = np.exp(g.uniform(np.log(0.5), np.log(2.0)))
    return max(8, int(round(s * np.sqrt(a)))), max(8, int(round(s / np.sqrt(a))))


def batch_config(params=None, n_images=256, iterations=200, lo=128, hi=1024):
    """Uneven batch: sides log-uniform on [128, 1024], aspect log-uniform on
    [0.5, 2], peaks uniform over {1, 2, 4, 8}; image i uses clean seed
    1000 + i and noise seed 5000 + i."""
    params = params or load_params()
    g = np.random.Generator(np.random.PCG64(4))
    jobs = []
    for i in range(n_images):
        h, w = _side_pair(g, lo, hi)
        peak = float(g.choice([1.0, 2.0, 4.0, 8.0]))
        jobs.append(_job(h, w, peak, 1000 + i, 5000 + i, iterations, params))
    return dict(m=7, n_filters=48, jobs=jobs)


def serving_stream(n_requests=10000, rate=1.0, params=None, lo=64, hi=2048,
                   it_lo=100, it_hi=300, seed=5):
    """Poisson-arrival request stream: exponential inter-arrival times at
    ``rate`` requests/s, sides log-uniform on [lo, hi] (aspect as the batch),
    peaks uniform over {0.5, 1, 2, 4, 8}, iterations uniform on
    [it_lo, it_hi].  Request j uses clean seed 100000 + j and noise seed
    200000 + j.  Returns (arrival_times, jobs)."""
    params = params or load_params()
    g = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    times, jobs = [], []
    for j in range(n_requests):
        t += g.exponential(1.0 / rate)
        h, w = _side_pair(g, lo, hi)
        peak = float(g.choice([0.5, 1.0, 2.0, 4.0, 8.0]))
        its = int(g.integers(it_lo, it_hi + 1))
        times.append(t)
        jobs.append(_job(h, w, peak, 100000 + j, 200000 + j, its, params))
    return np.array(times), jobs


def _job_counts(job):
    return job.arrays()[1]


def job_counts(jobs, workers=8):
    """Noisy counts of many jobs, generated on `workers` spawned host
    processes (they never touch a GPU); same values as job.arrays()[1]."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = list(jobs)
    if workers <= 1 or len(jobs) < 8:
        return [_job_counts(j) for j in jobs]
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_job_counts, jobs, chunksize=4))
