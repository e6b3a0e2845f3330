"""Serving: the continuous-batching server of libfe.so driven by a request
stream, with latency statistics.

    Server(prior, budget_bytes, iters_per_tick, max_active, ticks_in_flight)
    run_stream(server, arrivals, specs) -> per-request latencies

`python -m paper_1609_05722_amd.serving --requests N --loads 0.5,0.9` runs
the serving workload (Poisson arrivals, sides log-uniform on [64, 2048],
peaks {0.5, 1, 2, 4, 8}, 100-300 iterations) in two forms: continuous
batching with reduced-precision contractions, and one FP32 image at a time
(first in, first out), and prints images/s and p50/p99 latency per
offered load.
"""
import argparse
import ctypes
import json
import time

import numpy as np

from . import FeError, JobSpec, _Job, library, make_jobs


class _Cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("iters_per_tick", ctypes.c_int32),
                ("max_active", ctypes.c_int32), ("ticks_in_flight", ctypes.c_int32),
                ("tick_pixel_iters", ctypes.c_int64)]


class _Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


def _bind():
    lib = library()
    if getattr(lib, "_srv_bound", False):
        return lib
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.fe_server_create.argtypes = [vp, ctypes.POINTER(_Cfg), vp, ctypes.POINTER(vp)]
    lib.fe_server_create.restype = i32
    lib.fe_server_submit.argtypes = [vp, ctypes.POINTER(_Job), ctypes.c_uint64]
    lib.fe_server_submit.restype = i32
    lib.fe_server_poll.argtypes = [vp, ctypes.POINTER(_Completion), i32,
                                   ctypes.POINTER(i32), i32]
    lib.fe_server_poll.restype = i32
    lib.fe_server_load.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(ctypes.c_double)]
    lib.fe_server_load.restype = i32
    lib.fe_server_destroy.argtypes = [vp]
    lib.fe_server_destroy.restype = None
    lib.fe_server_last_error.argtypes = []
    lib.fe_server_last_error.restype = ctypes.c_char_p
    lib._srv_bound = True
    return lib


def _scheck(st):
    if st != 0:
        raise FeError(st, _bind().fe_server_last_error().decode())


class Server:
    """fe_server_create / submit / poll / destroy."""

    def __init__(self, prior, budget_bytes, iters_per_tick=20, max_active=4096,
                 ticks_in_flight=2, tick_pixel_iters=0):
        lib = _bind()
        self.prior = prior
        cfg = _Cfg(int(budget_bytes), int(iters_per_tick), int(max_active),
                   int(ticks_in_flight), int(tick_pixel_iters))
        h = ctypes.c_void_p()
        _scheck(lib.fe_server_create(prior.handle, ctypes.byref(cfg), None, ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self._keep = {}
        self._buf = (_Completion * 256)()

    def submit(self, spec, tag):
        arr, keep = make_jobs([spec])
        _scheck(self._lib.fe_server_submit(self._h, arr, int(tag)))
        self._keep[int(tag)] = keep[0]
        return keep[0][1], keep[0][2]   # (x_hat, u_hat or None) tensors

    def poll(self, wait_ms=0):
        n = ctypes.c_int32()
        _scheck(self._lib.fe_server_poll(self._h, self._buf, 256, ctypes.byref(n),
                                         int(wait_ms)))
        out = []
        for i in range(n.value):
            c = self._buf[i]
            out.append({"tag": c.tag, "iterations": c.iterations, "t_submit": c.t_submit,
                        "t_admit": c.t_admit, "t_done": c.t_done})
            self._keep.pop(int(c.tag), None)
        return out

    def load(self):
        p, a, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _scheck(self._lib.fe_server_load(self._h, ctypes.byref(p), ctypes.byref(a),
                                         ctypes.byref(t)))
        return p.value, a.value, t.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.fe_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: modules already torn down
            pass


def run_stream(server, arrivals, specs, timeout_s=600.0, progress_s=None):
    """Submit spec j at arrival time arrivals[j] (seconds from now) and
    collect every completion.  Returns (completions sorted by tag, outputs,
    wall seconds).  With progress_s, prints a progress line that often."""
    order = np.argsort(arrivals, kind="stable")
    done = {}
    outs = {}
    t0 = time.perf_counter()
    next_report = progress_s
    i = 0
    n = len(specs)
    while len(done) < n:
        if progress_s and time.perf_counter() - t0 >= next_report:
            print("serving: %.0f s, %d of %d submitted, %d done"
                  % (time.perf_counter() - t0, i, n, len(done)), flush=True)
            next_report += progress_s
        now = time.perf_counter() - t0
        while i < n and arrivals[order[i]] <= now:
            j = int(order[i])
            outs[j] = server.submit(specs[j], j)
            i += 1
        wait = 1 if i < n else 20
        if i < n:
            wait = max(0, min(20, int((arrivals[order[i]] - now) * 1e3)))
        for c in server.poll(wait_ms=wait):
            done[int(c["tag"])] = c
        if time.perf_counter() - t0 > timeout_s:
            raise TimeoutError("stream did not finish in %.0f s" % timeout_s)
    wall = time.perf_counter() - t0
    return [done[j] for j in range(n)], outs, wall


def latency_stats(comps, wall, pixel_iters):
    lat = np.array([c["t_done"] - c["t_submit"] for c in comps])
    t_first = min(c["t_submit"] for c in comps)
    t_last = max(c["t_done"] for c in comps)
    span = max(t_last - t_first, 1e-9)
    return {"requests": len(comps), "images_per_s": round(len(comps) / span, 2),
            "Mpixel_iter_per_s": round(pixel_iters / span / 1e6, 1),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "mean_ms": round(float(lat.mean()) * 1e3, 2), "span_s": round(span, 3),
            "wall_s": round(wall, 3)}


# ---------------------------------------------------------------------------
# the serving workload
_POOLS = {}


def _pool(side, peaks, n_clean=4, seed=77):
    """Noisy count images of side x side per peak, cropped per request.
    The clean images come from the synthetic generator (seeds 77..), one
    Poisson draw per (image, peak)."""
    from synth import clean_image, poisson_counts
    key = (side, tuple(peaks), n_clean, seed)
    if key in _POOLS:
        return _POOLS[key]
    pool = _POOLS[key] = {}
    for ci in range(n_clean):
        r = clean_image(seed + ci, side, side, 1.0)
        for pk in peaks:
            pool[(ci, pk)] = poisson_counts(1000 * (seed + ci) + int(pk * 10), pk * r)
    return pool


def build_requests(n, rate, precision, params=None, lo=64, hi=2048, pool_side=2048,
                   device="cuda", seed=5):
    """(arrival times, JobSpecs, pixel-iterations, crops) for n requests at
    `rate` requests/s.  Request j: size, peak and iteration count from
    synth.serving_stream; its counts are a crop at a seeded offset of the
    pool image for its peak (pool image j % 4).  crops[j] = (pool image,
    y, x, H, W, peak) locates its clean image for quality checks."""
    import torch
    from synth.workloads import serving_stream, step_size_for
    times, jobs = serving_stream(n, rate=rate, params=params, lo=lo, hi=hi, seed=seed)
    peaks = sorted({j.peak for j in jobs})
    pool = _pool(pool_side, peaks)
    tau, gamma = step_size_for(7, 48, params)
    specs, crops, pxit = [], [], 0
    for idx, j in enumerate(jobs):
        H, W = min(j.height, pool_side), min(j.width, pool_side)
        g = np.random.Generator(np.random.PCG64(100000 + idx))
        oy, ox = int(g.integers(0, pool_side - H + 1)), int(g.integers(0, pool_side - W + 1))
        crop = np.ascontiguousarray(pool[(idx % 4, j.peak)][oy:oy + H, ox:ox + W])
        specs.append(JobSpec(torch.from_numpy(crop).to(device), j.lam, j.iterations, tau,
                             gamma, data_term=j.data_term, peak=j.peak, precision=precision))
        crops.append((idx % 4, oy, ox, H, W, j.peak))
        pxit += H * W * j.iterations
    return times, specs, pxit, crops


_CLEAN = {}


def mean_psnr(outs, crops, pool_side=2048, n_clean=4, seed=77):
    """Mean PSNR (peak^2 / MSE in the count domain) of served outputs
    against the clean images they were cropped from."""
    import torch
    from synth import clean_image
    psnrs = []
    for j, (ci, oy, ox, H, W, pk) in enumerate(crops):
        key = (pool_side, seed + ci)
        if key not in _CLEAN:
            _CLEAN[key] = torch.from_numpy(
                clean_image(seed + ci, pool_side, pool_side, 1.0).astype(np.float32)).cuda()
        x = pk * _CLEAN[key][oy:oy + H, ox:ox + W]
        mse = torch.mean((outs[j][0] - x) ** 2).item()
        psnrs.append(10.0 * np.log10(pk * pk / max(mse, 1e-30)))
    return float(np.mean(psnrs))


# Work per tick of the batched form (pixel-iterations): 8 Mpx x 25
# iterations, a few milliseconds of device time, enough tiles to fill the
# chip; see serve().
TICK_WORK = 8 * (1 << 20) * 25


def serve(prior, times, specs, pxit, batched, budget_gb=64.0, iters_per_tick=25, crops=None,
          progress_s=None, tick_work=TICK_WORK):
    """One serving run; batched: continuous batching (oldest jobs first,
    tick_work pixel-iterations per tick, 0: every resident job every tick),
    else one job at a time."""
    import torch
    srv = Server(prior, int(budget_gb * (1 << 30)),
                 iters_per_tick=iters_per_tick if batched else 1 << 20,
                 max_active=4096 if batched else 1, ticks_in_flight=2,
                 tick_pixel_iters=tick_work if batched else 0)
    try:
        comps, outs, wall = run_stream(srv, times, specs, timeout_s=1200.0,
                                       progress_s=progress_s)
    finally:
        srv.close()
    torch.cuda.synchronize()
    stats = latency_stats(comps, wall, pxit)
    if crops is not None:
        stats["mean_psnr_db"] = round(mean_psnr(outs, crops), 4)
    return stats


def serving_report(prior, n_requests, loads=(0.9,), precision="bf16", max_side=2048,
                   log=None, forms=("batched", "single"), progress_s=None,
                   tick_work=TICK_WORK, same_rate_loads=()):
    """Both serving forms on the same request stream: saturation (every
    request at t = 0) and each offered load as a fraction of the form's own
    saturation rate; mean PSNR at saturation for the equal-quality check.
    same_rate_loads: the batched form also runs at these fractions of the
    one-image-at-a-time form's saturation rate (equal absolute arrival
    rates).  `log` receives one JSON line per finished run."""
    res = {"requests": n_requests, "contraction_precision": precision,
           "tick_pixel_iters": tick_work}
    runs = {"batched": ("batched_" + precision, True, precision),
            "single": ("single_fp32", False, "fp32")}
    # the one-image form first when both run: its rate sets the same-rate rows
    order = [f for f in ("single", "batched") if f in forms]
    for form in order:
        mode, batched, prec = runs[form]
        _, specs, pxit, crops = build_requests(n_requests, 1e9, prec, hi=max_side)
        sat = serve(prior, np.zeros(len(specs)), specs, pxit, batched, crops=crops,
                    progress_s=progress_s, tick_work=tick_work)
        del specs
        out = {"saturation": sat}
        if log:
            log(json.dumps({mode: {"saturation": sat}}))
        rows = [("load_%g" % ld, ld * sat["images_per_s"]) for ld in loads]
        if batched and "single_fp32" in res:
            rate1 = res["single_fp32"]["saturation"]["images_per_s"]
            rows += [("single_rate_%g" % ld, ld * rate1) for ld in same_rate_loads]
        for name, rate in rows:
            times, specs, pxit, _ = build_requests(n_requests, rate, prec, hi=max_side)
            out[name] = serve(prior, times, specs, pxit, batched, progress_s=progress_s,
                              tick_work=tick_work)
            out[name]["offered_per_s"] = round(rate, 2)
            del specs
            if log:
                log(json.dumps({mode: {name: out[name]}}))
        res[mode] = out
    if "batched_" + precision in res and "single_fp32" in res:
        b, f = res["batched_" + precision], res["single_fp32"]
        res["dpsnr_db"] = round(b["saturation"]["mean_psnr_db"]
                                - f["saturation"]["mean_psnr_db"], 4)
        res["speedup_images_per_s"] = round(b["saturation"]["images_per_s"]
                                            / f["saturation"]["images_per_s"], 3)
    return res


def main(argv=None):
    from . import Prior
    from synth.workloads import prior_for
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--loads", default="0.25,0.5,0.75,0.9,1.0,1.25")
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--max-side", type=int, default=2048)
    ap.add_argument("--progress", type=float, default=30.0,
                    help="seconds between progress lines during a run (0: none)")
    ap.add_argument("--forms", default="batched,single",
                    help="batched (continuous batching), single (one FP32 image at a time)")
    ap.add_argument("--tick-work", type=int, default=TICK_WORK,
                    help="pixel-iterations per tick of the batched form, oldest jobs "
                         "first (0: every resident job advances every tick)")
    ap.add_argument("--same-rate-loads", default="",
                    help="also run the batched form at these fractions of the "
                         "one-image form's saturation rate")
    a = ap.parse_args(argv)
    k, al = prior_for(7, 48)
    prior = Prior(k, al)
    same = [float(x) for x in a.same_rate_loads.split(",") if x]
    res = serving_report(prior, a.requests, [float(x) for x in a.loads.split(",")],
                         a.precision, a.max_side, log=lambda s: print(s, flush=True),
                         forms=tuple(a.forms.split(",")), progress_s=a.progress,
                         tick_work=a.tick_work, same_rate_loads=same)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
