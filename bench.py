"""Throughput benchmark of the FoE Poisson denoiser on one MI355X.

One step = one fe_denoise call over the FP32 baseline workload: one 512 x 512
synthetic clean image at peaks 1, 2, 4, 8 (four noisy images), 48 zero-mean
7 x 7 filters, 200 iPiano iterations each, symmetric boundary, data term by
peak (eq. 3.7).  Inputs are resident in HBM before timing starts.

Prints one JSON line:  value = whole-step Mpixel-iterations per second,
plus images/s, the roofline of the dominant kernel and the FP64 oracle
timed on the host cores on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FoE step Mpixel-iter/s vs roofline; served images/s + p50/p99 latency"
FP32_PEAK_TFLOPS = 157.3   # MI355X dense FP32 (matrix)
HBM_PEAK_GBS = 8000.0
MFMA16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 / fp16 matrix


def flops_per_px_it(m, nf):
    """Algorithmic contraction flops of one pixel-iteration: the forward and
    adjoint filter banks, 2 * 2 * N_f * m^2 (a multiply and an add per tap)."""
    return 4 * nf * m * m


VALU_LANE_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: one FP32 op per slot


def valu_slots_per_px_it(nf):
    """Algorithmic FP32 vector work of one pixel-iteration in lane issue
    slots: the influence of every filter, z / (1 + z^2) (an FMA, a reciprocal
    at a quarter of the full rate, so 4 slots, and a multiply), plus the
    inertial step (3) and the prox (about 10 with its square root)."""
    return nf * (1 + 4 + 1) + 3 + 10


def hbm_bytes_per_px_it():
    """Algorithmic HBM bytes of one pixel-iteration in FP32: read u^n,
    u^{n-1} and the counts y, write u^{n+1}."""
    return 16


KERNEL_SOURCE = os.path.join(ROOT, "paper_1609_05722_amd", "csrc", "kernels_fused.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_step_4x512_traffic.json")


def kernel_hash():
    from paper_1609_05722_amd.rocprof_summary import code_hash
    return code_hash(KERNEL_SOURCE)


def recorded_traffic(args):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes, if they were taken on this exact kernel
    source and workload; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_code_sha256_16") != kernel_hash() or rec.get("size") != args.size \
            or rec.get("iterations_checked") is None:
        return None
    return rec.get("bytes_per_launch")


def accuracy(gpu, uo, xo, clean, peak):
    """Errors of the library's outputs against the FP64 oracle's on the same
    image: max and RMS of x_hat and u_hat, the largest per-pixel relative
    error |gpu - oracle| / max(|oracle|, 1), and the PSNR of x_hat against the
    clean image (10 log10(peak^2 / MSE), count domain) minus the oracle's."""
    def psnr(xh):
        return 10.0 * np.log10(peak ** 2 / np.mean((xh - clean) ** 2))

    p0 = psnr(xo)
    out = {"oracle_psnr_db": round(float(p0), 4)}
    for prec, (xg, ug) in gpu.items():
        ex, eu = np.abs(xg - xo), np.abs(ug - uo)
        rel = max(float(np.max(ex / np.maximum(np.abs(xo), 1.0))),
                  float(np.max(eu / np.maximum(np.abs(uo), 1.0))))
        out[prec] = {"max_abs_err_x": float("%.3e" % ex.max()),
                     "rms_err_x": float("%.3e" % np.sqrt(np.mean(ex ** 2))),
                     "max_abs_err_u": float("%.3e" % eu.max()),
                     "rms_err_u": float("%.3e" % np.sqrt(np.mean(eu ** 2))),
                     "max_rel_err": float("%.3e" % rel),
                     "dpsnr_db": round(float(psnr(xg) - p0), 5)}
    return out


def cpu_baseline(args, k, a, job, tau, gamma, gpu=None):
    """The FP64 oracle timed on the host cores.  gpu: the library's (x_hat,
    u_hat) of the same job per precision; when the oracle runs the job's
    own iteration count, their errors against its result are reported."""
    import oracle
    threads = oracle.set_threads(len(os.sched_getaffinity(0)))
    clean, y = job.arrays()
    its = args.cpu_iters
    t0 = time.perf_counter()
    uo, xo = oracle.denoise(y, k, a, job.lam, tau, gamma, its, job.data_term)
    dt = time.perf_counter() - t0
    acc = None
    if gpu and its == job.iterations:
        acc = accuracy(gpu, uo, xo, clean, job.peak)
    px_it = job.height * job.width * its
    # the same image and iterations on one host thread
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.denoise(y, k, a, job.lam, tau, gamma, its, job.data_term)
    dt1 = time.perf_counter() - t1
    # the oracle-size case (64 x 64, peak 4, 24 filters of 5 x 5, 100 iterations)
    from synth.workloads import oracle_config, prior_for, step_size_for
    small = oracle_config()["jobs"][0]
    ks, as_ = prior_for(5, 24)
    ts, gs = step_size_for(5, 24)
    _, ys = small.arrays()
    small_rates = {}
    for n_thr in (1, threads):
        oracle.set_threads(n_thr)
        t2 = time.perf_counter()
        oracle.denoise(ys, ks, as_, small.lam, ts, gs, small.iterations, small.data_term)
        small_rates["cores_%d" % n_thr] = ys.size * small.iterations / (time.perf_counter() - t2) / 1e6
    oracle.set_threads(threads)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": px_it / dt / 1e6, "unit": "Mpixel-iter/s", "cores": threads,
            "kind": "oracle", "seconds": dt,
            "sample": "one %dx%d image (peak %g), %d iterations, %d %dx%d filters, FP64"
                      % (job.height, job.width, job.peak, its, k.shape[0], k.shape[1],
                         k.shape[2]),
            "cpu_model": model,
            "single_core": {"value": px_it / dt1 / 1e6, "unit": "Mpixel-iter/s",
                            "cores": 1, "seconds": dt1,
                            "images_per_s": 1.0 / dt1,
                            "sample": "the same image and iterations on one thread"},
            "images_per_s": 1.0 / dt,
            "oracle_size_case": dict(small_rates, unit="Mpixel-iter/s",
                                     sample="64x64, peak 4, 24 5x5 filters, 100 iterations"),
            "accuracy": acc}


def cpu_all_images(args, k, a, jobs, tau, gamma):
    """The oracle on every image of the FP32 baseline, on one thread and on
    all of them: Mpixel-iter/s per (image peak, threads)."""
    import oracle
    full = len(os.sched_getaffinity(0))
    out = {}
    for j in jobs:
        _, y = j.arrays()
        for n_thr in (1, full):
            oracle.set_threads(n_thr)
            t0 = time.perf_counter()
            oracle.denoise(y, k, a, j.lam, tau, gamma, args.cpu_iters, j.data_term)
            dt = time.perf_counter() - t0
            out["peak%g_cores%d" % (j.peak, n_thr)] = round(y.size * args.cpu_iters / dt / 1e6, 3)
            print(json.dumps({"cpu_oracle": {"peak": j.peak, "cores": n_thr, "seconds": dt}}),
                  file=sys.stderr, flush=True)
    oracle.set_threads(full)
    out["unit"] = "Mpixel-iter/s"
    out["iterations"] = args.cpu_iters
    return out


def batch_report(fe, torch, prior, args, tau, gamma, log=None):
    """Uneven batch: 256 images with sides log-uniform on [128, 1024],
    peaks {1, 2, 4, 8}, 200 iterations each, all in one launch per
    iteration.  Forms timed on the same inputs: one eager fe_denoise call
    (cost-model tile height), the same after fe_autotune, the tuned advance
    replayed as a captured HIP graph (fe_begin + replay + fe_end), and one
    fe_denoise call per image.  The graph form is the headline."""
    from synth.workloads import batch_config, job_counts
    cfg = batch_config(n_images=args.batch_images, iterations=args.iterations)
    jobs = cfg["jobs"]
    t0 = time.perf_counter()
    ys = job_counts(jobs)
    gen_s = time.perf_counter() - t0
    counts = [torch.from_numpy(y).cuda() for y in ys]
    del ys
    m, nf = cfg["m"], cfg["n_filters"]
    px = sum(j.height * j.width for j in jobs)
    px_it = sum(j.height * j.width * j.iterations for j in jobs)
    its = args.iterations
    stream = torch.cuda.current_stream()
    res = {"workload": "%d images, sides log-uniform on [128, 1024], aspect [0.5, 2], "
                       "peaks {1,2,4,8}, %d 7x7 filters, %d iterations"
                       % (len(jobs), nf, its),
           "pixels": px, "pixel_iterations": px_it, "input_generation_s": round(gen_s, 1)}

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def rate(ms):
        return {"ms": round(ms, 3), "Mpixel_iter_per_s": round(px_it / (ms * 1e-3) / 1e6, 1),
                "images_per_s": round(len(jobs) / (ms * 1e-3), 2)}

    for prec in args.batch_precisions.split(","):
        specs = [fe.JobSpec(c, j.lam, j.iterations, tau, gamma, data_term=j.data_term,
                            peak=j.peak, precision=prec) for c, j in zip(counts, jobs)]
        arr, keep = fe.make_jobs(specs)
        n = len(specs)
        ws = fe.alloc_workspace(fe.workspace_size(prior, arr, n), "cuda")
        lib = fe.library()

        def eager():
            fe._check(lib.fe_denoise(prior.handle, arr, n, fe._ptr(ws), ws.numel(),
                                     fe._stream_handle(stream)))

        out = {}
        eager()
        out["eager_cost_model"] = rate(timed(eager, 1))
        b = fe.Batch(prior, specs, stream=stream)
        t0 = time.perf_counter()
        b.autotune(4)
        torch.cuda.synchronize()
        out["autotune_s"] = round(time.perf_counter() - t0, 2)
        out["eager_tuned"] = rate(timed(eager, 1))
        b.begin()
        b.capture([its] * n)

        def graph_job():
            b.begin()
            b.replay()
            b.end()

        graph_job()
        out["graph_tuned"] = rate(timed(graph_job, max(1, args.batch_reps)))
        b.release_graph()
        if prec == "fp32" and not args.no_single:
            singles = []
            for sp in specs:
                a1, k1 = fe.make_jobs([sp])
                w1 = fe.alloc_workspace(fe.workspace_size(prior, a1, 1), "cuda")
                singles.append((a1, k1, w1))

            def one_at_a_time():
                for a1, _, w1 in singles:
                    fe._check(lib.fe_denoise(prior.handle, a1, 1, fe._ptr(w1), w1.numel(),
                                             fe._stream_handle(stream)))

            out["one_image_per_call"] = rate(timed(one_at_a_time, 1))
            del singles
        ach = flops_per_px_it(m, nf) * px_it / (out["graph_tuned"]["ms"] * 1e-3) / 1e12
        peak = FP32_PEAK_TFLOPS if prec == "fp32" else MFMA16_PEAK_TFLOPS
        out["achieved_TFLOPs"] = round(ach, 3)
        out["frac_of_peak"] = round(ach / peak, 4)
        res[prec] = out
        if log:
            log(json.dumps({"batch_" + prec: out}))
        del b, keep, ws
    return res


def energy_report(fe, torch, prior, cfg, counts, stream, reps=10):
    """fe_energy_grad_batch (the energy and its gradient, off the
    per-iteration path) over the four images of the workload in one call, at
    u = v (the Anscombe-domain start): gradient only (asynchronous, HIP events
    around `reps` calls) and energy + gradient (the energies return to the
    host, so each call synchronises; wall clock).  Algorithmic work per
    pixel: both filter banks, 2 * 2 * N_f * m^2 flops; HBM: read u and y,
    write the gradient, 12 bytes."""
    import ctypes
    lib = fe.library()
    m, nf = cfg["m"], cfg["n_filters"]
    H, W = counts[0].shape
    n = len(counts)
    px = H * W * n
    us = [2.0 * torch.sqrt(c + 0.375) for c in counts]
    grads = [torch.empty_like(u) for u in us]
    arr = (fe._GradJob * n)()
    for i, (c, u, g, j) in enumerate(zip(counts, us, grads, cfg["jobs"])):
        arr[i] = fe._GradJob(H, W, c.data_ptr(), u.data_ptr(), g.data_ptr(), float(j.lam),
                             int(j.data_term))
    sz = ctypes.c_size_t()
    st = lib.fe_energy_grad_batch_workspace_size(prior.handle, arr, n, ctypes.byref(sz))
    if st != 0:
        raise fe.FeError(st, lib.fe_last_error().decode())
    ws = fe.alloc_workspace(sz.value, "cuda")
    flop_px = flops_per_px_it(m, nf)
    bytes_px = 12
    out = {"workload": "%d images of %dx%d in one call, %d %dx%d filters, u = v"
                       % (n, H, W, nf, m, m),
           "flop_per_px": flop_px, "hbm_bytes_per_px": bytes_px}
    en = (ctypes.c_double * n)()
    for prec in ("fp32", "bf16", "fp16"):
        pr = fe._PREC[prec]

        def call(want_energy):
            r = lib.fe_energy_grad_batch(prior.handle, arr, n, pr,
                                         en if want_energy else None, fe._ptr(ws), ws.numel(),
                                         fe._stream_handle(stream))
            if r != 0:
                raise fe.FeError(r, lib.fe_last_error().decode())

        call(True)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            call(False)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_grad = ev0.elapsed_time(ev1) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            call(True)
        ms_both = (time.perf_counter() - t0) * 1e3 / reps
        peak = FP32_PEAK_TFLOPS if prec == "fp32" else MFMA16_PEAK_TFLOPS
        ach = flop_px * px / (ms_grad * 1e-3) / 1e12
        out[prec] = {"grad_ms_per_call": round(ms_grad, 4),
                     "energy_grad_ms_per_call": round(ms_both, 4),
                     "grad_Mpixel_per_s": round(px / (ms_grad * 1e-3) / 1e6, 1),
                     "achieved_TFLOPs": round(ach, 3),
                     "frac_of_matrix_peak": round(ach / peak, 4),
                     "matrix_peak_TFLOPs": peak,
                     "hbm_algorithmic_GBs": round(bytes_px * px / (ms_grad * 1e-3) / 1e9, 1)}
    del ws, us, grads
    return out


def binned_report(fe, torch, prior, cfg, counts, stream, tau, gamma, reps=3):
    """fe_denoise_binned (3 x 3 binning, the denoiser on the binned counts with
    the data term of 9x the peak, bilinear upsampling) on the four images of
    the workload, one call over all four, HIP events around each call."""
    import ctypes
    from synth.workloads import lambda_for_peak
    lib = fe.library()
    specs = [fe.JobSpec(c, lambda_for_peak(9 * j.peak), j.iterations, tau, gamma,
                        data_term="auto", peak=j.peak)
             for c, j in zip(counts, cfg["jobs"])]
    arr, keep = fe.make_jobs(specs)
    n = len(specs)
    sz = ctypes.c_size_t()
    st = lib.fe_binned_workspace_size(prior.handle, arr, n, ctypes.byref(sz))
    if st != 0:
        raise fe.FeError(st, lib.fe_last_error().decode())
    ws = fe.alloc_workspace(sz.value, "cuda")

    def call():
        r = lib.fe_denoise_binned(prior.handle, arr, n, fe._ptr(ws), ws.numel(),
                                  fe._stream_handle(stream))
        if r != 0:
            raise fe.FeError(r, lib.fe_last_error().decode())

    call()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        call()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    H, W = counts[0].shape
    hb, wb = (H + 2) // 3, (W + 2) // 3
    its = cfg["jobs"][0].iterations
    del ws, keep
    return {"workload": "%d images of %dx%d binned to %dx%d, %d iterations, one call" % (
                n, H, W, hb, wb, its),
            "ms_per_call": round(ms, 4), "images_per_s": round(n / (ms * 1e-3), 1),
            "binned_Mpixel_iter_per_s": round(n * hb * wb * its / (ms * 1e-3) / 1e6, 1),
            "full_res_Mpixel_per_s": round(n * H * W / (ms * 1e-3) / 1e6, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--iterations", type=int, default=200)
    ap.add_argument("--cpu-iters", type=int, default=200)
    ap.add_argument("--cpu-all-images", action="store_true",
                    help="also time the oracle on all four 512x512 images, on one and on "
                         "all host threads (minutes of CPU work; off by default)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the uneven-batch section (256 images under a HIP graph)")
    ap.add_argument("--batch-images", type=int, default=256)
    ap.add_argument("--batch-reps", type=int, default=2)
    ap.add_argument("--batch-precisions", default="fp32,bf16")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the one-image-per-call form of the batch section")
    ap.add_argument("--serving-requests", type=int, default=1000,
                    help="requests per serving run (the full 10,000-request workload "
                         "is python -m paper_1609_05722_amd.serving)")
    ap.add_argument("--serving-loads", default="0.5,0.75,0.9",
                    help="offered loads, fractions of each form's own saturation rate")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the bf16 / fp16 contraction timings")
    ap.add_argument("--no-energy", action="store_true",
                    help="skip the energy / gradient timing (fe_energy_grad)")
    ap.add_argument("--no-binned", action="store_true",
                    help="skip the binning-variant timing (fe_denoise_binned)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (a "
                         "known-size reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the denoiser's images are independent "
              "and the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1609_05722_amd as fe
    from synth.workloads import fp32_config, prior_for, step_size_for

    cfg = fp32_config(size=args.size, iterations=args.iterations)
    m, nf = cfg["m"], cfg["n_filters"]
    k, a = prior_for(m, nf)
    tau, gamma = step_size_for(m, nf)
    prior = fe.Prior(k, a, device=0)
    counts = [torch.from_numpy(j.arrays()[1]).cuda() for j in cfg["jobs"]]
    stream = torch.cuda.current_stream()
    lib = fe.library()
    its = max(j.iterations for j in cfg["jobs"])
    px_it = sum(j.height * j.width * j.iterations for j in cfg["jobs"])
    px_per_launch = sum(j.height * j.width for j in cfg["jobs"])

    def measure(precision, steps, warmup):
        specs = [fe.JobSpec(c, j.lam, j.iterations, tau, gamma, data_term=j.data_term,
                            peak=j.peak, precision=precision)
                 for c, j in zip(counts, cfg["jobs"])]
        arr, keep = fe.make_jobs(specs)
        n = len(specs)
        ws = fe.alloc_workspace(fe.workspace_size(prior, arr, n), "cuda")

        def step():
            st = lib.fe_denoise(prior.handle, arr, n, fe._ptr(ws), ws.numel(),
                                fe._stream_handle(stream))
            if st != 0:
                raise fe.FeError(st, lib.fe_last_error().decode())

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_per_step = ev0.elapsed_time(ev1) / steps
        # The dominant kernel: the fused step launches of one fe_advance call
        # (same jobs, same plan), timed with HIP events on the same stream.
        batch = fe.Batch(prior, specs, stream=stream)
        kern_ms = []
        for _ in range(max(1, steps)):
            batch.begin()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            batch.advance([j.iterations for j in cfg["jobs"]])
            e1.record(stream)
            torch.cuda.synchronize()
            kern_ms.append(e0.elapsed_time(e1) / its)
        return ms_per_step, float(np.mean(kern_ms)), wall, n

    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ms_per_step, launch_ms, wall, n = measure("fp32", args.steps, args.warmup)
    value = px_it / (ms_per_step * 1e-3) / 1e6
    achieved = flops_per_px_it(m, nf) * px_per_launch / (launch_ms * 1e-3) / 1e12
    traffic = recorded_traffic(args)
    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpixel-iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fp32 baseline: %dx%d synthetic image at peaks 1,2,4,8 "
                               "(4 jobs), %d 7x7 filters, %d iterations"
                               % (args.size, args.size, nf, args.iterations),
                   "images_per_step": n, "iterations": args.iterations,
                   "filters": "%dx%dx%d" % (nf, m, m)},
        "images_per_s": round(n / (ms_per_step * 1e-3), 2),
        "wall_s": round(wall, 3),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3),
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": traffic,
                     "kernel": "fused_step_kernel<7,MathF32<7,3,true>,0> (12 waves; one launch = one "
                               "iteration of all %d jobs)" % n,
                     "launch_us": round(launch_ms * 1e3, 2),
                     "flop_per_launch": flops_per_px_it(m, nf) * px_per_launch},
        "hbm_algorithmic_GBs": round(hbm_bytes_per_px_it() * px_per_launch
                                     / (launch_ms * 1e-3) / 1e9, 1),
    }
    def section(name, fn):
        """An optional part of the line; a Python error in it is reported in
        the line instead of losing the whole measurement."""
        try:
            result[name] = fn()
        except Exception as exc:  # noqa: BLE001 - reported, not hidden
            import traceback
            traceback.print_exc()
            result[name] = {"error": "%s: %s" % (type(exc).__name__, exc)}

    def mixed_section():
        mixed = {}
        for prec in ("bf16", "fp16"):
            ms_p, launch_p, _, _ = measure(prec, args.steps, 1)
            ach = flops_per_px_it(m, nf) * px_per_launch / (launch_p * 1e-3) / 1e12
            mixed[prec] = {"value": round(px_it / (ms_p * 1e-3) / 1e6, 2),
                           "unit": "Mpixel-iter/s", "ms_per_step": round(ms_p, 4),
                           "images_per_s": round(n / (ms_p * 1e-3), 2),
                           "launch_us": round(launch_p * 1e3, 2),
                           "achieved_TFLOPs": round(ach, 3),
                           "frac_of_mfma_peak": round(ach / MFMA16_PEAK_TFLOPS, 4)}
            # matrix and FP32 vector work one after the other (they overlap only
            # in part on gfx950): the bound of the reduced-precision step
            t_mfma = flops_per_px_it(m, nf) / (MFMA16_PEAK_TFLOPS * 1e12)
            t_valu = valu_slots_per_px_it(nf) / VALU_LANE_SLOTS_PER_S
            peak = 1.0 / (t_mfma + t_valu) / 1e9
            got = px_per_launch / (launch_p * 1e-3) / 1e9
            mixed[prec]["roofline_mfma_valu"] = {
                "bound": "mfma+alu", "unit": "Gpixel-iter/s", "achieved": round(got, 2),
                "peak": round(peak, 2), "frac": round(got / peak, 4),
                "valu_slots_per_px_it": valu_slots_per_px_it(nf),
                "mfma_flop_per_px_it": flops_per_px_it(m, nf)}
        return mixed

    def serving_section():
        from paper_1609_05722_amd.serving import serving_report
        loads = tuple(float(x) for x in args.serving_loads.split(","))
        return serving_report(prior, args.serving_requests, loads, "bf16",
                              same_rate_loads=(0.9,),
                              log=lambda t: print(t, file=sys.stderr, flush=True))

    def cpu_section():
        job4 = [j for j in cfg["jobs"] if j.peak == 4.0][0]
        # the library's outputs for the same image, one per precision
        gpu = {}
        c4 = counts[cfg["jobs"].index(job4)]
        for prec in ("fp32",) + (() if args.no_mixed else ("bf16", "fp16")):
            x4, u4 = fe.denoise(c4, prior, job4.lam, job4.iterations, tau, gamma,
                                data_term=job4.data_term, peak=job4.peak, precision=prec,
                                want_anscombe=True)
            torch.cuda.synchronize()
            gpu[prec] = (x4.cpu().numpy().astype(np.float64),
                         u4.cpu().numpy().astype(np.float64))
        out = cpu_baseline(args, k, a, job4, tau, gamma, gpu)
        if args.cpu_all_images:
            out["all_images"] = cpu_all_images(args, k, a, cfg["jobs"], tau, gamma)
        return out

    if not args.no_mixed:
        section("mixed_precision", mixed_section)
    if not args.no_energy:
        section("energy_grad", lambda: energy_report(fe, torch, prior, cfg, counts, stream))
    if not args.no_binned:
        section("binned", lambda: binned_report(fe, torch, prior, cfg, counts, stream,
                                                tau, gamma))
    if not args.no_batch:
        section("batch", lambda: batch_report(fe, torch, prior, args, tau, gamma,
                                              log=lambda t: print(t, file=sys.stderr,
                                                                  flush=True)))
    if not args.no_serving:
        section("serving", serving_section)
    if not args.no_cpu:
        section("cpu_baseline", cpu_section)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
