"""Python binding of libfe.so, the gfx950 FoE Poisson denoiser.

Argument marshalling only: every step of the scheme runs in the library's
HIP kernels.  PyTorch supplies device memory and the HIP stream.  If the
library has not been built, importing the binding's entry points raises
instead of falling back to anything else.

Entry points mirror include/fe.h:
  Prior(filters, weights, device=0)      fe_create / fe_destroy
  denoise(counts, prior, ...)            fe_denoise (one or many jobs)
  energy_grad(counts, u, prior, ...)     fe_energy_grad
  energy_grad_batch(items, prior, ...)   fe_energy_grad_batch
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfe.so")

FE_OK, FE_ERR_INVALID, FE_ERR_UNSUPPORTED, FE_ERR_NOMEM, FE_ERR_DEVICE = range(5)
DATA_AUTO, DATA_QUADRATIC, DATA_IDIV = 0, 1, 2
PREC_FP32, PREC_BF16, PREC_FP16 = 0, 1, 2
_PREC = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp16": PREC_FP16}
_DATA = {"auto": DATA_AUTO, "quadratic": DATA_QUADRATIC, "idiv": DATA_IDIV}

EXPORTS = ("fe_create", "fe_destroy", "fe_workspace_size", "fe_denoise",
           "fe_state_bytes", "fe_begin", "fe_advance_workspace_size", "fe_advance",
           "fe_end", "fe_binned_workspace_size", "fe_denoise_binned",
           "fe_energy_grad_workspace_size", "fe_energy_grad",
           "fe_energy_grad_batch_workspace_size", "fe_energy_grad_batch",
           "fe_server_create", "fe_server_submit", "fe_server_poll", "fe_server_load",
           "fe_server_destroy", "fe_server_last_error", "fe_autotune", "fe_tuning_save",
           "fe_tuning_load", "fe_advance_graph_create", "fe_graph_launch",
           "fe_graph_destroy", "fe_advance_noalloc", "fe_last_error")


class FeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("fe status %d: %s" % (status, msg))
        self.status = status


class _Prior(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n_filters", ctypes.c_int32),
                ("filters", ctypes.POINTER(ctypes.c_float)),
                ("weights", ctypes.POINTER(ctypes.c_float))]


class _Job(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("counts", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("out_anscombe", ctypes.c_void_p), ("lambda_", ctypes.c_float),
                ("iterations", ctypes.c_int32), ("data_term", ctypes.c_int32),
                ("peak", ctypes.c_float), ("tau", ctypes.c_float),
                ("gamma", ctypes.c_float), ("precision", ctypes.c_int32)]


class _GradJob(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("counts", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("grad", ctypes.c_void_p), ("lambda_", ctypes.c_float),
                ("data_term", ctypes.c_int32)]


_lib = None


def library():
    """Load libfe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfe.so is not built: run "
                              "python -m paper_1609_05722_amd.build or "
                              "__graft_entry__.build()")
        # PyTorch bundles its own HIP runtime under the same soname; loading
        # it first makes libfe.so bind to that one copy (a second runtime
        # loaded ahead of it leaves PyTorch without devices).
        _torch()
        lib = ctypes.CDLL(LIB_PATH)
        i32, vp, sz = ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
        lib.fe_create.argtypes = [ctypes.POINTER(_Prior), ctypes.c_int, ctypes.POINTER(vp)]
        lib.fe_create.restype = i32
        lib.fe_destroy.argtypes = [vp]
        lib.fe_destroy.restype = None
        lib.fe_workspace_size.argtypes = [vp, ctypes.POINTER(_Job), i32, ctypes.POINTER(sz)]
        lib.fe_workspace_size.restype = i32
        lib.fe_denoise.argtypes = [vp, ctypes.POINTER(_Job), i32, vp, sz, vp]
        lib.fe_denoise.restype = i32
        lib.fe_energy_grad_workspace_size.argtypes = [vp, i32, i32, ctypes.POINTER(sz)]
        lib.fe_energy_grad_workspace_size.restype = i32
        lib.fe_energy_grad.argtypes = [vp, i32, i32, vp, vp, ctypes.c_float, i32, i32,
                                       ctypes.POINTER(ctypes.c_double), vp, vp, sz, vp]
        lib.fe_energy_grad.restype = i32
        lib.fe_energy_grad_batch_workspace_size.argtypes = [vp, ctypes.POINTER(_GradJob), i32,
                                                            ctypes.POINTER(sz)]
        lib.fe_energy_grad_batch_workspace_size.restype = i32
        lib.fe_energy_grad_batch.argtypes = [vp, ctypes.POINTER(_GradJob), i32, i32,
                                             ctypes.POINTER(ctypes.c_double), vp, sz, vp]
        lib.fe_energy_grad_batch.restype = i32
        pp = ctypes.POINTER(ctypes.c_void_p)
        pi = ctypes.POINTER(ctypes.c_int32)
        lib.fe_state_bytes.argtypes = [vp, i32, i32, ctypes.POINTER(sz)]
        lib.fe_state_bytes.restype = i32
        lib.fe_begin.argtypes = [vp, ctypes.POINTER(_Job), pp, i32, vp]
        lib.fe_begin.restype = i32
        lib.fe_advance_workspace_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
        lib.fe_advance_workspace_size.restype = i32
        lib.fe_advance.argtypes = [vp, ctypes.POINTER(_Job), pp, pi, pi, i32, vp, sz, vp]
        lib.fe_advance.restype = i32
        lib.fe_advance_noalloc.argtypes = [vp, ctypes.POINTER(_Job), pp, pi, pi, i32, vp]
        lib.fe_advance_noalloc.restype = i32
        lib.fe_end.argtypes = [vp, ctypes.POINTER(_Job), pp, pi, i32, vp]
        lib.fe_end.restype = i32
        lib.fe_binned_workspace_size.argtypes = [vp, ctypes.POINTER(_Job), i32,
                                                 ctypes.POINTER(sz)]
        lib.fe_binned_workspace_size.restype = i32
        lib.fe_denoise_binned.argtypes = [vp, ctypes.POINTER(_Job), i32, vp, sz, vp]
        lib.fe_denoise_binned.restype = i32
        lib.fe_autotune.argtypes = [vp, ctypes.POINTER(_Job), i32, i32, vp]
        lib.fe_autotune.restype = i32
        lib.fe_tuning_save.argtypes = [vp, ctypes.c_char_p]
        lib.fe_tuning_save.restype = i32
        lib.fe_tuning_load.argtypes = [vp, ctypes.c_char_p]
        lib.fe_tuning_load.restype = i32
        lib.fe_advance_graph_create.argtypes = [vp, ctypes.POINTER(_Job), pp, pi, pi, i32, vp,
                                                sz, ctypes.POINTER(vp)]
        lib.fe_advance_graph_create.restype = i32
        lib.fe_graph_launch.argtypes = [vp, vp]
        lib.fe_graph_launch.restype = i32
        lib.fe_graph_destroy.argtypes = [vp]
        lib.fe_graph_destroy.restype = None
        lib.fe_last_error.argtypes = []
        lib.fe_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def _check(status):
    if status != FE_OK:
        raise FeError(status, library().fe_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Prior:
    """Filter bank and weights of eq. 2.5 uploaded to a device (fe_create)."""

    def __init__(self, filters, weights, device=0):
        f = np.ascontiguousarray(filters, dtype=np.float32)
        w = np.ascontiguousarray(weights, dtype=np.float32)
        if f.ndim != 3 or f.shape[1] != f.shape[2] or w.shape != (f.shape[0],):
            raise ValueError("filters must be [N_f, m, m] and weights [N_f]")
        self.m, self.n_filters = int(f.shape[1]), int(f.shape[0])
        self.device = int(device)
        pr = _Prior(self.m, self.n_filters,
                    f.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                    w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        h = ctypes.c_void_p()
        _check(library().fe_create(ctypes.byref(pr), self.device, ctypes.byref(h)))
        self._h = h
        self._lib = library()

    @property
    def handle(self):
        return self._h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.fe_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: modules already torn down
            pass


@dataclass
class JobSpec:
    """One image: device counts plus the scheme's parameters (eq. 3.7)."""
    counts: object            # torch float32 CUDA tensor, H x W
    lam: float
    iterations: int
    tau: float
    gamma: float
    data_term: str = "auto"
    peak: float = 0.0
    precision: str = "fp32"
    out: object = None        # optional preallocated outputs
    out_anscombe: object = None
    want_anscombe: bool = False


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _device_f32(t, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.dim() == 2 and t.is_contiguous()):
        raise ValueError(name + " must be a contiguous 2-D float32 CUDA tensor")
    return t


def make_jobs(specs):
    """Build the fe_job array (and output tensors) for a list of JobSpec."""
    torch = _torch()
    arr = (_Job * max(1, len(specs)))()
    keep = []
    for i, s in enumerate(specs):
        c = _device_f32(s.counts, "counts")
        H, W = c.shape
        out = s.out if s.out is not None else torch.empty_like(c)
        oa = s.out_anscombe
        if oa is None and s.want_anscombe:
            oa = torch.empty_like(c)
        for t, name in ((out, "out"), (oa, "out_anscombe")):
            if t is not None and (_device_f32(t, name).shape != c.shape
                                  or t.device != c.device):
                raise ValueError(name + " must match counts in shape and device")
        keep.append((c, out, oa))
        dt = _DATA[s.data_term] if isinstance(s.data_term, str) else int(s.data_term)
        pr = _PREC[s.precision] if isinstance(s.precision, str) else int(s.precision)
        arr[i] = _Job(H, W, c.data_ptr(), out.data_ptr(),
                      oa.data_ptr() if oa is not None else None,
                      float(s.lam), int(s.iterations), dt, float(s.peak),
                      float(s.tau), float(s.gamma), pr)
    return arr, keep


def workspace_size(prior, jobs_arr, n):
    sz = ctypes.c_size_t()
    _check(library().fe_workspace_size(prior.handle, jobs_arr, int(n), ctypes.byref(sz)))
    return int(sz.value)


def alloc_workspace(nbytes, device):
    torch = _torch()
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(256, int(nbytes)), dtype=torch.uint8, device=device)


def denoise_jobs(prior, specs, workspace=None, stream=None):
    """fe_denoise over several jobs in one call.  Returns a list of
    (x_hat, u_hat or None) tensors; asynchronous on the stream."""
    arr, keep = make_jobs(specs)
    n = len(specs)
    need = workspace_size(prior, arr, n)
    if workspace is None or workspace.numel() < need:
        workspace = alloc_workspace(need, specs[0].counts.device if n else "cuda")
    _check(library().fe_denoise(prior.handle, arr, n, _ptr(workspace),
                                workspace.numel(), _stream_handle(stream)))
    if stream is not None:
        # tensors freed here may be reused only after this stream's work
        workspace.record_stream(stream)
        for c, o, oa in keep:
            for t in (c, o, oa):
                if t is not None:
                    t.record_stream(stream)
    return [(o, oa) for (_, o, oa) in keep]


def denoise_binned_jobs(prior, specs, stream=None):
    """fe_denoise_binned over several jobs (the binning variant).  Returns a
    list of (x_hat H x W, binned u_hat or None); asynchronous."""
    arr, keep = make_jobs(specs)
    n = len(specs)
    sz = ctypes.c_size_t()
    _check(library().fe_binned_workspace_size(prior.handle, arr, n, ctypes.byref(sz)))
    ws = alloc_workspace(sz.value, specs[0].counts.device if n else "cuda")
    _check(library().fe_denoise_binned(prior.handle, arr, n, _ptr(ws), ws.numel(),
                                       _stream_handle(stream)))
    if stream is not None:
        ws.record_stream(stream)
    out = []
    for (c, o, oa) in keep:
        ub = None
        if oa is not None:
            Hb, Wb = (c.shape[0] + 2) // 3, (c.shape[1] + 2) // 3
            ub = oa.view(-1)[:Hb * Wb].view(Hb, Wb)
        out.append((o, ub))
    return out


def denoise(counts, prior, lam, iterations, tau, gamma, data_term="auto",
            peak=0.0, precision="fp32", want_anscombe=False, stream=None):
    """Denoise one image (eq. 3.7).  Returns x_hat, or (x_hat, u_hat)."""
    (x, u), = denoise_jobs(prior, [JobSpec(counts, lam, iterations, tau, gamma,
                                           data_term, peak, precision,
                                           want_anscombe=want_anscombe)],
                           stream=stream)
    return (x, u) if want_anscombe else x


def energy_grad(counts, u, prior, lam, data_term, want_energy=True,
                want_grad=True, stream=None, precision="fp32"):
    """E(u) and grad E(u) for counts y (v = f_A(y)) and an Anscombe-domain
    image u.  Returns (energy float or None, grad tensor or None)."""
    torch = _torch()
    c = _device_f32(counts, "counts")
    uu = _device_f32(u, "u")
    H, W = c.shape
    dt = _DATA[data_term] if isinstance(data_term, str) else int(data_term)
    sz = ctypes.c_size_t()
    _check(library().fe_energy_grad_workspace_size(prior.handle, H, W, ctypes.byref(sz)))
    ws = alloc_workspace(sz.value, c.device)
    grad = torch.empty_like(uu) if want_grad else None
    e = ctypes.c_double()
    pr = _PREC[precision] if isinstance(precision, str) else int(precision)
    _check(library().fe_energy_grad(prior.handle, H, W, _ptr(c), _ptr(uu), float(lam),
                                    dt, pr, ctypes.byref(e) if want_energy else None,
                                    _ptr(grad), _ptr(ws), ws.numel(),
                                    _stream_handle(stream)))
    return (e.value if want_energy else None), grad


def energy_grad_batch(items, prior, want_energy=True, want_grad=True, stream=None,
                      precision="fp32"):
    """fe_energy_grad_batch: items = [(counts, u, lam, data_term), ...] (CUDA
    tensors).  Returns (list of energies or None, list of gradients or
    None); one launch over every image."""
    torch = _torch()
    n = len(items)
    arr = (_GradJob * max(1, n))()
    grads = []
    for i, (c, u, lam, dt) in enumerate(items):
        c = _device_f32(c, "counts")
        u = _device_f32(u, "u")
        H, W = c.shape
        g = torch.empty_like(u) if want_grad else None
        grads.append(g)
        d = _DATA[dt] if isinstance(dt, str) else int(dt)
        arr[i] = _GradJob(H, W, c.data_ptr(), u.data_ptr(),
                          g.data_ptr() if g is not None else None, float(lam), d)
    sz = ctypes.c_size_t()
    _check(library().fe_energy_grad_batch_workspace_size(prior.handle, arr, n,
                                                         ctypes.byref(sz)))
    ws = alloc_workspace(sz.value, items[0][0].device if n else "cuda")
    en = (ctypes.c_double * max(1, n))()
    pr = _PREC[precision] if isinstance(precision, str) else int(precision)
    _check(library().fe_energy_grad_batch(prior.handle, arr, n, pr,
                                          en if want_energy else None, _ptr(ws), ws.numel(),
                                          _stream_handle(stream)))
    return ([en[i] for i in range(n)] if want_energy else None), \
        (grads if want_grad else None)


class Batch:
    """Jobs kept resident on the device between calls (fe_begin /
    fe_advance / fe_end): each job owns a state tensor of two H x W planes
    and a count of the iterations already applied."""

    def __init__(self, prior, specs, stream=None):
        torch = _torch()
        self.prior = prior
        self.specs = list(specs)
        self.n = len(self.specs)
        self.arr, self.keep = make_jobs(self.specs)
        self.states = [torch.empty((2,) + tuple(s.counts.shape), dtype=torch.float32,
                                   device=s.counts.device) for s in self.specs]
        self._sp = (ctypes.c_void_p * max(1, self.n))(*[t.data_ptr() for t in self.states])
        self.done = (ctypes.c_int32 * max(1, self.n))()
        sz = ctypes.c_size_t()
        _check(library().fe_advance_workspace_size(prior.handle, self.n, ctypes.byref(sz)))
        self.ws = alloc_workspace(sz.value, self.specs[0].counts.device if self.n else "cuda")
        self.stream = stream

    def begin(self):
        _check(library().fe_begin(self.prior.handle, self.arr, self._sp, self.n,
                                  _stream_handle(self.stream)))
        for i in range(self.n):
            self.done[i] = 0

    def advance(self, counts):
        """Apply counts[i] more iterations to job i (one call, shared launches)."""
        cnt = (ctypes.c_int32 * max(1, self.n))(*[int(c) for c in counts])
        _check(library().fe_advance(self.prior.handle, self.arr, self._sp, self.done, cnt,
                                    self.n, _ptr(self.ws), self.ws.numel(),
                                    _stream_handle(self.stream)))
        for i in range(self.n):
            self.done[i] += cnt[i]

    def advance_noalloc(self, counts):
        """advance() through fe_advance_noalloc: the job table goes to the
        library's static device array instead of this batch's workspace."""
        cnt = (ctypes.c_int32 * max(1, self.n))(*[int(c) for c in counts])
        _check(library().fe_advance_noalloc(self.prior.handle, self.arr, self._sp, self.done,
                                            cnt, self.n, _stream_handle(self.stream)))
        for i in range(self.n):
            self.done[i] += cnt[i]

    def capture(self, counts):
        """A HIP graph of one advance by counts (even) from the current
        iteration counts; each replay() applies them again."""
        self.release_graph()
        cnt = (ctypes.c_int32 * max(1, self.n))(*[int(c) for c in counts])
        h = ctypes.c_void_p()
        _check(library().fe_advance_graph_create(self.prior.handle, self.arr, self._sp,
                                                 self.done, cnt, self.n, _ptr(self.ws),
                                                 self.ws.numel(), ctypes.byref(h)))
        self._graph, self._graph_counts = h, list(counts)
        return h

    def replay(self):
        _check(library().fe_graph_launch(self._graph, _stream_handle(self.stream)))
        for i in range(self.n):
            self.done[i] += self._graph_counts[i]

    def release_graph(self):
        if getattr(self, "_graph", None) is not None:
            library().fe_graph_destroy(self._graph)
            self._graph = None

    def __del__(self):
        try:
            self.release_graph()
        except Exception:   # interpreter shutdown: modules already torn down
            pass

    def autotune(self, trial_iterations=4):
        _check(library().fe_autotune(self.prior.handle, self.arr, self.n,
                                     int(trial_iterations), _stream_handle(self.stream)))

    def end(self):
        _check(library().fe_end(self.prior.handle, self.arr, self._sp, self.done, self.n,
                                _stream_handle(self.stream)))
        return [(o, oa) for (_, o, oa) in self.keep]
