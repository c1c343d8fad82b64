"""MI355X-native FFT-based Morlet continuous wavelet transform (gfx950 HIP).

Python binding of libcwt (include/cwt.h).  torch supplies device memory and
streams; every step of the transform runs in libcwt's HIP kernels.

    import torch, paper_2506_07793_amd as cwt
    plan = cwt.Plan(n=4096, sfreq=1000.0, freqs=freqs, n_cycles=cyc)
    W = plan.execute(x)          # x: cuda float32 [C, n] -> complex64 [C, F, n]
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import CwtError  # noqa: F401

__all__ = ["Plan", "Batch", "CwtError", "cwt", "describe", "DEFAULT_BANDS"]

DEFAULT_BANDS = ((1.0, 4.0), (4.0, 8.0), (8.0, 13.0), (13.0, 30.0), (30.0, 100.0))


def _stream_handle(stream):
    import torch
    if stream is None:
        if not torch.cuda.is_available():
            return ctypes.c_void_p(0)
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _nbytes(t):
    return t.numel() * t.element_size()


def _check_dev(name, t, device=None, dtype=None, min_bytes=None, contiguous=True):
    """A tensor handed to the library as a device pointer: on a GPU, on
    `device` (when given), of `dtype` (when given), contiguous, and at least
    `min_bytes` long.  Raises before anything is launched."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise TypeError("%s must be a cuda tensor (got device %s)" % (name, t.device))
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if contiguous and not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if min_bytes is not None and _nbytes(t) < min_bytes:
        raise ValueError("%s holds %d bytes, the call writes or reads %d" % (
            name, _nbytes(t), min_bytes))
    return t


def _on_other_stream(stream):
    """True when `stream` is given and is not torch's current stream."""
    import torch
    return stream is not None and stream != torch.cuda.current_stream()


class TorchDeviceMemory:
    """Device-memory callbacks (cwt_alloc_fn / cwt_free_fn) served by torch's
    caching allocator, so that the library's own buffers (plan tables, a
    plan's workspace, stream rings) come from torch like the caller's tensors.

    alloc(bytes, stream) returns the storage of a uint8 tensor allocated on
    `stream` (torch's allocator then orders its reuse on that stream); free
    releases it, first marking it as used by the freeing stream when that is
    another one, so torch does not hand the memory out again before the work
    already enqueued there has finished (stream-ordered free).  Counts every
    byte that goes out and comes back."""

    def __init__(self, device=None):
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        self._blocks = {}
        self.bytes_out = 0
        self.bytes_back = 0
        self.alloc_fn = _lib.ALLOC_FN(self._alloc)
        self.free_fn = _lib.FREE_FN(self._free)

    def _torch_stream(self, handle):
        import torch
        if not handle:
            return torch.cuda.default_stream(self.device)
        return torch.cuda.ExternalStream(handle, device=self.device)

    def _alloc(self, nbytes, stream, ctx):
        import torch
        try:
            with torch.cuda.stream(self._torch_stream(stream)):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:  # the library reports CWT_E_NOMEM
            return None
        ptr = t.data_ptr()
        self._blocks[ptr] = (t, int(stream or 0), int(nbytes))
        self.bytes_out += int(nbytes)
        return ptr

    def _free(self, ptr, nbytes, stream, ctx):
        t, s_alloc, n = self._blocks.pop(int(ptr))
        if int(stream or 0) != s_alloc:
            t.record_stream(self._torch_stream(stream))
        self.bytes_back += n
        del t

    @property
    def outstanding(self):
        """Bytes handed out and not yet given back."""
        return self.bytes_out - self.bytes_back

    def fill(self, opts):
        opts.alloc = self.alloc_fn
        opts.free = self.free_fn
        opts.alloc_ctx = None


def _make_opts(lib, wavelet, pad, explicit_len, out, precision, bands, gmw_beta=17.5,
               gmw_gamma=3.0):
    opts = _lib.PlanOpts()
    lib.cwt_plan_opts_init(ctypes.byref(opts))
    opts.wavelet = _lib.WAVELET[wavelet]
    opts.gmw_beta = float(gmw_beta)
    opts.gmw_gamma = float(gmw_gamma)
    opts.pad = _lib.PAD[pad]
    opts.explicit_len = int(explicit_len)
    opts.out = _lib.OUT[out]
    opts.precision = _lib.PRECISION[precision]
    edges = None
    if bands is not None:
        edges = np.ascontiguousarray(np.asarray(bands, dtype=np.float64).ravel())
        opts.n_bands = len(edges) // 2
        opts.band_edges = edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return opts, edges


def _cycles(freqs, n_cycles, omega0, wavelet="morlet"):
    if wavelet == "gmw" and n_cycles is None and omega0 is None:
        return None, None, 0.0  # not used by the GMW
    if n_cycles is not None:
        cyc = np.asarray(n_cycles, dtype=np.float64)
        if cyc.ndim == 0:
            cyc = np.full(freqs.shape, float(cyc))
        cyc = np.ascontiguousarray(cyc.ravel())
        return cyc, cyc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.0
    if omega0 is None:
        raise ValueError("give n_cycles or omega0")
    return None, None, float(omega0)


def describe(n, sfreq, freqs, n_cycles=None, omega0=None, wavelet="morlet", pad="smooth7",
             explicit_len=0, out="complex64", precision="fp32", bands=None, gmw_beta=17.5,
             gmw_gamma=3.0):
    """Validate a plan request and describe it without a GPU (cwt_plan_describe)."""
    lib = _lib.load()
    freqs = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64).ravel())
    opts, edges = _make_opts(lib, wavelet, pad, explicit_len, out, precision, bands, gmw_beta,
                             gmw_gamma)
    cyc, cyc_ptr, om = _cycles(freqs, n_cycles, omega0, wavelet)
    desc = _lib.PlanDesc()
    _lib.check(lib.cwt_plan_describe(ctypes.byref(desc), int(n), float(sfreq),
                                     freqs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     len(freqs), cyc_ptr, om, ctypes.byref(opts)))
    return desc


class Plan:
    """A CWT plan: padded length, radix schedule and device-resident tables.

    n_cycles: one sigma per frequency (the paper's Morlet sigma), or None to
    use omega0 for every frequency.  wavelet: "morlet", "gabor" or "gmw" (the
    generalized Morse wavelet, gmw_beta / gmw_gamma; n_cycles not used).
    out: "complex64", "power" or "bandpower".
    """

    def __init__(self, n, sfreq, freqs, n_cycles=None, omega0=None, wavelet="morlet",
                 pad="smooth7", explicit_len=0, out="complex64", precision="fp32", bands=None,
                 stream=None, gmw_beta=17.5, gmw_gamma=3.0, max_channels=0, memory="torch"):
        """memory: "torch" (the plan's device memory from torch's caching
        allocator, the default), a TorchDeviceMemory, or None (HIP's
        stream-ordered pool).  max_channels > 0 gives the plan its own
        workspace for that many channels (execute without ws uses it)."""
        lib = _lib.load()
        self._lib = lib
        self.freqs = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64).ravel())
        opts, self._edges = _make_opts(lib, wavelet, pad, explicit_len, out, precision, bands,
                                       gmw_beta, gmw_gamma)
        opts.max_channels = int(max_channels)
        self.memory = TorchDeviceMemory() if memory == "torch" else memory
        if self.memory is not None:
            self.memory.fill(opts)
        self._cyc, cyc_ptr, om = _cycles(self.freqs, n_cycles, omega0, wavelet)
        handle = ctypes.c_void_p()
        self._ptr = None
        _lib.check(lib.cwt_plan_create(
            ctypes.byref(handle), int(n), float(sfreq),
            self.freqs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(self.freqs),
            cyc_ptr, om, ctypes.byref(opts), _stream_handle(stream)))
        self._finish(handle, out, sfreq)

    @classmethod
    def from_wavelets(cls, n, sfreq, freqs, wavelets, pad="smooth7", explicit_len=0,
                      out="complex64", bands=None, stream=None, max_channels=0,
                      memory="torch"):
        """Plan from sampled time-domain wavelets (cwt_plan_create_from_wavelets):
        wavelets [n_freqs, w_len] complex, sample j at time (j - w_len // 2) / sfreq,
        used as given; freqs label the rows (band grouping)."""
        self = cls.__new__(cls)
        lib = _lib.load()
        self._lib = lib
        self.freqs = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64).ravel())
        wv = np.ascontiguousarray(np.atleast_2d(np.asarray(wavelets, dtype=np.complex64)))
        if wv.shape[0] != len(self.freqs):
            raise ValueError("one wavelet per frequency")
        opts, self._edges = _make_opts(lib, "morlet", pad, explicit_len, out, "fp32", bands)
        opts.max_channels = int(max_channels)
        self.memory = TorchDeviceMemory() if memory == "torch" else memory
        if self.memory is not None:
            self.memory.fill(opts)
        self._cyc = None
        handle = ctypes.c_void_p()
        self._ptr = None
        _lib.check(lib.cwt_plan_create_from_wavelets(
            ctypes.byref(handle), int(n), float(sfreq),
            self.freqs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(self.freqs),
            wv.view(np.float32).ctypes.data_as(ctypes.POINTER(ctypes.c_float)), wv.shape[1],
            ctypes.byref(opts), _stream_handle(stream)))
        self._finish(handle, out, sfreq)
        return self

    def _finish(self, handle, out, sfreq):
        lib = self._lib
        self._ptr = handle
        desc = _lib.PlanDesc()
        _lib.check(lib.cwt_plan_info(self._ptr, ctypes.byref(desc)))
        self.desc = desc
        self.n = int(desc.n)
        self.L = int(desc.L)  # the padded length the transform is defined with
        self.n_segments = int(desc.n_segments)
        self.n_freqs = int(desc.n_freqs)
        self.n_bands = int(desc.n_bands)
        self.out_rows = int(desc.out_rows)
        self.out_mode = out
        self.sfreq = float(sfreq)

    # -- info ------------------------------------------------------------
    @property
    def radices(self):
        return [int(self.desc.radix[i]) for i in range(self.desc.n_passes)]

    def band_of_freq(self):
        out = np.empty(self.n_freqs, dtype=np.int32)
        _lib.check(self._lib.cwt_plan_band_of_freq(
            self._ptr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def workspace_size(self, C):
        return int(self._lib.cwt_workspace_size(self._ptr, int(C)))

    def tables(self, stream=None):
        """(H bins [spectrum_bins] f32 (complex64 for plans from sampled wavelets),
        band [F,3] int32, twiddles [L] complex64) on the host."""
        cplx = bool(self.desc.spectrum_complex)
        H = np.empty(max(1, int(self.desc.spectrum_bins)) * (2 if cplx else 1), dtype=np.float32)
        band = np.empty((self.n_freqs, 3), dtype=np.int32)
        tw = np.empty(2 * int(self.desc.segment_len), dtype=np.float32)
        _lib.check(self._lib.cwt_plan_copy_tables(
            self._ptr, H.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            band.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            tw.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream_handle(stream)))
        if cplx:
            return H.view(np.complex64)[: int(self.desc.spectrum_bins)], band, tw.view(np.complex64)
        return H[: int(self.desc.spectrum_bins)], band, tw.view(np.complex64)

    def batches_workspace_size(self, C):
        return int(self._lib.cwt_batches_workspace_size(self._ptr, int(C)))

    def alloc_batches_workspace(self, C, device="cuda"):
        """Double-buffered workspace for execute_batches."""
        import torch
        nbytes = max(256, self.batches_workspace_size(C))
        return torch.empty(nbytes, dtype=torch.uint8, device=device)

    def execute_batches(self, x, n_batches, out, ws, C, x_batch_stride=None,
                        out_batch_stride=None, stream=None):
        """n_batches batches of C channels (cwt_execute_batches): batch i
        reads x at i * x_batch_stride floats and writes out at
        i * out_batch_stride bytes (defaults: consecutive batches)."""
        import torch
        if x_batch_stride is None:
            x_batch_stride = int(C) * self.n
        if out_batch_stride is None:
            out_batch_stride = self.output_bytes(C)
        nb = max(int(n_batches), 1)
        _check_dev("x", x, dtype=torch.float32,
                   min_bytes=4 * (int(C) * self.n + (nb - 1) * int(x_batch_stride)))
        _check_dev("ws", ws, device=x.device, min_bytes=self.batches_workspace_size(C))
        _check_dev("out", out, device=x.device,
                   min_bytes=self.output_bytes(C) + (nb - 1) * int(out_batch_stride))
        _lib.check(self._lib.cwt_execute_batches(
            self._ptr, _dptr(x), int(x_batch_stride), int(n_batches), int(C), _dptr(out),
            int(out_batch_stride), _dptr(ws), _nbytes(ws), _stream_handle(stream)))
        return out

    def timing_start(self, max_launches):
        """Bind dispatch-timed event pairs to the next max_launches transform
        launches of this plan (cwt_plan_timing_start)."""
        _lib.check(self._lib.cwt_plan_timing_start(self._ptr, int(max_launches)))
        self._timing_cap = int(max_launches)

    def timing_stop(self):
        """Wait for the timed launches; their kernel durations in ms, in launch
        order (cwt_plan_timing_stop)."""
        cap = max(getattr(self, "_timing_cap", 0), 0)
        ms = np.zeros(max(cap, 1), dtype=np.float32)
        n = ctypes.c_int32(0)
        _lib.check(self._lib.cwt_plan_timing_stop(
            self._ptr, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), cap, ctypes.byref(n)))
        self._timing_cap = 0
        return ms[: min(n.value, cap)].astype(np.float64)

    def autotune(self, C, stream=None):
        """Time the candidate kernel configurations and keep the fastest (cwt_plan_autotune)."""
        r = _lib.TuneResult()
        _lib.check(self._lib.cwt_plan_autotune(self._ptr, int(C), _stream_handle(stream),
                                               ctypes.byref(r)))
        desc = _lib.PlanDesc()
        _lib.check(self._lib.cwt_plan_info(self._ptr, ctypes.byref(desc)))
        self.desc = desc
        return {"n_candidates": r.n_candidates, "kernel": r.kernel, "variant": r.variant,
                "threads": r.threads, "radix": [r.radix[i] for i in range(r.n_passes)],
                "best_ms": r.best_ms, "default_ms": r.default_ms}

    # -- execution -------------------------------------------------------
    def output_shape(self, C):
        return (int(C), self.out_rows, self.n)

    def output_bytes(self, C):
        elem = 8 if self.out_mode == "complex64" else 4
        return int(C) * self.out_rows * self.n * elem

    @property
    def out_dtype(self):
        import torch
        return torch.complex64 if self.out_mode == "complex64" else torch.float32

    def _check_x(self, x):
        """x: cuda float32 [C, n] contiguous; returns C."""
        import torch
        _check_dev("x", x, dtype=torch.float32)
        if x.dim() != 2 or x.shape[1] != self.n:
            raise ValueError("x must have shape [C, %d] (got %s)" % (self.n, tuple(x.shape)))
        return int(x.shape[0])

    def _check_out(self, out, C, device, n_batches=1, stride=None):
        need = self.output_bytes(C) + (n_batches - 1) * (stride or 0)
        _check_dev("out", out, device=device, min_bytes=need)
        if n_batches == 1 and stride is None:
            if out.dtype != self.out_dtype:
                raise TypeError("out must be %s for output mode %r (got %s)" % (
                    self.out_dtype, self.out_mode, out.dtype))
            if tuple(out.shape) != self.output_shape(C):
                raise ValueError("out must have shape %s (got %s)" % (
                    self.output_shape(C), tuple(out.shape)))

    def _check_ws(self, ws, device, need):
        _check_dev("ws", ws, device=device, min_bytes=need)

    def alloc_output(self, C, device="cuda"):
        import torch
        dt = torch.complex64 if self.out_mode == "complex64" else torch.float32
        return torch.empty(self.output_shape(C), dtype=dt, device=device)

    def alloc_workspace(self, C, device="cuda"):
        import torch
        nbytes = max(256, self.workspace_size(C))
        return torch.empty(nbytes, dtype=torch.uint8, device=device)

    def execute(self, x, out=None, ws=None, stream=None):
        """x: cuda float32 [C, n] (or [n]).  Returns the output tensor.

        out and ws (when given) must be cuda tensors on x's device: out of the
        plan's output dtype and shape, ws of at least workspace_size(C)
        bytes.  Tensors this call allocates are marked as used by `stream`
        so that torch's allocator does not reuse them before the launch has
        finished there."""
        import torch
        if isinstance(x, torch.Tensor) and x.dim() == 1:
            x = x[None, :]
        _check_dev("x", x, dtype=torch.float32, contiguous=False)
        if x.dim() != 2 or x.shape[1] != self.n:
            raise ValueError("x has shape %s, plan expects [C, %d]" % (tuple(x.shape), self.n))
        other = _on_other_stream(stream)
        made = []
        if not x.is_contiguous():
            x = x.contiguous()
            made.append(x)
        C = int(x.shape[0])
        if out is None:
            out = self.alloc_output(C, device=x.device)
        self._check_out(out, C, x.device)
        if ws is None and 0 < C <= int(self.desc.max_channels):
            # the plan's own workspace (calls using it are ordered on one stream)
            _lib.check(self._lib.cwt_execute(self._ptr, _dptr(x), C, _dptr(out), None, 0,
                                             _stream_handle(stream)))
            if other:
                for t in made:
                    t.record_stream(stream)
            return out
        if ws is None:
            ws = self.alloc_workspace(C, device=x.device)
            made.append(ws)
        self._check_ws(ws, x.device, self.workspace_size(C))
        _lib.check(self._lib.cwt_execute(self._ptr, _dptr(x), C, _dptr(out), _dptr(ws),
                                         _nbytes(ws), _stream_handle(stream)))
        if other:
            for t in made:
                t.record_stream(stream)
        return out

    def execute_noalloc(self, x, out, stream=None):
        """execute() without a workspace and without any device allocation
        (cwt_execute_noalloc): the workspace is the library's static device
        scratch of CWT_NOALLOC_SCRATCH_BYTES per GPU, shared by every call on
        that GPU, so calls that overlap on one GPU race.  x: cuda float32
        [C, n] contiguous; out: preallocated, the plan's output dtype and
        shape."""
        C = self._check_x(x)
        self._check_out(out, C, x.device)
        _lib.check(self._lib.cwt_execute_noalloc(self._ptr, _dptr(x), C, _dptr(out),
                                                 _stream_handle(stream)))
        return out

    def forward_spectra(self, x, ws, stream=None):
        """Stage 1 of execute: channel half spectra into ws (cwt_forward_spectra)."""
        C = self._check_x(x)
        self._check_ws(ws, x.device, self.workspace_size(C))
        _lib.check(self._lib.cwt_forward_spectra(self._ptr, _dptr(x), C, _dptr(ws),
                                                 _nbytes(ws), _stream_handle(stream)))

    def transform_spectra(self, C, out, ws, stream=None):
        """Stage 2 of execute: spectra in ws -> out (cwt_transform_spectra).
        out may be any cuda buffer of at least output_bytes(C) bytes."""
        _check_dev("ws", ws, min_bytes=self.workspace_size(C))
        _check_dev("out", out, device=ws.device, min_bytes=self.output_bytes(C))
        _lib.check(self._lib.cwt_transform_spectra(self._ptr, int(C), _dptr(out), _dptr(ws),
                                                   _nbytes(ws), _stream_handle(stream)))

    def close(self, stream=None):
        if getattr(self, "_ptr", None):
            try:
                self._lib.cwt_plan_destroy(self._ptr, _stream_handle(stream))
            finally:
                self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._ptr


class Batch:
    """Many (plan, x, out) items in one graph launch of persistent kernels."""

    def __init__(self, items):
        """items: list of (plan, x [C, n] cuda float32, out tensor)."""
        self.items = list(items)
        self._arr = (_lib.BatchItem * max(1, len(self.items)))()
        import torch
        self.device = None
        for i, (plan, x, out) in enumerate(self.items):
            _check_dev("item %d x" % i, x, device=self.device, dtype=torch.float32)
            self.device = x.device
            if x.dim() != 2 or x.shape[1] != plan.n:
                raise ValueError("item %d: x has shape %s, plan expects [C, %d]" % (
                    i, tuple(x.shape), plan.n))
            _check_dev("item %d out" % i, out, device=x.device, dtype=plan.out_dtype)
            if tuple(out.shape) != plan.output_shape(x.shape[0]):
                raise ValueError("item %d: out must have shape %s" % (
                    i, plan.output_shape(x.shape[0])))
            self._arr[i] = _lib.BatchItem(plan.handle.value, x.data_ptr(), int(x.shape[0]),
                                          out.data_ptr())
        self._lib = _lib.load()

    def workspace_size(self):
        return int(self._lib.cwt_batch_workspace_size(self._arr, len(self.items)))

    def alloc_workspace(self, device="cuda"):
        import torch
        return torch.empty(max(256, self.workspace_size()), dtype=torch.uint8, device=device)

    def execute(self, ws, stream=None):
        _check_dev("ws", ws, device=self.device, min_bytes=self.workspace_size())
        _lib.check(self._lib.cwt_execute_batch(self._arr, len(self.items), _dptr(ws),
                                               _nbytes(ws), _stream_handle(stream)))


def cwt(x, sfreq, freqs, n_cycles, **kw):
    """One-shot transform of a cuda float32 [C, n] tensor."""
    plan = Plan(x.shape[-1], sfreq, freqs, n_cycles=n_cycles, **kw)
    try:
        return plan.execute(x)
    finally:
        import torch
        torch.cuda.current_stream().synchronize()
        plan.close()
