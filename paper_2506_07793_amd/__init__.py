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
                 stream=None, gmw_beta=17.5, gmw_gamma=3.0):
        lib = _lib.load()
        self._lib = lib
        self.freqs = np.ascontiguousarray(np.asarray(freqs, dtype=np.float64).ravel())
        opts, self._edges = _make_opts(lib, wavelet, pad, explicit_len, out, precision, bands,
                                       gmw_beta, gmw_gamma)
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
                      out="complex64", bands=None, stream=None):
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
        self.L = int(desc.L)
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
        tw = np.empty(2 * self.L, dtype=np.float32)
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
        if x_batch_stride is None:
            x_batch_stride = int(C) * self.n
        if out_batch_stride is None:
            out_batch_stride = self.output_bytes(C)
        _lib.check(self._lib.cwt_execute_batches(
            self._ptr, _dptr(x), int(x_batch_stride), int(n_batches), int(C), _dptr(out),
            int(out_batch_stride), _dptr(ws), ws.numel() * ws.element_size(),
            _stream_handle(stream)))
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

    def output_bytes(self, C):
        elem = 8 if self.out_mode == "complex64" else 4
        return int(C) * self.out_rows * self.n * elem

    def alloc_output(self, C, device="cuda"):
        import torch
        dt = torch.complex64 if self.out_mode == "complex64" else torch.float32
        return torch.empty(self.output_shape(C), dtype=dt, device=device)

    def alloc_workspace(self, C, device="cuda"):
        import torch
        nbytes = max(256, self.workspace_size(C))
        return torch.empty(nbytes, dtype=torch.uint8, device=device)

    def execute(self, x, out=None, ws=None, stream=None):
        """x: cuda float32 [C, n] (or [n]).  Returns the output tensor."""
        import torch
        if x.dim() == 1:
            x = x[None, :]
        if x.dtype != torch.float32 or not x.is_cuda:
            raise TypeError("x must be a cuda float32 tensor")
        if x.shape[-1] != self.n:
            raise ValueError("x has %d samples, plan expects %d" % (x.shape[-1], self.n))
        x = x.contiguous()
        C = int(x.shape[0])
        if out is None:
            out = self.alloc_output(C, device=x.device)
        if tuple(out.shape) != self.output_shape(C) or not out.is_contiguous():
            raise ValueError("out must be contiguous with shape %s" % (self.output_shape(C),))
        if ws is None:
            ws = self.alloc_workspace(C, device=x.device)
        _lib.check(self._lib.cwt_execute(self._ptr, _dptr(x), C, _dptr(out), _dptr(ws),
                                         ws.numel() * ws.element_size(), _stream_handle(stream)))
        return out

    def forward_spectra(self, x, ws, stream=None):
        """Stage 1 of execute: channel half spectra into ws (cwt_forward_spectra)."""
        C = int(x.shape[0])
        _lib.check(self._lib.cwt_forward_spectra(self._ptr, _dptr(x), C, _dptr(ws),
                                                 ws.numel() * ws.element_size(),
                                                 _stream_handle(stream)))

    def transform_spectra(self, C, out, ws, stream=None):
        """Stage 2 of execute: spectra in ws -> out (cwt_transform_spectra)."""
        _lib.check(self._lib.cwt_transform_spectra(self._ptr, int(C), _dptr(out), _dptr(ws),
                                                   ws.numel() * ws.element_size(),
                                                   _stream_handle(stream)))

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
        for i, (plan, x, out) in enumerate(self.items):
            if x.dtype.is_floating_point is False or not x.is_contiguous():
                raise TypeError("x must be a contiguous float32 tensor")
            if x.shape[-1] != plan.n:
                raise ValueError("item %d: x has %d samples, plan expects %d" % (
                    i, x.shape[-1], plan.n))
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
        _lib.check(self._lib.cwt_execute_batch(self._arr, len(self.items), _dptr(ws),
                                               ws.numel() * ws.element_size(),
                                               _stream_handle(stream)))


def cwt(x, sfreq, freqs, n_cycles, **kw):
    """One-shot transform of a cuda float32 [C, n] tensor."""
    plan = Plan(x.shape[-1], sfreq, freqs, n_cycles=n_cycles, **kw)
    try:
        return plan.execute(x)
    finally:
        import torch
        torch.cuda.current_stream().synchronize()
        plan.close()
