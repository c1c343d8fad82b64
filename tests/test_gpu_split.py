"""Split-precision DFT-as-GEMM (MFMA) path: error against the FP64 oracle,
reported for every output kind, and compared with the FP32 path.

The bound asserted here is the reporting bar of this variant, not the FP32
gate: FP16 hi+lo splitting carries about 22 significant bits, BF16 hi+lo
about 16, so e_P <= 1e-5 (FP16) and <= 1e-4 (BF16)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_07793_amd as cwt
from paper_2506_07793_amd import _lib
import synth

pytestmark = pytest.mark.gpu
BOUND = {"split_f16": 1e-5, "split_bf16": 1e-4}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


@pytest.fixture(scope="module")
def data():
    d = synth.eeg_64ch(C=2)
    x = d["x"]
    ref = oracle.cwt(x.astype(np.float64), d["sfreq"], d["freqs"], d["n_cycles"])
    return d, ref


@pytest.mark.parametrize("prec", ["split_f16", "split_bf16"])
def test_split_complex_and_power(prec, data):
    d, ref = data
    xt = torch.from_numpy(d["x"]).cuda()
    res = {}
    for out in ("complex64", "power", "bandpower"):
        plan = cwt.Plan(4096, d["sfreq"], d["freqs"], n_cycles=d["n_cycles"], out=out,
                        precision=prec)
        got = plan.execute(xt).cpu().numpy()
        torch.cuda.synchronize()
        if out == "complex64":
            e_P, e_W = oracle.parity_errors(got, ref)
            res[out] = (e_P, e_W)
        else:
            P = oracle.power(ref)
            if out == "bandpower":
                P = oracle.band_power(P, oracle.band_groups(d["freqs"]))
            e_P = float(np.max(np.abs(got - P)) / P.max())
            res[out] = (e_P, None)
        plan.close()
    print("%s: complex e_P=%.3e e_W=%.3e | power e_P=%.3e | bandpower e=%.3e" % (
        prec, res["complex64"][0], res["complex64"][1], res["power"][0], res["bandpower"][0]))
    for out, (e_P, _) in res.items():
        assert e_P <= BOUND[prec], (out, e_P)


def test_split_full_size_sampled_rows():
    d = synth.eeg_64ch(C=64)
    xt = torch.from_numpy(d["x"]).cuda()
    rng = np.random.default_rng(12)
    rows = np.stack([rng.integers(0, 64, 16), rng.integers(0, 100, 16)], axis=1)
    ref = oracle.cwt(d["x"].astype(np.float64), d["sfreq"], d["freqs"], d["n_cycles"], rows=rows)
    for prec in ("split_f16", "split_bf16"):
        plan = cwt.Plan(4096, d["sfreq"], d["freqs"], n_cycles=d["n_cycles"], precision=prec)
        W = plan.execute(xt).cpu().numpy()
        e_P, e_W = oracle.parity_errors(W[rows[:, 0], rows[:, 1]], ref)
        print("%s 64ch sampled: e_P=%.3e e_W=%.3e" % (prec, e_P, e_W))
        assert e_P <= BOUND[prec]
        plan.close()


def test_split_needs_length_4096():
    with pytest.raises(cwt.CwtError) as ei:
        cwt.Plan(1000, 1000.0, [10.0, 20.0], n_cycles=5.0, precision="split_f16")
    assert ei.value.code == _lib.CWT_E_UNSUPPORTED


@pytest.mark.parametrize("prec", ["split_f16", "split_bf16"])
def test_split_band_first_stage(prec):
    """Rows whose band has at most L/16 = 256 bins compute the first stage
    directly (one input per butterfly) and run the MFMA stages from the
    second; wider rows run all three.  Grid as in the register-resident band
    test: bands of 1 to 256 bins, wrapping past bin 0, ending at the last
    positive bin, and whole-spectrum rows; every row against the oracle."""
    sfreq, L = 1000.0, 4096
    N = L - 37
    freqs = np.concatenate([synth.log_freqs(0.3, 480.0, 20), [499.0, 495.0]])
    cyc = np.concatenate([np.where(np.arange(20) % 2 == 0, 3.0, 12.0), [3.0, 240.0]])
    rng = np.random.default_rng(17)
    x = rng.normal(0, 20, size=(2, N)).astype(np.float32)
    plan = cwt.Plan(N, sfreq, freqs, n_cycles=cyc, pad="pow2", precision=prec)
    _, band, _ = plan.tables()
    K = band[:, 1]
    assert (K <= 256).any() and (K > 256).any() and (band[K <= 256, 0] < 0).any()
    got = plan.execute(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc, L=L)
    e_P, e_W = oracle.parity_errors(got, ref)
    print("%s band first stage: e_P=%.3e e_W=%.3e" % (prec, e_P, e_W))
    assert e_P <= BOUND[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["split_f16", "split_bf16"])
@pytest.mark.parametrize("C,N", [(3, 4096), (2, 3000)], ids=["odd-C", "zero-padded"])
def test_split_forward_spectra(prec, C, N):
    """The forward transform on MFMA: the half spectra of every channel (two
    real channels per complex transform, the last pair with one channel when
    C is odd; zero padding from N to 4096) against the FP64 FFT of the
    padded signal, and against the FP32 path's."""
    d = synth.eeg_64ch(C=C, N=N)
    x = d["x"]
    xt = torch.from_numpy(x).cuda()
    kw = dict(n_cycles=d["n_cycles"], pad="pow2")
    plan = cwt.Plan(N, d["sfreq"], d["freqs"], precision=prec, **kw)
    ref_plan = cwt.Plan(N, d["sfreq"], d["freqs"], **kw)
    assert plan.L == 4096
    Lh = plan.L // 2 + 1
    ws = plan.alloc_workspace(C)
    ws_ref = ref_plan.alloc_workspace(C)
    plan.forward_spectra(xt, ws)
    ref_plan.forward_spectra(xt, ws_ref)
    torch.cuda.synchronize()
    got = ws[: C * Lh * 8].view(torch.complex64).reshape(C, Lh).cpu().numpy()
    f32 = ws_ref[: C * Lh * 8].view(torch.complex64).reshape(C, Lh).cpu().numpy()
    exact = np.fft.rfft(x.astype(np.float64), n=plan.L, axis=1)
    scale = np.abs(exact).max(axis=1, keepdims=True)
    e = float(np.max(np.abs(got - exact) / scale))
    e32 = float(np.max(np.abs(f32 - exact) / scale))
    print("%s forward C=%d N=%d: max |err| / peak = %.3e (FP32 path %.3e)" % (prec, C, N, e, e32))
    assert e <= BOUND[prec] / 10
    plan.close()
    ref_plan.close()
