"""Autotuner: candidates are timed on the device, the fastest is kept, results
stay within the parity gate, and the cache file is applied to new plans."""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_07793_amd as cwt
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


@pytest.mark.parametrize("N,sfreq", [(2000, 1000.0), (4096, 1000.0), (10080, 2048.0)])
def test_autotune_keeps_parity_and_caches(N, sfreq, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("CWT_AUTOTUNE_CACHE", str(cache))
    freqs = synth.log_freqs(1.0, 100.0, 24)
    cyc = synth.eeg_cycles(freqs)
    x = synth.eeg(3, N, sfreq, seed=N)
    plan = cwt.Plan(N, sfreq, freqs, n_cycles=cyc, out="power")
    r = plan.autotune(8)
    print("L=%d: %d candidates, kernel %d, threads %d, radix %s, best %.4f ms (default %.4f ms)" % (
        plan.L, r["n_candidates"], r["kernel"], r["threads"], r["radix"], r["best_ms"],
        r["default_ms"]))
    assert r["n_candidates"] >= 2
    assert r["best_ms"] <= r["default_ms"]
    P = plan.execute(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = oracle.power(oracle.cwt(x.astype(np.float64), sfreq, freqs, cyc))
    e = float(np.max(np.abs(P - ref)) / ref.max())
    print("tuned e_P %.3e" % e)
    assert e <= 1e-5
    line = cache.read_text().strip().splitlines()[-1].split()
    assert line[0].startswith("gfx950") and int(line[1]) == plan.L
    # a new plan with the same key picks the cached choice
    plan2 = cwt.Plan(N, sfreq, freqs, n_cycles=cyc, out="power")
    assert plan2.desc.kernel == r["kernel"]
    if r["kernel"] == 0:
        assert plan2.radices == r["radix"] and plan2.desc.threads == r["threads"]
    plan.close()
    plan2.close()
