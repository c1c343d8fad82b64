"""Batched form on the GPU: heterogeneous recordings in one graph launch (one
launch pair per recording by default, or persistent class kernels), checked
against the FP64 oracle and against cwt_execute."""
import numpy as np
import pytest
import torch

import oracle
import paper_2506_07793_amd as cwt
import synth

pytestmark = pytest.mark.gpu
TOL_P = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def _items(specs, seed):
    out = []
    for k, (N, C, F, sfreq, mode) in enumerate(specs):
        freqs = synth.log_freqs(0.5, min(200.0, 0.45 * sfreq), F)
        cyc = synth.eeg_cycles(freqs)
        plan = cwt.Plan(N, sfreq, freqs, n_cycles=cyc, out=mode)
        x = synth.eeg(C, N, sfreq, seed + k)
        out.append(dict(plan=plan, x=x, xt=torch.from_numpy(x).cuda(), out=plan.alloc_output(C),
                        freqs=freqs, cyc=cyc, sfreq=sfreq, mode=mode))
    return out


def _check_item(it, got, rows, label):
    x64 = it["x"].astype(np.float64)
    if it["mode"] == "bandpower":
        ref = oracle.band_power(oracle.power(oracle.cwt(x64, it["sfreq"], it["freqs"], it["cyc"])),
                                oracle.band_groups(it["freqs"]))
        e = max(float(np.max(np.abs(got[:, b] - ref[:, b])) / ref[:, b].max())
                for b in range(ref.shape[1]))
    else:
        W = oracle.cwt(x64, it["sfreq"], it["freqs"], it["cyc"], rows=rows)
        g = np.stack([got[c, f] for c, f in rows])
        if it["mode"] == "power":
            P = oracle.power(W)
            e = float(np.max(np.abs(g - P)) / P.max())
        else:
            e = oracle.parity_errors(g, W)[0]
    print("%s: e=%.3e" % (label, e), flush=True)
    assert e <= TOL_P, label


SPECS = [(1000, 3, 20, 250.0, "complex64"), (4116, 2, 33, 1000.0, "power"),
         (777, 5, 40, 500.0, "complex64"), (2048, 1, 25, 2048.0, "bandpower"),
         (12000, 2, 21, 1000.0, "power"), (105, 4, 24, 250.0, "complex64"),
         (19999, 1, 20, 2048.0, "complex64"),
         # plans of the 32-value class (at most 768 threads): L = 19440 and 20412
         (19440, 3, 16, 1000.0, "power"), (20400, 2, 12, 2048.0, "complex64")]


@pytest.mark.parametrize("kernels", ["items", "persistent"])
@pytest.mark.parametrize("graph", ["1", "0"])
def test_heterogeneous_batch_matches_oracle(graph, kernels, monkeypatch):
    monkeypatch.setenv("CWT_BATCH_GRAPH", graph)
    monkeypatch.setenv("CWT_BATCH_KERNELS", kernels)
    its = _items(SPECS, seed=30)
    # the 32-value items run at most 768 threads per workgroup, also as a
    # persistent class
    assert sum(1 for it in its if it["plan"].desc.threads == 768 and it["plan"].L > 16384) == 2
    b = cwt.Batch([(it["plan"], it["xt"], it["out"]) for it in its])
    ws = b.alloc_workspace()
    b.execute(ws)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for k, it in enumerate(its):
        C = it["x"].shape[0]
        F = len(it["freqs"])
        rows = [(int(rng.integers(0, C)), int(rng.integers(0, F))) for _ in range(3)] + [(0, 0)]
        _check_item(it, it["out"].cpu().numpy(), rows, "item %d N=%d L=%d mode=%s" % (
            k, it["x"].shape[1], it["plan"].L, it["mode"]))
        # same numbers as the single-recording path's generic kernel (to rounding)
        ref = it["plan"].execute(it["xt"]).cpu().numpy()
        got = it["out"].cpu().numpy()
        scale = np.abs(ref).max()
        assert np.max(np.abs(got - ref)) <= 2e-6 * scale
    for it in its:
        it["plan"].close()


def test_graph_replays_with_new_inputs():
    """The captured graph is replayed for new inputs of the same shapes; eager
    work and synchronisations happen between replays, and each replay is
    checked against cwt_execute."""
    its = _items(SPECS[:4], seed=50)
    b = cwt.Batch([(it["plan"], it["xt"], it["out"]) for it in its])
    ws = b.alloc_workspace()
    for rep in range(3):
        for k, it in enumerate(its):
            it["xt"].copy_(torch.from_numpy(synth.eeg(it["x"].shape[0], it["x"].shape[1],
                                                       it["sfreq"], 1000 * rep + k)))
        torch.cuda.synchronize()
        b.execute(ws)
        torch.cuda.synchronize()
        for it in its:
            ref = it["plan"].execute(it["xt"]).cpu().numpy()
            got = it["out"].cpu().numpy()
            assert np.max(np.abs(got - ref)) <= 2e-6 * np.abs(ref).max(), rep
        _ = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work
    for it in its:
        it["plan"].close()


def test_seeded_recording_draw_subset():
    """First recordings of the seeded heterogeneous draw (lengths 500-20000, 1-128
    channels, 20-150 frequencies, four sampling rates), power output."""
    recs = synth.batch_recordings()[:12]
    its = []
    for k, r in enumerate(recs):
        C = min(r["C"], 8)  # keep the oracle's sampled rows cheap
        plan = cwt.Plan(r["N"], r["sfreq"], r["freqs"], n_cycles=r["n_cycles"], out="power")
        x = synth.eeg(C, r["N"], r["sfreq"], r["seed"])
        its.append(dict(plan=plan, x=x, xt=torch.from_numpy(x).cuda(), out=plan.alloc_output(C),
                        freqs=r["freqs"], cyc=r["n_cycles"], sfreq=r["sfreq"], mode="power"))
    b = cwt.Batch([(it["plan"], it["xt"], it["out"]) for it in its])
    ws = b.alloc_workspace()
    b.execute(ws)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    for k, it in enumerate(its):
        C, F = it["x"].shape[0], len(it["freqs"])
        rows = [(int(rng.integers(0, C)), int(rng.integers(0, F))) for _ in range(2)]
        _check_item(it, it["out"].cpu().numpy(), rows, "rec %d N=%d L=%d" % (
            k, it["x"].shape[1], it["plan"].L))
    for it in its:
        it["plan"].close()


def test_full_recording_draw_one_graph():
    """The benchmarked batch at its full size: all 256 recordings of the seeded
    draw (lengths 500-20000, their full 1-128 channels, power out) in one graph
    launch of the default form.  Every output is finite and non-negative; one
    row of the first recording of each padded length, and of every recording
    whose padded length exceeds 16 384 (a channel of structured synthetic EEG,
    the other channels EEG-scale white noise), is checked against the
    oracle."""
    recs = synth.batch_recordings()
    assert len(recs) == 256
    rng = np.random.default_rng(9)
    its, checks, seen_L = [], [], set()
    for k, r in enumerate(recs):
        C, N = r["C"], r["N"]
        x = rng.standard_normal((C, N), dtype=np.float32) * np.float32(synth.EEG_RMS_UV)
        plan = cwt.Plan(N, r["sfreq"], r["freqs"], n_cycles=r["n_cycles"], out="power")
        it = dict(plan=plan, xt=torch.from_numpy(x).cuda(), out=plan.alloc_output(C),
                  freqs=r["freqs"], cyc=r["n_cycles"], sfreq=r["sfreq"], mode="power")
        if plan.L not in seen_L or plan.L > 16384:
            seen_L.add(plan.L)
            c, f = int(rng.integers(0, C)), int(rng.integers(0, len(r["freqs"])))
            x_c = synth.eeg(1, N, r["sfreq"], r["seed"])
            it["xt"][c] = torch.from_numpy(x_c[0]).cuda()
            checks.append((k, c, f, x_c))
        its.append(it)
    b = cwt.Batch([(it["plan"], it["xt"], it["out"]) for it in its])
    ws = b.alloc_workspace()
    b.execute(ws)
    torch.cuda.synchronize()
    total = 0
    for it in its:
        o = it["out"]
        assert bool(torch.isfinite(o).all()) and float(o.min()) >= 0.0
        total += o.numel()
    n_long = sum(1 for k, _, _, _ in checks if its[k]["plan"].L > 16384)
    assert total > 1.4e10 and len(checks) > 100 and n_long > 40
    # oracle rows in parallel threads (each call releases the GIL)
    from concurrent.futures import ThreadPoolExecutor

    def ref_row(chk):
        k, c, f, x_c = chk
        it = its[k]
        return oracle.power(oracle.cwt(x_c.astype(np.float64), it["sfreq"], it["freqs"],
                                       it["cyc"], rows=[(0, f)]))[0]

    with ThreadPoolExecutor(max_workers=8) as pool:
        refs = list(pool.map(ref_row, checks))
    for (k, c, f, x_c), P in zip(checks, refs):
        it = its[k]
        got = it["out"][c, f].cpu().numpy().astype(np.float64)
        e = float(np.max(np.abs(got - P)) / P.max())
        print("rec %d N=%d L=%d ch %d f %d: e=%.3e" % (k, x_c.shape[1], it["plan"].L, c, f, e),
              flush=True)
        assert e <= TOL_P, k
    for it in its:
        it["plan"].close()
