#!/usr/bin/env python3
"""Throughput benchmark of the FFT-based Morlet CWT on one MI355X.

Workload (one step = the whole hot path on one batch, inputs resident in HBM):
64 channels x 4096 samples at 1000 Hz of synthetic EEG (pink noise 20 uV rms +
10 Hz alpha bursts, seed 2), 100 log-spaced frequencies 1-100 Hz,
n_cycles = clip(f/2, 3, 10), FP32 input, complex64 output [64, 100, 4096]:
forward real FFT of every channel, then per (channel, frequency) the spectral
multiply, inverse FFT, crop and store.  Each step writes its own 210 MB output
buffer of a 64-buffer ring (13.4 GB, beyond the 256 MB last-level cache), so
that the outputs reach HBM.  By default the K timed steps run as
cwt_execute_batches: one launch per step that transforms the step's batch and
computes the next batch's forward FFT (--serial: forward + transform launches
per step; the serial step time is reported either way).  Before the warm-up
steps a pre-roll of untimed pipelined steps runs until at least --preroll-ms
of GPU time has passed and two consecutive chunk means agree within 2% (on a
fresh device the first ~25 ms of work run 15-30% slower while the clock
ramps up); it is reported as `preroll`, and `warmup` stays what was asked.

Prints one JSON line with the throughput (output samples x frequencies per
second), the roofline of the dominant kernel (the transform launch, each timed
by events bound to its own dispatch on the stream it runs on) and the FP64
CPU oracle's throughput on a bounded sample of the same workload; beside them
the split-precision variants, the 256-recording batch, the length sweep, the
streaming server's latencies, and as context the same pipeline composed from
torch.fft on the same GPU and the paper's FFT method in FP64 on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published


PROFILES = {
    ("fused", "complex64"): os.path.join(ROOT, "profiles", "k_fixed_fused_64ch_4096x100f_complex64.md"),
    ("main", "complex64"): os.path.join(ROOT, "profiles", "k_fixed_main_64ch_4096x100f_complex64.md"),
    ("fused", "bandpower"): os.path.join(ROOT, "profiles", "k_fixed_fused_64ch_4096x100f_bandpower.md"),
}


def progress(msg):
    """One line on stderr as each leg ends (stdout carries only the JSON line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def committed_traffic(plan, out, kind):
    """HBM bytes per launch of the timed kernel from its committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when
    the kernel sources no longer hash to the profiled ones or the workload
    differs from the profiled one."""
    import hashlib
    path = PROFILES.get((kind, out))
    if plan.desc.kernel != 1 or not path or not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        k, _, v = line.strip().partition(": ")
        if k in ("traffic_bytes_per_launch", "kernel_sources_sha256", "kernel_sources"):
            fields[k] = v.strip()
    if len(fields) != 3:
        return None
    h = hashlib.sha256()
    for rel in fields["kernel_sources"].split():
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    if h.hexdigest() != fields["kernel_sources_sha256"]:
        return None
    return int(fields["traffic_bytes_per_launch"])


def oracle_single_thread(cfg, Cs):
    """The oracle's rate on one host thread (OMP_NUM_THREADS=1, in a child
    process, since the thread count is fixed when the oracle loads) over Cs
    channels x all frequencies of the 64-channel workload; None if the child
    fails.  (cfg is unused: the child regenerates the seeded input.)"""
    import subprocess
    code = (
        "import sys, time, json; sys.path.insert(0, %r)\n"
        "import numpy as np, synth, oracle\n"
        "d = synth.eeg_64ch(seed=2, C=%d)\n"
        "rows = [(c, f) for c in range(%d) for f in range(len(d['freqs']))]\n"
        "t0 = time.perf_counter()\n"
        "oracle.cwt(d['x'].astype(np.float64), d['sfreq'], d['freqs'], d['n_cycles'], rows=rows)\n"
        "dt = time.perf_counter() - t0\n"
        "print(json.dumps({'value': len(rows) * d['x'].shape[1] / dt, 'seconds': dt,\n"
        "                  'threads': oracle.num_threads(), 'channels': %d}))\n"
    ) % (ROOT, Cs, Cs, Cs)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                           text=True, timeout=300)
        return json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None


def cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_name(plan, fused):
    """The transform kernel the timed steps launch (the one the roofline prices)."""
    if plan.desc.kernel == 1 and fused:
        return ("k_fixed_fused (multiply + inverse FFT + store of one batch, forward FFT of "
                "the next, register-resident, L=%d)" % plan.L)
    if plan.desc.kernel == 1:
        return "k_fixed_main (multiply + inverse FFT + store, register-resident, L=%d)" % plan.L
    return "k_main (multiply + inverse FFT + store, runtime radices, L=%d)" % plan.L


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--out", default="complex64", choices=["complex64", "power", "bandpower"],
                    help="output of the timed transform (complex64: the headline; bandpower: the "
                         "five EEG bands' mean power [C, 5, N])")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing (profiling runs)")
    ap.add_argument("--cpu-channels", type=int, default=64,
                    help="channels of the oracle's timed sample (all 100 frequencies each)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="the oracle's sample is repeated until this much time has passed "
                         "(at most 8 passes)")
    ap.add_argument("--serial", action="store_true",
                    help="time K forward + transform pairs instead of the pipelined form")
    ap.add_argument("--graph", type=int, default=0,
                    help="1: replay the step as a captured HIP graph; 0: direct launches (default)")
    ap.add_argument("--batch-steps", type=int, default=3,
                    help="timed steps of the 256-recording batch run (0 skips it)")
    ap.add_argument("--stream-deadline-us", type=int, default=500,
                    help="streaming server's batching deadline in microseconds (the longest "
                         "a completed hop waits for others to share its launch)")
    ap.add_argument("--stream-seconds", type=float, default=6.0,
                    help="real-time length of each streaming run (0 skips the streaming runs; "
                         "60 gives the 60 s serving runs of the serving workload)")
    ap.add_argument("--length-sweep", type=int, default=1,
                    help="1: run the N = 100..2500 length sweep, the long recording, the "
                         "paper's workload and the epoch lengths (0 skips them)")
    ap.add_argument("--preroll-ms", type=float, default=300.0,
                    help="untimed pipelined steps before the warm-up until at least this much "
                         "GPU time has passed and two consecutive chunk means agree within 2%% "
                         "(the device clock ramps up over the first tens of ms of work)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (scales the HBM "
                         "byte counters of a profiler run)")
    return ap.parse_args()


def bench_batch(steps, n_rec=256):
    """Heterogeneous batch: 256 seeded recordings (lengths 500-20000, 1-128
    channels, 20-150 log frequencies 0.5 Hz-min(200, 0.45 sfreq), sfreq in {250,
    500, 1000, 2048}), power output, FP32.  One launch of the captured batch
    graph per step (a forward and a transform launch per recording inside it),
    against the sum of per-recording cwt_execute calls on the same data.
    Inputs are device normal noise at EEG scale (the timings do not depend on
    the values; the parity tests use the structured EEG generator)."""
    import torch

    import paper_2506_07793_amd as cwt
    import synth

    recs = synth.batch_recordings()[:n_rec]
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    items, plans = [], []
    pts = 0
    out_bytes = 0
    in_bytes = 0
    # Autotune the first plan of each padded length (on up to 16 channels);
    # later plans of that length take the choice from the tuning cache file.
    import tempfile
    tune_file = tempfile.NamedTemporaryFile(prefix="cwt_tune_", suffix=".txt", delete=False)
    tune_file.close()
    old_cache = os.environ.get("CWT_AUTOTUNE_CACHE")
    os.environ["CWT_AUTOTUNE_CACHE"] = tune_file.name
    tuned = {}
    t_tune = 0.0
    try:
        for r in recs:
            plan = cwt.Plan(r["N"], r["sfreq"], r["freqs"], n_cycles=r["n_cycles"], out="power")
            if plan.L not in tuned:
                t0 = time.perf_counter()
                tuned[plan.L] = plan.autotune(r["C"])
                t_tune += time.perf_counter() - t0
            x = torch.randn(r["C"], r["N"], device="cuda", generator=g) * 20.0
            out = plan.alloc_output(r["C"])
            items.append((plan, x, out))
            plans.append(plan)
            pts += r["C"] * r["F"] * r["N"]
            out_bytes += out.numel() * 4
            in_bytes += x.numel() * 4 + r["C"] * (plan.L // 2 + 1) * 8 * 2
    finally:
        if old_cache is None:
            os.environ.pop("CWT_AUTOTUNE_CACHE", None)
        else:
            os.environ["CWT_AUTOTUNE_CACHE"] = old_cache
        os.unlink(tune_file.name)
    batch = cwt.Batch(items)
    ws = batch.alloc_workspace()
    wss = [p.alloc_workspace(x.shape[0]) for p, x, _ in items]
    stream = torch.cuda.current_stream()
    batch.execute(ws)
    for (p, x, o), w in zip(items, wss):
        p.execute(x, out=o, ws=w)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        batch.execute(ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1) / steps
    e0.record(stream)
    for _ in range(steps):
        for (p, x, o), w in zip(items, wss):
            p.execute(x, out=o, ws=w)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_loop = e0.elapsed_time(e1) / steps
    # The persistent form (one persistent forward and one transform kernel
    # per workgroup-size class, tasks claimed through atomic counters) on the
    # same autotuned plans, for comparison with the default form.
    old_k = os.environ.get("CWT_BATCH_KERNELS")
    os.environ["CWT_BATCH_KERNELS"] = "persistent"
    try:
        batch.execute(ws)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            batch.execute(ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_pers = e0.elapsed_time(e1) / steps
    finally:
        if old_k is None:
            os.environ.pop("CWT_BATCH_KERNELS", None)
        else:
            os.environ["CWT_BATCH_KERNELS"] = old_k
    res = {"workload": "%d seeded heterogeneous recordings, power out" % len(recs),
           "autotune_s": t_tune, "distinct_lengths": len(tuned),
           "points": pts, "out_GB": out_bytes / 1e9,
           "batch_graph_ms": ms_batch, "batch_pts_per_s": pts / (ms_batch * 1e-3),
           "per_recording_ms": ms_loop, "per_recording_pts_per_s": pts / (ms_loop * 1e-3),
           "persistent_form_ms": ms_pers,
           "persistent_form_over_graph": ms_pers / ms_batch,
           "batch_hbm_frac": (out_bytes + in_bytes) / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS}
    del items, batch, ws, wss
    for p in plans:
        p.close()
    torch.cuda.empty_cache()
    return res


def bench_long_recording(reps=5):
    """A recording longer than one transform: 5 minutes of 64-channel EEG at
    1000 Hz (300 000 samples), the 100-frequency grid, power out (7.7 GB),
    run as a segmented plan (overlap-save over the full padded length).
    Times `reps` calls of cwt_execute with events."""
    import torch
    import paper_2506_07793_amd as cwt
    import synth
    n, sfreq, C = 300000, 1000.0, 64
    d = synth.eeg_64ch(C=1, N=16)
    x = torch.from_numpy(synth.eeg(C, n, sfreq, 45)).cuda()
    plan = cwt.Plan(n, sfreq, d["freqs"], n_cycles=d["n_cycles"], out="power")
    out = plan.alloc_output(C)
    ws = plan.alloc_workspace(C)
    plan.execute(x, out=out, ws=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.execute(x, out=out, ws=ws)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    res = {"workload": "64 ch x 300000 samples @1000 Hz, 100 log freqs 1-100 Hz, power out, "
                       "segmented plan",
           "padded_len": plan.L, "segments": plan.n_segments,
           "segment_len": int(plan.desc.segment_len),
           "segment_outputs": int(plan.desc.segment_outputs),
           "ms_per_call": ms, "samples_freqs_per_s": C * n * 100 / (ms * 1e-3),
           "out_GB": C * n * 100 * 4 / 1e9}
    del out, ws, x
    plan.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def bench_paper_workload(reps=10):
    """The paper's own throughput workload, for context beside its figure:
    64 channels x 10 s at 2048 Hz (20 480 samples), Morlet sigma 7 at 30-90 Hz
    in 1 Hz steps (61 frequencies), complex64 out (640 MB).  Two rates: inputs
    and outputs resident in HBM, and with the host transfers the paper's
    timing includes (pinned host input copied in, the whole output copied
    back to pinned host memory), each over `reps` calls timed with events."""
    import numpy as np
    import torch
    import paper_2506_07793_amd as cwt
    import synth
    C, sfreq, n = 64, 2048.0, 20480
    freqs = np.arange(30.0, 91.0)
    xh = torch.from_numpy(synth.eeg(C, n, sfreq, 46)).pin_memory()
    plan = cwt.Plan(n, sfreq, freqs, n_cycles=7.0)
    x = xh.cuda()
    out = plan.alloc_output(C)
    ws = plan.alloc_workspace(C)
    host_out = torch.empty(out.shape, dtype=out.dtype, pin_memory=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        plan.execute(x, out=out, ws=ws)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        plan.execute(x, out=out, ws=ws)
    e1.record()
    e1.synchronize()
    ms_dev = e0.elapsed_time(e1) / reps
    e0.record()
    for _ in range(reps):
        x.copy_(xh, non_blocking=True)
        plan.execute(x, out=out, ws=ws)
        host_out.copy_(out, non_blocking=True)
    e1.record()
    e1.synchronize()
    ms_host = e0.elapsed_time(e1) / reps
    pts = C * n * len(freqs)
    res = {"workload": "64 ch x 20480 samples (10 s @2048 Hz), Morlet sigma 7, 61 freqs 30-90 Hz, "
                       "complex64 out",
           "L": plan.L, "kernel": int(plan.desc.kernel),
           "ms_per_call_hbm_resident": ms_dev, "samples_freqs_per_s_hbm_resident": pts / (ms_dev * 1e-3),
           "ms_per_call_with_host_transfers": ms_host,
           "samples_freqs_per_s_with_host_transfers": pts / (ms_host * 1e-3),
           "paper_figure_context": "RTX 4060 Laptop GPU via CuPy, transfers included: "
                                   ">= 8.0e8 samples x freqs / s (10 runs in 1 s)"}
    del out, ws, x, host_out, xh
    plan.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def bench_length_sweep(reps=100):
    """Length sweep (section "Wavelength and flexibility", Figure 4): signals of
    N = 100 ... 2500 samples at 1000 Hz (every 100, the largest prime at or
    below each, and the powers of two in range), Morlet sigma 7 at 30-90 Hz in
    1 Hz steps (61 frequencies), complex64 out.  Each length: `reps` calls of
    cwt_execute (forward + transform) on 1 channel and on 64 channels, timed
    with events; plus the plan-creation time of the paper's Table 2 case
    (61 wavelets of 1 s at 1000 Hz).  Reports the times, a least-squares line
    through (N, time) and, for each prime, its time over the mean of the two
    nearest multiples of 100."""
    import numpy as np
    import torch

    import paper_2506_07793_amd as cwt
    import synth

    def is_prime(m):
        return m > 1 and all(m % d for d in range(2, int(m ** 0.5) + 1))

    rounds = list(range(100, 2501, 100))
    primes = sorted({max(p for p in range(2, n + 1) if is_prime(p)) for n in rounds})
    pows = [128, 256, 512, 1024, 2048]
    lengths = sorted(set(rounds) | set(primes) | set(pows))
    sfreq, freqs = 1000.0, np.arange(30.0, 91.0)
    stream = torch.cuda.Stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    x64 = torch.from_numpy(synth.eeg(64, 2500, sfreq, 7)).cuda()
    rows = []
    t_create = []
    for N in lengths:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = cwt.Plan(N, sfreq, freqs, n_cycles=7.0, stream=stream)
        stream.synchronize()
        t_create.append((N, (time.perf_counter() - t0) * 1e3))
        rec = {"N": N, "L": plan.L, "radices": plan.radices, "kernel": int(plan.desc.kernel),
               "kind": "prime" if is_prime(N) else ("pow2" if N in pows else "round")}
        for C in (1, 64):
            x = x64[:C, :N].contiguous()
            out = plan.alloc_output(C)
            ws = plan.alloc_workspace(C)
            with torch.cuda.stream(stream):
                for _ in range(5):
                    plan.execute(x, out=out, ws=ws, stream=stream)
                ev0.record(stream)
                for _ in range(reps):
                    plan.execute(x, out=out, ws=ws, stream=stream)
                ev1.record(stream)
                torch.cuda.synchronize()
            rec["ms_C%d" % C] = ev0.elapsed_time(ev1) / reps
        rows.append(rec)
        plan.close()
    res = {"workload": "N = 100..2500 at 1000 Hz, Morlet sigma 7, 61 freqs 30-90 Hz, complex64, "
                       "%d calls per length" % reps, "lengths": rows}
    for C in (1, 64):
        n = np.array([r["N"] for r in rows], float)
        t = np.array([r["ms_C%d" % C] for r in rows])
        a, b = np.polyfit(n, t, 1)
        pred = a * n + b
        r2 = 1 - np.sum((t - pred) ** 2) / np.sum((t - t.mean()) ** 2)
        by_n = {r["N"]: r["ms_C%d" % C] for r in rows}
        ratios = []
        for r in rows:
            if r["kind"] == "prime":
                lo, hi = (r["N"] // 100) * 100, (r["N"] // 100 + 1) * 100
                ref = [by_n[m] for m in (lo, hi) if m in by_n]
                if ref:
                    ratios.append(r["ms_C%d" % C] / np.mean(ref))
        res["C%d" % C] = {"ms_per_sample_slope": a, "ms_intercept": b, "r2_linear": r2,
                          "prime_over_neighbours_max": float(np.max(ratios)),
                          "prime_over_neighbours_mean": float(np.mean(ratios))}
    res["plan_create_ms_N1000_61_wavelets"] = dict(t_create)[1000]
    return res


def bench_epoch_lengths(reps=50):
    """EEG epochs of 4, 5, 8 and 10 s at 1000 Hz (L = 4000, 5000, 8000, 10000):
    64 channels, the 100-frequency EEG grid (1-100 Hz, n_cycles = f / 2 in
    [3, 10]), complex64 out; `reps` cwt_execute calls per length, timed with
    events, with the default plan (the mixed-radix register-resident kernel)
    and with CWT_GENERIC_ONLY=1 (the runtime-radix kernel)."""
    import os

    import torch

    import paper_2506_07793_amd as cwt
    import synth

    sfreq = 1000.0
    freqs = synth.log_freqs(1.0, 100.0, 100)
    cyc = synth.eeg_cycles(freqs)
    stream = torch.cuda.Stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for N in (4000, 5000, 8000, 10000):
        x = torch.from_numpy(synth.eeg(64, N, sfreq, 17)).cuda()
        rec = {"N": N}
        for label, generic in (("register", False), ("runtime_radix", True)):
            prev = os.environ.pop("CWT_GENERIC_ONLY", None)
            if generic:
                os.environ["CWT_GENERIC_ONLY"] = "1"
            try:
                plan = cwt.Plan(N, sfreq, freqs, n_cycles=cyc, stream=stream)
            finally:
                os.environ.pop("CWT_GENERIC_ONLY", None)
                if prev is not None:
                    os.environ["CWT_GENERIC_ONLY"] = prev
            out = plan.alloc_output(64)
            ws = plan.alloc_workspace(64)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                for _ in range(5):
                    plan.execute(x, out=out, ws=ws, stream=stream)
                ev0.record(stream)
                for _ in range(reps):
                    plan.execute(x, out=out, ws=ws, stream=stream)
                ev1.record(stream)
                torch.cuda.synchronize()
            rec[label] = {"L": plan.L, "kernel": int(plan.desc.kernel), "radices": plan.radices,
                          "ms": ev0.elapsed_time(ev1) / reps}
            del out, ws
            plan.close()
        rows.append(rec)
    return {"workload": "64 ch x N at 1000 Hz, 100 log freqs 1-100 Hz, complex64, %d calls "
                        "per length and kernel" % reps, "lengths": rows}


def bench_stream(n_sessions, C, sfreq, win_s, hop_s, seconds, seed, max_batch, deadline_us,
                 pad="smooth7"):
    """Real-time serving run: Poisson-arriving sessions push one hop each hop_s.

    n_sessions sessions are open at t = 0; new ones arrive at rate
    n_sessions / 20 s and live an exponential 20 s on average, so about
    n_sessions stay open.  Each session arrives with its window already
    filled (its past samples pushed at open), then pushes one hop every hop_s
    at a random phase.  Latency = result completion - push of the hop's last
    sample, both on CLOCK_MONOTONIC.
    """
    import numpy as np

    import paper_2506_07793_amd as cwt
    import synth
    from paper_2506_07793_amd.stream import Server, now_ns

    W = int(round(win_s * sfreq))
    hop = int(round(hop_s * sfreq))
    freqs = synth.log_freqs(1.0, 100.0, 40)
    plan = cwt.Plan(W, sfreq, freqs, n_cycles=synth.eeg_cycles(freqs), out="bandpower", pad=pad)
    pool = synth.eeg(C, int(30 * sfreq), sfreq, seed)  # shared signal, each session at its own offset
    T = pool.shape[1]
    sched = synth.session_schedule(n_sessions, seconds, hop_s=hop_s, seed=seed)
    srv = Server(64 << 30, max_batch=max_batch, deadline_us=deadline_us, max_pending=256)
    rng = np.random.default_rng(seed)
    events = []  # (time, kind, index)
    for i, (t_open, t_close, phase) in enumerate(sched):
        events.append((t_open, 0, i))
        events.append((min(t_close, seconds), 2, i))
    events.sort()
    sess, offs, nxt, outstanding = {}, {}, {}, {}
    lat = []
    lat_t = []  # push time of each result, s after the start
    t0 = time.perf_counter()
    t0_ns = now_ns()
    hop_times = []  # heap of (t, i)
    import heapq

    def drain(all_=False):
        for i, s in list(sess.items()):
            if outstanding.get(i, 0) == 0:
                continue
            while True:
                r = s.poll()
                if r is None:
                    break
                lat.append((r[3] - r[2]) * 1e-6)
                lat_t.append((r[2] - t0_ns) * 1e-9)
                outstanding[i] -= 1

    ev = 0
    last_drain = 0.0
    pushed = 0
    # The producer loop is Python: a full garbage collection in a process
    # with torch loaded takes 35-50 ms, which would hold back every push and
    # poll and hand the server a burst of hops afterwards.  The collector is
    # paused for the run (its long-lived objects frozen first).
    import gc
    gc.collect()
    gc.freeze()
    gc.disable()
    t0 = time.perf_counter()  # the schedule starts now
    t0_ns = now_ns()
    try:
        while True:
            now = time.perf_counter() - t0
            if now >= seconds:
                break
            while ev < len(events) and events[ev][0] <= now:
                _, kind, i = events[ev]
                ev += 1
                if kind == 0:
                    s = srv.open(plan, C, hop)
                    o = int(rng.integers(0, T - W))
                    s.push(pool[:, o:o + W - hop])  # history: the window minus one hop
                    sess[i], offs[i] = s, o + W - hop
                    outstanding[i] = 0
                    heapq.heappush(hop_times, (now + sched[i][2], i))
                elif i in sess:
                    s = sess.pop(i)
                    s.close()
            while hop_times and hop_times[0][0] <= now:
                t_h, i = heapq.heappop(hop_times)
                if i not in sess:
                    continue
                o = offs[i]
                if o + hop > T:
                    o = 0
                if sess[i].push(pool[:, o:o + hop]):
                    outstanding[i] += 1
                    pushed += 1
                offs[i] = o + hop
                heapq.heappush(hop_times, (t_h + hop_s, i))
            if now - last_drain > 0.005:
                drain()
                last_drain = now
            nt = min(hop_times[0][0] if hop_times else now + 0.001,
                     events[ev][0] if ev < len(events) else now + 0.001)
            if nt > now:
                time.sleep(min(nt - now, 0.001))
        srv.flush()
        drain()
    finally:
        gc.enable()
        gc.unfreeze()
    st = srv.stats()
    elapsed = time.perf_counter() - t0
    for s in list(sess.values()):
        s.close()
    srv.close()
    L_plan = plan.L
    plan.close()
    lat = np.array(lat)
    lat_t = np.array(lat_t)
    steady = lat[lat_t >= 2.0] if lat.size else lat
    # Hops slower than 5 ms, grouped into clusters of nearby push times, each
    # with the session arrivals and departures just before or during it.
    slow = np.nonzero(lat > 5.0)[0] if lat.size else np.zeros(0, int)
    clusters = []
    if slow.size:
        order = slow[np.argsort(lat_t[slow])]
        start = 0
        for j in range(1, order.size + 1):
            if j == order.size or lat_t[order[j]] - lat_t[order[j - 1]] > 0.1:
                idx = order[start:j]
                t_a, t_b = float(lat_t[idx].min()), float(lat_t[idx].max())
                near = [k for (t, k, _) in events if t_a - 0.2 <= t <= t_b + 0.05]
                clusters.append({"t_s": round(t_a, 3), "span_ms": round((t_b - t_a) * 1e3, 1),
                                 "hops": int(idx.size), "max_ms": round(float(lat[idx].max()), 2),
                                 "opens": near.count(0), "closes": near.count(2)})
                start = j
    worst_s = None
    if lat.size:
        sec = np.floor(lat_t).astype(int)
        p99s = [float(np.percentile(lat[sec == k], 99)) for k in np.unique(sec)]
        worst_s = {"second": int(np.unique(sec)[int(np.argmax(p99s))]), "p99_ms": max(p99s)}
    return {
        "workload": "%d sessions x %d ch @%g Hz, %g s window, %g ms hop, 40 log freqs 1-100 Hz, "
                    "band power, %s padding (L = %d)" % (n_sessions, C, sfreq, win_s, hop_s * 1e3,
                                                        pad, L_plan),
        "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
        "p999_ms": float(np.percentile(lat, 99.9)) if lat.size else None,
        # results of hops pushed after the first 2 s (the initial sessions'
        # histories and first windows have gone through by then)
        "steady_p50_ms": float(np.percentile(steady, 50)) if steady.size else None,
        "steady_p99_ms": float(np.percentile(steady, 99)) if steady.size else None,
        "steady_p999_ms": float(np.percentile(steady, 99.9)) if steady.size else None,
        "worst_second_p99": worst_s,
        "results": int(lat.size), "hops_pushed": pushed, "hops_per_s": pushed / elapsed,
        "batches": st["batches"], "mean_batch": st["hops"] / max(1, st["batches"]),
        "max_batch_hops": st["max_batch_hops"], "max_batch_ms": st["max_batch_ns"] * 1e-6,
        "slot_waits": st["slot_waits"],
        "slow_hops": {"over_ms": 5.0, "count": int(slow.size), "clusters": len(clusters),
                      "worst_clusters": sorted(clusters, key=lambda c: -c["hops"])[:8]},
        "seconds": seconds, "max_batch": max_batch, "deadline_us": deadline_us}


def bench_torch_fft(plan, x, C, N, F, stream, steps, W_ref):
    """Same-GPU library context: the pipeline composed from torch.fft (the ROCm
    FFT library) and one broadcast multiply, with the plan's own FP32 spectra
    scattered into a dense [F, L] table: forward FFT of each channel, product
    with every frequency's spectrum, batched inverse FFT, crop to N."""
    import numpy as np
    import torch
    L = plan.L
    H, band, _ = plan.tables()
    Hd = np.zeros((F, L), dtype=np.float32)
    for i, (lo, K, off) in enumerate(band):
        Hd[i, (lo + np.arange(K)) % L] = H[off:off + K]
    Hg = torch.from_numpy(Hd).to(x.device)

    def run():
        X = torch.fft.fft(x, n=L)                          # [C, L] complex64
        Y = X[:, None, :] * Hg[None, :, :]                 # [C, F, L]
        return torch.fft.ifft(Y, dim=-1, norm="forward")[..., :N]  # 1/L is in H

    with torch.cuda.stream(stream):
        W = run()
        torch.cuda.synchronize()
        e_W = float((W - W_ref).abs().max() / W_ref.abs().max())
        del W
        for _ in range(5):
            run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            run()
        e1.record(stream)
        e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return {"kind": "torch.fft (ROCm FFT library) composite of the same pipeline, same GPU",
            "ms_per_step": ms, "value": C * F * N / (ms * 1e-3),
            "max_rel_diff_vs_this_library": e_W}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus 1); the path would shard by channels, "
              "rows, recordings or stream sessions with no exchange step, one process per "
              "GPU, but only the one-GPU share is implemented and measured", file=sys.stderr)
        sys.exit(2)

    # The single-thread oracle timing runs in a child process, started here
    # before this process touches the GPU.
    single = None
    if not args.no_cpu_baseline and not args.copy_calibration:
        single = oracle_single_thread(None, 2)

    import numpy as np
    import torch

    import paper_2506_07793_amd as cwt
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "copies": 3}), flush=True)
        return
    C, N, F = 64, 4096, 100
    cfg = synth.eeg_64ch(seed=2, C=C, N=N, F=F)
    x = torch.from_numpy(cfg["x"]).to(dev)
    plan = cwt.Plan(N, cfg["sfreq"], cfg["freqs"], n_cycles=cfg["n_cycles"], out=args.out)
    out = plan.alloc_output(C, device=dev)
    ws = plan.alloc_workspace(C, device=dev)
    stream = torch.cuda.Stream()  # default priority

    # Every step runs the whole path on one batch (the same resident input)
    # and writes its own output buffer: the steps cycle through a ring of
    # RING output buffers (13.4 GB), far beyond the 256 MB last-level cache,
    # so that every step's output reaches HBM.  Overwriting one 210 MB buffer
    # each step can be partly absorbed by that cache (on some boxes it is);
    # that form is timed too and reported beside (`one_output_buffer`).
    ob = plan.output_bytes(C)
    RING = 64
    ring = torch.empty(RING * ob, dtype=torch.uint8, device=dev)
    slot = [0]

    def step():
        plan.forward_spectra(x, ws, stream=stream)
        i = slot[0]
        plan.transform_spectra(C, ring[i * ob:(i + 1) * ob], ws, stream=stream)
        slot[0] = (i + 1) % RING

    # Pipelined form (cwt_execute_batches): one launch per step that
    # transforms this step's batch and computes the next batch's forward FFT
    # into the other half of a double-buffered workspace; one call per pass
    # over the ring (its last step has no next batch to fuse).
    wsb = plan.alloc_batches_workspace(C, device=dev)

    def chunks(n):
        out_n = []
        while n > 0:
            out_n.append(min(RING, n))
            n -= out_n[-1]
        return out_n

    def batches(n):
        for m in chunks(n):
            plan.execute_batches(x, m, ring, wsb, C, x_batch_stride=0, out_batch_stride=ob,
                                 stream=stream)

    def batches_one_buffer(n):
        plan.execute_batches(x, n, out, wsb, C, x_batch_stride=0, out_batch_stride=0,
                             stream=stream)

    def timed(fn):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    def preroll(min_ms, tol=0.02, max_ms=3000.0):
        """Untimed pipelined steps, one ring pass per chunk, until at least
        min_ms of GPU time has passed and the last two chunk means agree
        within tol (at most max_ms)."""
        total, n, means = 0.0, 0, []
        while True:
            ms = timed(lambda: batches(RING))
            total += ms
            n += RING
            means.append(ms / RING)
            settled = len(means) >= 2 and abs(means[-1] - means[-2]) <= tol * means[-2]
            if (total >= min_ms and settled) or total >= max_ms:
                break
        return {"gpu_ms": total, "steps": n, "settled": settled,
                "last_two_chunk_ms_per_step": means[-2:]}

    K = args.steps
    serial = not args.graph and args.serial
    with torch.cuda.stream(stream):
        pre = preroll(args.preroll_ms) if args.preroll_ms > 0 else None
        for _ in range(args.warmup):
            step()
        batches(args.warmup)
        torch.cuda.synchronize()

        # Serial reference first (forward + transform per step, no
        # pipelining), so that the timed region runs on a warm device.
        ms_serial = timed(lambda: [step() for _ in range(K)]) / K

        # The timed region: K steps.  Default: K pipelined steps (one
        # cwt_execute_batches call); --serial: K forward + transform pairs;
        # --graph 1: K replays of a captured forward + transform step.
        if args.graph:
            # (a captured step writes the ring slot it was captured with)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                step()
            for _ in range(args.warmup):
                g.replay()

            def region():
                for _ in range(K):
                    g.replay()
        elif serial:
            def region():
                for _ in range(K):
                    step()
        else:
            def region():
                batches(K)
        ms_step = timed(region) / K

        # The kernel's launch durations: the same K steps once more, each
        # transform launch carrying a pair of events bound to its own
        # dispatch (cwt_plan_timing_start; no system-scope fence, so no
        # cache write-back), on the stream it runs on.  They widen the gap
        # between launches by about a microsecond, which is why the step
        # time above comes from a pass without them.  (A graph cannot carry
        # them: with --graph the kernel is timed on direct steps.)
        plan.timing_start(K)
        if args.graph or serial:
            ms_step_ev = timed(lambda: [step() for _ in range(K)]) / K
        else:
            ms_step_ev = timed(lambda: batches(K)) / K
        kernel_ms = plan.timing_stop()
        assert len(kernel_ms) == K, "timed %d of %d transform launches" % (len(kernel_ms), K)
        fused = not (args.graph or serial) and plan.desc.kernel == 1 and K > 1
        if fused:
            # the last step of each call has no next batch to fuse
            ends = set(np.cumsum(chunks(K)) - 1)
            kernel_ms = np.array([m for i, m in enumerate(kernel_ms) if i not in ends])
        ms_main = float(np.mean(kernel_ms))

        # Store ceiling: a plain device fill of one output buffer per step,
        # cycling through the ring like the steps.
        fills = [ring[i * ob:(i + 1) * ob].view(torch.float32) for i in range(RING)]
        for f_ in fills[:3]:
            f_.fill_(0.0)
        ms_fill = timed(lambda: [fills[i % RING].fill_(0.0) for i in range(K)]) / K

        # The same pipelined steps overwriting one output buffer.
        one_buf = None
        if not (args.graph or serial):
            batches_one_buffer(K)
            ms_one = timed(lambda: batches_one_buffer(K)) / K
            one_buf = {"ms_per_step": ms_one, "value": C * F * N / (ms_one * 1e-3),
                       "MB": ob / 1e6}

    pts = C * F * N
    value = pts / (ms_step * 1e-3)
    desc = plan.desc
    # Algorithmic flops of one transform launch: 5 L log2 L per inverse
    # transform (C x F of them) and 2 per stored spectrum bin per channel
    # (the complex-by-real multiply)
    import math
    transform_flops = C * F * 5.0 * plan.L * math.log2(plan.L) + C * 2.0 * int(desc.spectrum_bins)
    elem = 8 if args.out == "complex64" else 4
    out_elems = C * plan.out_rows * N  # F rows, or the bands' rows in band-power mode
    Lh = plan.L // 2 + 1
    # Algorithmic bytes of one launch of the transform kernel: every output
    # element written once, every channel half-spectrum and every stored
    # wavelet-spectrum bin read once; the pipelined launch also reads the
    # next batch's signal and writes its half spectra once.
    transform_bytes = out_elems * elem + C * Lh * 8 + int(desc.spectrum_bins) * 4
    main_bytes = transform_bytes + (C * N * 4 + C * Lh * 8 if fused else 0)
    achieved = main_bytes / (ms_main * 1e-3) / 1e9
    # Whole step: the input signal and the spectra round trip as well.
    step_bytes = out_elems * elem + C * Lh * 8 + int(desc.spectrum_bins) * 4 + C * N * 4 + C * Lh * 8

    if args.out == "bandpower":
        # 5.2 MB of output per step: arithmetic, not HBM, bounds this mode
        ach_tf = transform_flops / (ms_main * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": kernel_name(plan, fused), "achieved": ach_tf,
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach_tf / FP32_VECTOR_PEAK_TFLOPS,
                "traffic": committed_traffic(plan, args.out, "fused" if fused else "main"),
                "algorithmic_flops": transform_flops, "algorithmic_bytes": main_bytes,
                "avg_ms": ms_main, "median_ms": float(np.median(kernel_ms)),
                "kernel_avg_within_step": bool(ms_main <= ms_step)}
    else:
        roof = None
    result = {
        "metric": "CWT output samples x freqs per second (+ %HBM roofline; p99 stream window "
                  "latency)",
        "value": value,
        "unit": "samples*freqs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain CWT 64ch x 4096 @1000Hz, 100 log freqs 1-100 Hz, "
                               "n_cycles=clip(f/2,3,10), FP32 in, %s out" % args.out,
                   "channels": C, "samples": N, "freqs": F, "padded_len": plan.L,
                   "radices": plan.radices, "out": args.out,
                   "launch": ("hip graph replay of forward + transform" if args.graph else
                              "forward + transform per step" if serial else
                              "pipelined: one launch per step (transform + next forward)")},
        "roofline": {"bound": "hbm", "kernel": kernel_name(plan, fused),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": committed_traffic(plan, args.out, "fused" if fused else "main"),
                     "algorithmic_bytes": main_bytes, "avg_ms": ms_main,
                     "median_ms": float(np.median(kernel_ms)),
                     "p90_ms": float(np.percentile(kernel_ms, 90)),
                     # the kernel's launches cannot take longer than the steps that
                     # contain them; False flags a run whose clock changed between
                     # the timed pass and the event pass
                     "kernel_avg_within_step": bool(ms_main <= ms_step),
                     # the same algorithmic bytes over the whole step (launch gaps
                     # included), the figure the step clock gives
                     "step_frac": main_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS}
                    if roof is None else roof,
        "preroll": pre,
        "step_hbm_frac": step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "store_bytes_per_launch": out_elems * elem,
        "output_ring": {"buffers": RING, "MB": RING * ob / 1e6},
        "one_output_buffer": one_buf,
        "ms_per_step_with_timing_events": ms_step_ev,
        "serial_steps": {"ms_per_step": ms_serial, "value": pts / (ms_serial * 1e-3)},
        "store_ceiling": {"kernel": "torch fill_ of the output buffer",
                          "GBps": out.numel() * out.element_size() / (ms_fill * 1e-3) / 1e9,
                          "ms": ms_fill},
    }

    # Precision variants: the same 64-channel workload through the split-precision
    # DFT-as-GEMM (MFMA) transform kernel.  Their errors against the FP64
    # oracle are measured by tests/test_gpu_split.py.
    prec_runs = []
    W32 = plan.execute(x) if args.out == "complex64" else None
    for prec in ("split_f16", "split_bf16"):
        pp = cwt.Plan(N, cfg["sfreq"], cfg["freqs"], n_cycles=cfg["n_cycles"], out=args.out,
                      precision=prec)
        # its own workspace: band power on these kernels also holds chunk rows
        wsp = pp.alloc_workspace(C)
        with torch.cuda.stream(stream):
            pp.forward_spectra(x, wsp, stream=stream)
            for i in range(3):
                pp.transform_spectra(C, ring[i * ob:(i + 1) * ob], wsp, stream=stream)
            torch.cuda.synchronize()
            pp.timing_start(K)
            for i in range(K):
                j = i % RING
                pp.transform_spectra(C, ring[j * ob:(j + 1) * ob], wsp, stream=stream)
            ms_p = float(np.mean(pp.timing_stop()))
        run = {"precision": prec, "transform_ms": ms_p,
               "transform_pts_per_s": pts / (ms_p * 1e-3),
               "hbm_frac": transform_bytes / (ms_p * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if W32 is not None:
            # difference from the FP32 path's output on the same input (its
            # error against the FP64 oracle is what tests/test_gpu_split.py gates)
            Wp = pp.execute(x)
            torch.cuda.synchronize()
            P32, Pp = W32.abs() ** 2, Wp.abs() ** 2
            run["vs_fp32_path"] = {
                "max_rel_W": float((Wp - W32).abs().max() / W32.abs().max()),
                "max_rel_P": float((Pp - P32).abs().max() / P32.max()),
                "mean_rel_P": float((Pp - P32).abs().mean() / P32.max())}
            del Wp, P32, Pp
        prec_runs.append(run)
        pp.close()
    result["precision_variants"] = prec_runs
    del ring, fills, W32
    torch.cuda.empty_cache()

    # Outputs of every precision and output mode on the first PREC_C channels,
    # compared with the FP64 oracle in the CPU leg below.
    PREC_C = 2
    prec_out = {}
    for prec in ("fp32", "split_f16", "split_bf16"):
        for mode in ("complex64", "power", "bandpower"):
            pp = cwt.Plan(N, cfg["sfreq"], cfg["freqs"], n_cycles=cfg["n_cycles"], out=mode,
                          precision=prec)
            prec_out[(prec, mode)] = pp.execute(x[:PREC_C]).cpu().numpy()
            pp.close()
    torch.cuda.synchronize()

    if args.out == "complex64":
        W_ref = plan.execute(x)
        result["library_baseline"] = bench_torch_fft(plan, x, C, N, F, stream, min(K, 50), W_ref)
        result["library_baseline"]["speedup_of_this_library"] = (
            result["library_baseline"]["ms_per_step"] / ms_step)
        del W_ref
        torch.cuda.empty_cache()

    progress("plain transform done: %.4f ms per step" % ms_step)
    if args.batch_steps > 0:
        result["batch"] = bench_batch(args.batch_steps)
        progress("batch done")

    if args.length_sweep:
        result["length_sweep"] = bench_length_sweep()
        progress("length sweep done")
        result["long_recording"] = bench_long_recording()
        progress("long recording done")
        result["paper_workload"] = bench_paper_workload()
        progress("paper's workload done")
        result["epoch_lengths"] = bench_epoch_lengths()
        progress("epoch lengths done")

    if args.stream_seconds > 0:
        legs = [
            ((512, 64, 1000.0, 2.0, 0.05), 5, 512, {}),
            ((64, 256, 2048.0, 2.0, 102 / 2048.0), 6, 64, {}),
            # the first workload with linear-edge plans: no cyclic wrap of the
            # window's oldest samples reaches the trailing hop
            ((512, 64, 1000.0, 2.0, 0.05), 5, 512, {"pad": "linear"}),
        ]
        result["stream"] = []
        for (ns, sc, sf, win, hop), seed, mb, kw in legs:
            result["stream"].append(bench_stream(ns, sc, sf, win, hop, args.stream_seconds, seed,
                                                 mb, args.stream_deadline_us, **kw))
            progress("serving leg %d sessions x %d ch %s done" % (ns, sc, kw.get("pad", "")))
        result["p99_stream_ms"] = result["stream"][0]["p99_ms"]

    if not args.no_cpu_baseline:
        import oracle
        Cs = max(1, min(C, args.cpu_channels))
        rows = [(c, f) for c in range(Cs) for f in range(F)]
        xs = cfg["x"].astype(np.float64)
        passes = 0
        t0 = time.perf_counter()
        while True:
            oracle.cwt(xs, cfg["sfreq"], cfg["freqs"], cfg["n_cycles"], rows=rows)
            passes += 1
            dt = time.perf_counter() - t0
            if dt >= args.cpu_seconds or passes >= 8:
                break
        # Each precision's error against the FP64 oracle, per output kind,
        # on PREC_C channels x all frequencies x all samples (relative to the
        # largest reference value of that output).
        ref = oracle.cwt(xs[:PREC_C], cfg["sfreq"], cfg["freqs"], cfg["n_cycles"])
        P_ref = oracle.power(ref)
        BP_ref = oracle.band_power(P_ref, oracle.band_groups(cfg["freqs"]))
        pvo = {"sample": "%d channels x %d freqs x %d samples of the workload above" % (
            PREC_C, F, N)}
        for prec in ("fp32", "split_f16", "split_bf16"):
            Wg = prec_out[(prec, "complex64")].astype(np.complex128)
            e = {}
            dW = np.abs(Wg - ref) / np.abs(ref).max()
            e["complex"] = {"max_rel_W": float(dW.max()), "mean_rel_W": float(dW.mean())}
            for mode, R, key in (("power", P_ref, "power"), ("bandpower", BP_ref, "band_power")):
                d = np.abs(prec_out[(prec, mode)].astype(np.float64) - R) / R.max()
                e[key] = {"max_rel": float(d.max()), "mean_rel": float(d.mean())}
            dP = np.abs(oracle.power(Wg) - P_ref) / P_ref.max()
            e["power_of_complex"] = {"max_rel": float(dP.max()), "mean_rel": float(dP.mean())}
            pvo[prec] = e
        result["precision_vs_oracle"] = pvo
        result["cpu_baseline"] = {
            "value": passes * len(rows) * N / dt, "unit": "samples*freqs/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d pass(es) over %d of %d channels x %d freqs x %d samples (FP64 direct "
                      "cyclic convolution, %.1f s in all)" % (passes, Cs, C, F, N, dt),
            "cpu_model": cpu_model(),
            "single_thread": single}
        # Context: the paper's own method (FFT, multiply, inverse FFT) in FP64
        # on the same host cores, with the oracle's closed-form spectra.
        import scipy.fft as sfft
        L = plan.L
        Hb = oracle.wavelet_bank(L, cfg["sfreq"], cfg["freqs"], cfg["n_cycles"])
        nt = oracle.num_threads()
        t0 = time.perf_counter()
        for c in range(C):
            Xc = sfft.fft(xs[c], n=L)
            Wc = sfft.ifft(Xc[None, :] * Hb, axis=-1, workers=nt)[:, :N]
        dt_fft = time.perf_counter() - t0
        del Wc
        result["cpu_fft_context"] = {
            "kind": "scipy.fft FP64 pipeline of the paper's method (forward FFT, multiply, "
                    "inverse FFT per channel and frequency), whole job, host cores",
            "value": C * F * N / dt_fft, "unit": "samples*freqs/s", "threads": nt,
            "seconds": dt_fft}
    plan.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
