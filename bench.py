"""Throughput of the fused MRT stream-collide sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]

Headline workload: D2Q9 MRT, nonlinear anisotropic CDE with the Scheme-A
source on a periodic 1024 x 1024 grid (B = 0.5 phi^2 (1, 1),
K = K0 (1 + phi^2), R = 0.1 phi (1 - phi), phi0 = 0.5 + 0.1 U[-1, 1) seed 2),
distributions stored as FP32 offsets.  One step = one time step of every
node: one fused sweep, or half of a pass that runs two time steps (the
autotuner's choice where it is faster; the results are bit-identical).  The
value is the median of 5 timed regions of --steps steps each.  The roofline
object describes the kernel launched: algorithmic bytes per node update (one
read and one write of every population and of the phi history) times the
updates one launch performs, over the launch time; a two-step pass performs
two updates per node while moving the state once, so its fraction can exceed
1 (its fraction on its own bytes is reported beside it), and single sweeps
are reported beside it too.  The same run in FP64 storage, the
reversed (adjoint) sweep on the
512 x 512 adjoint workload, the D3Q19 sweep on 256^3 with walls, a plain copy
kernel (practical HBM ceiling) and the CPU oracle on a bounded sample are
reported beside it.  Inputs are synthetic and resident in HBM before timing.
Prints one JSON line.
"""
import argparse
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "MRT LBM MLUPS & % of HBM roofline (fwd+adjoint), FP32-store vs FP64 at fixed err"


def bytes_per_node(q, prec, src):
    """Algorithmic bytes of one node update: each population read once and
    written once, plus the phi history read and write for the Scheme-A source."""
    s = {"f64": 8, "f32": 4, "f16": 2}[prec]
    h = 8 if prec == "f64" else 4
    return 2 * q * s + (2 * h if src else 0)


def adjoint_bytes_per_node(q, prec, src):
    """Reversed sweep: read f_s and psi_{s+1} (q each), write psi_s (q); read
    pi_{s+1} and write pi_s (FP64); read the phi history (Scheme A)."""
    s = 8 if prec == "f64" else 4
    h = 8 if prec == "f64" else 4
    return 3 * q * s + 2 * 8 + (h if src else 0)


def kernel_hash():
    """Hash of the library's code, without its // comments and blank lines,
    so that an edit of a comment does not void the committed profiles (the
    sources contain no string literal with // in it)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1603_09577_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".h", ".hip")):
            for line in open(os.path.join(csrc, f), encoding="utf-8"):
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def profile_entry(kernel_key, kernel=None):
    """The committed rocprofv3 summary of a workload (HBM traffic per launch,
    VALU issue fraction), or None when it is missing, was taken on different
    kernel sources, or (with `kernel`) profiled another kernel variant."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    v = d.get("workloads", {}).get(kernel_key)
    if v is None or (kernel is not None and not v.get("kernel", "").startswith(kernel)):
        return None
    return v


SAMPLES = 5          # timed samples of `steps` steps each; the median is reported
PREROLL_CYCLES = 2_000_000


def time_steps(torch, sim, steps, warmup, samples=SAMPLES):
    """Time per step: the median over `samples` timed regions of `steps`
    steps each (HIP events on the stream the kernels run on), after `warmup`
    untimed steps.  Before each region a spin kernel holds the GPU for about
    a millisecond while the host enqueues the region's launches, so that a
    short region measures the sweeps back to back rather than the host's
    launch latency; the device synchronises before and after each region.
    Returns (median seconds per step, details)."""
    import statistics
    sim.step(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    per, walls = [], []
    for _ in range(samples):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(PREROLL_CYCLES)
        t0 = time.perf_counter()
        e0.record(st)
        sim.step(steps)
        e1.record(st)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        per.append(e0.elapsed_time(e1) / 1e3 / steps)
    med = statistics.median(per)
    return med, {"samples": samples, "ms_per_step_samples": [round(v * 1e3, 6) for v in per],
                 "ms_per_step_min": min(per) * 1e3, "ms_per_step_max": max(per) * 1e3,
                 "wall_s": sum(walls)}


# tile shape forced on D2Q9 two-step runs after tuning, with the XCD-aware
# order (--two-step-shape; None: the tuner's choices)
TWO_STEP_SHAPE = None
# whether the adjoint pair's trial also times every tile shape (--adjoint-tile-pick: no)
ADJ_TILE_TRIAL = True
# [(rows, waves), ...] two-step shapes forced on D3Q19 runs, the first the
# precision has (--two-step-3d; None: the tuner's choice between single
# sweeps and each shape)
TWO_STEP_3D = None


def run_forward(torch, lbm, spec, phi0, steps, warmup, label, tune=True, two_step=None):
    """Time `steps` sweeps.  With tune, the launch shape is the autotuner's
    (which may pick two time steps per pass); two_step forces that choice,
    TWO_STEP_SHAPE the tile shape of a two-step run."""
    sim = lbm.Lbm(spec).init(phi0)
    rep = sim.tune(reps=20).splitlines()[-1] if tune else "untuned"
    if two_step is not None:
        sim.set_two_step(two_step)
        rep += f"; two steps per pass forced {'on' if two_step else 'off'}"
    if TWO_STEP_3D is not None and sim.q == 19 and two_step is None:
        shapes = sim.two_step_shapes()
        pick = next((sh for sh in TWO_STEP_3D if sh in shapes), None)
        if pick is not None:
            sim.set_two_step(True, shapes.index(pick))
            r, w = pick
            rep = re.sub(r" two \d rows \d+ waves \d+", f" two 1 rows {r} waves {w}", rep)
            rep += f"; two steps per pass with shape {r} x {w} forced"
    elif TWO_STEP_SHAPE is not None and (" two 1" in rep if two_step is None else two_step):
        shapes = sim.two_step_shapes()
        if TWO_STEP_SHAPE < len(shapes):
            sim.set_two_step(True, TWO_STEP_SHAPE)
            sim.set_remap(True)
            r, w = shapes[TWO_STEP_SHAPE]
            rep = re.sub(r" rows \d+ waves \d+", f" rows {r} waves {w}", rep)
            rep = re.sub(r" remap \d", " remap 1", rep) + f"; shape {r} x {w} and XCD order forced"
    two = (" two 1" in rep) if two_step is None else bool(two_step)
    m = re.search(r" rows (\d+) waves (\d+)", rep)
    rows = f"{m.group(1)} rows x {m.group(2)} waves" if (two and m) else None
    per, tinfo = time_steps(torch, sim, steps, warmup)
    N = sim.N
    prec = spec.get("precision", "f64")
    src = bool(spec.get("rpoly")) and spec.get("scheme", "A") == "A"   # Scheme B keeps no phi history
    bpn = bytes_per_node(sim.q, prec, src)
    out = {
        "label": label, "nodes": N, "steps": steps, "ms_per_step": per * 1e3,
        "mlups": N / per / 1e6, "bytes_per_node": bpn, "two_step": two, "tile_rows": rows,
        "timing": tinfo, "tuner": rep,
    }
    # algorithmic bytes of the launched kernel: a single sweep reads and writes
    # the state once per step; a two-step pass once per two steps
    launch_bytes = bpn * N
    launch_s = 2 * per if two else per
    out["achieved_gbs"] = launch_bytes / launch_s / 1e9
    out["hbm_frac"] = out["achieved_gbs"] / PEAK_HBM_GBS
    # per node update at the single-sweep bytes (the HBM roofline of one sweep per step)
    out["per_update_hbm_frac"] = bpn * N / per / 1e9 / PEAK_HBM_GBS
    phi = sim.phi()
    r = sim.reduce(phi)
    out["nonfinite"] = int(r["nonfinite"])
    return out, sim, phi


def adjoint_pair_bytes_per_node(q, prec, src):
    """Two reversed sweeps per launch: one sweep's bytes plus the second
    forward state (f_{s-1} and its phi history); psi_s and pi_s stay on chip."""
    s = 8 if prec == "f64" else 4
    h = 8 if prec == "f64" else 4
    return adjoint_bytes_per_node(q, prec, src) + q * s + (h if src else 0)


def time_diagnostics(torch, sim, head_ms_per_step, every=100, reps=50):
    """Cost of the FP64 diagnostics on a forward state: phi in FP64
    (lbm_get_phi) and the FP64 sums, min/max and non-finite count
    (lbm_reduce, which returns its results to the host), per call, and as a
    fraction of the sweeps when taken every `every` steps."""
    import time
    phi = sim.phi()
    for _ in range(5):
        sim.reduce(sim.phi(out=phi))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.reduce(sim.phi(out=phi))
    per = (time.perf_counter() - t0) / reps
    # the same work without waiting (lbm_reduce_async: results stay on the device)
    out = torch.empty(8, dtype=torch.float64, device=phi.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sim.reduce_async(sim.phi(out=phi), out=out)
    e1.record()
    torch.cuda.synchronize()
    per_async = e0.elapsed_time(e1) / 1e3 / reps
    # phi formed inside the reduction (lbm_reduce_state: one pass over the state)
    e0.record()
    for _ in range(reps):
        sim.reduce_state(out=out)
    e1.record()
    torch.cuda.synchronize()
    per_state = e0.elapsed_time(e1) / 1e3 / reps
    return {"ms_per_call": per * 1e3, "every_steps": every,
            "ms_per_call_state": per_state * 1e3,
            "fraction_of_sweep_time_state": per_state * 1e3 / (every * head_ms_per_step),
            "fraction_of_sweep_time": per * 1e3 / (every * head_ms_per_step),
            "ms_per_call_async": per_async * 1e3,
            "fraction_of_sweep_time_async": per_async * 1e3 / (every * head_ms_per_step),
            "what": "phi to FP64 plus FP64 sum, sum of squares, min, max and non-finite count; "
                    "synchronous (lbm_reduce, results on the host), without waiting (lbm_reduce_async), "
                    "and in one pass over the state without a phi field (lbm_reduce_state)"}


def run_adjoint(torch, lbm, spec, phi0, steps, warmup, label, pairs=True):
    """Time the reversed sweep on a fixed forward state: `steps` sweeps
    captured in a HIP graph (through torch's graph capture, which records the
    library's launches on the capture stream) and replayed.  Where the
    rollout would take two reversed sweeps per launch (they apply and its
    timed trial prefers them), they are what is timed, and the one-sweep
    kernel beside them."""
    sim = lbm.Lbm(spec).init(phi0)
    sim.step(10)
    which, _ = sim.current()
    f_s, p_s = sim.f[which], sim.p
    # the pair's second forward state sits in other buffers, as in the rollout
    # (the other distribution buffer holds the state one sweep earlier)
    f_m, p_m = sim.f[1 - which], sim.p.clone()
    psi_a, pi = sim.adjoint_buffers()
    psi_b, pi_b = sim.adjoint_buffers()
    g = torch.full(sim.shape, 1e-3, dtype=torch.float64, device=sim.device)
    use_pairs = pairs and steps % 2 == 0 and sim.adjoint_pairs_faster(shapes=ADJ_TILE_TRIAL)
    sim.adjoint_seed(g, psi_a, pi)

    def launches(n):
        a, b, pa, pb = psi_a, psi_b, pi, pi_b
        if use_pairs:
            for i in range(n // 2):
                sim.adjoint_step2(f_s, p_s, f_m, p_m, a, pa, b, pb)
                a, b, pa, pb = b, a, pb, pa
        else:
            for i in range(n):
                sim.adjoint_step(f_s, p_s, a, pa, b, pa)
                a, b = b, a

    launches(warmup - warmup % 2)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    with torch.cuda.graph(graph, stream=cap):
        launches(steps)
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    per = e0.elapsed_time(e1) / 1e3 / (steps * reps)
    prec = spec.get("precision", "f64")
    src = bool(spec.get("rpoly"))
    bpn1 = adjoint_bytes_per_node(sim.q, prec, src)
    out = {"label": label, "nodes": sim.N, "steps": steps, "ms_per_step": per * 1e3,
           "mlups": sim.N / per / 1e6, "pairs": use_pairs}
    if use_pairs:
        r, w = sim.adjoint_tile_shapes()[sim.adjoint_tile]
        out["tile"] = f"{r} rows x {w} waves"
        bpl = adjoint_pair_bytes_per_node(sim.q, prec, src)
        gbs = bpl * sim.N / (2 * per) / 1e9
        out.update({"bytes_per_node": bpl, "bytes_per_node_note": "per launch of two reversed sweeps",
                    "achieved_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS,
                    "per_update_hbm_frac": bpn1 * sim.N / per / 1e9 / PEAK_HBM_GBS})
        del graph
        out["single_sweep"] = run_adjoint(torch, lbm, spec, phi0, steps, warmup, label, pairs=False)
    else:
        gbs = bpn1 * sim.N / per / 1e9
        out.update({"bytes_per_node": bpn1, "achieved_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS,
                    "per_update_hbm_frac": gbs / PEAK_HBM_GBS})
    return out


def run_batch(torch, lbm, W, steps):
    """The batched workload: 512 D2Q9 instances (FP32 offsets), autotuned
    launch shape, `steps` steps of every instance; aggregate MLUPS."""
    items = W.batch_specs()
    b = lbm.Batch([s for s, _ in items]).init([p for _, p in items])
    rep = b.tune(reps=3)
    per, tinfo = time_steps(torch, b, steps, 32, samples=3)
    N = b.total_nodes
    bpn = bytes_per_node(9, "f32", False)
    fin = torch.isfinite(b.phi()).all().item()
    shape = b.get_shape()
    two = shape["npt"] < 0        # two time steps per launch: the state crosses HBM once per two steps
    launch_gbs = bpn * N / ((2 if two else 1) * per) / 1e9
    return {"instances": len(items), "nodes": N, "steps": steps, "ms_per_step": per * 1e3,
            "mlups": N / per / 1e6, "bytes_per_node": bpn, "two_step": two, "achieved_gbs": launch_gbs,
            "hbm_frac": launch_gbs / PEAK_HBM_GBS, "per_update_hbm_frac": bpn * N / per / 1e9 / PEAK_HBM_GBS,
            "shape": shape, "tuner": rep.splitlines()[-1], "finite": bool(fin), "timing": tinfo}


def copy_probe(torch, lbm, nbytes=1 << 30, reps=20):
    """Plain device copy (the library's 16-byte-per-lane copy kernel) of a
    buffer much larger than the caches: read + write bytes per second."""
    n = nbytes // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    out = {"bytes_per_copy": 2 * nbytes}
    for grid in (0, 256 * 16):
        for _ in range(3):
            lbm.probe_copy(a, b, grid)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            lbm.probe_copy(a, b, grid)
        e1.record()
        torch.cuda.synchronize()
        per = e0.elapsed_time(e1) / 1e3 / reps
        out["gbs_one_chunk_per_workgroup" if grid == 0 else f"gbs_grid{grid}"] = 2 * nbytes / per / 1e9
    out["gbs"] = max(v for k, v in out.items() if k.startswith("gbs_"))
    return out


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(spec, phi0, target_s=12.0, single_s=6.0):
    """The oracle as it stands, on the host cores, on a bounded number of
    steps of the same workload; MLUPS over the timed steps, with OpenMP on
    every thread the box grants (OMP_NUM_THREADS) and on one thread."""
    import oracle as orc
    p = orc.params_from_spec(dict(spec, precision="f64"))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    f, pp = orc.init(p, phi0)
    t0 = time.perf_counter()
    orc.step(p, f, pp, nthreads=threads)
    one = time.perf_counter() - t0
    n = max(1, min(200, int(target_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    for _ in range(n):
        orc.step(p, f, pp, nthreads=threads)
    dt = time.perf_counter() - t0
    N = orc.nodes(p)
    phi_after = orc.phi(p, f)
    # one thread, continuing from the same state (a separate sample)
    t0 = time.perf_counter()
    orc.step(p, f, pp, nthreads=1)
    one1 = time.perf_counter() - t0
    n1 = max(1, min(50, int(single_s / max(one1, 1e-3))))
    t0 = time.perf_counter()
    for _ in range(n1):
        orc.step(p, f, pp, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": N * n / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "single_thread_mlups": N * n1 / dt1 / 1e6, "cpu_model": cpu_model(),
            "host_threads_visible": os.cpu_count(),
            "sample": f"{n + 1} steps of the 1024x1024 D2Q9 headline workload in FP64 "
                      f"(first step untimed), OpenMP over nodes on {threads} threads; then "
                      f"{n1 + 1} steps on one thread (first untimed)"}, phi_after, n + 1


# ---------------------------------------------------------------------------
# rocprofv3 summaries: the committed profiles are written from the raw CSVs
# of the three profiled runs named in PROFILE_COMMANDS.
# ---------------------------------------------------------------------------

PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats -d gpurun_out/prof_trace -o trace --output-format csv -- "
             "python3 bench.py --no-cpu --steps 1000 --warmup 50 --two-step-shape 1 --two-step-3d 14x16,6x8 "
             "--adjoint-tile-pick",
    "fetch": "rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_fetch -o fetch --output-format csv -- "
             "python3 bench.py --no-cpu --steps 20 --warmup 0 --only adjoint,d3q19,batch --two-step-shape 1 --two-step-3d 14x16,6x8 "
             "--adjoint-tile-pick",
    "write": "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_write -o write --output-format csv -- "
             "python3 bench.py --no-cpu --steps 20 --warmup 0 --only adjoint,d3q19,batch --two-step-shape 1 --two-step-3d 14x16,6x8 "
             "--adjoint-tile-pick",
    "valu": "rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVES -d gpurun_out/pmc_valu -o valu "
            "--output-format csv -- python3 bench.py --no-cpu --steps 20 --warmup 0 --only adjoint,d3q19 "
            "--two-step-shape 1 --two-step-3d 14x16,6x8 --adjoint-tile-pick",
    "stall": "rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY "
             "SQ_WAIT_INST_LDS -d gpurun_out/pmc_stall -o stall --output-format csv -- "
             "python3 bench.py --no-cpu --steps 20 --warmup 0 --only adjoint,d3q19 --two-step-shape 1 "
             "--two-step-3d 14x16,6x8 --adjoint-tile-pick",
    "l2": "rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum -d gpurun_out/pmc_l2 -o l2 --output-format csv -- "
          "python3 bench.py --no-cpu --steps 20 --warmup 0 --only adjoint,d3q19 --two-step-shape 1 "
          "--two-step-3d 14x16,6x8 --adjoint-tile-pick",
}
# vector-ALU issue peak without packed FP32: each SIMD issues one 64-lane
# instruction every 4 clocks (16 lanes per clock), 4 SIMDs per CU, so one
# wave-instruction per CU per clock: 256 CUs x 2.4 GHz
VALU_ISSUE_PEAK = 256 * 2.4e9

# nodes of the 512-instance batch workload (sides 32..512, seed 4)
BATCH_NODES = 44439067

# workload label -> (kernel name prefix in the trace, algorithmic bytes per launch)
PROFILED = {
    "nonlinear2d-1024 f32 two-step": ("k_sweep2<float, float, true, true, 3, ",
                                      bytes_per_node(9, "f32", True) * 1024 * 1024),
    "nonlinear2d-1024 f64 two-step": ("k_sweep2<double, double, true, true, 3, ",
                                      bytes_per_node(9, "f64", True) * 1024 * 1024),
    "nonlinear2d-1024 f32": ("k_sweep<9, float, float, true, true, true, false, 3, false, ",
                             bytes_per_node(9, "f32", True) * 1024 * 1024),
    "nonlinear2d-1024 f64": ("k_sweep<9, double, double, true, true, true, false, 3, false, ",
                             bytes_per_node(9, "f64", True) * 1024 * 1024),
    "d3q19-256 f32": ("k_sweep<19, float, float, true, false, false, true, ",
                      bytes_per_node(19, "f32", False) * 256 ** 3),
    "d3q19-256 f64": ("k_sweep<19, double, double, true, false, false, true, ",
                      bytes_per_node(19, "f64", False) * 256 ** 3),
    "d3q19-256 f32 two-step": ("k_sweep2_3d<float, float, ", bytes_per_node(19, "f32", False) * 256 ** 3),
    "d3q19-256 f64 two-step": ("k_sweep2_3d<double, double, ", bytes_per_node(19, "f64", False) * 256 ** 3),
    "batch-512 f32 two-step": ("k_batch_sweep2<float, float, ", bytes_per_node(9, "f32", False) * BATCH_NODES),
    "adjoint2d-512 f64": ("k_adjoint<9, double, double, true, true, true, false, 3, ",
                          adjoint_bytes_per_node(9, "f64", True) * 512 * 512),
    "adjoint2d-512 f32": ("k_adjoint<9, float, float, true, true, true, false, 3, ",
                          adjoint_bytes_per_node(9, "f32", True) * 512 * 512),
    "adjoint2d-512 f64 pairs": ("k_adjoint2<double, double, true, true, 3, ",
                                adjoint_pair_bytes_per_node(9, "f64", True) * 512 * 512),
    "adjoint2d-512 f32 pairs": ("k_adjoint2<float, float, true, true, 3, ",
                                adjoint_pair_bytes_per_node(9, "f32", True) * 512 * 512),
}


def summarize_profiles(gdir, copy_bytes=1 << 30):
    """Write profiles/pmc_traffic.json, profiles/sweep_kernels_kernel_trace.md
    and profiles/sweep_kernels_hbm_traffic.md from the CSV output of the
    three runs in PROFILE_COMMANDS (under `gdir`).  FETCH_SIZE and WRITE_SIZE
    are scaled by what they read for the library copy kernel moving
    `copy_bytes` each way."""
    import csv
    import statistics as stats

    def kname(n):
        return n.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").strip()

    trace = list(csv.DictReader(open(os.path.join(gdir, "prof_trace", "trace_kernel_stats.csv"))))
    avg_us = {kname(r["Name"]): float(r["AverageNs"]) / 1e3 for r in trace}
    # per-dispatch durations: the median is not moved by the autotuner's trials
    durs = {}
    by_grid = {}   # (kernel, launch grid in threads) -> durations: one kernel may run on several grids
    tpath = os.path.join(gdir, "prof_trace", "trace_kernel_trace.csv")
    if os.path.exists(tpath):
        for r in csv.DictReader(open(tpath)):
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            durs.setdefault(kname(r["Kernel_Name"]), []).append(d)
            grid = tuple(int(r.get(f"Grid_Size_{a}", 1) or 1) for a in "XYZ")
            by_grid.setdefault((kname(r["Kernel_Name"]), grid), []).append(d)
    med_us = {k: stats.median(v) for k, v in durs.items()}

    def counters(sub, stem, cname):
        agg = {}
        for r in csv.DictReader(open(os.path.join(gdir, sub, f"{stem}_counter_collection.csv"))):
            if r.get("Counter_Name") == cname:
                agg.setdefault(kname(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return agg

    fetch = counters("pmc_fetch", "fetch", "FETCH_SIZE")
    write = counters("pmc_write", "write", "WRITE_SIZE")
    copy = next(k for k in fetch if "k_copy16" in k)
    fscale = copy_bytes / (stats.median(fetch[copy]) * 1024)
    wscale = copy_bytes / (stats.median(write[copy]) * 1024)
    out = {"kernel_hash": kernel_hash(), "fetch_scale": fscale, "write_scale": wscale,
           "calibration": f"library copy kernel k_copy16 of {copy_bytes} bytes each way",
           "commands": PROFILE_COMMANDS, "workloads": {}}
    rows = []
    for label, (kn, alg) in PROFILED.items():
        # the variant with the most dispatches (the timed run, not the tuners'
        # trials); the profiled runs pin the two-step tile shape, so the
        # trace and the counter runs time the same kernel
        prefix = kn
        hits = sorted((k for k in fetch if prefix in k and k in write), key=lambda k: -len(fetch[k]))
        if not hits:
            continue
        k = hits[0]
        kn = k.replace("lbm::", "")
        fv, wv = stats.median(fetch[k]), stats.median(write[k])
        t = fv * 1024 * fscale + wv * 1024 * wscale
        tk = sorted((n for n in durs if prefix in n), key=lambda n: -len(durs[n]))
        tr = med_us.get(tk[0]) if tk else None
        if tr is None:
            tr = next((v for n, v in avg_us.items() if kn in n), None)
        if tk and tk[0] != k:
            kn = f"{kn} (counters); {tk[0].replace('lbm::', '')} (trace)"
        out["workloads"][label] = {"kernel": kn, "fetch_kib": fv, "write_kib": wv,
                                   "traffic_bytes_per_launch": t, "algorithmic_bytes_per_launch": alg,
                                   "dispatches": len(fetch[k]), "trace_median_us": tr}
        rows.append((label, kn, len(fetch[k]), fv, wv, t, alg, tr))
    pdir = os.path.join(ROOT, "profiles")
    with open(os.path.join(pdir, "pmc_traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)

    md = ["# HBM traffic of the sweep and adjoint kernels (rocprofv3 counters)", "",
          "Two passes, one counter each, from the repository root with `TMPDIR=/tmp`:", "",
          "    " + PROFILE_COMMANDS["fetch"], "    " + PROFILE_COMMANDS["write"], "",
          "Summarised by `python3 bench.py --summarize-profiles gpurun_out`.", "",
          f"Calibration: the same run executes the library copy kernel `k_copy16`, which reads and "
          f"writes {copy_bytes / 2**30:g} GiB. FETCH_SIZE reads {1 / fscale:.4f} of the bytes it "
          f"fetches (scale x{fscale:.3f}); WRITE_SIZE reads {1 / wscale:.4f} of the bytes it writes "
          f"(scale x{wscale:.3f}).", "",
          "Values are medians per dispatch. Traffic = scaled fetch + scaled write. Algorithmic bytes = "
          "bytes per node update x nodes per launch (a two-step pass: one read and one write of the state "
          "for two updates); the trace column is the median kernel time from the kernel-trace run and the "
          "bandwidth is algorithmic bytes over it.", "",
          "| workload | kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | traffic MB | "
          "algorithmic MB | traffic / algorithmic | trace median us | GB/s (algorithmic) |",
          "|---|---|---|---|---|---|---|---|---|---|"]
    for label, kn, nd, fv, wv, t, alg, tr in rows:
        bw = f"{alg / (tr * 1e-6) / 1e9:.0f}" if tr else "-"
        trs = f"{tr:.2f}" if tr else "-"
        md.append(f"| {label} | `{kn}` | {nd} | {fv:.1f} | {wv:.1f} | {t / 1e6:.2f} | {alg / 1e6:.2f} | "
                  f"{t / alg:.3f} | {trs} | {bw} |")
    md += ["", f"Kernel-source hash `{out['kernel_hash']}`; `bench.py` reports `traffic` only while the "
           "sources hash to it. Machine-readable copy: `pmc_traffic.json`."]
    with open(os.path.join(pdir, "sweep_kernels_hbm_traffic.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")

    tl = ["# Kernel trace: fused sweep, adjoint and batch kernels (MI355X, gfx950)", "",
          "From the repository root with `TMPDIR=/tmp`:", "", "    " + PROFILE_COMMANDS["trace"], "",
          "Summarised by `python3 bench.py --summarize-profiles gpurun_out`. The run includes the "
          "autotuners' trial launches. Template arguments of the sweep:", "",
          "    k_sweep<Q, storage, compute, equal-rate, source, K(phi), walls, polynomial length, non-temporal>",
          "", "| kernel | calls | avg us | median us | min us | max us | share % |", "|---|---|---|---|---|---|---|"]
    for r in trace[:20]:
        med = med_us.get(kname(r["Name"]))
        tl.append(f"| `{kname(r['Name'])[:110]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                  f"{'-' if med is None else f'{med:.2f}'} | "
                  f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                  f"{float(r['Percentage']):.1f} |")
    # one kernel instantiation can serve several workloads (the two-step pass
    # runs the 1024^2 and the 4096^2 grids), so the per-workload figures take
    # the dispatches of the workload's kernel on its most frequent launch grid
    tl += ["", "## Per workload", "",
           "Dispatches of each workload's kernel on its own launch grid (the grid with the most dispatches "
           "of that kernel; tuner trials of the same kernel on the same grid are the same work and are "
           "included). GB/s = algorithmic bytes per launch over the average duration.", "",
           "| workload | kernel | launch grid (threads) | dispatches | avg us | median us | "
           "algorithmic MB per launch | GB/s (avg) | fraction of 8 TB/s |", "|---|---|---|---|---|---|---|---|---|"]
    per_wl = {}
    for label, (prefix, alg) in PROFILED.items():
        groups = sorted(((k, g) for (k, g) in by_grid if prefix in k), key=lambda kg: -len(by_grid[kg]))
        if not groups:
            continue
        k, grid = groups[0]
        v = by_grid[(k, grid)]
        avg, med = stats.mean(v), stats.median(v)
        per_wl[label] = {"kernel": k.replace("lbm::", ""), "grid": grid, "dispatches": len(v),
                         "avg_us": avg, "median_us": med, "gbs_avg": alg / (avg * 1e-6) / 1e9}
        gx = " x ".join(str(x) for x in grid if x > 1) or "1"
        tl.append(f"| {label} | `{k.replace('lbm::', '')}` | {gx} | {len(v)} | {avg:.2f} | {med:.2f} | "
                  f"{alg / 1e6:.2f} | {alg / (avg * 1e-6) / 1e9:.0f} | {alg / (avg * 1e-6) / 8e12:.3f} |")
    # the profiled run's own bench line: its roofline figure for the headline
    # kernel comes from HIP events around the timed region of the same run
    blog = os.path.join(gdir, "trace.log")
    head = "nonlinear2d-1024 f32 two-step"
    if os.path.exists(blog) and head in per_wl:
        line = next((ln for ln in open(blog) if ln.startswith('{"metric"')), None)
        if line:
            rf = json.loads(line)["roofline"]
            per_launch_us = rf["launch_us"]
            w = per_wl[head]
            tl += ["", f"The bench line of this profiled run reports `roofline.launch_us` = {per_launch_us:.2f} us "
                   f"per launch of `{rf['kernel']}` (HIP events over the timed region, median of the samples; "
                   f"`roofline.achieved` = {rf['achieved']:.0f} GB/s at {rf['bytes_per_node']} B per node "
                   f"update x {rf['steps_per_launch']} updates of {rf['nodes_per_launch']} nodes per launch); "
                   f"the trace gives {w['avg_us']:.2f} us average and {w['median_us']:.2f} us median "
                   f"per dispatch of that kernel on the same grid."]
    out["trace_per_workload"] = per_wl
    with open(os.path.join(pdir, "sweep_kernels_kernel_trace.md"), "w") as fh:
        fh.write("\n".join(tl) + "\n")

    vpath = os.path.join(gdir, "pmc_valu", "valu_counter_collection.csv")
    if os.path.exists(vpath):
        vals = {}
        for r in csv.DictReader(open(vpath)):
            vals.setdefault(kname(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
        vl = ["# Instruction issue of the sweep and adjoint kernels (rocprofv3 counters)", "",
              "From the repository root with `TMPDIR=/tmp`:", "", "    " + PROFILE_COMMANDS["valu"], "",
              "Summarised by `python3 bench.py --summarize-profiles gpurun_out`. Medians per dispatch of "
              "the variant with the most dispatches. The issue fraction is SQ_INSTS_VALU (wave-instructions "
              "per dispatch) over the trace median time of the same workload times the vector issue peak: "
              "with packed FP32 off, each SIMD issues one 64-lane instruction every 4 clocks, so a CU issues "
              "one wave-instruction per clock, 256 x 2.4e9 = 6.14e11 per second. Lane-instructions per "
              "update = SQ_INSTS_VALU x 64 / node updates per dispatch.", "",
              "| workload | kernel | waves | VALU | SALU | LDS | VALU lane-instructions per update | "
              "trace median us | VALU issue fraction |", "|---|---|---|---|---|---|---|---|---|"]
        for label, (prefix, alg) in PROFILED.items():
            want = "lbm::" + out["workloads"].get(label, {}).get("kernel", "")
            hits = sorted((k for k in vals if prefix in k and "SQ_INSTS_VALU" in vals[k]),
                          key=lambda k: -len(vals[k]["SQ_INSTS_VALU"]))
            if not hits:
                continue
            k = want if want in vals and "SQ_INSTS_VALU" in vals[want] else hits[0]
            m = {c: stats.median(v) for c, v in vals[k].items()}
            w = out["workloads"].get(label, {})
            tr = w.get("trace_median_us")
            nodes = {"nonlinear2d-1024": 1024 * 1024, "adjoint2d-512": 512 * 512,
                     "d3q19-256": 256 ** 3, "batch-512": BATCH_NODES}[label.split(" ")[0]]
            upd = nodes * (2 if ("two-step" in label or "pairs" in label) else 1)
            frac = m["SQ_INSTS_VALU"] / (tr * 1e-6 * VALU_ISSUE_PEAK) if tr else None
            w.update({"sq_insts_valu": m["SQ_INSTS_VALU"], "valu_issue_fraction": frac})
            vl.append(f"| {label} | `{k.replace('lbm::', '')}` | {m.get('SQ_WAVES', 0):.0f} | "
                      f"{m['SQ_INSTS_VALU']:.0f} | {m.get('SQ_INSTS_SALU', 0):.0f} | {m.get('SQ_INSTS_LDS', 0):.0f} | "
                      f"{m['SQ_INSTS_VALU'] * 64 / upd:.0f} | {'-' if tr is None else f'{tr:.2f}'} | "
                      f"{'-' if frac is None else f'{frac:.2f}'} |")
        vl += ["", f"Kernel-source hash `{out['kernel_hash']}`."]
        with open(os.path.join(pdir, "sweep_kernels_valu_issue.md"), "w") as fh:
            fh.write("\n".join(vl) + "\n")

    def per_kernel(sub, stem):
        path = os.path.join(gdir, sub, f"{stem}_counter_collection.csv")
        if not os.path.exists(path):
            return None
        vals = {}
        for r in csv.DictReader(open(path)):
            vals.setdefault(kname(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
        return vals

    stall, l2 = per_kernel("pmc_stall", "stall"), per_kernel("pmc_l2", "l2")
    if stall:
        sl = ["# Where the waves of the sweep and adjoint kernels wait (rocprofv3 counters)", "",
              "From the repository root with `TMPDIR=/tmp`:", "", "    " + PROFILE_COMMANDS["stall"]]
        if l2:
            sl += ["    " + PROFILE_COMMANDS["l2"]]
        sl += ["", "Summarised by `python3 bench.py --summarize-profiles gpurun_out`. Medians per dispatch of "
               "the variant with the most dispatches (the profiled runs pin the tile shapes, so this is the "
               "timed kernel). The counters are taken as the hardware reports them, summed over the waves "
               "of a dispatch; the ratios compare kernels with each other and are not calibrated shares of "
               "time. `wait` = SQ_WAIT_ANY / SQ_WAVE_CYCLES (waves held at a wait on memory, LDS or a "
               "barrier counter), `issue wait` = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES (waves ready but not "
               "issued), `LDS wait` = SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES; `cycles per wave` = "
               "SQ_WAVE_CYCLES / SQ_WAVES. L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS), summed over the L2 "
               "channels.", "",
               "| workload | kernel | waves | cycles per wave | wait | issue wait | LDS wait | L2 hit |",
               "|---|---|---|---|---|---|---|---|"]
        for label, (prefix, alg) in PROFILED.items():
            want = "lbm::" + out["workloads"].get(label, {}).get("kernel", "")
            hits = sorted((k for k in stall if prefix in k and "SQ_WAVE_CYCLES" in stall[k]),
                          key=lambda k: -len(stall[k]["SQ_WAVE_CYCLES"]))
            if not hits:
                continue
            k = want if want in stall and "SQ_WAVE_CYCLES" in stall[want] else hits[0]
            m = {c: stats.median(v) for c, v in stall[k].items()}
            wc = m["SQ_WAVE_CYCLES"] or 1.0
            hit = None
            if l2 and k in l2 and "TCC_HIT_sum" in l2[k]:
                h, ms = stats.median(l2[k]["TCC_HIT_sum"]), stats.median(l2[k].get("TCC_MISS_sum", [0.0]))
                hit = h / (h + ms) if h + ms else None
            w = out["workloads"].setdefault(label, {})
            w.update({"wait_ratio": m.get("SQ_WAIT_ANY", 0) / wc, "issue_wait_ratio": m.get("SQ_WAIT_INST_ANY", 0) / wc,
                      "lds_wait_ratio": m.get("SQ_WAIT_INST_LDS", 0) / wc, "l2_hit": hit})
            waves = m.get("SQ_WAVES", 0)
            sl.append(f"| {label} | `{k.replace('lbm::', '')}` | {waves:.0f} | "
                      f"{'-' if not waves else f'{wc / waves:.0f}'} | {m.get('SQ_WAIT_ANY', 0) / wc:.2f} | "
                      f"{m.get('SQ_WAIT_INST_ANY', 0) / wc:.2f} | {m.get('SQ_WAIT_INST_LDS', 0) / wc:.2f} | "
                      f"{'-' if hit is None else f'{hit:.2f}'} |")
        sl += ["", f"Kernel-source hash `{out['kernel_hash']}`."]
        with open(os.path.join(pdir, "sweep_kernels_stalls.md"), "w") as fh:
            fh.write("\n".join(sl) + "\n")
        with open(os.path.join(pdir, "pmc_traffic.json"), "w") as fh:
            json.dump(out, fh, indent=1)
        with open(os.path.join(pdir, "pmc_traffic.json"), "w") as fh:
            json.dump(out, fh, indent=1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--quick", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--only", default="",
                    help="comma list of secondary workloads to run: adjoint,d3q19,batch,hbm (default: all)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30,
                    help="size of the plain copy (practical bandwidth, counter calibration)")
    ap.add_argument("--two-step-shape", type=int, default=None,
                    help="after tuning, run two-step passes with this tile shape (lbm_two_step_shape index) "
                         "and the XCD-aware order; the profiles pin 1 with that order, the tuner's usual choice, "
                         "so that every profiled run times the same kernel")
    ap.add_argument("--two-step-3d", metavar="ROWSxWAVES[,...]", default=None,
                    help="run the D3Q19 legs with two steps per pass in the first of these tile shapes that the "
                         "precision has (14x16 FP32/FP16 only, 6x8 all), so that the profiled runs time one kernel "
                         "whatever the tuner picks")
    ap.add_argument("--adjoint-tile-pick", action="store_true",
                    help="keep the adjoint pair's tile shape picked at creation instead of timing every shape, so "
                         "that the profiled runs, whose timings the counters disturb, time the same kernel")
    ap.add_argument("--summarize-profiles", metavar="DIR", default=None,
                    help="write the profiles/ summaries from rocprofv3 output under DIR and exit (no GPU)")
    args = ap.parse_args()
    if args.summarize_profiles:
        out = summarize_profiles(args.summarize_profiles, args.copy_bytes)
        print(json.dumps({k: v["traffic_bytes_per_launch"] / v["algorithmic_bytes_per_launch"]
                          for k, v in out["workloads"].items()}))
        return
    global TWO_STEP_SHAPE, TWO_STEP_3D, ADJ_TILE_TRIAL
    TWO_STEP_SHAPE = args.two_step_shape
    ADJ_TILE_TRIAL = not args.adjoint_tile_pick
    if args.two_step_3d:
        TWO_STEP_3D = [tuple(int(v) for v in sh.split("x")) for sh in args.two_step_3d.lower().split(",")]
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU (the library has no multi-GPU path); run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_1603_09577_amd import lbm, workloads as W

    torch.cuda.set_device(0)
    K, Wm = args.steps, args.warmup
    spec32, phi0, _ = W.nonlinear_2d(1024, precision="f32")
    spec64, _, _ = W.nonlinear_2d(1024, precision="f64")

    head, sim32, phi32 = run_forward(torch, lbm, spec32, phi0, K, Wm, "nonlinear2d-1024 f32")
    single32, s1, _ = run_forward(torch, lbm, spec32, phi0, K, Wm, "nonlinear2d-1024 f32 single", two_step=False)
    del s1
    print(f"# nonlinear2d-1024 f32: {head['mlups']:.0f} MLUPS, {head['achieved_gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    f64, sim64, phi64 = run_forward(torch, lbm, spec64, phi0, K, Wm, "nonlinear2d-1024 f64")
    print(f"# nonlinear2d-1024 f64: {f64['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    # both ran warmup + K steps from the same phi0: error of FP32 storage
    # against the FP64 path after the same number of steps
    err32 = float(torch.linalg.norm(phi32 - phi64) / torch.linalg.norm(phi64))
    spec16, _, _ = W.nonlinear_2d(1024, precision="f16")
    f16, sim16, phi16 = run_forward(torch, lbm, spec16, phi0, K, Wm, "nonlinear2d-1024 f16")
    err16 = float(torch.linalg.norm(phi16 - phi64) / torch.linalg.norm(phi64))
    del sim16, phi16
    print(f"# nonlinear2d-1024 f16: {f16['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    diag = time_diagnostics(torch, sim32, head["ms_per_step"])
    # the paper's default source scheme (Remark II, Scheme B) on the same
    # workload: Eq. 35 is then a quadratic in phi, solved at every node
    schemeb = {}
    for prec, sp in (("f32", spec32), ("f64", spec64)):
        rb, sb, phib = run_forward(torch, lbm, dict(sp, scheme="B"), phi0, K, Wm, f"nonlinear2d-1024 {prec} scheme B")
        schemeb[prec] = {"mlups": rb["mlups"], "ms_per_step": rb["ms_per_step"], "achieved_gbs": rb["achieved_gbs"],
                         "hbm_frac": rb["hbm_frac"], "bytes_per_node": rb["bytes_per_node"], "tuner": rb["tuner"],
                         "nonfinite": rb["nonfinite"]}
        del sb, phib
    print(f"# nonlinear2d-1024 scheme B: f32 {schemeb['f32']['mlups']:.0f} / f64 {schemeb['f64']['mlups']:.0f} MLUPS",
          file=sys.stderr, flush=True)

    extra = {}
    only = set(w for w in args.only.split(",") if w) or {"adjoint", "d3q19", "batch", "hbm"}
    if args.quick:
        only = set()
    if "adjoint" in only:
        spec5, p5, _, _ = W.adjoint_2d()
        extra["adjoint_f64"] = run_adjoint(torch, lbm, spec5, p5, 200, 20, "adjoint2d-512 f64")
        spec5f, _, _, _ = W.adjoint_2d(precision="f32")
        extra["adjoint_f32"] = run_adjoint(torch, lbm, spec5f, p5, 200, 20, "adjoint2d-512 f32")
        print(f"# adjoint f64 {extra['adjoint_f64']['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        # the same physics on 1024^2: four rounds of workgroups instead of one,
        # where the two-sweep launches are no longer held to one round's phases
        big = {}
        for prec in ("f64", "f32"):
            specb, pb, _, _ = W.adjoint_2d(1024, precision=prec)
            big[prec] = run_adjoint(torch, lbm, specb, pb, 100, 10, f"adjoint2d-1024 {prec}")
        extra["adjoint_1024"] = dict(big, note="not the 512^2 adjoint workload: the same physics on 1024^2, "
                                               "reported beside it")
        torch.cuda.empty_cache()
    if "d3q19" in only:
        spec3, p3, _ = W.d3q19_walls(precision="f32")
        d3, s3, _ = run_forward(torch, lbm, spec3, p3, 200, 20, "d3q19-256 f32")
        del s3
        extra["d3q19_f32"] = d3
        spec3d, _, _ = W.d3q19_walls(precision="f64")
        d3d, s3d, _ = run_forward(torch, lbm, spec3d, p3, 100, 10, "d3q19-256 f64")
        del s3d
        extra["d3q19_f64"] = d3d
        print(f"# d3q19-256 f32 {d3['mlups']:.0f} / f64 {d3d['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        # reversed sweep of the same D3Q19 workload (walls, full K)
        extra["adjoint_d3q19_f32"] = run_adjoint(torch, lbm, spec3, p3, 40, 4, "adjoint d3q19-256 f32")
        torch.cuda.empty_cache()
        extra["adjoint_d3q19_f64"] = run_adjoint(torch, lbm, spec3d, p3, 20, 2, "adjoint d3q19-256 f64")
        print(f"# adjoint d3q19-256 f32 {extra['adjoint_d3q19_f32']['mlups']:.0f} / "
              f"f64 {extra['adjoint_d3q19_f64']['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if "batch" in only:
        extra["batch_f32"] = run_batch(torch, lbm, W, 1000 if args.steps >= 1000 else args.steps)
    if "hbm" in only:
        # the headline grid's state (79 MB) fits in the 256 MB Infinity Cache;
        # the same workload at 4096^2 (1.2 GB) is bound by HBM proper
        spec4, _, _ = W.nonlinear_2d(4096, precision="f32")
        p4 = W.noise_field((4096, 4096), 2)
        big, sb, _ = run_forward(torch, lbm, spec4, p4, 200, 64, "nonlinear2d-4096 f32")
        del sb
        one, s1, _ = run_forward(torch, lbm, spec4, p4, 200, 64, "nonlinear2d-4096 f32 single", two_step=False)
        del s1
        extra["hbm_resident_4096_f32"] = {
            "mlups": big["mlups"], "two_step": big["two_step"], "tile_rows": big["tile_rows"],
            "per_update_hbm_frac": big["per_update_hbm_frac"], "hbm_frac": big["hbm_frac"],
            "single_sweep_mlups": one["mlups"], "single_sweep_hbm_frac": one["hbm_frac"],
            "state_bytes": 2 * 9 * 4 * 4096 * 4096 + 4 * 4096 * 4096}
        print(f"# nonlinear2d-4096 f32: {big['mlups']:.0f} MLUPS (single sweep {one['mlups']:.0f})",
              file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        print(f"# batch {extra['batch_f32']['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    extra["copy_probe"] = copy_probe(torch, lbm, args.copy_bytes)

    cpu = None
    if not args.no_cpu:
        cpu, phi_cpu, ncpu = cpu_baseline(spec64, phi0)
        # same number of steps on the GPU for an oracle comparison of both paths
        errs = {}
        for name, sp in (("f64", spec64), ("f32", spec32)):
            s = lbm.Lbm(sp).init(phi0)
            s.step(ncpu)
            ph = s.phi().cpu().numpy()
            errs[name] = float(np.linalg.norm(ph - phi_cpu) / np.linalg.norm(phi_cpu))
        extra["rel_l2_vs_oracle"] = {"steps": ncpu, **errs}

    per = head["ms_per_step"] / 1e3
    if head["two_step"]:
        m = re.match(r"(\d+) rows x (\d+) waves", head["tile_rows"] or "")
        prof = profile_entry("nonlinear2d-1024 f32 two-step",
                             f"k_sweep2<float, float, true, true, 3, {m.group(1)}, {m.group(2)}," if m else "?")
    else:
        prof = profile_entry("nonlinear2d-1024 f32")
    traffic = prof.get("traffic_bytes_per_launch") if prof else None
    line = {
        "metric": METRIC,
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "D2Q9 MRT nonlinear anisotropic CDE with Scheme-A source, periodic 1024x1024, "
                        "FP32 offset storage (headline); FP64 storage beside it",
            "lattice": "D2Q9", "grid": [1024, 1024], "storage": "f32 offsets f - w phi_ref",
            "scheme": "A", "grid_spacing": W.NONLINEAR_DX, "time_step": W.NONLINEAR_DT,
        },
        "roofline": {
            # algorithmic bytes per launch = bytes per node update (one read and
            # one write of every population plus the phi history) x the node
            # updates one launch performs (2 N for a two-step pass), over the
            # launch time
            "bound": "hbm", "achieved": head["per_update_hbm_frac"] * PEAK_HBM_GBS, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": head["per_update_hbm_frac"], "traffic": traffic,
            "frac_own_bytes": head["hbm_frac"],
            "note": ("frac counts the bytes one sweep per step would move; a two-step pass moves the "
                     "state through HBM once per two updates (frac_own_bytes: its own bytes over its time), "
                     "and the 79 MB state also fits the 256 MB Infinity Cache, so frac can exceed 1. "
                     "HBM-resident evidence: hbm_resident_4096_f32 and d3q19_f32/f64"
                     if head["two_step"] else
                     "the 79 MB state fits the 256 MB Infinity Cache; HBM-resident evidence: "
                     "hbm_resident_4096_f32 and d3q19_f32/f64"),
            "kernel": (f"k_sweep2<float, float, SRC, KVAR, 3-term polynomials, {head['tile_rows']}> "
                       "(two steps per pass)"
                       if head["two_step"] else "k_sweep<9, float, float, EQR, SRC, KVAR, !WALL, 3-term polynomials>"),
            "bytes_per_node": head["bytes_per_node"], "nodes_per_launch": head["nodes"],
            "steps_per_launch": 2 if head["two_step"] else 1,
            "launch_us": head["ms_per_step"] * (2 if head["two_step"] else 1) * 1e3,
            # measured vector-instruction issue of the same kernel (rocprofv3
            # SQ_INSTS_VALU over its trace time) against 6.14e11 wave-instructions/s
            # (256 CUs x 2.4 GHz, one 64-lane instruction per CU per clock without packed FP32)
            "valu_issue_frac": prof.get("valu_issue_fraction") if prof else None,
        },
        "single_step": {"mlups": single32["mlups"], "ms_per_step": single32["ms_per_step"],
                        "achieved_gbs": single32["achieved_gbs"], "hbm_frac": single32["hbm_frac"]},
        "cpu_baseline": cpu,
        "tuner": head["tuner"],
        "timing": head["timing"],
        "fp64": {"mlups": f64["mlups"], "ms_per_step": f64["ms_per_step"], "two_step": f64["two_step"],
                 "tile_rows": f64["tile_rows"], "achieved_gbs": f64["achieved_gbs"], "hbm_frac": f64["hbm_frac"],
                 "per_update_hbm_frac": f64["per_update_hbm_frac"]},
        "fp32_vs_fp64_mlups": head["mlups"] / f64["mlups"],
        "fp32_rel_l2_vs_fp64_after_run": err32,
        "fp16": {"mlups": f16["mlups"], "ms_per_step": f16["ms_per_step"], "two_step": f16["two_step"],
                 "tile_rows": f16["tile_rows"], "achieved_gbs": f16["achieved_gbs"],
                 "hbm_frac": f16["hbm_frac"], "rel_l2_vs_fp64_after_run": err16,
                 "storage": "f16 offsets, re-centred every 256 steps"},
        "nonfinite": head["nonfinite"] + f64["nonfinite"] + f16["nonfinite"],
        "diagnostics_fp64": diag,
        "scheme_b": dict(schemeb, note="Scheme B (no phi history: bytes per node without it); the tuned "
                                       "3-term kernels with the closed-form root of Eq. 35 per node; "
                                       "hbm_frac is per launch (a two-step pass: its own bytes)"),
        **extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
