"""Benchmark: Floquet steps/s of the BP-gauged simple-update kicked Ising simulation.

Workload: the 127-qubit Eagle heavy-hex lattice (144 edges, greedy 3-colouring), chi = 64,
theta_h = the first of 8 angles drawn uniformly in [0, pi/2] with numpy default_rng(2306),
BP tolerance 1e-12.  One bench "step" is one whole Floquet step of the resident state: X
rotations, the three simple-update gate layers, BP to convergence, <Z_v> on every site.
The first --warmup steps (default 6: bonds saturate at chi = 64 after 6 steps) are untimed; the
next --steps steps are timed, so the default run is steps 7..20 of the 20-step circuit.

The JSON line also carries:
  roofline     : the kernel with the most time in the step, chosen from three profiled kernels by
                 their HIP-event-timed launch durations (every 7th launch of each kernel in the
                 timed window): gemm_kernel (tiled GEMM), gemm_stream_kernel (the leg absorptions of BP
                 and the gate layers) and bp_close_kernel (the BP messages: per degree-3 site a
                 pair closing of two absorbed copies of its tensor, 8 chi^3 (chi + 1) flops and
                 2 x 2 chi^3 x 16 bytes per message; per degree-2 site the absorption and closing
                 fused).  Algorithmic flops (8 per complex multiply-add, a Hermitian output counted
                 by its distinct entries) and algorithmic bytes (operands read once, outputs
                 written once) of the sampled launches over their summed durations; bound "mfma"
                 (TFLOP/s against the FP64 dense peak 78.6) when the flops per byte reach the
                 ridge point 78.6 / 8, else "hbm" (GB/s against 8 TB/s).  traffic = HBM bytes per
                 launch from the committed rocprofv3 counter summary of that kernel (null once its
                 source has changed); achievable = measured roofs on this GPU (MFMA chains
                 without memory traffic, a 1 GiB copy) and frac_of_achievable against them (MFMA:
                 x 4/3, the 3M complex product issuing 3/4 of the algorithmic real flops).
                 other_kernels: the same for the other two.
  mixed        : the same window in mixed precision (BP tolerance MIXED_TOL), with max / median
                 |<Z>| difference to FP64, the FP64 mode at the same tolerance (the FP32
                 arithmetic's own gain) and the roofline of its dominant FP32 kernel as above
                 (against the FP32 MFMA peak 157.3 TFLOP/s or HBM).
  config1      : the chi = 32 configuration: nine theta_h, 20 steps each, FP64, the lattice-average
                 magnetisation after every step.
  chi128       : the same workload at chi = 128, steps 8..10 (FP64).
  precision_form, precision_form_chi128 (opt-in): the eight seeded theta_h with 64 seeded Pauli
                 strings each, 20 steps, FP64 and mixed, the mixed run's error in every <Z> and
                 string; at chi = 64 and (opt-in) chi = 128.
  weight10     : the paper's weight-10 observable after 5 steps at the eight theta_h, measured by
                 the extended time evolution (5 steps, then 5 steps of U(pi/2)^dagger, <Z_13>).
  theta_batch  : the eight theta_h values of the workload (20 steps each) solved together, one
                 serving slot each: aggregate Floquet steps/s.
  serving      : the seeded request stream, 256 requests by default (see serving_bench).
  cpu_baseline : the FP64 oracle on this host's cores, BLAS at all cores and at one thread, as
                 Floquet steps/s of the same workload from a bounded per-unit sample (gates of each
                 edge type, message updates and <Z> of sites of each degree on a seeded random
                 chi = 64 state, scaled by their counts per step, with the BP sweep count measured
                 here); --cpu-config1 adds a whole oracle run of the chi = 32 configuration.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# every 7th launch of each profiled kernel in the timed window is bracketed by HIP events (an
# event pair on every launch would slow the timed steps by ~4%)
PROFILE_STRIDE = 7
HBM_PEAK_GBPS = 8000.0
GEMM_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "gemm_kernel_hbm_traffic.md")
STREAM_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "gemm_stream_kernel_hbm_traffic.md")
CLOSE_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "bp_close_kernel_hbm_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2306_14887_amd", "csrc", "hip_backend.hip")
# the source spans (kernel, host launch code) that the recorded counters belong to
GEMM_SPANS = (("constexpr int BM = 64, BN = 64, BK = 16, PAD = 1;",
               "// Twelve independent MFMA accumulation chains per wave"),
              ("  void gemm(const GemmDesc &d, const double *const *A",
               "  void bp_close(const BpCloseDesc &d,"))
CLOSE_SPANS = (("// Fused BP closing at chi = CH = 64 or 32 (BpCloseDesc).",
                "// Hermitian Jacobi eigensolver"),
               ("  void bp_close(const BpCloseDesc &d,", "  void *splitk_ws(size_t need) {"))


def kernel_source_hash(spans) -> str:
    import hashlib
    src = open(KERNEL_SOURCE).read()
    return hashlib.sha256("".join(src[src.index(a):src.index(b)] for a, b in spans)
                          .encode()).hexdigest()


def recorded_traffic(profile: str, spans):
    """HBM bytes per launch from a committed FETCH_SIZE / WRITE_SIZE summary, or None when the
    kernel or its launch code has changed since those counters were taken (their hash is
    recorded)."""
    try:
        rec = {}
        for line in open(profile):
            if ":" in line:
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        if rec.get("kernel_source_sha256") != kernel_source_hash(spans):
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


# the three profiled kernels: (name, committed HBM-traffic summary, source spans of its hash)
PROFILED = {0: ("gemm_kernel", GEMM_TRAFFIC_PROFILE, GEMM_SPANS),
            1: ("bp_close_kernel", CLOSE_TRAFFIC_PROFILE, CLOSE_SPANS),
            2: ("gemm_stream_kernel", STREAM_TRAFFIC_PROFILE, GEMM_SPANS)}


def kernel_roofline(p: dict, kernel: int, prec: int, peaks: dict | None) -> dict:
    """Roofline of one profiled kernel's bracketed launches: algorithmic flops and bytes over their
    summed HIP-event durations.  Bound by the MFMA when its flops per byte reach the ridge point of
    the dense peak over the 8 TB/s HBM peak, else by HBM."""
    name, prof_path, spans = PROFILED[kernel]
    peak_tf = FP32_PEAK_TFLOPS if prec else FP64_PEAK_TFLOPS
    sec = p["ms"] * 1e-3
    tf = p["flops"] / sec / 1e12 if sec > 0 else 0.0
    gbps = p["bytes"] / sec / 1e9 if sec > 0 else 0.0
    intensity = p["flops"] / p["bytes"] if p["bytes"] > 0 else float("inf")
    ridge = peak_tf * 1e12 / (HBM_PEAK_GBPS * 1e9)
    mfma = intensity >= ridge
    r = {"bound": "mfma" if mfma else "hbm",
         "kernel": f"{name}<{'float' if prec else 'double'}>",
         "achieved": tf if mfma else gbps, "peak": peak_tf if mfma else HBM_PEAK_GBPS,
         "unit": "TFLOP/s" if mfma else "GB/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r.update({"tflops": tf, "gbps": gbps, "flops_per_byte": intensity,
              "ridge_flops_per_byte": ridge, "launches": p["launches"],
              "avg_launch_ms": p["ms"] / max(1, p["launches"]), "ms_sampled": p["ms"],
              "traffic": recorded_traffic(prof_path, spans) if not prec else None,
              "traffic_unit": "bytes per launch (HBM, calibrated)",
              "algorithmic_bytes_per_launch": p["bytes"] / max(1, p["launches"])})
    if peaks:
        if mfma and peaks.get("mfma_f64_tflops") and not prec:
            # the 3M complex product issues 3/4 of the algorithmic real flops
            r["frac_of_achievable"] = tf / (peaks["mfma_f64_tflops"] * 4.0 / 3.0)
        elif mfma and peaks.get("mfma_f32_tflops") and prec:
            r["frac_of_achievable"] = tf / (peaks["mfma_f32_tflops"] * 4.0 / 3.0)
        elif not mfma and peaks.get("hbm_copy_gbps"):
            r["frac_of_achievable"] = gbps / peaks["hbm_copy_gbps"]
    return r


def dominant_roofline(prof: dict, prec: int, peaks: dict | None) -> dict:
    """The roofline of the kernel with the most time (its average sampled launch duration times
    all its launches), the other kernels beside it."""
    rl = {k: kernel_roofline(prof[(k, prec)], k, prec, peaks) for k in PROFILED}
    for k in rl:
        rl[k]["all_launches"] = prof[(k, prec)]["all_launches"]
        rl[k]["est_total_ms"] = rl[k]["avg_launch_ms"] * prof[(k, prec)]["all_launches"]
    dom = max(rl, key=lambda k: rl[k]["est_total_ms"])
    out = dict(rl[dom])
    out["other_kernels"] = {rl[k]["kernel"]: rl[k] for k in rl if k != dom}
    return out


def _cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:
        n = os.cpu_count() or 1
    for var in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS"):
        v = os.environ.get(var)
        if v and v.isdigit():
            n = min(n, int(v))
    return n


def _oracle_step_time(lat, chi: int, theta: float, sweeps: float, samples: int = 6):
    """The FP64 oracle's time for one Floquet step of the workload, from per-unit timings on a
    seeded random full-bond state: the X rotations (all sites), `samples` gates of each edge type
    (by the degrees of the endpoints), the message updates of `samples` sites of each degree (all
    messages they send) and <Z> of `samples` sites of each degree, each unit scaled by its count
    per step; BP enters with the measured number of sweeps."""
    import numpy as np

    from oracle import bp_tns as O

    rng = np.random.default_rng(7)
    net = O.Network(lat.n_sites, lat.edges, lat.colour)
    for v in range(net.n):
        d = len(net.nb[v])
        shape = (2,) + (chi,) * d
        net.T[v] = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / chi
    for k in list(net.M):
        X = rng.standard_normal((chi, chi)) + 1j * rng.standard_normal((chi, chi))
        M = X @ X.conj().T
        net.M[k] = M / np.trace(M)
    deg = lat.degrees()
    opt = O.Options(chi=chi)
    t0 = time.perf_counter()
    net.apply_rx(theta)
    t_rx = time.perf_counter() - t0
    kinds = {}
    for u, v in lat.edges.tolist():
        kinds.setdefault(tuple(sorted((int(deg[u]), int(deg[v])))), []).append((u, v))
    t_gates = 0.0
    for es in kinds.values():
        t0 = time.perf_counter()
        for u, v in es[:samples]:
            net.simple_update(u, v, opt)
        t_gates += len(es) * (time.perf_counter() - t0) / min(samples, len(es))
    t_sweep = t_obs = 0.0
    for d in sorted(set(deg.tolist())):
        sites = [v for v in range(lat.n_sites) if deg[v] == d]
        t0 = time.perf_counter()
        for v in sites[:samples]:
            for w in net.nb[v]:
                net.message(v, w, net.M)
        t_sweep += len(sites) * (time.perf_counter() - t0) / min(samples, len(sites))
        t0 = time.perf_counter()
        for v in sites[:samples]:
            net.expect_site(v, 3)
        t_obs += len(sites) * (time.perf_counter() - t0) / min(samples, len(sites))
    return {"rx_s": t_rx, "gates_s": t_gates, "bp_sweep_s": t_sweep, "observe_s": t_obs,
            "step_s": t_rx + t_gates + sweeps * t_sweep + t_obs}


def cpu_baseline(lat, chi: int, theta: float, bp_sweeps_per_step: float) -> dict:
    """The FP64 oracle on this host's cores (BLAS at all cores, and at one thread), as Floquet
    steps/s of the benchmark workload estimated from a bounded per-unit sample."""
    import threadpoolctl

    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = "unknown BLAS"
    try:
        info = [i for i in threadpoolctl.threadpool_info() if i.get("user_api") == "blas"]
        if info:
            blas = ", ".join(f"{i.get('internal_api')} {i.get('version')} "
                             f"({i.get('num_threads')} threads)" for i in info)
    except Exception:
        pass
    t0 = time.perf_counter()
    allc = _oracle_step_time(lat, chi, theta, bp_sweeps_per_step)
    with threadpoolctl.threadpool_limits(1):
        one = _oracle_step_time(lat, chi, theta, bp_sweeps_per_step)
    wall = time.perf_counter() - t0
    return {
        "value": 1.0 / allc["step_s"], "unit": "Floquet steps/s", "cores": _cores(),
        "kind": "oracle", "cpu": model, "blas": blas,
        "one_thread": {"value": 1.0 / one["step_s"], "cores": 1, "phases_s": one},
        "phases_s": allc,
        "sample": (f"FP64 numpy oracle, 127-qubit lattice, seeded random chi={chi} state: the X "
                   f"rotations, 6 gates of each edge type, the messages of 6 sites and <Z> of 6 "
                   f"sites of each degree, each scaled by its count per step, with "
                   f"{bp_sweeps_per_step:.1f} BP sweeps per step (measured on the GPU); BLAS at "
                   f"all cores, then at one thread ({wall:.1f} s in all)"),
    }


MIXED_TOL = 1e-10  # mixed-mode BP tolerance: the stated bound (|<Z> - FP64| <= 1e-5) holds there


def serving_bench(n: int, slots: int) -> dict:
    """Serving workload: ``n`` requests from the seeded serving stream (lattices (3,9), (5,11),
    (7,15); theta ~ U[0, pi/2]; depth ~ U{1..20}; chi ~ U{8,16,32,64}).
    1. comparator: every request solved one at a time in plain FP64 (BP tolerance 1e-12); its
       latency under the arrivals of step 3 follows from the measured service times by the FIFO
       queue of one server (finish = max(arrival, previous finish) + service: one solve at a
       time on an idle device);
    2. capacity: all requests submitted at once to the serving slots in mixed precision (FP32 BP,
       FP64 polish to MIXED_TOL): solves/s = n / makespan, with cross-request packing (the library
       default: chi <= 16, up to 16 per pack, requests that would otherwise wait) and without;
       and the same capacity run served in FP64 on the same slots;
    3. latency: the served mixed run with Poisson arrivals at 0.5, 1 and 2 times the comparator's
       solve rate (p50 / p99 of finish - arrival; the top-level latency keys are the 2x run), and
       the served FP64 run at 2x.
    Reports the largest |<Z>| deviation of a served result from its FP64 solve alone."""
    import numpy as np

    from paper_2306_14887_amd import bpki
    from paper_2306_14887_amd import lattice as L

    reqs = L.serving_requests(n, seed=0, rate=1.0)
    lats = {}
    specs64, specsmx = [], []
    for r in reqs:
        key = (r.rows, r.row_len)
        if key not in lats:
            lats[key] = L.heavy_hex(*key)
        specs64.append(bpki.spec_from_lattice(lats[key], r.theta, r.depth, r.chi))
        specsmx.append(bpki.spec_from_lattice(lats[key], r.theta, r.depth, r.chi,
                                              precision=bpki.BPKI_FP32, bp_tol=MIXED_TOL))
    ref = []
    with bpki.Context(0) as ctx:
        t0 = time.perf_counter()
        service = []
        for s in specs64:
            a = time.perf_counter()
            ref.append(ctx.solve(s)["z"])
            service.append(time.perf_counter() - a)
        t_seq = time.perf_counter() - t0
    service = np.array(service)
    rate = n / t_seq
    print(f"serving: sequential FP64 {rate:.2f} solves/s", file=sys.stderr, flush=True)

    def served(specs, arrivals, pack=True):
        with bpki.Context(0) as ctx:
            ctx.serving_config(slots)
            if not pack:
                ctx.serving_packing(1)
            tickets = [None] * n
            t0 = time.perf_counter()
            for i, s in enumerate(specs):
                wait = arrivals[i] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                tickets[i] = ctx.submit(s)
            while not all(t.poll() for t in tickets):
                time.sleep(0.0005)
            times = np.array([t.times() for t in tickets])
            packs = np.array([t.pack_size() for t in tickets])
            outs = [t.wait() for t in tickets]
        err = max(float(np.abs(o["z"] - z).max()) for o, z in zip(outs, ref))
        return times, err, packs

    def lat_ms(times):
        lat = times[:, 2] - times[:, 0]
        return 1e3 * float(np.percentile(lat, 50)), 1e3 * float(np.percentile(lat, 99))

    def sequential_latency(arrivals):
        fin, prev = np.empty(n), 0.0
        for i in range(n):
            prev = max(arrivals[i], prev) + service[i]
            fin[i] = prev
        lat = fin - arrivals
        return 1e3 * float(np.percentile(lat, 50)), 1e3 * float(np.percentile(lat, 99))

    zero = np.zeros(n)
    times_sat, err_sat, packs_sat = served(specsmx, zero)
    cap = n / (times_sat[:, 2].max() - times_sat[:, 0].min())
    times_np, err_np, _ = served(specsmx, zero, pack=False)
    cap_np = n / (times_np[:, 2].max() - times_np[:, 0].min())
    times_64, err_64, _ = served(specs64, zero)
    cap_64 = n / (times_64[:, 2].max() - times_64[:, 0].min())
    print(f"serving: capacity mixed {cap:.2f}, FP64 {cap_64:.2f} solves/s", file=sys.stderr,
          flush=True)
    gaps = np.array([r.arrival for r in reqs])
    sweep, errs = [], []
    arrivals = gaps * 0
    for f in (0.5, 1.0, 2.0):
        lam = f * rate
        arrivals = gaps / gaps[-1] * (n / lam) if n > 1 else gaps * 0
        times, err, packs = served(specsmx, arrivals)
        errs.append(err)
        p50, p99 = lat_ms(times)
        s50, s99 = sequential_latency(arrivals)
        sweep.append({"rate_factor": f, "arrival_rate_per_s": lam, "p50_ms": p50, "p99_ms": p99,
                      "requests_packed": int((packs > 1).sum()),
                      "sequential_fp64_p50_ms": s50, "sequential_fp64_p99_ms": s99})
        print(f"serving: poisson {f}x p99 {p99:.0f} ms (sequential FP64 {s99:.0f} ms)",
              file=sys.stderr, flush=True)
    times_64p, err_64p, _ = served(specs64, arrivals)
    f50, f99 = lat_ms(times_64p)
    return {
        "requests": n, "slots": slots, "mixed_bp_tol": MIXED_TOL,
        "served_mixed_solves_per_s": cap,
        "served_mixed_solves_per_s_without_packing": cap_np,
        "served_fp64_solves_per_s": cap_64,
        "requests_packed_capacity_run": int((packs_sat > 1).sum()),
        "mean_pack_size_capacity_run": float(packs_sat.mean()),
        "requests_packed_poisson_run": sweep[-1]["requests_packed"],
        "sequential_fp64_solves_per_s": rate,
        "speedup_vs_sequential_fp64": cap / rate,
        "speedup_vs_served_fp64": cap / cap_64,
        "poisson_arrival_rate_per_s": sweep[-1]["arrival_rate_per_s"],
        "served_p50_ms": sweep[-1]["p50_ms"], "served_p99_ms": sweep[-1]["p99_ms"],
        "sequential_fp64_p50_ms": sweep[-1]["sequential_fp64_p50_ms"],
        "sequential_fp64_p99_ms": sweep[-1]["sequential_fp64_p99_ms"],
        "sequential_latency": "FIFO queue of one server fed with the measured FP64 service times",
        "served_fp64_p50_ms": f50, "served_fp64_p99_ms": f99,
        "poisson_sweep": sweep,
        "max_abs_dz_vs_fp64": max(errs + [err_sat, err_np]),
        "max_abs_dz_served_fp64_vs_alone": max(err_64, err_64p),
    }


def _window(lat, theta, chi, warmup, steps, precision, tol, profile=False):
    """Steps warmup+1 .. warmup+steps of the workload in one session: steps/s, sweeps, <Z> rows
    and (profile) the sampled GEMM launches of each arithmetic."""
    import numpy as np

    from paper_2306_14887_amd import bpki

    with bpki.Context(0) as ctx:
        sess = ctx.session(bpki.spec_from_lattice(lat, theta, warmup + steps, chi,
                                                  precision=precision, bp_tol=tol))
        for _ in range(warmup):
            sess.step(observe=True)
        if profile:
            sess.profile(True, stride=PROFILE_STRIDE)
        iters, zs = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            r = sess.step(observe=True)
            iters.append(r["bp_iters"])
            zs.append(r["z"])
        wall = time.perf_counter() - t0
        prof = ({(k, q): sess.profile_read_kernel(k, q) for k in PROFILED for q in (0, 1)}
                if profile else None)
        sess.close()
    return steps / wall, float(np.mean(iters)), np.array(zs), prof


def mixed_window(lat, theta, chi, warmup, steps) -> dict:
    """The same steps in mixed precision (FP32 BP on FP32 copies of the tensors until the FP32
    rounding level, FP64 sweeps to MIXED_TOL), the FP64 mode at the same BP tolerance (so the
    FP32 arithmetic's own gain is separated from the tolerance), and the roofline of the FP32
    GEMM launches against the FP32 MFMA peak."""
    from paper_2306_14887_amd import bpki

    v32, it32, z32, prof = _window(lat, theta, chi, warmup, steps, bpki.BPKI_FP32, MIXED_TOL,
                                   profile=True)
    v64, it64, _, _ = _window(lat, theta, chi, warmup, steps, bpki.BPKI_FP64, MIXED_TOL)
    rl32 = dominant_roofline(prof, 1, None)
    rl32["fp64_launches_of_the_window"] = {
        kernel_roofline(prof[(k, 0)], k, 0, None)["kernel"]: kernel_roofline(prof[(k, 0)], k, 0, None)
        for k in PROFILED}
    return {"value": v32, "unit": "Floquet steps/s", "ms_per_step": 1e3 / v32,
            "bp_sweeps_per_step": it32, "bp_tol": MIXED_TOL,
            "dtype": "c64 BP contractions on c64 copies until the FP32 level, then c128",
            "fp64_same_tol": {"value": v64, "bp_sweeps_per_step": it64,
                              "mixed_speedup": v32 / v64},
            "roofline": rl32,
            "_z": z32}


def config1(chi: int = 32, depth: int = 20) -> dict:
    """The 127-qubit lattice at chi = 32, 20 Floquet steps, FP64, at the nine theta_h of the
    configuration (0, 0.2, ..., 1.4, pi/2): the lattice-average magnetisation after every step
    (Fig. 3a's quantity) and the steps/s of each run."""
    import numpy as np

    from paper_2306_14887_amd import bpki
    from paper_2306_14887_amd import lattice as L

    lat = L.eagle()
    runs = []
    with bpki.Context(0) as ctx:
        for th in L.theta_grid_config1():
            t0 = time.perf_counter()
            r = ctx.solve(bpki.spec_from_lattice(lat, th, depth, chi))
            wall = time.perf_counter() - t0
            runs.append({"theta_h": th, "steps_per_s": depth / wall,
                         "bp_sweeps": int(np.sum(r["bp_iters"])),
                         "magnetisation_per_step": [round(float(x), 8)
                                                    for x in r["z"].mean(axis=1)],
                         "z62_last_step": float(r["z"][-1][62])})
    return {"lattice": "127-qubit heavy hex", "chi": chi, "steps": depth, "precision": "fp64",
            "runs": runs,
            "aggregate_steps_per_s": len(runs) * depth / sum(depth / r["steps_per_s"]
                                                             for r in runs)}


def achievable_peaks(ctx) -> dict:
    """Micro-benchmarks of the two roofs on this GPU: independent MFMA chains with no memory
    traffic (the library's probe) and a 1 GiB device-to-device copy (read + write)."""
    out = {"mfma_f64_tflops": ctx.test_mfma_rate(0, 1024, 2000),
           "mfma_f32_tflops": ctx.test_mfma_rate(1, 1024, 2000)}
    try:
        import torch
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(8):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        out["hbm_copy_gbps"] = 8 * 2 * n * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del src, dst
        torch.cuda.empty_cache()
    except Exception:
        out["hbm_copy_gbps"] = None
    return out


def weight10(lat, chi: int) -> dict:
    """The paper's weight-10 observable X13,29,31 Y9,30 Z8,12,17,28,32 after 5 steps, by the
    extended time evolution: it equals U^5(pi/2) Z_13 U^5(pi/2)^dagger (with phase +1), so it is
    <Z_13> after 5 steps at theta_h and 5 steps of U(pi/2)^dagger.  One 10-step solve per seeded
    theta_h (FP64, chi as given)."""
    import numpy as np

    from paper_2306_14887_amd import bpki
    from paper_2306_14887_amd import lattice as L

    vals, secs = [], []
    with bpki.Context(0) as ctx:
        for th in L.theta_draw():
            t0 = time.perf_counter()
            r = ctx.solve(bpki.spec_from_lattice(lat, th, 5, chi, clifford_steps=5,
                                                 record_every_step=False))
            secs.append(time.perf_counter() - t0)
            vals.append(float(r["z"][-1][13]))
    return {"observable": "X13,29,31 Y9,30 Z8,12,17,28,32 after 5 steps", "chi": chi,
            "steps": "5 + 5 (extended time evolution)",
            "theta_h": [float(t) for t in L.theta_draw()], "value": vals,
            "seconds_per_solve_mean": float(np.mean(secs))}


def theta_batch(lat, chi: int, depth: int) -> dict:
    """The eight theta_h values of the workload solved together (one serving slot each): the
    aggregate Floquet steps/s of the batch (8 * depth / makespan)."""
    from paper_2306_14887_amd import bpki
    from paper_2306_14887_amd import lattice as L

    thetas = L.theta_draw(8, 2306)
    with bpki.Context(0) as ctx:
        ctx.serving_config(len(thetas))
        ctx.serving_packing(1)
        t0 = time.perf_counter()
        tickets = [ctx.submit(bpki.spec_from_lattice(lat, float(t), depth, chi)) for t in thetas]
        outs = [t.wait() for t in tickets]
        wall = time.perf_counter() - t0
    return {"thetas": len(thetas), "depth": depth, "chi": chi, "precision": "fp64",
            "aggregate_steps_per_s": len(thetas) * depth / wall, "makespan_s": wall,
            "bp_sweeps_per_step": float(sum(sum(o["bp_iters"]) for o in outs)) / (len(thetas) * depth)}


def precision_form(lat, chi: int, depth: int) -> dict:
    """The precision form of the workload: the eight seeded theta_h values (one serving slot
    each), with the 64 seeded Pauli strings (weight 3..17, tree clusters, X/Y/Z uniform) measured
    after the last step, in FP64 and in mixed precision (FP32 BP contractions, MIXED_TOL):
    the absolute error of every <Z_v>(t) and every string of the mixed run against the FP64 run,
    and the wall time of each batch (steps and strings)."""
    import numpy as np

    from paper_2306_14887_amd import bpki
    from paper_2306_14887_amd import lattice as L

    thetas = L.theta_draw(8, 2306)
    strings = [(p.sites, p.ops) for p in L.random_pauli_strings(lat, 64, seed=14887)]
    res = {}
    for name, prec, tol in (("fp64", bpki.BPKI_FP64, 1e-12), ("mixed", bpki.BPKI_FP32, MIXED_TOL)):
        with bpki.Context(0) as ctx:
            ctx.serving_config(len(thetas))
            ctx.serving_packing(1)
            t0 = time.perf_counter()
            tickets = [ctx.submit(bpki.spec_from_lattice(lat, float(t), depth, chi, precision=prec,
                                                         bp_tol=tol, pauli=strings))
                       for t in thetas]
            outs = [t.wait() for t in tickets]
            res[name] = (outs, time.perf_counter() - t0)
    (o64, w64), (o32, w32) = res["fp64"], res["mixed"]
    dz = np.abs(np.array([o["z"] for o in o32]) - np.array([o["z"] for o in o64]))
    dp = np.abs(np.array([o["pauli"] for o in o32]) - np.array([o["pauli"] for o in o64]))
    return {"thetas": len(thetas), "depth": depth, "chi": chi, "pauli_strings": len(strings),
            "fp64_batch_s": w64, "mixed_batch_s": w32,
            "abs_dz_max": float(dz.max()), "abs_dz_median": float(np.median(dz)),
            "abs_dpauli_max": float(dp.max()), "abs_dpauli_median": float(np.median(dp)),
            "pauli_abs_max_fp64": float(np.abs(np.array([o["pauli"] for o in o64])).max())}


def chi128_window(lat, theta: float, warmup: int = 7, steps: int = 3) -> dict:
    """The same workload at chi = 128 (bonds saturate after 7 steps): FP64 steps/s over `steps`
    steps after `warmup`."""
    import numpy as np

    from paper_2306_14887_amd import bpki

    with bpki.Context(0) as ctx:
        sess = ctx.session(bpki.spec_from_lattice(lat, theta, warmup + steps, 128))
        for _ in range(warmup):
            sess.step(observe=True)
        iters = []
        phase = np.zeros(4)
        t0 = time.perf_counter()
        for _ in range(steps):
            iters.append(sess.step(observe=True)["bp_iters"])
            phase += sess.last_timing()
        wall = time.perf_counter() - t0
        sess.close()
    return {"chi": 128, "value": steps / wall, "unit": "Floquet steps/s",
            "ms_per_step": 1e3 * wall / steps, "steps_timed": f"{warmup + 1}..{warmup + steps}",
            "bp_sweeps_per_step": float(np.mean(iters)),
            "phase_ms_per_step": {k: float(v / steps) for k, v in
                                  zip(("rx", "gate_layers", "bp", "observe"), phase)}}


def infinite_lattice(chi: int, depth: int = 30) -> dict:
    """The thermodynamic limit ("Dynamics of the infinite heavy-hex lattice", Fig. 4): the 5-site
    periodic cell (degree-3 sites A, B and three bridges) at theta_h in {pi/8, pi/4, 3pi/8},
    `depth` Floquet steps, FP64 (BP tolerance 1e-12) and mixed precision (FP32 MFMA BP, MIXED_TOL):
    <Z> per sublattice per step, the bond entropies after the last step and the time per step."""
    import math

    import numpy as np

    from paper_2306_14887_amd import bpki
    from paper_2306_14887_amd import lattice as L

    cell = L.infinite_cell()
    thetas = [math.pi / 8, math.pi / 4, 3 * math.pi / 8]
    runs, zs = [], {}
    with bpki.Context(0) as ctx:
        for prec, tol, name in ((bpki.BPKI_FP64, 1e-12, "fp64"),
                                (bpki.BPKI_FP32, MIXED_TOL, "mixed")):
            for th in thetas:
                t0 = time.perf_counter()
                r = ctx.solve(bpki.spec_from_lattice(cell, th, depth, chi, precision=prec,
                                                     bp_tol=tol, bond_entropy=True))
                wall = time.perf_counter() - t0
                z = r["z"]
                zs[(name, th)] = z
                runs.append({
                    "theta_h": th, "precision": name, "status": int(r["status"]),
                    "ms_per_step": 1e3 * wall / depth,
                    "bp_sweeps_per_step": float(np.mean(r["bp_iters"][:depth])),
                    "z_A": [round(float(x), 6) for x in z[:, 0]],
                    "z_B": [round(float(x), 6) for x in z[:, 1]],
                    "z_bridges": [round(float(x), 6) for x in z[:, 2:].mean(axis=1)],
                    "bond_entropy_last_step": [round(float(x), 6)
                                               for x in r["bond_entropy"][-1]],
                })
                print(f"infinite cell {name} theta={th:.4f}: {1e3 * wall / depth:.1f} ms/step",
                      file=sys.stderr, flush=True)
    for run in runs:
        if run["precision"] == "mixed":
            dz = np.abs(zs[("mixed", run["theta_h"])] - zs[("fp64", run["theta_h"])])
            run["abs_dz_vs_fp64_max"] = float(dz.max())
    # the three FP64 runs packed into one problem on the union of three cells (serving path):
    # a small request on the same lattice holds the one slot while the three queue up
    with bpki.Context(0) as ctx:
        ctx.serving_config(1)
        ctx.serving_packing(len(thetas), chi)
        hold = ctx.submit(bpki.spec_from_lattice(cell, 0.1, 1, 2))
        tickets = [ctx.submit(bpki.spec_from_lattice(cell, th, depth, chi, bond_entropy=True))
                   for th in thetas]
        hold.wait()
        while not all(t.poll() for t in tickets):
            time.sleep(0.002)
        times = np.array([t.times() for t in tickets])      # a ticket is released by wait()
        packs = [t.pack_size() for t in tickets]
        outs = [t.wait() for t in tickets]
    span = float(times[:, 2].max() - times[:, 1].min())
    packed = {"pack_sizes": packs, "aggregate_steps_per_s": len(thetas) * depth / span,
              "makespan_s": span,
              "sequential_steps_per_s": len(thetas) * depth / (1e-3 * depth * sum(
                  r["ms_per_step"] for r in runs if r["precision"] == "fp64")),
              "abs_dz_vs_alone_max": float(max(np.abs(o["z"] - zs[("fp64", th)]).max()
                                               for o, th in zip(outs, thetas)))}
    return {"lattice": "heavy-hex 5-site periodic cell (edges A-C_d colour d, C_d-B colour "
                       "(d+1) mod 3)", "chi": chi, "steps": depth, "runs": runs,
            "fp64_packed": packed}


def infinite_lattice_chi256(depth: int) -> dict:
    """The periodic heavy-hex cell at chi = 256 (the largest bond dimension of the thermodynamic-limit
    workload; truncation eigenproblems of n = 512): theta_h = pi/4, `depth` Floquet steps, FP64
    (BP tolerance 1e-12) and mixed precision (MIXED_TOL): <Z> per sublattice per step, the bond
    entropies after the last step and the time per step over the saturated steps (9..depth)."""
    import math

    import numpy as np

    from paper_2306_14887_amd import bpki
    from paper_2306_14887_amd import lattice as L

    cell = L.infinite_cell()
    th = math.pi / 4
    runs, zs = [], {}
    with bpki.Context(0) as ctx:
        for prec, tol, name in ((bpki.BPKI_FP64, 1e-12, "fp64"),
                                (bpki.BPKI_FP32, MIXED_TOL, "mixed")):
            sess = ctx.session(bpki.spec_from_lattice(cell, th, depth, 256, precision=prec,
                                                      bp_tol=tol))
            z, iters, sat = [], [], []
            for t in range(depth):
                t0 = time.perf_counter()
                r = sess.step()
                dt = time.perf_counter() - t0
                if t >= 8:
                    sat.append(dt)
                z.append(r["z"])
                iters.append(r["bp_iters"])
            ent = sess.observe_bond_entropy()
            sess.close()
            z = np.array(z)
            zs[name] = z
            runs.append({
                "precision": name, "ms_per_step_saturated": 1e3 * float(np.mean(sat)) if sat else None,
                "bp_sweeps_per_step": float(np.mean(iters)),
                "z_A": [round(float(x), 6) for x in z[:, 0]],
                "z_B": [round(float(x), 6) for x in z[:, 1]],
                "z_bridges": [round(float(x), 6) for x in z[:, 2:].mean(axis=1)],
                "bond_entropy_last_step": [round(float(x), 6) for x in ent],
            })
            print(f"infinite cell chi=256 {name}: {runs[-1]['ms_per_step_saturated']:.1f} ms/step",
                  file=sys.stderr, flush=True)
    runs[1]["abs_dz_vs_fp64_max"] = float(np.abs(zs["mixed"] - zs["fp64"]).max())
    return {"chi": 256, "theta_h": th, "steps": depth, "runs": runs}


def bp_error_ring(steps: int = 5, chi: int = 4) -> dict:
    """The BP error estimate (Eq. "BPErrorEstimate") on one heavy hexagon (the 12-qubit ring, the
    paper's smallest loop): after each of `steps` Floquet steps at theta_h in {0, pi/8, pi/4,
    3pi/8, pi/2}, the estimate on every edge (FP64, chi as given); reports the mean and the
    largest over the edges, per step."""
    import math

    import numpy as np

    from paper_2306_14887_amd import bpki
    from paper_2306_14887_amd import lattice as L

    ring = L.hexagon_ring()
    out = []
    t0 = time.perf_counter()
    with bpki.Context(0) as ctx:
        for th in (0.0, math.pi / 8, math.pi / 4, 3 * math.pi / 8, math.pi / 2):
            sess = ctx.session(bpki.spec_from_lattice(ring, th, steps, chi))
            mean, worst = [], []
            for _ in range(steps):
                sess.step(observe=False)
                errs = [sess.bp_error(e)[0] for e in range(ring.n_edges)]
                mean.append(float(np.mean(errs)))
                worst.append(float(np.max(errs)))
            sess.close()
            out.append({"theta_h": th, "mean_per_step": mean, "max_per_step": worst})
    return {"lattice": "12-qubit heavy hexagon (ring)", "chi": chi, "steps": steps,
            "runs": out, "seconds": time.perf_counter() - t0}


def oracle_config1_run(chi: int = 32, theta: float = 0.8, depth: int = 20) -> dict:
    """The oracle on one whole run of the chi = 32 configuration (127 qubits, 20 steps), BLAS at
    all cores: Floquet steps/s of the run."""
    from oracle import bp_tns as O
    from paper_2306_14887_amd import lattice as L

    lat = L.eagle()
    net = O.Network(lat.n_sites, lat.edges, lat.colour)
    sweeps = 0
    t0 = time.perf_counter()
    for t in range(depth):                # one step at a time on the same network
        r = O.solve(lat.n_sites, lat.edges, lat.colour, theta, 1, O.Options(chi=chi), net=net)
        sweeps += int(sum(r.bp_iters))
        print(f"oracle chi={chi} step {t + 1}/{depth}: {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    return {"chi": chi, "theta_h": theta, "steps": depth, "seconds": wall,
            "value": depth / wall, "unit": "Floquet steps/s", "cores": _cores(),
            "bp_sweeps": sweeps}


def copy_probe(mib: int) -> int:
    """8 launches of torch's device copy kernel, each reading and writing ``mib`` MiB."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(8):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": n * 8, "launches": 8}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=14)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--chi", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving", type=int, default=256,
                    help="requests in the serving measurement (0 = skip; 256 = the full stream)")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision window")
    ap.add_argument("--chi128", type=int, default=1,
                    help="1: also time steps 8..10 of the workload at chi = 128")
    ap.add_argument("--weight10", type=int, default=1,
                    help="1: also the weight-10 observable at the 8 theta_h (extended evolution)")
    ap.add_argument("--theta-batch", type=int, default=1,
                    help="1: also solve the eight theta_h values together (aggregate steps/s)")
    ap.add_argument("--infinite", type=int, default=128, metavar="CHI",
                    help="bond dimension of the infinite-lattice section (5-site periodic cell, "
                         "3 theta_h x 30 steps, FP64 and mixed; 0 = skip)")
    ap.add_argument("--precision-form", type=int, default=1,
                    help="1: also the 8 theta_h with 64 Pauli strings each, FP64 vs mixed errors")
    ap.add_argument("--precision-form-chi128", type=int, default=0,
                    help="1: also the precision form at chi = 128 (minutes of GPU time)")
    ap.add_argument("--infinite256", type=int, default=30, metavar="STEPS",
                    help="steps of the infinite-lattice cell at chi = 256 (theta_h = pi/4, FP64 and "
                         "mixed; 0 = skip)")
    ap.add_argument("--bp-error", type=int, default=1,
                    help="1: also the BP error estimate on the 12-qubit ring (5 theta_h, 5 steps)")
    ap.add_argument("--config1", type=int, default=1,
                    help="1: also the chi = 32 configuration (9 theta_h, 20 steps, magnetisation)")
    ap.add_argument("--cpu-config1", type=int, default=0,
                    help="1: also time the oracle on a whole chi = 32 run (theta_h 0.8, 20 steps; "
                         "minutes of CPU)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 8 plain device-to-device copies of MIB MiB and exit "
                         "(calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.copy_probe > 0:
        return copy_probe(args.copy_probe)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the per-request "
              "work does not span devices in this build.", file=sys.stderr)
        return 2

    import numpy as np

    from paper_2306_14887_amd import bpki
    from paper_2306_14887_amd import lattice as L

    lat = L.eagle()
    theta = L.theta_draw(8, 2306)[0]
    chi = args.chi
    depth = args.warmup + args.steps
    try:
        import torch
        have_torch = torch.cuda.is_available()
    except Exception:
        have_torch = False

    ctx = bpki.Context(0)
    spec = bpki.spec_from_lattice(lat, theta, depth, chi)
    sess = ctx.session(spec)
    for t in range(args.warmup):
        sess.step(observe=True)
        print(f"warmup step {t + 1}/{args.warmup}", file=sys.stderr, flush=True)
    if have_torch:
        torch.cuda.synchronize()
    sess.profile(True, stride=PROFILE_STRIDE)
    iters, zsteps = [], []
    phase = np.zeros(4)
    t0 = time.perf_counter()
    for t in range(args.steps):
        r = sess.step(observe=True)
        iters.append(r["bp_iters"])
        zsteps.append(r["z"])
        phase += sess.last_timing()
        print(f"step {t + 1}/{args.steps}: bp sweeps {r['bp_iters']}", file=sys.stderr,
              flush=True)
    if have_torch:
        torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = sess.profile_read()
    pk = {(k, 0): sess.profile_read_kernel(k, 0) for k in PROFILED}
    sess.profile(False)
    z = r["z"]
    sess.close()
    peaks = achievable_peaks(ctx)
    ctx.close()

    steps_per_s = args.steps / wall
    roof = dominant_roofline(pk, 0, peaks)
    roof.update({"launches_in_window": prof["all_launches"], "sampling_stride": PROFILE_STRIDE,
                 "achievable": peaks})
    out = {
        "metric": "Floquet steps/s at 127q chi=64",
        "value": steps_per_s,
        "unit": "Floquet steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {
            "workload": "eagle127 kicked Ising, BP-gauged simple update",
            "chi": chi, "theta_h": theta, "precision": "fp64", "bp_tol": 1e-12,
            "steps_timed": f"{args.warmup + 1}..{depth}",
            "bp_sweeps_per_step": float(np.mean(iters)),
            "phase_ms_per_step": {k: float(v / args.steps) for k, v in
                                  zip(("rx", "gate_layers", "bp", "observe"), phase)},
            "mean_z_last_step": float(np.mean(z)),
        },
        "roofline": roof,
    }
    if not args.no_mixed:
        mixed = mixed_window(lat, theta, chi, args.warmup, args.steps)
        dz = np.abs(mixed.pop("_z") - np.array(zsteps))
        mixed["abs_dz_vs_fp64_max"] = float(dz.max())
        mixed["abs_dz_vs_fp64_median"] = float(np.median(dz))
        mixed["bound"] = 1e-5
        out["mixed"] = mixed
        print("mixed-precision window done", file=sys.stderr, flush=True)
    if args.config1:
        out["config1"] = config1()
        print("chi=32 configuration done", file=sys.stderr, flush=True)
    if args.chi128:
        out["chi128"] = chi128_window(lat, theta)
        print("chi=128 window done", file=sys.stderr, flush=True)
    if args.weight10:
        out["weight10"] = weight10(lat, chi)
        print("weight-10 observable done", file=sys.stderr, flush=True)
    if args.theta_batch:
        out["theta_batch"] = theta_batch(lat, chi, args.warmup + args.steps)
        print("theta batch done", file=sys.stderr, flush=True)
    if args.precision_form:
        out["precision_form"] = precision_form(lat, chi, args.warmup + args.steps)
        print("precision form done", file=sys.stderr, flush=True)
    if args.precision_form_chi128:
        out["precision_form_chi128"] = precision_form(lat, 128, 20)
        print("precision form at chi = 128 done", file=sys.stderr, flush=True)
    if args.bp_error:
        out["bp_error_ring"] = bp_error_ring()
        print("BP error estimate done", file=sys.stderr, flush=True)
    if args.infinite > 0:
        out["infinite_lattice"] = infinite_lattice(args.infinite)
        print("infinite lattice done", file=sys.stderr, flush=True)
    if args.infinite256 > 0:
        out["infinite_lattice_chi256"] = infinite_lattice_chi256(args.infinite256)
        print("infinite lattice chi=256 done", file=sys.stderr, flush=True)
    if args.serving > 0:
        out["serving"] = serving_bench(args.serving, args.slots)
        print("serving done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(lat, chi, theta, float(np.mean(iters)))
        if args.cpu_config1:
            out["cpu_baseline"]["config1_run"] = oracle_config1_run()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
