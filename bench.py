#!/usr/bin/env python3
"""Benchmark of the direct-summation hot path on one MI355X.

Default workload: a single Plummer cluster of N = 262144 equal masses (eps = 1e-4, no external
field) advanced by the kick-drift-kick leapfrog with dt = 2^-11, pair arithmetic in mode fp32dl
(particles sorted along a Hilbert curve, coordinates local to each work item, FP32 on far j-tiles
and double-single on near ones, FP64-folded tile sums).  One "step" = one leapfrog step = one full
force evaluation (N^2 pair interactions, j = i counted as the paper counts N^2) plus the O(N)
sort, far-tile and kick/drift kernels.  Throughput is pair interactions per second of the whole step.

Prints ONE JSON line.  Besides the contract fields it carries:
  roofline      the pair kernel (dominant, about 98% of the step) against the FP32 vector peak, with
                its duration measured by HIP events recorded around every pair-kernel launch on
                the stream the kernel runs on, over the timed region;
  cpu_baseline  the FP64 oracle timed on this host's cores on a bounded sample of the same
                workload (a block of rows against all N sources);
  modes         the same step timed in the other precision modes;
  accel_error_on_fp64_trajectory  every mode's accuracy (paper_1003_3896_amd.accuracy: the a_rms,
                per-particle, L2 and S_i metrics) on states of the FP64 trajectory;
  c1, c2, c4, c5  short runs of the other configurations (default run only; --no-extras skips
                them): C1 with step graphs on and off, the C2 step with its accuracy on the state
                after 50 FP64 sym6 steps, the C4 ensemble batched against per-cluster launches, and a
                bounded C5 served stream with p50/p99 latency beside its throughput.
Other workloads (--workload c1|c2|c4|c5|paper|bh) run their own configurations in full.
"""
import argparse
import hashlib

import numpy as np
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_INTERACTION = 20  # the paper's convention for one pair force (Sect. 4.1)
PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 vector peak (256 CU, 2.4 GHz)
PEAK_FP64_TFLOPS = 78.6
# Issue-rate ceiling of the pair loop (FP32 modes, no packed FP32): a wave64 FP32 FMA every 2.9 SIMD
# cycles and v_rsq_f32 adding 6.2 cycles at 6 waves per SIMD (timed instruction-stream
# microbenchmark on gfx950); VALU instructions per term of the fastest loop a workload runs, counted
# in the compiled code (the rest of the kernel, staging, folds and near tiles, only adds to it).
CYCLES_PER_FMA, RSQ_EXTRA_CYCLES = 2.9, 6.2
LOOP_VALU = {("fp32dl", True): 10.19, ("fp32dl", False): 12.19, ("fp32ds", True): 17.09,
             ("fp32ds", False): 18.09}
METRIC = "G pair-interactions/s & %FP32 VALU peak; batched p50/p99 job latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's own step count; C3 1000, C2 200, C1 and C4 100)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5", "paper", "bh"])
    ap.add_argument("--sizes", default=None, help="paper: comma-separated N (default 480*2^k .. 1,536,000)")
    ap.add_argument("--ratios", default=None, help="bh: comma-separated black-hole to cluster mass ratios")
    ap.add_argument("--jobs", type=int, default=120, help="c5: jobs in the open-loop stream")
    ap.add_argument("--sat-jobs", type=int, default=48, help="c5: jobs in the closed-loop saturation run")
    ap.add_argument("--warm-jobs", type=int, default=None,
                    help="c5: first jobs left out of the latency statistics (default: jobs / 20)")
    ap.add_argument("--load", type=float, default=0.8, help="c5: offered load as a fraction of saturation")
    ap.add_argument("--policy", default="srpt", choices=["srpt", "all"], help="c5: which active jobs a round advances")
    ap.add_argument("--fill", type=float, default=2.0 ** 30, help="c5: pair interactions a round gathers (srpt)")
    ap.add_argument("--prec", default=None, help="fp32 | fp32c | fp32ds | fp32dl | fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the c1/c2/c4/c5 keys of the c3 run, the graph A/B of c1/c2 and the per-cluster "
                         "baseline of c4 (profiling runs)")
    ap.add_argument("--extra-jobs", type=int, default=120, help="c3 extras: jobs of the bounded C5 stream")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    return ap.parse_args()


def workload(name):
    from paper_1003_3896_amd import inputs
    if name == "c1":
        return inputs.c1(), "fp64"
    # the fastest mode that meets the 1e-6 accuracy gate over a whole step: the local double-single
    # mode for the large clusters, plain double-single for the ensemble of small ones (where the
    # local mode's pair kernel is no faster and its sort costs a few percent of the step); the
    # other mode is reported beside it
    if name == "c2":
        return inputs.c2(), "fp32dl"
    if name == "c3":
        return inputs.c3(), "fp32dl"
    return inputs.c4(), "fp32ds"


ACCEL_ROWS = 2048  # rows of the per-mode accuracy table


PROFILE_TAG = {"c3": "plummer262144", "c2": "salpeter65536", "c4": "ensemble512"}  # committed counter summaries

# sources that decide what a pair-kernel launch does (its code, work items and split rule)
PAIR_SOURCES = [os.path.join(ROOT, "paper_1003_3896_amd", "csrc", f)
                for f in ("pair_kernel.h", "nb_device.h", "nb_internal.h", "runtime.hip")]


def pair_source_hash():
    """Hash of the code of PAIR_SOURCES with // comments and blank lines removed (editing a comment
    does not change a kernel)."""
    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        for line in open(f, encoding="utf-8"):
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def profile_summary(prec, tile=None, workload="c3"):
    """Fields of the committed counter summary of this workload's pair kernel, or None if there is
    none, or the kernel sources or the launch shape have changed since the counters were taken."""
    if workload not in PROFILE_TAG:
        return None
    path = os.path.join(ROOT, "profiles", "pair_%s_%s.md" % (prec, PROFILE_TAG[workload]))
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            v = v.split()
            fields[k.strip()] = v[0].strip("`") if v else ""
    if fields.get("kernel_source_sha256") != pair_source_hash():
        return None
    if tile is not None and fields.get("tile") != ",".join(str(v) for v in tile):
        return None
    return fields


def traffic_from_profile(prec, tile=None, workload="c3"):
    """HBM bytes per pair-kernel launch (FETCH_SIZE and WRITE_SIZE calibrated against a plain
    copy) from the committed summary, or None (see profile_summary)."""
    f = profile_summary(prec, tile, workload)
    try:
        return float(f["hbm_bytes_per_launch"]) if f else None
    except (KeyError, ValueError):
        return None


def issue_counters(prec, tile=None, workload="c3"):
    """The pair kernel's instruction mix and cycles per wave-interaction (20 at the FP32 vector peak)
    from the committed counter summary, or None."""
    f = profile_summary(prec, tile, workload)
    try:
        return {"valu_per_wave_interaction": float(f["valu_per_wave_interaction"]),
                "trans_per_wave_interaction": float(f["trans_per_wave_interaction"]),
                "busy_clock_ghz": float(f["busy_clock_ghz"]),
                "source": "rocprofv3 counters of the committed summary (another run of the same kernel)"}
    except (TypeError, KeyError, ValueError):
        return None


def time_steps(sim, integrator, dt, steps, warmup, torch):
    from paper_1003_3896_amd import nbody
    sim.accel()
    if warmup:
        sim.step(integrator, dt, warmup)
    torch.cuda.synchronize()
    nbody.nbody_timing_read(sim.ctx)  # drop anything recorded so far
    nbody.nbody_timing_enable(sim.ctx, True)
    t0 = time.perf_counter()
    sim.step(integrator, dt, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nbody.nbody_timing_enable(sim.ctx, False)
    kms, nlaunch = nbody.nbody_timing_read(sim.ctx)
    return t1 - t0, kms, nlaunch


def energy_fp64(sim):
    """Library FP64 diagnostics of cluster 0: (E, E_int, Lz) with E_int = K_cm-frame + W."""
    e = sim.energy(prec="fp64")[0].cpu().numpy()
    K, W, Uext, E = e[0], e[1], e[2], e[3]
    P = e[4:7]
    M = e[13]
    return E, K - 0.5 * float(P @ P) / M + W, e[9]


def drift_report(e0, e1):
    return {"dE_over_E0": float(abs(e1[0] - e0[0]) / abs(e0[0])),
            "dE_over_Eint0": float(abs(e1[0] - e0[0]) / abs(e0[1])),
            "dLz_over_Lz0": float(abs(e1[2] - e0[2]) / abs(e0[2])) if e0[2] != 0 else None}


def per_cluster_baseline(batch, integrator, dt, steps, torch):
    """The same kernels launched cluster by cluster (one single-cluster system per call, one stream,
    no graphs): what the batched persistent launch is compared against."""
    from paper_1003_3896_amd import nbody
    sim = nbody.Simulation(batch, "fp32ds")
    ctx = sim.ctx
    nbody.nbody_use_graphs(ctx, False)
    sizes = np.diff(batch.offsets)
    big = int(sizes.max())
    one = nbody.System([0, big], [batch.eps[0]], None, batch.G, batch.galaxy, "fp32ds")
    wsb = nbody.nbody_workspace_bytes(ctx, one)
    ws = torch.empty(wsb + 256, dtype=torch.uint8, device="cuda")
    wsa = (ws.data_ptr() + 255) & ~255
    systems = [nbody.System([0, int(n)], [batch.eps[c]], None if batch.field is None else [batch.field[c]],
                            batch.G, batch.galaxy, "fp32ds") for c, n in enumerate(sizes)]
    fn = nbody.nbody_step_leapfrog if integrator == "leapfrog" else nbody.nbody_step_sym6
    P, V, M, A = (sim.pos.data_ptr(), sim.vel.data_ptr(), sim.mass.data_ptr(), sim.acc.data_ptr())
    sim.accel()

    def run(nst):
        for c, sysc in enumerate(systems):
            o = int(batch.offsets[c])
            fn(ctx, sysc, P + 24 * o, V + 24 * o, M + 8 * o, A + 24 * o, dt, nst, wsa, wsb)

    run(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.close()
    return el


def cpu_baseline(batch, pos_all, target_s, a_gpu):
    """Time the FP64 oracle on a block of rows of the first cluster against all of its sources, at
    the positions the GPU run ended with (so the same rows double as a parity sample)."""
    import numpy as np
    import oracle
    oracle.build()
    n = int(batch.offsets[1])
    pos, mass, eps = pos_all[:n], batch.mass[:n], float(batch.eps[0])
    probe = max(1, min(n, 256))
    oracle.accel(pos, mass, batch.G, eps, rows=(0, probe))  # starts the thread pool
    t0 = time.perf_counter()
    oracle.accel(pos, mass, batch.G, eps, rows=(0, probe))
    tp = max(time.perf_counter() - t0, 1e-6)
    rows = int(max(probe, min(n, probe * target_s / tp)))
    t0 = time.perf_counter()
    ref, absa = oracle.accel(pos, mass, batch.G, eps, rows=(0, rows), want_abs=True)
    el = time.perf_counter() - t0
    inter = rows * n
    if batch.field[0]:
        ae, _ = oracle.ext_field(pos[:rows], batch.G, batch.galaxy)
        ref = ref + ae
        absa = absa + np.linalg.norm(ae, axis=1)
    err = np.linalg.norm(a_gpu[:rows] - ref, axis=1) / absa
    cores = oracle.num_threads()
    # one thread, on a sample of about 3 s
    oracle.set_threads(1)
    rows1 = max(1, min(n, int(3.0 * rows / (max(el, 1e-6) * max(cores, 1)))))
    t0 = time.perf_counter()
    oracle.accel(pos, mass, batch.G, eps, rows=(0, rows1))
    el1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    return {
        "value": inter / el / 1e9,
        "unit": "G pair-interactions/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "rows [0,%d) of the first cluster (N=%d) against all its sources, one FP64 force evaluation, "
                  "%.1f s" % (rows, n, el),
        "single_thread_value": rows1 * n / el1 / 1e9,
        "single_thread_sample": "rows [0,%d), %.1f s" % (rows1, el1),
        "cpu_model": _cpu_model(),
    }, {"rows": rows, "max": float(err.max()), "median": float(np.median(err))}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def sample_rows(n, nrows):
    """About nrows rows of a cluster of n, in three blocks: its start, middle and end."""
    if nrows >= n:
        return np.arange(n)
    per = max(1, nrows // 3)
    h = n // 2
    blocks = [(0, per), (max(per, h - per // 2), max(per, h - per // 2) + per), (max(0, n - per), n)]
    idx = np.unique(np.concatenate([np.arange(a, min(b, n)) for a, b in blocks]))
    return idx


def oracle_rows(batch, pos, idx):
    """Oracle acceleration (internal + field) and S_i of rows idx of the first cluster at pos."""
    import oracle
    n = int(batch.offsets[1])
    refs, scales = [], []
    # contiguous runs of idx, one oracle call each
    cuts = np.nonzero(np.diff(idx) != 1)[0] + 1
    for run in np.split(idx, cuts):
        r0, r1 = int(run[0]), int(run[-1]) + 1
        ref, absa = oracle.accel(pos[:n], batch.mass[:n], batch.G, float(batch.eps[0]), rows=(r0, r1),
                                 want_abs=True)
        if batch.field[0]:
            ae, _ = oracle.ext_field(pos[r0:r1], batch.G, batch.galaxy)
            ref = ref + ae
            absa = absa + np.linalg.norm(ae, axis=1)
        refs.append(ref)
        scales.append(absa)
    return np.concatenate(refs), np.concatenate(scales)


def sampled_state_errors(batch, modes, integrator, dt, targets, nrows, torch):
    """Accuracy of every mode's force evaluation on states of the FP64-mode trajectory (after each
    step count in targets), against the oracle on the same state, on sampled rows of the first
    cluster; a_rms from the library's FP64 evaluation of the whole cluster (pinned to the oracle by
    the tests).  All metrics of paper_1003_3896_amd.accuracy."""
    from paper_1003_3896_amd import accuracy, nbody
    n = int(batch.offsets[1])
    idx = sample_rows(n, nrows)
    ref_sim = nbody.Simulation(batch, "fp64")
    ref_sim.accel()
    sims = {m: nbody.Simulation(batch, m) for m in modes}
    out, done = {}, 0
    for target in sorted(set(targets)):
        if target > done:
            ref_sim.step(integrator, dt, target - done)
            done = target
        torch.cuda.synchronize()
        pos = ref_sim.pos.cpu().numpy()
        a64 = ref_sim.acc.cpu().numpy()[:n]
        arms = [float(np.sqrt(np.mean((a64 * a64).sum(1))))]
        ref, scale = oracle_rows(batch, pos, idx)
        row = {}
        for m, sm in sims.items():
            sm.pos.copy_(ref_sim.pos)
            a = sm.accel().cpu().numpy()[idx]
            row[m] = accuracy.short(accuracy.accel_error(a, ref, offsets=[0, n], scale=scale, rows=idx, arms=arms))
        out[str(target)] = row
    for sm in list(sims.values()) + [ref_sim]:
        sm.close()
    return out


def all_particle_errors(batch, pos, modes, torch):
    """Every mode's force evaluation at positions pos against the library's FP64 evaluation of the
    same state, over ALL particles (the FP64 mode matches the oracle to 1e-15 in the tests): the
    a_rms, per-particle and L2 metrics of paper_1003_3896_amd.accuracy (no S_i: that needs the
    oracle)."""
    from paper_1003_3896_amd import accuracy, nbody
    ref = nbody.Simulation(batch, "fp64")
    ref.pos.copy_(torch.as_tensor(pos, dtype=torch.float64, device="cuda"))
    a64 = ref.accel().cpu().numpy()
    out = {}
    for m in modes:
        sm = nbody.Simulation(batch, m)
        sm.pos.copy_(ref.pos)
        out[m] = accuracy.short(accuracy.accel_error(sm.accel().cpu().numpy(), a64, offsets=batch.offsets))
        sm.close()
    ref.close()
    return out


def graph_ab(batch, prec, integrator, dt, steps, torch):
    """Wall-clock ms per step of the same run with step graphs on and off (no per-kernel events)."""
    from paper_1003_3896_amd import nbody
    gres = {}
    for use in (True, False):
        s3 = nbody.Simulation(batch, prec)
        nbody.nbody_use_graphs(s3.ctx, use)
        s3.accel()
        s3.step(integrator, dt, steps)  # the same call as the timed one: graphs captured here
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s3.step(integrator, dt, steps)
        torch.cuda.synchronize()
        gres["graphs_on" if use else "graphs_off"] = round((time.perf_counter() - t0) / steps * 1e3, 4)
        s3.close()
    return gres


def equal_masses(batch):
    """True when every cluster's masses are all equal (the pair loops then leave the mass out)."""
    return all(np.all(batch.mass[batch.offsets[c]:batch.offsets[c + 1]] == batch.mass[batch.offsets[c]])
               for c in range(len(batch.offsets) - 1) if batch.offsets[c + 1] > batch.offsets[c])


def rsq_ceiling(prec, equal_masses):
    """The issue-rate ceiling of the fastest pair loop of this mode, as a fraction of the FP32 peak
    (20 SIMD cycles per wave-interaction), or None where no loop count is recorded."""
    n = LOOP_VALU.get((prec, bool(equal_masses)))
    if n is None:
        return None
    cyc = n * CYCLES_PER_FMA + RSQ_EXTRA_CYCLES
    return {"frac": round(FLOPS_PER_INTERACTION / cyc, 4), "cycles_per_wave_interaction": round(cyc, 2),
            "valu_per_term": n, "cycles_per_fma": CYCLES_PER_FMA, "rsq_extra_cycles": RSQ_EXTRA_CYCLES}


def pair_roofline(prec, inter_per_eval, pair_ms, tile=None, workload="c3", equal_masses=None):
    achieved = FLOPS_PER_INTERACTION * inter_per_eval / (pair_ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved / peak, 4), "traffic": traffic_from_profile(prec, tile, workload),
           "kernel": "pair (%s)" % prec, "kernel_ms": round(pair_ms, 4)}
    if equal_masses is not None:
        out["rsq_ceiling"] = rsq_ceiling(prec, equal_masses)
    return out


def extra_c1(torch):
    """C1 (N = 1024 Plummer, FP64, 100 leapfrog steps of 1/1024): launch-bound; graphs on and off."""
    from paper_1003_3896_amd import inputs, nbody
    b = inputs.c1()
    sim = nbody.Simulation(b, "fp64")
    wall, kms, nl = time_steps(sim, "leapfrog", b.meta["dt"], 100, 3, torch)
    sim.close()
    return {"workload": "plummer-1024, fp64, leapfrog, 100 steps", "ms_per_step": round(wall / 100 * 1e3, 4),
            "G_interactions_per_s": round(b.n * b.n * 100 / wall / 1e9, 3),
            "pair_kernel_ms": round(kms / max(nl, 1), 4),
            "ms_per_step_graphs": graph_ab(b, "fp64", "leapfrog", b.meta["dt"], 100, torch)}


def extra_c2(torch, steps=5):
    """C2 (N = 65536 Salpeter + galaxy, sym6): a few whole steps in the local double-single mode, and
    every FP32 mode's accuracy on the state after 50 FP64 sym6 steps."""
    from paper_1003_3896_amd import autotune, inputs, nbody
    b = inputs.c2()
    prec = "fp32dl"
    dt = b.meta["dt"]
    sim = nbody.Simulation(b, prec)
    tile = nbody.nbody_get_tile(sim.ctx, prec, autotune.size_class(b.n))
    e0 = energy_fp64(sim)
    wall, kms, nl = time_steps(sim, "sym6", dt, steps, 1, torch)
    e1 = energy_fp64(sim)
    sim.close()
    ipe = b.interactions_per_eval()
    out = {"workload": "plummer-salpeter-65536, galaxy field, sym6, dt 2^-11", "precision_mode": prec,
           "steps": steps, "ms_per_step": round(wall / steps * 1e3, 4),
           "G_interactions_per_s": round(ipe * 7 * steps / wall / 1e9, 3),
           "roofline": pair_roofline(prec, ipe, kms / max(nl, 1), tile, "c2", equal_masses(b)),
           "energy": dict(drift_report(e0, e1), steps=steps + 1)}
    out["accel_error_after_50_fp64_steps"] = sampled_state_errors(
        b, ["fp32dl", "fp32ds", "fp32c"], "sym6", dt, [50], 768, torch)["50"]
    return out


def c4_accuracy(batch, torch):
    """The batched launch and single-cluster launches of the same clusters (smallest, largest, two
    in between) against the oracle: the accuracy the throughput comparison is made at."""
    import oracle
    from paper_1003_3896_amd import accuracy, inputs, nbody
    sizes = np.diff(batch.offsets)
    order = np.argsort(sizes, kind="stable")
    pick = sorted({int(order[0]), int(order[-1]), int(order[len(order) // 3]), int(order[2 * len(order) // 3])})
    sim = nbody.Simulation(batch, "fp32ds")
    a_b = sim.accel().cpu().numpy()
    sim.close()
    got = {"batched": [], "per_cluster": []}
    refs, scales = [], []
    for c in pick:
        s, e = int(batch.offsets[c]), int(batch.offsets[c + 1])
        ref, absa = oracle.accel(batch.pos[s:e], batch.mass[s:e], batch.G, float(batch.eps[c]), want_abs=True)
        refs.append(ref)
        scales.append(absa)
        got["batched"].append(a_b[s:e])
        one = nbody.Simulation(inputs.single(batch.pos[s:e], batch.vel[s:e], batch.mass[s:e], batch.eps[c]), "fp32ds")
        got["per_cluster"].append(one.accel().cpu().numpy())
        one.close()
    offs = np.concatenate([[0], np.cumsum([len(r) for r in refs])])
    ref, scale = np.concatenate(refs), np.concatenate(scales)
    out = {k: accuracy.short(accuracy.accel_error(np.concatenate(v), ref, offsets=offs, scale=scale))
           for k, v in got.items()}
    out["clusters"] = [int(sizes[c]) for c in pick]
    return out


def extra_c4(torch, steps=3, base_steps=2):
    """C4 (512 Plummer clusters, 256..16384, sym6, FP32DS): the persistent ragged launch against the
    same kernels launched cluster by cluster, a few steps each, and their accuracy."""
    from paper_1003_3896_amd import autotune, inputs, nbody
    b = inputs.c4()
    prec = "fp32ds"
    dt = b.meta["dt"]
    sim = nbody.Simulation(b, prec)
    tile = nbody.nbody_get_tile(sim.ctx, prec, autotune.size_class(int(np.diff(b.offsets).max())))
    wall, kms, nl = time_steps(sim, "sym6", dt, steps, 1, torch)
    sim.close()
    ipe = b.interactions_per_eval()
    value = ipe * 7 * steps / wall / 1e9
    el = per_cluster_baseline(b, "sym6", dt, base_steps, torch)
    per = ipe * 7 * base_steps / el / 1e9
    return {"workload": "512 Plummer clusters, N log-uniform [256,16384], eps 1e-3, sym6", "precision_mode": prec,
            "steps": steps, "ms_per_step": round(wall / steps * 1e3, 4), "G_interactions_per_s": round(value, 3),
            "roofline": pair_roofline(prec, ipe, kms / max(nl, 1), tile, "c4", equal_masses(b)),
            "per_cluster_launches": {"G_interactions_per_s": round(per, 3), "steps": base_steps,
                                     "ms_per_step": round(el / base_steps * 1e3, 4)},
            "batched_over_per_cluster": round(value / per, 2),
            "accel_error": c4_accuracy(b, torch)}


def extra_c5(args):
    """A bounded C5 served stream (the full stream is --workload c5)."""
    import argparse
    a = argparse.Namespace(**vars(args))
    a.jobs, a.sat_jobs, a.prec, a.load, a.policy, a.fill = args.extra_jobs, 32, "fp32ds", 0.8, "srpt", 2.0 ** 30
    r = bench_c5(a)
    keep = ("value", "unit", "latency_s", "stretch", "saturation_G_interactions_per_s", "rounds", "jobs_done",
            "jobs_failed", "max_rel_energy_error", "config")
    return {k: r[k] for k in keep}


def serve_requests(jobs):
    from paper_1003_3896_amd.serve import Request
    reqs = []
    for j in jobs:
        p, v, m = j.initial_state()
        reqs.append(Request(j.jid, p, v, m, j.steps, j.integrator, j.dt, j.eps, j.field, j.arrival))
    return reqs


def bench_c5(args):
    """Served stream: closed-loop saturation throughput first, then Poisson arrivals at the given
    fraction of it; latency = arrival -> final state and energy on the host."""
    import torch
    from paper_1003_3896_amd import inputs
    from paper_1003_3896_amd.serve import HipExecutor, Server, latency_stats
    torch.cuda.set_device(0)
    cap, maxb = 1 << 20, 256
    ex = HipExecutor(cap, maxb, args.prec or "fp32ds")
    # saturation: all jobs present at t = 0; throughput over the rounds with a backlog
    sat = serve_requests(inputs.c5_jobs(args.sat_jobs, 0.0, seed=5006))
    for r in sat:
        r.arrival = 0.0
    srv = Server(ex, energy=False, policy=args.policy, fill=args.fill)
    t0 = time.perf_counter()
    res = srv.run(sat)
    el = time.perf_counter() - t0
    work = sum(r.interactions() for r in sat if res[r.jid].status == "done")
    xsat = work / el
    print("c5: saturation %.3e int/s over %d jobs in %.1f s" % (xsat, len(sat), el), file=sys.stderr, flush=True)
    # the stream's sizes and step counts do not depend on the rate: take its own mean work, so the
    # offered load is the stated fraction of the measured saturation throughput
    probe = inputs.c5_jobs(args.jobs, 1.0)
    mean_work = sum(j.n * j.n * j.steps * (1 if j.integrator == "leapfrog" else 7) for j in probe) / len(probe)
    rate = args.load * xsat / mean_work
    jobs = inputs.c5_jobs(args.jobs, rate)
    reqs = serve_requests(jobs)
    count = [0]

    def progress(r):
        count[0] += 1
        if count[0] % 20 == 0:
            print("c5: %d / %d jobs done" % (count[0], len(reqs)), file=sys.stderr, flush=True)

    srv = Server(ex, energy=True, policy=args.policy, fill=args.fill, on_result=progress)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    el = time.perf_counter() - t0
    done = [r for r in reqs if res[r.jid].status == "done"]
    work = sum(r.interactions() for r in done)
    warm = args.warm_jobs if args.warm_jobs is not None else max(1, args.jobs // 20)
    lat = latency_stats(res, skip=warm)
    dE = [res[r.jid].rel_energy_error for r in done]
    # stretch: latency over the job's own work at the saturation rate
    stretch = sorted(res[r.jid].latency / (r.interactions() / xsat) for r in done if r.jid >= warm)
    ex.close()
    return {
        "metric": METRIC,
        "value": round(work / el / 1e9, 3),
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": len(done),
        "warmup": warm,
        "ms_per_step": round(el / max(len(done), 1) * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Plummer jobs, Poisson arrivals)",
        "config": {"workload": "served stream: N log-uniform [1024,65536], steps U[10,1000], leapfrog/sym6 "
                               "50/50, galaxy field on half, eps=1e-3, dt=2^-11, " + (args.prec or "fp32ds"),
                   "jobs": args.jobs, "offered_load": args.load, "arrival_rate_per_s": round(rate, 4),
                   "arena_particles": cap, "max_clusters": maxb, "policy": args.policy,
                   "fill": args.fill},
        "latency_s": {"p50": round(lat["p50"], 4), "p99": round(lat["p99"], 4), "mean": round(lat.get("mean", 0), 4),
                      "jobs_counted": lat["n"]},
        "stretch": {"p50": round(float(np.percentile(stretch, 50)), 3),
                    "p99": round(float(np.percentile(stretch, 99)), 3)} if stretch else None,
        "saturation_G_interactions_per_s": round(xsat / 1e9, 3),
        "rounds": srv.rounds,
        "jobs_done": len(done),
        "jobs_failed": sum(1 for r in reqs if res[r.jid].status != "done"),
        "max_rel_energy_error": float(np.nanmax(dE)) if dE else None,
    }


def bench_paper(args):
    """The paper's timing set-up (Sect. 5): a uniform sphere with virial ratio 0.3, softening
    0.005 R / N^(1/3), in the galaxy, leapfrog steps of 5e-4, for N = 480 * 2^k up to 1,536,000:
    time per step and pair interactions per second at every N (the analog of its timing curves)."""
    import numpy as np
    import torch
    from paper_1003_3896_amd import inputs, nbody
    torch.cuda.set_device(0)
    prec = args.prec or "fp32dl"
    sizes = [int(x) for x in args.sizes.split(",")] if args.sizes else inputs.PAPER_SIZES
    scan = []
    last = None
    for n in sizes:
        batch = inputs.paper_timing(n)
        sim = nbody.Simulation(batch, prec)
        steps = max(1, min(args.steps or 30, int(2e12 / max(n * n, 1))))  # about a second of pair work each
        wall, kms, nl = time_steps(sim, "leapfrog", batch.meta["dt"], steps, 1, torch)
        row = {"n": n, "steps": steps, "ms_per_step": round(wall / steps * 1e3, 4),
               "G_interactions_per_s": round(n * n * steps / wall / 1e9, 3),
               "pair_kernel_ms": round(kms / max(nl, 1), 4)}
        print("paper N=%d %s" % (n, row), file=sys.stderr, flush=True)
        scan.append(row)
        if n == sizes[-1]:
            last = (batch, sim.pos.cpu().numpy(), sim.acc.cpu().numpy(), row, wall, steps)
        sim.close()
    batch, pos_final, a_gpu, row, wall, steps = last
    pair_ms = row["pair_kernel_ms"]
    achieved = FLOPS_PER_INTERACTION * row["n"] ** 2 / (pair_ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
    result = {
        "metric": METRIC,
        "value": row["G_interactions_per_s"],
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": row["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic (seeded uniform spheres)",
        "config": {"workload": "uniform sphere, virial ratio 0.3, eps = 0.005/N^(1/3), galaxy field, leapfrog "
                               "dt = 5e-4; N = %d..%d" % (sizes[0], sizes[-1]),
                   "precision_mode": prec, "value_at_n": row["n"]},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": None, "kernel": "pair (%s)" % prec,
                     "kernel_ms": pair_ms, "flops_per_interaction": FLOPS_PER_INTERACTION},
        "scan": scan,
    }
    # the paper's own figure for this workload and N (one Tesla C1060, Table 3 at 20 flops per
    # interaction): another machine's number, reported as context
    paper = {"fp64": 22.0 / 20}.get(prec, 423.0 / 20)  # G interactions/s
    if row["n"] == 1536000:
        result["vs_baseline"] = round(row["G_interactions_per_s"] / paper, 2)
        result["vs_baseline_basis"] = ("the paper's single-GPU %s figure for N = 1,536,000 (%.1f G interactions/s, "
                                       "Tesla C1060); other hardware" % ("FP64" if prec == "fp64" else "FP32", paper))
    if not args.no_cpu_baseline:
        cb, parity = cpu_baseline(batch, pos_final, args.cpu_seconds, a_gpu)
        result["cpu_baseline"] = cb
        result["parity_sample"] = parity
    return result


def bench_black_hole(args):
    """The stiff collisions of Sect. 6.2 (Table 8): an N = 15360 uniform sphere falling through a
    central point mass of 0.1, 1, 50 and 105 cluster masses from (10, 0, 0), sym6 with dt = 1e-4;
    energy and angular-momentum changes (FP64 diagnostics) after the given number of steps (the
    paper's runs are 4e4 steps, t = [0, 4]; the default here covers the first 4000)."""
    import numpy as np
    import torch
    from paper_1003_3896_amd import inputs, nbody
    torch.cuda.set_device(0)
    prec = args.prec or "fp32ds"
    steps = args.steps or 4000
    rows, tot_int, tot_wall = [], 0.0, 0.0
    ratios = [float(x) for x in args.ratios.split(",")] if args.ratios else inputs.BH_RATIOS
    for ratio in ratios:
        b = inputs.paper_black_hole(ratio)
        sim = nbody.Simulation(b, prec)
        e0 = sim.energy(prec="fp64")[0].cpu().numpy().copy()
        sim.accel()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:  # in slices, so a long run prints its progress
            k = min(2000, steps - done)
            sim.step("sym6", b.meta["dt"], k)
            torch.cuda.synchronize()
            done += k
            print("bh ratio %g: %d / %d steps" % (ratio, done, steps), file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        e1 = sim.energy(prec="fp64")[0].cpu().numpy().copy()
        L0, L1 = e0[7:10], e1[7:10]
        row = {"mbh_over_m": ratio, "steps": steps, "t_end": round(steps * b.meta["dt"], 6),
               "dE_over_E0": float(abs(e1[3] - e0[3]) / abs(e0[3])),
               "dL_over_L0": float(np.linalg.norm(L1 - L0) / np.linalg.norm(L0)),
               "dLz_over_Lz0": float(abs(L1[2] - L0[2]) / abs(L0[2])),
               "ms_per_step": round(wall / steps * 1e3, 4), "finite": bool(e1[19] == 0)}
        rows.append(row)
        tot_int += b.interactions_per_eval() * 7 * steps
        tot_wall += wall
        sim.close()
    return {
        "metric": METRIC,
        "value": round(tot_int / tot_wall / 1e9, 3),
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": round(tot_wall / (steps * len(rows)) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic (seeded uniform sphere)",
        "config": {"workload": "cluster-black hole collisions: N = 15360 uniform sphere, virial ratio 0.3, "
                               "from (10, 0, 0) at 0.001 v_c, black hole of 0.1/1/50/105 cluster masses, "
                               "sym6 dt = 1e-4", "precision_mode": prec},
        "table8": rows,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(asked for --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "c5":
        print(json.dumps(bench_c5(args)), flush=True)
        return
    if args.workload == "paper":
        print(json.dumps(bench_paper(args)), flush=True)
        return
    if args.workload == "bh":
        print(json.dumps(bench_black_hole(args)), flush=True)
        return
    import torch
    from paper_1003_3896_amd import inputs, nbody

    torch.cuda.set_device(0)
    batch, prec = workload(args.workload)
    prec = args.prec or prec
    if args.steps is None:
        args.steps = int(batch.meta["steps"])
    integrator = batch.meta["integrator"]
    dt = batch.meta["dt"]
    evals_per_step = 1 if integrator == "leapfrog" else 7
    inter_per_eval = batch.interactions_per_eval()

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    sim = nbody.Simulation(batch, prec)
    from paper_1003_3896_amd import autotune
    tile_used = nbody.nbody_get_tile(sim.ctx, prec, autotune.size_class(int(np.diff(batch.offsets).max())))
    e_start = energy_fp64(sim) if args.workload in ("c1", "c2", "c3") else None
    nrows = min(int(batch.offsets[1]), ACCEL_ROWS)
    wall, kms, nlaunch = time_steps(sim, integrator, dt, args.steps, args.warmup, torch)
    e_end = energy_fp64(sim) if e_start is not None else None
    inter = inter_per_eval * evals_per_step * args.steps
    value = inter / wall / 1e9
    pair_ms = kms / max(nlaunch, 1)
    roofline = pair_roofline(prec, inter_per_eval, pair_ms, tile_used, args.workload, equal_masses(batch))
    prof = profile_summary(prec, tile_used, args.workload)
    roofline.update({
        "busy_clock_ghz_profiled": float(prof["busy_clock_ghz"]) if prof and "busy_clock_ghz" in prof else None,
        "issue_counters": issue_counters(prec, tile_used, args.workload),
        "tile": {"k": tile_used[0], "waves_per_group": tile_used[1], "tile": tile_used[2],
                 "blocks_per_cu": tile_used[3], "phased": tile_used[4]},
        "launches": nlaunch,
        "flops_per_interaction": FLOPS_PER_INTERACTION,
        "interactions_per_launch": inter_per_eval,
    })
    a_gpu = sim.acc.cpu().numpy()
    pos_final = sim.pos.cpu().numpy()
    sim.close()

    modes = {}
    if not args.no_modes and args.workload in ("c2", "c3", "c4"):
        others = {"c3": ("fp32ds", "fp32c", "fp32", "fp64"), "c2": ("fp32ds", "fp32c", "fp64"), "c4": ("fp32dl",)}
        for m in others[args.workload]:
            if m == prec:
                continue
            s2 = nbody.Simulation(batch, m)
            a0 = energy_fp64(s2)
            w2, k2, n2 = time_steps(s2, integrator, dt, args.steps, args.warmup, torch)
            modes[m] = {"G_interactions_per_s": round(inter_per_eval * evals_per_step * args.steps / w2 / 1e9, 2),
                        "pair_kernel_ms": round(k2 / max(n2, 1), 4),
                        "energy": dict(drift_report(a0, energy_fp64(s2)), steps=args.steps + args.warmup)}
            s2.close()

    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic (seeded Plummer initial conditions)",
        "config": {
            "workload": batch.meta.get("name", args.workload),
            "n_particles": batch.n,
            "clusters": batch.B,
            "integrator": integrator,
            "dt": dt,
            "eps": float(batch.eps[0]),
            "precision_mode": prec,
            "force_evals_per_step": evals_per_step,
        },
        "pct_fp32_valu_peak": round(100 * value * 1e9 * FLOPS_PER_INTERACTION / (PEAK_FP32_TFLOPS * 1e12), 2),
        "roofline": roofline,
    }
    if e_start is not None:
        # horizon: the warm-up plus the timed steps of this run (not the configuration's full count)
        result["energy"] = dict(drift_report(e_start, e_end), steps=args.steps + args.warmup,
                                measured_in="fp64 library diagnostics")
    if modes:
        result["modes"] = modes
    if args.workload in ("c1", "c2") and not args.no_extras:
        result["ms_per_step_graphs"] = graph_ab(batch, prec, integrator, dt, args.steps, torch)
    if args.workload == "c4" and not args.no_extras:
        bsteps = max(1, min(args.steps, 3))
        el = per_cluster_baseline(batch, integrator, dt, bsteps, torch)
        per = inter_per_eval * evals_per_step * bsteps / el / 1e9
        result["per_cluster_launches"] = {"G_interactions_per_s": round(per, 3), "steps": bsteps,
                                          "batched_over_per_cluster": round(value / per, 2)}
        result["accel_error"] = c4_accuracy(batch, torch)
    if not args.no_cpu_baseline:
        cb, parity = cpu_baseline(batch, pos_final, args.cpu_seconds, a_gpu)
        result["cpu_baseline"] = cb
        result["parity_sample"] = parity
    if args.workload in ("c2", "c3", "c4"):
        result["accel_error_all_particles_vs_fp64"] = dict(
            all_particle_errors(batch, pos_final, [prec] + [m for m in modes if m != "fp64"], torch),
            state="the final state of the timed run")
    if not args.no_cpu_baseline and args.workload in ("c2", "c3"):
        result["accel_error_on_fp64_trajectory"] = sampled_state_errors(
            batch, [prec] + [m for m in modes], integrator, dt, [0, min(args.steps, 100) // 2, min(args.steps, 100)],
            nrows, torch)
    if args.workload == "c3" and not args.no_extras:
        for key, fn in (("c1", lambda: extra_c1(torch)), ("c2", lambda: extra_c2(torch)),
                        ("c4", lambda: extra_c4(torch)), ("c5", lambda: extra_c5(args))):
            print("extras: %s" % key, file=sys.stderr, flush=True)
            result[key] = fn()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
