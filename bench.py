"""Benchmark: SU(3) heat-bath + overrelaxation link updates per second on
32^4 lattices, FP32 batched against FP64 single-lattice, on one MI355X.

A step is one sweep (1 Cabibbo-Marinari heat-bath pass with
Kennedy-Pendleton draws + 4 overrelaxation passes, even/odd checkerboard per
direction, plus the fp64 plaquette of the sweep) over every lattice of the
workload.  One link update = one link through one pass, so a 32^4 sweep is
5 * 4 * 32^4 = 20,971,520 link updates.  Inputs are synthetic hot starts
(Haar links from Philox) at beta = 6.0, resident in HBM before timing.

Printed: one JSON line (rank 0) with the headline value (FP32-R12 batched
link updates/s), the FP64 single-lattice figure, the roofline of the
dominant kernel (the overrelaxation phase) from HIP events recorded around
each run of same-kind phase launches, and the FP64 CPU oracle timed on a
bounded sample, together with its timings on bounded samples of every
workload configuration at 1 and all host threads.  Extra reports: HMC at
32^4, a multiscale step (16^4 -> 32^4 prolongation, rethermalization,
flow), the Wilson flow and the 48-lattice batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LINK_BYTES = {"fp64": 144, "fp32": 72, "fp32_r12": 48}
PHASE_RECORDS = 9  # 8 link records read + 1 written per updated link (4V reads + V/2 writes per phase)
# Sources that determine the phase kernel's code; the committed counter
# summary records their hash, and its HBM traffic is reported only while
# they are unchanged.
KERNEL_SOURCES = ["paper_1510_04675_amd/csrc/phase.hpp", "paper_1510_04675_amd/csrc/device.hpp",
                  "paper_1510_04675_amd/csrc/kernels.hpp", "paper_1510_04675_amd/csrc/k_phase_f32.hip",
                  "paper_1510_04675_amd/csrc/k_phase_f64.hip", "paper_1510_04675_amd/build.py"]
TRAFFIC_SUMMARY = "profiles/k_phase_hb_or_32x4.md"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_variant(m, torch, prec, n_lat, dims, steps, warmup, beta=6.0, n_or=4, streaming_steps=5):
    """Time `steps` sweeps of n_lat lattices as one batched call (one graph
    of `steps` sweeps, replayed; the graph is built by an untimed call of the
    same size first), then the same number of one-sweep calls with HIP events
    between them (median per call, host round trip included), then more
    sweeps launched eagerly with HIP events to get kernel durations."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    fields = [m.Field(dims, prec) for _ in range(n_lat)]
    for i, f in enumerate(fields):
        m.su3_init_hot(f, 3, i)
    params = m.hb_params(n_or=n_or, n_hb_hits=1, hb_max_tries=64, reunit_every=10 if prec != "fp64" else 0)
    betas = [beta] * n_lat
    seeds = [3] * n_lat
    lids = list(range(n_lat))
    sweep = 0
    plaq_first = None
    warm_sweeps = 0
    for _ in range(max(warmup, 1)):
        pw = m.su3_batch_sweep_hb_or(fields, betas, seeds, lids, sweep, 1, params)
        if plaq_first is None:
            plaq_first = float(pw[0, 0])
        sweep += 1
        warm_sweeps += 1
    # untimed call of the timed call's size: builds its graph
    m.su3_batch_sweep_hb_or(fields, betas, seeds, lids, sweep, steps, params)
    sweep += steps
    warm_sweeps += steps
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    plaq = m.su3_batch_sweep_hb_or(fields, betas, seeds, lids, sweep, steps, params)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    sweep += steps
    # one sweep per call: events at the call boundaries (each call ends with
    # a synchronization of the fields' stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        m.su3_batch_sweep_hb_or(fields, betas, seeds, lids, sweep, 1, params)
        ev[i + 1].record(stream)
        sweep += 1
    torch.cuda.synchronize()
    step_ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    # kernel durations: same kernels launched eagerly with events around each
    # run of same-kind phases (heat bath, overrelaxation, plaquette)
    m.su3_profile_enable(True)
    for _ in range(steps):
        m.su3_batch_sweep_hb_or(fields, betas, seeds, lids, sweep, 1, params)
        sweep += 1
    torch.cuda.synchronize()
    hb_ms, hb_n = m.su3_profile_read(0)
    or_ms, or_n = m.su3_profile_read(1)
    pl_ms, pl_n = m.su3_profile_read(2)
    m.su3_profile_enable(False)
    stream_or_us = None
    if n_lat > 1 and streaming_steps > 0:
        # the same kernels with the batch swept phase by phase (one launch
        # over all lattices, n_lat x the last-level cache's worth of links):
        # the overrelaxation launch then streams from HBM
        m.su3_set_group_bytes(0)
        m.su3_profile_enable(True)
        for _ in range(streaming_steps):
            m.su3_batch_sweep_hb_or(fields, betas, seeds, lids, sweep, 1, params)
            sweep += 1
        torch.cuda.synchronize()
        s_ms, s_n = m.su3_profile_read(1)
        m.su3_profile_enable(False)
        m.su3_set_group_bytes(224 << 20)
        stream_or_us = 1e3 * s_ms / max(s_n, 1)
    updates = (1 + n_or) * 4 * V * n_lat * steps
    cfg = m.su3_get_config(fields)
    out = {
        "prec": prec, "n_lat": n_lat, "launch": cfg, "wall_s": wall, "event_ms": ev_ms,
        "ms_per_step": wall * 1e3 / steps, "updates_per_s": updates / wall,
        "step_ms_median": step_ms[len(step_ms) // 2], "step_ms_min": step_ms[0], "warmup_sweeps": warm_sweeps,
        "streaming_or_kernel_us": stream_or_us,
        # algorithmic bytes of one step: 9 link records per link update
        "bytes_per_step": (1 + n_or) * 4 * V * n_lat * PHASE_RECORDS * LINK_BYTES[prec],
        "hb_kernel_us": 1e3 * hb_ms / max(hb_n, 1), "or_kernel_us": 1e3 * or_ms / max(or_n, 1),
        "plaq_kernel_us": 1e3 * pl_ms / max(pl_n, 1),
        "hb_launches": hb_n, "or_launches": or_n, "plaq_last": float(plaq[-1].mean()),
        "phase_links": V // 2 * n_lat, "plaq_first": plaq_first,
        # algorithmic bytes of all overrelaxation launches of the profiled steps
        "or_bytes_total": steps * n_or * 8 * (V // 2 * n_lat) * PHASE_RECORDS * LINK_BYTES[prec],
        "sweeps_per_s": n_lat * steps / wall,
        # heat-bath link updates per second of heat-bath kernel time
        "hb_updates_per_s": steps * 8 * (V // 2 * n_lat) / max(1e-3 * hb_ms, 1e-12),
    }
    for f in fields:
        f.close()
    return out


def run_hmc(m, torch, dims, n_traj=20, n_steps=40, beta=6.0, therm=200, prec="fp32"):
    """HMC on one lattice: cold start + `therm` HB+OR sweeps at beta (seed 5),
    then n_traj unit trajectories of n_steps leapfrog steps (fp32 molecular
    dynamics, fp64 Hamiltonian and Metropolis test)."""
    f = m.Field(dims, prec)
    m.su3_init_cold(f)
    m.su3_sweep_hb_or(f, beta, 5, 0, 0, therm, m.hb_params(n_or=4, reunit_every=10), record=False)
    # deviation from fp64: one trajectory of the same start in both precisions
    a32, a64 = m.Field(dims, prec), m.Field(dims, "fp64")
    m.su3_field_copy(a32, f)
    m.su3_field_copy(a64, f)
    _, dh32 = m.su3_hmc_trajectory(a32, beta, 1.0, n_steps, 5, 0, 10**6, 0)
    _, dh64 = m.su3_hmc_trajectory(a64, beta, 1.0, n_steps, 5, 0, 10**6, 0)
    a32.close()
    a64.close()
    m.su3_hmc_trajectory(f, beta, 1.0, n_steps, 5, 0, 10**6 + 1, 1)  # warm-up (allocates the field's scratch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dh, acc = [], 0
    for t in range(n_traj):
        a, d = m.su3_hmc_trajectory(f, beta, 1.0, n_steps, 5, 0, t, 1)
        acc += a
        dh.append(d)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    import math
    out = {"lattice": f"{dims[0]}^4", "beta": beta, "tau": 1.0, "n_steps": n_steps, "trajectories": n_traj,
           "precision": f"{prec} molecular dynamics, fp64 Hamiltonian", "trajectories_per_s": round(n_traj / wall, 3),
           "ms_per_trajectory": round(1e3 * wall / n_traj, 3), "acceptance": acc / n_traj,
           "mean_dH": round(sum(dh) / n_traj, 5), "mean_exp_minus_dH": round(sum(math.exp(-x) for x in dh) / n_traj, 5),
           "plaquette": round(m.su3_plaquette(f), 8),
           "dH_same_start": {prec: dh32, "fp64": dh64, "abs_dev": abs(dh32 - dh64)},
           "start": f"cold + {therm} HB+OR sweeps at beta {beta}"}
    f.close()
    return out


def run_multiscale(m, torch, L=32, beta_c=5.7, beta=6.0, n_coarse=20, n_sweeps=20, every=4):
    """One multiscale step at L^4: a coarse (L/2)^4 hot start (seed 11)
    thermalized by n_coarse sweeps at beta_c, prolongated (c = 0.05,
    tolerance 1e-5) in fp64, rounded to R12 and rethermalized at beta; reports
    the stage times and the displaced 2x2 loops (their spread measures how far
    translational symmetry is from restored)."""
    c = m.Field([L // 2] * 4, "fp64")
    m.su3_init_hot(c, 11, 0)
    m.su3_sweep_hb_or(c, beta_c, 11, 0, 0, n_coarse, m.hb_params(n_or=4), record=False)
    f64 = m.Field([L] * 4, "fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = m.su3_prolongate(c, f64, 0.05, 1e-5, 10000)
    torch.cuda.synchronize()
    t_pro = time.perf_counter() - t0
    t0 = time.perf_counter()
    dl = m.su3_displaced_loops(f64)
    t_loops = time.perf_counter() - t0
    f = m.Field([L] * 4, "fp32_r12")
    m.su3_field_copy(f, f64)
    f64.close()
    c.close()
    curve = [[0, float(dl.max() - dl.min())]]
    # a call without sweeps runs the launch-shape autotuner (when enabled)
    # for this field shape, outside the timed rethermalization
    m.su3_sweep_hb_or(f, beta, 11, 0, 1000, 0, m.hb_params(n_or=4, reunit_every=10), record=False)
    t_sw = 0.0
    for k in range(0, n_sweeps, every):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.su3_sweep_hb_or(f, beta, 11, 0, 1000 + k, every, m.hb_params(n_or=4, reunit_every=10), record=False)
        torch.cuda.synchronize()
        t_sw += time.perf_counter() - t0
        d = m.su3_displaced_loops(f)
        curve.append([k + every, float(d.max() - d.min())])
    # measurement after flow of the rethermalized field, R12 against FP64 from
    # the same links: adaptive flow (tolerance 0.01, maximum step 0.2) to t = 1
    g = m.Field([L] * 4, "fp64")
    m.su3_field_copy(g, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E12, Q12, na, nr = m.su3_wilson_flow_adaptive(f, 1.0, 0.01, 0.2, 0.01, [0.5, 1.0])
    torch.cuda.synchronize()
    t_flow = time.perf_counter() - t0
    E64, Q64, _, _ = m.su3_wilson_flow_adaptive(g, 1.0, 0.01, 0.2, 0.01, [0.5, 1.0])
    p12, p64 = m.su3_plaquette(f), m.su3_plaquette(g)
    g.close()
    out = {"coarse": f"{L // 2}^4 hot start (seed 11), {n_coarse} sweeps at beta {beta_c}",
           "fine": f"{L}^4, R12 rethermalization at beta {beta}",
           "flow_to_t1_ms_r12": round(1e3 * t_flow, 2), "flow_steps": [na, nr],
           "after_flow_r12_vs_fp64": {"plaquette": [p12, p64, abs(p12 - p64)], "E": [float(E12[-1]), float(E64[-1])],
                                      "Q": [float(Q12[-1]), float(Q64[-1]), abs(float(Q12[-1] - Q64[-1]))]},
           "prolongation_ms": round(1e3 * t_pro, 2), "ape_steps_per_stage": [int(x) for x in iters],
           "displaced_loops_ms": round(1e3 * t_loops, 3),
           "displaced_2x2_after_prolongation": [round(float(x), 6) for x in dl],
           "displaced_spread_vs_sweeps": curve,
           "rethermalization_sweeps_per_s": round(n_sweeps / t_sw, 1)}
    f.close()
    return out


def run_flow(m, torch, L=32, n_steps=20, eps=0.02):
    """Fixed-step RK3 Wilson flow (Sec. IV.B) of a thermalized L^4 lattice in
    R12 and FP64: ms per flow step and the flow stage kernel against 8 TB/s.
    Algorithmic bytes per link of one step: the first stage reads W and
    writes W' and X (8 reals), the other two also read X; a link record is
    rec bytes, so 3 (2 rec) + 8 r (1 + 2 + 2) with r the real size
    (R12: 448 B, FP64: 1184 B); the staple neighbours are counted as the
    field read once."""
    out = {}
    base = m.Field([L] * 4, "fp32_r12")
    m.su3_init_cold(base)
    m.su3_sweep_hb_or(base, 6.0, 9, 0, 0, 50, m.hb_params(n_or=4, reunit_every=10), record=False)
    for prec, rec, r in (("fp32_r12", 48, 4), ("fp64", 144, 8)):
        f = m.Field([L] * 4, prec)
        m.su3_field_copy(f, base)
        m.su3_wilson_flow(f, eps, 1)  # allocates the flow buffers
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.su3_wilson_flow(f, eps, n_steps)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / n_steps
        links = 4 * L ** 4
        alg = links * (3 * 2 * rec + 8 * r * 5)
        out[prec] = {"ms_per_step": round(ms, 4), "algorithmic_bytes_per_step": alg,
                     "achieved_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
                     "frac_of_8TBps": round(alg / (ms * 1e-3) / 8e12, 4),
                     "plaquette_after": m.su3_plaquette(f), "Q_after": m.su3_topological_charge(f)}
        f.close()
    base.close()
    out["flow"] = f"{n_steps} RK3 steps of eps {eps} from a {L}^4 lattice (cold start + 50 R12 sweeps at beta 6.0)"
    return out


def run_batch48(m, torch, prec="fp32", n_sweeps=100):
    """48 prolongated lattices of uneven sizes (16 each of 12^4, 16^4, 20^4),
    beta_i uniform in [5.9, 6.2] (numpy PCG64 seed 4), coarse (L/2)^4 hot
    starts (seed 4, lattice id i) with 20 sweeps at beta_i - 0.36, then
    n_sweeps HB+OR sweeps of all 48 in one batched graph launch."""
    import synth_inputs as si
    sizes = [12] * 16 + [16] * 16 + [20] * 16
    betas = si.batch_betas(48, 4)
    fields = []
    for i, L in enumerate(sizes):
        c = m.Field([L // 2] * 4, "fp64")
        m.su3_init_hot(c, 4, i)
        m.su3_sweep_hb_or(c, betas[i] - 0.36, 4, i, 0, 20, m.hb_params(n_or=4), record=False)
        f = m.Field([L] * 4, prec)
        m.su3_prolongate(c, f, 0.05, 1e-5, 10000)
        c.close()
        fields.append(f)
    p = m.hb_params(n_or=4, reunit_every=10)
    m.su3_batch_sweep_hb_or(fields, betas, [4] * 48, list(range(48)), 0, n_sweeps, p)  # builds the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = m.su3_batch_sweep_hb_or(fields, betas, [4] * 48, list(range(48)), n_sweeps, n_sweeps, p)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    links = sum(4 * L**4 for L in sizes)
    out = {"lattices": "16 x 12^4 + 16 x 16^4 + 16 x 20^4", "links": links, "storage": prec, "sweeps": n_sweeps,
           "seconds": round(dt, 4), "link_updates_per_s": round(5 * links * n_sweeps / dt, 1),
           "plaquette_last_sweep_by_beta": [[round(float(b), 4), round(float(x), 6)]
                                            for b, x in sorted(zip(betas, h[-1]))][::8]}
    for f in fields:
        f.close()
    return out


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def launch_str(c):
    return f"{c['block']},{c['xcd_remap']},{c['ty']},{c['tz']},{c['tt']}"


def recorded_traffic(v, lattice):
    """HBM bytes per launch of the OR phase kernel (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, each scaled by a plain copy's reading), from the committed
    summary, if it was taken with these kernel sources, this workload and this
    launch shape; otherwise None."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_SUMMARY)) as fh:
            recs = [json.loads(line.split(":", 1)[1]) for line in fh if line.startswith("traffic-record:")]
    except (OSError, ValueError):
        return None
    sha = kernel_sources_hash()
    for rec in recs:
        if (rec.get("sources_sha256") == sha and rec.get("launch") == launch_str(v["launch"])
                and rec.get("prec") == v["prec"] and rec.get("n_lat") == v["n_lat"] and rec.get("lattice") == lattice):
            return rec.get("hbm_bytes_per_launch")
    return None


def roofline(v, lattice=32):
    # a batch may be swept in lattice groups, one launch per group and phase:
    # bytes per launch = all overrelaxation bytes / overrelaxation launches
    per_launch = v["or_bytes_total"] / max(v["or_launches"], 1)
    achieved = per_launch / (v["or_kernel_us"] * 1e-6) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(v, lattice),
           "traffic_unit": "bytes per launch", "traffic_source": TRAFFIC_SUMMARY,
           "kernel": f"k_phase<{v['prec']}, OR>", "algorithmic_bytes_per_launch": round(per_launch),
           "avg_launch_us": round(v["or_kernel_us"], 2)}
    if v["n_lat"] > 1:
        out["note"] = ("batch swept in lattice groups of at most 224 MiB: each lattice stays in the 256 MB "
                       "last-level cache across its phases, so this launch is cache-resident; "
                       "'streaming' is the same kernel with the batch swept phase by phase from HBM")
        if v.get("streaming_or_kernel_us"):
            # one launch over all lattices: n_lat lattices' bytes per launch
            s_bytes = per_launch * v["n_lat"]
            s_ach = s_bytes / (v["streaming_or_kernel_us"] * 1e-6) / 1e9
            out["streaming"] = {"achieved": round(s_ach, 1), "frac": round(s_ach / HBM_PEAK_GBS, 4),
                                "avg_launch_us": round(v["streaming_or_kernel_us"], 2),
                                "algorithmic_bytes_per_launch": round(s_bytes)}
    return out


def sweep_level(v):
    """The whole step against the roofline: algorithmic bytes of all its
    phases (9 link records per link update) over the measured step time."""
    ach = v["bytes_per_step"] / (v["ms_per_step"] * 1e-3) / 1e9
    return {"algorithmic_bytes_per_step": v["bytes_per_step"], "achieved": round(ach, 1), "unit": "GB/s",
            "peak": HBM_PEAK_GBS, "frac": round(ach / HBM_PEAK_GBS, 4),
            "step_ms_mean": round(v["ms_per_step"], 4),
            "one_sweep_per_call": {
                "step_ms_median": round(v["step_ms_median"], 4),
                "frac_at_median": round(v["bytes_per_step"] / (v["step_ms_median"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def cpu_baseline(dims, threads, n_sweeps=4):
    """The FP64 oracle (as it stands) on n_sweeps sweeps (1 HB + 4 OR) of one
    lattice of the benchmark's shape from a hot start (about 10-15 s on 16
    host threads); the hot start is not timed."""
    import oracle
    oracle.set_threads(threads)
    U = oracle.init_hot(dims, 3, 0)
    t0 = time.perf_counter()
    oracle.sweep_hb_or(dims, U, 6.0, 3, 0, 0, n_sweeps, n_or=4)
    dt = time.perf_counter() - t0
    V = dims[0] * dims[1] * dims[2] * dims[3]
    return {"value": round(n_sweeps * 5 * 4 * V / dt, 1), "unit": "link updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_sweeps} sweeps (1 HB + 4 OR) of one {dims[0]}^4 FP64 lattice from a hot start, "
                      f"{threads} OpenMP threads, {dt:.1f} s"}


def oracle_timing(threads_list=(1, 16)):
    """The FP64 oracle (as it stands) on bounded samples of each workload
    configuration, host only, at each thread count: measured seconds and the
    full configuration extrapolated from the sample (per sweep for sweeps, per
    step for the prolongation and the flow, by volume for HMC).  Prints one
    progress line per item."""
    import oracle

    def cpu_model():
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
        except OSError:
            pass
        return "unknown"

    def timed(fn):
        t0 = time.perf_counter()
        r = fn()
        return time.perf_counter() - t0, r

    out = {"host": {"cpu": cpu_model(), "logical_cpus": os.cpu_count()}, "runs": []}
    for th in threads_list:
        oracle.set_threads(th)

        def rec(config, sample, secs, full_secs, how):
            out["runs"].append({"threads": th, "config": config, "sample": sample, "seconds": round(secs, 3),
                                "full_config_seconds": round(full_secs, 1), "extrapolation": how})
            log(f"bench: oracle {th} thread(s) {config}: {secs:.2f} s for {sample}; full config ~{full_secs:.1f} s")

        d4, d8, d16 = [4] * 4, [8] * 4, [16] * 4
        U = oracle.init_hot(d4, 1, 0)
        t, _ = timed(lambda: oracle.sweep_hb_or(d4, U, 6.0, 1, 0, 0, 10, n_or=4))
        rec("C1 4^4 FP64, 10 sweeps", "the whole configuration", t, t, "none")
        U = oracle.init_cold(d16)
        t, _ = timed(lambda: oracle.sweep_hb_or(d16, U, 6.0, 2, 0, 0, 5, n_or=4))
        rec("C2 16^4 cold, 200 sweeps", "5 sweeps", t, t * 40, "x40 sweeps")
        Uc = oracle.init_hot(d8, 7, 0)
        t1, _ = timed(lambda: oracle.sweep_hb_or(d8, Uc, 5.8, 7, 0, 0, 20, n_or=4))
        its = (156, 69, 39)  # steps the paper's tolerance takes on this input
        t2, _ = timed(lambda: oracle.prolongate(d8, Uc, 0.05, 1e-5, 10))
        Uf, _ = oracle.prolongate(d8, Uc, 0.05, 1e-5, 1)
        t3, _ = timed(lambda: oracle.sweep_hb_or(d16, Uf, 6.0, 7, 0, 100, 5, n_or=4))
        t4, _ = timed(lambda: oracle.wilson_flow(d16, Uf, 0.01, 5))
        rec("C3 8^4 x 100 sweeps -> prolongation -> 16^4 x 50 sweeps -> 100 flow steps",
            "20 coarse sweeps, 10 steps per prolongation stage, 5 fine sweeps, 5 flow steps",
            t1 + t2 + t3 + t4, t1 * 5 + t2 * sum(its) / 30 + t3 * 10 + t4 * 20,
            "coarse sweeps x5, prolongation x(156+69+39)/30 steps, fine sweeps x10, flow x20")
        tot, tsample = 0.0, 0.0
        for L in (12, 16, 20):
            dl = [L] * 4
            U = oracle.init_hot(dl, 4, 0)
            t, _ = timed(lambda: oracle.sweep_hb_or(dl, U, 6.0, 4, 0, 0, 2, n_or=4))
            tsample += t
            tot += t * 50 * 16
        rec("C4 16 x (12^4, 16^4, 20^4), 100 sweeps", "2 sweeps of one lattice per size", tsample, tot,
            "x50 sweeps x16 lattices per size")
        rate = 5 * 4 * 16 ** 4 * 5 / max(t3, 1e-9)  # link updates/s of the 16^4 sweeps of C3
        rec("M0 32^4, 1 sweep (1 HB + 4 OR)", "no run: the 16^4 sweep rate of C3", 0.0, 5 * 4 * 32 ** 4 / rate,
            "by link updates at the 16^4 rate")
        U = oracle.init_cold(d8)
        oracle.sweep_hb_or(d8, U, 6.0, 5, 0, 0, 5, n_or=4)
        t, _ = timed(lambda: oracle.hmc_trajectory(d8, U, 6.0, 1.0, 40, 5, 0, 0, 0))
        rec("C5 32^4 HMC, 20 trajectories of 40 steps", "one 8^4 trajectory", t, t * 256 * 20, "x256 volume x20")
    return out


def copy_calibration(torch, gib=1.0):
    """A plain device-to-device copy of known size (for scaling HBM counters)."""
    n = int(gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lattice", type=int, default=32)
    ap.add_argument("--batch", type=int, default=4, help="lattices in the FP32 batched run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="", help="comma list of parts to run (fp64,fp32,fp32_r12,fp32_batch,r12_batch,hmc,multiscale,flow,batch48)")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="time the oracle on bounded samples of each configuration (host only) and exit")
    ap.add_argument("--no-oracle-configs", action="store_true",
                    help="skip the oracle's per-configuration timing in the bench line")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--no-hmc", action="store_true", help="skip the HMC report")
    ap.add_argument("--no-hmc-r12", action="store_true", help="skip the HMC run with 12-real links")
    ap.add_argument("--no-multiscale", action="store_true", help="skip the prolongation / displaced-loop report")
    ap.add_argument("--no-batch48", action="store_true", help="skip the 48-lattice batched run")
    ap.add_argument("--no-flow", action="store_true", help="skip the Wilson flow report")
    ap.add_argument("--launch", default="", help="fix the launch shape block,xcd_remap,ty,tz,tt (implies --no-tune)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(independent lattices would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)
    if a.oracle_timing:  # host only: no GPU needed
        print(json.dumps({"oracle_timing": oracle_timing()}), flush=True)
        return
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import paper_1510_04675_amd as m
    m.lib()
    if a.copy_calibration:
        copy_calibration(torch)
        return
    L = a.lattice
    dims = [L, L, L, L]
    if a.launch:
        b, r, ty, tz, tt = (int(x) for x in a.launch.split(","))
        m.su3_set_launch(b, r)
        m.su3_set_tile(ty, tz, tt)
    m.su3_autotune(not (a.no_tune or a.launch))
    want = set(a.only.split(",")) if a.only else {"fp64", "fp32", "fp32_r12", "fp32_batch", "r12_batch"}
    res = {}
    plan = [("fp64", "fp64", 1), ("fp32", "fp32", 1), ("fp32_r12", "fp32_r12", 1),
            ("fp32_batch", "fp32", a.batch), ("r12_batch", "fp32_r12", a.batch)]
    for name, prec, n in plan:
        if name not in want:
            continue
        log(f"bench: {name} ({n} x {L}^4) ...")
        res[name] = run_variant(m, torch, prec, n, dims, a.steps, a.warmup)
        log(f"bench: {name}: {res[name]['updates_per_s']:.3e} link updates/s, "
            f"OR kernel {res[name]['or_kernel_us']:.1f} us, HB kernel {res[name]['hb_kernel_us']:.1f} us, "
            f"plaquette kernel {res[name]['plaq_kernel_us']:.1f} us")
    head = res.get("r12_batch") or next(iter(res.values()), None)
    hmc = None
    if not a.no_hmc and (not a.only or "hmc" in want):
        log("bench: hmc (32^4, tau 1, 40 steps, 20 trajectories) ...")
        hmc = run_hmc(m, torch, dims)
        log(f"bench: hmc {hmc['trajectories_per_s']} traj/s, acceptance {hmc['acceptance']}")
        if not a.no_hmc_r12:
            # the same run with 12-real links (re-orthonormalized at every drift)
            r12 = run_hmc(m, torch, dims, prec="fp32_r12")
            hmc["fp32_r12_links"] = {k: r12[k] for k in ("trajectories_per_s", "acceptance", "mean_dH",
                                                          "dH_same_start")}
            log(f"bench: hmc r12 {r12['trajectories_per_s']} traj/s, dH vs fp64 from the same start "
                f"{r12['dH_same_start']['abs_dev']:.2e}")
    ms = None
    if not a.no_multiscale and (not a.only or "multiscale" in want):
        log("bench: multiscale (16^4 -> 32^4 prolongation, displaced loops) ...")
        ms = run_multiscale(m, torch, L)
        log(f"bench: prolongation {ms['prolongation_ms']} ms, displaced spread {ms['displaced_spread_vs_sweeps']}")
    fl = None
    if not a.no_flow and (not a.only or "flow" in want):
        log("bench: Wilson flow (32^4, R12 and FP64, 20 RK3 steps) ...")
        fl = run_flow(m, torch, L)
        log("bench: flow " + ", ".join(f"{k} {v['ms_per_step']} ms/step ({v['frac_of_8TBps']:.2f} of 8 TB/s)"
                                       for k, v in fl.items() if isinstance(v, dict)))
    b48 = None
    if not a.no_batch48 and (not a.only or "batch48" in want):
        log("bench: 48 prolongated lattices (12^4, 16^4, 20^4), 100 sweeps in one graph ...")
        b48 = {prec: run_batch48(m, torch, prec) for prec in ("fp32", "fp32_r12")}
        log("bench: batch48 " + ", ".join(f"{k} {v['link_updates_per_s']:.3e} link updates/s" for k, v in b48.items()))
    if head is None:  # only the HMC / multiscale / batch48 parts were asked for
        print(json.dumps({"hmc": hmc, "multiscale": ms, "flow": fl, "batch48": b48}), flush=True)
        return
    cpu = None
    if not a.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        log(f"bench: cpu baseline (oracle, {threads} threads) ...")
        cpu = cpu_baseline(dims, threads)
        log(f"bench: cpu baseline {cpu['value']:.3e} link updates/s")
    orc_cfg = None
    if not (a.no_cpu_baseline or a.no_oracle_configs):
        thr = min(16, os.cpu_count() or 1)
        log(f"bench: oracle per configuration (bounded samples, 1 and {thr} threads) ...")
        try:
            orc_cfg = oracle_timing((1, thr) if thr > 1 else (1,))
        except Exception as e:  # the bench line is printed regardless
            orc_cfg = {"error": repr(e)}
    line = {
        "metric": "SU(3) link updates/s (HB+OR, 32^4) FP32-batched vs FP64; % HBM roofline",
        "value": round(head["updates_per_s"], 1),
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "timing": (f"the {a.steps} steps are one call of {a.steps} sweeps (a replayed HIP graph) between two "
                   f"synchronizations; its graph is built by an untimed call of the same size after the "
                   f"{a.warmup} warm-up sweeps"),
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head["prec"] != "fp64" else "f64",
        "data": "synthetic (Haar hot start from Philox seed 3, beta 6.0)",
        "config": {"workload": f"HB+OR sweeps (1 HB + 4 OR), {head['n_lat']} x {L}^4, {head['prec']} links",
                   "lattice": f"{L}^4", "n_lattices": head["n_lat"], "storage": head["prec"], "beta": 6.0,
                   "n_or": 4, "sampler": "Kennedy-Pendleton", "parallelism": "single GPU"},
        "roofline": roofline(head, L),
        "sweep_roofline": sweep_level(head),
        "cpu_baseline": cpu,
        "variants": {k: {"link_updates_per_s": round(v["updates_per_s"], 1), "ms_per_step": round(v["ms_per_step"], 4),
                         "or_kernel_us": round(v["or_kernel_us"], 2), "hb_kernel_us": round(v["hb_kernel_us"], 2),
                         "plaq_kernel_us": round(v["plaq_kernel_us"], 2),
                         "sweeps_per_s": round(v["sweeps_per_s"], 2),
                         "hb_kernel_link_updates_per_s": round(v["hb_updates_per_s"], 1),
                         "first_sweep_plaquette_lattice0": v["plaq_first"],
                         "or_hbm_frac": roofline(v, L)["frac"], "plaq_after": round(v["plaq_last"], 8),
                         "step_ms_median": round(v["step_ms_median"], 4),
                         "sweep_frac": sweep_level(v)["frac"],
                         "launch": v["launch"]}
                     for k, v in res.items()},
    }
    if orc_cfg is not None:
        line["oracle_configs"] = orc_cfg
    if hmc is not None:
        line["hmc"] = hmc
    if ms is not None:
        line["multiscale"] = ms
    if fl is not None:
        line["flow"] = fl
    if b48 is not None:
        line["batch48"] = b48
    if "fp64" in res:
        # every variant's lattice 0 starts from the same hot start and draws the
        # same uniforms, so its first sweep is comparable with the fp64 one
        p64 = res["fp64"]["plaq_first"]
        line["first_sweep_plaquette_dev_vs_fp64"] = {k: abs(v["plaq_first"] - p64) for k, v in res.items()
                                                      if k != "fp64" and p64 is not None and v["plaq_first"] is not None}
        line["fp64_single_link_updates_per_s"] = round(res["fp64"]["updates_per_s"], 1)
        line["speedup_fp32_batched_vs_fp64"] = round(head["updates_per_s"] / res["fp64"]["updates_per_s"], 3)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
