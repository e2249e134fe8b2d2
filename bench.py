"""Throughput of the dynamic-bonding Langevin MD step on one GPU.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload gel|telechelic|small]

Prints one JSON line: particle-timesteps/s of db_step (bonding sweeps
included) on a synthetic workload already resident on the GPU (the 200k
gel in its bonded state, reached by an untimed equilibration), the roofline
position of the dominant kernel (k_step, timed with HIP events on the stream
it runs on), of the whole step and of the list build and proposal kernels,
the small and telechelic workloads on their own, replicas/hour of a
parameter-sweep batch run by db_step_batch under its autotuned plan against
the same replicas run one by one with db_step, and the FP64 CPU oracle timed
on a bounded sample of the same workload (one core) and of the replicas (all
cores at once).
"""

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_gel200k_traffic.txt")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10000)
    p.add_argument("--warmup", type=int, default=200)
    p.add_argument("--workload", default="gel", choices=["gel", "gel-lattice", "telechelic", "small"])
    p.add_argument("--n", type=int, default=0, help="particle count for the gel workload (default 200000)")
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-steps", type=int, default=20)
    p.add_argument("--equilibrate", type=int, default=5000,
                   help="untimed steps from the initial state before the warm-up (the bonded state is the input)")
    p.add_argument("--tune-steps", type=int, default=200, help="steps per autotuner trial of the batch")
    p.add_argument("--no-other-configs", action="store_true", help="skip the small and telechelic lines")
    p.add_argument("--profile-steps", type=int, default=2000)
    p.add_argument("--skin", type=float, default=None, help="neighbour-list skin (default: the library's)")
    p.add_argument("--step-threads", type=int, default=0,
                   help="threads per particle in the step kernel (0: the library's choice)")
    p.add_argument("--modifier", default="none", choices=["none", "slip", "melt"],
                   help="rate modifier on every reaction: slip bonds (a = 1) or melting with T_melt = kT")
    p.add_argument("--list-batch", type=int, default=0,
                   help="list entries per thread loaded up front in the step kernel (0: the library's choice)")
    p.add_argument("--replicas", type=int, default=1024,
                   help="replicas of the parameter-sweep batch (0 skips the batched-vs-plain measurement)")
    p.add_argument("--replica-steps", type=int, default=20000)
    p.add_argument("--plain-sample", type=int, default=32,
                   help="replicas (spread over the size range) timed one after another with db_step")
    p.add_argument("--plain-steps", type=int, default=2000)
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="first run one plain device-to-device copy of this many MiB (the reference "
                        "kernel that scales rocprofv3 FETCH_SIZE / WRITE_SIZE to bytes)")
    return p.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("device.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2609_21204_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_tag):
    """HBM bytes per k_step launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source and this workload."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    src = re.search(r"kernel_source_hash:\s*(\S+)", text)
    wl = re.search(r"workload:\s*(\S+)", text)
    val = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (src and wl and val) or src.group(1) != kernel_source_hash() or wl.group(1) != workload_tag:
        return None
    return float(val.group(1))


def algorithmic_bytes_per_particle(w):
    """Minimum bytes one k_step launch must move per particle: position and
    velocity read + write (4 x 12 B), the type (1 B), and the 5 B bond slot
    words (4 B partner + 1 B type) the particle's valence and static bonds
    span."""
    import numpy as np
    cap = np.array([t[0] for t in w.types])[w.type_id]
    stat = np.zeros(w.n)
    if len(w.static_pairs):
        np.add.at(stat, w.static_pairs.reshape(-1).astype(np.int64), 1)
    slots = float(np.mean(cap + stat))
    return 48.0 + 1.0 + 5.0 * slots, slots


def sweep_trials_per_particle(w):
    """Reactive-site trials per particle and sweep: every site of a
    reaction's types proposes once per reaction (a homotypic reaction counts
    its type once)."""
    import numpy as np
    t = np.asarray(w.type_id)
    tot = 0
    for r in w.reactions:
        types = {r["type_a"], r["type_b"]}
        tot += int(np.isin(t, list(types)).sum())
    return tot / w.n


def host_cpu():
    """Host CPU as /proc/cpuinfo names it, with the logical CPUs the OS shows
    and those this process may run on."""
    model, mhz = "unknown", None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name") and model == "unknown":
                model = ln.split(":", 1)[1].strip()
            elif ln.startswith("cpu MHz") and mhz is None:
                mhz = float(ln.split(":", 1)[1])
    except (OSError, ValueError):
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return (f"{model}" + (f" @ {mhz:.0f} MHz" if mhz else "")
            + f"; {os.cpu_count()} logical CPUs visible, {usable} usable by this process")


def cpu_baseline(w, state, steps):
    """The FP64 oracle, single-threaded, on `steps` steps of the same
    workload from the state the GPU run reached (positions, velocities and
    bonds read back), so that it times the same bonded state."""
    from threadpoolctl import threadpool_limits
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import oracle_from_workload
    step0, pos, vel, bonds = state
    with threadpool_limits(limits=1):
        o = oracle_from_workload(w)
        o.set_state(step0, pos, vel, bonds[:, :2], bonds[:, 2])
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
    return {"value": w.n * steps / dt, "unit": "particle-timesteps/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu(),
            "sample": f"{steps} FP64 oracle steps of the {w.name} workload (N={w.n}, {steps // w.period} "
                      f"bonding sweeps) from the GPU run's state at step {step0} ({len(bonds)} bonds), "
                      f"one thread, {dt:.1f} s"}


def _oracle_replica_worker(args):
    """One replica run by the oracle for `steps` steps in its own process
    (one thread); returns the seconds it took."""
    root, seed, n, eps, rho, cap, kind, steps = args
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    sys.path.insert(0, root)
    sys.path.insert(0, os.path.join(root, "tests"))
    from helpers import oracle_from_workload
    from paper_2609_21204_amd import inputs
    w = inputs.replica(seed, n, eps, rho, cap, kind)
    o = oracle_from_workload(w)
    t0 = time.perf_counter()
    o.step(steps)
    return time.perf_counter() - t0


def cpu_replica_baseline(a, inputs, steps=100):
    """Oracle replicas/hour on every host core: one oracle process per core
    (at most 16), all running at once, each on one replica of the set
    (replicas spread over the size range), `steps` steps each; the mean time
    of a replica under that load, scaled to the batch's step count, gives
    the all-core rate (and one core's)."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16)
    reps = inputs.replica_set(seed=a.seed, count=a.replicas)
    by_size = sorted(reps, key=lambda w: w.n)
    sample = [by_size[int((k + 0.5) * len(by_size) / cores)] for k in range(cores)]
    jobs = [(ROOT, w.seed, w.n, w.extra["eps"], w.extra["density"], w.extra["cap_b"], w.extra["kind"], steps)
            for w in sample]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        secs = pool.map(_oracle_replica_worker, jobs)
    wall = time.perf_counter() - t0
    per_replica_s = sum(secs) / len(secs) * (a.replica_steps / steps)
    return {"replicas_per_hour_1core": 3600.0 / per_replica_s,
            "replicas_per_hour_all_cores": cores * 3600.0 / per_replica_s,
            "host_cores": cores, "host_cpu": host_cpu(),
            "replica_sample": f"{cores} oracle processes at once, one per core, each one replica (N "
                              f"{min(w.n for w in sample)}..{max(w.n for w in sample)}, spread over the set) for "
                              f"{steps} steps; mean {sum(secs) / len(secs):.2f} s per replica, {wall:.1f} s wall; "
                              f"scaled to {a.replica_steps} steps"}


def copy_bandwidth(torch, mib=1024, reps=10):
    """Achievable HBM bandwidth: a plain device-to-device copy of `mib` MiB
    (far larger than the 256 MB last-level cache), read + write bytes over
    the time of `reps` copies."""
    src = torch.empty(mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del src, dst
    return 2.0 * (mib << 20) * reps / dt / 1e9


def timed_steps(s, torch, k):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(k)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def batch_vs_plain(a, db, inputs, torch):
    """Replicas/hour of the parameter-sweep batch run by db_step_batch (one
    graph, one launch chain per size class) under the plan the autotuner
    picks on these replicas (its trials are ordinary steps of the run and
    are timed separately), against the same replicas run one after another
    with db_step.  The plain cost is measured on a sample spread over the
    size range and scaled to the whole set."""
    reps = inputs.replica_set(seed=a.seed, count=a.replicas)
    n_tot = sum(w.n for w in reps)
    systems = [db.System.from_workload(w) for w in reps]
    hs = [s.h for s in systems]
    try:
        db.db_step_batch(hs, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan, tuned_steps, trial_ms = db.db_batch_autotune(hs, a.tune_steps)
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        db.db_step_batch(hs, a.replica_steps)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        # each size class of the plan alone, for the makespan picture
        classes = []
        lo = 0
        for k, (nmax, thr) in enumerate(plan):
            last = k == len(plan) - 1
            mine = [s.h for s, w in zip(systems, reps) if w.n > lo and (w.n <= nmax or last)]
            lo = nmax
            if not mine:
                continue
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            db.db_step_batch_plan(mine, 1000, plan)
            torch.cuda.synchronize()
            classes.append({"n_max": nmax, "threads": thr, "systems": len(mine),
                            "ms_per_1000_steps_alone": 1000.0 * (time.perf_counter() - t0)})
        by_size = sorted(range(len(reps)), key=lambda k: reps[k].n)
        stride = max(1, len(reps) // max(1, a.plain_sample))
        sample = by_size[stride // 2::stride][:a.plain_sample]
        for k in sample:
            systems[k].step(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in sample:
            systems[k].step(a.plain_steps)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
    finally:
        for s in systems:
            s.close()
    plain_total = tp / len(sample) * len(reps) * (a.replica_steps / a.plain_steps)
    return {
        "replicas": len(reps), "particles": n_tot, "steps": a.replica_steps,
        "batched_s": tb, "batched_replicas_per_hour": len(reps) * 3600.0 / tb,
        "batched_ptps": n_tot * a.replica_steps / tb,
        "plan": plan, "tuning_s": tune_s, "tuning_steps": tuned_steps,
        "tuning_trial_ms": [round(x, 2) for x in trial_ms], "classes": classes,
        "plain_sample": len(sample), "plain_sample_steps": a.plain_steps, "plain_sample_s": tp,
        "plain_s_estimated": plain_total, "plain_replicas_per_hour": len(reps) * 3600.0 / plain_total,
        "speedup": plain_total / tb,
        "equal_accuracy": "bitwise equal to db_step (tests/test_gpu_parity.py::test_batched_systems_match_plain_runs)",
        "workload": "parameter-sweep replicas: N log-uniform in [256, 8192], eps ~ U[2, 10], density ~ U[0.05, 0.4], "
                    "B valence 1/2/4, monomers or telechelic chains",
    }


def other_configs(db, inputs, torch, oracle=True):
    """The small and telechelic workloads on their own (absolute numbers
    only): small over its whole 1000-step run from the initial state (one
    db_step call: for 512 particles its first 200 steps time the grid
    kernels and a batch of one, 100 steps each, and the rest runs on the
    faster), telechelic over 2000 steps after 500 (grid kernels,
    launch-bound).  With `oracle`, the
    FP64 oracle (one thread) on the same starting state: the whole 1000
    small steps, and a 100-step window of telechelic."""
    import numpy as np
    out = {}
    for name, equil, steps, osteps in (("small", 0, 1000, 1000), ("telechelic", 500, 2000, 100)):
        w = inputs.WORKLOADS[name](seed=1)
        with db.System.from_workload(w) as s:
            s.step(equil)
            state = (s.step_count, s.positions(), s.velocities(), s.bonds().astype(np.int64))
            dt = timed_steps(s, torch, steps)
            out[name] = {"n_particles": w.n, "steps": steps, "after_steps": equil,
                         "ms_per_step": 1000.0 * dt / steps, "particle_timesteps_per_s": w.n * steps / dt,
                         # db_step runs long calls on a system of at most 768 particles
                         # on whichever of a batch of one (one workgroup) and the grid
                         # kernels its first long call measured faster
                         "path": "measured: one workgroup or grid kernels" if w.n <= 768 else "grid kernels"}
        if oracle:
            ob = cpu_baseline(w, state, osteps)
            out[name]["oracle_particle_timesteps_per_s"] = ob["value"]
            out[name]["oracle_sample"] = ob["sample"]
    return out


def kernel_roofline(alg_bytes, avg_us):
    gbs = alg_bytes / (avg_us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "alg_bytes": alg_bytes, "avg_us": avg_us}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(spatial sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2609_21204_amd import dybond as db
    from paper_2609_21204_amd import inputs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}))
        sys.exit(1)
    if a.workload == "gel":
        w = inputs.gel(seed=a.seed, n=a.n or 200000)
    elif a.workload == "gel-lattice":
        w = inputs.gel_lattice(seed=a.seed, n=a.n or 200000)
    else:
        w = inputs.WORKLOADS[a.workload](seed=a.seed)
    if a.modifier != "none":
        ndt = w.period * w.dt
        for r in w.reactions:
            if a.modifier == "slip":
                r["slip"] = 1.0
            else:                       # half bound at T_melt = kT: k_on_melt 0, k_off_melt = k_on - k_off
                k_on = r["p_on0"] / ndt
                r["melt"] = (5.0, w.kT, 0.0, k_on - k_on * math.exp(-r["epsilon"]))
    tag = f"{w.name}{w.n // 1000}k"
    if a.calibrate_copy:
        src = torch.empty(a.calibrate_copy << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    copy_gbs = copy_bandwidth(torch)
    s = db.System.from_workload(w, device=0, skin=a.skin)
    if a.step_threads or a.list_batch:
        db.db_set_step_shape(s.h, a.step_threads, a.list_batch)
    # the synthetic input is the workload's bonded state: the random initial
    # placement relaxes and bonds form over the first thousands of steps
    s.step(a.equilibrate)
    s.step(a.warmup)
    b0 = db.db_read_list_builds(s.h)
    elapsed = timed_steps(s, torch, a.steps)
    builds = db.db_read_list_builds(s.h) - b0
    value = w.n * a.steps / elapsed
    ms_per_step = 1000.0 * elapsed / a.steps

    # per-kernel HIP-event timing on the library's stream (graph replay off)
    db.db_kernel_timing(s.h, 1)
    b1 = db.db_read_list_builds(s.h)
    s.step(max(a.profile_steps, 1))
    prof_builds = db.db_read_list_builds(s.h) - b1
    kern = {}
    for name in ("k_step", "k_binr", "k_nlist", "k_propose", "k_claim", "k_kill", "k_finish", "k_break",
                 "k_cell_scan_blocks", "k_scan_bsum", "k_sort_assign", "k_sort_scatter", "k_sort_copyback",
                 "k_clear_counts", "k_bin"):
        cnt, ms = db.db_read_kernel_time(s.h, name)
        if cnt:
            kern[name] = {"launches": cnt, "avg_us": 1000.0 * ms / cnt, "total_ms": ms}
    db.db_kernel_timing(s.h, 0)
    obs = s.observables()
    tpp, qb = db.db_get_step_shape(s.h)
    state = (s.step_count, s.positions(), s.velocities(), s.bonds().astype(np.int64))
    mean_nb = None
    s.close()

    bpp, slots = algorithmic_bytes_per_particle(w)
    trials = sweep_trials_per_particle(w)
    sweep_bpp = 24.0 * trials / w.period
    step_us = kern["k_step"]["avg_us"]
    achieved = bpp * w.n / (step_us * 1e-6) / 1e9
    traffic = measured_traffic(tag)
    whole_gbs = (bpp + sweep_bpp) * w.n / (ms_per_step * 1e-3) / 1e9
    # list build: read each position (12 B), write its list (4 B per entry
    # of 1.7 on average in the gel, plus the count); spread over the builds
    # of the profiled steps (idle launches included in the kernel time)
    nl_bytes = (12.0 + 4.0 * 1.7 + 4.0) * w.n * max(prof_builds, 1)
    nl = kern.get("k_nlist"), kern.get("k_binr")
    sub = {}
    if nl[0]:
        t_us = 1000.0 * (nl[0]["total_ms"] + (nl[1]["total_ms"] if nl[1] else 0.0)) / max(prof_builds, 1)
        sub["k_binr+k_nlist"] = dict(kernel_roofline(nl_bytes / max(prof_builds, 1), t_us),
                                     per="build", builds_per_step=prof_builds / max(a.profile_steps, 1))
    if "k_propose" in kern:
        # one launch per reaction and sweep: 24 B per proposing site (its
        # position, occupancy and the candidates' positions it reads)
        prop_bytes = 24.0 * trials / max(len(w.reactions), 1) * w.n
        sub["k_propose"] = dict(kernel_roofline(prop_bytes, kern["k_propose"]["avg_us"]), per="launch")
    line = {
        "metric": "particle-timesteps/sec with bonding (1 GPU); batched vs plain replicas/hour",
        "value": value,
        "unit": "particle-timesteps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": tag, "n_particles": w.n, "box_L": round(w.L, 4),
                   "types": len(w.types), "reactions": len(w.reactions),
                   "sweep_period": w.period, "dt": w.dt, "kT": w.kT, "gamma": w.gamma,
                   "equilibration_steps": a.equilibrate,
                   "parallelism": "single GPU", **({"modifier": a.modifier} if a.modifier != "none" else {})},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "copy_gbs": copy_gbs,
                     "traffic": traffic,
                     "kernel": "k_step", "kernel_avg_us": step_us, "threads_per_particle": tpp, "list_batch": qb,
                     "alg_bytes_per_particle": bpp, "bond_slots_per_particle": slots,
                     "whole_step": {"alg_bytes_per_particle": bpp + sweep_bpp, "sweep_bytes_per_particle": sweep_bpp,
                                    "achieved": whole_gbs, "frac": whole_gbs / HBM_PEAK_GBS},
                     "other_kernels": sub},
        "kernels": kern,
        "list_builds_per_step": builds / a.steps,
        "state": {"step": state[0], "bonds": obs["n_bonds"].tolist(), "bonded_fraction": obs["bonded_fraction"].tolist(),
                  "T_kin": obs["T_kin"]},
    }
    if a.workload == "gel" and not a.no_other_configs:
        line["other_configs"] = other_configs(db, inputs, torch, oracle=not a.no_cpu_baseline)
    if a.replicas > 0:
        line["batch"] = batch_vs_plain(a, db, inputs, torch)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, state, a.cpu_steps)
        if a.replicas > 0:
            line["cpu_baseline"].update(cpu_replica_baseline(a, inputs))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
