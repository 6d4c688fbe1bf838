#!/usr/bin/env python3
"""Throughput of the fused D2Q9 thermal pseudopotential LB step on one GPU.

Workload: the 2048 x 2048 flat two-phase slab (liquid in the middle half,
Carnahan-Starling EOS at 0.85 T_c, walls at 0.80 T_c and 0.90 T_c, periodic
in x), corrected temperature treatment (Eq. (24)), EOS at the local
temperature, distributions stored in FP32 with a per-node density reference
(the storage form that meets the FP64 oracle's tolerances).  A step is the
fused update (moments, psi, force, collision of f and g, streaming with
bounce-back walls); the library runs two steps per launch (the two-step
kernel) unless `--no-pair`; the FP64 reduction check runs every 100 steps
(an even interval, so no pair straddles a check) and the FP64 moments are
exported once at the end of the timed region.

Prints one JSON line.  `value` is MLUPS (lattice updates per second / 1e6)
with the state resident in HBM.  `roofline` prices the dominant kernel's
algorithmic bytes (18 distributions read + written per node and step, 144
B in FP32, times the steps per launch) against the 8 TB/s HBM peak, gives
the launch time measured with HIP events on the launch stream (its own
100-step warm-up, then the median of five runs of 200 launches, with their
min and max, whatever --steps is; this leg runs first, so the timed region
also starts on a warm device), and the counter-measured HBM
bytes per launch (`traffic`, from the profile summary while the kernel and
tiling sources are unchanged) with the rate they imply (`measured_GBs`);
`cpu_baseline` times the FP64 oracle on the host cores over a bounded
number of steps of the same workload, and again on one core
(`single_core`, a child process with one OpenMP thread).  Side sections:
`by_precision` (FP64 and FP32 global-shift storage on the same slab,
timed like the roofline leg), `by_treatment` (the slab with each of the
three temperature treatments), `small_lattices` (64^2 and 256^2 droplets,
latency-bound), `interface_jump` (the slab's temperature
jump across its interfaces after 20,000 steps of each treatment, the
forcing-term effect of Eq. (23)), `batched` (256 uneven lattices stepped
together, autotuned, against the same lattices one at a time in the same
storage form and in FP64) and
`steady_state` (wall time of held-out steady-state solves to a 1e-8
residual: one lattice at a time, batched, warm-started, and started at
rest in the forcing scheme's velocity).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALG_BYTES = {"fp32local": 144, "fp32dev": 144, "fp64": 288}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_traffic_wall_slab_2048.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1405_2232_amd", "csrc", f)
                  for f in ("lbm_device.hip", "lbm_device.h", "lbm_api.hip")]
# (lbm_api.hip holds the default tilings: a changed tiling changes the traffic)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fp:
            h.update(fp.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--nx", type=int, default=2048)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--precision", default="fp32local", choices=sorted(ALG_BYTES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extra", action="store_true", help="skip the FP64/FP32-global side runs")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-lattice batch section")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--no-steady", action="store_true", help="skip the steady-state (residual) section")
    ap.add_argument("--no-jump", action="store_true", help="skip the interface temperature jump section")
    ap.add_argument("--jump-steps", type=int, default=20000)
    ap.add_argument("--steady-cases", type=int, default=8)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run the plain copy kernel 10 times on BYTES (counter calibration)")
    ap.add_argument("--no-pair", action="store_true",
                    help="one step per launch (the two-step kernel off)")
    ap.add_argument("--traffic-out", default=TRAFFIC_FILE,
                    help="where --traffic-from writes its summary")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="only summarise two rocprofv3 --pmc runs of this script (FETCH_SIZE, "
                         "then WRITE_SIZE) into the step kernel's HBM traffic file")
    return ap.parse_args()


def copy_rate(nbytes):
    """Ten launches of the plain streaming copy over `nbytes`: the reference
    for scaling byte counters and the practical bandwidth ceiling.
    Returns (ms per copy, GB/s counting read + write)."""
    import torch
    from paper_1405_2232_amd.lbm import copy_probe
    a = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    copy_probe(b, a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        copy_probe(b, a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    return ms, 2 * nbytes / ms / 1e6


def copy_probe_only(nbytes):
    ms, gbs = copy_rate(nbytes)
    print(json.dumps({"copy_bytes": nbytes, "ms": round(ms, 5), "GBs": round(gbs, 1)}), flush=True)


def _counter_rows(d):
    """(kernel name, counter value) of every dispatch in the rocprofv3
    counter-collection CSVs under directory d."""
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(f) as fp:
            for r in csv.DictReader(fp):
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit("no counter_collection.csv under " + d)
    return rows


def traffic_summary(args):
    """HBM bytes per step-kernel launch from a FETCH_SIZE and a WRITE_SIZE
    run of this script.  Each counter is scaled by what it reads for the
    1 GiB plain copy kernel the same run launches (1 GiB read, 1 GiB
    written), then the per-launch mean over the step kernel's dispatches is
    written with the hash of the kernel sources it was taken on."""
    import re
    step = re.compile(r"lbmdev::k_tile<(\d+), (\d+), 0, (\d+)>|lbmdev::k_pair<(\d+), (\d+)(?:, \w+)?>")
    out = {"precision": args.precision, "nx": args.nx, "ny": args.ny,
           "layout": "row-interleaved", "kernel_hash": kernel_hash()}
    copy_kib = float(1 << 20)
    for key, d in (("fetch", args.traffic_from[0]), ("write", args.traffic_from[1])):
        rows = _counter_rows(d)
        copies = [v for k, v in rows if "lbmdev::k_copy" in k]
        steps = {}
        for k, v in rows:
            m = step.search(k)
            if m:
                steps.setdefault(m.group(0), []).append(v)
        if not copies or not steps:
            raise SystemExit("no copy or step-kernel dispatches in " + d)
        name, vals = max(steps.items(), key=lambda kv: len(kv[1]))
        scale = copy_kib / (sum(copies) / len(copies))
        raw = sum(vals) / len(vals)
        out["kernel"] = name
        out["steps_per_launch"] = 2 if "k_pair" in name else 1
        out[key + "_kib_raw"] = round(raw, 1)
        out[key + "_scale"] = round(scale, 4)
        out[key + "_bytes"] = int(raw * scale * 1024)
        out[key + "_launches"] = len(vals)
    out["bytes_per_launch"] = out["fetch_bytes"] + out["write_bytes"]
    out["bytes_per_node"] = round(out["bytes_per_launch"] / (args.nx * args.ny), 1)
    out["bytes_per_node_step"] = round(out["bytes_per_node"] / out["steps_per_launch"], 1)
    with open(args.traffic_out, "w") as fp:
        json.dump(out, fp, indent=1)
        fp.write("\n")
    print(json.dumps(out), flush=True)


def batch_section(steps, torch):
    """The 256 uneven periodic droplet lattices (sides 64..512, seed 2):
    every lattice advanced `steps` steps by one launch per two steps
    replayed from hipGraphs, FP32 per-node-reference storage, autotuned
    band height (the one-step tile shape is tuned too; it serves odd steps);
    against the same lattices advanced one after another by single-lattice
    launches, in the same storage form (the gain of batching alone) and in
    FP64 (timed over fewer steps per lattice and scaled: the cost per step
    is constant)."""
    from paper_1405_2232_amd import autotune, inputs
    from paper_1405_2232_amd.lbm import CORRECTED, Batch, Lattice
    cases = inputs.batch_lattices()
    cells = sum(p["nx"] * p["ny"] for p, _, _ in cases)
    refs = [(float(r.mean()), float(t.mean())) for _, r, t in cases]

    def make():
        b = Batch([c[0] for c in cases], "fp32local", refs=refs)
        for m, (p, rho, T) in zip(b.members, cases):
            m.init_fields(rho, T)
        return b

    sizes = [(p["nx"], p["ny"]) for p, _, _ in cases]
    (bx, rows), tried = autotune.tune(make, "batch", "fp32local", sizes, CORRECTED)
    prows, ptried = autotune.tune_pair_rows(make, "batch", "fp32local", sizes, CORRECTED)
    b = make()
    b.set_tiling(bx, rows)
    if prows:
        b.set_step_pairing(True, prows)
    b.use_graph(10)
    b.step(50, CORRECTED)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    b.step(steps, CORRECTED)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = b.sync()
    if status != 0:
        raise SystemExit("the batch reported status %d" % status)
    batch_ms = e0.elapsed_time(e1)
    del b

    # the same lattices one after another, single-lattice launches, in the
    # batch's storage form (the batching gain alone) and in FP64
    seq_steps = 500
    seq = {}
    for prec in ("fp32local", "fp64"):
        seq_ms = 0.0
        for (p, rho, T), ref in zip(cases, refs):
            g = Lattice(p, prec, rho_ref=ref[0], T_ref=ref[1]) if prec != "fp64" else Lattice(p, prec)
            g.init_fields(rho, T)
            g.step(10, CORRECTED)
            seq_ms += timed_steps(g, seq_steps, CORRECTED, torch) * steps
            del g
        seq[prec] = seq_ms
    return {"lattices": len(cases), "nodes": cells, "steps": steps,
            "fp32local_graph_s": round(batch_ms / 1e3, 3), "wall_s": round(wall, 3),
            "mlups": round(cells * steps / (batch_ms / 1e3) / 1e6, 1),
            "alg_GBs": round(ALG_BYTES["fp32local"] * cells * steps / (batch_ms / 1e3) / 1e9, 1),
            "tile": [bx, rows], "autotune_ms_per_step": tried,
            "pair_rows": prows, "autotune_pair_ms_per_step": ptried,
            "sequential_fp32local_s": round(seq["fp32local"] / 1e3, 3),
            "sequential_fp32local_mlups": round(cells * steps / (seq["fp32local"] / 1e3) / 1e6, 1),
            "speedup_same_storage": round(seq["fp32local"] / batch_ms, 2),
            "sequential_fp64_s": round(seq["fp64"] / 1e3, 3),
            "sequential_fp64_mlups": round(cells * steps / (seq["fp64"] / 1e3) / 1e6, 1),
            "speedup_vs_fp64": round(seq["fp64"] / batch_ms, 2),
            "sequential_note": "single-lattice launches, %d timed steps per lattice (after 10), "
                               "scaled to %d: the cost per step is constant" % (seq_steps, steps)}


def timed_steps(g, steps, treatment, torch):
    """Average duration of one step launch, from HIP events on the stream
    the library launches on (torch's current stream)."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    g.step(steps, treatment)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def kernel_timing(g, treatment, torch, warm=100, runs=5, launches=200):
    """Launch time of the step kernel alone: `warm` untimed steps, then
    `runs` runs of `launches` launches each, every run bracketed by HIP
    events on the launch stream (torch's current stream; no periodic check
    inside).  Returns the median, min and max ms per launch and the steps
    one launch advances."""
    g.set_check_interval(0)
    per = 2 if g.get_step_pairing()[0] else 1
    g.step(warm + (warm & 1), treatment)
    times = sorted(timed_steps(g, launches * per, treatment, torch) * per for _ in range(runs))
    return {"median": times[runs // 2], "min": times[0], "max": times[-1],
            "steps_per_launch": per, "runs": runs, "launches": launches, "warmup": warm}


def treatment_section(p, rho, T, args, torch, warm=100, runs=5, steps=200):
    """The slab in the benchmark's storage form with each temperature
    treatment: ms per step (median of `runs` event-timed runs of `steps`
    steps after `warm` untimed ones, no periodic check) and MLUPS.  The
    plain treatment holds the EOS at T0 (with the EOS at the local
    temperature it leaves the EOS domain); the finite-difference treatment
    runs the one-step kernel for f and two stencil passes for T per step."""
    from paper_1405_2232_amd.lbm import CORRECTED, FD_RK2, PLAIN, Lattice
    cells = p["nx"] * p["ny"]
    out = {}
    for name, treatment, fixed in (("plain_eq7_eos_at_T0", PLAIN, True), ("corrected_eq24", CORRECTED, False),
                                   ("finite_difference_eq26", FD_RK2, False)):
        q = dict(p, eos_fixed_T=fixed)
        g = Lattice(q, args.precision)
        g.init_fields(rho, T)
        if args.no_pair:
            g.set_step_pairing(False)
        g.set_check_interval(0)
        g.step(warm, treatment)
        times = sorted(timed_steps(g, steps, treatment, torch) for _ in range(runs))
        ms = times[runs // 2]
        out[name] = {"ms_per_step": round(ms, 5), "mlups": round(cells / ms / 1e3, 1),
                     "steps_per_launch": 2 if (g.get_step_pairing()[0] and treatment != FD_RK2) else 1}
        del g
    return out


def small_section(torch, steps=2000, runs=3):
    """Lattices too small to fill the device, which are bound by latency,
    not HBM (a roofline fraction means nothing there): the 64^2 periodic
    droplet for its 2000 steps with each treatment in FP64 (the two-treatment
    parity workload), and a 256^2 droplet (the size of the warm-start
    workload's boxes in the survey's recipe).  MLUPS from the median of
    `runs` event-timed runs of `steps` steps."""
    from paper_1405_2232_amd import inputs
    from paper_1405_2232_amd.lbm import CORRECTED, PLAIN, Lattice
    out = {}
    for n, radius in ((64, 16.0), (256, 64.0)):
        p, rho, T = inputs.static_droplet(nx=n, ny=n, radius=radius)
        # the plain treatment with the EOS at T0, as in the parity workload
        # (with the EOS at the local temperature it leaves the EOS domain)
        for name, treatment, fixed in (("plain_eos_at_T0", PLAIN, True), ("corrected", CORRECTED, False)):
            g = Lattice(dict(p, eos_fixed_T=fixed), "fp64")
            g.init_fields(rho, T)
            g.set_check_interval(0)
            g.step(100, treatment)
            ms = sorted(timed_steps(g, steps, treatment, torch) for _ in range(runs))[runs // 2]
            out["droplet_%d_fp64_%s" % (n, name)] = {"us_per_step": round(ms * 1e3, 2),
                                                      "mlups": round(n * n / ms / 1e3, 1),
                                                      "two_step": g.get_step_pairing()[0]}
            del g
    return out


def cpu_baseline(p, rho, T, treatment, seconds):
    """FP64 oracle on the host cores: time whole steps of the same workload
    until about `seconds` have passed."""
    from oracle import Oracle
    o = Oracle(p)
    o.init_fields(rho, T)
    o.step(1, treatment)  # first touch
    n = 0
    t0 = time.perf_counter()
    while True:
        o.step(1, treatment)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    cells = p["nx"] * p["ny"]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": round(cells * n / el / 1e6, 3), "unit": "MLUPS", "cores": cores,
           "kind": "oracle", "cpu_model": host_cpu_model(),
           "sample": "%d steps of the %dx%d slab (FP64 oracle, %d OpenMP threads, %.1f s)"
                     % (n, p["nx"], p["ny"], cores, el)}
    out["single_core"] = single_core_baseline(p["nx"], p["ny"], treatment, seconds / 2)
    return out


def host_cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fp:
            for line in fp:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def single_core_baseline(nx, ny, treatment, seconds):
    """The same oracle steps on one host core, in a child process started
    with OMP_NUM_THREADS=1 (the OpenMP runtime reads it at start-up); the
    child imports no GPU code."""
    import subprocess
    code = ("import json, sys, time; sys.path.insert(0, %r)\n"
            "from oracle import Oracle\n"
            "from paper_1405_2232_amd import inputs\n"
            "p, rho, T = inputs.wall_slab(nx=%d, ny=%d)\n"
            "o = Oracle(p); o.init_fields(rho, T); o.step(1, %d)\n"
            "n = 0; t0 = time.perf_counter()\n"
            "while True:\n"
            "    o.step(1, %d); n += 1; el = time.perf_counter() - t0\n"
            "    if el >= %r: break\n"
            "print(json.dumps({'steps': n, 's': el}))\n"
            % (ROOT, nx, ny, treatment, treatment, float(seconds)))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=120 + 4 * seconds)
        d = json.loads(r.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None
    return {"value": round(nx * ny * d["steps"] / d["s"] / 1e6, 3), "unit": "MLUPS", "cores": 1,
            "sample": "%d steps of the %dx%d slab (FP64 oracle, 1 thread, %.1f s)"
                      % (d["steps"], nx, ny, d["s"])}


def interface_jump_section(nx, ny, steps, torch):
    """The forcing-term effect on the slab (Eq. (23)): the 2048^2 wall
    slab run `steps` steps with each treatment (FP32 per-node-reference
    storage; the plain treatment with the EOS at T0, since with the EOS at
    the local temperature it leaves the EOS domain), then at each of the two
    interfaces the temperature and density 8 nodes into the vapour and into
    the liquid from where the density crosses its mid value.  The plain
    treatment diffuses rho cv T rather than T, so across an interface it
    drives T_v/T_l towards rho_l/rho_v; the corrected one keeps T
    continuous (T_v/T_l near 1)."""
    from paper_1405_2232_amd import inputs
    from paper_1405_2232_amd.lbm import CORRECTED, PLAIN, Lattice
    out = {"nx": nx, "ny": ny, "steps": steps, "storage": "fp32local", "probe_depth": 8}
    for name, treatment, fixed in (("corrected", CORRECTED, False), ("plain_eos_at_T0", PLAIN, True)):
        p, rho, T = inputs.wall_slab(nx=nx, ny=ny)
        p["eos_fixed_T"] = fixed
        g = Lattice(p, "fp32local")
        g.init_fields(rho, T)
        g.set_check_interval(1000)
        g.step(steps, treatment)
        r, _, _, t = (a[:, 0] for a in g.moments())
        del g
        mid = 0.5 * (r[ny // 2] + r[ny // 8])
        liquid = r > mid
        cross = [int(k) for k in range(1, ny) if liquid[k] != liquid[k - 1]]
        sides = []
        for k in cross:
            lo, hi = k - 1, k  # the crossing lies between rows lo and hi
            v, l = (lo - 8, hi + 8) if liquid[hi] else (hi + 8, lo - 8)
            sides.append({"row": k, "T_v_over_T_l": round(float(t[v] / t[l]), 4),
                          "rho_l_over_rho_v": round(float(r[l] / r[v]), 4),
                          "T_v_over_Tc": round(float(t[v] / inputs.cs_tc()), 4),
                          "T_l_over_Tc": round(float(t[l] / inputs.cs_tc()), 4)})
        out[name] = sides
    return out


WARM_WEIGHTS = os.path.join(ROOT, "paper_1405_2232_amd", "warmstart_64.npz")


def steady_section(count, torch, n=64, target=1e-8, cap=600000):
    """Wall time to a one-step residual of `target` on held-out steady-state
    cases (seeds 100000.., n x n, 1-3 droplets between Dirichlet walls, EOS
    at T0, FP64 storage): plain = one lattice at a time from the initial
    fields; batched = all cases in one batch; warm = batched, started from
    the trained network's prediction (inference and screening timed in);
    physical_start = the batched runs again, each lattice started at rest
    in the forcing scheme's velocity (stored momentum -F/2)."""
    from paper_1405_2232_amd import inputs, warmstart
    cases = [inputs.warmstart_case(100000 + s, n=n, max_drops=3) for s in range(count)]
    plain = warmstart.solve_single(cases, target=target, cap=cap)
    cold = warmstart.solve(cases, target=target, cap=cap, keep=False)
    out = {"cases": count, "n": n, "target": target, "cap": cap, "storage": "f64",
           "plain_s": round(plain["wall_s"], 2), "plain_converged": sum(s is not None for s in plain["steps"]),
           "batched_cold_s": round(cold["wall_s"], 2),
           "batched_cold_converged": sum(s is not None for s in cold["steps"])}
    if os.path.exists(WARM_WEIGHTS):
        t0 = time.perf_counter()
        ws = warmstart.WarmStart(n, params=warmstart.load_params(WARM_WEIGHTS))
        preds = ws.predict(cases)
        inits, rp, rc = warmstart.screen(cases, preds)
        t_inf = time.perf_counter() - t0
        warm = warmstart.solve(cases, inits=inits, target=target, cap=cap, keep=False)
        both = [i for i in range(count) if cold["steps"][i] is not None and warm["steps"][i] is not None]
        out.update({
            "warm_s": round(warm["wall_s"] + t_inf, 2), "warm_inference_s": round(t_inf, 3),
            "warm_converged": sum(s is not None for s in warm["steps"]),
            "warm_accepted": sum(p is not None for p in inits),
            "steps_cold_vs_warm_on_both": [sum(cold["steps"][i] for i in both), sum(warm["steps"][i] for i in both)],
            "speedup_warm_vs_plain": round(plain["wall_s"] / (warm["wall_s"] + t_inf), 2)})
    out["speedup_batched_vs_plain"] = round(plain["wall_s"] / cold["wall_s"], 2)
    coldp = warmstart.solve(cases, target=target, cap=cap, keep=False, physical=True)
    both = [i for i in range(count) if cold["steps"][i] is not None and coldp["steps"][i] is not None]
    ps = {"cold_s": round(coldp["wall_s"], 2),
          "cold_converged": sum(s is not None for s in coldp["steps"]),
          "steps_cold_vs_physical_on_both": [sum(cold["steps"][i] for i in both),
                                             sum(coldp["steps"][i] for i in both)],
          "speedup_vs_plain": round(plain["wall_s"] / coldp["wall_s"], 2)}
    if os.path.exists(WARM_WEIGHTS):
        t0 = time.perf_counter()
        preds = ws.predict(cases)
        inits, _, _ = warmstart.screen(cases, preds, physical=True)
        t_inf = time.perf_counter() - t0
        warmp = warmstart.solve(cases, inits=inits, target=target, cap=cap, keep=False, physical=True)
        rawp = warmstart.solve(cases, inits=preds, target=target, cap=cap, keep=False, physical=True)
        capped = lambda st: sum(cap if s is None else s for s in st)  # noqa: E731
        ps.update({"warm_s": round(warmp["wall_s"] + t_inf, 2),
                   "warm_converged": sum(s is not None for s in warmp["steps"]),
                   "warm_accepted": sum(p is not None for p in inits),
                   "steps_capped_cold_vs_warm": [capped(coldp["steps"]), capped(warmp["steps"])],
                   "every_prediction_s": round(rawp["wall_s"] + t_inf, 2),
                   "every_prediction_converged": sum(s is not None for s in rawp["steps"]),
                   "steps_capped_every_prediction": capped(rawp["steps"]),
                   "speedup_warm_vs_plain": round(plain["wall_s"] / (warmp["wall_s"] + t_inf), 2)})
    out["physical_start"] = ps
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (a lattice would "
              "shard as y-slabs exchanging three halo rows per two-step launch; batches would "
              "split by lattice)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe_only(args.copy_probe)
        return
    if args.traffic_from:
        traffic_summary(args)
        return
    import torch
    from paper_1405_2232_amd import inputs
    from paper_1405_2232_amd.lbm import CORRECTED, Lattice

    torch.cuda.set_device(0)
    p, rho, T = inputs.wall_slab(nx=args.nx, ny=args.ny)
    cells = args.nx * args.ny
    treatment = CORRECTED

    g = Lattice(p, args.precision)
    g.init_fields(rho, T)
    if args.no_pair:
        g.set_step_pairing(False)

    # step kernel alone (the roofline): its own warm-up, then the median of
    # five event-timed runs, whatever --steps and --warmup are; this also
    # brings the device to its working clocks before the timed region
    kt = kernel_timing(g, treatment, torch)
    per_launch = kt["steps_per_launch"]
    paired = per_launch == 2
    launch_ms = kt["median"]
    kernel_ms = launch_ms / per_launch
    achieved = ALG_BYTES[args.precision] * cells * per_launch / (launch_ms * 1e-3) / 1e9

    g.set_check_interval(100)
    if args.warmup > 0:
        g.step(args.warmup, treatment)
    out = [torch.empty((args.ny, args.nx), dtype=torch.float64, device="cuda") for _ in range(4)]
    torch.cuda.synchronize()

    # timed region: K steps (with the periodic FP64 check) + one moments export
    t0 = time.perf_counter()
    g.step(args.steps, treatment)
    g.moments_device(*out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = g.sync()
    if status != 0:
        raise SystemExit("the run reported status %d" % status)
    ms_per_step = wall * 1e3 / args.steps
    mlups = cells * args.steps / wall / 1e6

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fp:
            tr = json.load(fp)
        if tr.get("kernel_hash") == kernel_hash() and tr.get("precision") == args.precision \
                and tr.get("nx") == args.nx and tr.get("ny") == args.ny \
                and tr.get("steps_per_launch", 1) == per_launch:
            traffic = tr.get("bytes_per_launch")

    # the same K steps with the boundary's host transfers timed in: FP64
    # host fields in (lbm_init_fields), K steps, FP64 host moments out
    # (lbm_moments); never `value`, whose state is resident in HBM
    g.set_check_interval(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.init_fields(rho, T)
    g.step(args.steps, treatment)
    g.moments()
    wall_h = time.perf_counter() - t0
    host_inclusive = {"mlups": round(cells * args.steps / wall_h / 1e6, 1), "ms": round(wall_h * 1e3, 2),
                      "what": "host rho, T in; %d steps; host rho, u, T out" % args.steps}
    del g

    copy_ms, copy_gbs = copy_rate(1 << 30)

    extra = {}
    if not args.no_extra:
        for prec in ("fp64", "fp32dev"):
            if prec == args.precision:
                continue
            h = Lattice(p, prec)
            h.init_fields(rho, T)
            if args.no_pair:
                h.set_step_pairing(False)
            ht = kernel_timing(h, treatment, torch)
            ms = ht["median"] / ht["steps_per_launch"]
            extra[prec] = {"mlups": round(cells / ms / 1e3, 1),
                           "alg_GBs": round(ALG_BYTES[prec] * cells / ms / 1e6, 1),
                           "launch_ms": [round(ht[k], 5) for k in ("median", "min", "max")],
                           "steps_per_launch": ht["steps_per_launch"]}
            del h
        extra[args.precision] = {"mlups": round(cells / kernel_ms / 1e3, 1),
                                 "alg_GBs": round(achieved, 1),
                                 "launch_ms": [round(kt[k], 5) for k in ("median", "min", "max")],
                                 "steps_per_launch": per_launch}

    by_treatment = {} if args.no_extra else treatment_section(p, rho, T, args, torch)
    small = {} if args.no_extra else small_section(torch)

    line = {
        "metric": "MLUPS (FP64 vs FP32-dev, % HBM roofline); wall-time to 1e-8 residual vs plain",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage": {"fp32local": "f32 + f16 node reference", "fp32dev": "f32",
                    "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "wall_slab_%dx%d_corrected_%s" % (args.nx, args.ny, args.precision),
                   "nx": args.nx, "ny": args.ny, "treatment": "corrected (Eq. 24)",
                   "eos": "Carnahan-Starling at local T", "T0": "0.85 Tc",
                   "walls": "0.80 Tc / 0.90 Tc", "check_every": 100},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_pair" if paired else "k_tile",
                     "steps_per_launch": per_launch,
                     "launch_ms": round(launch_ms, 5),
                     "launch_ms_min_max": [round(kt["min"], 5), round(kt["max"], 5)],
                     "timing": "median of %d runs of %d launches after %d warm-up steps, HIP events"
                               % (kt["runs"], kt["launches"], kt["warmup"]),
                     "kernel_ms": round(kernel_ms, 5),
                     "bytes_per_node": ALG_BYTES[args.precision],
                     "measured_GBs": (round(traffic / (launch_ms * 1e-3) / 1e9, 1)
                                      if traffic else None),
                     "copy_GBs": round(copy_gbs, 1)},
        "by_precision": extra,
        "by_treatment": by_treatment,
        "small_lattices": small,
        "host_inclusive": host_inclusive,
    }
    if not args.no_jump:
        line["interface_jump"] = interface_jump_section(args.nx, args.ny, args.jump_steps, torch)
    if not args.no_batch:
        line["batched"] = batch_section(args.batch_steps, torch)
    if not args.no_steady:
        line["steady_state"] = steady_section(args.steady_cases, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, rho, T, treatment, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
