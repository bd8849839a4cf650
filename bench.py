#!/usr/bin/env python3
"""Throughput of the free-surface LBM hot path on one MI355X.

One step = one full lattice update of the 512x512x1024 bubble column with 1e5
spheres (fused stream-collide with free-surface and particle boundaries, cell
conversions, bubble model, particle update and coverage).  Prints one JSON line:
box MLUPS (all box cells counted), the HBM roofline of the dominant kernel
(timed with HIP events on the library's stream) and the FP64 oracle timed on a
bounded sample of the same workload on the host cores.

Also reported: the storage forms (shifted binary16 / bfloat16 populations) on the
same column with their error against the oracle on the 128^3 pool with 1,400
spheres after 1,000 steps; the differentiation form (adjoint MLUPS of the
summed-drag window, 64^3 and 256^3); the column with surface tension (curvature
pass); the bubble-splitting test and labelling pass; single rising bubbles in the
four regimes of the bubble-regime table; and a plain device copy's bandwidth beside
the roofline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0
METRIC = "FSLBM MLUPS + achieved HBM GB/s vs peak; FP16-storage and adjoint MLUPS"
STORAGES = {"f32": 0, "f16s": 1, "bf16s": 2}
DTYPE = {0: "f32", 1: "f16-shifted storage, f32 arithmetic", 2: "bf16-shifted storage, f32 arithmetic"}
ELEM = {0: 4, 1: 2, 2: 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name, storage):
    from paper_1712_07028_amd import workloads as W

    if name == "column":
        w = W.bubble_column_large()
    elif name == "column_nospheres":
        w = W.bubble_column_large().replace(particles=None, name="column512x512x1024_bubble40_no_spheres")
    elif name == "bed128":
        w = W.bubble_bed_128()
    elif name == "pool32":
        w = W.bubble_column_small()
    else:
        raise SystemExit(f"unknown workload {name}")
    return w.replace(storage=storage)


TRAFFIC_FILE = os.path.join(HERE, "profiles", "k_stream_collide_column_traffic.json")
KERNEL_SOURCES = [os.path.join(HERE, "paper_1712_07028_amd", "csrc", f)
                  for f in ("k_stream_collide.hpp", "fsl_device.hpp")]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(path, storage):
    """HBM bytes per stream-collide launch from the counter runs recorded in path,
    or None when they were taken on other kernel sources or another storage."""
    if not path or not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernel_hash") != kernel_hash() or t.get("storage") != storage:
        return None
    return t.get("bytes_per_launch")


def precision_errors(fsl, W, storage):
    """Errors of one storage form against the oracle's stored results on the 128^3
    pool with one bubble and 1,400 spheres after 1,000 steps."""
    ref = json.load(open(os.path.join(HERE, "tests", "golden", "precision_bed128.json")))
    T = ref["steps"]
    w = W.bubble_bed_128(storage=storage)
    n = w.particles.n
    s = fsl.Sim(w)
    M0 = s.mass()[0]
    s.step(T - 10)
    b0 = s.bubbles()
    drag = []
    for _ in range(10):
        s.step(1)
        drag.append(float(s.particles_get(n)["F"][:, 2].mean()))
    b1 = s.bubbles()
    M1 = s.mass()[0]
    s.close()
    rise = (b1[1]["centroid"][2] - b0[1]["centroid"][2]) / 10.0
    return {"workload": ref["workload"], "steps": T,
            "mass_drift": abs(M1 / M0 - 1.0), "mass_vs_oracle": abs(M1 / ref["mass"] - 1.0),
            "rise_velocity_rel_err": abs(rise / ref["rise_velocity"] - 1.0),
            "mean_drag_rel_err": abs(float(np.mean(drag)) / ref["mean_drag_z"] - 1.0)}


def adjoint_rate(fsl, W, torch, n, n_particles, T=200, k=20):
    """Summed-drag window: forward (T steps with checkpoints) and the adjoint sweep
    (recompute + reverse), MLUPS = box cells x T / time."""
    w = W.adjoint_window(n=n, n_particles=n_particles)
    s = fsl.Sim(w, window=(T, k))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = s.window_forward(T, k)
    t1 = time.perf_counter()
    dtau, dg = s.window_backward(1.0)
    t2 = time.perf_counter()
    flags = s.get(fsl.FIELD_FLAGS)
    n_liq = int((flags == fsl.LIQ).sum())
    s.close()
    N = w.cells
    # adjoint step kernel: s_{t-1} pulled, mu_{t+1} gathered, mu_t written (FP32)
    return {"workload": w.name, "steps": T, "checkpoint_every": k,
            "forward_mlups": round(N * T / (t1 - t0) / 1e6, 1),
            "adjoint_mlups": round(N * T / (t2 - t1) / 1e6, 1),
            "backward_ms": round((t2 - t1) * 1e3, 2),
            "adjoint_bytes_per_step": 3 * 19 * 4 * n_liq + N,
            "J": J, "dJ_dtau": dtau, "dJ_dg": [float(v) for v in dg]}


def surface_tension_rate(fsl, torch, w, steps, sigma=0.005):
    """The column with surface tension: whole step and the curvature pass."""
    ws = w.replace(sigma=sigma)
    s = fsl.Sim(ws, face_forces=False)
    s.step(5)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # phase times from a separate bracketed run, so the events do not enter the rate
    s.profile(True)
    s.profile_get()
    s.step(20)
    prof = s.profile_get()
    s.close()
    torch.cuda.empty_cache()
    return {"sigma": sigma, "steps": steps, "mlups": round(ws.cells * steps / dt / 1e6, 1),
            "ms_per_step": round(dt / steps * 1e3, 4),
            "curvature_ms": round(prof["curvature"][0] / max(prof["curvature"][1], 1), 4)}


def split_pass_cost(fsl, torch, w, reps=3):
    """The column's bubble-splitting labelling when it runs: a forced pass over the
    state after 5 steps (setting the bubble table labels every gas cell)."""
    s = fsl.Sim(w, face_forces=False)
    s.step(5)
    s.sync()
    b = s.bubbles()
    s.profile(True)
    s.profile_get()
    for _ in range(reps):
        s.bubbles_set([x["M"] for x in b], list(range(len(b))), [x["alive"] for x in b])
    prof = s.profile_get()
    s.close()
    torch.cuda.empty_cache()
    return round(prof["split"][0] / max(prof["split"][1], 1), 4)


def bubble_regimes(fsl, W, torch, steps=8000, every=50, z_stop=70.0):
    """Single rising bubbles in the regimes of Table tab:Annaland (free-slip sides,
    no-slip floor, pressure at the top): the bubble Reynolds number Re = u d / nu from
    the rise velocity of the main bubble's centroid over the last third of the run, d
    the diameter of a sphere of its volume, beside the paper's numbers."""
    out = {}
    for case, p in W.BUBBLE_REGIMES.items():
        w = W.bubble_regime(case)
        nu = (w.tau - 0.5) / 3.0
        s = fsl.Sim(w)
        track = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = 0
        full = None
        while t < steps:
            s.step(every)
            t += every
            try:
                b = s.bubbles()
            except fsl.FslError as e:
                # the skirted bubble sheds tens of satellites, each holding an id of the
                # 64-entry table until it vanishes: the run ends where the table is full
                if "overflowed" not in str(e):
                    raise
                full = t
                break
            # the main bubble: the largest gas part other than the atmosphere (id 0); a
            # split can leave id 1 to a fragment
            m = max((x for x in b[1:] if x["alive"]), key=lambda x: x["V"], default=None)
            if m is None:  # the bubble has vanished
                break
            track.append((t, m["centroid"][2], m["V"], len([x for x in b if x["alive"]])))
            if m["centroid"][2] > z_stop:
                break
        dt = time.perf_counter() - t0
        s.close()
        if len(track) < 2:
            out[case] = {"re": None, "re_paper": p["re_paper"], "re_fan": p["re_fan"], "steps": int(t)}
            continue
        tr = np.array(track)
        k = max(2, len(tr) // 3)
        u = np.polyfit(tr[-k:, 0], tr[-k:, 1], 1)[0]
        d = (6.0 * tr[-k:, 2].mean() / np.pi) ** (1.0 / 3.0)
        out[case] = {"re": round(float(u * d / nu), 3), "re_paper": p["re_paper"], "re_fan": p["re_fan"],
                     "u": float(u), "d": round(float(d), 3), "steps": int(tr[-1, 0]), "bubbles_alive": int(tr[-1, 3]),
                     "mlups": round(w.cells * t / dt / 1e6, 1)}
        if full is not None:
            out[case]["bubble_table_full_at_step"] = int(full)
    return out


def copy_bandwidth(torch, gib=2.0, reps=5):
    """A plain device copy of a large buffer on the same GPU, for context beside the
    roofline: bytes read plus bytes written over the copy time (HIP events)."""
    n = int(gib * (1 << 30))
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return round(2.0 * n / (ms / 1e3) / 1e9, 1)


def ceiling_bandwidth(torch, n=(512, 512, 256), reps=5):
    """The D3Q19 pull with no arithmetic (libfsl_ceiling.so) over a closed FP32 box on
    torch's current stream: 152 B per cell over its time (HIP events), the ceiling
    that the stream-collide kernel's access shape allows."""
    import ctypes

    from paper_1712_07028_amd import build as B

    lib = ctypes.CDLL(B.CEILING_LIB)
    lib.fsl_ceiling_pull.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_longlong, ctypes.c_void_p]
    N = n[0] * n[1] * n[2]
    S = (N + 255) // 256 * 256
    a = torch.zeros(19 * S, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()

    def launch():
        rc = lib.fsl_ceiling_pull(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n[0], n[1], n[2], S,
                                  ctypes.c_void_p(stream.cuda_stream))
        if rc:
            raise RuntimeError(f"fsl_ceiling_pull failed ({rc})")

    launch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        launch()
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return round(152.0 * N / (ms / 1e3) / 1e9, 1)


def suspension(fsl, W, torch, phis, re_p, warm, steps, every):
    """The sheared suspension of Sec. 3.1 on the paper's box: for each volume fraction
    the plate force F_x (the mean of the two plates' x forces, bottom minus top) is
    sampled every `every` steps over `steps` steps after `warm` steps of start-up,
    mu_s = <F_x> / (A gamma), against Eq. Eilers."""
    out = {}
    for phi in phis:
        w, wall = W.sheared_suspension(phi, re_p=re_p)
        n = w.n
        U = wall[2][1][0]
        gamma, A, mu = 2.0 * U / n[2], n[0] * n[1], (w.tau - 0.5) / 3.0
        s = fsl.Sim(w, wall_u=wall)
        log(f"suspension phi {phi}: {w.particles.n if w.particles is not None else 0} spheres, tau {w.tau:.4f}, "
            f"{warm} + {steps} steps")
        t0 = time.perf_counter()
        done = 0
        while done < warm:
            k = min(50000, warm - done)
            s.step(k)
            s.sync()
            done += k
            log(f"  start-up {done}/{warm}, {time.perf_counter() - t0:.0f} s")
        samples = []
        done = 0
        while done < steps:
            s.step(every)
            Wf = s.walls()
            samples.append(0.5 * (Wf[2, 0, 0] - Wf[2, 1, 0]))
            done += every
            if done % 50000 < every:
                log(f"  averaging {done}/{steps}, mu_s/mu so far {np.mean(samples) / (A * gamma) / mu:.4f}, "
                    f"{time.perf_counter() - t0:.0f} s")
        wall_s = time.perf_counter() - t0
        s.close()
        f = np.array(samples)
        half = len(f) // 2
        rel = f.mean() / (A * gamma) / mu
        out[f"{phi:g}"] = {
            "workload": w.name, "spheres": w.particles.n if w.particles is not None else 0, "tau": w.tau,
            "re_p": re_p, "gamma_T": gamma * steps, "startup_steps": warm, "steps": steps, "sample_every": every,
            "mu_s_over_mu": round(float(rel), 4),
            # the two halves of the averaging window, as a check that the mean has settled
            "halves": [round(float(f[:half].mean() / (A * gamma) / mu), 4),
                       round(float(f[half:].mean() / (A * gamma) / mu), 4)],
            "eilers": round(float(W.eilers(phi)), 4), "mlups": round(w.cells * (warm + steps) / wall_s / 1e6, 1),
        }
        log(f"  phi {phi}: mu_s/mu = {rel:.4f}, Eilers {W.eilers(phi):.4f}")
    return out


def host_threads():
    """Threads the host grants this job: OMP_NUM_THREADS when the job scheduler sets
    it, else the CPUs in the process's affinity mask."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, steps):
    """The FP64 oracle on the host: the headline value on a bounded sample of the
    column (its lowest 16 layers, all granted threads), plus the small-box and
    128^3-bed configurations at one thread and at all granted threads."""
    import oracle
    from paper_1712_07028_amd import workloads as W

    oracle.build(force=False)
    threads = host_threads()

    def timed(wl, n, th):
        o = oracle.Oracle(wl, n_threads=th)
        t0 = time.perf_counter()
        o.step(n)
        dt = time.perf_counter() - t0
        o.close()
        return {"workload": wl.name, "box": list(wl.n), "steps": n, "threads": th,
                "seconds": round(dt, 3), "MLUPS": round(wl.cells * n / dt / 1e6, 4)}

    s = W.slab_of(w, 16) if w.n[2] > 16 else w
    head = timed(s, steps, threads)
    small, bed = W.bubble_column_small(), W.bubble_bed_128()
    runs = [timed(small, small.steps, 1), timed(small, small.steps, threads),
            timed(bed, 3, 1), timed(bed, 10, threads), timed(s, 1, 1)]
    return {"value": head["MLUPS"], "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{s.n[0]}x{s.n[1]}x{s.n[2]} bottom slab of the column "
                      f"({s.particles.n if s.particles is not None else 0} spheres), {steps} steps, FP64",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(), "runs": runs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="column")
    ap.add_argument("--storage", default="f32", choices=list(STORAGES))
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the storage forms and the differentiation form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the differentiation form (for kernel profiles)")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--regimes-only", action="store_true",
                    help="only the single rising bubbles of the bubble-regime table")
    ap.add_argument("--suspension", default="",
                    help="only the sheared suspension: comma-separated volume fractions")
    ap.add_argument("--susp-re", type=float, default=0.1, help="particle Reynolds number of the suspension")
    ap.add_argument("--susp-warm", type=int, default=150000, help="start-up steps of the suspension")
    ap.add_argument("--susp-steps", type=int, default=900000, help="averaging steps (gamma T = 100 at 900,000)")
    ap.add_argument("--susp-every", type=int, default=50, help="steps between plate-force samples")
    ap.add_argument("--traffic", default=TRAFFIC_FILE,
                    help="JSON file with measured HBM bytes per stream-collide launch")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="after the run, copy a buffer of this many GiB three times with the "
                         "runtime's copy and three times 4 bytes per lane (device copies of known "
                         "size, for scaling hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the multi-GPU slab decomposition is a design, "
              "not code (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1712_07028_amd as fsl

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    fsl.load_library()

    if args.suspension:
        from paper_1712_07028_amd import workloads as W

        phis = [float(v) for v in args.suspension.split(",")]
        res = suspension(fsl, W, torch, phis, args.susp_re, args.susp_warm, args.susp_steps, args.susp_every)
        print(json.dumps({"sheared_suspension": res}), flush=True)
        return

    if args.regimes_only:
        from paper_1712_07028_amd import workloads as W

        print(json.dumps({"bubble_regimes": bubble_regimes(fsl, W, torch)}), flush=True)
        return

    if args.adjoint_only:
        from paper_1712_07028_amd import workloads as W

        res = {f"{n}^3": adjoint_rate(fsl, W, torch, n, npart) for n, npart in ((64, 20), (256, 1280))}
        print(json.dumps({"adjoint": res}), flush=True)
        return

    st = STORAGES[args.storage]
    t0 = time.perf_counter()
    w = workload(args.workload, st)
    log(f"workload {w.name}: {w.n}, {w.particles.n if w.particles is not None else 0} spheres "
        f"(placement {time.perf_counter() - t0:.1f} s)")

    def run(storage, steps, warmup, profile):
        ww = w.replace(storage=storage)
        # the column's step without the face-force diagnostic (the plate force of the
        # suspension experiment), which nothing here reads
        sim = fsl.Sim(ww, face_forces=False)
        sim.step(warmup)
        sim.sync()
        flags = sim.get(fsl.FIELD_FLAGS)
        n_active = int(((flags == fsl.LIQ) | (flags == fsl.IFC)).sum())
        del flags
        if profile:
            sim.profile(True)
            sim.profile_get()  # reset
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        sim.sync()
        prof = sim.profile_get() if profile else None
        sim.close()
        del sim
        torch.cuda.empty_cache()
        return dt, n_active, prof

    log(f"warmup {args.warmup}, timed {args.steps} steps, storage {args.storage}")
    dt, n_active, prof = run(st, args.steps, args.warmup, True)
    N = w.cells
    mlups = N * args.steps / dt / 1e6
    ms_sc, n_sc = prof["stream_collide"]
    avg_s = ms_sc / max(n_sc, 1) / 1e3
    alg_bytes = 2 * 19 * ELEM[st] * n_active + N  # populations in and out + cell types
    achieved = alg_bytes / avg_s / 1e9
    traffic = measured_traffic(args.traffic, args.storage)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": "k_stream_collide", "kernel_ms": round(avg_s * 1e3, 4),
            "algorithmic_bytes_per_launch": int(alg_bytes), "active_cells": n_active,
            "copy_GBs": copy_bandwidth(torch),
            "ceiling_GBs": ceiling_bandwidth(torch),
            "ceiling_kernel": "k_pull_ceiling: D3Q19 pull, 19 FP32 SoA plane reads + 19 writes, no arithmetic, "
                              "512x512x256 closed box"}
    breakdown = {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()}
    log(f"{mlups:.0f} MLUPS, stream-collide {avg_s * 1e3:.3f} ms, {achieved:.0f} GB/s, "
        f"breakdown ms/step {breakdown}")

    forms = {}
    adjoint = {}
    surface = None
    split = None
    regimes = None
    if not args.no_forms:
        from paper_1712_07028_amd import workloads as W

        for name, s2 in STORAGES.items():
            if s2 == st:
                d2, na2, p2 = dt, n_active, prof
            else:
                d2, na2, p2 = run(s2, args.steps, args.warmup, True)
            ms2, n2 = p2["stream_collide"]
            a2 = (2 * 19 * ELEM[s2] * na2 + N) / (ms2 / max(n2, 1) / 1e3) / 1e9
            forms[name] = {"mlups": round(N * args.steps / d2 / 1e6, 1),
                           "speedup_vs_f32": None, "stream_collide_GBs": round(a2, 1),
                           "stream_collide_ms": round(ms2 / max(n2, 1), 4),
                           "error_vs_oracle": precision_errors(fsl, W, s2)}
            log(name, forms[name])
        for name in forms:
            forms[name]["speedup_vs_f32"] = round(forms[name]["mlups"] / forms["f32"]["mlups"], 3)
        for n, npart in ((64, 20), (256, 1280)):
            adjoint[f"{n}^3"] = adjoint_rate(fsl, W, torch, n, npart)
            log("adjoint", adjoint[f"{n}^3"])
        surface = surface_tension_rate(fsl, torch, w.replace(storage=0), min(args.steps, 100))
        log("surface tension", surface)
        split = {"step_ms": breakdown.get("split"),
                 "labelling_pass_ms": split_pass_cost(fsl, torch, w.replace(storage=0))}
        log("bubble splitting", split)
        regimes = bubble_regimes(fsl, W, torch)
        log("bubble regimes", regimes)

    if args.calibrate_copy_gib > 0:
        nbytes = int(args.calibrate_copy_gib * (1 << 30))
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        b2 = torch.empty_like(a)
        for _ in range(3):
            b2.copy_(a)
        # the same bytes moved with 4 bytes per lane: views one float off the
        # allocation's alignment keep torch's elementwise kernel from vectorising
        a32, b32 = a.view(torch.float32)[1:], b2.view(torch.float32)[1:]
        for _ in range(3):
            torch.mul(a32, 1.0, out=b32)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {nbytes} bytes, then 3 of {nbytes - 4} bytes 4 bytes per lane")
        del a, b2, a32, b32
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        cpu = cpu_baseline(w, args.cpu_steps)

    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[st],
        "data": "synthetic",
        "config": {"workload": w.name, "box": list(w.n),
                   "particles": w.particles.n if w.particles is not None else 0,
                   "collision": "TRT" if w.trt else "SRT", "tau": w.tau,
                   "storage": args.storage, "face_forces": False, "step_ms_breakdown": breakdown},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if forms:
        out["forms"] = forms
    if adjoint:
        out["adjoint"] = adjoint
    if surface:
        out["surface_tension"] = surface
    if split:
        out["bubble_splitting"] = split
    if regimes:
        out["bubble_regimes"] = regimes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
