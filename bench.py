"""Benchmark of the FDTD-PIC step on one MI355X.

One step is the whole hot path on one batch of synthetic input: cell sort
(every 20 steps), H update, gather + Boris push + Esirkepov deposit of every
live particle, Drude J + E update, FP64 probe DFT.  The default workload is
the 512x256x256-cell (33.5M), 1 nm, 12-cell-CPML grating run with a
1e7-particle 100 keV bunch; all inputs are resident in HBM before timing.

Prints one JSON line: whole-step Gcell-updates/s as `value`, particle
pushes/s, the roofline of the dominant kernel (its VALU instruction issue rate
against the chip's issue peak when committed counters exist for its current
source, with its HBM fraction on algorithmic bytes beside it), the FP64
oracle timed on the host's cores on the whole workload, and the rest of the
metric: the 256x128x128 production run's rates, the 16-instance batched sweep
against its 16 plain runs, and pic_grad against the plain forward run.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Gcell-updates/s + particle-pushes/s (FP32) and % HBM roofline; "
          "batched/adjoint vs plain")
HBM_PEAK_GBS = 8000.0
# wave64 VALU instructions the chip can issue: 256 CUs x 4 SIMDs, one wave64
# instruction per SIMD every 4 cycles (16 lanes a cycle) at 2.4 GHz
VALU_PEAK_G = 256 * 4 * 2.4 / 4
FAMILIES = ("h_update", "push_deposit", "e_update", "probe", "sort", "field_sweep")
KERNEL_SOURCES = {"h_update": "kernels_fields.hip", "e_update": "kernels_fields.hip",
                  "push_deposit": "kernels_particles.hip", "sort": "kernels_particles.hip",
                  "probe": "kernels_diag.hip", "field_sweep": "kernels_fused.hip"}


def workload(name):
    import pic_inputs as pi
    table = {"grating40nm_512x256x256_cpml12": pi.grating_large,
             "film30nm_256x128x128_cpml8": pi.film_production,
             "film20nm_128x64x64_cpml8": pi.film_adjoint,
             "grating40nm_shard2of8_64x256x256": pi.grating_shard,
             "slab20nm_32x32x32_pec": pi.slab_tiny}
    return table[name]()


def cpml_memberships(w):
    """Sum over CPML axes of the cells inside that axis's two absorbing slabs."""
    n = (w.nx, w.ny, w.nz)
    tot = 0
    for a in range(3):
        if w.bc[a] == 2:
            tot += 2 * w.npml * (w.cells // n[a])
    return tot


def metal_box_cells(w):
    import numpy as np
    m = w.wp_map > 0
    if not m.any():
        return 0
    idx = [np.where(m.any(axis=tuple(b for b in range(3) if b != a)))[0] for a in range(3)]
    return int(np.prod([i.max() - i.min() + 1 for i in idx]))


def algorithmic_bytes(w, fam, pushes_per_step, pbox):
    """Bytes the method must move per launch (FP32 state, read + write).

    h_update : 36 B/cell (read E, read H, write H) + 16 B per CPML layer-axis
               membership (two psi, read + write)
    e_update : 36 B/cell + 16 B per membership + 32 B per metal-box cell
               (J_pol read + write, (cb, d)) + 24 B per bunch-box cell (J_b read + clear)
    push     : 48 B per live particle (x, u read + write)
    field_sweep : the one-pass E + H update: 48 B/cell (read E, H; write E,
               H) + the two updates' CPML, Drude and bunch-current bytes
    """
    N = w.cells
    mem = cpml_memberships(w)
    if fam == "h_update":
        return 36 * N + 16 * mem
    if fam == "e_update":
        box = 1
        for d in range(3):
            box *= max(0, pbox[3 + d] - pbox[d] + 1)
        return 36 * N + 16 * mem + 32 * metal_box_cells(w) + 24 * box
    if fam == "push_deposit":
        return 48 * pushes_per_step
    if fam == "field_sweep":
        return (algorithmic_bytes(w, "h_update", pushes_per_step, pbox) +
                algorithmic_bytes(w, "e_update", pushes_per_step, pbox) - 24 * N)
    return None


def source_sha(fam):
    """Hash of the kernel's source file and of the shared header that fixes its
    launch shapes and argument blocks."""
    csrc = os.path.join(ROOT, "paper_1505_04007_amd", "csrc")
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES[fam], "pic_internal.hpp"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def counters_for(fam, wname):
    """The committed rocprofv3 counter record of a kernel on a workload (HBM
    bytes per launch, VALU instructions per launch), or {} when none exists or
    the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return {}
    try:
        rec = json.load(open(path)).get(wname, {}).get(fam)
    except (ValueError, OSError):
        return {}
    if not rec or rec.get("source_sha") != source_sha(fam):
        return {}
    return rec


def traffic_for(fam, wname):
    return counters_for(fam, wname).get("bytes_per_launch")


def cpu_baseline(w, steps=6):
    """The FP64 oracle on the whole workload (full grid, every particle) for
    `steps` steps after one untimed step, its field loops and its particle
    chunks spread over the host's threads."""
    from oracle import pic_oracle as po
    b = w.bunch
    o = po.OracleSim(w.nx, w.ny, w.nz, w.dx, w.dt, bc=w.bc, npml=w.npml, pml=w.pml,
                     wp_map=w.wp_map, gamma_map=w.gamma_map)
    o.set_particles(b.x, b.y, b.z, b.ux, b.uy, b.uz, b.q, b.m, b.w)
    o.set_probes(w.probes, w.omega)
    o.step(1)  # first touch of the arrays, not timed
    t0 = o.timing()
    o.step(steps)
    t1 = o.timing()
    field_s = t1["field_s"] - t0["field_s"]
    part_s = t1["particle_s"] - t0["particle_s"]
    pushes = t1["pushes"] - t0["pushes"]
    return {"value": w.cells * steps / (field_s + part_s) / 1e9, "unit": "Gcell-updates/s",
            "cores": t1["threads"], "kind": "oracle",
            "sample": (f"the whole workload: {w.nx}x{w.ny}x{w.nz} grid and all {b.n} particles, "
                       f"{steps} steps after one untimed step; fields {field_s / steps:.3f} s and "
                       f"particles {part_s / steps:.3f} s per step, both parallel over "
                       f"{t1['threads']} threads"),
            "particle_pushes_per_s": pushes / part_s if part_s > 0 else None}


def step_bytes(w):
    """Algorithmic bytes of one whole step (H + E+Drude + pushes), bunch box excluded."""
    npart = w.bunch.n if w.bunch is not None else 0
    return (algorithmic_bytes(w, "h_update", 0, (0, 0, 0, -1, -1, -1)) +
            algorithmic_bytes(w, "e_update", 0, (0, 0, 0, -1, -1, -1)) + 48 * npart)


def run_batched(steps, warmup, tune_reps):
    """16 film/energy instances of uneven size: 16 sequential plain runs vs one
    batch (one launch per kernel family per step, captured sort-period graph).
    Both sides tuned (tune_reps > 0) or on the default tile."""
    import torch
    import pic_inputs as pi
    from paper_1505_04007_amd import native

    ws = pi.batched_sweep()
    cells = sum(w.cells for w in ws)
    pushes_total = 0
    plain_s = 0.0
    for w in ws:
        sim = native.from_workload(w)
        if tune_reps > 0:
            sim.tune(reps=tune_reps)
        sim.step(warmup)
        torch.cuda.synchronize()
        p0 = sim.stats()["pushes"]
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        plain_s += time.perf_counter() - t0
        pushes_total += sim.stats()["pushes"] - p0
        sim.close()
        del sim
    sims = [native.from_workload(w) for w in ws]
    batch = native.Batch(sims, use_graph=True)
    tune = batch.tune(reps=tune_reps) if tune_reps > 0 else batch.tune(force=0)
    batch.step(warmup)
    torch.cuda.synchronize()
    p0 = sum(s.stats()["pushes"] for s in sims)
    t0 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    pushes = sum(s.stats()["pushes"] for s in sims) - p0
    batch.close()
    for s_ in sims:
        s_.close()
    return {"ws": ws, "cells": cells, "steps": steps, "plain_s": plain_s, "batched_s": secs,
            "plain_pushes": pushes_total, "batched_pushes": pushes, "tile": tune}


def bench_batched(args):
    """The batched sweep as its own bench line."""
    r = run_batched(args.steps, args.warmup, 0 if args.no_tune else 5)
    ws, cells, secs, plain_s = r["ws"], r["cells"], r["batched_s"], r["plain_s"]
    tune, pushes, pushes_total = r["tile"], r["batched_pushes"], r["plain_pushes"]
    print(f"[bench] 16 plain runs: {plain_s:.3f} s, batched: {secs:.3f} s", file=sys.stderr, flush=True)
    gcells = cells * args.steps / secs / 1e9
    plain_g = cells * args.steps / plain_s / 1e9
    sb = sum(step_bytes(w) for w in ws)
    ach = sb * args.steps / secs / 1e9
    out = {"metric": METRIC, "value": round(gcells, 3), "unit": "Gcell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * secs / args.steps, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batched16_film5-80nm_128x64x64-192x96x96", "instances": len(ws),
                      "cells": cells, "particles": sum(w.bunch.n for w in ws), "sort_every": 20,
                      "field_tile": [tune["fx"], tune["fy"], tune["order"]], "parallelism": "single-gpu"},
           "particle_pushes_per_s": round(pushes / secs, 1),
           "plain_sequential": {"value": round(plain_g, 3), "unit": "Gcell-updates/s",
                                "particle_pushes_per_s": round(pushes_total / plain_s, 1)},
           "batched_vs_plain": round(gcells / plain_g, 3),
           "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "whole batched step (H + push + E+Drude, algorithmic bytes)"},
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def run_adjoint(N, warmup):
    """pic_grad on the 128x64x64, 20 nm film, 1e5-particle workload: the
    differentiated run (a forward run that keeps what the reverse pass needs:
    every step's metal-box state when that fits in half the free device
    memory, else checkpoints and a replay; then the adjoint) against the plain
    forward run of the same steps."""
    import torch
    import pic_inputs as pi
    from paper_1505_04007_amd import native

    w = pi.film_adjoint()
    N = w.steps if N is None else N
    w0 = w.meta["omega0"]
    warm = native.from_workload(w)
    warm.grad(w0, max(warmup, 1))
    warm.close()
    plain = native.from_workload(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain.step(N)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    pushes = plain.stats()["pushes"]
    plain.close()
    sim = native.from_workload(w)
    # pic_grad's automatic choice: every step's metal-box snapshot kept from the
    # forward run when they fit in half the free memory, else sqrt(N) checkpoints
    free_b, _ = torch.cuda.mem_get_info()
    replay = ("snapshots of every step, no replay" if N * 24 * metal_box_cells(w) <= free_b / 2
              else f"checkpoints every {int(np.ceil(np.sqrt(N)))} steps, replayed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L, gw, gg = sim.grad(w0, N)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    sim.close()
    return {"w": w, "N": N, "plain_s": tf, "grad_s": tg, "pushes": pushes, "L": L, "gw": gw, "gg": gg,
            "replay": replay}


def bench_adjoint(args):
    """The adjoint workload as its own bench line."""
    r = run_adjoint(args.steps, args.warmup)
    w, N, tf, tg, pushes, L, gw, gg, replay = (r["w"], r["N"], r["plain_s"], r["grad_s"], r["pushes"],
                                               r["L"], r["gw"], r["gg"], r["replay"])
    print(f"[bench] plain {N} steps: {tf:.3f} s; pic_grad {tg:.3f} s, L = {L:.4e}", file=sys.stderr, flush=True)
    gcells = w.cells * N / tg / 1e9
    out = {"metric": METRIC, "value": round(gcells, 3), "unit": "Gcell-updates/s", "n_gpus": 1,
           "steps": N, "warmup": args.warmup, "ms_per_step": round(1e3 * tg / N, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": w.name + "_adjoint", "cells": w.cells, "particles": w.bunch.n,
                      "sort_every": w.sort_every, "objective": "sum_p |F_p(0.68 wp)|^2",
                      "reverse_pass": replay, "parallelism": "single-gpu"},
           "plain_forward": {"value": round(w.cells * N / tf / 1e9, 3), "unit": "Gcell-updates/s",
                             "seconds": round(tf, 4), "particle_pushes_per_s": round(pushes / tf, 1)},
           "grad_seconds": round(tg, 4),
           "adjoint_vs_plain": round(tg / tf, 3),
           "grad_norms": {"dL_dwp": float(np.linalg.norm(gw)), "dL_dgamma": float(np.linalg.norm(gg)),
                          "L": L},
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def run_production(steps, warmup):
    """The 256x128x128, 2 nm, 8-cell-CPML production run (30 nm film, 1e6
    particles at 50 keV): whole-step Gcell-updates/s and pushes/s, every
    particle live over the timed steps.  Its state (~0.15 GB) fits in the
    256 MB Infinity Cache, so its rates are not an HBM measurement."""
    import torch
    import pic_inputs as pi
    from paper_1505_04007_amd import native

    w = pi.film_production()
    sim = native.from_workload(w)
    tune = sim.tune(reps=5)
    sim.step(warmup)
    torch.cuda.synchronize()
    p0 = sim.stats()["pushes"]
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = sim.stats()
    sim.close()
    return {"workload": w.name, "cells": w.cells, "particles": w.bunch.n, "steps": steps,
            "value": round(w.cells * steps / secs / 1e9, 3), "unit": "Gcell-updates/s",
            "particle_pushes_per_s": round((st["pushes"] - p0) / secs, 1),
            "live_particles": st["live"], "ms_per_step": round(1e3 * secs / steps, 4),
            "field_tile": [tune["fx"], tune["fy"], tune["order"]]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 200; the adjoint workload: its 2000)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="grating40nm_512x256x256_cpml12")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the production, batched and adjoint legs of the default line")
    ap.add_argument("--deposit-mode", type=int, default=0)
    ap.add_argument("--field-sweep", type=int, default=0,
                    help="1: the one-pass E + H field sweep instead of the separate launches")
    ap.add_argument("--timing-every", type=int, default=7,
                    help="time the kernels of every this many steps with HIP events (every sort "
                         "too); 1 = every step.  Coprime to the sort interval, so the sample covers "
                         "every phase of it")
    ap.add_argument("--sort-every", type=int, default=None,
                    help="override the workload's cell-sort interval")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default field tile instead of running the autotuner")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                          "GBps_read_plus_write": round(2 * (1 << 30) / dt / 1e9, 1)}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1505_04007_amd import native

    if args.workload == "batched16":
        torch.cuda.set_device(0)
        args.steps = 200 if args.steps is None else args.steps
        bench_batched(args)
        return
    if args.workload == "adjoint":
        torch.cuda.set_device(0)
        bench_adjoint(args)
        return
    args.steps = 200 if args.steps is None else args.steps
    if args.steps < args.timing_every:
        # fewer steps than the interval might hold no sampled step at all
        args.timing_every = 1
    w = workload(args.workload)
    torch.cuda.set_device(0)
    if args.sort_every is not None:
        w.sort_every = args.sort_every
    sim = native.from_workload(w, timing=args.timing_every, deposit_mode=args.deposit_mode,
                               field_sweep=args.field_sweep)
    tune = sim.tune(force=0) if args.no_tune else sim.tune(reps=10)
    if not args.no_tune:
        print("[bench] tile variants ms per H+E pair: " + " ".join(f"{m:.3f}" for m in tune["ms"]),
              file=sys.stderr, flush=True)
    print(f"[bench] {w.name}: {w.cells} cells, {w.bunch.n if w.bunch else 0} particles, "
          f"warmup {args.warmup}, field tile {tune['fx']}x{tune['fy']} order {tune['order']}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    p0 = sim.stats()["pushes"]
    sim.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sim.stats()
    fams = sim.timing(reset=True)
    sim.step(0)
    pushes = st["pushes"] - p0
    secs = t1 - t0
    ms_per_step = 1e3 * secs / args.steps
    gcells = w.cells * args.steps / secs / 1e9
    print(f"[bench] timed {args.steps} steps in {secs:.3f} s", file=sys.stderr, flush=True)

    # device time of each family over the timed region: the sampled steps'
    # launches stand for timing_every steps each; every sort is timed
    est = {f: fams[f][0] * (1 if f == "sort" else args.timing_every) for f in FAMILIES}
    dom = max(est, key=est.get)
    ms_tot, launches = fams[dom]
    avg_s = ms_tot / 1e3 / max(launches, 1)
    per_step_push = pushes / args.steps
    algo = algorithmic_bytes(w, dom, per_step_push, st["pbox"])
    roof = None
    if algo is not None and avg_s > 0:
        ach = algo / avg_s / 1e9
        rec = counters_for(dom, w.name)
        hbm = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": rec.get("bytes_per_launch")}
        roof = dict(hbm, kernel=dom, algorithmic_bytes_per_launch=algo, avg_launch_ms=round(avg_s * 1e3, 4))
        if rec.get("valu_per_launch"):
            # VALU-issue bound: committed SQ_INSTS_VALU per launch over the live launch time
            va = rec["valu_per_launch"] / avg_s / 1e9
            roof = {"bound": "alu", "achieved": round(va, 1), "peak": VALU_PEAK_G,
                    "unit": "G wave64-VALU-instructions/s", "frac": round(va / VALU_PEAK_G, 4),
                    "traffic": rec.get("bytes_per_launch"), "kernel": dom,
                    "valu_per_launch": rec["valu_per_launch"], "avg_launch_ms": round(avg_s * 1e3, 4),
                    "hbm": {k: hbm[k] for k in ("achieved", "peak", "unit", "frac")},
                    "algorithmic_bytes_per_launch": algo}
    kernels = {}
    for f in FAMILIES:
        ms, n = fams[f]
        if n == 0:
            continue
        b = algorithmic_bytes(w, f, per_step_push, st["pbox"])
        kernels[f] = {"avg_ms": round(ms / n, 4), "launches_timed": n,
                      "share": round(est[f] / max(sum(est.values()), 1e-12), 3)}
        if b is not None:
            kernels[f]["algo_GBps"] = round(b / (ms / n / 1e3) / 1e9, 1)

    del sim
    extra = {}
    if not args.no_extras and args.workload == "grating40nm_512x256x256_cpml12":
        # the rest of the metric, each on its own workload
        prod = run_production(100, 20)
        print(f"[bench] production {prod['workload']}: {prod['value']} Gcell/s, "
              f"{prod['particle_pushes_per_s']:.3e} pushes/s", file=sys.stderr, flush=True)
        bt = run_batched(100, 20, 5)
        cells_b = bt["cells"]
        plain_g = cells_b * bt["steps"] / bt["plain_s"] / 1e9
        batch_g = cells_b * bt["steps"] / bt["batched_s"] / 1e9
        print(f"[bench] batched16: {batch_g:.2f} vs plain {plain_g:.2f} Gcell/s", file=sys.stderr, flush=True)
        ad = run_adjoint(None, 5)
        print(f"[bench] adjoint: pic_grad {ad['grad_s']:.3f} s vs plain {ad['plain_s']:.3f} s",
              file=sys.stderr, flush=True)
        extra = {
            "production": prod,
            "batched_vs_plain": round(batch_g / plain_g, 3),
            "batched": {"workload": "batched16_film5-80nm_128x64x64-192x96x96", "instances": len(bt["ws"]),
                        "cells": cells_b, "steps": bt["steps"], "value": round(batch_g, 3),
                        "plain_sequential_value": round(plain_g, 3), "unit": "Gcell-updates/s",
                        "particle_pushes_per_s": round(bt["batched_pushes"] / bt["batched_s"], 1),
                        "field_tile": [bt["tile"]["fx"], bt["tile"]["fy"], bt["tile"]["order"]]},
            "adjoint_vs_plain": round(ad["grad_s"] / ad["plain_s"], 3),
            "adjoint": {"workload": ad["w"].name, "steps": ad["N"], "grad_seconds": round(ad["grad_s"], 4),
                        "plain_forward_seconds": round(ad["plain_s"], 4), "reverse_pass": ad["replay"],
                        "note": "ratio = time of pic_grad (forward + reverse) / time of the plain forward run"},
        }

    cpu = None
    if not args.no_cpu_baseline and w.bunch is not None:
        print("[bench] timing the oracle on host cores", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w)

    out = {"metric": METRIC, "value": round(gcells, 3), "unit": "Gcell-updates/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "cells": w.cells,
                      "particles": w.bunch.n if w.bunch else 0, "sort_every": w.sort_every,
                      "deposit_mode": args.deposit_mode, "field_sweep": args.field_sweep,
                      "kernels_timed_every": args.timing_every,
                      "field_tile": [tune["fx"], tune["fy"], tune["order"]],
                      "parallelism": "single-gpu"},
           "particle_pushes_per_s": round(pushes / secs, 1),
           "roofline": roof, "kernels": kernels, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
