"""Benchmark of the FDTD-PIC step on one MI355X.

One step is the whole hot path on one batch of synthetic input: cell sort
(every 20 steps), H update, gather + Boris push + Esirkepov deposit of every
live particle, Drude J + E update, FP64 probe DFT.  The default workload is
the 512x256x256-cell (33.5M), 1 nm, 12-cell-CPML grating run with a
1e7-particle 100 keV bunch; all inputs are resident in HBM before timing.

Prints one JSON line: whole-step Gcell-updates/s as `value`, particle
pushes/s, the HBM roofline of the dominant kernel (algorithmic bytes per
launch / HIP-event launch time), and the FP64 oracle timed on host cores on a
bounded sample of the same workload.
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
FAMILIES = ("h_update", "push_deposit", "e_update", "probe", "sort")
KERNEL_SOURCES = {"h_update": "kernels_fields.hip", "e_update": "kernels_fields.hip",
                  "push_deposit": "kernels_particles.hip", "sort": "kernels_particles.hip",
                  "probe": "kernels_diag.hip"}


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
    return None


def source_sha(fam):
    """Hash of the kernel's source file and of the shared header that fixes its
    launch shapes and argument blocks."""
    csrc = os.path.join(ROOT, "paper_1505_04007_amd", "csrc")
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES[fam], "pic_internal.hpp"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(fam, wname):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when no summary exists or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(wname, {}).get(fam)
    except (ValueError, OSError):
        return None
    if not rec or rec.get("source_sha") != source_sha(fam):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(w, nsub=200_000, steps=16):
    """The FP64 oracle on the full grid of the same workload for `steps` steps
    with a 1/(n/nsub) subsample of the bunch; the per-push time is scaled to
    the full bunch to give the per-step time of the whole workload."""
    import numpy as np
    from oracle import pic_oracle as po
    b = w.bunch
    idx = np.arange(0, b.n, max(1, b.n // nsub))[:nsub]
    sub = b.subset(idx)
    o = po.OracleSim(w.nx, w.ny, w.nz, w.dx, w.dt, bc=w.bc, npml=w.npml, pml=w.pml,
                     wp_map=w.wp_map, gamma_map=w.gamma_map)
    o.set_particles(sub.x, sub.y, sub.z, sub.ux, sub.uy, sub.uz, sub.q, b.m, b.w)
    o.set_probes(w.probes, w.omega)
    o.step(steps)
    t = o.timing()
    field_s = t["field_s"] / steps
    push_s = t["particle_s"] / max(t["pushes"], 1)
    step_s = field_s + push_s * b.n
    return {"value": w.cells / step_s / 1e9, "unit": "Gcell-updates/s", "cores": t["threads"],
            "kind": "oracle",
            "sample": (f"full {w.nx}x{w.ny}x{w.nz} grid, {steps} steps, {len(idx)} of {b.n} "
                       f"particles; field time per step {field_s:.2f} s measured, push time "
                       f"{push_s * 1e6:.2f} us/push scaled to the full bunch"),
            "particle_pushes_per_s": 1.0 / push_s}


def step_bytes(w):
    """Algorithmic bytes of one whole step (H + E+Drude + pushes), bunch box excluded."""
    npart = w.bunch.n if w.bunch is not None else 0
    return (algorithmic_bytes(w, "h_update", 0, (0, 0, 0, -1, -1, -1)) +
            algorithmic_bytes(w, "e_update", 0, (0, 0, 0, -1, -1, -1)) + 48 * npart)


def bench_batched(args):
    """16 film/energy instances of uneven size: 16 sequential plain runs vs one
    batch (one launch per kernel family per step, captured sort-period graph)."""
    import torch
    import pic_inputs as pi
    from paper_1505_04007_amd import native

    ws = pi.batched_sweep()
    cells = sum(w.cells for w in ws)
    pushes_total = 0
    plain_s = 0.0
    for w in ws:
        sim = native.from_workload(w)
        if not args.no_tune:
            sim.tune(reps=5)
        sim.step(args.warmup)
        torch.cuda.synchronize()
        p0 = sim.stats()["pushes"]
        t0 = time.perf_counter()
        sim.step(args.steps)
        torch.cuda.synchronize()
        plain_s += time.perf_counter() - t0
        pushes_total += sim.stats()["pushes"] - p0
        sim.close()
        del sim
    print(f"[bench] 16 plain runs: {plain_s:.3f} s", file=sys.stderr, flush=True)
    sims = [native.from_workload(w) for w in ws]
    batch = native.Batch(sims, use_graph=True)
    tune = batch.tune(force=0) if args.no_tune else batch.tune(reps=5)
    batch.step(args.warmup)
    torch.cuda.synchronize()
    p0 = sum(s.stats()["pushes"] for s in sims)
    t0 = time.perf_counter()
    batch.step(args.steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    pushes = sum(s.stats()["pushes"] for s in sims) - p0
    print(f"[bench] batched: {secs:.3f} s", file=sys.stderr, flush=True)
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


def bench_adjoint(args):
    """pic_grad on the 128x64x64, 20 nm film, 1e5-particle workload: the
    differentiated run (a forward run that keeps what the reverse pass needs:
    every step's metal-box state when that fits in half the free device
    memory, else checkpoints and a replay; then the adjoint) against the plain
    forward run of the same steps."""
    import torch
    import pic_inputs as pi
    from paper_1505_04007_amd import native

    w = pi.film_adjoint()
    N = args.steps if args.steps is not None else w.steps
    w0 = w.meta["omega0"]
    warm = native.from_workload(w)
    warm.grad(w0, max(args.warmup, 1))
    warm.close()
    plain = native.from_workload(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain.step(N)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    pushes = plain.stats()["pushes"]
    plain.close()
    print(f"[bench] plain {N} steps: {tf:.3f} s", file=sys.stderr, flush=True)
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
    print(f"[bench] pic_grad {N} steps: {tg:.3f} s, L = {L:.4e}", file=sys.stderr, flush=True)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 200; the adjoint workload: its 2000)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="grating40nm_512x256x256_cpml12")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--deposit-mode", type=int, default=0)
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
    w = workload(args.workload)
    torch.cuda.set_device(0)
    if args.sort_every is not None:
        w.sort_every = args.sort_every
    sim = native.from_workload(w, timing=True, deposit_mode=args.deposit_mode)
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

    # dominant kernel family by total device time
    dom = max(fams, key=lambda f: fams[f][0])
    ms_tot, launches = fams[dom]
    avg_s = ms_tot / 1e3 / max(launches, 1)
    per_step_push = pushes / args.steps
    algo = algorithmic_bytes(w, dom, per_step_push, st["pbox"])
    roof = None
    if algo is not None:
        ach = algo / avg_s / 1e9
        tr = traffic_for(dom, w.name)
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": tr, "kernel": dom,
                "algorithmic_bytes_per_launch": algo, "avg_launch_ms": round(avg_s * 1e3, 4)}
    kernels = {}
    for f in FAMILIES:
        ms, n = fams[f]
        if n == 0:
            continue
        b = algorithmic_bytes(w, f, per_step_push, st["pbox"])
        kernels[f] = {"avg_ms": round(ms / n, 4), "launches": n,
                      "share": round(ms / max(sum(v[0] for v in fams.values()), 1e-12), 3)}
        if b is not None:
            kernels[f]["algo_GBps"] = round(b / (ms / n / 1e3) / 1e9, 1)

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
                      "deposit_mode": args.deposit_mode, "field_tile": [tune["fx"], tune["fy"], tune["order"]],
                      "parallelism": "single-gpu"},
           "particle_pushes_per_s": round(pushes / secs, 1),
           "roofline": roof, "kernels": kernels, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
