"""Throughput of diffusion-based coarse graining on one MI355X.

One step = one cgd_coarse_grain call over the dense particle bed: PCM
deposition of 20M particles into a 256 x 256 x 512 hex mesh (box 1 x 1 x 2,
h = 1/256), then 4 backward-Euler pseudo-steps of T = b^2/4 with b = 4h,
each a conjugate-gradient solve (preconditioned by a Chebyshev polynomial of
the operator) to rtol 1e-6.  Inputs are resident in HBM before timing.
value = fields coarse-grained per second.

Prints one JSON line.  Also reports:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                mean duration (HIP events on the library's stream), vs 8 TB/s
  cpu_baseline  the CPU oracle timed on a bounded sample of the same recipe
  rel_l2        accuracy of the timed result against the float64 oracle
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coarse-grained fields/sec at 256^3, 20M particles, rel L2<=1e-5 vs FP64"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fields", type=int, default=1, help="1: volume; 4: volume + 3 drag components")
    ap.add_argument("--particles", type=int, default=20_000_000)
    ap.add_argument("--shape", default="256,256,512")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=4)
    ap.add_argument("--no-check", action="store_true", help="skip the float64 accuracy check")
    ap.add_argument("--scheme", default="be", choices=["be", "cn"],
                    help="dense workload's integrator: backward Euler (the headline) or Crank-Nicolson")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="dense workload only: skip the other workloads' short runs")
    ap.add_argument("--profile-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--workload", default="dense", choices=["dense", "batched", "unstructured", "learned", "stretched"],
                    help="dense: the headline metric; batched: 64 snapshots x 4 fields on 128^3 in one "
                         "persistent launch; unstructured: 100^3 x 6 jittered tets; learned: train the "
                         "initial-guess network on advected snapshots, then compare initial guesses")
    ap.add_argument("--snapshots", type=int, default=64)
    ap.add_argument("--train-snapshots", type=int, default=1500)
    ap.add_argument("--test-snapshots", type=int, default=500)
    ap.add_argument("--lr", type=float, default=1e-3)
    return ap.parse_args()


# Sources the hex sweep kernels are built from, in the order their bytes are
# hashed for the counter summary's source_sha256.
SWEEP_SOURCES = ("cg_hex.hip", "stencil_tile.h", "precond_lds.h", "cg_common.h", "cg_common.hip")


def sweep_source_sha():
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_1409_0001_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_from_profiles():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current sweep sources (else None)."""
    path = os.path.join(ROOT, "profiles", "cg_sweep_traffic_dense_bed.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256") != sweep_source_sha():
        return None
    return d


# Timed kernels (cgd_timing_read kinds) that are one kernel each; "deposit"
# spans several and is split into its stages.
SOLVE_KERNELS = ("cg_sweep1", "cg_sweep2", "cg_precond_pass1", "cg_precond_pass_mid", "cg_precond_pass_last",
                 "cg_first_sweep1", "cg_first_sweep2", "cg_first_precond_pass1", "cg_first_precond_pass_mid",
                 "cg_first_precond_pass_last")
DEPOSIT_KERNELS = ("deposit_bin", "deposit_scatter", "deposit_accum")


def roofline_of(tim, ms_per_field):
    """Every timed kernel ranked by its total time on the last timed step;
    the dominant one (most total time) gives the roofline line: its
    algorithmic bytes per launch over its mean launch time, against 8 TB/s.
    Also the whole solve's and the whole call's algorithmic bytes over their
    time."""
    rows = []
    for k in SOLVE_KERNELS + DEPOSIT_KERNELS:
        n, ms, bpl = tim[k]
        if n:
            rows.append((k, n, ms, bpl))
    rows.sort(key=lambda r: -r[2])
    dom, launches, total_ms, bpl = rows[0]
    avg_ms = total_ms / launches
    achieved = bpl / (avg_ms * 1e-3) / 1e9
    tr = traffic_from_profiles()
    traffic = None
    if tr and dom in tr.get("kernels", {}):
        traffic = tr["kernels"][dom]["hbm_bytes_per_launch"]
    ranked = [{"kernel": k, "launches": n, "total_us": round(ms * 1e3, 1), "avg_us": round(ms / n * 1e3, 2),
               "algorithmic_bytes_per_launch": b, "achieved_GBs": round(b / (ms / n * 1e-3) / 1e9, 1),
               "frac": round(b / (ms / n * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)} for k, n, ms, b in rows]
    sb = sum(b * n for k, n, ms, b in rows if k in SOLVE_KERNELS)
    st = sum(ms for k, n, ms, b in rows if k in SOLVE_KERNELS)
    db = sum(b * n for k, n, ms, b in rows if k in DEPOSIT_KERNELS)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": dom, "launches": launches, "avg_us": round(avg_ms * 1e3, 2),
            "algorithmic_bytes_per_launch": bpl,
            "whole_solve": {"algorithmic_GB": round(sb / 1e9, 3), "kernel_ms": round(st, 3),
                            "achieved_GBs": round(sb / (st * 1e-3) / 1e9, 1),
                            "frac": round(sb / (st * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "whole_call_wall": {"algorithmic_GB": round((sb + db) / 1e9, 3), "ms": round(ms_per_field, 3),
                                "frac": round((sb + db) / (ms_per_field * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "kernels_by_total_time": ranked}


def host_cpu():
    """CPU model and the number of cores the process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(args):
    """The oracle as it stands (float64, scipy CG), single thread, on the
    dense-bed recipe at 1/8 of the cells and particles; scaled to fields/s
    of the full workload by the cell ratio."""
    from threadpoolctl import threadpool_limits

    from oracle import cgd_oracle as O
    from paper_1409_0001_amd import inputs
    nx, ny, nz = (int(v) for v in args.shape.split(","))
    sx, sy, sz = nx // 2, ny // 2, nz // 2
    ratio = (nx * ny * nz) / (sx * sy * sz)
    w = inputs.dense_bed(n_particles=int(args.particles / ratio), shape=(sx, sy, sz), n_fields=1)
    with threadpool_limits(1):
        t = time.perf_counter()
        O.coarse_grain_hex(w.particles.pos, w.particles.values, w.box.lo, w.box.hi, w.box.shape,
                           w.bandwidth, w.n_steps, rtol=1e-12, scheme=args.scheme)
        dt = time.perf_counter() - t
    model, nproc = host_cpu()
    return {"value": 1.0 / (dt * ratio), "unit": "fields/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_nproc": nproc,
            "sample": f"dense-bed recipe at {sx}x{sy}x{sz} cells, {w.particles.pos.shape[0]} particles "
                      f"(1/{ratio:g} of the workload), 1 field, deposit + 4 "
                      f"{'backward-Euler' if args.scheme == 'be' else 'Crank-Nicolson'} steps by "
                      f"float64 CG to 1e-12; {dt:.1f} s, scaled by the cell ratio"}


def bench_batched(args):
    """64 snapshots on a 128^3 hex mesh, particle counts U{0.5M..4M}, 4 fields
    each (volume + 3 drag components), all 256 right-hand sides per call; and
    the same work as 64 single-snapshot calls for comparison."""
    import numpy as np
    import torch

    import paper_1409_0001_amd as cgd
    from paper_1409_0001_amd import inputs
    t0 = time.perf_counter()
    snaps = [inputs.batched_snapshot(j) for j in range(args.snapshots)]
    counts = [len(p.pos) for p in snaps]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    pos = torch.from_numpy(np.concatenate([p.pos for p in snaps])).cuda()
    vals = torch.from_numpy(np.concatenate([p.values for p in snaps], axis=1)).cuda()
    print(f"[bench] {args.snapshots} snapshots, {int(off[-1])} particles in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    shape = (128, 128, 128)
    mesh = cgd.HexMesh(shape)
    b, steps, F = 4.0 / 128, 4, 4
    n_rhs = args.snapshots * F
    fields = torch.empty((args.snapshots, F, mesh.cells), dtype=torch.float32, device="cuda")
    chosen, tune_ms = cgd.autotune_batched(mesh, n_rhs)
    # warm-up with the timed call's arguments (its graph is captured there)
    for _ in range(max(1, args.warmup)):
        cgd.coarse_grain_batched(mesh, off, pos, vals, b, steps, rtol=args.rtol, fields=fields)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        cgd.coarse_grain_batched(mesh, off, pos, vals, b, steps, rtol=args.rtol, fields=fields)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    # the same call with per-snapshot statistics (untimed)
    _, iters, bstats = cgd.coarse_grain_batched(mesh, off, pos, vals, b, steps, rtol=args.rtol, fields=fields,
                                                return_iters=True, stats=True)
    # the same batched call with plain (unpreconditioned) CG
    _, iters_plain = cgd.coarse_grain_batched(mesh, off, pos, vals, b, steps, rtol=args.rtol, fields=fields,
                                              return_iters=True, precond=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        cgd.coarse_grain_batched(mesh, off, pos, vals, b, steps, rtol=args.rtol, fields=fields, precond=1)
    torch.cuda.synchronize()
    dt_plain = (time.perf_counter() - t) / args.steps
    # the same right-hand sides, one cgd_coarse_grain call per snapshot
    single = torch.empty((F, mesh.cells), dtype=torch.float32, device="cuda")
    p0 = [pos[off[j]:off[j + 1]].contiguous() for j in range(args.snapshots)]
    v0 = [vals[:, off[j]:off[j + 1]].contiguous() for j in range(args.snapshots)]
    cgd.coarse_grain(mesh, p0[0], v0[0], b, steps, rtol=args.rtol, field=single)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for j in range(args.snapshots):
        cgd.coarse_grain(mesh, p0[j], v0[j], b, steps, rtol=args.rtol, field=single)
    torch.cuda.synchronize()
    dt_loop = time.perf_counter() - t
    it_total = int(iters.sum())
    # preconditioned CG: 8 (z = M r) + 12 (direction) + 20 (update) bytes per cell and iteration
    alg_bytes = 40.0 * mesh.cells * it_total
    rel = None
    if not args.no_check:
        from oracle import cgd_oracle as O
        out = fields.cpu().numpy()
        rng = np.random.default_rng(7)
        rels = []
        for j in rng.choice(args.snapshots, min(8, args.snapshots), replace=False):
            p = snaps[j]
            dep = O.deposit_hex(p.pos, p.values, (0, 0, 0), (1, 1, 1), shape)
            ref = O.diffuse_hex_dct(dep["field64"], (0, 0, 0), (1, 1, 1), shape, b, steps)
            f = int(rng.integers(F))
            rels.append(float(np.linalg.norm(out[j, f] - ref[f]) / np.linalg.norm(ref[f])))
        rel = max(rels)
    line = {"metric": "coarse-grained fields/sec, batched 64 snapshots x 4 fields on 128^3",
            "value": round(n_rhs / dt, 2), "unit": "fields/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 2), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"batched {args.snapshots} snapshots x {F} fields, 128^3 hex, "
                                   f"{int(off[-1])} particles, b=4h, 4 backward-Euler steps, "
                                   f"polynomial-preconditioned CG rtol {args.rtol:g}",
                       "right_hand_sides": n_rhs, "cg_iters_total": it_total,
                       "cg_iters_per_rhs_step_mean": round(it_total / (n_rhs * steps), 2),
                       "autotune_choice": chosen, "autotune_ms": [round(x, 3) for x in tune_ms]},
            "looped_single_calls": {"value": round(n_rhs / dt_loop, 2), "unit": "fields/s",
                                    "ms": round(dt_loop * 1e3, 2)},
            "batched_plain_cg": {"value": round(n_rhs / dt_plain, 2), "unit": "fields/s",
                                 "ms": round(dt_plain * 1e3, 2),
                                 "cg_iters_per_rhs_step_mean": round(int(iters_plain.sum()) / (n_rhs * steps), 2)},
            "speedup_vs_plain_cg": round(dt_plain / dt, 3),
            "speedup_vs_looped": round(dt_loop / dt, 3),
            "solver_GBs_algorithmic_over_whole_call": round(alg_bytes / dt / 1e9, 1),
            "rel_l2_sampled": rel,
            "stats_sample": {"snapshot0_frac_bits": bstats[0].frac_bits, "snapshot0_n_dropped": bstats[0].n_dropped,
                             "max_rel_mass_change": max(abs(a - b_) / max(abs(b_), 1e-300)
                                                        for st_ in bstats for a, b_ in zip(st_.mass_after,
                                                                                           st_.mass_before))}}
    return line


def bench_unstructured(args):
    """100^3 hexes x 6 jittered tets (6M cells), 5M particles, b = 0.04,
    4 backward-Euler steps, polynomial-preconditioned CG rtol 1e-6."""
    import numpy as np
    import torch

    import paper_1409_0001_amd as cgd
    from paper_1409_0001_amd import inputs
    t0 = time.perf_counter()
    xyz, tets, parts, b, steps, rtol = inputs.unstructured()
    mesh = cgd.TetMesh(xyz, tets)
    print(f"[bench] tet mesh {len(tets)} cells, nnz {mesh.nnz}, built in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    pos = torch.from_numpy(parts.pos).cuda()
    vals = torch.from_numpy(parts.values).cuda()
    out = torch.empty((1, mesh.cells), dtype=torch.float32, device="cuda")
    for _ in range(max(1, args.warmup)):
        _, st = cgd.coarse_grain(mesh, pos, vals, b, steps, rtol=rtol, field=out, stats=True)
    cgd.timing_read(mesh, reset=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        if i == args.steps - 1:  # events on the last timed step only (as for the dense bed)
            cgd.timing_enable(mesh, True)
        cgd.coarse_grain(mesh, pos, vals, b, steps, rtol=rtol, field=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    cgd.timing_enable(mesh, False)
    tim = cgd.timing_read(mesh, reset=True)
    rl = {}
    for k in ("pcg_spmv_sweep", "pcg_update_sweep", "pcg_poly_pass_bv", "pcg_poly_pass_factor", "deposit"):
        n, ms, bpl = tim[k]
        if n:
            rl[k] = {"launches": n, "avg_us": round(ms / n * 1e3, 2), "total_ms": round(ms, 3),
                     "achieved_GBs": round(bpl / (ms / n * 1e-3) / 1e9, 1)}
    # one application of the polynomial per iteration that ran (timed: the
    # update sweeps after each step's first, plus the first); each takes
    # degree / 2 passes w = B v
    apps = tim["pcg_update_sweep"][0] + steps
    degree = 2 * tim["pcg_poly_pass_bv"][0] // max(1, apps)
    line = {"metric": "coarse-grained fields/sec, unstructured 6M tets, 5M particles",
            "value": round(1.0 / dt, 3), "unit": "fields/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 2), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "100^3 hexes x 6 jittered Kuhn tets, 5M particles, b=0.04, 4 backward-Euler "
                                   "steps, CG rtol 1e-6 preconditioned by a Chebyshev polynomial of the "
                                   "Jacobi-scaled operator", "cells": int(mesh.cells), "nnz": mesh.nnz,
                       "poly_degree": int(degree), "pcg_iters_per_step": [r[0] for r in st.iters]},
            "kernels": rl}
    return line


def bench_stretched(args):
    """Stretched hex mesh with a cell-wise diffusivity: the dense-bed box and
    particles (1 x 1 x 2, 20M particles) on 256 x 256 x 512 cells whose x
    widths grow by 1 % per cell away from the centre plane (3.5 : 1 from the
    centre to the walls), diffusivity 0 in the outermost cells (|x - 1/2| >
    0.45: PCM there), b = 4/256, 4 backward-Euler steps, rtol 1e-6 (the
    diffusivity depends on x only, so the stencil sweeps with per-axis
    factors run it, preconditioned by the Chebyshev polynomial of the
    scaled operator)."""
    import numpy as np
    import torch

    import paper_1409_0001_amd as cgd
    from paper_1409_0001_amd import inputs
    t0 = time.perf_counter()
    w = inputs.dense_bed(n_particles=args.particles, shape=(256, 256, 512), n_fields=1)
    wx = 1.01 ** np.arange(128)
    wx *= 0.5 / wx.sum()
    half = np.concatenate(([0.0], np.cumsum(wx)))
    ex = np.concatenate((0.5 - half[::-1], 0.5 + half[1:]))
    ex[0], ex[-1] = 0.0, 1.0
    ey, ez = np.linspace(0.0, 1.0, 257), np.linspace(0.0, 2.0, 513)
    xc = 0.5 * (ex[1:] + ex[:-1])
    D = np.broadcast_to((np.abs(xc - 0.5) <= 0.45).astype(np.float32), (512, 256, 256)).ravel()
    mesh = cgd.RectMesh(ex, ey, ez, diffusivity=D)
    print(f"[bench] stretched mesh {mesh.cells} cells, nnz {mesh.nnz}, inputs in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    pos = torch.from_numpy(w.particles.pos).cuda()
    vals = torch.from_numpy(w.particles.values).cuda()
    out = torch.empty((1, mesh.cells), dtype=torch.float32, device="cuda")
    b, steps, rtol = 4.0 / 256.0, 4, args.rtol
    for _ in range(max(1, args.warmup)):
        _, st = cgd.coarse_grain(mesh, pos, vals, b, steps, rtol=rtol, field=out, stats=True)
    cgd.timing_read(mesh, reset=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        if i == args.steps - 1:
            cgd.timing_enable(mesh, True)
        cgd.coarse_grain(mesh, pos, vals, b, steps, rtol=rtol, field=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    cgd.timing_enable(mesh, False)
    tim = cgd.timing_read(mesh, reset=True)
    rl = {}
    for k, v in tim.items():
        n, ms, bpl = v
        if n:
            rl[k] = {"launches": n, "avg_us": round(ms / n * 1e3, 2),
                     "achieved_GBs": round(bpl / (ms / n * 1e-3) / 1e9, 1)}
    line = {"metric": "coarse-grained fields/sec, stretched hex 256x256x512, 20M particles",
            "value": round(1.0 / dt, 3), "unit": "fields/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 2), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "dense-bed particles on a 256x256x512 rectilinear mesh, x widths +1 %/cell "
                                   "from the centre plane, diffusivity 0 where |x - 1/2| > 0.45, b=4/256, "
                                   f"4 backward-Euler steps, rtol {rtol:g} (separable diffusivity: stencil "
                                   "sweeps with per-axis factors, Chebyshev-preconditioned CG)",
                       "cells": int(mesh.cells), "nnz": mesh.nnz,
                       "pcg_iters_per_step": [r[0] for r in st.iters]},
            "kernels": rl}
    return line


def bench_learned(args):
    """Learned initial guess on 128^3 (unit cube, 2M particles advected by a
    divergence-free flow, b = 4h, 4 backward-Euler steps, rtol 1e-6): train
    on the step pairs of the first snapshots, then coarse-grain the next
    ones with the zero, previous-step and network guesses."""
    import numpy as np
    import torch

    import paper_1409_0001_amd as cgd
    from paper_1409_0001_amd import inputs, warmstart
    n, steps, rtol = 128, 4, args.rtol
    b = 4.0 / n
    mesh = cgd.HexMesh((n, n, n))
    net = cgd.UNet((n, n, n), seed=14090105)
    snaps = inputs.AdvectedSnapshots(n_particles=2_000_000, n_cells_x=n, stride=4, device="cuda")
    t0 = time.perf_counter()
    losses = warmstart.train(net, mesh, snaps, args.train_snapshots, b, steps, lr=args.lr, lr_final=args.lr / 10,
                             log_every=400, log=lambda m: print(m, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"[bench] trained on {args.train_snapshots} snapshots in {t_train:.1f}s", file=sys.stderr, flush=True)
    # parity sample: the first test snapshot against the float64 oracle
    first = snaps.current()
    first_pos, first_vals = first[0].cpu().numpy(), first[1].cpu().numpy()
    t0 = time.perf_counter()
    cases = [(m, pc) for pc in (0, 1) for m in (0, 1, 3)]
    res = warmstart.evaluate(mesh, net, snaps, args.test_snapshots, b, steps, rtol=rtol, cases=cases,
                             keep_fields=1)
    print(f"[bench] evaluated {args.test_snapshots} snapshots x {len(cases)} (guess, solver) cases in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    rel = None
    names = {0: "zero", 1: "previous_step", 3: "network"}
    solvers = {0: "preconditioned_cg", 1: "plain_cg"}
    if not args.no_check:
        from oracle import cgd_oracle as O
        lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
        dep = O.deposit_hex(first_pos, first_vals, lo, hi, (n, n, n))
        ref = O.diffuse_hex_dct(dep["field64"], lo, hi, (n, n, n), b, steps)[0]
        rel = {f"{solvers[pc]}/{names[m]}":
               float(np.linalg.norm(res[(m, pc)]["fields"][0].cpu().numpy() - ref) / np.linalg.norm(ref))
               for m, pc in cases}
    ntest = args.test_snapshots
    modes = {solvers[pc]: {names[m]: {"cg_iters_per_step": [round(v / ntest, 2) for v in res[(m, pc)]["iters"]],
                                      "cg_iters_total_per_field": round(sum(res[(m, pc)]["iters"]) / ntest, 2),
                                      "ms_per_field": round(res[(m, pc)]["ms"] / ntest, 3),
                                      "fallbacks": res[(m, pc)]["fallbacks"]}
                           for m in (0, 1, 3)}
             for pc in (0, 1)}
    t_fwd = []
    x = res[(0, 0)]["fields"][0]
    y = torch.empty_like(x)
    for _ in range(20):
        torch.cuda.synchronize()
        t = time.perf_counter()
        net.forward(x, y)
        torch.cuda.synchronize()
        t_fwd.append(time.perf_counter() - t)
    net_ms = res[(3, 0)]["ms"] / ntest
    line = {"metric": "coarse-grained fields/sec, learned-guess workload 128^3, 2M particles",
            "value": round(1e3 / net_ms, 3), "unit": "fields/s", "n_gpus": 1, "steps": ntest,
            "warmup": 0, "ms_per_step": round(net_ms, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 (solver), bf16 (network)", "data": "synthetic",
            "config": {"workload": "unit cube 128^3 hex, 2M particles advected by a 16-mode divergence-free "
                                   "flow (4 sub-steps between snapshots), b=4h, 4 backward-Euler steps, "
                                   f"polynomial-preconditioned CG rtol {rtol:g} seeded by the network; "
                                   f"network trained on {args.train_snapshots} snapshots "
                                   f"({args.train_snapshots * steps} step pairs), tested on the next {ntest}",
                       "cells": n ** 3, "train_snapshots": args.train_snapshots, "test_snapshots": ntest},
            "guesses": modes,
            "network_forward_ms": round(1e3 * float(np.median(t_fwd)), 3),
            "train": {"seconds": round(t_train, 1), "loss_first": losses[0][1], "loss_last": losses[-1][1],
                      "pairs": args.train_snapshots * steps},
            "rel_l2_first_test_snapshot": rel}
    return line


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the multi-GPU layout of the "
              "path is a design, not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1409_0001_amd as cgd
    from paper_1409_0001_amd import inputs

    one = {"batched": bench_batched, "unstructured": bench_unstructured, "stretched": bench_stretched,
           "learned": bench_learned}
    if args.workload in one:
        print(json.dumps(one[args.workload](args)), flush=True)
        return
    if args.profile_copy:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1.0)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}))
        return

    shape = tuple(int(v) for v in args.shape.split(","))
    t0 = time.perf_counter()
    w = inputs.dense_bed(n_particles=args.particles, shape=shape, n_fields=args.fields)
    print(f"[bench] inputs {w.name} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    pos = torch.from_numpy(w.particles.pos).cuda()
    vals = torch.from_numpy(w.particles.values).cuda()
    mesh = cgd.HexMesh(w.box.shape, w.box.lo, w.box.hi)
    r = run_dense(args, w, mesh, pos, vals, args.scheme, args.steps, args.warmup, check=not args.no_check)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args)
    line = {
        "metric": METRIC, "value": round(r["value"], 3), "unit": "fields/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms_per_field"] * args.fields, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"dense bed {shape[0]}x{shape[1]}x{shape[2]} hex, box 1x1x2, "
                               f"{args.particles} particles, F={args.fields}, b=4h, 4 "
                               f"{'backward-Euler' if args.scheme == 'be' else 'Crank-Nicolson'} "
                               f"steps, CG preconditioned by a Chebyshev polynomial of A (degree 4, 8 or 12 by predicted "
                               f"cost{'; 12 at dtau/h^2 = 1' if args.scheme == 'be' else ''}), rtol {args.rtol:g}",
                   "particles": args.particles, "cells": int(mesh.cells), "fields": args.fields,
                   "cg_iters_per_step": r["iters"]},
        "rel_l2": r["rel_l2"],
        "deposit_bit_exact": r["deposit_bit_exact"],
        "roofline": r["roofline"],
        "cpu_baseline": cpu,
    }
    if not args.no_secondary and args.workload == "dense" and shape == (256, 256, 512) and args.fields == 1:
        line["secondary"] = secondary(args, w, mesh, pos, vals)
    print(json.dumps(line), flush=True)
    if r["deposit_bit_exact"] is False or (r["rel_l2"] is not None and r["rel_l2"] > 1e-5):
        print("[bench] accuracy gate failed", file=sys.stderr, flush=True)
        sys.exit(1)


def run_dense(args, w, mesh, pos, vals, scheme, steps, warmup, check=True):
    """Timed coarse_grain calls of one hex workload: throughput, per-kernel
    roofline from the last timed call, and (check) rel L2 against the oracle
    and the deposit bit for bit."""
    import numpy as np
    import torch

    import paper_1409_0001_amd as cgd
    F = int(vals.shape[0])
    out = torch.empty((F, mesh.cells), dtype=torch.float32, device="cuda")
    kw = dict(rtol=args.rtol, check_every=args.check_every, field=out, scheme=scheme)
    for _ in range(warmup):
        cgd.coarse_grain(mesh, pos, vals, w.bandwidth, w.n_steps, **kw)
    _, st = cgd.coarse_grain(mesh, pos, vals, w.bandwidth, w.n_steps, stats=True, **kw)
    iters = [row[0] for row in st.iters]
    print(f"[bench] {w.name} {scheme}: CG iterations per step {iters}", file=sys.stderr, flush=True)
    # The per-kernel HIP events bracket the launches of the last timed step
    # only: each event pair idles the queue for a few microseconds, which
    # would otherwise be charged to every step's throughput.
    cgd.timing_read(mesh, reset=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(steps):
        if i == steps - 1:
            cgd.timing_enable(mesh, True)
        cgd.coarse_grain(mesh, pos, vals, w.bandwidth, w.n_steps, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    cgd.timing_enable(mesh, False)
    tim = cgd.timing_read(mesh, reset=True)
    ms_per_field = 1e3 * dt / (steps * F)
    value = F * steps / dt
    print(f"[bench] {w.name} {scheme}: {ms_per_field:.2f} ms per field, {value:.2f} fields/s",
          file=sys.stderr, flush=True)
    res = {"value": value, "ms_per_field": ms_per_field, "iters": iters, "roofline": roofline_of(tim, ms_per_field),
           "rel_l2": None, "deposit_bit_exact": None}
    if check:
        from oracle import cgd_oracle as O
        dep = O.deposit_hex(w.particles.pos, w.particles.values, w.box.lo, w.box.hi, w.box.shape)
        ref = O.diffuse_hex_dct(dep["field64"], w.box.lo, w.box.hi, w.box.shape, w.bandwidth, w.n_steps,
                                scheme=scheme)
        got = out.cpu().numpy().astype(np.float64)
        res["rel_l2"] = max(float(np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f])) for f in range(F))
        print(f"[bench] rel L2 vs float64 oracle {res['rel_l2']:.3e}", file=sys.stderr, flush=True)
        # the timed call's deposit, repeated with its accumulators written out,
        # against the oracle's: int64 sums and float32 field bit for bit
        acc = torch.empty((F, mesh.cells), dtype=torch.int64, device="cuda")
        dfield, dst = cgd.deposit(mesh, pos, vals, acc=acc, stats=True)
        res["deposit_bit_exact"] = bool(
            dst.frac_bits == list(dep["S"]) and np.array_equal(acc.cpu().numpy(), dep["acc"])
            and np.array_equal(dfield.cpu().numpy().view(np.uint32), dep["field32"].view(np.uint32)))
        del acc, dfield
        print(f"[bench] deposit bit-exact vs oracle: {res['deposit_bit_exact']}", file=sys.stderr, flush=True)
    return res


def secondary(args, w, mesh, pos, vals):
    """The other workloads, at their full sizes with few timed calls, so that
    the default run reports them too: Crank-Nicolson on the dense bed, the
    literal 256^3 cube, the dense bed turned to 512-cell rows, the batched
    launch, the unstructured and stretched meshes, and a reduced
    learned-guess sample."""
    import torch

    import paper_1409_0001_amd as cgd
    from paper_1409_0001_amd import inputs
    out = {}

    def guarded(name, fn):
        t = time.perf_counter()
        try:
            out[name] = fn()
        except Exception as e:  # a failing secondary workload must not hide the headline
            out[name] = {"error": f"{type(e).__name__}: {e}"}
        print(f"[bench] secondary {name} done in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)

    def cn():
        r = run_dense(args, w, mesh, pos, vals, "cn", 5, 1, check=True)
        return {"workload": "dense bed 256x256x512, 20M particles, 4 Crank-Nicolson steps", "unit": "fields/s",
                "value": round(r["value"], 2), "ms_per_field": round(r["ms_per_field"], 3),
                "cg_iters_per_step": r["iters"], "rel_l2": r["rel_l2"],
                "roofline_dominant": {k: r["roofline"][k] for k in ("kernel", "avg_us", "frac")},
                "whole_solve_frac": r["roofline"]["whole_solve"]["frac"]}

    def cube():
        wc = inputs.dense_bed(n_particles=10_000_000, shape=(256, 256, 256), depth=1.0)
        mc = cgd.HexMesh(wc.box.shape, wc.box.lo, wc.box.hi)
        pc = torch.from_numpy(wc.particles.pos).cuda()
        vc = torch.from_numpy(wc.particles.values).cuda()
        r = run_dense(args, wc, mc, pc, vc, "be", 5, 1, check=True)
        mc.close()
        return {"workload": "dense bed in the unit cube, 256^3 hex (h = 1/256), 10M particles, 4 backward-Euler "
                            "steps", "unit": "fields/s", "value": round(r["value"], 2),
                "ms_per_field": round(r["ms_per_field"], 3), "cg_iters_per_step": r["iters"],
                "rel_l2": r["rel_l2"], "deposit_bit_exact": r["deposit_bit_exact"],
                "roofline_dominant": {k: r["roofline"][k] for k in ("kernel", "avg_us", "frac")},
                "whole_solve_frac": r["roofline"]["whole_solve"]["frac"]}

    def wide():
        # the dense bed turned so that its long axis is x: 512 x 256 x 256 cells
        # in a 2 x 1 x 1 box (h = 1/256), rows wider than one wave covers
        import numpy as np
        wd = inputs.dense_bed(n_particles=20_000_000, shape=(256, 256, 512))
        ww = inputs.Workload("dense-bed-turned-512x256x256", inputs.HexBox((0.0, 0.0, 0.0), (2.0, 1.0, 1.0),
                                                                          (512, 256, 256)),
                             inputs.Particles(np.ascontiguousarray(wd.particles.pos[:, ::-1]), wd.particles.values),
                             wd.bandwidth, wd.n_steps, wd.rtol)
        del wd
        mw = cgd.HexMesh(ww.box.shape, ww.box.lo, ww.box.hi)
        pw = torch.from_numpy(ww.particles.pos).cuda()
        vw = torch.from_numpy(ww.particles.values).cuda()
        r = run_dense(args, ww, mw, pw, vw, "be", 5, 1, check=True)
        mw.close()
        return {"workload": "the dense bed turned so that its long axis is x: 512 x 256 x 256 hex in a 2 x 1 x 1 "
                            "box (h = 1/256), 20M particles, 4 backward-Euler steps (rows of 512 cells: solved with "
                            "x and y exchanged)", "unit": "fields/s", "value": round(r["value"], 2),
                "ms_per_field": round(r["ms_per_field"], 3), "cg_iters_per_step": r["iters"],
                "rel_l2": r["rel_l2"], "deposit_bit_exact": r["deposit_bit_exact"],
                "roofline_dominant": {k: r["roofline"][k] for k in ("kernel", "avg_us", "frac")},
                "whole_solve_frac": r["roofline"]["whole_solve"]["frac"]}

    def sub(fn, **over):
        a = argparse.Namespace(**vars(args))
        for k, v in over.items():
            setattr(a, k, v)
        return fn(a)

    guarded("dense_crank_nicolson", cn)
    guarded("cube_256", cube)
    guarded("wide_512", wide)
    guarded("stretched", lambda: sub(bench_stretched, steps=2, warmup=1, no_check=False))
    guarded("unstructured", lambda: sub(bench_unstructured, steps=3, warmup=1))
    guarded("batched", lambda: sub(bench_batched, steps=2, warmup=1, snapshots=64, no_check=False))
    guarded("learned_reduced", lambda: sub(bench_learned, train_snapshots=100, test_snapshots=16, no_check=False))
    return out


if __name__ == "__main__":
    main()
