"""Benchmark: pair Poisson solves/s and ms per E_xx + D_xx step on one MI355X.

Workload (default): 64 water-like molecules, 256 localized orbitals in a
12.4 A cube on a 128^3 grid, R_pair = 5 A, R_PE = 4 A, R_ME = 5 A, FP64,
CG to 1e-10 relative residual (seeded synthetic orbitals; see synth.py).
One step = exx_solve + exx_energy_potential over every pair of the step.

Prints ONE JSON line.  `roofline` describes the dominant kernel (the
persistent CG kernel): algorithmic bytes per launch (64 B per unknown per
CG iteration in FP64) over its HIP-event duration on the launch stream.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload's pairs on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = {"none": os.path.join(ROOT, "profiles", "cg_traffic.json"),
                   "mg": os.path.join(ROOT, "profiles", "cg_traffic_mg.json")}
KERNEL_SRC = os.path.join(ROOT, "paper_1911_10630_amd", "csrc", "exx_kernels.hip")


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def oracle_orbitals(wl, idx, origins):
    """The orbitals the GPU sees, as full FP64 grids for the oracle: box
    values placed into zero grids (box storage), rounded to FP32 first when
    the workload stores FP32."""
    from paper_1911_10630_amd import synth as S
    if origins is None:
        vals = S.orbitals_np(wl, idx)
    else:
        vals = S.embed_boxes(S.orbitals_np(wl, idx, origins=origins), [origins[k] for k in idx], wl.n_grid)
    if wl.orbital_dtype == "f32":
        vals = vals.astype(np.float32).astype(np.float64)
    return vals


def cpu_baseline(wl, pi, pj, n_sample, threads, seed=0, origins=None):
    """FP64 oracle on a stratified sample of the workload's pairs."""
    from oracle import oracle as O
    from paper_1911_10630_amd import synth as S
    rng = np.random.default_rng(seed)
    self_idx = np.nonzero(pi == pj)[0]
    ns_idx = np.nonzero(pi != pj)[0]
    n_self = max(1, int(round(n_sample * len(self_idx) / len(pi))))
    pick = np.concatenate([rng.choice(self_idx, n_self, replace=False),
                           rng.choice(ns_idx, n_sample - n_self, replace=False)])
    orbs = sorted(set(pi[pick].tolist()) | set(pj[pick].tolist()))
    phis = dict(zip(orbs, oracle_orbitals(wl, orbs, origins)))
    t0 = time.perf_counter()
    res = O.solve_pairs(wl.n_grid, wl.cell, wl.r_pe, wl.r_me, wl.orbitals.centers, phis, pi[pick], pj[pick],
                        tol=wl.cg_rtol, nthreads=threads)
    dt = time.perf_counter() - t0
    return dict(value=len(pick) / dt, unit="pair Poisson solves/s", cores=int(res["threads"]),
                kind="oracle",
                sample=f"{len(pick)} of {len(pi)} pairs ({n_self} self), FP64, {dt:.1f} s wall, "
                       f"mean {float(np.mean(res['iters'])):.0f} CG iterations"), pick, res


def train_model(args, wl, ctx):
    """Trains the learned-guess model before anything is timed, on the same
    configuration with other orbital seeds (the evaluation seed is never
    seen).  Each seed: one solve, then Adam epochs over its pairs."""
    import torch
    from paper_1911_10630_amd import synth as S
    dev = torch.device("cuda:0")
    ctx.model_init(args.coarsen, seed=5)
    t0 = time.perf_counter()
    n_samples, loss, train_s = 0, None, 0.0
    for k in range(args.train_seeds):
        wl_k = S.WORKLOADS[args.workload](seed=9001 + k)
        if args.precision:
            wl_k.precision = args.precision
        n = ctx.pairs(wl_k.orbitals.centers)
        phi = S.orbitals_torch(wl_k, device=dev, origins=ctx.box_origins() if wl_k.box else None)
        ctx.step(phi)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for ep in range(args.train_epochs):
            loss = ctx.model_train(epochs=1, batch=args.train_batch, lr=args.train_lr, seed=1000 * k + ep)
            log(f"[bench]   epoch {ep + 1}/{args.train_epochs}: loss {loss:.4g}, {time.perf_counter() - t1:.1f} s")
        train_s += time.perf_counter() - t1
        n_samples += n
        log(f"[bench] trained on seed {9001 + k}: {n} pairs x {args.train_epochs} epochs, loss {loss:.4g}, "
            f"{time.perf_counter() - t1:.1f} s")
        del phi
    return dict(coarsen=args.coarsen, edge=ctx.model_edge(), train_seeds=args.train_seeds,
                train_pairs=n_samples, epochs=args.train_epochs, batch=args.train_batch, lr=args.train_lr,
                last_loss=loss, train_s=round(train_s, 1), total_s=round(time.perf_counter() - t0, 1))


def md_run(args, wl):
    """Synthetic MD: centres random-walk by N(0, (0.02 A)^2) per component per
    step, orbitals rebuilt, pair list rebuilt, every step solved with the
    requested initial guess.  One JSON line with per-step iterations."""
    import torch
    from paper_1911_10630_amd import exx as X
    from paper_1911_10630_amd import synth as S
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(2718)
    orbs = wl.orbitals
    ctx = X.Exx.from_workload(wl, block_threads=args.block, cg_cols=args.cols, inner_rtol=args.inner_rtol,
                              guess=args.guess)
    learned = train_model(args, wl, ctx) if args.guess == "learned" else None
    stream = torch.cuda.current_stream(dev)
    steps = []
    t_all = 0.0
    n_all = 0
    # orbitals and D first: the pair waves are sized from the memory left
    shape = (orbs.n,) + tuple(reversed(wl.box or wl.n_grid))
    phi = torch.empty(shape, dtype=torch.float64 if wl.orbital_dtype == "f64" else torch.float32, device=dev)
    dxx = torch.empty_like(phi)
    for k in range(args.md_steps):
        wl_k = S.Workload(wl.name, wl.n_grid, wl.cell, orbs, wl.r_pair, wl.r_pe, wl.r_me,
                          orbital_dtype=wl.orbital_dtype, precision=wl.precision, box=wl.box)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = ctx.pairs(orbs.centers)
        t_pairs = time.perf_counter() - t0
        # the step's orbitals (input, not timed): on their boxes when stored so
        S.orbitals_torch(wl_k, device=dev, origins=ctx.box_origins() if wl.box else None, out=phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.solve(phi, stream)
        E = ctx.energy_potential(dxx, stream)
        torch.cuda.synchronize()
        dt = t_pairs + time.perf_counter() - t0
        st = ctx.stats()
        steps.append(dict(step=k, n_pairs=n, seconds=round(dt, 3), iters_mean=round(st["iters_total"] / n, 2),
                          outer_mean=round(st["outer_total"] / n, 2), cg_ms=round(st["cg_ms"], 1),
                          guess_ms=round(st["guess_ms"], 1), E_xx=E))
        log(f"[bench] md step {k}: {n} pairs, {dt:.2f} s, mean iterations {st['iters_total'] / n:.1f}, E {E:.12f}")
        if k > 0:                        # step 0 has no history for any guess
            t_all += dt
            n_all += n
        orbs = S.md_displace(orbs, wl.cell[0], rng)
    line = dict(metric="pair Poisson solves/s (MD steps 1..)", value=round(n_all / t_all, 2) if t_all else None,
                unit="pair Poisson solves/s", n_gpus=1, steps=args.md_steps, warmup=1, higher_is_better=True,
                dtype="f64" if wl.precision == "fp64" else "f32+f64", data="synthetic",
                config=dict(workload=wl.name, guess=args.guess, precision=wl.precision,
                            n_orbitals=wl.orbitals.n, grid=list(wl.n_grid)),
                md=steps)
    if learned:
        line["learned"] = learned
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32_refine"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cols", type=int, default=0, help="CG columns per thread (-1: flat kernel)")
    ap.add_argument("--inner-rtol", type=float, default=1e-5, help="FP32 inner CG tolerance (refinement)")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0: 6 per thread, about 15 s of CPU work)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--md-steps", type=int, default=0,
                    help="run a synthetic MD trajectory of this many steps instead (initial-guess comparison)")
    ap.add_argument("--guess", default="zero", choices=["zero", "previous", "extrap", "learned"])
    ap.add_argument("--precond", default="none", choices=["none", "mg"],
                    help="FP64 CG preconditioner: none (the paper's CG) or a multigrid V-cycle")
    ap.add_argument("--omega-scale", type=float, default=0.0,
                    help="per-pair subdomain classes: Omega_i radius = this x the orbital spread (0: the two "
                         "fixed classes)")
    ap.add_argument("--class-radii", default="3.5,4.5,6.0,7.56",
                    help="per-pair classes: PE radii (bohr), ascending; ME radius = PE + 1.9 bohr")
    ap.add_argument("--graph", action="store_true",
                    help="launch each solve as a captured HIP graph (the CG kernel is then timed with the whole solve)")
    ap.add_argument("--coarsen", type=int, default=2, help="learned guess: grid points per coarse cell edge")
    ap.add_argument("--train-seeds", type=int, default=2, help="learned guess: training configurations")
    ap.add_argument("--train-epochs", type=int, default=2)
    ap.add_argument("--train-batch", type=int, default=8)
    ap.add_argument("--train-lr", type=float, default=1e-3)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="(profiling) also run a plain device copy of this many MiB, 3 times, to calibrate "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU path "
              "(each GPU a share of the pair list, D summed over GPUs) is designed but not implemented",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_10630_amd import exx as X
    from paper_1911_10630_amd import synth as S

    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 3 x {args.copy_probe_mb} MiB device-to-device")
        del src, dst

    wl = S.WORKLOADS[args.workload]()
    if args.precision:
        wl.precision = args.precision
    if args.md_steps:
        return md_run(args, wl)
    dev = torch.device("cuda:0")
    guess = "learned" if args.guess == "learned" else "zero"
    classed = args.omega_scale > 0.0
    ckw = {}
    if classed:
        radii = [float(v) for v in args.class_radii.split(",")]
        ckw = dict(classes=[(r, r + 1.9) for r in radii], omega_scale=args.omega_scale)
    ctx = X.Exx.from_workload(wl, block_threads=args.block, cg_cols=args.cols, inner_rtol=args.inner_rtol,
                              guess=guess, graph=args.graph, precond=args.precond, **ckw)
    learned = train_model(args, wl, ctx) if guess == "learned" else None
    # orbitals and D first: the pair waves are sized from the memory left
    shape = (wl.orbitals.n,) + tuple(reversed(wl.box or wl.n_grid))
    fdt = torch.float64 if wl.orbital_dtype == "f64" else torch.float32
    phi = torch.empty(shape, dtype=fdt, device=dev)
    dxx = torch.empty_like(phi)
    if classed:
        n_pairs = ctx.pairs_spread(wl.orbitals.centers, S.spreads(wl.orbitals))
    else:
        n_pairs = ctx.pairs(wl.orbitals.centers)
    origins = ctx.box_origins() if wl.box else None
    log(f"[bench] workload {wl.name}: generating {wl.orbitals.n} orbitals on {dev}"
        + (f" on {wl.box} boxes" if wl.box else ""))
    S.orbitals_torch(wl, device=dev, origins=origins, out=phi)
    info = ctx.pair_info(results=False)
    stream = torch.cuda.current_stream(dev)
    log(f"[bench] {n_pairs} pairs; warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.solve(phi, stream)
        E = ctx.energy_potential(dxx, stream)
        log(f"[bench] warmup step done, E_xx = {E:.12f}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx.solve(phi, stream)
        E = ctx.energy_potential(dxx, stream)
        log(f"[bench] step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.stats()
    ms_per_step = 1e3 * dt / args.steps
    value = n_pairs * args.steps / dt

    # dominant kernel: persistent CG (one launch per step when one wave holds every pair)
    cg_ms = st["cg_ms"] if st["cg_ms"] > 0 else st["solve_ms"]
    achieved = st["cg_bytes"] / (cg_ms * 1e-3) / 1e9
    traffic = None
    ptr = PROFILE_TRAFFIC[args.precond]
    if os.path.exists(ptr):
        tr = json.load(open(ptr))
        if (tr.get("kernel_hash") == kernel_hash() and tr.get("workload") == wl.name and guess == "zero"
                and not classed):
            for v in tr.get("variants", []):
                if v["variant"] == [st["solve_block"], st["cg_cols"]]:
                    # measured HBM bytes of the same launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
                    # calibrated on a device copy); FP64 iteration counts are deterministic
                    traffic = int(v["bytes_per_launch"])
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic)

    line = dict(metric="pair Poisson solves/s", value=round(value, 2), unit="pair Poisson solves/s",
                n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_per_step, 2),
                higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f64" if wl.precision == "fp64" else "f32+f64",
                data="synthetic",
                config=dict(workload=wl.name, n_orbitals=wl.orbitals.n, n_pairs=n_pairs,
                            grid=list(wl.n_grid), r_pair_bohr=round(wl.r_pair, 4),
                            r_pe_bohr=[round(v, 4) for v in wl.r_pe], r_me_bohr=[round(v, 4) for v in wl.r_me],
                            n_pe=st["n_pe"], n_me=st["n_me"], cg_rtol=wl.cg_rtol, precision=wl.precision,
                            parallelism="1 GPU, persistent work-group per pair"),
                roofline=roofline,
                detail=dict(E_xx=E, iters_mean=st["iters_total"] / n_pairs, iters_min=st["iters_min"],
                            iters_max=st["iters_max"], relres_max=st["relres_max"],
                            solve_ms=round(st["solve_ms"], 2), prep_ms=round(st["prep_ms"], 2),
                            cg_ms=round(st["cg_ms"], 2), dxx_ms=round(st["dxx_ms"], 2),
                            energy_ms=round(st["energy_ms"], 3), cg_bytes=st["cg_bytes"],
                            dxx_gbs=round(st["dxx_bytes"] / (st["dxx_ms"] * 1e-3) / 1e9, 1) if st["dxx_ms"] > 0 else None,
                            grid=st["solve_grid"], block=st["solve_block"], waves=st["n_waves"],
                            autotuned_variants=st["tuned"], tune_ms=round(st["tune_ms"], 1),
                            graph_launches=st["graph_launches"],
                            cg_cols=st["cg_cols"], cg_bands=st["cg_bands"], outer_total=st["outer_total"],
                            inner_rtol=args.inner_rtol if wl.precision != "fp64" else None,
                            kernel_hash=kernel_hash()))
    if args.precond != "none":
        line["config"]["precond"] = args.precond
    if classed:
        nc = st["n_classes"]
        # the subdomains are the classes', not the workload's fixed pair
        line["config"].update(r_pe_bohr=[round(c[0], 4) for c in ckw["classes"]],
                              r_me_bohr=[round(c[1], 4) for c in ckw["classes"]],
                              n_pe=st["class_n_pe"][:nc], n_me=st["class_n_me"][:nc])
        line["config"]["pair_classes"] = dict(omega_scale=args.omega_scale,
                                              pairs=st["class_pairs"][:nc], capped=st["class_capped"])
    if learned:
        line["config"]["guess"] = "learned"
        learned["guess_ms"] = round(st["guess_ms"], 2)
        line["learned"] = learned

    if not args.no_cpu_baseline and not classed:       # the oracle leg runs the two fixed classes
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        n_sample = args.cpu_sample or 6 * threads
        n_sample = min(n_sample, n_pairs)
        log(f"[bench] CPU oracle baseline: {n_sample} pairs on {threads} threads")
        cb, pick, res = cpu_baseline(wl, info["i"], info["j"], n_sample, threads, origins=origins)
        line["cpu_baseline"] = cb
        pinfo = ctx.pair_info()
        rel = np.abs(pinfo["e"][pick] - res["e"]) / np.abs(res["e"])
        line["detail"]["sample_pair_energy_max_rel_vs_oracle"] = float(rel.max())
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
