"""Benchmark: pair Poisson solves/s and ms per E_xx + D_xx step on one MI355X.

Default workload: 512 water-like molecules (2048 localized orbitals) in a
24.8 A cube on a 256^3 grid, orbitals stored FP32 on 160^3 local boxes,
R_pair = 5 A (79,753 pairs), each pair on the smallest of four subdomain
classes that holds its domain Omega_ij (the uneven truncated subdomains of
the paper's outlook), CG preconditioned by a multigrid V-cycle in FP64 to
||b - A x|| <= 1e-10 ||b|| (seeded synthetic orbitals; see synth.py).
One step = exx_solve + exx_energy_potential over every pair, replayed as a
captured HIP graph.

Prints ONE JSON line.  `roofline` describes the dominant kernel (the
persistent CG kernel): its algorithmic bytes per step over its span on the
device wall clock (first work-group start to last work-group end, summed
over the launch waves; the same span rocprofv3 reports).  `cpu_baseline`
times the FP64 CPU oracle on a bounded sample of the same workload's pairs.
After the timed steps, untimed extras on the same workload:
`two_class_reference` (one step with the two fixed subdomain classes, the
paper's self / non-self pair) and `learned_vs_plain` (the learned initial
guess against the zero guess, plain and multigrid-preconditioned CG, on a
subsystem of the same water, the model trained on a subsystem of another
seed).
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair Poisson solves/s and ms per E_xx+D_xx step; learned vs plain CG @1e-7 rel E_xx"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "cg_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1911_10630_amd", "csrc", "exx_kernels.hip")
CLASS_RADII = "3.5,4.5,6.0,7.56"     # per-pair classes: PE radii (bohr); ME = PE + 1.9 bohr


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def host_cpu() -> str:
    """CPU model and logical core count of the host running the oracle."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical cores visible"


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


def nearest_orbitals(wl, n_keep, point=None):
    """Indices of the n_keep orbitals nearest `point` (the cell centre by
    default), minimum image."""
    L = np.asarray(wl.cell, float)
    p = L / 2 if point is None else np.asarray(point, float)
    d = wl.orbitals.centers - p
    d -= L * np.round(d / L)
    return np.sort(np.argsort(np.sum(d * d, axis=1), kind="stable")[:n_keep])


def subsystem(wl, keep, name_suffix):
    """The workload restricted to the orbitals `keep` (same cell, grid,
    radii, storage and shapes)."""
    from paper_1911_10630_amd import synth as S
    o = wl.orbitals
    sub = S.OrbitalSet(centers=o.centers[keep], kind=o.kind[keep], alpha=o.alpha[keep], u=o.u[keep], a=o.a[keep],
                       B=o.B[keep])
    return dataclasses.replace(wl, orbitals=sub, name=wl.name + name_suffix)


def class_list(args):
    radii = [float(v) for v in args.class_radii.split(",")]
    return [(r, r + 1.9) for r in radii]


def cpu_baseline_fixed(wl, pi, pj, n_sample, threads, seed=0, origins=None):
    """FP64 oracle on a stratified sample of the workload's pairs (two fixed
    classes)."""
    from oracle import oracle as O
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


def cpu_baseline_classed(wl, classes, omega, spreads, pi, pj, n_cluster, n_sample, threads, seed=0,
                         origins=None):
    """FP64 oracle on a bounded sample of a per-pair-class workload: pairs
    among the n_cluster orbitals nearest the cell centre (so the sample
    needs few orbital grids), at most n_sample of them, each on the class the
    oracle assigns it (pair_domain_radius against the class radii)."""
    from oracle import oracle as O
    keep = set(nearest_orbitals(wl, n_cluster).tolist())
    cand = np.nonzero([(i in keep and j in keep) for i, j in zip(pi.tolist(), pj.tolist())])[0]
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(cand, min(n_sample, len(cand)), replace=False))
    C = wl.orbitals.centers
    r_pe = [c[0] for c in classes]
    cls = np.zeros(len(pick), np.int32)
    for t, p in enumerate(pick):
        i, j = int(pi[p]), int(pj[p])
        g = O.pair_origin(C[i], C[j], wl.cell, wl.n_grid)
        r = O.pair_domain_radius(C[i], C[j], omega * spreads[i], omega * spreads[j], g, wl.cell, wl.n_grid, i == j)
        k = 0
        while k < len(r_pe) and r_pe[k] < r:
            k += 1
        cls[t] = min(k, len(r_pe) - 1)
    orbs = sorted(set(pi[pick].tolist()) | set(pj[pick].tolist()))
    phis = dict(zip(orbs, oracle_orbitals(wl, orbs, origins)))
    t0 = time.perf_counter()
    res = O.solve_pairs_classed(wl.n_grid, wl.cell, classes, C, phis, pi[pick], pj[pick], cls, tol=wl.cg_rtol,
                                nthreads=threads)
    dt = time.perf_counter() - t0
    mix = np.bincount(cls, minlength=len(classes)).tolist()
    return dict(value=len(pick) / dt, unit="pair Poisson solves/s", cores=int(res["threads"]), kind="oracle",
                sample=f"{len(pick)} of {len(pi)} pairs, those among the {n_cluster} orbitals nearest the cell "
                       f"centre (per class {mix}), FP64 plain CG, {dt:.1f} s wall, mean "
                       f"{float(np.mean(res['iters'])):.0f} CG iterations"), pick, res


def step_timed(ctx, phi, dxx, stream, n):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        ctx.solve(phi, stream)
        E = ctx.energy_potential(dxx, stream)
    torch.cuda.synchronize()
    return E, (time.perf_counter() - t0) / max(n, 1)


def two_class_reference(wl, phi, dxx, origins, E_head, args):
    """One step of the same workload with the two fixed subdomain classes
    (self pairs R_PE = 4 A, the others 3.33 A), eager launches."""
    import torch
    from paper_1911_10630_amd import exx as X
    ctx = X.Exx.from_workload(wl, precond=args.precond, precision="fp64")
    n = ctx.pairs(wl.orbitals.centers)
    assert np.array_equal(ctx.box_origins(), origins) if origins is not None else True
    stream = torch.cuda.current_stream(phi.device)
    E, dt = step_timed(ctx, phi, dxx, stream, 1)
    st = ctx.stats()
    ctx.close()
    return dict(subdomains="two fixed classes: self pairs R_PE 4 A, others 10/3 A (R_ME + 1 A)",
                n_pairs=n, ms_per_step=round(1e3 * dt, 1), solves_per_s=round(n / dt, 1), E_xx=E,
                iters_mean=round(st["iters_total"] / n, 2), cg_clock_ms=round(st["cg_clock_ms"], 1),
                rel_diff_E_vs_headline=abs(E - E_head) / abs(E))


def learned_full(wl, phi, dxx, spreads, classes, head, args):
    """The headline configuration (every pair, per-pair classes, multigrid
    PCG) with the learned initial guess, in FP64 and in FP32 with FP64
    residual replacement (the latter beside its zero-guess run): one warm-up
    step (graph build) and one timed step each.  The model is trained on the
    same-size subsystem of the workload drawn with another seed, on the same
    classes."""
    import torch
    from paper_1911_10630_amd import exx as X
    from paper_1911_10630_amd import synth as S
    dev = phi.device
    stream = torch.cuda.current_stream(dev)
    ckw = dict(classes=classes, omega_scale=args.omega_scale, precond="mg")
    t0 = time.perf_counter()
    tw = S.WORKLOADS[args.workload](seed=9001)
    tw = subsystem(tw, nearest_orbitals(tw, args.lvp_orbitals), "-train")
    tw.precision = "fp64"
    tr = X.Exx.from_workload(tw, guess="learned", **ckw)
    n_tr = tr.pairs_spread(tw.orbitals.centers, S.spreads(tw.orbitals))
    shape = (tw.orbitals.n,) + tuple(reversed(tw.box or tw.n_grid))
    phi_t = torch.empty(shape, dtype=phi.dtype, device=dev)
    S.orbitals_torch(tw, device=dev, origins=tr.box_origins() if tw.box else None, out=phi_t)
    tr.model_init(args.coarsen, seed=5)
    tr.step(phi_t)
    loss0 = tr.model_loss(batch=args.train_batch)
    loss = None
    for ep in range(args.train_epochs):
        loss = tr.model_train(epochs=1, batch=args.train_batch, lr=args.train_lr, seed=ep)
    blob = tr.model_save()
    train_s = time.perf_counter() - t0
    tr.close()
    del phi_t
    log(f"[bench] learned guess (classes): trained on {n_tr} pairs x {args.train_epochs} epochs in {train_s:.1f} s, "
        f"loss {loss0:.3g} -> {loss:.3g}")
    rows = {"mg": dict(ms_per_step=head["ms_per_step"], solves_per_s=head["solves_per_s"],
                       iters_mean=head["iters_mean"], cg_clock_ms=head["cg_clock_ms"], E_xx=head["E_xx"],
                       rel_diff_E_vs_mg=0.0, note="the timed headline steps")}
    variant = {"mg": tuple(head["variant"])}   # the zero-guess run's CG variant, forced on its learned twin
    for name, kw in (("mg+learned", dict(guess="learned")), ("mg_fp32", dict(precision="fp32_refine")),
                     ("mg_fp32+learned", dict(guess="learned", precision="fp32_refine"))):
        base = name.split("+")[0]
        if name != base and base in variant:
            kw = dict(kw, block_threads=variant[base][0], cg_cols=variant[base][1])
        w = dataclasses.replace(wl)
        w.precision = kw.pop("precision", "fp64")
        ctx = X.Exx.from_workload(w, graph=True, **ckw, **kw)
        n = ctx.pairs_spread(wl.orbitals.centers, spreads)
        if "learned" in name:
            ctx.load_model(blob)
        step_timed(ctx, phi, dxx, stream, 1)                     # warm-up: graph build
        E, dt = step_timed(ctx, phi, dxx, stream, 1)
        st = ctx.stats()
        if name == base:
            variant[name] = (st["solve_block"], st["cg_cols"])
        rows[name] = dict(ms_per_step=round(1e3 * dt, 2), solves_per_s=round(n / dt, 1),
                          iters_mean=round(st["iters_total"] / n, 2), guess_ms=round(st["guess_ms"], 2),
                          cg_clock_ms=round(st["cg_clock_ms"], 2), E_xx=E,
                          rel_diff_E_vs_mg=abs(E - head["E_xx"]) / abs(head["E_xx"]),
                          variant=[st["solve_block"], st["cg_cols"]])
        ctx.close()
        log(f"[bench] {name}: {1e3 * dt:.0f} ms, {rows[name]['iters_mean']} iterations")
    base = rows["mg"]["ms_per_step"]
    for r in rows.values():
        r["speedup_vs_mg"] = round(base / r["ms_per_step"], 3)
    return dict(config="the headline workload and classes, multigrid PCG to 1e-10, HIP graph",
                model=dict(coarsen=args.coarsen, train_pairs=n_tr, epochs=args.train_epochs, train_s=round(train_s, 1),
                           loss_before=loss0, loss_after=loss,
                           train_set=f"the {args.lvp_orbitals} orbitals nearest the centre, orbital seed 9001, "
                                     "same classes"),
                accuracy_point="every mode stops on ||b - A x|| <= 1e-10 ||b||; |dE_xx|/|E_xx| against the "
                               "headline is listed per mode (the bar is 1e-7)",
                modes=rows)


def learned_vs_plain(wl, args):
    """The learned initial guess against the zero guess, for plain and
    multigrid-preconditioned FP64 CG, on the n_sub orbitals nearest the cell
    centre (all their pairs, two fixed classes); the model is trained on the
    same-size subsystem of the workload drawn with another seed."""
    import torch
    from paper_1911_10630_amd import exx as X
    from paper_1911_10630_amd import synth as S
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    train_wl = subsystem(S.WORKLOADS[args.workload](seed=9001), nearest_orbitals(S.WORKLOADS[args.workload](seed=9001),
                                                                                 args.lvp_orbitals), "-train")
    eval_wl = subsystem(wl, nearest_orbitals(wl, args.lvp_orbitals), "-eval")
    for w in (train_wl, eval_wl):
        w.precision = "fp64"

    def make(w, **kw):
        ctx = X.Exx.from_workload(w, **kw)
        n = ctx.pairs(w.orbitals.centers)
        shape = (w.orbitals.n,) + tuple(reversed(w.box or w.n_grid))
        phi = torch.empty(shape, dtype=torch.float32 if w.orbital_dtype == "f32" else torch.float64, device=dev)
        S.orbitals_torch(w, device=dev, origins=ctx.box_origins() if w.box else None, out=phi)
        return ctx, n, phi

    t0 = time.perf_counter()
    tr, n_tr, phi_tr = make(train_wl, guess="learned")
    tr.model_init(args.coarsen, seed=5)
    tr.step(phi_tr)
    loss0 = tr.model_loss(batch=args.train_batch)
    loss = None
    for ep in range(args.train_epochs):
        loss = tr.model_train(epochs=1, batch=args.train_batch, lr=args.train_lr, seed=ep)
    blob = tr.model_save()
    train_s = time.perf_counter() - t0
    tr.close()
    del phi_tr
    log(f"[bench] learned guess: trained on {n_tr} pairs x {args.train_epochs} epochs in {train_s:.1f} s, "
        f"loss {loss0:.3g} -> {loss:.3g}")
    rows = {}
    E_plain = None
    variant = {}   # the zero-guess run's CG variant, forced on its learned twin
    for name, kw in (("plain", dict()), ("plain+learned", dict(guess="learned")), ("mg", dict(precond="mg")),
                     ("mg+learned", dict(precond="mg", guess="learned"))):
        base = name.split("+")[0]
        if name != base and base in variant:
            kw = dict(kw, block_threads=variant[base][0], cg_cols=variant[base][1])
        ctx, n, phi = make(eval_wl, **kw)
        if "learned" in name:
            ctx.load_model(blob)
        dxx = torch.empty_like(phi)
        step_timed(ctx, phi, dxx, stream, 1)                     # warm-up (first graph-free launch)
        E, dt = step_timed(ctx, phi, dxx, stream, 1)
        st = ctx.stats()
        if name == base:
            variant[name] = (st["solve_block"], st["cg_cols"])
        if E_plain is None:
            E_plain = E
        rows[name] = dict(ms_per_step=round(1e3 * dt, 2), solves_per_s=round(n / dt, 1),
                          iters_mean=round(st["iters_total"] / n, 2), guess_ms=round(st["guess_ms"], 2),
                          cg_clock_ms=round(st["cg_clock_ms"], 2), E_xx=E,
                          rel_diff_E_vs_plain=abs(E - E_plain) / abs(E_plain),
                          variant=[st["solve_block"], st["cg_cols"]])
        ctx.close()
        del phi, dxx
    base = rows["plain"]["ms_per_step"]
    for r in rows.values():
        r["speedup_vs_plain"] = round(base / r["ms_per_step"], 3)
    return dict(subsystem=f"the {args.lvp_orbitals} orbitals nearest the cell centre, all {n} of their pairs, two "
                          f"fixed classes, FP64, CG to 1e-10",
                model=dict(coarsen=args.coarsen, train_pairs=n_tr, epochs=args.train_epochs, train_s=round(train_s, 1),
                           loss_before=loss0, loss_after=loss, train_set="same-size subsystem, orbital seed 9001"),
                accuracy_point="every mode stops on ||b - A x|| <= 1e-10 ||b||; |dE_xx|/|E_xx| against plain "
                               "CG is listed per mode (the bar is 1e-7)",
                modes=rows)


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
                              guess=args.guess, precond=args.precond)
    learned = None
    if args.guess == "learned":
        ctx.model_init(args.coarsen, seed=5)
        for k in range(args.train_seeds):
            wl_k = S.WORKLOADS[args.workload](seed=9001 + k)
            wl_k.precision = wl.precision
            ctx.pairs(wl_k.orbitals.centers)
            phi = S.orbitals_torch(wl_k, device=dev, origins=ctx.box_origins() if wl_k.box else None)
            ctx.step(phi)
            for ep in range(args.train_epochs):
                loss = ctx.model_train(epochs=1, batch=args.train_batch, lr=args.train_lr, seed=1000 * k + ep)
            log(f"[bench] trained on seed {9001 + k}, loss {loss:.4g}")
            del phi
        learned = dict(coarsen=args.coarsen, train_seeds=args.train_seeds, epochs=args.train_epochs)
    stream = torch.cuda.current_stream(dev)
    steps = []
    t_all = 0.0
    n_all = 0
    shape = (orbs.n,) + tuple(reversed(wl.box or wl.n_grid))
    phi = torch.empty(shape, dtype=torch.float64 if wl.orbital_dtype == "f64" else torch.float32, device=dev)
    dxx = torch.empty_like(phi)
    for k in range(args.md_steps):
        wl_k = dataclasses.replace(wl, orbitals=orbs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = ctx.pairs(orbs.centers)
        t_pairs = time.perf_counter() - t0
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
        if k > 0:
            t_all += dt
            n_all += n
        orbs = S.md_displace(orbs, wl.cell[0], rng)
    line = dict(metric="pair Poisson solves/s (MD steps 1..)", value=round(n_all / t_all, 2) if t_all else None,
                unit="pair Poisson solves/s", n_gpus=1, steps=args.md_steps, warmup=1, higher_is_better=True,
                dtype="f64" if wl.precision == "fp64" else "f32+f64", data="synthetic",
                config=dict(workload=wl.name, guess=args.guess, precision=wl.precision, precond=args.precond,
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
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_refine"])
    ap.add_argument("--precond", default="mg", choices=["none", "mg"],
                    help="CG preconditioner: mg (multigrid V-cycle, default) or none (the paper's plain CG)")
    ap.add_argument("--omega-scale", type=float, default=5.0,
                    help="per-pair subdomain classes: Omega_i radius = this x the orbital spread (0: the two "
                         "fixed classes)")
    ap.add_argument("--class-radii", default=CLASS_RADII,
                    help="per-pair classes: PE radii (bohr), ascending; ME radius = PE + 1.9 bohr")
    ap.add_argument("--no-graph", action="store_true", help="launch each solve eagerly instead of as a HIP graph")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cols", type=int, default=0, help="CG columns per thread (-1: flat kernel)")
    ap.add_argument("--inner-rtol", type=float, default=1e-5, help="FP32 inner CG tolerance (refinement)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle sample size (0: 6 pairs per thread, about 15 s of CPU work)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the untimed two-class reference step and the learned-vs-plain comparison")
    ap.add_argument("--lvp-orbitals", type=int, default=96, help="learned vs plain: subsystem size (orbitals)")
    ap.add_argument("--md-steps", type=int, default=0,
                    help="run a synthetic MD trajectory of this many steps instead (initial-guess comparison)")
    ap.add_argument("--guess", default="zero", choices=["zero", "previous", "extrap", "learned"])
    ap.add_argument("--coarsen", type=int, default=4, help="learned guess: grid points per coarse cell edge")
    ap.add_argument("--train-seeds", type=int, default=1, help="learned guess (MD mode): training configurations")
    ap.add_argument("--train-epochs", type=int, default=12)
    ap.add_argument("--train-batch", type=int, default=8)
    ap.add_argument("--train-lr", type=float, default=1e-3)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="(profiling) also run a plain device copy of this many MiB, 3 times, to calibrate "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--stream-probe", action="store_true",
                    help="print the device's measured streaming rates (read / copy / triad / CG mix, GB/s) as one "
                         "JSON line and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU path "
              "(each GPU a share of the pair list, D summed over GPUs) is designed but not implemented",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_10630_amd import exx as X
    from paper_1911_10630_amd import synth as S

    if args.stream_probe:
        print(json.dumps(X.stream_rates(0)), flush=True)
        return

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
    wl.precision = args.precision
    if args.md_steps:
        return md_run(args, wl)
    dev = torch.device("cuda:0")
    classed = args.omega_scale > 0.0
    classes = class_list(args) if classed else None
    ckw = dict(classes=classes, omega_scale=args.omega_scale) if classed else {}
    graph = not args.no_graph
    ctx = X.Exx.from_workload(wl, block_threads=args.block, cg_cols=args.cols, inner_rtol=args.inner_rtol,
                              graph=graph, precond=args.precond, **ckw)
    # orbitals and D first: the pair waves are sized from the memory left
    shape = (wl.orbitals.n,) + tuple(reversed(wl.box or wl.n_grid))
    fdt = torch.float64 if wl.orbital_dtype == "f64" else torch.float32
    phi = torch.empty(shape, dtype=fdt, device=dev)
    dxx = torch.empty_like(phi)
    spreads = S.spreads(wl.orbitals)
    t0 = time.perf_counter()
    n_pairs = ctx.pairs_spread(wl.orbitals.centers, spreads) if classed else ctx.pairs(wl.orbitals.centers)
    t_pairs = time.perf_counter() - t0
    origins = ctx.box_origins() if wl.box else None
    log(f"[bench] workload {wl.name}: {n_pairs} pairs ({t_pairs:.2f} s); generating {wl.orbitals.n} orbitals"
        + (f" on {wl.box} boxes" if wl.box else ""))
    S.orbitals_torch(wl, device=dev, origins=origins, out=phi)
    info = ctx.pair_info(results=False)
    stream = torch.cuda.current_stream(dev)
    log(f"[bench] warmup {args.warmup}")
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
    pinfo = ctx.pair_info()
    ms_per_step = 1e3 * dt / args.steps
    value = n_pairs * args.steps / dt

    # dominant kernel: the persistent CG kernel, its span on the device clock
    # (per launch wave, summed), which graph replays keep
    cg_ms = st["cg_clock_ms"] if st["cg_clock_ms"] > 0 else (st["cg_ms"] if st["cg_ms"] > 0 else st["solve_ms"])
    achieved = st["cg_bytes"] / (cg_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        tr = json.load(open(PROFILE_TRAFFIC))
        for entry in tr.get("entries", []):
            if (entry.get("kernel_hash") == kernel_hash() and entry.get("workload") == wl.name
                    and entry.get("precond") == args.precond and entry.get("omega_scale") == args.omega_scale
                    and entry.get("precision", "fp64") == wl.precision
                    and entry.get("algorithmic_bytes_per_step") == st["cg_bytes"]
                    and entry.get("variant") == [st["solve_block"], st["cg_cols"]]):
                # measured HBM bytes of the same launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
                # calibrated on a device copy); FP64 iteration counts are deterministic
                traffic = int(entry["bytes_per_step"])
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic)
    method = ("CG preconditioned by a symmetric multigrid V-cycle" if args.precond == "mg"
              else "plain CG (the paper's Step IV)")
    method += ", FP64" if wl.precision == "fp64" else ", FP32 with FP64 residual replacement"
    config = dict(workload=wl.name, method=method,
                  orbital_storage=(f"{'FP32' if wl.orbital_dtype == 'f32' else 'FP64'} on "
                                   f"{wl.box[0]}^3 local boxes" if wl.box else
                                   f"{'FP32' if wl.orbital_dtype == 'f32' else 'FP64'} full grids"),
                  n_orbitals=wl.orbitals.n, n_pairs=n_pairs, grid=list(wl.n_grid),
                  r_pair_bohr=round(wl.r_pair, 4), cg_rtol=wl.cg_rtol, precision=wl.precision,
                  precond=args.precond, guess="zero", launch="HIP graph" if graph else "eager",
                  parallelism="1 GPU, persistent work-group per pair, pairs in waves sized to HBM")
    if classed:
        nc = st["n_classes"]
        config["subdomains"] = dict(kind="per-pair classes: the smallest whose PE sphere holds Omega_ij",
                                    omega_scale=args.omega_scale, r_pe_bohr=[round(c[0], 4) for c in classes],
                                    r_me_bohr=[round(c[1], 4) for c in classes], n_pe=st["class_n_pe"][:nc],
                                    pairs=st["class_pairs"][:nc], capped=st["class_capped"])
    else:
        config["subdomains"] = dict(kind="two fixed classes (self / other)",
                                    r_pe_bohr=[round(v, 4) for v in wl.r_pe], r_me_bohr=[round(v, 4) for v in wl.r_me],
                                    n_pe=st["n_pe"])
    line = dict(metric=METRIC, value=round(value, 2), unit="pair Poisson solves/s",
                n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_per_step, 2),
                higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f64" if wl.precision == "fp64" else "f32+f64", data="synthetic",
                config=config, roofline=roofline,
                detail=dict(E_xx=E, iters_mean=st["iters_total"] / n_pairs, iters_min=st["iters_min"],
                            iters_max=st["iters_max"], relres_max=st["relres_max"], n_not_converged=st["n_not_converged"],
                            pairs_build_s=round(t_pairs, 3), solve_ms=round(st["solve_ms"], 2),
                            cg_clock_ms=round(st["cg_clock_ms"], 2), cg_event_ms=round(st["cg_ms"], 2),
                            dxx_in_energy_potential_ms=round(st["dxx_ms"], 2), energy_ms=round(st["energy_ms"], 3),
                            dxx_bytes=st["dxx_bytes"],
                            # algorithmic rate of the D kernel; in waves D is summed inside the solve
                            # and the timing above covers only the final rounding
                            dxx_gbs=round(st["dxx_bytes"] / st["dxx_ms"] / 1e6, 1)
                            if st["n_waves"] == 1 and st["dxx_ms"] > 0 else None,
                            cg_bytes=st["cg_bytes"], grid=st["solve_grid"], block=st["solve_block"],
                            cg_cols=st["cg_cols"], cg_bands=st["cg_bands"], waves=st["n_waves"],
                            autotuned_variants=st["tuned"], tune_ms=round(st["tune_ms"], 1),
                            graph_builds=st["graph_builds"], graph_launches=st["graph_launches"],
                            outer_total=st["outer_total"], kernel_hash=kernel_hash(),
                            bytes_per_unknown_iteration="72 (multigrid, FP64 r and x) + the V-cycle's"
                            if args.precond == "mg" else "64 (plain FP64 CG)"))
    ctx.close()

    if not args.no_extras:
        t1 = time.perf_counter()
        if classed:
            log("[bench] two-class reference step (untimed)")
            line["two_class_reference"] = two_class_reference(wl, phi, dxx, origins, E, args)
            if args.precond == "mg" and wl.precision == "fp64":
                log("[bench] learned guess on the headline configuration (untimed)")
                head = dict(ms_per_step=round(ms_per_step, 2), solves_per_s=round(value, 1),
                            iters_mean=round(st["iters_total"] / n_pairs, 2), cg_clock_ms=round(st["cg_clock_ms"], 2),
                            E_xx=E, variant=[st["solve_block"], st["cg_cols"]])
                line["learned_full"] = learned_full(wl, phi, dxx, spreads, classes, head, args)
        log("[bench] learned vs plain on a subsystem (untimed)")
        del phi, dxx
        torch.cuda.empty_cache()
        line["learned_vs_plain"] = learned_vs_plain(wl, args)
        line["detail"]["extras_s"] = round(time.perf_counter() - t1, 1)

    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        n_sample = min(args.cpu_sample or 6 * threads, n_pairs)
        log(f"[bench] CPU oracle baseline: up to {n_sample} pairs on {threads} threads")
        if classed:
            cb, pick, res = cpu_baseline_classed(wl, classes, args.omega_scale, spreads, info["i"], info["j"], 24,
                                                 n_sample, threads, origins=origins)
        else:
            cb, pick, res = cpu_baseline_fixed(wl, info["i"], info["j"], n_sample, threads, origins=origins)
        line["cpu_baseline"] = cb
        line["detail"]["host_cpu"] = host_cpu()
        rel = np.abs(pinfo["e"][pick] - res["e"]) / np.abs(res["e"])
        line["detail"]["sample_pair_energy_max_rel_vs_oracle"] = float(rel.max())
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
