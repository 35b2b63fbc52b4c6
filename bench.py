#!/usr/bin/env python3
"""Benchmark of one linearized pseudo-4D DFN Jacobian solve on one MI355X.

Workload: the homogeneous cube cell, 64 x 64 x 192 nodes (anode / separator /
cathode 80 / 32 / 80 layers), 20 radial points per particle, N = 15,335,424
unknowns; FP64 restarted FGMRES(30) with the particle-Schur block
preconditioner to a true relative residual of 1e-8.  One step = preconditioner
setup + solve (what each Newton step of a simulation has to pay), with the
inputs already resident in device memory.

Prints one JSON line: the metric is DOF*iter/s = N * iterations / step time.
Extra fields report the FP32-preconditioned solve on the same input and on the
lognormal-conductivity cube, the block-Jacobi and block Gauss-Seidel
preconditioners (all 24 orderings of the latter), the Krylov iteration over
the Schur complement of the particle blocks, the adjoint solve with gradients,
the batched solve of 64 uneven cells, per-kernel times and bandwidths measured
with HIP events inside the timed region, and the CPU oracle timed on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_cube64x64x192_hbm_traffic.txt")
# the timed headline steps time one event pair in SAMPLE_EVERY of the
# dominant kernel class (a pair of the level-0 smoother spans its launches
# on one side of a V-cycle's coarse correction; odd, so both sides are
# sampled)
SAMPLE_EVERY = 13


def measured_traffic(kernel_class):
    """HBM bytes per launch of a kernel class from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or
    None when there is none or the kernel's source changed since."""
    import hashlib
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        f = ln.split()
        if len(f) < 2 or f[0] != "traffic" or f[1] != kernel_class:
            continue
        kv = dict(x.split("=", 1) for x in f[2:] if "=" in x)
        try:
            src = open(os.path.join(ROOT, kv["source"]), "rb").read()
        except (OSError, KeyError):
            return None
        if hashlib.sha256(src).hexdigest() != kv.get("sha256"):
            return None
        return float(kv["bytes_per_launch"])
    return None


FIELD_NAMES = ("phi_s", "phi_e", "c_e", "c_s")


def cpu_model():
    """CPU model name of the host (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def field_errors(p, x, ref):
    """Relative error of x against ref overall and per field block."""
    o = list(p.offsets)
    names = ("phi_s", "phi_e", "c_e", "c_s_anode", "c_s_cathode")
    out = {"all": float(np.linalg.norm(x - ref) / np.linalg.norm(ref))}
    for nm, a, b in zip(names, o[:-1], o[1:]):
        nb = np.linalg.norm(ref[a:b])
        out[nm] = float(np.linalg.norm(x[a:b] - ref[a:b]) / (nb if nb > 0 else 1.0))
    return out


def bgs_sweep(s, b, base):
    """Block Gauss-Seidel (eq. PGS) in each of the 24 field orderings (the
    ordering study of Sec. 5): iterations and time of one step each (setup +
    solve, after one untimed step), two-pass Gram-Schmidt."""
    import itertools
    from paper_2602_07225_amd import _lib as L
    rows = []
    for fields in itertools.permutations(range(4)):
        order = sum(f << (2 * q) for q, f in enumerate(fields))
        opts = dict(base, pc=L.P4D_PC_BGS, bgs_order=order, cgs2=1)
        try:
            _, info, it, t, _ = timed_steps(s, b, opts, 1, 1)
            rows.append({"ordering": [FIELD_NAMES[f] for f in fields], "iters": it,
                         "ms_per_step": round(1e3 * t, 3)})
        except RuntimeError as ex:
            rows.append({"ordering": [FIELD_NAMES[f] for f in fields], "error": str(ex)})
    ok = [r for r in rows if "iters" in r]
    ok.sort(key=lambda r: (r["iters"], r["ms_per_step"]))
    paper = [r for r in rows if r["ordering"] == ["phi_e", "c_s", "phi_s", "c_e"]]
    return {"best": ok[0] if ok else None, "worst": ok[-1] if ok else None,
            "paper_ordering": paper[0] if paper else None,
            "iters_spread": (ok[-1]["iters"] / ok[0]["iters"] - 1.0) if ok else None,
            "all": rows}


def event_pair_us(n=200):
    """Mean elapsed time of an event pair with nothing between them, on the
    stream the library's launches use (the current torch stream)."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for e0, e1 in evs:
        e0.record()
        e1.record()
    torch.cuda.synchronize()
    return 1e3 * sum(e0.elapsed_time(e1) for e0, e1 in evs) / n


def byte_split(p64, p32, steps):
    """Per timed kernel class (coarse multigrid levels are not a class): the
    algorithmic bytes and time per step with the FP64 and the FP32
    preconditioner, and the class's share of the FP64 step's timed bytes
    (the part FP32 storage can shrink is the preconditioner's)."""
    def per_step(p, k, key):
        return p[k][key] * (p[k]["launches"] if key == "bytes_per_launch" else 1) / steps if k in p else 0.0
    tot64 = sum(per_step(p64, k, "bytes_per_launch") for k in p64)
    out = {}
    for k in sorted(set(p64) | set(p32)):
        b64, b32 = per_step(p64, k, "bytes_per_launch"), per_step(p32, k, "bytes_per_launch")
        out[k] = {"fp64_MB": b64 / 1e6, "fp32_MB": b32 / 1e6,
                  "fp64_ms": per_step(p64, k, "ms_total"), "fp32_ms": per_step(p32, k, "ms_total"),
                  "share_of_fp64_bytes": b64 / tot64 if tot64 else None}
    return out


def timed_steps(s, b, opts, steps, warmup, profile_mask=0, every=1):
    """Time `steps` setup + solve steps; with profile_mask, HIP event pairs
    around one launch in `every` of those kernel classes (a pair costs the
    stream a few microseconds, so the headline pass times a sample)."""
    import torch
    from paper_2602_07225_amd import _lib as L
    for _ in range(warmup):
        s.setup(**opts)
        s.solve(b)
    torch.cuda.synchronize()
    if profile_mask:
        L.p4d_profile(s.ctx, profile_mask)
        L.p4d_profile_every(s.ctx, every)
    iters = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        s.setup(**opts)
        x, info = s.solve(b)
        iters += info.iters
        if info.status != 0:
            raise RuntimeError(f"solve did not converge: status {info.status}")
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    prof = {}
    if profile_mask:
        for k, name in L.KERNEL_CLASSES.items():
            ms, n, by = L.p4d_profile_read(s.ctx, k)
            if n:
                prof[name] = {"ms_total": ms, "launches": n, "avg_us": 1e3 * ms / n,
                              "bytes_per_launch": by / n,
                              "GBps": (by / 1e9) / (ms / 1e3) if ms > 0 else None}
        L.p4d_profile(s.ctx, 0)
        L.p4d_profile_every(s.ctx, 1)
    return x, info, iters, t, prof


def bench_batch(steps):
    """64 independent cells of uneven size (sides 16..48, N_r in {8, 16, 32}),
    FP32 preconditioner with autotuned smoother tiles, FGMRES(30) to 1e-8 in
    lockstep.  Solve time per batch with the batched stage launches and with
    per-cell launches of the same kernels; setup timed separately."""
    import torch
    import p4d_inputs as pi
    from paper_2602_07225_amd import P4DBatch
    from paper_2602_07225_amd import _lib as L
    cells = pi.make_batch(64)
    ntot = sum(p.N for p in cells)
    log(f"[bench] C4: {len(cells)} cells, {ntot} DOF")
    B = P4DBatch(cells, pc_prec=L.P4D_FP32)
    bs = [torch.as_tensor(p.b, device="cuda") for p in cells]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.setup(rtol=1e-8)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    tiles = B.autotune()
    out = {"cells": len(cells), "dof_total": ntot, "setup_ms": 1e3 * t_setup,
           "tiles": sorted(set(tiles))}
    for mode, name in ((0, "batched_stage_launches"), (2, "persistent_launch"), (1, "per_cell_launches")):
        B.set_pc_mode(mode)
        B.solve(bs)
        torch.cuda.synchronize()
        if mode == 0:
            B.profile(sum(1 << k for k in L.KERNEL_CLASSES))
        t0 = time.perf_counter()
        dof_it = 0
        for _ in range(steps):
            _, infos = B.solve(bs)
            dof_it += sum(p.N * i.iters for p, i in zip(cells, infos))
            if any(i.status != 0 for i in infos):
                raise RuntimeError("a batched cell did not converge")
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[name] = {"solve_ms": 1e3 * t / steps, "DOF_iter_per_s": dof_it / t,
                     "iters_min_max": [min(i.iters for i in infos), max(i.iters for i in infos)]}
        if mode == 0:
            kern = {}
            for k, kn in L.KERNEL_CLASSES.items():
                ms, n, by = B.profile_read(k)
                if n:
                    kern[kn] = {"ms_total": ms, "launch_groups": n, "avg_us": 1e3 * ms / n,
                                "GBps": (by / 1e9) / (ms / 1e3) if ms > 0 else None}
            out[name]["kernels"] = kern
            B.profile(0)
        log(f"[bench] C4 {name}: {1e3 * t / steps:.1f} ms/solve, {dof_it / t:.3e} DOF*iter/s")
    B.set_pc_mode(0)
    out["speedup_batched_vs_per_cell"] = (out["per_cell_launches"]["solve_ms"] /
                                          out["batched_stage_launches"]["solve_ms"])
    out["speedup_persistent_vs_stage_launches"] = (out["batched_stage_launches"]["solve_ms"] /
                                                   out["persistent_launch"]["solve_ms"])
    # per mesh side, the cell with the fewest unknowns: its FP32-preconditioned
    # solution, for the comparison with the oracle in the CPU leg
    xs, _ = B.solve(bs)
    pick = {}
    for i, p in enumerate(cells):
        if p.nx not in pick or p.N < cells[pick[p.nx]].N:
            pick[p.nx] = i
    out["_sample"] = [(i, xs[i].cpu().numpy()) for i in sorted(pick.values())]
    B.close()
    return out


def bench_newton(n=64, nr=(10, 10), steps=30, hetero=False, krylov=0):
    """The physical cube cell (Case I: 225 um cube, 100/25/100 um layers,
    appendix parameters, Gaussian 1C discharge current; with hetero, Case II:
    volume fractions per element from seeded random fields, uniform
    current): `steps` backward-Euler steps of 60 s, each by Newton
    iterations on the GPU (FGMRES over all unknowns, or with krylov = 1 over
    the Schur complement of the particle blocks)."""
    import torch
    from p4d_inputs import phys as ph
    from paper_2602_07225_amd import PhysCell
    from paper_2602_07225_amd import _lib as L
    case = ph.case2(n, nr, seed=2) if hetero else ph.PhysCase(n=n, nr=nr)
    q = [ph.F / 3600.0 * e.eps_s * case.electrode_volume * e.cs_max for e in case.electrodes]
    current = -case.c_rate * min(q)
    cell = PhysCell(case, current, coarse_max=64)
    u = cell.initial_state()
    o = cell.offsets
    top = slice(o[1] - n * n, o[1])          # phi_s on the top face (positive collector)
    v0 = u[top].mean().item()
    cell.step(u)                              # warm-up (compiles nothing, touches every kernel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    newton, lin = [], 0
    for _ in range(steps):
        u, info = cell.step(u, krylov=krylov)
        if info.status != 0:
            raise RuntimeError(f"Newton did not converge: status {info.status}")
        newton.append(info.iters)
        lin += info.lin_iters
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out = {"nodes_per_edge": n, "nr": list(nr), "dof": cell.N, "steps": steps, "dt_s": case.dt,
           "applied_current_A": current, "total_ms": 1e3 * t, "ms_per_step": 1e3 * t / steps,
           "newton_iters_per_step": float(np.mean(newton)), "newton_iters_max": int(max(newton)),
           "fgmres_iters_per_newton": lin / max(1, sum(newton)),
           "voltage_start_V": v0, "voltage_end_V": u[top].mean().item(),
           "krylov": "schur_complement" if krylov else "full"}
    cell.close()
    return out


def bench_case3(steps=2, warmup=1):
    """Case III-like flattened roll (the paper's element edges along the
    roll and the height, 60 elements through the 120 um stack, 1801 x 86 x
    61 nodes, N_r = 10): FGMRES(30) to 1e-8 with the SCHUR preconditioner and
    z-line multigrid.  Beside it, a 225 x 11-element section of the roll
    solved with both smoothers (the point-smoothed one capped at 1000
    iterations)."""
    import torch
    import p4d_inputs as pi
    from paper_2602_07225_amd import P4DSolver
    from paper_2602_07225_amd import _lib as L
    p = pi.make_case3_like()
    zl = dict(pc=L.P4D_PC_SCHUR, pc_prec=L.P4D_FP64, rtol=1e-8, restart=30,
              smoother=L.P4D_SMOOTH_ZLINE, coarse_max=64, cheb_degree=1)
    s = P4DSolver(p, smoother=L.P4D_SMOOTH_ZLINE, coarse_max=64)
    b = torch.as_tensor(p.b, device="cuda")
    t0 = time.perf_counter()
    s.setup(**zl)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    x, info, iters, t, prof = timed_steps(s, b, zl, steps, warmup, profile_mask=(1 << L.P4D_K_SMOOTH0))
    out = {"nodes": [p.nx, p.ny, p.nz], "nr": list(p.nr), "dof": p.N,
           "element_aspect": [p.hxy[0] / p.h, p.hxy[1] / p.h], "setup_ms": setup_ms,
           "sweeps_per_side": 1, "ms_per_solve": 1e3 * t / steps, "iters_per_solve": iters / steps,
           "DOF_iter_per_s": p.N * iters / t, "relres_true": info.relres_true,
           "zline_level0_pass": prof.get("smooth0")}
    _, _, it2, t2, _ = timed_steps(s, b, dict(zl, cheb_degree=2), steps, 1)
    out["two_sweeps_per_side"] = {"ms_per_solve": 1e3 * t2 / steps, "iters_per_solve": it2 / steps}
    _, i3, it3, t3, _ = timed_steps(s, b, dict(zl, krylov=L.P4D_KRYLOV_SCHUR), steps, 1)
    out["schur_krylov"] = {"ms_per_solve": 1e3 * t3 / steps, "iters_per_solve": it3 / steps,
                           "relres_true": i3.relres_true}
    del s, x, b
    torch.cuda.empty_cache()
    q = pi.make_case3_like(nx=226, ny=12)
    sec = {"nodes": [q.nx, q.ny, q.nz], "dof": q.N}
    bq = torch.as_tensor(q.b, device="cuda")
    for name, sm in (("zline", L.P4D_SMOOTH_ZLINE), ("chebyshev", L.P4D_SMOOTH_CHEB)):
        o = dict(zl, smoother=sm, maxit=1000, cheb_degree=2)
        sq = P4DSolver(q, smoother=sm, coarse_max=64)
        sq.setup(**o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, inf = sq.solve(bq)
        torch.cuda.synchronize()
        sec[name] = {"iters": inf.iters, "status": inf.status, "relres_true": inf.relres_true,
                     "ms": 1e3 * (time.perf_counter() - t0)}
        del sq
    out["section_225x11"] = sec
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extras", action="store_true", help="only the headline solve")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 64-cell batched solve (prints its JSON fields; for profiling)")
    ap.add_argument("--bgs-only", action="store_true",
                    help="only the block Gauss-Seidel solve of the cube in the paper's ordering "
                         "(prints its JSON fields; for profiling)")
    ap.add_argument("--schur-only", action="store_true",
                    help="only the cube solve with the Krylov space reduced to the Schur complement "
                         "of the particle blocks (prints its JSON fields; for profiling)")
    ap.add_argument("--newton-only", action="store_true",
                    help="only the Newton steps of the physical cube cell (prints its JSON fields)")
    ap.add_argument("--case3-only", action="store_true",
                    help="only the Case III-like flattened roll with z-line multigrid (prints its JSON)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 512 MiB device copy first (a reference of known size "
                         "for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the solver has no multi-GPU sharding)", file=sys.stderr)
        sys.exit(2)

    global np
    import numpy as np
    import torch

    import p4d_inputs as pi
    from paper_2602_07225_amd import P4DSolver
    from paper_2602_07225_amd import _lib as L

    torch.cuda.set_device(0)
    if args.batch_only:
        bat = bench_batch(args.steps)
        bat.pop("_sample", None)
        print(json.dumps({"C4_batch_64_cells": bat}), flush=True)
        return
    if args.case3_only:
        print(json.dumps({"case3_like_roll": bench_case3()}), flush=True)
        return
    if args.newton_only:
        print(json.dumps({"newton_case_I_cube": bench_newton(),
                          "newton_case_I_cube_schur_krylov": bench_newton(krylov=1),
                          "newton_case_II_cube": bench_newton(hetero=True)}), flush=True)
        return
    if args.schur_only:
        p = pi.make_config(2)
        s = P4DSolver(p, restart=30)
        b = torch.as_tensor(p.b, device="cuda")
        red = dict(pc=L.P4D_PC_SCHUR, krylov=L.P4D_KRYLOV_SCHUR, rtol=1e-8, restart=30,
                   pc_prec=L.P4D_FP64)
        mask = sum(1 << k for k in L.KERNEL_CLASSES)
        _, info, it, t, prof = timed_steps(s, b, red, args.steps, args.warmup, mask)
        print(json.dumps({"schur_krylov_C2": {
            "ms_per_step": 1e3 * t / args.steps, "iters_per_solve": it / args.steps,
            "DOF_iter_per_s": p.N * it / t, "kernels": prof}}), flush=True)
        return
    if args.bgs_only:
        p = pi.make_config(2)
        s = P4DSolver(p, restart=30)
        b = torch.as_tensor(p.b, device="cuda")
        bgs = dict(pc=L.P4D_PC_BGS, bgs_order=L.P4D_BGS_PAPER_ORDER, cgs2=1, rtol=1e-8,
                   restart=30, pc_prec=L.P4D_FP64)
        mask = sum(1 << k for k in L.KERNEL_CLASSES)
        _, info, it, t, prof = timed_steps(s, b, bgs, args.steps, args.warmup, mask)
        print(json.dumps({"block_gauss_seidel_C2": {
            "ms_per_step": 1e3 * t / args.steps, "iters_per_solve": it / args.steps,
            "kernels": prof}}), flush=True)
        return
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p = pi.make_config(2)
    N = p.N
    log(f"[bench] C2 N={N}: building solver")
    s = P4DSolver(p, restart=30)
    b = torch.as_tensor(p.b, device="cuda")
    # V(3,3): degree-3 Chebyshev smoothing (8 iterations instead of 9 with
    # degree 2 on this cube; the fastest degree measured)
    fp64 = dict(pc=L.P4D_PC_SCHUR, pc_prec=L.P4D_FP64, rtol=1e-8, restart=30, cheb_degree=3)
    mask = sum(1 << k for k in L.KERNEL_CLASSES)
    # a first pass with events around every launch of every kernel class
    # gives the per-class table and the dominant class; the timed steps then
    # record one event pair in SAMPLE_EVERY of that class only (every
    # launch of that class does the same work; all its pairs would add to
    # the headline step)
    _, _, _, _, prof = timed_steps(s, b, fp64, args.steps, args.warmup, mask)
    dom = max(prof, key=lambda k: prof[k]["ms_total"]) if prof else None
    dom_mask = (1 << next(k for k, v in L.KERNEL_CLASSES.items() if v == dom)) if dom else 0
    x64, info, iters, t, prof_dom = timed_steps(s, b, fp64, args.steps, 1, dom_mask, SAMPLE_EVERY)
    ms_step = 1e3 * t / args.steps
    value = N * iters / t
    log(f"[bench] FP64: {iters / args.steps:.1f} it/step, {ms_step:.2f} ms/step, "
        f"{value:.3e} DOF*iter/s")

    # dominant kernel class of the timed region
    roofline = None
    if dom and dom in prof_dom:
        d = prof_dom[dom]
        roofline = {"kernel": dom, "bound": "hbm", "achieved": d["GBps"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": d["GBps"] / HBM_PEAK_GBS,
                    "traffic": measured_traffic(dom),
                    "avg_launch_us": d["avg_us"], "bytes_per_launch": d["bytes_per_launch"],
                    "timed_launches": d["launches"], "sampled_every": SAMPLE_EVERY}
        # an event pair also times its own processing on the queue, shared by
        # the launches it spans (for the level-0 smoother the steps on one
        # side of a coarse correction): measured here with nothing between
        # the events, for context; avg_launch_us keeps it (the conservative
        # figure; the kernel trace in profiles/ gives the durations alone)
        roofline["event_pair_us"] = event_pair_us()

    # setup and solve split (one extra, untimed-in-the-headline run)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.setup(**fp64)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    # GPU solutions kept on the host for the comparison with the oracle
    keep = {"C2_fp64": x64.cpu().numpy()}
    extras = {"setup_ms": 1e3 * t_setup,
              "solve_ms": ms_step - 1e3 * t_setup,
              "iters_per_solve": iters / args.steps,
              "solve_only_DOF_iter_per_s": N * iters / args.steps / max(1e-9, (t / args.steps - t_setup)),
              "kernels": prof}

    if not args.no_extras:
        # FP32 preconditioner (radial eliminations + V-cycle storage); the Z
        # basis stays FP64 (its near-null component would swamp FP32 storage)
        fp32 = dict(fp64, pc_prec=L.P4D_FP32)
        x32, i32, it32, t32, _ = timed_steps(s, b, fp32, args.steps, 1)
        keep["C2_fp32"] = x32.cpu().numpy()
        err = (torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64)).item()
        # per kernel class: the bytes each precision moves per step (a pass
        # with events around every launch, as for the FP64 table)
        _, _, _, _, prof32 = timed_steps(s, b, fp32, args.steps, 1, mask)
        extras["fp32_precond_C2"] = {"ms_per_step": 1e3 * t32 / args.steps,
                                     "iters_per_solve": it32 / args.steps,
                                     "DOF_iter_per_s": N * it32 / t32,
                                     "rel_err_vs_fp64_gpu": err,
                                     "speedup_vs_fp64": t / t32,
                                     "byte_split": byte_split(prof, prof32, args.steps)}
        log(f"[bench] FP32-PC C2: {1e3 * t32 / args.steps:.2f} ms/step, {it32 / args.steps:.1f} it")
        # block-Jacobi preconditioner (the paper's eq. PJ) on the same input
        # (Chebyshev degree 2: BJ and BGS take fewer iterations with it)
        bj = dict(fp64, pc=L.P4D_PC_BJ, cgs2=1, cheb_degree=2)
        try:
            _, ibj, itbj, tbj, _ = timed_steps(s, b, bj, 2, 1)
            extras["block_jacobi_C2"] = {"ms_per_step": 1e3 * tbj / 2, "iters_per_solve": itbj / 2}
            log(f"[bench] BJ C2: {1e3 * tbj / 2:.2f} ms/step, {itbj / 2:.1f} it")
        except RuntimeError as ex:
            extras["block_jacobi_C2"] = {"error": str(ex)}
        # block Gauss-Seidel (eq. PGS), the paper's ordering, both precisions;
        # then all 24 orderings
        bgs = dict(fp64, pc=L.P4D_PC_BGS, bgs_order=L.P4D_BGS_PAPER_ORDER, cgs2=1, cheb_degree=2)
        try:
            _, _, itg, tg, _ = timed_steps(s, b, bgs, 2, 1)
            _, _, itg32, tg32, _ = timed_steps(s, b, dict(bgs, pc_prec=L.P4D_FP32), 2, 1)
            extras["block_gauss_seidel_C2"] = {
                "ordering": ["phi_e", "c_s", "phi_s", "c_e"],
                "fp64": {"ms_per_step": 1e3 * tg / 2, "iters_per_solve": itg / 2},
                "fp32_precond": {"ms_per_step": 1e3 * tg32 / 2, "iters_per_solve": itg32 / 2}}
            log(f"[bench] BGS C2: {1e3 * tg / 2:.2f} ms/step, {itg / 2:.1f} it; "
                f"FP32-PC {1e3 * tg32 / 2:.2f} ms/step")
        except RuntimeError as ex:
            extras["block_gauss_seidel_C2"] = {"error": str(ex)}
        # Krylov space reduced to the Schur complement of the particle blocks
        # (the same system and tolerance; FGMRES over the 2.2 M electrode-level
        # unknowns), both preconditioner precisions
        sk = dict(fp64, krylov=L.P4D_KRYLOV_SCHUR, cheb_degree=2)   # its fastest degree
        xs64, is64, its64, ts64, profs = timed_steps(s, b, sk, args.steps, 1, mask)
        xs32, is32, its32, ts32, _ = timed_steps(s, b, dict(sk, pc_prec=L.P4D_FP32), args.steps, 1)
        keep["C2_schur_krylov_fp64"] = xs64.cpu().numpy()
        keep["C2_schur_krylov_fp32"] = xs32.cpu().numpy()
        extras["schur_krylov_C2"] = {
            "fp64": {"ms_per_step": 1e3 * ts64 / args.steps, "iters_per_solve": its64 / args.steps,
                     "DOF_iter_per_s": N * its64 / ts64, "relres_true": is64.relres_true,
                     "rel_diff_vs_full_space": (torch.linalg.norm(xs64 - x64) /
                                                torch.linalg.norm(x64)).item()},
            "fp32_precond": {"ms_per_step": 1e3 * ts32 / args.steps,
                             "iters_per_solve": its32 / args.steps,
                             "DOF_iter_per_s": N * its32 / ts32,
                             "rel_diff_vs_full_space": (torch.linalg.norm(xs32 - x64) /
                                                        torch.linalg.norm(x64)).item()},
            "speedup_vs_full_space": t / ts64,
            "kernels": profs}
        log(f"[bench] Schur-Krylov C2: fp64 {1e3 * ts64 / args.steps:.2f} ms ({its64 / args.steps:.0f} it), "
            f"fp32-PC {1e3 * ts32 / args.steps:.2f} ms ({its32 / args.steps:.0f} it)")
        del xs64, xs32
        extras["bgs_orderings_C2"] = bgs_sweep(s, b, dict(fp64, cheb_degree=2))
        log(f"[bench] BGS orderings C2: best {extras['bgs_orderings_C2']['best']}, "
            f"worst {extras['bgs_orderings_C2']['worst']}")
        # lognormal cube, both precisions
        p3 = pi.make_config(3)
        s3 = P4DSolver(p3, restart=30)
        b3 = torch.as_tensor(p3.b, device="cuda")
        xa, ia, ita, ta, _ = timed_steps(s3, b3, fp64, args.steps, 1)
        xb, ib, itb, tb, _ = timed_steps(s3, b3, fp32, args.steps, 1)
        keep["C3_fp64"], keep["C3_fp32"] = xa.cpu().numpy(), xb.cpu().numpy()
        extras["C3_lognormal"] = {
            "fp64": {"ms_per_step": 1e3 * ta / args.steps, "iters_per_solve": ita / args.steps},
            "fp32_precond": {"ms_per_step": 1e3 * tb / args.steps, "iters_per_solve": itb / args.steps,
                             "rel_err_vs_fp64_gpu":
                                 (torch.linalg.norm(xb - xa) / torch.linalg.norm(xa)).item()},
            "speedup_fp32_vs_fp64": ta / tb}
        log(f"[bench] C3: fp64 {1e3 * ta / args.steps:.2f} ms, fp32 {1e3 * tb / args.steps:.2f} ms")
        xc, _, itc, tc3, _ = timed_steps(s3, b3, dict(sk), args.steps, 1)
        xc32, _, itc32, tc332, _ = timed_steps(s3, b3, dict(sk, pc_prec=L.P4D_FP32), args.steps, 1)
        keep["C3_schur_krylov_fp64"] = xc.cpu().numpy()
        keep["C3_schur_krylov_fp32"] = xc32.cpu().numpy()
        del xc, xc32
        extras["schur_krylov_C3"] = {
            "fp64": {"ms_per_step": 1e3 * tc3 / args.steps, "iters_per_solve": itc / args.steps},
            "fp32_precond": {"ms_per_step": 1e3 * tc332 / args.steps,
                             "iters_per_solve": itc32 / args.steps}}
        log(f"[bench] Schur-Krylov C3: fp64 {1e3 * tc3 / args.steps:.2f} ms, "
            f"fp32-PC {1e3 * tc332 / args.steps:.2f} ms")
        extras["bgs_orderings_C3"] = bgs_sweep(s3, b3, dict(fp64, cheb_degree=2))
        log(f"[bench] BGS orderings C3: best {extras['bgs_orderings_C3']['best']}, "
            f"worst {extras['bgs_orderings_C3']['worst']}")
        del s3
        # adjoint solve + gradients on C2 (J = mean phi_s on the cathode top face)
        w = torch.as_tensor(pi.functional_weights(p), device="cuda")
        s.setup(**fp64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, ia = s.solve_adjoint(w)
        gs, gD = s.gradient(x64, lam)
        torch.cuda.synchronize()
        extras["adjoint_C2"] = {"ms": 1e3 * (time.perf_counter() - t0), "iters": ia.iters,
                                "status": ia.status}

    if not args.no_extras:
        # large cell: forward + adjoint solves and gradients (68 M unknowns)
        p5 = pi.make_config(5)
        s5 = P4DSolver(p5, restart=30)
        b5 = torch.as_tensor(p5.b, device="cuda")
        w5 = torch.as_tensor(pi.functional_weights(p5), device="cuda")
        s5.setup(**fp64)
        s5.solve(b5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s5.setup(**fp64)
        x5, f5 = s5.solve(b5)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        l5, a5 = s5.solve_adjoint(w5)
        g5, gD5 = s5.gradient(x5, l5)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        extras["C5_forward_adjoint"] = {
            "dof": p5.N, "forward_ms": 1e3 * (t1 - t0), "forward_iters": f5.iters,
            "adjoint_plus_gradient_ms": 1e3 * (t2 - t1), "adjoint_iters": a5.iters,
            "DOF_iter_per_s_forward": p5.N * f5.iters / (t1 - t0)}
        log(f"[bench] C5: forward {1e3 * (t1 - t0):.1f} ms ({f5.iters} it), adjoint+grad "
            f"{1e3 * (t2 - t1):.1f} ms ({a5.iters} it)")
        # the same with the Krylov space reduced to the Schur complement
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s5.setup(**fp64)
        x5r, f5r = s5.solve(b5, krylov=L.P4D_KRYLOV_SCHUR)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        l5r, a5r = s5.solve_adjoint(w5, krylov=L.P4D_KRYLOV_SCHUR)
        g5r, gD5r = s5.gradient(x5r, l5r)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        extras["schur_krylov_C5"] = {
            "forward_ms": 1e3 * (t1 - t0), "forward_iters": f5r.iters,
            "adjoint_plus_gradient_ms": 1e3 * (t2 - t1), "adjoint_iters": a5r.iters,
            "DOF_iter_per_s_forward": p5.N * f5r.iters / (t1 - t0),
            "rel_diff_vs_full_space": {
                "x": (torch.linalg.norm(x5r - x5) / torch.linalg.norm(x5)).item(),
                "lambda": (torch.linalg.norm(l5r - l5) / torch.linalg.norm(l5)).item(),
                "dJ_dsigma": (torch.linalg.norm(g5r - g5) / torch.linalg.norm(g5)).item()}}
        log(f"[bench] Schur-Krylov C5: forward {1e3 * (t1 - t0):.1f} ms ({f5r.iters} it), "
            f"adjoint+grad {1e3 * (t2 - t1):.1f} ms ({a5r.iters} it)")
        del s5, x5, l5, g5, x5r, l5r, g5r

    if not args.no_extras:
        extras["C4_batch_64_cells"] = bench_batch(args.steps)
        try:
            extras["case3_like_roll"] = e = bench_case3()
            log(f"[bench] Case III-like roll N={e['dof']}: z-line {e['ms_per_solve']:.1f} ms/solve, "
                f"{e['iters_per_solve']:.1f} it (Schur-Krylov {e['schur_krylov']['ms_per_solve']:.1f} ms); "
                f"section: z-line {e['section_225x11']['zline']['iters']} it, "
                f"point {e['section_225x11']['chebyshev']['iters']} it "
                f"(status {e['section_225x11']['chebyshev']['status']})")
        except RuntimeError as ex:
            extras["case3_like_roll"] = {"error": str(ex)}
        for key, het, kry in (("newton_case_I_cube", False, 0), ("newton_case_I_cube_schur_krylov", False, 1),
                              ("newton_case_II_cube", True, 0)):
            try:
                extras[key] = e = bench_newton(hetero=het, krylov=kry)
                log(f"[bench] Newton {'Case II' if het else 'Case I'}{' (Schur-Krylov)' if kry else ''}: "
                    f"{e['steps']} steps, "
                    f"{e['ms_per_step']:.1f} ms/step, {e['newton_iters_per_step']:.1f} Newton it/step, "
                    f"V {e['voltage_start_V']:.4f} -> {e['voltage_end_V']:.4f}")
            except RuntimeError as ex:
                extras[key] = {"error": str(ex)}

    cpu = None
    if not args.no_cpu:
        import oracle as O
        log("[bench] CPU oracle: two full C2 steps")
        t0 = time.perf_counter()
        its = 0
        for _ in range(2):
            orc = O.Oracle(p).setup(rtol=1e-8, cheb_degree=fp64["cheb_degree"])
            xo, io = orc.solve(p.b)
            its += io.iters
        tc = time.perf_counter() - t0
        vs = {k: field_errors(p, v, xo) for k, v in keep.items() if k.startswith("C2")}
        cpu = {"value": N * its / tc, "unit": "DOF*iter/s", "cores": O.num_threads(),
               "cpu_model": cpu_model(), "kind": "oracle",
               "sample": f"two full steps of the same workload (setup + {io.iters} FGMRES iterations "
                         f"to rtol 1e-8, each), {tc:.1f} s",
               "gpu_vs_oracle_rel_err": vs["C2_fp64"]["all"],
               "gpu_vs_oracle_rel_err_per_field": vs}
        log(f"[bench] oracle: {tc:.1f} s, {io.iters} it, rel err gpu vs oracle {vs['C2_fp64']['all']:.2e}")
        if "C3_fp64" in keep:
            # the lognormal cube: one oracle step (timed), and the error of
            # every GPU solution of it against the oracle's
            p3 = pi.make_config(3)
            t0 = time.perf_counter()
            orc = O.Oracle(p3).setup(rtol=1e-8, cheb_degree=fp64["cheb_degree"])
            xo3, io3 = orc.solve(p3.b)
            tc3 = time.perf_counter() - t0
            extras["oracle_C3"] = {
                "value": p3.N * io3.iters / tc3, "unit": "DOF*iter/s", "cores": O.num_threads(),
                "iters": io3.iters, "seconds": tc3,
                "gpu_vs_oracle_rel_err_per_field": {k: field_errors(p3, v, xo3) for k, v in keep.items()
                                                    if k.startswith("C3")}}
            log(f"[bench] oracle C3: {tc3:.1f} s, {io3.iters} it")
        bat = extras.get("C4_batch_64_cells", {})
        if bat.get("_sample"):
            # a sample of the batch: per mesh side, the cell with the fewest
            # unknowns, against its oracle solve
            rows = []
            for i, xc in bat.pop("_sample"):
                pc = pi.make_batch(64)[i]
                xoc, _ = O.Oracle(pc).setup(rtol=1e-8).solve(pc.b)
                rows.append({"cell": i, "side": pc.nx, "nr": list(pc.nr), "dof": pc.N,
                             **field_errors(pc, xc, xoc)})
            bat["fp32_vs_oracle_sample"] = rows
    extras.get("C4_batch_64_cells", {}).pop("_sample", None)

    out = {
        "metric": "P4D Jacobian solve time & DOF*iter/s; FP32-precond vs FP64; HBM GB/s",
        "value": value,
        "unit": "DOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "homogeneous cube cell 64x64x192 nodes, Nr=20, 15,335,424 DOF; "
                               "FP64 FGMRES(30) + particle-Schur block preconditioner (V(3,3) "
                               "Chebyshev multigrid) to rtol 1e-8; step = setup + solve",
                   "nodes": [p.nx, p.ny, p.nz], "layers": [p.na, p.ns, p.nc], "nr": list(p.nr),
                   "dof": N, "restart": 30, "rtol": 1e-8, "pc": "schur", "cheb_degree": 3},
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
