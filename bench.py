#!/usr/bin/env python3
"""Throughput of the tau-preconditioned GMRES time stepper on one MI355X.

A step is one Crank-Nicolson time step of the 2-D workload (N = 1023 per axis,
alpha = (1.3, 1.7), kappa = (1, 0.5), e = 2 + sin(pi x) sin(pi y) cos t, f = 8x8
sine modes with seeded N(0,1) amplitudes, psi = 0, dt = 1/32, GMRES(30) to
rtol 1e-10, FP64): evaluate e at t_{m+1/2}, form the right-hand side and run
the preconditioned GMRES solve on the device.  Inputs are resident in HBM before
the timed region starts.  The timed steps run in the library's own time loop
(rsfde_solve_range), one call for all of them.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-steps/sec (PGMRES to 1e-10) on 2D 1023²; HBM GB/s of FFT/DST kernels"
HBM_PEAK_GBS = 8000.0
KCLASS_NAMES = ("mv_first", "mv_mid", "mv_last", "dst", "dsd", "dots", "orth_dots", "orth_norm", "update")
KCLASS_KERNELS = {
    "mv_first": "rsfde_pass_kernel, first-axis operator pass (B stencil on e.v and v, Toeplitz product)",
    "mv_mid": "rsfde_pass_kernel, middle-axis operator pass",
    "mv_last": "rsfde_pass_kernel, last-axis operator pass (B stencil, Toeplitz product, sine transform)",
    "dst": "rsfde_dst_kernel, sine-transform pass",
    "dsd": "rsfde_dst_kernel, sine transform + 1/mu scaling + sine transform",
    "dots": "k_sweep1 (Arnoldi sweep A: basis dot products)",
    "orth_dots": "k_sweepB (Arnoldi sweep B: delayed second projection, first projection)",
    "orth_norm": "(unused)",
    "update": "k_update (Givens resolve + solution update)",
}
WORKLOAD_TEXT = {
    "C1": "C1: 1-D N=511, alpha=1.5, kappa=1, e=1+x^2(1+t), manufactured u=e^-t x^2(1-x)^2, "
          "dt=1/64, GMRES(20) rtol 1e-12, FP64",
    "C2": "C2: 2-D N=1023x1023, alpha=(1.3,1.7), kappa=(1,0.5), e=2+sin(pi x)sin(pi y)cos t, "
          "f=8x8 seeded sine modes, psi=0, dt=1/32, GMRES(30) rtol 1e-10, FP64",
    "C3": "C3: 3-D N=255^3, alpha=(1.2,1.5,1.8), kappa=(1,1,1), e=1+0.5xyz(1+t), manufactured "
          "u=e^-t prod x_i^2(1-x_i)^2, dt=1/16, GMRES(30) rtol 1e-10, FP64",
    "C5": "C5: 3-D N=511^3, alpha=(1.4,1.6,1.9), kappa=(1,0.8,0.6), e=2+prod sin(pi x_i) cos t, "
          "f=8x8x8 seeded sine modes, psi=0, dt=1/8, GMRES(20) rtol 1e-10, FP64",
    "C4": "C4: 64 independent 2-D instances, N_i in {127,255,383,511} per axis (6.5M unknowns), "
          "alpha_i~U(1.1,1.9), kappa_i~U(0.2,2), e=1+U*g, f=8x8 seeded sine modes, psi=0, dt=1/16, "
          "GMRES(30) rtol 1e-10, FP64, batched launches; a step advances all 64",
}


def pass_symbol(R, h, inst, kclass: str):
    """Kernel instantiation the autotuner picked for a pencil-pass class (the name
    rocprofv3 reports: the length argument is the plan code, L or L + 65536), or
    None for the other classes."""
    d = inst.d
    where = {"mv_first": (0, 0), "mv_mid": (1, 0), "mv_last": (d - 1, 0), "dsd": (0, 1),
             "dst": (d - 1, 1)}.get(kclass)
    if where is None or where[0] >= d:
        return None
    L, F = R.rsfde_get_pass_shape(h, 0, where[0], R.RSFDE_FP64, where[1])
    code, _ = R.rsfde_get_pass_plan(h, 0, where[0], R.RSFDE_FP64, where[1])
    kern = "rsfde_dst_kernel" if where[1] else "rsfde_pass_kernel"
    return f"{kern}<double, {code}, {F}, {'true' if where[0] > 0 else 'false'}>"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2404_10221_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str, symbol: str):
    """HBM bytes per launch of one kernel instantiation from the committed rocprofv3
    counter summary, when it was taken on the current kernel sources, on this
    workload and on this very instantiation (tile shape included); else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or not symbol:
        return None
    with open(path) as fh:
        data = json.load(fh)
    if data.get("source_hash") != kernel_source_hash():
        return None
    ent = data.get("workloads", {}).get(workload, {}).get(symbol)
    return None if ent is None else ent.get("bytes_per_launch")


def copy_ceilings():
    """Device-copy bandwidth (read + write bytes per second) measured on this GPU with
    torch events: a 1 GiB copy (HBM-resident) and a repeated 48 MiB copy (96 MiB of
    source and destination: past the 32 MiB of L2 caches, inside the 256 MiB
    Infinity Cache, like the 2-D workload's vectors)."""
    import torch
    out = {}
    for name, nbytes, ring, reps in (("hbm", 1 << 30, 1, 4), ("mall", 48 << 20, 1, 64)):
        n = nbytes // 8
        src = [torch.ones(n, dtype=torch.float64, device="cuda") for _ in range(ring)]
        dst = [torch.empty_like(x) for x in src]
        for k in range(ring):
            dst[k].copy_(src[k])
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for r in range(reps):
            dst[r % ring].copy_(src[r % ring])
        b.record()
        b.synchronize()
        out[name + "_copy_gbs"] = 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
        del src, dst
    torch.cuda.empty_cache()
    return out


def host_info():
    """CPU model, logical cores and RAM of the host."""
    model, ram = "unknown", None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:  # pragma: no cover
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "host_ram_gib": ram}


class Stepper:
    """Owns a handle on one or more instances (several: batched launches) and steps
    them together with device-evaluated fields."""

    def __init__(self, insts, graphs=False, **over):
        import torch
        from paper_2404_10221_amd import rsfde as R
        self.R = R
        self.insts = list(insts) if isinstance(insts, (list, tuple)) else [insts]
        self.inst = self.insts[0]
        self.S = R.Solver([R.params_from_instance(i, **over) for i in self.insts])
        if graphs:
            R.rsfde_set_graph(self.S.h, True)
        self.us, self.es, self.fs = [], [], []
        for k, inst in enumerate(self.insts):
            R.rsfde_set_fields(self.S.h, k, inst.e, inst.f, inst.psi)
            R.rsfde_prescan_ebar(self.S.h, k, inst.M)
            ncl = 1
            for v in inst.n:
                ncl *= v + 2
            self.us.append(torch.empty(inst.size, dtype=torch.float64, device="cuda"))
            self.es.append(torch.empty(inst.size, dtype=torch.float64, device="cuda"))
            self.fs.append(torch.empty(ncl, dtype=torch.float64, device="cuda"))
            R.rsfde_eval_field(self.S.h, k, R.WHICH_PSI, 0.0, self.us[k])
            R.rsfde_eval_field(self.S.h, k, R.WHICH_F, 0.5 * inst.dt, self.fs[k])
            R.rsfde_eval_field(self.S.h, k, R.WHICH_E, 0.5 * inst.dt, self.es[k])
        self.u = self.us[0]
        self.m = 0
        self.iters = 0
        self.sweeps = 0
        self.true_res = -1.0
        self.status = 0

    def step(self):
        # e and f at t_{m+1/2}; a field that does not depend on t keeps its first evaluation
        R = self.R
        th = (self.m + 0.5) * self.inst.dt
        if len(self.insts) > 1 and all(i.dt == self.inst.dt for i in self.insts):
            if any(i.e.time_dependent for i in self.insts):
                R.rsfde_eval_field_batch(self.S.h, R.WHICH_E, th, self.es)  # one launch for all
            if any(i.f.time_dependent for i in self.insts):
                R.rsfde_eval_field_batch(self.S.h, R.WHICH_F, th, self.fs)
        else:
            for k, inst in enumerate(self.insts):
                tk = (self.m + 0.5) * inst.dt
                if inst.e.time_dependent:
                    R.rsfde_eval_field(self.S.h, k, R.WHICH_E, tk, self.es[k])
                if inst.f.time_dependent:
                    R.rsfde_eval_field(self.S.h, k, R.WHICH_F, tk, self.fs[k])
        s, st = R.rsfde_step(self.S.h, self.m * self.inst.dt, self.es, self.fs, self.us)
        self.status = max(self.status, s)
        self.iters += sum(x["iters"] for x in st)
        self.sweeps += sum(x["outer_sweeps"] for x in st)
        self.true_res = max([self.true_res] + [x["rel_true_res"] for x in st])
        self.m += 1

    def run(self, k):
        # k steps in the library's own time loop (rsfde_solve_range from step m, the
        # registered fields sampled on the device at each midpoint): the same
        # kernels and time levels as k calls of step(), without a host round trip
        # per step.  true_res keeps the largest last-step value over the calls.
        if k <= 0:
            return
        R = self.R
        s, st = R.rsfde_solve_range(self.S.h, self.m, k, self.us)
        self.status = max(self.status, s)
        self.iters += sum(x["iters"] for x in st)
        self.sweeps += sum(x["outer_sweeps"] for x in st)
        self.true_res = max([self.true_res] + [x["rel_true_res"] for x in st])
        self.m += k

    def close(self):
        self.S.close()


def cpu_baseline_batch(insts, nsample: int):
    """Many-instance workload: time the FP64 oracle on one step of the first
    `nsample` instances and scale to the whole batch by unknown count; parity of
    the batched GPU step on the same instances."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    sample = insts[:nsample]
    t0 = time.perf_counter()
    refs = []
    for inst in sample:
        P = O.OracleProblem(inst)
        u, _ = P.step(P.psi(), 0)
        refs.append(u.ravel())
    dt = time.perf_counter() - t0
    n_s = sum(i.size for i in sample)
    n_all = sum(i.size for i in insts)
    g = Stepper(insts)
    g.step()
    par = 0.0
    for k, ref in enumerate(refs):
        got = g.us[k].cpu().numpy()
        par = max(par, float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)))
    g.close()
    out = {
        "value": (n_s / n_all) / dt, "unit": "time-steps/s", "cores": int(threads), "kind": "oracle",
        "sample": f"first step of instances 0..{nsample - 1} ({n_s} of {n_all} unknowns) in {dt:.1f} s, "
                  f"scaled to the whole batch by unknown count",
        "parity_rel_diff_gpu_vs_oracle": par,
    }
    out.update(host_info())
    return out


def _oracle_steps(O, inst, steps, rtol=None):
    from dataclasses import replace
    if rtol is not None:
        inst = replace(inst, rtol=rtol, max_cycles=max(inst.max_cycles, 20))
    P = O.OracleProblem(inst)
    u = P.psi()
    its = []
    t0 = time.perf_counter()
    big = inst.size > 4_000_000

    def progress(k, r):
        # the large grids take seconds per oracle iteration: report each one
        if big:
            print(f"oracle step {len(its)}: iteration {k}, residual {r:.2e}, "
                  f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)

    for m in range(steps):
        u, st = P.step(u, m, progress=progress)
        its.append(st["iters"])
    return u.ravel(), its, time.perf_counter() - t0


def cpu_baseline(inst, steps: int, tight: bool = True, one_thread_steps: int = 1):
    """Time the FP64 oracle on `steps` steps from psi on the host cores, and on
    `one_thread_steps` steps with one thread; run the GPU's FP64 and mixed forms on the
    same steps for parity figures: FP64 against the oracle (same Krylov sequence),
    mixed against the oracle solved to 1e-13 (the mixed form iterates along another
    sequence, so it is held to the exact solution of each step's system)."""
    import numpy as np
    import oracle as O
    from paper_2404_10221_amd import rsfde as R
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threadpool_limits = None
        threads = os.cpu_count() or 1
    ref, its, dt = _oracle_steps(O, inst, steps)

    def rel(a, b):
        return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))

    def gpu(**over):
        g = Stepper(inst, **over)
        for _ in range(steps):
            g.step()
        got = g.u.cpu().numpy()
        g.close()
        return got

    out = {
        "value": steps / dt, "unit": "time-steps/s", "cores": int(threads), "kind": "oracle",
        "sample": f"first {steps} of the {inst.M} steps from psi (dense-matrix FP64 oracle, "
                  f"{sum(its)} GMRES iterations); {dt:.1f} s wall",
        "parity_rel_diff_gpu_vs_oracle": rel(gpu(), ref),
    }
    out.update(host_info())
    if tight:
        ref_t, its_t, dt_t = _oracle_steps(O, inst, steps, rtol=1e-13)
        out["parity_rel_diff_mixed_gpu_vs_oracle_rtol_1e-13"] = rel(gpu(precision=R.RSFDE_MIXED), ref_t)
        out["rel_diff_oracle_vs_oracle_rtol_1e-13"] = rel(ref, ref_t)
    if one_thread_steps and threadpool_limits is not None:
        with threadpool_limits(limits=1):
            _, its1, dt1 = _oracle_steps(O, inst, one_thread_steps)
        out["one_thread"] = {"value": one_thread_steps / dt1, "unit": "time-steps/s",
                             "sample": f"first {one_thread_steps} step(s), {sum(its1)} GMRES "
                                       f"iterations, {dt1:.1f} s wall"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-strang", action="store_true",
                    help="skip the run with the Strang circulant preconditioner")
    ap.add_argument("--no-two-sided", action="store_true",
                    help="skip the run of the two-sided form (eq. Pls)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="skip the run with graph replay of the Arnoldi steps")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--cpu-instances", type=int, default=4,
                    help="instances of a many-instance workload the oracle baseline samples")
    ap.add_argument("--workload", default="C2", choices=("C1", "C2", "C3", "C4", "C5"))
    ap.add_argument("--timing-every", type=int, default=8,
                    help="time one launch in this many of the dominant kernel class (a stamped "
                         "dispatch waits about 5 us longer to start)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_10221_amd import rsfde as R
    from rsfde_workloads import config

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = (1 << 30) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                          "launches": 3}), flush=True)
        return
    cfg = config(args.workload)
    insts = cfg if isinstance(cfg, list) else [cfg]
    inst = insts[0]
    unknowns = sum(i.size for i in insts)
    K, W = args.steps, args.warmup

    # ---- FP64 form: warm-up with every kernel class timed (to find the dominant one)
    g = Stepper(insts)
    R.rsfde_set_timing(g.S.h, (1 << len(KCLASS_NAMES)) - 1, 1)
    g.run(W)
    tot = {}
    for c, name in enumerate(KCLASS_NAMES):
        n, ms, by = R.rsfde_get_timing(g.S.h, c)
        tot[name] = (n, ms, by)
    dom = max(tot, key=lambda k: tot[k][1])
    dom_cls = KCLASS_NAMES.index(dom)
    # ---- timed region: time one launch in `timing_every` of the dominant class
    R.rsfde_set_timing(g.S.h, 1 << dom_cls, args.timing_every)
    it0 = g.iters
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.run(K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n, ms, by = R.rsfde_get_timing(g.S.h, dom_cls)
    R.rsfde_set_timing(g.S.h, 0, 1)
    elapsed = t1 - t0
    iters = g.iters - it0
    u64 = [u.clone() for u in g.us]
    status = g.status
    symbol = pass_symbol(R, g.S.h, inst, dom) if len(insts) == 1 else None
    g.close()
    achieved = (by / n) / ((ms / n) * 1e-3) / 1e9 if n else 0.0
    traffic = read_traffic(args.workload, symbol)
    ceil = copy_ceilings()
    out = {
        "metric": METRIC,
        "value": K / elapsed,
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "instances": len(insts), "unknowns": unknowns, "gmres_iters_per_step": iters / K,
                   "status": status},
        "roofline": {
            "bound": "hbm", "kernel": dom, "kernel_symbol": symbol or KCLASS_KERNELS.get(dom, dom),
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "launches_timed": n, "avg_launch_us": 1e3 * ms / n if n else None,
            "algorithmic_bytes_per_launch": by / n if n else None,
            "copy_ceilings_gbs": {k: round(v, 1) for k, v in ceil.items()},
            "frac_of_hbm_copy": achieved / ceil["hbm_copy_gbs"],
            "frac_of_mall_copy": achieved / ceil["mall_copy_gbs"],
            "launches": "launches that exited on the status word past the end of their "
                        "GMRES cycle are left out",
        },
        # every kernel class over the fully timed warm-up: launches that did work,
        # total and average time, and the HBM fraction of its algorithmic bytes
        "kernel_classes_warmup": {
            k: {"launches": v[0], "ms": round(v[1], 4),
                "avg_us": round(1e3 * v[1] / v[0], 2),
                "frac": round((v[2] / v[0]) / ((v[1] / v[0]) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            for k, v in tot.items() if v[0] > 0 and v[1] > 0},
    }

    def rel(xs, ys):
        return max(float((a - b).abs().max() / b.abs().max().clamp_min(1e-300)) for a, b in zip(xs, ys))

    def timed_leg(**over):
        gl = Stepper(insts, **over)
        gl.run(W)
        it0, sw0 = gl.iters, gl.sweeps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gl.run(K)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        us = [u.clone() for u in gl.us]
        res = {"value": K / el, "unit": "time-steps/s", "ms_per_step": 1e3 * el / K,
               "gmres_iters_per_step": (gl.iters - it0) / K,
               "outer_sweeps_per_step": (gl.sweeps - sw0) / K,
               "max_rel_true_res": gl.true_res, "status": gl.status}
        gl.close()
        return res, us

    # ---- mixed FP32 operator + FP64 refinement on the same steps, at equal accuracy:
    # every form's distance from a tight solve (FP64 to rtol 1e-14) of the same steps,
    # and the FP64 form run to the mixed form's own stopping bound (rtol / 10 on the
    # FP64 preconditioned residual)
    if not args.no_mixed:
        _, tight = timed_leg(rtol=1e-14, max_cycles=50)
        res, um = timed_leg(precision=R.RSFDE_MIXED)
        res["rel_diff_vs_fp64_gpu"] = rel(um, u64)
        res["rel_diff_vs_tight_solve"] = rel(um, tight)
        res["outer_rtol"] = 0.1 * inst.rtol
        out["mixed"] = res
        res, ub = timed_leg(rtol=0.1 * inst.rtol)
        res["rel_diff_vs_tight_solve"] = rel(ub, tight)
        out["fp64_at_mixed_bound"] = res
        out["config"]["rel_diff_vs_tight_solve"] = rel(u64, tight)

    # ---- two-sided form (eq. Pls, FP64) on the same steps: more passes per iteration
    if not args.no_two_sided:
        gt = Stepper(insts, method=R.RSFDE_TPGM)
        gt.run(W)
        it0 = gt.iters
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gt.run(K)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        diff = max(float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))
                   for a, b in zip(gt.us, u64))
        out["two_sided"] = {"value": K / el, "unit": "time-steps/s", "ms_per_step": 1e3 * el / K,
                            "gmres_iters_per_step": (gt.iters - it0) / K,
                            "rel_diff_vs_one_sided_gpu": diff, "status": gt.status}
        gt.close()

    # ---- the paper's comparison solver: Strang circulant preconditioner (FP64)
    if not args.no_strang:
        gs = Stepper(insts, method=R.RSFDE_SPGM)
        gs.run(W)
        it0 = gs.iters
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gs.run(K)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        diff = max(float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))
                   for a, b in zip(gs.us, u64))
        out["strang"] = {"value": K / el, "unit": "time-steps/s", "ms_per_step": 1e3 * el / K,
                         "gmres_iters_per_step": (gs.iters - it0) / K,
                         "rel_diff_vs_tau_gpu": diff, "status": gs.status}
        gs.close()

    # ---- FP64 form with graph replay of the Arnoldi steps (no kernel timing)
    if not args.no_graphs:
        gg = Stepper(insts, graphs=True)
        gg.run(W)
        it0 = gg.iters
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gg.run(K)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        same = all(bool(torch.equal(a, b)) for a, b in zip(gg.us, u64))
        out["graph_replay"] = {"value": K / el, "unit": "time-steps/s", "ms_per_step": 1e3 * el / K,
                               "gmres_iters_per_step": (gg.iters - it0) / K,
                               "bitwise_equal_to_direct": same, "status": gg.status}
        gg.close()

    if not args.no_cpu_baseline:
        if len(insts) > 1:
            out["cpu_baseline"] = cpu_baseline_batch(insts, args.cpu_instances)
        else:
            # bounded samples: the 3-D workloads take seconds (255^3) to a minute
            # (511^3) per oracle step on the host
            steps = {"C3": 2, "C5": 1}.get(args.workload, args.cpu_steps)
            small = args.workload in ("C1", "C2")
            out["cpu_baseline"] = cpu_baseline(inst, steps, tight=small,
                                               one_thread_steps=1 if small else 0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
