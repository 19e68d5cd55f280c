"""Benchmark of the fine-grid hot path on one MI355X.

Workload (the headline single-GPU configuration): 2-D convection-diffusion
-u_xx - u_yy + 100 u_x on the unit square, 5-point centred differences, fine
grid 1023 x 1023 (n = 1,046,529), coarse grid 511 x 511, b ~ N(0,1) (seed 2).
Setup (untimed, reported separately): GMRES-DR(80,30) on the coarse grid until
30 harmonic Ritz pairs have relative residual <= 1e-8, prolongation and
orthonormalisation of the 30 vectors, H = V^T A V.  A step is one fine solve,
BiCGStab(20)-Proj(30) in float64 from the prolongated coarse solution to true
relative residual ||b - A x|| / ||b|| <= 1e-8, with every input already in
device memory.

Prints one JSON line.  `value` is seconds per fine solve (lower is better).
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

METRIC = "fine-solve time to rel.resid 1e-8 (s) + stencil HBM GB/s; FP32/batched vs FP64"
HBM_PEAK_GBS = 8000.0


def log(*m):
    print("[bench]", *m, file=sys.stderr, flush=True)


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle CPU sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--solve-only", action="store_true",
                    help="setup, warm-up and timed solves only (for hardware-counter runs)")
    ap.add_argument("--workload", choices=("2d", "3d", "mg"), default="2d",
                    help="with --solve-only: 2d = 1023^2 FP64 (the headline), 3d = 255^3 FP32 inner + FP64 "
                         "refinement, mg = the multigrid preconditioner of the kappa = 100 Helmholtz workload "
                         "alone (--steps applications)")
    ap.add_argument("--method", choices=("bicgstab", "idr", "gmres"), default="bicgstab",
                    help="with --solve-only --workload 2d: the fine solver (idr = IDR(4), gmres = GMRES(50); "
                         "FP64)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 512 MiB device buffer three times (counter scale of a plain copy)")
    return ap.parse_args()


def kernel_hash():
    h = hashlib.sha256()
    for f in ("step_kernel.h", "kernels_step2d.hip", "march3d.h", "device_common.h", "tgdk_shared.h"):
        with open(os.path.join(ROOT, "paper_2005_03070_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles():
    """HBM bytes per launch of the step kernel from the committed counter
    summary (FETCH_SIZE scaled by the copy-kernel factor, plus WRITE_SIZE), if
    it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "k_step_f64_1023sq_counters.txt")
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if ":" in line and not line.startswith((" ", "#", "`")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU design is "
              "documented but not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if a.solve_only and a.workload == "3d":
        import paper_2005_03070_amd as tg
        import workloads as W
        c3 = W.CONFIGS["C3"]
        op3 = tg.Operator.const_cd(c3["n"], c3["beta"])
        b3 = torch.tensor(W.rhs(op3.n, c3["seed"]), device="cuda:0")
        s3 = tg.TwoGridSolver(op3, m=c3["m"], k=c3["k"], nev=c3["nev"], rtolev=1e-4, maxcyc=12,
                              store=torch.float32)
        x03 = s3.setup(b3)
        kw = dict(x0=x03, precision="fp32_ir", rtol=c3["rtol"], ncyc=c3["ncyc"], max_extra=40)
        for _ in range(a.warmup):
            s3.solve(b3, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            x3, r3 = s3.solve(b3, **kw)
        torch.cuda.synchronize()
        log(f"255^3 fp32_ir: {(time.perf_counter() - t0) / a.steps * 1e3:.1f} ms/solve, mvps {r3[0].mvp_inner}, "
            f"relres {r3[0].relres_true:.2e}")
        return

    if a.solve_only and a.workload == "mg":
        import paper_2005_03070_amd as tg
        import workloads as W
        c5 = W.CONFIGS["H2"]
        shifted = tg.Operator.const_cd(c5["n"], c5["beta"], sigma=-c5["sigma"])
        mg = tg.Multigrid(shifted, cycles=c5["mg_cycles"], nu=c5["mg_nu"])
        b5 = torch.tensor(W.rhs(shifted.n, c5["seed"]), device="cuda:0")
        for _ in range(a.warmup):
            mg.apply(b5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            mg.apply(b5)
        torch.cuda.synchronize()
        log(f"multigrid {c5['n'][0]}^2, {mg.levels} levels, {c5['mg_cycles']} V-cycles: "
            f"{(time.perf_counter() - t0) / a.steps * 1e3:.3f} ms per application")
        return

    if a.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {src.numel() * 8 / 2**20:.0f} MiB three times")
        return

    import paper_2005_03070_amd as tg
    from paper_2005_03070_amd import _lib as L
    from paper_2005_03070_amd.api import context
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    c = W.CONFIGS["C2"]
    nx, ny = c["n"]
    n = nx * ny
    b_np = W.rhs(n, c["seed"])
    b = torch.tensor(b_np, device=dev)
    op = tg.Operator.const_cd((nx, ny), c["beta"])
    ctx, _ = context(dev)

    # ---------------------------------------------------------------- setup
    t0 = time.perf_counter()
    coarse = op.coarsen()
    bc = tg.restrict(op, coarse, b)
    xc, cspace, srep = tg.coarse_setup(coarse, bc, c["m"], c["k"], c["nev"], c["rtolev"], 1e-8, 300)
    space = tg.defl_prolongate(cspace, op)
    x0 = tg.prolongate(coarse, op, xc)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup {setup_s:.2f}s: GMRES-DR cycles={srep.cycles} nconv={srep.nconv} mvps={srep.mvps}")

    def fine_solve(**kw):
        kw.setdefault("ncyc", c["ncyc"])
        kw.setdefault("rtol", c["rtol"])
        kw.setdefault("defl", space)
        return tg.solve(op, b, x0=x0, **kw)

    if a.solve_only and a.method == "idr":
        shadow = torch.tensor(W.shadow_draw(n, 4, 5), device=dev)
        for _ in range(a.warmup):
            tg.solve_idr(op, b, s=4, shadow=shadow, x0=x0, defl=space, ncyc=c["ncyc"], rtol=c["rtol"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            xi, ri = tg.solve_idr(op, b, s=4, shadow=shadow, x0=x0, defl=space, ncyc=c["ncyc"], rtol=c["rtol"])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        log(f"fp64 IDR(4)(20)-Proj(30): {dt*1e3:.1f} ms/solve, mvps {ri.mvp_inner}, cycles {ri.cycles}, "
            f"relres {ri.relres_true:.2e}, {dt*1e6/max(ri.mvp_inner, 1):.1f} us per inner mvp")
        return

    if a.solve_only and a.method == "gmres":
        for _ in range(a.warmup):
            fine_solve(method="gmres", m3=c["m3"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            xg, rg = fine_solve(method="gmres", m3=c["m3"])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        log(f"fp64 GMRES(50)-Proj(30): {dt*1e3:.1f} ms/solve, mvps {rg[0].mvp_inner}, cycles {rg[0].cycles}, "
            f"relres {rg[0].relres_true:.2e}, {dt*1e6/max(rg[0].mvp_inner, 1):.1f} us per inner mvp")
        return

    def true_relres(x):
        r = b - op.apply(x)
        return float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))

    # ------------------------------------------------------- headline steps
    for _ in range(a.warmup):
        fine_solve()
    torch.cuda.synchronize()
    times = []
    reps = None
    t_start = time.perf_counter()
    for _ in range(a.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, reps = fine_solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    total = time.perf_counter() - t_start
    rr = true_relres(x)
    assert reps[0].status == 0 and rr <= c["rtol"], (reps[0].status_name, rr)
    sec = total / a.steps
    log(f"fp64 BiCGStab(20)-Proj(30): {sec*1e3:.1f} ms/solve, mvps {reps[0].mvp_inner}, relres {rr:.2e}")
    head = reps[0]
    if a.solve_only:
        return

    # ------------------------------------------- live kernel timing (roofline)
    # One more solve with the library's measurement on: every step launch
    # stamps its first workgroup start and last workgroup end on the device
    # wall clock and logs what it did (phase A, phase B, cycle boundary, ...);
    # each action has its own algorithmic byte count.  (A HIP event pair around
    # every launch would add about 4 us to a 20 us launch.)  HIP events on the
    # solve's stream bracket the whole solve, giving the share of its GPU time
    # spent inside step kernels.
    import ctypes as C
    kdefl = space.k
    w8, v8 = 8, 8  # float64 inner vectors and stored deflation vectors
    act_bytes = {  # algorithmic HBM bytes per grid point of one launch
        "A": 10 * w8,               # reads s, t, p, v, e, r^; writes r, e, p, v
        "A0": 5 * w8,               # reads r, r^; writes p, v, e
        "B": 5 * w8,                # reads r, v, r^; writes s, t
        "RES": 8 + 3 * w8 + 8 + kdefl * v8 + 8,    # reads x, e p s, b, V; writes r
        "REDUCE": 0,                # partial sums only
        "APPLY": 16 + 3 * w8 + kdefl * v8 + 16 + w8,  # reads x r, e p s, V; writes x r, r^
        "FIN": 16 + 3 * w8,         # reads x, e p s; writes x
        "FIN_A0": 16 + 3 * w8 + 5 * w8,
        "APPLYW": 8 + 3 * w8 + kdefl * v8 + 16,   # 3-D only: reads x, e p s, V; writes x, w
    }
    codes = {"A": 1, "A0": 2, "B": 3, "RES": 4, "REDUCE": 5, "APPLY": 6, "FIN": 7, "FIN_A0": 8, "APPLYW": 9}
    L.check(L.lib().tgdk_ctx_time_kernel(ctx, 1))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    fine_solve()
    ev1.record()
    torch.cuda.synchronize()
    solve_event_ms = ev0.elapsed_time(ev1)
    per_act = {}
    for name, code in codes.items():
        ms = np.zeros(1)
        cnt = np.zeros(1, dtype=np.int64)
        L.check(L.lib().tgdk_ctx_kernel_time(ctx, code, ms.ctypes.data_as(L.DP),
                                             cnt.ctypes.data_as(C.POINTER(C.c_longlong))))
        if cnt[0]:
            per_act[name] = (float(ms[0]), int(cnt[0]))
    L.check(L.lib().tgdk_ctx_time_kernel(ctx, 0))
    tot_ms = sum(v[0] for v in per_act.values())
    tot_cnt = sum(v[1] for v in per_act.values())
    tot_bytes = sum(act_bytes[k] * n * v[1] for k, v in per_act.items())
    step_us = tot_ms * 1e3 / max(tot_cnt, 1)
    step_bytes = tot_bytes / max(tot_cnt, 1)
    ach_step = tot_bytes / (tot_ms * 1e-3) / 1e9
    act_table = {k: {"launches": v[1], "avg_launch_us": v[0] * 1e3 / v[1],
                     "algorithmic_bytes_per_launch": act_bytes[k] * n,
                     "achieved_GBs": (act_bytes[k] * n / (v[0] * 1e-3 / v[1]) / 1e9) if act_bytes[k] else None}
                 for k, v in per_act.items()}
    log("step kernel: " + ", ".join(f"{k} {v['avg_launch_us']:.1f} us x{v['launches']}"
                                     + (f" {v['achieved_GBs']:.0f} GB/s" if v["achieved_GBs"] else "")
                                     for k, v in act_table.items()))
    log(f"step kernel overall: {step_us:.1f} us/launch, {ach_step:.0f} GB/s algorithmic; "
        f"{tot_ms:.1f} ms of step kernels in a {solve_event_ms:.1f} ms solve (HIP events)")

    # ------------------------------------------------------------ variants
    variants = {}
    if not a.no_variants:
        def run(name, steps, **kw):
            fine_solve(**kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                xv, rv = fine_solve(**kw)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / steps
            variants[name] = {"seconds": dt, "relres_true": true_relres(xv), "status": rv[0].status_name,
                              "cycles": rv[0].cycles, "mvp_inner": rv[0].mvp_inner,
                              "mvp_boundary": rv[0].mvp_boundary}
            log(f"{name}: {dt*1e3:.1f} ms, mvps {rv[0].mvp_inner}, relres {variants[name]['relres_true']:.2e}")

        run("fp32_inner_fp64_refinement", max(3, a.steps // 2), precision="fp32_ir")
        run("gmres50_proj30_fp64", 2, method="gmres", m3=c["m3"])

        # IDR(4)(20)-Proj(30): IDR(s) in place of BiCGStab in the same cycles
        def run_idr(name, steps, **kw):
            f = lambda: tg.solve_idr(op, b, s=4, x0=x0, defl=space, ncyc=c["ncyc"], rtol=c["rtol"], **kw)
            f()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                xv, rv = f()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / steps
            variants[name] = {"seconds": dt, "relres_true": true_relres(xv), "status": rv.status_name,
                              "cycles": rv.cycles, "mvp_inner": rv.mvp_inner, "mvp_boundary": rv.mvp_boundary,
                              "us_per_inner_mvp": dt * 1e6 / max(rv.mvp_inner, 1)}
            log(f"{name}: {dt*1e3:.1f} ms, mvps {rv.mvp_inner}, relres {variants[name]['relres_true']:.2e}")

        run_idr("idr4_proj30_fp64", 2)

        # phase 2: Arnoldi-E(80,30) on the moved vectors until the 24 leading
        # pairs are below 1e-4 (the paper's Table 5.1 improves until its first
        # 80 are below 1e-3), at most 40 cycles; then the same fine solve
        t = time.perf_counter()
        space_imp, arep = space.improve(m=c["m"], nev=c["nev"], tol=1e-4, maxcyc=40)
        torch.cuda.synchronize()
        imp_s = time.perf_counter() - t
        log(f"Arnoldi-E({c['m']},{c['k']}): {arep['cycles']} cycles, {arep['mvps']} mvps, {imp_s*1e3:.0f} ms; "
            f"max eigen-residual of the {c['nev']} leading pairs {arep['eigres_start'].max():.1e} -> "
            f"{arep['eigres'][:c['nev']].max():.1e}")
        run("bicgstab20_proj30_after_arnoldie_fp64", 2, defl=space_imp)
        variants["bicgstab20_proj30_after_arnoldie_fp64"]["arnoldie"] = {
            "seconds": imp_s, "cycles": arep["cycles"], "mvps": arep["mvps"], "nconv": arep["nconv"],
            "max_eigres_start": float(arep["eigres_start"].max()),
            "max_eigres_end": float(arep["eigres"][:c["nev"]].max())}
        del space_imp

        # MinRes projection (H = (AV)^T AV, c = (AV)^T r) on the same V
        space_minres = space.minres()
        run("bicgstab20_proj30_minres_fp64", 2, defl=space_minres)
        # variable restarting (Sec. 4.3): GMRES cycle j as long as the headline
        # BiCGStab's cycle j (capped at 128), and seeded random lengths 1..100
        lens_b = [min(max(v, 1), 128) for v in head.cycle_mvps]
        run("gmres_restarted_as_bicgstab_proj30_fp64", 1, method="gmres", m3=128, cycle_lengths=lens_b)
        variants["gmres_restarted_as_bicgstab_proj30_fp64"]["cycle_lengths"] = lens_b
        lens_r = [int(v) for v in np.random.default_rng(9).integers(1, 101, size=200)]
        run("gmres_random_lengths_1to100_proj30_fp64", 1, method="gmres", m3=100, cycle_lengths=lens_r)
        del space_minres
        # no deflation, from zero: the restarted BiCGStab baseline
        t = time.perf_counter()
        x_nd, r_nd = tg.solve(op, b, rtol=c["rtol"], ncyc=c["ncyc"], max_extra=40)
        torch.cuda.synchronize()
        variants["bicgstab20_no_deflation_fp64"] = {
            "seconds": time.perf_counter() - t, "relres_true": true_relres(x_nd), "status": r_nd[0].status_name,
            "cycles": r_nd[0].cycles, "mvp_inner": r_nd[0].mvp_inner}

    # --------------------------- the other workloads: 3-D, batched right-hand sides
    workloads = {}
    if not a.no_variants:
        def act_times(ctx_):
            out = {}
            for name, code in codes.items():
                ms = np.zeros(1)
                cnt = np.zeros(1, dtype=np.int64)
                L.check(L.lib().tgdk_ctx_kernel_time(ctx_, code, ms.ctypes.data_as(L.DP),
                                                     cnt.ctypes.data_as(C.POINTER(C.c_longlong))))
                if cnt[0]:
                    out[name] = (float(ms[0]) * 1e3 / int(cnt[0]), int(cnt[0]))
            return out

        def timed(fn, reps=2):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                res = fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps, res

        # 3-D: 255^3, 40+ vectors stored in float32, FP32 inner + FP64 refinement vs FP64
        c3 = W.CONFIGS["C3"]
        op3 = tg.Operator.const_cd(c3["n"], c3["beta"])
        b3 = torch.tensor(W.rhs(op3.n, c3["seed"]), device=dev)
        t = time.perf_counter()
        s3 = tg.TwoGridSolver(op3, m=c3["m"], k=c3["k"], nev=c3["nev"], rtolev=1e-4, maxcyc=12, store=torch.float32)
        x03 = s3.setup(b3)
        torch.cuda.synchronize()
        w3 = {"setup_seconds": time.perf_counter() - t, "k": s3.defl.k}
        for prec in ("fp64", "fp32_ir"):
            kw = dict(x0=x03, precision=prec, rtol=c3["rtol"], ncyc=c3["ncyc"], max_extra=40)
            sec3, (x3, r3) = timed(lambda: s3.solve(b3, **kw))
            L.check(L.lib().tgdk_ctx_time_kernel(ctx, 1))
            s3.solve(b3, **kw)
            acts = act_times(ctx)
            L.check(L.lib().tgdk_ctx_time_kernel(ctx, 0))
            wv = 4 if prec == "fp32_ir" else 8
            per = {k: {"avg_launch_us": us, "launches": cnt,
                       "achieved_GBs": ({"A": 10, "B": 5, "A0": 5}[k] * wv * op3.n / (us * 1e-6) / 1e9)
                       if k in ("A", "B", "A0") else None}
                   for k, (us, cnt) in acts.items()}
            w3[prec] = {"seconds": sec3, "mvp_inner": r3[0].mvp_inner, "cycles": r3[0].cycles,
                        "relres_true": r3[0].relres_true, "status": r3[0].status_name, "step_by_action": per}
            log(f"255^3 {prec}: {sec3*1e3:.1f} ms, mvps {r3[0].mvp_inner}, relres {r3[0].relres_true:.2e}; "
                + ", ".join(f"{k} {v['avg_launch_us']:.0f} us" + (f" {v['achieved_GBs']:.0f} GB/s" if v["achieved_GBs"] else "")
                            for k, v in per.items()))
        workloads["3d_255cube_k40_f32V"] = w3
        del s3, x03, b3, op3
        torch.cuda.empty_cache()

        # batched: 32 right-hand sides on 511^2 sharing 30 vectors
        c4 = W.CONFIGS["C4"]
        op4 = tg.Operator.const_cd(c4["n"], c4["beta"])
        B4 = torch.tensor(W.rhs_block(op4.n, c4["seeds"]).T.copy(), device=dev)
        s4 = tg.TwoGridSolver(op4, m=c4["m"], k=c4["k"], nev=c4["nev"], rtolev=1e-6, maxcyc=60)
        s4.setup(B4[0].contiguous())
        w4 = {}
        for prec in ("fp64", "fp32_ir"):
            secb, (X4, r4) = timed(lambda: s4.solve(B4, precision=prec), reps=1)
            ok = all(q.status == 0 for q in r4) and max(q.relres_true for q in r4) <= c4["rtol"]
            w4[f"batched32_{prec}_seconds"] = secb
            w4[f"batched32_{prec}_all_converged"] = ok
            log(f"511^2 x 32 RHS batched {prec}: {secb*1e3:.1f} ms (all converged: {ok})")
        seqs, _ = timed(lambda: [s4.solve(B4[j].contiguous(), precision="fp64") for j in range(32)], reps=1)
        w4["sequential32_fp64_seconds"] = seqs
        log(f"511^2 x 32 RHS one after another fp64: {seqs*1e3:.1f} ms")
        workloads["batched_32rhs_511sq_k30"] = w4
        del s4, B4, op4
        torch.cuda.empty_cache()

        # Helmholtz (indefinite): IDR(s)-Proj against the other fine solvers on
        # one moved space, and IDR(20) without deflation (capped)
        ch = W.CONFIGS["H1"]
        oph = tg.Operator.const_cd(ch["n"], ch["beta"], sigma=ch["sigma"])
        bh = torch.tensor(W.rhs(oph.n, ch["seed"]), device=dev)
        t = time.perf_counter()
        coarse_h = oph.coarsen()
        xch, csh, srh = tg.coarse_setup(coarse_h, tg.restrict(oph, coarse_h, bh), ch["m"], ch["k"], ch["nev"],
                                        ch["rtolev"], ch["rtol"], 300)
        sph = tg.defl_prolongate(csh, oph)
        x0h = tg.prolongate(coarse_h, oph, xch)
        torch.cuda.synchronize()
        wh = {"setup_seconds": time.perf_counter() - t, "gmresdr_cycles": srh.cycles, "nconv": srh.nconv,
              "k": sph.k}
        log(f"Helmholtz 511^2 kappa 25: coarse GMRES-DR({ch['m']},{ch['k']}) {srh.cycles} cycles, "
            f"{srh.nconv} converged, {wh['setup_seconds']:.2f} s")
        shadows = {sd: torch.tensor(W.shadow_draw(oph.n, sd, ch["seed"] + sd), device=dev) for sd in (4, 20)}

        def hrun(name, fn):
            sec, (xv, rv) = timed(fn, reps=1)
            rv = rv[0] if isinstance(rv, list) else rv
            rr = float(torch.linalg.vector_norm(bh - oph.apply(xv)) / torch.linalg.vector_norm(bh))
            wh[name] = {"seconds": sec, "status": rv.status_name, "cycles": rv.cycles, "mvp_inner": rv.mvp_inner,
                        "relres_true": rr}
            log(f"  {name}: {sec*1e3:.0f} ms, {rv.status_name}, {rv.cycles} cycles, mvps {rv.mvp_inner}, "
                f"relres {rr:.2e}")

        hk = dict(x0=x0h, defl=sph, rtol=ch["rtol"], ncyc=ch["ncyc"], max_extra=20)
        hrun("idr20_proj60_fp64", lambda: tg.solve_idr(oph, bh, s=20, shadow=shadows[20], **hk))
        hrun("idr4_proj60_fp64", lambda: tg.solve_idr(oph, bh, s=4, shadow=shadows[4], **hk))
        hrun("bicgstab_proj60_fp64", lambda: tg.solve(oph, bh, **hk))
        hrun("gmres100_proj60_fp64", lambda: tg.solve(oph, bh, x0=x0h, defl=sph, method="gmres", m3=100,
                                                      rtol=ch["rtol"], max_extra=150))
        t = time.perf_counter()
        sph_i, arep_h = sph.improve(m=ch["m"], nev=ch["nev"], tol=1e-4, maxcyc=20)
        torch.cuda.synchronize()
        wh["arnoldie"] = {"seconds": time.perf_counter() - t, "cycles": arep_h["cycles"], "mvps": arep_h["mvps"],
                          "nconv": arep_h["nconv"], "max_eigres_start": float(arep_h["eigres_start"].max()),
                          "max_eigres_end": float(arep_h["eigres"][:ch["nev"]].max())}
        log(f"  Arnoldi-E({ch['m']},{ch['k']}): {arep_h['cycles']} cycles, {arep_h['mvps']} mvps, "
            f"{wh['arnoldie']['seconds']*1e3:.0f} ms, eigen-residuals {wh['arnoldie']['max_eigres_start']:.1e} -> "
            f"{wh['arnoldie']['max_eigres_end']:.1e}")
        hrun("idr20_proj60_after_arnoldie_fp64", lambda: tg.solve_idr(oph, bh, s=20, shadow=shadows[20], x0=x0h,
                                                                      defl=sph_i, rtol=ch["rtol"], ncyc=ch["ncyc"],
                                                                      max_extra=20))
        del sph_i
        sph_m = sph.minres()
        hrun("idr20_proj60_minres_fp64", lambda: tg.solve_idr(oph, bh, s=20, shadow=shadows[20], x0=x0h, defl=sph_m,
                                                              rtol=ch["rtol"], ncyc=ch["ncyc"], max_extra=20))
        hrun("gmres100_proj60_minres_fp64", lambda: tg.solve(oph, bh, x0=x0h, defl=sph_m, method="gmres", m3=100,
                                                             rtol=ch["rtol"], max_extra=150))
        del sph_m
        hrun("idr20_no_deflation_10x1000", lambda: tg.solve_idr(oph, bh, s=20, shadow=shadows[20], rtol=ch["rtol"],
                                                                ncyc=10, max_extra=0, maxit_cycle=1000))
        workloads["helmholtz_511sq_kappa25_k60"] = wh
        del oph, bh, sph, csh, coarse_h, x0h, shadows
        torch.cuda.empty_cache()

        # Example 5: multigrid-preconditioned Helmholtz, kappa = 100 on 511^2
        # (each solve once: they take seconds)
        c5 = W.CONFIGS["H2"]
        kap2 = -c5["sigma"]
        op5 = tg.Operator.const_cd(c5["n"], c5["beta"], sigma=c5["sigma"])
        b5 = torch.tensor(W.rhs(op5.n, c5["seed"]), device=dev)
        t = time.perf_counter()
        mg5 = tg.Multigrid(tg.Operator.const_cd(c5["n"], c5["beta"], sigma=kap2), cycles=c5["mg_cycles"],
                           nu=c5["mg_nu"])
        coarse5 = op5.coarsen()
        mg5c = tg.Multigrid(tg.Operator.const_cd(coarse5.dims, c5["beta"], sigma=kap2), cycles=c5["mg_cycles"],
                            nu=c5["mg_nu"])
        xc5, cs5, sr5 = tg.coarse_setup(coarse5, tg.restrict(op5, coarse5, b5), c5["m"], c5["k"], c5["nev"],
                                        c5["rtolev"], c5["rtol"], 300, precond=mg5c)
        sp5 = tg.defl_prolongate(cs5, op5).precond(mg5)
        x05 = tg.prolongate(coarse5, op5, xc5)
        torch.cuda.synchronize()
        w5 = {"setup_seconds": time.perf_counter() - t, "gmresdr_cycles": sr5.cycles, "nconv": sr5.nconv,
              "k": sp5.k}
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            mg5.apply(b5)
        torch.cuda.synchronize()
        w5["mg_apply_ms"] = (time.perf_counter() - t) / 5 * 1e3
        log(f"Helmholtz 511^2 kappa 100, multigrid-preconditioned: coarse GMRES-DR({c5['m']},{c5['k']}) on A M^-1 "
            f"{sr5.cycles} cycles, {sr5.nconv} converged, {w5['setup_seconds']:.2f} s; M^-1 {w5['mg_apply_ms']:.2f} ms")
        sh5 = torch.tensor(W.shadow_draw(op5.n, c5["s"], c5["seed"] + c5["s"]), device=dev)

        def once(name, fn):
            torch.cuda.synchronize()
            t0_ = time.perf_counter()
            xv, rv = fn()
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0_
            rr = float(torch.linalg.vector_norm(b5 - op5.apply(xv)) / torch.linalg.vector_norm(b5))
            w5[name] = {"seconds": sec, "status": rv.status_name, "cycles": rv.cycles, "mvp_inner": rv.mvp_inner,
                        "relres_true": rr}
            log(f"  {name}: {sec*1e3:.0f} ms, {rv.status_name}, {rv.cycles} cycles, mvps {rv.mvp_inner}, "
                f"relres {rr:.2e}")

        once("idr5_5cyc_proj60_mg_fp64", lambda: tg.solve_idr(op5, b5, s=c5["s"], shadow=sh5, x0=x05, defl=sp5,
                                                               rtol=c5["rtol"], ncyc=c5["ncyc"], max_extra=20,
                                                               precond=mg5))
        once("idr5_mg_no_deflation_fp64", lambda: tg.solve_idr(op5, b5, s=c5["s"], shadow=sh5, x0=x05,
                                                                rtol=c5["rtol"], ncyc=c5["ncyc"], max_extra=20,
                                                                precond=mg5))
        workloads["helmholtz_mg_511sq_kappa100_k60"] = w5
        del op5, b5, mg5, mg5c, coarse5, cs5, sp5, x05, sh5
        torch.cuda.empty_cache()

    # ------------------------------------------ standalone stencil bandwidth
    def stencil_gbs(opx, dtype, rotate_bytes=2 << 30):
        es = torch.tensor([], dtype=dtype).element_size()
        per = 2 * opx.n * es
        nbuf = max(2, int(rotate_bytes // per))
        xs = [torch.randn(opx.n, dtype=dtype, device=dev) for _ in range(nbuf)]
        ys = [torch.empty_like(xs[0]) for _ in range(nbuf)]
        for i in range(nbuf):
            ys[i] = opx.apply(xs[i])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps_ = 3 * nbuf
        e0.record()
        for i in range(reps_):
            j = i % nbuf
            ys[j] = opx.apply(xs[j])
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps_
        del xs, ys
        return per / (ms * 1e-3) / 1e9, ms * 1e3

    st_c2, us_c2 = stencil_gbs(op, torch.float64)
    op3 = tg.Operator.const_cd((255, 255, 255), (50.0, 20.0, 10.0))
    st_c3, us_c3 = stencil_gbs(op3, torch.float32)
    log(f"stencil 1023^2 f64 {st_c2:.0f} GB/s ({us_c2:.1f} us); 255^3 f32 {st_c3:.0f} GB/s ({us_c3:.1f} us)")

    # -------------------------------------------------- oracle CPU baseline
    cpu = None
    if not a.no_cpu:
        from oracle import bicgstab as OB, operators as OO
        oop = OO.const_cd((nx, ny), c["beta"])
        r0 = b_np - OO.apply(oop, x0.cpu().numpy())
        t = time.perf_counter()
        iters = 0
        chunk = 20
        while time.perf_counter() - t < a.cpu_seconds:
            res = OB.bicgstab_inner(lambda z: OO.apply(oop, z), r0, 0.0, chunk)
            iters += res.iters
        dt = time.perf_counter() - t
        per_mvp = dt / (2 * iters)
        total_mvps = head.mvp_inner + head.mvp_boundary
        cpu = {"value": per_mvp * total_mvps, "unit": "s", "cores": 1, "kind": "oracle",
               "sample": (f"numpy float64 Bi-CGSTAB iterations of the oracle on the same 1023^2 operator: "
                          f"{2 * iters} mvps in {dt:.1f} s ({per_mvp * 1e3:.2f} ms per mvp with its vector ops), "
                          f"scaled to the GPU solve's {total_mvps} mvps; projection and setup not included; "
                          f"single-threaded numpy on a host with {os.cpu_count()} cores")}
        log(f"cpu oracle {per_mvp*1e3:.2f} ms/mvp -> {cpu['value']:.1f} s per solve")

    out = {
        "metric": METRIC,
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2-D conv-diff -Lap(u)+100u_x, 5-pt, fine 1023^2 (n=1,046,529), coarse 511^2, "
                               "GMRES-DR(80,30) -> 30 vectors, BiCGStab(20)-Proj(30) fp64, rtol 1e-8 true residual",
                   "n": n, "k": space.k, "ncyc": c["ncyc"], "seed": c["seed"]},
        "roofline": {"bound": "hbm", "achieved": ach_step, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach_step / HBM_PEAK_GBS, "traffic": traffic_from_profiles(),
                     "kernel": "k_step1 (BiCGStab step kernel of a one-system group: phase A / phase B / cycle boundary), f64, one solve",
                     "algorithmic_bytes_per_launch": step_bytes, "avg_launch_us": step_us,
                     "launches_timed": tot_cnt, "timing": "device wall clock per launch",
                     "step_kernel_ms": tot_ms, "solve_ms_hip_events": solve_event_ms},
        "kernels": {"step_by_action": act_table,
                    "stencil_1023sq_f64_GBs": st_c2, "stencil_255cube_f32_GBs": st_c3},
        "solve": {"relres_true": rr, "cycles": head.cycles, "mvp_inner": head.mvp_inner,
                  "mvp_boundary": head.mvp_boundary, "min_s": min(times), "max_s": max(times)},
        "setup": {"seconds": setup_s, "gmresdr_cycles": srep.cycles, "nconv": srep.nconv, "mvps": srep.mvps},
        "variants": variants,
        "workloads": workloads,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
