"""Benchmark of the Krylov phi combination on one MI355X.

One timed step = one full phi_combo call (stage, hybrid low-synchronisation
Arnoldi, small Pade exponential, on-device substep controller, combine) on the
Allen-Cahn Jacobian workload: A = 0.01 Lap + diag(1 - 3u^2) on a 1024 x 1024
periodic grid (N = 1,048,576), p = 2, h = 0.1, tol = 1e-8, m <= 64, H-GSMGS.
The whole call is one cooperative kernel launch.

Printed: one JSON line with Arnoldi steps/s (whole job), phi_combo/s, the
roofline of the persistent kernel (algorithmic HBM bytes per launch over its
average duration, HIP events on the launch stream), a fixed-m microbenchmark
(one substep of exactly 64 Arnoldi steps) with its error against the float64
CPU oracle, and the oracle's own speed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Arnoldi steps/s and phi_combo/s at N=1M,m=64; HBM GB/s vs peak; err vs FP64"
KERNEL = "kp::k_run<double>"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_run_allen_cahn_1024_traffic.txt")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_batch_uneven_512_traffic.txt")
CSRC = os.path.join(ROOT, "paper_2410_14917_amd", "csrc")


def kernel_source_hash():
    """sha256 over the kernel sources (the counters are void once they change)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(path=None, key="hbm_bytes_per_launch"):
    """HBM bytes per launch of the persistent kernel (or, with the batched
    summary, per batched call) from the committed PMC summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by the factor the same counter gives for a plain
    device copy of known size), or None when the summary is missing or was
    taken on other kernel sources."""
    try:
        kv = {}
        with open(path or TRAFFIC_FILE) as f:
            for line in f:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != kernel_source_hash():
            return None
        return float(kv[key])
    except (OSError, KeyError, ValueError):
        return None


def basis_bytes_per_call(schedule, p, c, n, s):
    """Algorithmic HBM bytes of one call with basis elements of s bytes (the
    state vector, B, the fields and out stay float64): per Arnoldi step jj the
    matvec reads x_j (s), p columns of B and c fields (8 each) and jj basis
    columns (s), writes w (s); the update reads w and jj+1 columns (s) and
    writes x_{j+1} (s); combine reads m columns (s) and writes u (8); stage
    reads p+1 columns and writes u (8); the last combine writes out (8)."""
    total = 8 * ((p + 1) + 1)
    for _, m in schedule:
        total += sum(s * (2 * jj + 5) + 8 * (p + c) for jj in range(m)) + s + s * m + 8
    return (total + 8) * n


def vectors_per_call(schedule, p, c):
    """Algorithmic vector passes (each N float64) of one phi_combo call.

    Arnoldi step jj (0-based): matvec+dots reads x_j, p columns of B, c field
    vectors and jj basis columns, writes w (the first step also writes column
    0); update reads w and jj+1 columns, writes x_{j+1}:  2 jj + p + c + 5.
    Combine: m reads + 1 write.  Stage: p+1 reads + 1 write.  The last
    combine also writes out."""
    total = (p + 1) + 1
    for _, m in schedule:
        total += sum(2 * jj + p + c + 5 for jj in range(m)) + 1 + (m + 1)
    return total + 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--orth", default="h-gsmgs")
    ap.add_argument("--basis", default="f64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fixed", action="store_true", help="skip the fixed-m microbenchmark")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32-basis leg (2 x 2048^2 Brusselator)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint leg (advection-diffusion 1024^2, least-squares loss)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched leg (512 uneven advection-diffusion-reaction problems)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    import paper_2410_14917_amd as kp

    dev = "cuda:0"
    torch.cuda.set_device(0)
    pr = W.config2(side=args.side)
    N, p = pr.op.n, pr.p
    c_fields = 1                                   # Allen-Cahn reads u
    op = kp.Operator.from_host(pr.op, device=dev)
    B = torch.as_tensor(np.ascontiguousarray(pr.B.T), device=dev)
    out = torch.empty(N, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    # ---- adaptive phi_combo: the timed steps --------------------------------
    ctx = kp.Context(orth=args.orth, basis=args.basis, stream=stream)
    info = None
    for _ in range(args.warmup):
        _, info = ctx.phi_combo(op, B, pr.h, tol=pr.tol, m_max=pr.m_max, out=out, info=True)
    sched = ctx.schedule()
    _, info = ctx.phi_combo(op, B, pr.h, tol=pr.tol, m_max=pr.m_max, out=out, info=True)
    sched = ctx.schedule()
    print(f"[bench] adaptive call: {info}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev0[k].record(stream)
        ctx.phi_combo(op, B, pr.h, tol=pr.tol, m_max=pr.m_max, out=out)
        ev1[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
    avg_ms = float(np.mean(launch_ms))
    steps_per_call = info["arnoldi_steps"]
    value = steps_per_call * args.steps / wall
    vec = vectors_per_call(sched, p, c_fields)
    bytes_per_call = vec * 8.0 * N
    achieved = bytes_per_call / (avg_ms * 1e-3) / 1e9
    print(f"[bench] {args.steps} calls: wall {wall:.3f}s, event avg {avg_ms:.3f} ms/launch, "
          f"{vec} vector passes/call", file=sys.stderr, flush=True)

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Arnoldi steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.basis == "f64" else "f32-basis/f64",
        "data": "synthetic",
        "config": {"workload": f"Allen-Cahn Jacobian 0.01*Lap+diag(1-3u^2), {args.side}x{args.side} "
                               f"periodic, N={N}, p={p}, h={pr.h}, tol={pr.tol}, m<=64 adaptive, "
                               f"{args.orth}, one persistent launch per call",
                   "N": N, "p": p, "m_max": pr.m_max, "tol": pr.tol, "h": pr.h,
                   "orth": args.orth, "basis": args.basis, "seed": pr.seed},
        "phi_combo_per_s": round(args.steps / wall, 4),
        "per_call": {"substeps": info["substeps"], "rejected": info["rejected"],
                     "arnoldi_steps": steps_per_call, "expm_evals": info["expm_evals"],
                     "n_fallback": info["n_fallback"], "status": info["status"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(), "kernel": KERNEL,
                     "bytes_per_launch": bytes_per_call, "avg_launch_ms": round(avg_ms, 4)},
    }

    if args.calib_copy:
        # a plain elementwise kernel of known size: dst = -src reads 1 GiB and
        # writes 1 GiB (the HBM-counter calibration of the profiles)
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # ---- fixed m = 64: one substep, Arnoldi throughput + error vs oracle ------
    y_fixed = None
    if not args.no_fixed:
        fctx = kp.Context(orth=args.orth, basis=args.basis, fixed_m=64, fixed_substeps=1,
                          stream=stream)
        for _ in range(max(1, args.warmup)):
            fctx.phi_combo(op, B, pr.h, m_max=64, out=out)
        nrep = max(3, args.steps)
        e0 = [torch.cuda.Event(enable_timing=True) for _ in range(nrep)]
        e1 = [torch.cuda.Event(enable_timing=True) for _ in range(nrep)]
        torch.cuda.synchronize()
        for k in range(nrep):
            e0[k].record(stream)
            fctx.phi_combo(op, B, pr.h, m_max=64, out=out)
            e1[k].record(stream)
        torch.cuda.synchronize()
        fms = float(np.mean([a.elapsed_time(b) for a, b in zip(e0, e1)]))
        fvec = vectors_per_call([(pr.h, 64)], p, c_fields)
        y_fixed = out.cpu().numpy().copy()
        result["fixed_m64"] = {
            "ms_per_substep": round(fms, 4),
            "arnoldi_steps_per_s": round(64 / (fms * 1e-3), 1),
            "achieved_GBps": round(fvec * 8.0 * N / (fms * 1e-3) / 1e9, 1),
            "frac": round(fvec * 8.0 * N / (fms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_launch": fvec * 8.0 * N,
        }
        fctx.close()
    ctx.close()

    # ---- FP32 basis against the FP64 path (2 x 2048^2 Brusselator) ----------
    if not args.no_fp32:
        del B, out
        torch.cuda.empty_cache()
        p3 = W.config3()
        op3 = kp.Operator.from_host(p3.op, device=dev)
        B3 = torch.as_tensor(np.ascontiguousarray(p3.B.T), device=dev)
        o3 = torch.empty(p3.op.n, dtype=torch.float64, device=dev)
        leg = {"workload": f"Brusselator Jacobian (A=1, B=3, D=0.02/0.01), 2x2048^2, "
                           f"N={p3.op.n}, p={p3.p}, h={p3.h}, tol={p3.tol}, m<=64 adaptive"}
        ys = {}
        for basis, sz in (("f64", 8), ("f32", 4)):
            c3 = kp.Context(orth=args.orth, basis=basis, stream=stream)
            _, inf3 = c3.phi_combo(op3, B3, p3.h, tol=p3.tol, m_max=p3.m_max, out=o3, info=True)
            sch3 = c3.schedule()
            nrep = 3
            e0 = [torch.cuda.Event(enable_timing=True) for _ in range(nrep)]
            e1 = [torch.cuda.Event(enable_timing=True) for _ in range(nrep)]
            torch.cuda.synchronize()
            for k in range(nrep):
                e0[k].record(stream)
                c3.phi_combo(op3, B3, p3.h, tol=p3.tol, m_max=p3.m_max, out=o3)
                e1[k].record(stream)
            torch.cuda.synchronize()
            ms3 = float(np.mean([a.elapsed_time(b) for a, b in zip(e0, e1)]))
            ys[basis] = o3.double().cpu().numpy().copy()
            byts = basis_bytes_per_call(sch3, p3.p, 2, p3.op.n, sz)
            leg[basis] = {"ms_per_call": round(ms3, 3), "arnoldi_steps": inf3["arnoldi_steps"],
                          "substeps": inf3["substeps"], "rejected": inf3["rejected"],
                          "arnoldi_steps_per_s": round(inf3["arnoldi_steps"] / (ms3 * 1e-3), 1),
                          "modelled_GBps": round(byts / (ms3 * 1e-3) / 1e9, 1),
                          "frac": round(byts / (ms3 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "status": inf3["status"]}
            c3.close()
            print(f"[bench] fp32 leg {basis}: {leg[basis]}", file=sys.stderr, flush=True)
        leg["rel_err_f32_vs_f64"] = float(np.linalg.norm(ys["f32"] - ys["f64"]) /
                                          np.linalg.norm(ys["f64"]))
        leg["speedup_f32_over_f64"] = round(leg["f64"]["ms_per_call"] / leg["f32"]["ms_per_call"], 3)
        result["fp32_basis"] = leg
        del B3, o3

    # ---- adjoint: loss ||phi_combo - y||^2, gradients in B and nu ------------
    # (the nu-gradient of this constant-coefficient operator is one plain solve
    # with p + 2 right-hand sides: the direction commutes with A)
    if not args.no_adjoint:
        from paper_2410_14917_amd import autograd as kpa
        torch.cuda.empty_cache()
        p5 = W.config5()
        op5 = kp.Operator.from_host(p5.op, device=dev)
        B5 = torch.as_tensor(np.ascontiguousarray(p5.B.T), device=dev).requires_grad_(True)
        nu5 = torch.tensor(p5.op.nu, dtype=torch.float64, device=dev, requires_grad=True)
        y5 = torch.as_tensor(p5.y, device=dev)

        def loss5():
            return ((kpa.phi_combo(B5, nu5, op5, p5.h, tol=p5.tol, m_max=p5.m_max,
                                   orth=args.orth) - y5) ** 2).sum()

        def timed(fn, nrep=3):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(nrep):
                fn()
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - t) / nrep

        def fwd():
            with torch.no_grad():
                loss5()

        def fwd_bwd():
            B5.grad = nu5.grad = None
            loss5().backward()

        ms_f, ms_fb = timed(fwd), timed(fwd_bwd)
        # the solves one by one (forward, the p+1 transposed solves, the tangent)
        c5 = kp.Context(orth=args.orth, stream=stream)
        opt5 = kp.Operator(op5.kind, op5.nx, op5.ny, nu=op5.nu, ax=op5.ax, ay=op5.ay,
                           react=op5.react, transpose=True, dx=op5.dx, dy=op5.dy)
        dop5 = kp.Operator(op5.kind, op5.nx, op5.ny, nu=1.0, dx=op5.dx, dy=op5.dy)
        Bd = B5.detach()
        g5 = torch.randn(p5.op.n, dtype=torch.float64, device=dev)
        solves = {}
        _, inf = c5.phi_combo(op5, Bd, p5.h, tol=p5.tol, m_max=p5.m_max, info=True)
        solves["forward"] = (timed(lambda: c5.phi_combo(op5, Bd, p5.h, tol=p5.tol,
                                                        m_max=p5.m_max)), inf)
        for k in range(p5.p + 1):
            Bk = torch.zeros((k + 1, p5.op.n), dtype=torch.float64, device=dev)
            Bk[k] = g5
            _, inf = c5.phi_combo(opt5, Bk, p5.h, tol=p5.tol, m_max=p5.m_max, info=True)
            solves[f"transposed_k{k}"] = (timed(lambda: c5.phi_combo(
                opt5, Bk, p5.h, tol=p5.tol, m_max=p5.m_max)), inf)
        _, _, inf = c5.phi_combo_backward(op5, Bd, p5.h, g5, tol=p5.tol, m_max=p5.m_max,
                                          want_B=False, coefs=("nu",), info=True)
        solves["nu_gradient"] = (timed(lambda: c5.phi_combo_backward(
            op5, Bd, p5.h, g5, tol=p5.tol, m_max=p5.m_max, want_B=False, coefs=("nu",))), inf)
        _, _, inf = c5.phi_combo_tangent(op5, dop5, Bd, p5.h, tol=p5.tol, m_max=p5.m_max,
                                         info=True)
        solves["tangent_for_reference"] = (timed(lambda: c5.phi_combo_tangent(
            op5, dop5, Bd, p5.h, tol=p5.tol, m_max=p5.m_max)), inf)
        c5.close()
        kpa.release_contexts()
        result["adjoint"] = {
            "workload": f"advection-diffusion nu={p5.op.nu}, a=({p5.op.ax},{p5.op.ay}), "
                        f"{p5.op.nx}x{p5.op.ny}, p={p5.p}, h={p5.h}, tol={p5.tol}, "
                        f"loss ||phi_combo - y||^2, gradients in b_0..b_{p5.p} and nu",
            "forward_ms": round(ms_f, 3), "forward_backward_ms": round(ms_fb, 3),
            "backward_over_forward": round((ms_fb - ms_f) / ms_f, 3),
            "solves": {k: {"ms": round(v[0], 3), "arnoldi_steps": v[1]["arnoldi_steps"],
                           "substeps": v[1]["substeps"], "status": v[1]["status"]}
                       for k, v in solves.items()},
        }
        print(f"[bench] adjoint leg: {result['adjoint']}", file=sys.stderr, flush=True)
        del B5, y5

    # ---- batched uneven problems: one launch vs one call per problem --------
    if not args.no_batch:
        torch.cuda.empty_cache()
        probs4 = W.config4()
        ops4 = [kp.Operator.from_host(q.op, device=dev) for q in probs4]
        Bs4 = [torch.as_tensor(np.ascontiguousarray(q.B.T), device=dev) for q in probs4]
        hs4 = [q.h for q in probs4]
        outs4 = [torch.empty(q.op.n, dtype=torch.float64, device=dev) for q in probs4]
        tol4, mm4 = probs4[0].tol, probs4[0].m_max
        c4 = kp.Context(orth=args.orth, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, inf4 = c4.phi_combo_batched(ops4, Bs4, hs4, tol=tol4, m_max=mm4, outs=outs4, info=True)
        first_s = time.perf_counter() - t0
        nrep = 3
        e0 = [torch.cuda.Event(enable_timing=True) for _ in range(nrep)]
        e1 = [torch.cuda.Event(enable_timing=True) for _ in range(nrep)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(nrep):
            e0[k].record(stream)
            c4.phi_combo_batched(ops4, Bs4, hs4, tol=tol4, m_max=mm4, outs=outs4)
            e1[k].record(stream)
        torch.cuda.synchronize()
        batch_wall = (time.perf_counter() - t0) / nrep
        batch_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(e0, e1)]))
        steps4 = sum(r["arnoldi_steps"] for r in inf4)
        bytes4 = sum(vectors_per_call(c4.batch_schedule(i), q.p, 0) * 8.0 * q.op.n
                     for i, q in enumerate(probs4))
        _, _, plan_s, work_s = kp.batch_plan([q.op for q in probs4], [q.p for q in probs4], hs4,
                                             m_max=mm4, n_wg=256)
        # one plain call per problem (the largest first, so the workspace is
        # allocated before the timed loop)
        big = max(range(len(probs4)), key=lambda i: probs4[i].op.n)
        c4.phi_combo(ops4[big], Bs4[big], hs4[big], tol=tol4, m_max=mm4, out=outs4[big])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(len(probs4)):
            c4.phi_combo(ops4[i], Bs4[i], hs4[i], tol=tol4, m_max=mm4, out=outs4[i])
        torch.cuda.synchronize()
        seq_s = time.perf_counter() - t0
        c4.close()
        traffic4 = measured_traffic(BATCH_TRAFFIC_FILE, "hbm_bytes_per_call")
        result["batched"] = {
            "workload": f"{len(probs4)} advection-diffusion-reaction problems, sides U{{32..512}}, "
                        f"N total {sum(q.op.n for q in probs4)}, nu logU[1e-3,1e-1], r U[-1,1], "
                        f"h={hs4[0]}, p={probs4[0].p}, tol={tol4}, m<={mm4}",
            "batched_ms": round(batch_ms, 2), "batched_wall_ms": round(1e3 * batch_wall, 2),
            "first_call_s": round(first_s, 3),
            "sequential_ms": round(1e3 * seq_s, 1),
            "speedup_vs_sequential": round(1e3 * seq_s / batch_ms, 2),
            "arnoldi_steps": steps4,
            "arnoldi_steps_per_s": round(steps4 / (batch_ms * 1e-3), 1),
            "modelled_GBps": round(bytes4 / (batch_ms * 1e-3) / 1e9, 1),
            "frac": round(bytes4 / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": traffic4,
            "measured_GBps": (round(traffic4 / (batch_ms * 1e-3) / 1e9, 1)
                              if traffic4 else None),
            "plan_makespan_ms": round(1e3 * plan_s, 1),
            "plan_balanced_ms": round(1e3 * work_s / 256, 1),
            "status_ok": all(r["status"] == 0 for r in inf4),
        }
        print(f"[bench] batched leg: {result['batched']}", file=sys.stderr, flush=True)
        del Bs4, outs4

    # ---- CPU oracle baseline (bounded sample) --------------------------------
    if not args.no_cpu:
        from oracle import krylov
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        except Exception:
            cores = 1
        reps = 5   # ~10-15 s of oracle work on the host cores
        t0 = time.perf_counter()
        for _ in range(reps):
            ref, _ = krylov.phi_combo(pr.op, pr.B, pr.h, p, fixed_m=64, fixed_substeps=1,
                                      m_max=64)
        cw = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": round(64 * reps / cw, 3), "unit": "Arnoldi steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{reps} x one substep of 64 MGS Arnoldi steps + Taylor expm + combine "
                      f"on the same N={N} workload (numpy float64), {cw:.1f} s"}
        if y_fixed is not None:
            err = float(np.linalg.norm(y_fixed - ref) / np.linalg.norm(ref))
            result["fixed_m64"]["rel_err_vs_oracle"] = err
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
