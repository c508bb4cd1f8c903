"""Benchmark of the batched trajectory cost + adjoint and solver on one GPU.

Workload: 32 seeds x 32 waypoints x 8 line-search candidates, 7-DOF arm with
52 collision spheres, 40 oriented cuboids (seeded synthetic inputs standing in
for the paper's datasets).  One step = one full solve: 100 L-BFGS iterations
(direction, 8-candidate cost + adjoint evaluation, noisy line search, best
tracking), replayed as hipGraphs of 25 iterations.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line: evals/s (seed x waypoint x candidate cost+gradient
evaluations per second), ms per solve batched (graph) and plain (direct
launches), the evaluation kernel's roofline figures and the FP64 reference
timed on the host cores.
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

PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0


def flops_per_eval(M, N, L, D, M_active=0):
    """Algorithmic FP32 operations of one (seed, waypoint, candidate) cost +
    gradient evaluation, counted as every pair is tested (FMA = 2, other
    operations = 1, sqrt/sin/cos = 1):
      37 per sphere-cuboid pair (box-frame transform 18, |p| - h 3, clamp 3,
         squared norm 5, inner max/min 3, add/compare 3, clearance 1),
      18 per sphere (centre), 2 x 85 per link (chain forward and again for
         the adjoint), 200 per joint (limits, stencils, smoothness, forward
         and adjoint), 300 per evaluation (pose), 70 per sphere within reach
         of a cuboid (its gradient through the joints above it; 0 here, a
         lower bound)."""
    return 37 * M * N + 18 * M + 2 * 85 * L + 200 * D + 300 + 70 * M_active


def flops_per_eval_executed(M, N, L, D, pose_at_row_fraction):
    """A closer count of what the culling kernel executes per evaluation:
    24 per pair face test (box-frame transform 18, |p|-h 3, max3 2, compare
    1), 33 per sphere (centre 18, wrench 15), 180 per link, 120 per joint,
    150 per pose evaluation (last waypoint only)."""
    return 24 * M * N + 33 * M + 180 * L + 120 * D + 150 * pose_at_row_fraction


def pct(samples):
    """median and p90 of a list of timings."""
    a = np.asarray(samples, dtype=np.float64)
    return {"median": float(np.median(a)), "p90": float(np.percentile(a, 90)), "n": int(a.size)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", choices=["eval", "solve", "copy", "large"],
                    help="profiling driver instead of the benchmark: 'eval' runs --launches "
                         "line searches of the benchmark shape (one evaluation launch each), "
                         "'solve' --launches solves of the benchmark (graph replay), "
                         "'large' one particle round and --launches line searches of the large "
                         "two-arm workload, 'copy' copies 256 MiB five times (HBM byte-counter "
                         "calibration)")
    ap.add_argument("--launches", type=int, default=10)
    ap.add_argument("--layout", type=int, choices=[0, 1, 2, 3, 4], default=None,
                    help="force the evaluation layout (0 lane per link, 1 wave per link, "
                         "2 two waves per link, 3 two slot groups per wave, 4 four slot groups "
                         "per wave) instead of the autotuner's choice")
    ap.add_argument("--slices", type=int, choices=[0, 1, 2, 4, 8, 16], default=0,
                    help="with --layout: cuboid slices (0 automatic)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the uneven-batch, inverse-kinematics, large, motion-generation and "
                         "planning measurements")
    ap.add_argument("--plan-only", action="store_true", help="only the geometric planning measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding over several "
              "GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.profile == "copy":
        return profile_copy()
    if args.profile == "large":
        return profile_large(args.launches, args.layout)
    if args.plan_only:
        print(json.dumps({"plan": bench_plan(args.warmup)}), flush=True)
        return

    import torch
    from paper_2310_17274_amd import workloads as wl
    from paper_2310_17274_amd.binding import Context

    robot, worlds, batch, meta = wl.cfg_cost_adjoint()
    robot, worlds, batch = wl.robot_f32(robot), wl.worlds_f32(worlds), wl.to_f32(batch)
    alpha = meta["alpha"]
    iters = meta["iters"]
    K = len(alpha)
    D = robot.dof
    S, T = int(batch.seeds[0]), int(batch.horizon[0])

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = Context(robot)
    ctx.mg_set_worlds(worlds)
    b = ctx.batch(batch.seeds, batch.horizon, batch.world, K_max=K, m_max=4)
    q_start = torch.as_tensor(batch.q_start, dtype=torch.float32, device=dev).contiguous()
    goal = torch.as_tensor(batch.goal.reshape(batch.n_problems, -1), dtype=torch.float32, device=dev).contiguous()
    x0 = torch.as_tensor(batch.x0.reshape(-1, D), dtype=torch.float32, device=dev).contiguous()
    x = x0.clone()
    outs = (torch.empty(b.n_seeds, dtype=torch.float32, device=dev),
            torch.empty(b.P, dtype=torch.int32, device=dev),
            torch.empty(b.P, dtype=torch.int32, device=dev))

    # launch-shape autotuner: fastest evaluation layout for this batch
    c0, g0, _ = ctx.mg_cost_grad(b, q_start, goal, x0)
    dvec = ctx.mg_lbfgs_step(b, 4, True, x0, g0)
    if args.layout is None:
        layout = layout_name(ctx.mg_autotune(b, q_start, goal, x0, dvec, alpha))
    else:
        b.mg_batch_set_layout(args.layout, args.slices)
        layout = ({2: "two_waves_per_link", 3: "two_slot_groups", 4: "four_slot_groups"}[args.layout]
                  if args.layout >= 2 else
                  ["lane_per_link", "wave_per_link"][args.layout] + "/" +
                  (str(args.slices) if args.slices else "auto"))

    if args.profile == "eval":
        return profile_eval(ctx, b, q_start, goal, x0, c0, g0, dvec, alpha, args.launches, layout)
    fused = ctx.mg_solve_fuses(b, K, 4, x0)

    def solve(use_graph, n=iters):
        x.copy_(x0)
        ctx.mg_solve(b, q_start, goal, x, n, 4, alpha, mode=1, graph_inner=25,
                     use_graph=use_graph, outputs=outs)

    if args.profile == "solve":
        for _ in range(args.launches):
            solve(True)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "solve", "solves": args.launches, "fused": fused, "layout": layout,
                          "kernel_digest": kernel_digest()}), flush=True)
        return

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        solve(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for i in range(args.steps):
        solve(True)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_batched = evs[0].elapsed_time(evs[-1]) / args.steps
    step_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # plain path: the same solve with every kernel launched directly
    for _ in range(max(1, args.warmup // 2)):
        solve(False)
    torch.cuda.synchronize()
    ev0.record(stream)
    n_plain = max(3, args.steps // 4)
    for _ in range(n_plain):
        solve(False)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_plain = ev0.elapsed_time(ev1) / n_plain

    # the evaluation kernel alone: HIP events on the launch stream around 30
    # back-to-back launches of the solve's evaluation kernel and grid
    # (32 seeds x 32 waypoints x 8 candidates, cost + adjoint)
    n_ev = 30
    ctx.mg_time_eval(b, q_start, goal, x0, dvec, alpha, launches=3)
    plain_eval_us = ctx.mg_time_eval(b, q_start, goal, x0, dvec, alpha, launches=n_ev)

    def t_solve(n, use_graph=True, reps=10):
        solve(use_graph, n)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            solve(use_graph, n)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    # With the choice folded in, each iteration after the first is one
    # launch of the evaluation kernel that also makes the previous choice:
    # its time per launch is the difference of two graph-replayed solve
    # lengths (HIP events on the launch stream), which includes the gap
    # between launches.  The same solve with separate choice launches, for
    # comparison.
    half = iters // 2
    if fused:
        eval_us = (t_solve(iters) - t_solve(half)) * 1e3 / (iters - half)
        b.mg_batch_set_fusion(False)
        ms_separate = t_solve(iters)
        b.mg_batch_set_fusion(True)
    else:
        eval_us, ms_separate = plain_eval_us, None

    best = outs[0].cpu().numpy()
    evals_per_step = S * T * K * iters
    value = evals_per_step / (ms_batched * 1e-3)
    N = int(worlds.pose.shape[0])
    fl = flops_per_eval(robot.n_spheres, N, robot.n_links, D)
    fl_x = flops_per_eval_executed(robot.n_spheres, N, robot.n_links, D, 1.0 / T)
    achieved = fl * S * T * K / (eval_us * 1e-6) / 1e12 if eval_us > 0 else 0.0

    line = {
        "metric": "seed*timestep*candidate cost+grad evals/s (full L-BFGS solve)",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batched,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"cost+adjoint solve: {S} seeds x T={T} x K={K} candidates, "
                               f"{D}-DOF arm, {robot.n_spheres} spheres, {worlds.pose.shape[0]} "
                               f"oriented cuboids, {iters} L-BFGS iterations (graph_inner 25; a graph "
                               f"holds 26 when the choice is folded into the evaluation)",
                   "seeds": S, "horizon": T, "candidates": K, "iterations": iters,
                   "spheres": robot.n_spheres, "cuboids": int(worlds.pose.shape[0])},
        "ms_per_solve_batched": ms_batched,
        "ms_per_step_pct": pct(step_ms),
        "ms_per_solve_plain": ms_plain,
        "choice_folded_into_evaluation": fused,
        "ms_per_solve_choice_separate": ms_separate,
        "speedup_batched_vs_plain": ms_plain / ms_batched,
        "wall_s_timed": wall,
        "best_cost_min": float(best.min()),
        "roofline": {"bound": "alu",
                     "kernel": ("eval_wl_fs_kernel (cost + adjoint, 8 candidates, the previous line-search "
                                "choice and L-BFGS direction folded in)" if fused else
                                ("eval_kernel" if layout.startswith("lane") else "eval_wl_kernel")
                                + " (cost + adjoint, 8 candidates)"),
                     "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(layout, fused),
                     "eval_kernel_us": eval_us,
                     "eval_kernel_timing": ("(t(%d it.) - t(%d it.)) / %d of graph-replayed solves, 10 each"
                                            % (iters, half, iters - half)) if fused else
                                           "%d back-to-back launches (mg_time_eval)" % n_ev,
                     "plain_eval_kernel_us": plain_eval_us,
                     "plain_eval_frac": fl * S * T * K / (plain_eval_us * 1e-6) / 1e12 / PEAK_FP32_TFLOPS
                     if plain_eval_us > 0 else 0.0,
                     "layout": layout,
                     "flop_per_eval": fl, "flop_count": "every pair tested (37 M N + 18 M + 170 L + 200 D + 300)",
                     "flop_per_eval_executed": fl_x,
                     "frac_executed": fl_x * S * T * K / (eval_us * 1e-6) / 1e12 / PEAK_FP32_TFLOPS
                     if eval_us > 0 else 0.0,
                     "frac_unpacked_peak": achieved / (PEAK_FP32_TFLOPS / 2),
                     "evals_per_launch": S * T * K},
    }

    if not args.no_extra:
        line["plain"] = bench_plain(args.warmup)
        line["uneven"] = bench_uneven(args.warmup)
        line["ik"] = bench_ik(args.warmup)
        line["large"] = bench_large(args.warmup)
        line["motion_gen"] = bench_motion_gen(args.warmup)
        line["plan"] = bench_plan(args.warmup)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(robot, worlds, batch, alpha, iters, args.cpu_seconds)
    print(json.dumps(line), flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "eval_kernel_cost_adjoint_32x32x8_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2310_17274_amd", "csrc", f)
                  for f in ("mg_eval.h", "mg_eval_wl.h", "mg_device.h", "mg_internal.h", "mg_solver.h")]


def kernel_digest():
    """sha256 over the evaluation kernel's sources."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def layout_name(tuned):
    """The autotuner's choice as 'lane_per_link/<slices>',
    'wave_per_link/<workgroups per 64 evaluations>', 'two_waves_per_link',
    'two_slot_groups' or 'four_slot_groups'."""
    if tuned == -8:
        return "two_waves_per_link"
    if tuned == -16:
        return "two_slot_groups"
    if tuned == -32:
        return "four_slot_groups"
    return f"lane_per_link/{tuned}" if tuned > 0 else f"wave_per_link/{-tuned}"


def measured_traffic(layout, fused=False):
    """HBM bytes per evaluation launch of `layout` (`fused`: the launch that
    also makes the previous choice, key `fused/<layout>`) from the committed
    FETCH_SIZE / WRITE_SIZE counter summary (one `hbm_bytes_per_launch[<key>]`
    line per profiled launch), or None when the kernel sources changed since
    the counters were taken, the launch was not profiled, or no summary
    exists."""
    try:
        with open(TRAFFIC_FILE) as fh:
            fields = dict((k.strip(), v.strip()) for k, v in
                          (line.split(":", 1) for line in fh if ":" in line and not line.startswith("#")))
    except OSError:
        return None
    if fields.get("source_digest") != kernel_digest():
        return None
    v = fields.get(f"hbm_bytes_per_launch[{'fused/' if fused else ''}{layout}]")
    return float(v) if v is not None else None


def _inputs(robot, batch, dev):
    import torch
    D = robot.dof
    q_start = torch.as_tensor(batch.q_start, dtype=torch.float32, device=dev).contiguous()
    goal = torch.as_tensor(batch.goal.reshape(batch.n_problems, -1), dtype=torch.float32, device=dev).contiguous()
    x0 = torch.as_tensor(batch.x0.reshape(-1, D), dtype=torch.float32, device=dev).contiguous()
    return q_start, goal, x0


def _time_solves(ctx, b, q_start, goal, x0, iters, alpha, use_graph, reps, warmup, samples=None):
    """Mean ms per call of mg_solve over `reps` calls (HIP events on the
    current stream between calls), and the last call's outputs; each call's
    ms is appended to `samples` when given."""
    import torch
    x = x0.clone()
    dev = x0.device
    outs = (torch.empty(b.n_seeds, dtype=torch.float32, device=dev),
            torch.empty(b.P, dtype=torch.int32, device=dev),
            torch.empty(b.P, dtype=torch.int32, device=dev))

    def run():
        x.copy_(x0)
        ctx.mg_solve(b, q_start, goal, x, iters, 4, alpha, mode=1, graph_inner=25,
                     use_graph=use_graph, outputs=outs)
    for _ in range(warmup):
        run()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(reps):
        run()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    if samples is not None:
        samples.extend(evs[i].elapsed_time(evs[i + 1]) for i in range(reps))
    return evs[0].elapsed_time(evs[-1]) / reps, outs


def bench_plain(warmup, reps=20):
    """The plain method on one problem: 7-DOF arm, 20 spheres, 10
    axis-aligned cuboids, 4 seeds x T=32, K=4, 100 iterations.  Latency-bound:
    ms per solve and us per iteration, graph replays against direct
    launches."""
    import torch
    from paper_2310_17274_amd import workloads as wl
    from paper_2310_17274_amd.binding import Context
    robot, worlds, batch, meta = wl.cfg_plain()
    robot, worlds, batch = wl.robot_f32(robot), wl.worlds_f32(worlds), wl.to_f32(batch)
    dev = torch.device("cuda:0")
    ctx = Context(robot)
    ctx.mg_set_worlds(worlds)
    alpha, iters = meta["alpha"], meta["iters"]
    b = ctx.batch(batch.seeds, batch.horizon, batch.world, K_max=len(alpha), m_max=4)
    q_start, goal, x0 = _inputs(robot, batch, dev)
    c0, g0, _ = ctx.mg_cost_grad(b, q_start, goal, x0)
    dvec = ctx.mg_lbfgs_step(b, 4, True, x0, g0)
    layout = layout_name(ctx.mg_autotune(b, q_start, goal, x0, dvec, alpha))
    sg, sp = [], []
    ms_g, outs = _time_solves(ctx, b, q_start, goal, x0, iters, alpha, True, reps, max(1, warmup), sg)
    ms_p, _ = _time_solves(ctx, b, q_start, goal, x0, iters, alpha, False, reps, max(1, warmup), sp)
    return {"workload": f"1 problem, {int(batch.seeds[0])} seeds x T={int(batch.horizon[0])}, "
                        f"{robot.n_spheres} spheres, {int(worlds.offsets[-1])} axis-aligned cuboids, "
                        f"K={len(alpha)}, {iters} iterations",
            "ms_per_solve_batched": pct(sg), "ms_per_solve_plain": pct(sp),
            "us_per_iteration_batched": 1000.0 * ms_g / iters, "us_per_iteration_plain": 1000.0 * ms_p / iters,
            "speedup_batched_vs_plain": ms_p / ms_g, "best_cost_min": float(outs[0].min().item()),
            "layout": layout}


def bench_uneven(warmup):
    """64 problems of uneven size (seeds U{4..64}, T in {24,32,48}, worlds of
    U{5..200} cuboids, K = 4): one batched graph solve of all problems against
    64 sequential per-problem solves with direct launches."""
    import torch
    from paper_2310_17274_amd import workloads as wl
    from paper_2310_17274_amd.binding import Context
    robot, worlds, batch, meta = wl.cfg_uneven()
    robot, worlds, batch = wl.robot_f32(robot), wl.worlds_f32(worlds), wl.to_f32(batch)
    dev = torch.device("cuda:0")
    ctx = Context(robot)
    ctx.mg_set_worlds(worlds)
    alpha, iters, P, D = meta["alpha"], meta["iters"], batch.n_problems, robot.dof
    b = ctx.batch(batch.seeds, batch.horizon, batch.world, K_max=len(alpha), m_max=4)
    q_start, goal, x0 = _inputs(robot, batch, dev)
    c0, g0, _ = ctx.mg_cost_grad(b, q_start, goal, x0)
    dvec = ctx.mg_lbfgs_step(b, 4, True, x0, g0)
    layout = layout_name(ctx.mg_autotune(b, q_start, goal, x0, dvec, alpha))
    sb = []
    ms_b, _ = _time_solves(ctx, b, q_start, goal, x0, iters, alpha, True, 20, max(1, warmup), sb)
    # plain: one batch per problem, every kernel launched directly
    singles, r0 = [], 0
    for p in range(P):
        n = int(batch.seeds[p]) * int(batch.horizon[p])
        bp = ctx.batch([batch.seeds[p]], [batch.horizon[p]], [batch.world[p]], K_max=len(alpha), m_max=4)
        outs = (torch.empty(bp.n_seeds, dtype=torch.float32, device=dev),
                torch.empty(1, dtype=torch.int32, device=dev), torch.empty(1, dtype=torch.int32, device=dev))
        singles.append((bp, q_start[p:p + 1].contiguous(), goal[p:p + 1].contiguous(),
                        x0[r0:r0 + n].clone(), outs))
        r0 += n
    xs = [s[3].clone() for s in singles]

    def plain():
        for (bp, qs, gl, xp, outs), x in zip(singles, xs):
            x.copy_(xp)
            ctx.mg_solve(bp, qs, gl, x, iters, 4, alpha, mode=1, use_graph=False, outputs=outs)
    plain()
    torch.cuda.synchronize()
    reps = 20
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    evs[0].record(torch.cuda.current_stream())
    for i in range(reps):
        plain()
        evs[i + 1].record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    sp = [evs[i].elapsed_time(evs[i + 1]) for i in range(reps)]
    ms_p = evs[0].elapsed_time(evs[-1]) / reps
    evals = int(np.sum(batch.seeds * batch.horizon)) * len(alpha) * iters
    return {"workload": f"{P} problems, seeds U{{4..64}} (total {int(batch.seeds.sum())}), T in {{24,32,48}}, "
                        f"{int(worlds.offsets[-1])} cuboids in {P} worlds, K={len(alpha)}, {iters} iterations",
            "ms_per_solve_batched": ms_b / P, "ms_per_solve_plain": ms_p / P,
            "speedup_batched_vs_plain": ms_p / ms_b, "evals_per_s_batched": evals / (ms_b * 1e-3),
            "ms_per_batch_batched": pct(sb), "ms_per_batch_plain": pct(sp),
            "layout": layout}


def bench_ik(warmup):
    """Collision-free inverse kinematics: 4096 goal poses x 32 seeds (T = 1),
    40 oriented cuboids, K = 4, 100 iterations as graphs of 25.  Timed on the
    configured goals (positions uniform in the 0.3-0.8 m shell, uniform
    orientation: many are unreachable or in collision), with the success
    fraction on them, and the success fraction on a feasible set: end-effector
    poses of collision-free random configurations (reachable and
    collision-free by construction)."""
    import torch
    from paper_2310_17274_amd import workloads as wl
    from paper_2310_17274_amd.binding import Context
    robot, worlds, batch, meta = wl.cfg_ik()
    robot, worlds, batch = wl.robot_f32(robot), wl.worlds_f32(worlds), wl.to_f32(batch)
    dev = torch.device("cuda:0")
    ctx = Context(robot)
    ctx.mg_set_worlds(worlds)
    alpha, iters, P = meta["alpha"], meta["iters"], batch.n_problems
    b = ctx.batch(batch.seeds, batch.horizon, batch.world, K_max=len(alpha), m_max=4)
    q_start, goal, x0 = _inputs(robot, batch, dev)
    c0, g0, _ = ctx.mg_cost_grad(b, q_start, goal, x0)
    dvec = ctx.mg_lbfgs_step(b, 4, True, x0, g0)
    layout = layout_name(ctx.mg_autotune(b, q_start, goal, x0, dvec, alpha))
    samples = []
    ms, outs = _time_solves(ctx, b, q_start, goal, x0, iters, alpha, True, 20, max(1, warmup), samples)
    ok_cfg = outs[2].float().mean().item()
    # feasible goals: poses of collision-free random configurations (the
    # library's own kinematics and clearance at T = 1)
    cand = wl.goal_configs(robot, 33, 32 * P)
    qc = torch.as_tensor(cand, dtype=torch.float32, device=dev).contiguous()
    bc = ctx.batch([cand.shape[0]], [1], [0], K_max=1, m_max=0)
    _, _, clear = ctx.mg_cost_grad(bc, q_start[:1].contiguous(), goal[:1].contiguous(), qc, grad=False)
    free = torch.nonzero(clear >= 0.0).flatten()
    n_free = int(free.numel())
    pick = free[:P] if n_free >= P else torch.cat([free, torch.argsort(clear, descending=True)[:P - n_free]])
    goal_f = ctx.mg_ee_pose(qc[pick].contiguous()).reshape(P, -1).contiguous()
    ms_f, outs_f = _time_solves(ctx, b, q_start, goal_f, x0, iters, alpha, True, 3, 1)
    ok_f = outs_f[2].float().mean().item()
    return {"workload": f"{P} goals x {int(batch.seeds[0])} seeds, T=1, {int(worlds.offsets[-1])} oriented "
                        f"cuboids, K={len(alpha)}, {iters} iterations (graphs of 25)",
            "ik_per_s": P / (ms * 1e-3), "ms_per_batch": ms, "ms_per_batch_pct": pct(samples),
            "success_fraction": ok_cfg,
            "success_fraction_feasible": ok_f, "ms_per_batch_feasible": ms_f,
            "feasible_goals_collision_free_configs": min(n_free, P),
            "evals_per_s": int(batch.seeds.sum()) * len(alpha) * iters / (ms * 1e-3),
            "layout": layout,
            "note": "success = best seed within 5 mm / 0.05 rad of the goal and collision free. "
                    "success_fraction: goals as configured (positions uniform in the 0.3-0.8 m shell, "
                    "uniform orientation; reachability and clearance not enforced). "
                    "success_fraction_feasible: goals at end-effector poses of collision-free "
                    "configurations U(-2.5,2.5)^7 (reachable and collision free by construction)"}


def bench_motion_gen(warmup):
    """Motion generation (IK -> seeds -> two-pass trajectory optimization ->
    choice) on the 7-DOF arm with 52 spheres among 40 oriented cuboids:
    one problem alone, then 64 problems in one call.  IK 32 seeds x 100
    iterations; trajectories 12 seeds x T=32, 100 + 100 iterations."""
    import torch
    from paper_2310_17274_amd import workloads as wl
    from paper_2310_17274_amd.binding import Context
    robot, worlds, batch, meta = wl.cfg_cost_adjoint()
    robot, worlds = wl.robot_f32(robot), wl.worlds_f32(worlds)
    dev = torch.device("cuda:0")
    ctx = Context(robot)
    ctx.mg_set_worlds(worlds)
    alpha, D = wl.ALPHA_4, robot.dof
    vmax, amax, jmax = [2.175] * 4 + [2.61] * 3, [15.0, 7.5, 10.0, 12.5, 15.0, 20.0, 20.0], \
        [7500.0, 3750.0, 5000.0, 6250.0, 7500.0, 10000.0, 10000.0]
    rng = np.random.default_rng(60)
    out = {}
    for P in (1, 64):
        # collision-free starts and reachable collision-free goals: the
        # clearest of 128 random configurations per problem (the library's
        # own kinematics and clearance), alternately start and goal
        cand = wl.goal_configs(robot, 61 + P, 128 * P)
        qc = torch.as_tensor(cand, dtype=torch.float32, device=dev).contiguous()
        bc = ctx.batch([cand.shape[0]], [1], [0], K_max=1, m_max=0)
        z = torch.zeros((1, D), dtype=torch.float32, device=dev)
        zg = ctx.mg_ee_pose(z).reshape(1, -1).contiguous()
        _, _, clear = ctx.mg_cost_grad(bc, z, zg, qc, grad=False)
        order = torch.argsort(clear, descending=True, stable=True)[:2 * P]
        free = (clear[order] >= 0.0).float().mean().item()
        q_start = qc[order[0::2]].contiguous()
        goal = ctx.mg_ee_pose(qc[order[1::2]].contiguous()).reshape(P, -1).contiguous()
        ik = ctx.batch(np.full(P, 32), np.ones(P, int), np.zeros(P, int), K_max=4, m_max=4)
        to = ctx.batch(np.full(P, 12), np.full(P, 32), np.zeros(P, int), K_max=4, m_max=4)
        x_ik0 = torch.as_tensor(rng.uniform(-2.5, 2.5, (P * 32, D)), dtype=torch.float32, device=dev)
        x_ik = torch.empty_like(x_ik0)
        x_to = torch.empty((to.rows, D), dtype=torch.float32, device=dev)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        calls = []
        for rep in range(max(1, warmup) + 20):
            x_ik.copy_(x_ik0)
            torch.cuda.synchronize()
            ev0.record()
            _, ik_ok, bs, ok, mt, dts = ctx.mg_motion_gen(ik, to, q_start, goal, x_ik, 100, 100, 100, 4, alpha,
                                                          vmax, amax, jmax, x_to=x_to)
            ev1.record()
            torch.cuda.synchronize()
            if rep >= max(1, warmup):
                calls.append(ev0.elapsed_time(ev1))
        ms = float(np.median(calls))
        out[f"P{P}"] = {"ms_per_call": ms, "ms_per_call_pct": pct(calls), "ms_per_problem": ms / P,
                        "ik_found_fraction": ik_ok.float().mean().item(),
                        "success_fraction": ok.float().mean().item(),
                        "mean_motion_time_s": mt.mean().item(), "dt_opt": dts[0], "dt_final": dts[1],
                        "start_goal_collision_free": free}
    out["workload"] = ("7-DOF arm, 52 spheres, 40 oriented cuboids; IK 32 seeds x 100 iterations (K=4), "
                       "12 linear seeds x T=32, 100 iterations at dt 0.25 without jerk, retime, 100 "
                       "iterations at the retimed dt with rescaled weights, retime, choice")
    out["note"] = ("starts and goal configurations are the clearest of 128 random configurations "
                   "U(-2.5,2.5)^7 per problem (about 6% of random configurations are collision free "
                   "in this world); success = goal within 5 mm / 0.05 rad and collision free")
    return out


def _connected_queries(ctx, robot, nq, seed, res, n_max):
    """nq start/goal pairs known to be joined by a collision-free path: both
    ends in the largest connected component of a dense roadmap (the free
    ones of 200000 uniform configurations, each steered to its 10 nearest),
    built with the library's own clearance, k-nearest search and steering,
    and with the direct edge between them blocked."""
    import torch
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from paper_2310_17274_amd.binding import mg_knn
    dev, D = torch.device("cuda:0"), robot.dof
    rng = np.random.default_rng(seed)
    Q = rng.uniform(robot.q_lo, robot.q_hi, (200000, D)).astype(np.float32)
    qd = torch.as_tensor(Q, device=dev).contiguous()
    z = torch.zeros((1, D), dtype=torch.float32, device=dev)
    zg = ctx.mg_ee_pose(z).reshape(1, -1).contiguous()
    _, _, clear = ctx.mg_cost_grad(ctx.batch([Q.shape[0]], [1], [0], K_max=1, m_max=0), z, zg, qd, grad=False)
    nodes = Q[clear.cpu().numpy() >= 0]
    k, E = 10, 512
    idx, _ = mg_knn(torch.as_tensor(nodes, device=dev), torch.as_tensor(nodes, device=dev), k + 1)
    src = np.repeat(np.arange(len(nodes)), k)
    dst = idx.cpu().numpy()[:, 1:].reshape(-1)
    b = ctx.batch([E * (n_max + 1)], [1], [0], K_max=1, m_max=0)

    def steer_ok(a, c):
        ok = np.zeros(len(a), bool)
        for e0 in range(0, len(a), E):
            fa, fb = a[e0:e0 + E], c[e0:e0 + E]
            n = len(fa)
            fa = np.concatenate([fa, np.repeat(fa[-1:], E - n, 0)])
            fb = np.concatenate([fb, np.repeat(fb[-1:], E - n, 0)])
            _, last, _ = ctx.mg_steer(b, torch.as_tensor(fa, device=dev), torch.as_tensor(fb, device=dev), res, n_max)
            steps = np.floor(np.abs(fb[:n] - fa[:n]).max(1) / res).astype(int) + 1
            ok[e0:e0 + n] = last.cpu().numpy()[:n] == steps
        return ok
    ok = steer_ok(nodes[src], nodes[dst])
    m = coo_matrix((np.ones(ok.sum()), (src[ok], dst[ok])), shape=(len(nodes), len(nodes)))
    _, lab = connected_components(m, directed=False)
    big = np.flatnonzero(lab == np.bincount(lab).argmax())
    pairs = []
    while len(pairs) < nq:
        a, c = nodes[rng.choice(big, 2, replace=False)]
        if not steer_ok(a[None], c[None])[0]:
            pairs.append((a, c))
    return (np.stack([p[0] for p in pairs]), np.stack([p[1] for p in pairs]),
            {"free_samples": int(len(nodes)), "largest_component": int(len(big))})


def bench_plan(warmup, reps=20):
    """Geometric planning (Alg.2, steering by Alg.3) on the 7-DOF arm with
    52 spheres among 40 oriented cuboids, one call per query set, each call
    seeded anew.  Two query sets: starts and goals that are the clearest of
    64 random configurations each (some pairs lie in different free-space
    components: no path exists), and pairs known to be connected with their
    direct edge blocked.  One query alone, then 16 on one shared roadmap."""
    import torch
    from paper_2310_17274_amd import workloads as wl
    from paper_2310_17274_amd.binding import Context
    robot, worlds, _, _ = wl.cfg_cost_adjoint()
    robot, worlds = wl.robot_f32(robot), wl.worlds_f32(worlds)
    dev = torch.device("cuda:0")
    ctx = Context(robot)
    ctx.mg_set_worlds(worlds)
    D = robot.dof
    n_edges, n_max, res = 256, 128, 0.05
    b = ctx.batch([n_edges * (n_max + 1)], [1], [0], K_max=1, m_max=0)
    z = torch.zeros((1, D), dtype=torch.float32, device=dev)
    zg = ctx.mg_ee_pose(z).reshape(1, -1).contiguous()
    cs, cg, info = _connected_queries(ctx, robot, 16, 90, res, n_max)
    out = {"connected_queries": info}
    for kind in ("clearest", "connected"):
        for nq in (1, 16):
            if kind == "clearest":
                cand = wl.goal_configs(robot, 80 + nq, 64 * 2 * nq)
                qc = torch.as_tensor(cand, dtype=torch.float32, device=dev).contiguous()
                bc = ctx.batch([cand.shape[0]], [1], [0], K_max=1, m_max=0)
                _, _, clear = ctx.mg_cost_grad(bc, z, zg, qc, grad=False)
                clear = clear.cpu().numpy().reshape(2 * nq, 64)
                pick = cand.reshape(2 * nq, 64, D)[np.arange(2 * nq), clear.argmax(1)]
                starts, goals = pick[0::2], pick[1::2]
            else:
                starts, goals = cs[:nq], cg[:nq]
            calls, solved, wps = [], [], []
            for rep in range(max(1, warmup) + reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                paths = ctx.mg_plan_batch(b, starts, goals, res, n_max, n_samples=64, k_near=4, max_rounds=40,
                                          refine_rounds=4, seed=1000 + rep)
                torch.cuda.synchronize()
                if rep >= max(1, warmup):
                    calls.append((time.perf_counter() - t0) * 1e3)
                    solved += [len(p) > 0 for p in paths]
                    wps += [len(p) for p in paths if len(p)]
            out[f"{kind}_Q{nq}"] = {"ms_per_call": float(np.median(calls)), "ms_per_call_pct": pct(calls),
                                    "success_fraction": float(np.mean(solved)), "calls": len(calls),
                                    "mean_waypoints": float(np.mean(wps)) if wps else 0.0}
    out["workload"] = ("7-DOF arm, 52 spheres, 40 oriented cuboids (about 6% of configurations collision "
                       "free); steering at 0.05 rad, up to 128 steps, 256 edges per launch; 64 collision-free "
                       "samples (of 32x as many candidates) and 4 neighbours per round, growing on failure; at "
                       "most 40 rounds, 4 refine rounds once every query is solved")
    out["note"] = ("host wall clock per call (host roadmap; device clearance, k-nearest search and "
                   "steering); 'connected' pairs lie in the largest component of a dense roadmap "
                   "(200000 uniform samples) with their direct edge blocked")
    return out


def bench_large(warmup, reps=20):
    """Two-arm tree (14 joints, 120 spheres), 500 oriented cuboids, swept
    collision (4 trace steps), 128 seeds x 48 waypoints: the particle stage
    (2 rounds x 256 particles per seed, noise drawn on the device) then 100
    L-BFGS iterations with 4 line-search candidates (graphs of 25)."""
    import torch
    from paper_2310_17274_amd import workloads as wl
    from paper_2310_17274_amd.binding import Context, default_params
    robot, worlds, batch, meta = wl.cfg_large()
    robot, worlds, batch = wl.robot_f32(robot), wl.worlds_f32(worlds), wl.to_f32(batch)
    dev = torch.device("cuda:0")
    ctx = Context(robot, default_params(swept=1, sweep_steps=4))
    ctx.mg_set_worlds(worlds)
    alpha, iters, P, D = meta["alpha"], meta["iters"], batch.n_problems, robot.dof
    S, T, N, R = int(batch.seeds[0]), int(batch.horizon[0]), 256, 2
    b = ctx.batch(batch.seeds, batch.horizon, batch.world, K_max=len(alpha), m_max=4)
    b.mg_batch_reserve_particles(N)
    q_start, goal, x0 = _inputs(robot, batch, dev)
    c0, g0, _ = ctx.mg_cost_grad(b, q_start, goal, x0)
    dvec = ctx.mg_lbfgs_step(b, 4, True, x0, g0)
    layout = layout_name(ctx.mg_autotune(b, q_start, goal, x0, dvec, alpha, launches=3))
    mean, var = x0.clone(), torch.empty_like(x0)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    stream = torch.cuda.current_stream()
    tp, ts = [], []
    for rep in range(max(1, warmup) + reps):
        mean.copy_(x0)
        var.fill_(0.05 ** 2)
        torch.cuda.synchronize()
        e0.record(stream)
        ctx.mg_particles_seeded(b, q_start, goal, mean, var, N, R, 55)
        e1.record(stream)
        ctx.mg_solve(b, q_start, goal, mean, iters, 4, alpha, mode=1, graph_inner=25, use_graph=True)
        e2.record(stream)
        torch.cuda.synchronize()
        if rep >= max(1, warmup):
            tp.append(e0.elapsed_time(e1))
            ts.append(e1.elapsed_time(e2))
    ms_p, ms_s = float(np.mean(tp)), float(np.mean(ts))
    return {"workload": f"two-arm tree ({D} joints, {robot.n_spheres} spheres), {int(worlds.offsets[-1])} "
                        f"oriented cuboids, swept collision (4 steps), {S} seeds x T={T}; particle stage "
                        f"{R} x {N} (device Philox noise), then {iters} L-BFGS iterations with K={len(alpha)} (graphs of 25)",
            "ms_particle_stage": ms_p, "ms_lbfgs_solve": ms_s, "ms_per_solve": ms_p + ms_s,
            "particle_evals_per_s": R * N * S * T / (ms_p * 1e-3),
            "lbfgs_evals_per_s": S * T * len(alpha) * iters / (ms_s * 1e-3),
            "ms_particle_stage_pct": pct(tp), "ms_lbfgs_solve_pct": pct(ts),
            "layout": layout}


def profile_eval(ctx, b, q_start, goal, x0, c0, g0, dvec, alpha, launches, layout):
    """Evaluation launches of the benchmark shape for hardware-counter runs."""
    import torch
    for _ in range(launches):
        ctx.mg_linesearch(b, q_start, goal, x0, c0, g0, dvec, alpha, 1)
    torch.cuda.synchronize()
    print(json.dumps({"profile": "eval", "launches": launches, "kernel_digest": kernel_digest(),
                      "layout": layout}), flush=True)


def profile_large(launches, layout=None):
    """The large two-arm workload for hardware-counter runs: one particle
    round (256 particles per seed, device noise) and `launches` line searches
    (one evaluation launch each, K = 4)."""
    import torch
    from paper_2310_17274_amd import workloads as wl
    from paper_2310_17274_amd.binding import Context, default_params
    robot, worlds, batch, meta = wl.cfg_large()
    robot, worlds, batch = wl.robot_f32(robot), wl.worlds_f32(worlds), wl.to_f32(batch)
    dev = torch.device("cuda:0")
    ctx = Context(robot, default_params(swept=1, sweep_steps=4))
    ctx.mg_set_worlds(worlds)
    alpha = meta["alpha"]
    b = ctx.batch(batch.seeds, batch.horizon, batch.world, K_max=len(alpha), m_max=4)
    b.mg_batch_reserve_particles(256)
    q_start, goal, x0 = _inputs(robot, batch, dev)
    c0, g0, _ = ctx.mg_cost_grad(b, q_start, goal, x0)
    dvec = ctx.mg_lbfgs_step(b, 4, True, x0, g0)
    if layout is None:
        tuned = layout_name(ctx.mg_autotune(b, q_start, goal, x0, dvec, alpha, launches=3))
    else:
        b.mg_batch_set_layout(layout, 0)
        tuned = f"forced {layout}"
    mean, var = x0.clone(), torch.full_like(x0, 0.05 ** 2)
    ctx.mg_particles_seeded(b, q_start, goal, mean, var, 256, 1, 55)
    for _ in range(launches):
        ctx.mg_linesearch(b, q_start, goal, x0, c0, g0, dvec, alpha, 1)
    torch.cuda.synchronize()
    print(json.dumps({"profile": "large", "launches": launches, "layout": tuned}), flush=True)


def profile_copy():
    """Plain device-to-device copy of 256 MiB, five times: the reference
    reading of the HBM byte counters."""
    import torch
    n = 64 * 1024 * 1024
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profile": "copy", "bytes": n * 4, "copies": 5}), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_solve_rate(r, boxes, q0, goal, T, x, K, alpha, iters, threads, seconds):
    """Oracle evaluations per second of whole solves repeated to fill about
    `seconds` (each solve of n iterations evaluates n S T K candidates plus
    the initial S T)."""
    S = x.size // (T * r.robot.dof)
    t0 = time.perf_counter()
    r.solve(boxes, q0, goal, T, x, 1, 4, alpha, nthreads=threads)
    one = time.perf_counter() - t0
    n = int(max(1, min(iters, seconds / max(one, 1e-6))))
    reps = int(max(1, seconds / max(one * n, 1e-6)))
    t0 = time.perf_counter()
    for _ in range(reps):
        r.solve(boxes, q0, goal, T, x, n, 4, alpha, nthreads=threads)
    dt = time.perf_counter() - t0
    return reps * (n * S * T * K + S * T) / dt, reps, n, dt


def cpu_baseline(robot, worlds, batch, alpha, iters, seconds):
    """The FP64 reference solve on the host cores, on bounded samples: the
    same 32-seed problem on all threads of the machine's CPU share (16 at most)
    and on one thread, and seeded subsets of the IK, uneven and large
    workloads with their whole-workload solve times extrapolated."""
    from oracle import ref
    from paper_2310_17274_amd import workloads as wl
    threads = min(16, os.cpu_count() or 1)
    r = ref.Ref(robot)
    T, S, K = int(batch.horizon[0]), int(batch.seeds[0]), len(alpha)
    boxes = worlds.world(0)
    v, reps, n, dt = _oracle_solve_rate(r, boxes, batch.q_start[0], batch.goal[0], T, batch.x0, K, alpha, iters,
                                        threads, seconds)
    v1, reps1, n1, dt1 = _oracle_solve_rate(r, boxes, batch.q_start[0], batch.goal[0], T, batch.x0, K, alpha,
                                            iters, 1, seconds / 2)
    subsets = {}
    # IK: 4 goals x 32 seeds; uneven: problems 0 and 1; large: 2 seeds
    for name, (rb, wd, bt, meta), pick, sw in (
            ("ik", wl.cfg_ik(), lambda bt: [(p, 32) for p in range(4)], 0),
            ("uneven", wl.cfg_uneven(), lambda bt: [(0, int(bt.seeds[0])), (1, int(bt.seeds[1]))], 0),
            ("large", wl.cfg_large(), lambda bt: [(0, 2)], 1)):
        rb, wd, bt = wl.robot_f32(rb), wl.worlds_f32(wd), wl.to_f32(bt)
        rr = ref.Ref(rb, swept=sw, sweep_steps=4)
        offs = bt.row_offsets(rb.dof)
        seed0 = np.concatenate([[0], np.cumsum(bt.seeds)])
        evals, secs = 0.0, 0.0
        for p, ns in pick(bt):
            Tp = int(bt.horizon[p])
            a, b_ = offs[seed0[p]], offs[seed0[p] + ns]
            rate, rp, nn, tt = _oracle_solve_rate(rr, wd.world(int(bt.world[p])), bt.q_start[p], bt.goal[p], Tp,
                                                  bt.x0[a:b_], len(meta["alpha"]), meta["alpha"], meta["iters"],
                                                  threads, seconds / 6)
            evals += rate * tt
            secs += tt
        rate = evals / secs
        total = float(np.sum(bt.seeds * bt.horizon)) * len(meta["alpha"]) * meta["iters"]
        subsets[name] = {"evals_per_s": rate, "sample_s": secs,
                         "extrapolated_solve_s": total / rate, "sample": str([q for q in pick(bt)]) +
                         " (problem, seeds) solved with the oracle"}
    return {"value": v, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 reference solve of the same problem, {reps} x {n} of {iters} iterations, "
                      f"{S} seeds in parallel over {threads} threads ({dt:.1f} s)",
            "single_thread": {"value": v1, "unit": "evals/s", "cores": 1,
                              "sample": f"{reps1} x {n1} iterations on one thread ({dt1:.1f} s)"},
            "cpu_model": _cpu_model(),
            "subsets_extrapolated": subsets}


if __name__ == "__main__":
    main()
