#!/usr/bin/env python3
"""Condensed MPC steps/s on one MI355X: 1000-node chain, horizon N = 20.

One step is one pass of the whole hot path of Algorithm 1 on resident inputs:
linearize the GNN (forward pass + forward-mode Jacobians, BF16 MLPs with FP32
accumulation), condense (S_k / Gx_k recursion, H, g, 200 node-position rows,
FP32) and solve the condensed box QP (ADMM, FP32).  The plain form (analytic
mass-spring-damper Jacobians on the same graph) is timed beside it.  The
step is captured once as a HIP graph and replayed (``--eager`` times eager
launches instead).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--eager] [--only-step]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "condensed MPC steps/s, 1000 nodes N=20 (GNN vs plain); % HBM roofline"
BF16_DENSE_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak
HBM_PEAK_GBS = 8000.0


def jacobian_flops(P):
    """Algorithmic FLOPs of one GNN linearization: exact forward mode restricted
    to each seed's receptive support.  Per tangent column of seed s and round l:
    [W_a; W_b] on every node of V_{l-1}(s) (4 Hd^2), W_n2 on every node of V_l(s)
    and W_n1 on those also in V_{l-1}(s) (2 Hd^2 each), then the 3 used decoder
    rows on V_L(s) (6 Hd); V_l(s) = nodes within l hops downstream of s."""
    Hd, L, M = P.gnn.Hd, P.gnn.L, P.M
    outn = [[] for _ in range(M)]
    for i in range(M):
        for j in P.col[P.row_ptr[i]:P.row_ptr[i + 1]]:
            outn[j].append(i)
    act = set(int(a) for a in P.act)
    total = 0.0
    for s in range(M):
        V = [{s}]
        for _ in range(L):
            nxt = set(V[-1])
            for j in V[-1]:
                nxt.update(outn[j])
            V.append(nxt)
        per_col = sum(4 * Hd * Hd * len(V[l - 1]) + 2 * Hd * Hd * (len(V[l]) + len(V[l - 1]))
                      for l in range(1, L + 1)) + 6 * Hd * len(V[L])
        total += per_col * (6 + (3 if s in act else 0))
    return total * P.N


def measured_traffic():
    """HBM bytes per launch of the Jacobian kernel from the counter summary in
    profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a
    copy of known size), or None when the kernel source has changed since the
    counters were taken (the summary records the SHA-256 of the source file)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "jvp_mfma2_kernel_chain1000_counters.md")
    src = os.path.join(ROOT, "paper_2602_17601_amd", "csrc", "gnn.hip")
    try:
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line and line.strip().startswith("- "):
                    k, v = line.strip()[2:].split(":", 1)
                    fields[k.strip()] = v.strip().strip("`")
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if fields.get("source_sha256") != sha:
            return None
        return int(fields["fetch_bytes_per_launch"]) + int(fields["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _host_cpu():
    """CPU model name and the number of cores this process may run on."""
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


def _oracle_lin_sample(job):
    """Worker of the multi-core oracle timing: the FP64 GNN linearization of the
    1000-node workload on the given (stage, node) sample, one BLAS thread."""
    stages, nodes = job
    from threadpoolctl import threadpool_limits
    from oracle.gnn import gnn_linearize
    from paper_2602_17601_amd import workloads as wl
    P = wl.gnn1000_bf16()
    Wr = P.gnn.rounded_bf16(biases="f32")
    with threadpool_limits(1):
        t0 = time.perf_counter()
        gnn_linearize(P.xhat, P.uhat, Wr, P.row_ptr, P.col, P.act, stages=stages, nodes=nodes)
        return time.perf_counter() - t0


def _oracle_plain_step(P):
    """One plain-form step of the FP64 oracle: analytic linearization,
    per-node condensing recursion and the interior-point QP (seconds)."""
    from oracle.condense import condense_local
    from oracle.msd import msd_linearize
    from oracle.qp import qp_ipm
    t0 = time.perf_counter()
    prow, pcol, A, B, c = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    l = condense_local(A, B, c, prow, pcol, P.x0, P.costs.Q, P.costs.q, P.costs.R, P.costs.r, P.rows)
    if P.rows.n:
        qp_ipm(l["H"], l["g"], P.lb, P.ub, l["Ct"], np.full(P.rows.n, -np.inf), l["dt"])
    else:
        qp_ipm(l["H"], l["g"], P.lb, P.ub)
    return time.perf_counter() - t0


def cpu_baseline(P, Pm):
    """The FP64 oracle on the host cores, on a bounded sample of the step.

    GNN form: the per-node linearization timed on a sample of node-stages
    (1000 on one thread; 1000 per core on all cores, split over one worker
    process per core) and extrapolated to all N*M node-stages, plus one full
    condensing on the 13-wide GNN pattern and one QP solve, which the oracle
    runs on one thread.  The condensing takes the analytic mass-spring-damper
    Jacobians of the same chain placed into the wider GNN pattern, so the
    blocks have the dynamics' magnitudes.  Plain form: whole oracle steps
    (linearize, condense, QP) of the 10-, 100- and 1000-node workloads."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle.condense import condense_local
    from oracle.graph import jacobian_pattern
    from oracle.msd import msd_linearize
    from oracle.qp import qp_ipm
    from paper_2602_17601_amd import workloads as wl
    cpu, cores = _host_cpu()
    stages = [3, 7, 11, 15, 19]
    sample1 = (stages, list(range(300, 500)))
    with threadpool_limits(1):
        t_lin1 = _oracle_lin_sample(sample1) / 1000 * P.N * P.M
        prow, pcol = jacobian_pattern(P.row_ptr, P.col, P.M, P.gnn.L)
        mrow, mcol, Am, Bm, cm = msd_linearize(Pm.xhat, Pm.uhat, Pm.row_ptr, Pm.col, Pm.act, Pm.msd)
        A = np.zeros((P.N, len(pcol), 6, 6))
        for i in range(P.M):
            cols = pcol[prow[i]:prow[i + 1]]
            for e in range(mrow[i], mrow[i + 1]):
                A[:, prow[i] + int(np.searchsorted(cols, mcol[e]))] = Am[:, e]
        t0 = time.perf_counter()
        l = condense_local(A, Bm, cm, prow, pcol, Pm.x0, Pm.costs.Q, Pm.costs.q, Pm.costs.R, Pm.costs.r, Pm.rows)
        t_cond = time.perf_counter() - t0
        t0 = time.perf_counter()
        qp_ipm(l["H"], l["g"], Pm.lb, Pm.ub, l["Ct"], np.full(Pm.rows.n, -np.inf), l["dt"])
        t_qp = time.perf_counter() - t0
        plain = {name: 1.0 / _oracle_plain_step(prob) for name, prob in
                 (("msd10_fp64", wl.msd10_fp64()), ("msd100", wl.gnn100_fp32("msd")), ("msd1000", Pm))}
    # all cores: one worker process per core, 200 nodes x 5 stages each
    jobs = [(stages, [(300 + 200 * w + t) % P.M for t in range(200)]) for w in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_lin_sample, jobs)
    t_lin_n = (time.perf_counter() - t0) / (1000 * cores) * P.N * P.M
    step1 = t_lin1 + t_cond + t_qp
    stepn = t_lin_n + t_cond + t_qp
    return {"value": 1.0 / stepn, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "cpu": cpu, "value_1_thread": 1.0 / step1, "plain_form_steps_per_s": plain,
            "sample": (f"FP64 oracle (numpy) on {cpu}, {cores} cores: GNN linearization timed on 1000 "
                       f"node-stages per core in {cores} worker processes, including their start-up "
                       f"({t_lin_n / (P.N * P.M) * 1e3:.2f} ms per node-stage; 1 thread: "
                       f"{t_lin1 / (P.N * P.M) * 1e3:.1f} ms), extrapolated to {P.N * P.M}; one full "
                       f"condensing on the {len(pcol)}-block GNN pattern ({t_cond:.2f} s, 1 thread) and "
                       f"one QP ({t_qp:.2f} s, 1 thread); plain form: whole oracle steps on 1 thread")}


# Published MI355X peaks used by the per-phase rooflines.
FP32_MATRIX_PEAK_TFLOPS = 157.3   # dense FP32 (matrix cores)
FP32_VECTOR_PEAK_TFLOPS = 157.3   # FP32 vector (packed); the library builds without packed FP32, i.e. half
CU_COUNT = 256


def phase_rooflines(P, nnz, phase_ms, jac_flops):
    """Per-phase attainable-roofline fractions of the GNN step: algorithmic
    FLOPs and HBM bytes of each phase, t_roof = max(bytes / HBM peak,
    FLOPs / peak of the binding unit), against the measured phase time."""
    M, N, nu, Hd, L = P.M, P.N, P.nu, P.gnn.Hd, P.gnn.L
    E = int(P.col.shape[0])
    f4 = 4
    A_bytes, B_bytes, c_bytes = N * nnz * 36 * f4, N * M * 6 * nu * f4, N * M * 6 * f4
    # forward: encoder and decoder per node, per round [W_a; W_b] h and W_n [h; agg] per node (8 Hd^2,
    # the edge MLP in factored form) plus the per-edge combine, ReLU and sum (3 Hd)
    fwd_flops = N * (M * (2 * 9 * Hd + 2 * Hd * 6) + L * (M * 8 * Hd * Hd + E * 3 * Hd))
    n = N * nu
    prop_flops = 72 * nnz * nu * N * (N - 1) / 2 + 72 * nnz * N
    gram_flops = sum(6 * M * (k * nu) * (k * nu + 1) + 2 * 6 * M * k * nu for k in range(1, N + 1))
    rows_flops = 2 * 6 * P.rows.n * n
    qp_flops = 2 * (n ** 3) / 3 + 10 * (2 * n * n + 4 * n * P.rows.n)
    cu_peak = FP32_MATRIX_PEAK_TFLOPS / CU_COUNT
    ph = [
        # phase, flops, bytes, binding unit, peak TFLOP/s
        ("gnn_forward", fwd_flops, P.xhat.size * f4 + 2 * N * M * 6 * f4, "mfma_bf16", BF16_DENSE_PEAK_TFLOPS),
        ("gnn_stage_images", 0, 0, "none (implementation traffic: the Jacobian kernel's stage copies)", None),
        ("gnn_jacobian", jac_flops, A_bytes + B_bytes, "mfma_bf16", BF16_DENSE_PEAK_TFLOPS),
        ("gnn_assembly", 2 * N * (nnz * 36 + M * 6 * nu), A_bytes + B_bytes + c_bytes, "hbm", None),
        ("condense_propagate", prop_flops, A_bytes + B_bytes + c_bytes, "fp32_vector", FP32_VECTOR_PEAK_TFLOPS),
        ("condense_gram", gram_flops, n * n * f4, "fp32_matrix", FP32_MATRIX_PEAK_TFLOPS),
        ("condense_rows", rows_flops, P.rows.n * 6 * n * f4 + P.rows.n * n * f4, "hbm", None),
        ("qp", qp_flops, n * n * f4 + P.rows.n * n * f4, "fp32_matrix_one_cu", cu_peak),
    ]
    out = {}
    tot_roof = tot_meas = 0.0
    for name, fl, by, unit, peak in ph:
        t_mem = by / (HBM_PEAK_GBS * 1e9)
        t_cmp = fl / (peak * 1e12) if peak else 0.0
        t_roof = max(t_mem, t_cmp)
        bound = unit if t_roof == 0 else ("hbm" if t_mem >= t_cmp else unit)
        t_meas = phase_ms.get(name, 0.0) * 1e-3
        out[name] = {"flops": fl, "hbm_bytes": by, "bound": bound, "t_roof_us": t_roof * 1e6,
                     "t_meas_us": t_meas * 1e6, "frac": t_roof / t_meas if t_meas > 0 else None}
        tot_roof += t_roof
        tot_meas += t_meas
    out["step"] = {"t_roof_us": tot_roof * 1e6, "t_meas_us": tot_meas * 1e6,
                   "frac": tot_roof / tot_meas if tot_meas > 0 else None}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead of the single instance: K independent instances of uneven size "
                         "(M ~ U{50..1000}, N ~ U{10..30}) in one batched step; prints its own JSON line")
    ap.add_argument("--surrogate", action="store_true",
                    help="instead of the step: the learned-surrogate pipeline (simulator data set, GNN training, "
                         "500-step closed loop with GNN against analytic Jacobians); prints its own JSON line")
    ap.add_argument("--surrogate-steps", type=int, default=2000, help="Adam steps of the --surrogate training")
    ap.add_argument("--eager", action="store_true",
                    help="time eagerly launched steps instead of replays of the step captured as a HIP graph")
    ap.add_argument("--only-step", action="store_true",
                    help="time the step (GNN and plain forms) only, without the side measurements (tangent maps, "
                         "simulator, closed loop, paper model, training, interior-point QP); for profiler runs")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB 5 times (the reference kernel "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters to bytes) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs the hot path on one GPU only; multi-GPU runs are not supported "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_mib:
        nb = args.copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb, "launches": 5}), flush=True)
        return
    from paper_2602_17601_amd import gnmpc as gn
    from paper_2602_17601_amd import workloads as wl

    if args.batch:
        bench_batch(args, torch, gn, wl)
        return
    if args.surrogate:
        from paper_2602_17601_amd import surrogate
        res = surrogate.run(surrogate.SurrogateConfig(steps=args.surrogate_steps),
                            log=lambda m: print(m, file=sys.stderr, flush=True))
        print(json.dumps({"metric": "learned-surrogate pipeline: one-step RMSE, Jacobian error, closed loop",
                          "n_gpus": 1, "data": "synthetic (simulator)", **res}), flush=True)
        return

    dev = "cuda"
    P = wl.gnn1000_bf16()
    Pm = wl.gnn1000_bf16(model="msd")
    # the host baseline runs before the GPU is touched (its worker processes start clean)
    cpu = None if args.no_cpu_baseline else cpu_baseline(P, Pm)
    n = P.N * P.nu

    def t(a):
        return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev).contiguous()

    def make(Pr, gnn):
        plan = gn.Plan(Pr.M, Pr.nu, Pr.N, Pr.rows.n, gn.F32)
        plan.graph_set(Pr.row_ptr, Pr.col, Pr.gnn.L if gnn else 1)
        if gnn:
            plan.model_set_gnn(Pr.gnn, Pr.act, dtype=gn.BF16)
        else:
            plan.model_set_msd(Pr.msd, Pr.act)
        plan.rows_set(Pr.rows.node, Pr.rows.stage)
        bufs = dict(xhat=t(Pr.xhat), uhat=t(Pr.uhat), x0=t(Pr.x0), Q=t(Pr.costs.Q), q=t(Pr.costs.q),
                    R=t(Pr.costs.R), r=t(Pr.costs.r), rowC=t(Pr.rows.C), rowd=t(Pr.rows.d), lb=t(Pr.lb),
                    ub=t(Pr.ub),
                    A=torch.empty(Pr.N, plan.nnz, 6, 6, device=dev), B=torch.empty(Pr.N, Pr.M, 6, Pr.nu, device=dev),
                    c=torch.empty(Pr.N, Pr.M, 6, device=dev), H=torch.empty(n, n, device=dev),
                    g=torch.empty(n, device=dev), Ct=torch.empty(Pr.rows.n, n, device=dev),
                    dt=torch.empty(Pr.rows.n, device=dev), u=torch.empty(n, device=dev),
                    info=torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device=dev))
        return plan, bufs

    settings = gn.default_admm_settings()

    def step(plan, b):
        plan.linearize(b["xhat"], b["uhat"], b["A"], b["B"], b["c"])
        plan.condense(b["A"], b["B"], b["c"], b["x0"], b["Q"], b["q"], b["R"], b["r"], b["rowC"], b["rowd"],
                      b["H"], b["g"], b["Ct"], b["dt"])
        plan.solve_box_qp(b["H"], b["g"], b["lb"], b["ub"], b["Ct"], None, b["dt"], b["u"], b["info"],
                          settings=settings)

    def timed(plan, b):
        """Throughput over exactly args.steps steps: replays of the whole step
        captured once as a HIP graph (or eager launches with --eager), with no
        event records in the timed stream.  Then the eager throughput, the
        per-step median and p95 of the replays (an event pair around each),
        and the per-phase HIP-event timers on eager steps (the events add
        gaps, so they stay out of `value`)."""
        for _ in range(args.warmup):
            step(plan, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(plan, b)
        torch.cuda.synchronize()
        el_eager = time.perf_counter() - t0
        graph = None
        if not args.eager:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                step(plan, b)
            for _ in range(args.warmup):
                graph.replay()
            torch.cuda.synchronize()
        run = graph.replay if graph is not None else (lambda: step(plan, b))
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        for e0, e1 in ev:
            e0.record()
            run()
            e1.record()
        torch.cuda.synchronize()
        per = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        stats = {"median_ms": per[len(per) // 2], "p95_ms": per[min(len(per) - 1, int(0.95 * len(per)))],
                 "eager_steps_per_s": args.steps / el_eager}
        plan.timers_enable(True)
        for _ in range(args.steps):
            step(plan, b)
        torch.cuda.synchronize()
        phases = plan.timers_read()
        plan.timers_enable(False)
        return el, phases, stats

    plan_g, bg = make(P, True)
    plan_m, bm = make(Pm, False)

    def tune(plan, b):
        """The library's condensing autotuner on this step's own blocks (setup, untimed)."""
        plan.linearize(b["xhat"], b["uhat"], b["A"], b["B"], b["c"])
        chosen, entries = plan.autotune_condense(b["A"], b["B"], b["c"], b["x0"], b["Q"], b["q"], b["R"], b["r"],
                                                 b["rowC"], b["rowd"], b["H"], b["g"], b["Ct"], b["dt"], reps=5)
        names = {0: "per-node kernel", 1: "node blocks, one stage per launch", 2: "node blocks, two stages per launch"}
        return {"chosen": chosen, "candidates": [
            {"variant": names[e["variant"]], "block_nodes": e["block_nodes"], "us": round(e["us"], 1)} for e in entries]}

    tuning = {"gnn": tune(plan_g, bg), "plain": tune(plan_m, bm)}
    el_g, ph_g, st_g = timed(plan_g, bg)
    el_m, ph_m, st_m = timed(plan_m, bm)
    qpi = gn.qp_info(bg["info"])
    steps_g = args.steps / el_g
    steps_m = args.steps / el_m

    jac_ms, jac_n = ph_g["gnn_jacobian"]
    jac_avg_s = jac_ms / max(jac_n, 1) * 1e-3
    flops = jacobian_flops(P)
    achieved = flops / jac_avg_s / 1e12 if jac_avg_s > 0 else 0.0
    roofline = {"kernel": "gnn_jacobian", "bound": "mfma", "achieved": achieved,
                "peak": BF16_DENSE_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / BF16_DENSE_PEAK_TFLOPS,
                "traffic": measured_traffic(), "algorithmic_flops_per_launch": flops,
                "avg_launch_ms": jac_avg_s * 1e3}

    def phase_avg(ph):
        return {k: (v[0] / v[1] if v[1] else 0.0) for k, v in ph.items() if v[1]}

    out = {
        "metric": METRIC,
        "value": steps_g,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el_g / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32",
        "data": "synthetic",
        "config": {"workload": ("1000-node 1-2-hop chain, GNN Hd=128 L=3 (BF16 MLPs, FP32 accumulate), "
                                "n_u=12 at 4 nodes, N=20, 200 node-position rows, FP32 condensing, ADMM box QP"),
                   "M": P.M, "N": P.N, "nu": P.nu, "nnz_blocks": int(plan_g.nnz), "state_rows": P.rows.n},
        "timing": ("eager launches" if args.eager else "HIP graph replay of the whole step") +
                  " on inputs resident in HBM (x0, nominal trajectory, costs, rows uploaded once before timing; "
                  "u stays on the device)",
        "median_ms_per_step": st_g["median_ms"],
        "p95_ms_per_step": st_g["p95_ms"],
        "eager_steps_per_s": st_g["eager_steps_per_s"],
        "plain_steps_per_s": steps_m,
        "plain_ms_per_step": el_m / args.steps * 1e3,
        "plain_median_ms_per_step": st_m["median_ms"],
        "plain_eager_steps_per_s": st_m["eager_steps_per_s"],
        "phase_ms_gnn": phase_avg(ph_g),
        "phase_ms_plain": phase_avg(ph_m),
        "qp_iters_gnn": qpi.iters,
        "condense_tuning": tuning,
        "qp_status_gnn": qpi.status,
        "roofline": roofline,
        "phase_roofline_gnn": phase_rooflines(P, int(plan_g.nnz), phase_avg(ph_g), flops),
        "cpu_baseline": cpu,
    }
    if not args.only_step:
        out.update({
            "tangent": tangent_rates(gn, plan_g, bg, args.steps),
            "simulator": simulator_rate(torch, gn, wl),
            "closed_loop": {"workload": "1000-node chain, N=20, 200 obstacle rows, spring-damper plant",
                            "plain": closed_loop_rate(torch, gn, wl, "msd"),
                            "gnn": closed_loop_rate(torch, gn, wl, "gnn")},
            "paper_model": paper_model_rate(torch, gn, wl),
            "ipm": ipm_rate(torch, gn, plan_g, bg, settings),
            "training": training_rate(torch, gn, wl),
        })
    print(json.dumps(out), flush=True)


def ipm_rate(torch, gn, plan, b, settings, reps=10):
    """The interior-point QP solver on the GNN step's own condensed QP (as left in
    b by the timed steps: 240 inputs, 200 state rows), against ADMM on it."""
    u = torch.empty_like(b["u"])
    info = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device=u.device)
    admm = lambda: plan.solve_box_qp(b["H"], b["g"], b["lb"], b["ub"], b["Ct"], None, b["dt"], b["u"], b["info"],
                                     settings=settings)
    out = {"workload": "condensed QP of the GNN step: 240 inputs, box bounds, 200 one-sided state rows"}
    for name, fn in [("admm", admm)] + [
            (f"ipm_tol_{tol:g}", (lambda tol=tol: plan.solve_qp_ipm(b["H"], b["g"], b["lb"], b["ub"], b["Ct"], None,
                                                                    b["dt"], u, info, tol=tol)))
            for tol in (1e-6, 1e-10)]:
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        inf = gn.qp_info(info if name != "admm" else b["info"])
        out[name] = {"ms": e0.elapsed_time(e1) / reps, "iters": inf.iters, "status": inf.status}
    out["ipm_vs_admm_rel"] = float((u - b["u"]).norm() / b["u"].norm().clamp_min(1e-30))
    return out


def tangent_rates(gn, plan, b, reps):
    """gnmpc_jvp and gnmpc_vjp on the step's GNN blocks (A, B of all 20 stages),
    timed with HIP events on the stream they run on; algorithmic HBM bytes per call
    (each block read once, each vector read or written once) over the average time."""
    import torch
    N, M, nu, nnz = plan.N, plan.M, plan.nu, plan.nnz
    A, B = b["A"], b["B"]
    dx = torch.randn(N, M, 6, device="cuda")
    du = torch.randn(N, nu, device="cuda")
    out = torch.empty(N, M, 6, device="cuda")
    gx = torch.empty(N, M, 6, device="cuda")
    gu = torch.empty(N, nu, device="cuda")
    blocks = 4 * (N * nnz * 36 + N * M * 6 * nu)
    vec = 4 * (N * M * 6)
    res = {}
    for name, fn, nbytes in (("jvp", lambda: plan.jvp(A, B, dx, du, out), blocks + 2 * vec + 4 * N * nu),
                             ("vjp", lambda: plan.vjp(A, B, out, gx, gu), blocks + 2 * vec + 4 * N * nu)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms": ms, "bytes": nbytes, "GB_per_s": nbytes / (ms * 1e-3) / 1e9,
                     "hbm_frac": nbytes / (ms * 1e-3) / 8e12}
    # reverse mode through the GNN's layers (forward pass recomputed, then the layers backwards)
    if getattr(plan, "model", None) == "gnn":
        for _ in range(3):
            plan.gnn_vjp(b["xhat"], b["uhat"], out, gx, gu)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.gnn_vjp(b["xhat"], b["uhat"], out, gx, gu)
        e1.record()
        torch.cuda.synchronize()
        res["gnn_vjp_reverse_mode"] = {"ms": e0.elapsed_time(e1) / reps,
                                       "note": "forward pass recomputed at the point, then L rounds backwards"}
    return res


def simulator_rate(torch, gn, wl, reps=3):
    """Trajectories of the nonlinear spring-damper chain for the surrogate's data set
    (4096 trajectories x 100 steps x 1000 nodes, FP32): time per call with HIP events
    on the stream it runs on, and the HBM rate of its algorithmic traffic (x0 and u
    read once, every state written once)."""
    B, T, M = 4096, 100, 1000
    S = wl.simulator_batch(B, T, M)
    plan = gn.Plan(M, S.nu, 1, 1, gn.F32)
    plan.graph_set(S.row_ptr, S.col, 1)
    plan.model_set_msd(S.msd, S.act)
    x0 = torch.tensor(S.x0, dtype=torch.float32, device="cuda")
    u = torch.tensor(S.u, dtype=torch.float32, device="cuda")
    X = torch.empty(B, T + 1, M, 6, dtype=torch.float32, device="cuda")
    plan.msd_simulate(x0, u, X)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.msd_simulate(x0, u, X)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 4 * (x0.numel() + u.numel() + X.numel())
    del X
    return {"workload": f"{B} trajectories x {T} steps, {M}-node 1-2-hop chain, cubic springs k3=50, gravity",
            "ms": ms, "node_steps_per_s": B * T * M / (ms * 1e-3), "bytes": nbytes,
            "GB_per_s": nbytes / (ms * 1e-3) / 1e9, "hbm_frac": nbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}


def closed_loop_rate(torch, gn, wl, model="msd", iters=50):
    """Algorithm 1 in closed loop on the 1000-node workload: each iteration is one
    gnmpc_rti_step of the controller (linearize, condense, QP, rollout of the
    optimum, shift; 200 obstacle rows) and one step of the spring-damper simulator
    as the plant, all on one stream with nothing copied to the host.  The
    controller's model is the plant's own spring-damper model (analytic
    Jacobians, model="msd") or the GNN (model="gnn": seeded random weights, which
    do not describe the plant, so the loop drifts and its QPs get harder; timing
    of the path only)."""
    P = wl.gnn1000_bf16(model=model)
    Pm = wl.gnn1000_bf16(model="msd")
    N, M, nu, n = P.N, P.M, P.nu, P.N * P.nu

    def t(a):
        return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()

    plan = gn.Plan(M, nu, N, P.rows.n, gn.F32)
    if model == "gnn":
        plan.graph_set(P.row_ptr, P.col, P.gnn.L)
        plan.model_set_gnn(P.gnn, P.act, dtype=gn.BF16)
    else:
        plan.graph_set(P.row_ptr, P.col, 1)
        plan.model_set_msd(P.msd, P.act)
    plan.rows_set(P.rows.node, P.rows.stage)
    plant = gn.Plan(M, nu, 1, 1, gn.F32)
    plant.graph_set(Pm.row_ptr, Pm.col, 1)
    plant.model_set_msd(Pm.msd, Pm.act)
    e = lambda *sh: torch.empty(*sh, device="cuda")
    b = dict(xhat=t(np.repeat(P.x0[None], N + 1, axis=0)), uhat=torch.zeros(N, nu, device="cuda"), x0=t(P.x0),
             Q=t(P.costs.Q), q=t(P.costs.q), R=t(P.costs.R), r=t(P.costs.r), rowC=t(P.rows.C), rowd=t(P.rows.d),
             lb=t(P.lb), ub=t(P.ub), A=e(N, plan.nnz, 6, 6), B=e(N, M, 6, nu), c=e(N, M, 6), H=e(n, n), g=e(n),
             Ct=e(P.rows.n, n), dt=e(P.rows.n), u=e(n), uc=None,
             info=torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda"))
    b["uc"] = b["dt"]
    xpred, X = e(N + 1, M, 6), e(1, 2, M, 6)
    settings = gn.default_admm_settings()

    def iteration():
        gn.rti_step(plan, b, xpred, settings=settings)
        plant.msd_simulate(b["x0"].view(1, M, 6), b["u"][:nu].view(1, 1, nu), X)
        b["x0"].copy_(X[0, 1])

    for _ in range(5):
        iteration()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        iteration()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    info = gn.qp_info(b["info"])
    return {"controller": "spring-damper model (analytic Jacobians)" if model == "msd" else
            "GNN Hd=128 L=3 BF16, random weights", "iterations": iters, "ms_per_iteration": ms,
            "iterations_per_s": 1e3 / ms, "qp_status_last": info.status, "qp_iters_last": info.iters,
            "qp_used_fp64_last": info.used_fp64}


def paper_model_rate(torch, gn, wl, iters=50):
    """The paper's own model on its robot's shape (interaction network, 4 nodes with
    2 neighbours, psi 4 x 50, phi 8 x 250, n_u = 6, N = 20, FP32): time of the
    linearization alone and of one GNN-MPC iteration (gnmpc_rti_step), HIP events on
    the stream both run on."""
    P = wl.trunk_inet()
    N, M, nu, n = P.N, P.M, P.nu, P.N * P.nu
    plan = gn.Plan(M, nu, N, 0, gn.F32)
    plan.graph_set(P.row_ptr, P.col, 1)
    plan.model_set_inet(P.inet)

    def t(a):
        return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()

    e = lambda *sh: torch.empty(*sh, device="cuda")
    b = dict(xhat=t(P.xhat), uhat=t(P.uhat), x0=t(P.x0), Q=t(P.costs.Q), q=t(P.costs.q), R=t(P.costs.R),
             r=t(P.costs.r), lb=t(P.lb), ub=t(P.ub), A=e(N, plan.nnz, 6, 6), B=e(N, M, 6, nu), c=e(N, M, 6),
             H=e(n, n), g=e(n), u=e(n), info=torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda"))
    xpred, xn, un = e(N + 1, M, 6), e(N + 1, M, 6), e(N, nu)

    def timed(fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / iters

    lin_ms = timed(lambda: plan.linearize(b["xhat"], b["uhat"], b["A"], b["B"], b["c"]))
    rti_ms = timed(lambda: gn.rti_step(plan, b, xpred, xn, un))
    qp_iters = gn.qp_info(b["info"]).iters
    # the iteration's condensed QP (120 inputs, box bounds) by the interior-point solver and by ADMM
    u_ipm = e(n)
    info_ipm = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda")
    ipm_ms = timed(lambda: plan.solve_qp_ipm(b["H"], b["g"], b["lb"], b["ub"], None, None, None, u_ipm, info_ipm,
                                             tol=1e-8))
    admm_ms = timed(lambda: plan.solve_box_qp(b["H"], b["g"], b["lb"], b["ub"], None, None, None, b["u"], b["info"]))
    return {"workload": "interaction network (psi 4x50, phi 8x250), 4 nodes x 2 neighbours, n_u=6, N=20, FP32",
            "linearize_ms": lin_ms, "rti_step_ms": rti_ms, "rti_steps_per_s": 1e3 / rti_ms,
            "qp_iters": qp_iters, "qp_ipm_ms": ipm_ms, "qp_ipm_iters": gn.qp_info(info_ipm).iters,
            "qp_admm_ms": admm_ms}


def training_rate(torch, gn, wl, iters=10):
    """One training step (loss, gradient with respect to every parameter, Adam) of
    the 1000-node GNN (Hd = 128, L = 3, FP32) on a batch of 20 samples from the
    spring-damper simulator; HIP events on the stream the step runs on."""
    M, B, T = 1000, 5, 4
    sim = wl.simulator_batch(B, T, M=M)
    S = B * T
    splan = gn.Plan(M, sim.nu, 1, 0, gn.F32)
    splan.graph_set(sim.row_ptr, sim.col, 1)
    splan.model_set_msd(sim.msd, sim.act)
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()
    X = torch.empty(B, T + 1, M, 6, device="cuda")
    splan.msd_simulate(t(sim.x0), t(sim.u), X)
    x, xn = X[:, :T].reshape(S, M, 6).contiguous(), X[:, 1:].reshape(S, M, 6).contiguous()
    u = t(sim.u).reshape(S, sim.nu)
    W = wl.gnn_weights(3, 128, 3, dt=sim.msd.dt)
    plan = gn.Plan(M, sim.nu, S, 0, gn.F32)
    plan.graph_set(sim.row_ptr, sim.col, 3)
    # training reads the plan's graph, sizes and inputs only (theta is its own FP32
    # array); the BF16 setting is the one whose Jacobian tables fit this graph
    plan.model_set_gnn(W, sim.act, dtype=gn.BF16)
    n, wb = plan.gnn_train_sizes()
    theta = t(gn.gnn_flat(W))
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    grad, m, v = (torch.zeros(n, device="cuda") for _ in range(3))
    loss = torch.empty(1, device="cuda")
    O = [1, 1, 1, 1, 1, 1]

    def step(k):
        plan.gnn_loss_grad(theta, x, u, xn, O, 1e-6, ws, loss, grad)
        gn.adam_step(theta, grad, m, v, k, 1e-3)

    step(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(iters):
        step(k + 2)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    return {"workload": f"GNN Hd=128 L=3, {M}-node chain, {S} samples per step, FP32", "params": n,
            "ms_per_step": ms, "samples_per_s": S * 1e3 / ms, "node_samples_per_s": S * M * 1e3 / ms}


def bench_batch(args, torch, gn, wl):
    """K uneven instances (one shared BF16 GNN, Hd=128, L=2) per batched step,
    captured once as a HIP graph and replayed; the same instances one after
    another on one stream are timed beside it."""
    probs = wl.batch_instances(args.batch, seed=4)

    def t(a):
        return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()

    setups = []
    for P in probs:
        plan = gn.Plan(P.M, P.nu, P.N, 1, gn.F32)
        plan.graph_set(P.row_ptr, P.col, P.gnn.L)
        plan.model_set_gnn(P.gnn, P.act, dtype=gn.BF16)
        n = P.N * P.nu
        b = dict(xhat=t(P.xhat), uhat=t(P.uhat), x0=t(P.x0), Q=t(P.costs.Q), q=t(P.costs.q), R=t(P.costs.R),
                 r=t(P.costs.r), lb=t(P.lb), ub=t(P.ub),
                 A=torch.empty(P.N, plan.nnz, 6, 6, device="cuda"), B=torch.empty(P.N, P.M, 6, P.nu, device="cuda"),
                 c=torch.empty(P.N, P.M, 6, device="cuda"), H=torch.empty(n, n, device="cuda"),
                 g=torch.empty(n, device="cuda"), u=torch.empty(n, device="cuda"),
                 info=torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda"))
        setups.append((plan, b))
    descs = [gn.step_desc(plan, b) for plan, b in setups]

    def sequential():
        for plan, b in setups:
            plan.linearize(b["xhat"], b["uhat"], b["A"], b["B"], b["c"])
            plan.condense(b["A"], b["B"], b["c"], b["x0"], b["Q"], b["q"], b["R"], b["r"], None, None, b["H"],
                          b["g"], None, None)
            plan.solve_box_qp(b["H"], b["g"], b["lb"], b["ub"], None, None, None, b["u"], b["info"])

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    el_b = timed(lambda: gn.step_batched(descs))
    el_s = timed(sequential)
    K = len(setups)
    status = [gn.qp_info(b["info"]).status for _, b in setups]
    out = {
        "metric": "batched condensed MPC instance-steps/s (uneven GNN instances)",
        "value": args.steps * K / el_b,
        "unit": "instance-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_batch": el_b / args.steps * 1e3,
        "higher_is_better": True,
        "dtype": "bf16+f32",
        "data": "synthetic",
        "config": {"workload": f"{K} instances: M ~ U{{50..1000}}, N ~ U{{10..30}}, 2-4 actuated nodes, "
                               "shared GNN Hd=128 L=2 (BF16 MLPs), FP32 condensing, ADMM box QP, no state rows",
                   "instances": K, "total_nodes": int(sum(P.M for P in probs)),
                   "total_node_stages": int(sum(P.M * P.N for P in probs))},
        "sequential_instance_steps_per_s": args.steps * K / el_s,
        "qp_solved": int(sum(1 for s_ in status if s_ == gn.QP_SOLVED)),
        "timing": "HIP graph replay (batched: one captured step_batched call; sequential: the same "
                  "instances one after another on one stream)",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
