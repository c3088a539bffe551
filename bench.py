"""Benchmark: numeric assembly throughput of the nonlocal P1 stiffness matrix.

One step = one nla_assemble (pair quadrature, segmented sum into the CSR of
D, extraction of A, load vector) of the 8-arc-cap retriangulated-ball
workload on the jittered h = delta/8 mesh (delta = 0.1, constant kernel,
7-point outer x 16-point inner rules, FP64), inputs resident on the GPU.
The same line carries the learned-cap comparison on that mesh (network
trained on the GPU first, outside the timed region): FP32 learned-cap
assembly time against this FP64 exact-cap time, and the solutions' L2
differences.  Prints one JSON line.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-learned]
       [--config c2|c3|c4|c5|paper]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "element-pair quadratures/s + assembly time, learned/FP32 vs FP64 plain at L2 err"
FP64_PEAK_TFLOPS = 78.6    # MI355X vector FP64 (published)
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (published; packed FP32, which this build does not use)
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix cores (published, no sparsity)
LEARNED_TARGET_SPEEDUP = 3.0
LEARNED_TARGET_L2 = 1e-4

# Algorithmic FP64 operations of the pair kernel per unit of work (counted
# from the arithmetic the method needs per unit; an FMA counts 2, sqrt, div
# and transcendental calls count 1).  With an inner rule exact for quadratics
# (constant kernel) a partial item is integrated through its boundary: the
# counter "subtriangles" then counts boundary segments.
COST = dict(item=15,           # classification: 3 squared vertex distances
            whole=6,           # whole item: outer-weight sums and S0
            partial=114,       # polygon walk (3 edge quadratics, roots) + owner accumulation
            subtriangle=81,    # inner rule on one subtriangle from its vertex basis values (area, S1, S2),
                               # symmetric-rule form
            cap=30,            # arc span, chord midpoint, rotation by half angles
            arc_point=16,      # one rotated arc point and its basis values
            pair=45)           # per-pair accumulator set-up and output
COST_BOUNDARY = dict(item=15, whole=6,
                     partial=114 + 60,   # walk + owner accumulation + moments to S0, S1, S2
                     subtriangle=26,     # one boundary segment: cross product, first and second moment terms
                     cap=30,             # arc span, rotation by half angles
                     arc_point=6,        # one rotated arc point
                     pair=45)


# A deep pair (every item whole, R35) is not classified item by item in the
# pair kernel: the plan's vertex-distance test selects it and the kernel adds
# its inner element's area into the element sum and into the row-block
# columns of its three nodes.
COST_DEEP_PAIR = 4


def algorithmic_flops(info, n_pairs, ncap, cost=COST, nq=7):
    """Work of the pair kernel per launch: the per-unit costs above times the
    plan's counters.  Deep pairs count COST_DEEP_PAIR each instead of their
    items' classification (their items appear in the whole count)."""
    it = info["items"]
    n_deep = info.get("n_deep", 0)
    whole = it["whole"] - n_deep * nq
    items = whole + it["partial"] + it["empty"]
    return (cost["item"] * items + cost["whole"] * whole + cost["partial"] * it["partial"] +
            cost["subtriangle"] * info["subtriangles"] + cost["cap"] * info["caps"] +
            cost["arc_point"] * info["caps"] * max(ncap - 1, 0) + cost["pair"] * (n_pairs - n_deep) +
            COST_DEEP_PAIR * n_deep)


def method_point_flops(info, n_in, ncap):
    """The method's work with every region retriangulated and every partial
    subtriangle integrated point by point (the per-unit costs of the method:
    15 flops to classify an item and 31 to accumulate it; a partial item's
    polygon walk 66; a cap's arc points 14 each; a subtriangle 10 plus 40 per
    inner point; whole items by their closed form, 0 per point).  With a rule
    exact for quadratics and the constant kernel the pair kernel integrates
    the same regions through their boundaries (R27), which needs a fraction of
    this: the ratio of the two is how much the boundary form saves.  The
    subtriangle count follows from the kernel's counters: a partial item with
    n polygon vertices and c caps has n - 2 + ncap c subtriangles and
    n - c + ncap c boundary segments."""
    it = info["items"]
    items = it["whole"] + it["partial"] + it["empty"]
    subtri = info["subtriangles"] + info["caps"] - 2 * it["partial"]
    return 46 * items + 66 * it["partial"] + 14 * ncap * info["caps"] + (10 + 40 * n_in) * subtri


def fp32_point_flops(info, n_pairs, n_in, ncap, frac):
    """FP32 pair kernel with the point rule (fractional kernel): per inner point
    61 flops (map 12, basis 18, distance 3, weight 3, sums 25) and, with the
    fractional kernel, 2 transcendentals (log2, exp2); per subtriangle 20 set-up
    flops; whole items integrate all of E_k' by the rule; classification 15
    and accumulation 30 per item; polygon walk 114; cap 30 + 16 per arc point;
    pair 45.  Returns (flops, transcendentals)."""
    it = info["items"]
    items = it["whole"] + it["partial"] + it["empty"]
    tris = it["whole"] + info["subtriangles"]
    flops = (15 * items + 30 * (it["whole"] + it["partial"]) + 114 * it["partial"] + (20 + 61 * n_in) * tris +
             (30 + 16 * max(ncap - 1, 0)) * info["caps"] + 45 * n_pairs)
    return flops, (2 * n_in * tris if frac else 0)


def l2_error(mesh, U, u_exact):
    """||u - u_h|| on Omega with the degree-5 7-point rule (exact for quadratic u)."""
    from workloads import get_rule
    r = get_rule("dunavant7")
    ks = np.nonzero(mesh.tri_in_omega)[0]
    V = mesh.xy[mesh.tri[ks]]                       # [n,3,2]
    a2 = np.abs((V[:, 1, 0] - V[:, 0, 0]) * (V[:, 2, 1] - V[:, 0, 1]) -
                (V[:, 1, 1] - V[:, 0, 1]) * (V[:, 2, 0] - V[:, 0, 0]))
    X = np.einsum("qa,nac->nqc", r.lam, V)
    uh = np.einsum("qa,na->nq", r.lam, U[mesh.tri[ks]])
    e = (u_exact(X[..., 0], X[..., 1]) - uh) ** 2
    return float(math.sqrt(np.sum(e * r.w[None, :] * a2[:, None])))


def source_digest():
    """Digest of every source the FP64 pair kernel is compiled from, and of
    the plan that orders its launch: counters taken on other source are not
    reported."""
    h = hashlib.sha256()
    for name in ("nla_numeric.hip", "nla_device.hpp", "nla_internal.hpp", "nla_plan.hip"):
        with open(os.path.join(ROOT, "paper_2005_10775_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    with open(os.path.join(ROOT, "include", "nlasm.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel, digest):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the summary is missing or was taken on other source."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    e = d.get(kernel)
    if not e or e.get("source_digest") != digest:
        return None
    return e.get("bytes_per_launch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads():
    """Threads this job may use on the host: the cores it is bound to, capped
    by OMP_NUM_THREADS when that is set (the host's share for this job)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_baseline(mesh, prob, sample_elems, sample_elems_1t):
    """The FP64 oracle (pair search by an all-pairs loop with a conservative
    reject, then every pair's local blocks) timed on a bounded sample of outer
    elements with all their pairs: on every thread this job may use, and on
    one thread over a smaller sample."""
    import oracle
    oracle.build(force=False)
    op = oracle.OracleProblem(mesh, prob)
    K = mesh.n_triangles
    threads = _host_threads()

    def run(n, nthreads):
        n = min(n, K)
        k0 = (K - n) // 2        # a band of whole mesh rows through the middle (layer and Omega)
        t0 = time.perf_counter()
        total, _ = oracle.blocks_range(op, k0, k0 + n, nthreads)
        dt = time.perf_counter() - t0
        return total / dt, "outer elements [%d, %d) of %d with all their pairs (%d pairs), %.2f s wall" % (
            k0, k0 + n, K, total, dt)

    v1, s1 = run(sample_elems_1t, 1)
    vn, sn = run(sample_elems, threads)
    return {"value": vn, "unit": "pairs/s", "cores": threads, "kind": "oracle", "sample": sn,
            "single_thread": {"value": v1, "sample": s1},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "what": "pair search + local blocks (no CSR merge), FP64, gcc -O2 -ffp-contract=off, OpenMP over "
                    "outer elements"}


def bench_batch(args):
    """64 uneven instances: one persistent launch + hipGraph replay (autotuned)
    against the same instances assembled one after the other."""
    import torch
    from paper_2005_10775_amd import Batch
    from workloads import batch_instances, manufactured
    inst = batch_instances()
    u, f = manufactured("quadratic")
    t0 = time.perf_counter()
    b = Batch(inst)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    fs, gs = [], []
    for (mesh, prob), plan in zip(b.instances, b.plans):
        xq = plan.outer_points()
        fs.append(f(xq[..., 0], xq[..., 1]).contiguous())
        gs.append(torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda"))
    tune = b.autotune()
    stream = torch.cuda.current_stream()

    def timed(mode):
        for _ in range(args.warmup):
            b.assemble(mode, fs, gs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            b.assemble(mode, fs, gs)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms = timed(1)
    ms_seq = timed(0)
    info = b.info()
    # work of the regular pairs over all instances (each plan's counters); the
    # batched step also integrates the singular pairs, so this fraction of the
    # FP32 peak is a lower bound for the pair kernels
    from workloads import get_rule
    flops = trans = 0
    for (mesh, prob), plan in zip(b.instances, b.plans):
        pi = plan.info()
        ncap = prob.cap_edges if prob.ball == "retri" else 0
        if prob.kernel == "fractional":
            fl, tr = fp32_point_flops(pi, pi["n_pairs"], get_rule(prob.inner).n, ncap, True)
        else:
            fl, tr = algorithmic_flops(pi, pi["n_pairs"], ncap, COST, get_rule(prob.outer).n), 0
        flops += fl
        trans += tr
    ach = flops / (ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "whole batched step (pair kernels + singular pairs + sums)",
                "achieved": ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS,
                "traffic": None, "flops_per_launch": flops, "transcendentals_per_launch": trans,
                "kernel_ms": ms}
    pairs = info["total_pairs"]
    ks = [m.n_triangles for m, _ in inst]
    return {"metric": METRIC, "value": pairs / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "c4: 64 uneven instances (delta in [0.05,0.2], h = delta/k, k in 2..8; "
                                   "half constant / half s=0.4 kernel; barycenter 7x7 and 8-arc retri 7x16), FP32",
                       "instances": len(inst), "total_pairs": pairs, "total_elements": info["total_elements"],
                       "near_pairs": info["total_near"], "K_min": min(ks), "K_max": max(ks)},
            "batched_ms": ms, "sequential_ms": ms_seq, "sequential_value": pairs / (ms_seq * 1e-3),
            "speedup_vs_sequential": ms_seq / ms, "autotune": {"chunk": tune["chunk"], "grid": tune["grid"]},
            "plan_ms": plan_ms, "roofline": roofline}


def _timed_assembly(plan, fo, g, steps, warmup):
    """Milliseconds per assembly over `steps` assemblies with no phase events
    among them, then the per-phase times from a second pass of `steps`
    assemblies with the plan's phase events on."""
    import torch
    for _ in range(warmup):
        plan.assemble(fo, g)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.assemble(fo, g)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan.set_timing(steps)
    for _ in range(steps):
        plan.assemble(fo, g)
    torch.cuda.synchronize()
    phase, n = plan.timings()
    plan.set_timing(0)
    return ms, phase


def _solve(plan, mesh, u):
    U, its, rel = plan.cg(plan.load(), rtol=1e-12)
    Ufull = u(mesh.xy[:, 0], mesh.xy[:, 1]).copy()
    Ufull[plan.free_nodes().cpu().numpy()] = U.cpu().numpy()
    return Ufull, (its, rel)


def _l2_diff(mesh, U1, U2):
    return l2_error(mesh, U1 - U2, lambda x, y: 0.0 * x)


def train_network(args):
    """The learned-cap network trained on the GPU with the workload's recipe
    (samples of the h = delta/8 family labelled by the FP64 8-arc caps)."""
    import torch
    from paper_2005_10775_amd import Mlp
    from workloads.learned import TRAIN
    t0 = time.perf_counter()
    feat, lab = Mlp.samples(int(TRAIN["samples"] / 0.17), TRAIN["seed"], L=TRAIN["L"], jitter=TRAIN["jitter"],
                            band=TRAIN["band"], cap_edges=TRAIN["cap_edges"])
    feat, lab = feat[:TRAIN["samples"]].contiguous(), lab[:TRAIN["samples"]].contiguous()
    torch.cuda.synchronize()
    t_samples = time.perf_counter() - t0
    net = Mlp(seed=TRAIN["seed"])
    t0 = time.perf_counter()
    log = net.train(feat, lab, epochs=args.epochs, batch=TRAIN["batch"], lr=TRAIN["lr"], seed=TRAIN["seed"])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    fh, lh = Mlp.samples(400_000, TRAIN["seed"], first=10 ** 9)
    w, sc = net.get_weights()
    pred = net.forward(fh) * sc
    held = float(torch.sqrt(torch.mean((pred - lh) ** 2)) / torch.sqrt(torch.mean(lh ** 2)))
    info = {"samples": int(feat.shape[0]), "epochs": args.epochs, "batch": TRAIN["batch"], "samples_s": t_samples,
            "train_s": t_train, "loss_first": log[0], "loss_last": log[-1], "heldout_rel_rms": held, "scale": sc}
    return net, feat, info


def network_roofline(net, feat, n_items, steps):
    """k_mlp_fwd alone on n_items inputs (the count one learned assembly
    routes), timed with HIP events on the launch stream: 2 (128*128 + 3*128)
    matrix-core flops per item against the dense bf16 peak (the 6 -> 128 first
    layer and the 256 activations run on the vector unit and are not counted)."""
    import torch
    n = min(n_items, feat.shape[0])
    if n <= 0:
        return None
    x = feat[:n].contiguous()
    stream = torch.cuda.current_stream()
    for _ in range(3):
        net.forward(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        net.forward(x)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    flops = n * 2.0 * (128 * 128 + 3 * 128)
    ach = flops / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": "k_mlp_fwd", "achieved": ach, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / BF16_PEAK_TFLOPS, "traffic": None, "flops_per_launch": flops, "kernel_ms": ms,
            "items": n}


def learned_compare(args, mesh, p64, man, fp64_ms, U_exact):
    """The learned-cap form on the headline mesh against the FP64 exact-cap
    assembly already timed (fp64_ms, solution U_exact): train, then time the
    FP32 learned assembly; solve; compare with the exact-cap and the FP32
    no-cap solutions (what the network gains)."""
    import torch
    from dataclasses import replace
    from paper_2005_10775_amd import Plan
    from workloads import manufactured
    u, f = manufactured(man)
    net, feat, tinfo = train_network(args)
    res = {}
    sols = {}
    for name, prob in (("fp32_learned", replace(p64, precision="learned")),
                       ("fp32_nocaps", replace(p64, precision="fp32", cap_edges=0))):
        plan = Plan(mesh, prob, mlp=net if prob.precision == "learned" else None)
        xq = plan.outer_points()
        fo = f(xq[..., 0], xq[..., 1]).contiguous()
        g = torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda")
        ms, phase = _timed_assembly(plan, fo, g, args.steps, args.warmup)
        info = plan.info()
        sols[name], _ = _solve(plan, mesh, u)
        res[name] = {"ms": ms, "phase_ms": phase, "items": info["items"]}
        plan.close()
    L = res["fp32_learned"]
    d_learn = _l2_diff(mesh, sols["fp32_learned"], U_exact)
    d_nocap = _l2_diff(mesh, sols["fp32_nocaps"], U_exact)
    speedup = fp64_ms / L["ms"]
    return {"workload": "c5: the headline mesh and rules; caps outside the 0.02 delta band and inside the "
                        "network's training domain from a 6-128-128-3 tanh-GELU network (bf16 matrix cores), "
                        "the rest exact; FP32 compensated sums",
            "fp64_exactcap_ms": fp64_ms, "fp32_learned_ms": L["ms"], "fp32_nocaps_ms": res["fp32_nocaps"]["ms"],
            "speedup_vs_fp64_exactcap": speedup, "target_speedup": LEARNED_TARGET_SPEEDUP,
            "speedup_target_met": speedup >= LEARNED_TARGET_SPEEDUP,
            "l2_learned_vs_exactcap": d_learn, "l2_nocaps_vs_exactcap": d_nocap, "target_l2": LEARNED_TARGET_L2,
            "l2_target_met": d_learn <= LEARNED_TARGET_L2,
            "gain_vs_nocaps": d_nocap / d_learn if d_learn > 0 else None,
            "routed_items": L["items"]["learned"], "partial_items": L["items"]["partial"],
            "network_phase_ms": L["phase_ms"]["mlp"], "learned_phase_ms": L["phase_ms"],
            "network_roofline": network_roofline(net, feat, L["items"]["learned"], args.steps),
            "train": tinfo}


def bench_learned(args):
    """--config c5: the FP64 exact-cap assembly of the headline mesh, then the
    learned comparison; the line's value is the learned form's pairs/s."""
    import torch
    from paper_2005_10775_amd import Plan
    from workloads import make_config, manufactured
    mesh, p64, man = make_config("c2")
    u, f = manufactured(man)
    plan = Plan(mesh, p64)
    xq = plan.outer_points()
    fo = f(xq[..., 0], xq[..., 1]).contiguous()
    g = torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda")
    ms64, _ = _timed_assembly(plan, fo, g, args.steps, args.warmup)
    n_pairs = plan.info()["n_pairs"]
    U64, _ = _solve(plan, mesh, u)
    plan.close()
    cmp = learned_compare(args, mesh, p64, man, ms64, U64)
    ms = cmp["fp32_learned_ms"]
    return {"metric": METRIC, "value": n_pairs / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
            "config": {"workload": cmp["workload"], "n_pairs": n_pairs},
            "roofline": cmp["network_roofline"], "learned": cmp}


PAPER_BALLS = ("exactcaps", "approxcaps", "nocaps", "barycenter", "overlap", "shifted", "barynocaps",
               "baryapproxcaps", "analyticcaps")


def bench_paper(args):
    """The workloads of Sec. 8 (grid (a), delta = 0.1, u = x1^2 x2 + x2^2, the
    paper's rules and outer-rule switch) at the paper's finest grid
    h = 0.00625 (K = 73,728): per ball, the FP64 assembly time, pairs, solution
    L2 error next to the printed one, and the time relative to the slowest ball
    (the paper's 'time [%]' column is relative to its slowest run, exactcaps at
    this h).  "analyticcaps" is the exact ball (caps in closed form), which the
    paper recommends without running it."""
    import torch
    from paper_2005_10775_amd import Plan
    from workloads import manufactured, paper_workload
    here = os.path.dirname(os.path.abspath(__file__))
    printed = {}
    for name in ("paper_sec8_table.json", "paper_sec8_other_balls.json"):
        with open(os.path.join(here, "tests", "golden", name)) as fh:
            tab = json.load(fh)
        for ball, vals in tab["l2"].items():
            printed[ball] = dict(zip(tab["h"], vals))
    h = args.paper_h
    rows = {}
    balls = args.paper_balls.split(",") if args.paper_balls else PAPER_BALLS
    for ball in balls:
        if ball not in PAPER_BALLS:
            raise SystemExit("unknown ball %r: choose from %s" % (ball, ", ".join(PAPER_BALLS)))
        mesh, prob, man = paper_workload(h, ball)
        u, f = manufactured(man)
        t0 = time.perf_counter()
        plan = Plan(mesh, prob)
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t0) * 1e3
        xq = plan.outer_points()
        fo = f(xq[..., 0], xq[..., 1]).contiguous()
        g = torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda")
        ms, phase = _timed_assembly(plan, fo, g, args.steps, args.warmup)
        info = plan.info()
        U, (its, _) = _solve(plan, mesh, u)
        l2 = l2_error(mesh, U, u)
        rows[ball] = {"assembly_ms": ms, "pairs_ms": phase["pairs"], "plan_ms": plan_ms,
                      "n_pairs": info["n_pairs"], "pairs_per_s": info["n_pairs"] / (ms * 1e-3),
                      "items": info["items"], "l2": l2, "l2_printed": printed.get(ball, {}).get(h), "cg_iters": its}
        print("paper %-15s h=%g K=%d pairs=%d assembly %.3f ms L2 %.3e (printed %s)" % (
            ball, h, mesh.n_triangles, info["n_pairs"], ms, l2, rows[ball]["l2_printed"]), file=sys.stderr,
            flush=True)
        del plan
        torch.cuda.empty_cache()
    slow = max(r["assembly_ms"] for r in rows.values())
    for r in rows.values():
        r["time_pct"] = 100.0 * r["assembly_ms"] / slow
    ms = sum(r["assembly_ms"] for r in rows.values())
    n = sum(r["n_pairs"] for r in rows.values())
    return {"metric": "paper Sec. 8 workloads: FP64 assembly time per ball", "value": n / (ms * 1e-3),
            "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "Sec. 8 grid (a): delta=0.1 h=%g K=%d, balls %s, 7/4-pt outer with switch "
                                   "(4-pt for shifted, barycenter support), 3-pt inner" % (
                                       h, mesh.n_triangles, ",".join(balls))},
            "balls": rows}


def pair_roofline(prob, info, n_pairs, phase):
    """Roofline line of the configuration's dominant kernel, the pair
    quadrature: FP64 boundary form (constant kernel, intersection ball, rule
    exact for quadratics), otherwise the point-rule kernels (FP64 or FP32)."""
    from workloads import get_rule
    ri = get_rule(prob.inner)
    ncap = prob.cap_edges if prob.ball == "retri" else 0
    nq = get_rule(prob.outer).n
    q2 = abs(ri.w.sum() - 0.5) < 1e-14 and all(abs((ri.w * ri.lam[:, i]).sum() - 1 / 6) < 1e-14 for i in range(3))
    t = phase["pairs"] * 1e-3
    if prob.precision == "fp64":
        boundary = prob.ball == "retri" and q2 and prob.kernel == "constant"
        flops = algorithmic_flops(info, n_pairs, ncap, COST_BOUNDARY if boundary else COST, nq)
        ach = flops / t / 1e12
        digest = source_digest()
        out = {"bound": "alu", "kernel": "k_pairs_const_fp64", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
               "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
               "traffic": traffic_from_profile("k_pairs_const_fp64", digest) if boundary else None,
               "flops_per_launch": flops, "kernel_ms": phase["pairs"],
               "cost_model": "boundary form (partial items by boundary moments)" if boundary else "point rule"}
        if boundary:
            mf = method_point_flops(info, ri.n, ncap)
            out["method_point_flops"] = mf
            out["method_point_frac"] = mf / t / 1e12 / FP64_PEAK_TFLOPS
        return out
    flops, trans = fp32_point_flops(info, n_pairs, ri.n, ncap, prob.kernel == "fractional")
    ach = flops / t / 1e12
    return {"bound": "alu", "kernel": "k_pairs_fp32", "achieved": ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP32_PEAK_TFLOPS, "traffic": None, "flops_per_launch": flops,
            "transcendentals_per_launch": trans,
            "transcendentals_per_s": trans / t if trans else 0.0, "kernel_ms": phase["pairs"],
            "note": "FP32 peak is the packed rate; packed FP32 is disabled in this build, so unpacked FP32 "
                    "issues at half of it"}


def bench_plan(args):
    """Wall time of plan creation (pair build, pattern, codes, processing order):
    the first plan in the process also loads the library's code objects and
    warms the allocator, the later ones show the steady cost.  A kernel and
    runtime-call trace of this run splits the time further."""
    import torch
    from paper_2005_10775_amd import Plan
    from workloads import make_config
    mesh, prob, _ = make_config(args.config)
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        plan = Plan(mesh, prob)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        info = plan.info()
        plan.close()
    return {"config": args.config, "plan_first_ms": times[0], "plan_later_ms": times[1:],
            "n_pairs": info["n_pairs"], "nnz_full": info["nnz_full"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="c2: leave out the learned-cap comparison")
    ap.add_argument("--duffy", type=int, default=0, help="override the singular-pair rule order")
    ap.add_argument("--cpu-sample", type=int, default=12288, help="outer elements in the CPU-baseline sample")
    ap.add_argument("--cpu-sample-1t", type=int, default=3072,
                    help="outer elements in the single-thread CPU-baseline sample")
    ap.add_argument("--epochs", type=int, default=20, help="learned caps: training epochs")
    ap.add_argument("--paper-h", type=float, default=0.00625, help="paper: grid spacing of the Sec. 8 workloads")
    ap.add_argument("--paper-balls", default="", help="paper: comma-separated subset of the balls (default: all)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-MiB device buffer 3 times (reference kernel for HBM counters)")
    ap.add_argument("--plan-only", action="store_true",
                    help="time plan creation only: the first plan of the process, then two more of the same mesh")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU; splitting the outer elements over several GPUs is not built, "
              "so run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_10775_amd import Plan
    from workloads import make_config, manufactured

    torch.cuda.set_device(0)
    if args.plan_only:
        print(json.dumps(bench_plan(args)))
        return
    if args.config == "c4":
        print(json.dumps(bench_batch(args)))
        return
    if args.config == "c5":
        print(json.dumps(bench_learned(args)))
        return
    if args.config == "paper":
        print(json.dumps(bench_paper(args)))
        return
    mesh, prob, man = make_config(args.config)
    if args.duffy:
        from dataclasses import replace
        prob = replace(prob, duffy_order=args.duffy)
    u, f = manufactured(man)
    t0 = time.perf_counter()
    plan = Plan(mesh, prob)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    xq = plan.outer_points()
    fo = f(xq[..., 0], xq[..., 1]).contiguous()
    g = torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda")
    # K timed steps with no phase events among them, then K more with the
    # plan's per-phase HIP events on its launch stream (the pair kernel's
    # duration for the roofline line comes from these)
    ms, phase = _timed_assembly(plan, fo, g, args.steps, args.warmup)
    info = plan.info()
    n_pairs = info["n_pairs"]
    value = n_pairs / (ms * 1e-3)
    roofline = pair_roofline(prob, info, n_pairs, phase)

    # validation solve and L2 error (outside the timed region)
    Ufull, (its, rel) = _solve(plan, mesh, u)
    l2 = l2_error(mesh, Ufull, u)

    out = {"metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if prob.precision == "fp64" else "f32", "data": "synthetic",
           "config": {"workload": "%s: delta=%g h=%g K=%d %s%s %sx%s %s kernel" % (
               args.config, prob.delta, mesh.h, mesh.n_triangles, prob.ball,
               "-%d-arc caps" % prob.cap_edges if prob.ball == "retri" else "", prob.outer, prob.inner, prob.kernel),
               "n_pairs": n_pairs, "nnz_full": info["nnz_full"], "n_free": info["n_free"],
               "jitter": mesh.meta.get("jitter", 0.0)},
           "assembly_ms": ms, "plan_ms": plan_ms, "phase_ms": phase,
           "items": info["items"], "n_deep": info["n_deep"], "subtriangles": info["subtriangles"],
           "caps": info["caps"], "l2_err": l2, "cg": {"iters": its, "relres": rel},
           "roofline": roofline, "source_digest": source_digest()}
    if args.config == "c2" and not args.no_learned:
        plan.close()
        torch.cuda.empty_cache()
        out["learned"] = learned_compare(args, mesh, prob, man, ms, Ufull)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, prob, args.cpu_sample, args.cpu_sample_1t)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = n
    print(json.dumps(out))


if __name__ == "__main__":
    main()
