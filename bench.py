#!/usr/bin/env python3
"""Benchmark of the MI355X FMM hot path on one GPU.

One step = the whole path on one synthetic point set: plan (root cube, keys, sort,
octree, dual traversal, operator grouping), forward evaluation (P2M, M2M, M2L, L2L,
L2P, P2P, un-permute), a rebuilt plan and the adjoint (the same FMM with charges
w = dL/dphi, plus dL/dx = w grad phi + q grad psi).  `value` is whole-step
particles/s (forward + adjoint); the forward-only and evaluation-only rates are
reported beside it.  Inputs are resident in device memory before timing starts.

Prints one JSON line.  Accuracy is checked after the timed region against the exact
FP64 direct sum on 1000 sampled targets (the result counts only at <= 1e-4).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import hashlib  # noqa: E402

import numpy as np  # noqa: E402

MFMA_FP32_PEAK_TFLOPS = 157.3      # MI355X dense FP32 MFMA
MFMA_FP16_PEAK_TFLOPS = 2500.0     # MI355X dense FP16 MFMA
# HBM bytes of one M2L launch on the uniform-1M workload (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0,
# factors from a 1 GiB plain copy), measured with rocprofv3 on the M2L kernel source whose
# sha256 prefix is given (the text of k_gemm in eval.hip) and on the plan's grouping (its
# entry and work-item counts); reported only while both are unchanged.
M2L_TRAFFIC = {"kernel_sha256": "6a28cdac88939087", "workload": "uniform-1M", "p": 10, "theta": 0.4,
               "entries": 285444, "work_items": 4556, "bytes": 15.35e9}
VALU_FP32_PACKED_PEAK_TFLOPS = 157.3   # MI355X FP32 vector with packed (2-wide) FMA
VALU_FP32_PEAK_TFLOPS = 78.6           # 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz, packed FP32 not used
P2P_ISSUE_PEAK_TFLOPS = 47.6           # the same lanes at 16.5 issue slots per 20-flop interaction


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform-1M")
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "mixed"])
    ap.add_argument("--m2l-tol", type=float, default=0.0,
                    help="variable-order M2L tolerance (0: dense operators, the configuration's method)")
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--skip-accuracy", action="store_true")
    ap.add_argument("--accuracy-sweep", default=None, metavar="P_LIST",
                    help="instead of the benchmark line: error against the direct sum and throughput for each "
                         "order in P_LIST (e.g. 2,4,6,8,10,12) at theta 0.4 and 0.5, one JSON line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    return ap.parse_args()


def m2l_kernel_sha():
    """sha256 prefix of the M2L kernel's source text (the k_gemm template in eval.hip)."""
    src = open(os.path.join(ROOT, "paper_1602_02244_amd", "csrc", "eval.hip")).read()
    a = src.index("template <int P, bool ADD, bool MASKED")
    b = src.index("// ---", a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def m2l_roofline(precision, m2l_tflops, traffic):
    """The M2L kernel against the MFMA peak of the type it computes in.  The split-FP16
    form runs three FP16 products (hi hi, hi lo, lo hi) per algorithmic one."""
    if precision == "mixed":
        achieved = 3.0 * m2l_tflops
        return {"kernel": "k_m2l_f16 (split-FP16 MFMA grouped GEMM, 3 products)", "bound": "mfma",
                "achieved": achieved, "peak": MFMA_FP16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / MFMA_FP16_PEAK_TFLOPS,
                "fp32_equivalent": m2l_tflops, "traffic": None}
    return {"kernel": "k_m2l (FP32 MFMA grouped GEMM)", "bound": "mfma", "achieved": m2l_tflops,
            "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": m2l_tflops / MFMA_FP32_PEAK_TFLOPS,
            "traffic": traffic}


def m2l_traffic(workload, p, theta, st):
    t = M2L_TRAFFIC
    if (m2l_kernel_sha() == t["kernel_sha256"] and (workload, p, theta) == (t["workload"], t["p"], t["theta"])
            and (st["m2l_entries"], st["m2l_work_items"]) == (t["entries"], t["work_items"])):
        return t["bytes"]
    return None


def direct_reference(xt, qt, targets, chunk=None):
    """Exact potential and gradient at the sampled targets: plain FP64 direct summation
    (torch on the device; skips the target itself and coincident points)."""
    import torch
    x = xt.double()
    q = qt.double()
    if chunk is None:
        chunk = max(1, min(64, int(2e8 // x.shape[0])))     # bounds the pairwise temporaries
    phi = np.empty(len(targets))
    grad = np.empty((len(targets), 3))
    for c0 in range(0, len(targets), chunk):
        idx = torch.as_tensor(np.asarray(targets[c0:c0 + chunk]), device=x.device)
        d = x[idx][:, None, :] - x[None, :, :]
        r2 = (d * d).sum(-1)
        rinv = torch.where(r2 > 0, r2.rsqrt(), torch.zeros_like(r2))
        phi[c0:c0 + chunk] = (rinv * q).sum(1).cpu().numpy()
        grad[c0:c0 + chunk] = (-(rinv ** 3 * q)[:, :, None] * d).sum(1).cpu().numpy()
    return phi, grad


def accuracy_sweep(args, xt, qt, wt, n, ncrit, reps=5):
    """Error against the exact direct sum (1000 sampled targets) and throughput of the forward
    (plan + eval) and forward + adjoint (plan + eval + plan + adjoint) steps, per (theta, p)."""
    import torch
    from paper_1602_02244_amd import FMM, inputs
    samp = inputs.sample_targets(n, 1000)
    dphi, dgrad = direct_reference(xt, qt, samp)
    rows = []
    for theta in (0.4, 0.5):
        for p in (int(v) for v in args.accuracy_sweep.split(",")):
            FMM(xt, ncrit, p, theta, args.precision).close()          # operator tables for this (p, theta)
            fwd, step = [], []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan = FMM(xt, ncrit, p, theta, args.precision)
                phi, grad = plan.eval(qt)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                plan.close()
                plan2 = FMM(xt, ncrit, p, theta, args.precision)
                plan2.adjoint(qt, wt, gradient_fwd=grad)
                plan2.close()
                torch.cuda.synchronize()
                fwd.append(t1 - t0)
                step.append(time.perf_counter() - t0)
            e_phi = rel_l2(phi.cpu().numpy()[samp], dphi)
            e_grad = rel_l2(grad.cpu().numpy()[samp], dgrad)
            rows.append({"theta": theta, "p": p, "err_phi": e_phi, "err_grad": e_grad,
                         "fwd_particles_per_s": n / float(np.median(fwd)),
                         "step_particles_per_s": n / float(np.median(step))})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    best = {}
    for th in (0.4, 0.5):
        ok = [r for r in rows if r["theta"] == th and max(r["err_phi"], r["err_grad"]) <= 1e-4]
        if ok:
            best[str(th)] = min(ok, key=lambda r: r["p"])["p"]
    return {"sweep": rows, "smallest_p_at_1e-4": best, "workload": args.workload, "precision": args.precision}


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1602_02244_amd import FMM, inputs

    n0, dist, p, ncrit, theta = inputs.WORKLOADS[args.workload]
    p = args.p if args.p is not None else p
    theta = args.theta if args.theta is not None else theta
    x, q = inputs.workload(args.workload)
    n = x.shape[0]
    w = inputs.adjoint_weights(n)
    dev = torch.device("cuda:0")
    xt, qt, wt = (torch.from_numpy(a).to(dev) for a in (x, q, w))
    if args.calibrate_copy:
        # 1 GiB source, then 1 GiB of other writes so that none of it stays in the
        # 256 MB last-level cache, then one plain copy: FETCH_SIZE and WRITE_SIZE of
        # that copy should each read 1 GiB (1048576 KiB)
        src = torch.ones(256 << 20, device=dev, dtype=torch.float32)
        evict = torch.full((256 << 20,), 2.0, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        dst.copy_(src)
        del src, dst, evict
    torch.cuda.synchronize()
    if args.accuracy_sweep:
        print(json.dumps(accuracy_sweep(args, xt, qt, wt, n, ncrit)), flush=True)
        return

    def step(record):
        t0 = time.perf_counter()
        plan = FMM(xt, ncrit, p, theta, args.precision, m2l_tol=args.m2l_tol)
        if record is not None:
            torch.cuda.synchronize()
            record["plan"].append(time.perf_counter() - t0)
            plan.set_timing(True)
        phi, grad = plan.eval(qt)
        if record is not None:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            record["fwd"].append(t1 - t0)
            record["eval_phases"].append(plan.phase_times())
            record["stats"] = plan.stats()
        plan.close()
        plan2 = FMM(xt, ncrit, p, theta, args.precision, m2l_tol=args.m2l_tol)
        if record is not None:
            plan2.set_timing(True)
        dq, dx = plan2.adjoint(qt, wt, gradient_fwd=grad)
        if record is not None:
            record["adj_phases"].append(plan2.phase_times())
        plan2.close()
        return phi, grad, dq, dx

    # the first plan of a process also builds the (p, theta) operator tables, a cached constant
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    FMM(xt, ncrit, p, theta, args.precision, m2l_tol=args.m2l_tol).close()
    torch.cuda.synchronize()
    first_plan_ms = 1e3 * (time.perf_counter() - t0)
    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    rec = {"fwd": [], "plan": [], "eval_phases": [], "adj_phases": []}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step(rec)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    phi, grad, dq, dx = out

    ms_step = 1e3 * total / args.steps
    st = rec["stats"]
    ph = {k: float(np.mean([d[k] for d in rec["eval_phases"] + rec["adj_phases"]])) for k in rec["eval_phases"][0]}
    eval_ms = float(np.mean([d["total"] for d in rec["eval_phases"]]))
    m2l_ms = ph["m2l"]
    p2p_ms = ph["p2p"]
    # with a variable-order M2L only the applied operator blocks count as work
    m2l_tflops = st["m2l_flops"] * st["m2l_kept_fraction"] / (m2l_ms * 1e-3) / 1e12
    p2p_tflops = st["p2p_flops"] / (p2p_ms * 1e-3) / 1e12
    result = {
        "metric": "Laplace FMM particles/s at 1e-4 rel err (fwd, fwd+adjoint); P2P TFLOP/s",
        "value": n / (ms_step * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "mixed(f16x3 MFMA, f32, f64)",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "distribution": dist, "p": p, "ncrit": ncrit, "theta": theta,
                   "precision": args.precision, "m2l_tol": args.m2l_tol, "step": "plan + eval + plan + adjoint"},
        "fwd_particles_per_s": n / float(np.mean(rec["fwd"])),
        "eval_particles_per_s": n / (eval_ms * 1e-3),
        "phase_ms": ph,
        "plan_ms": 1e3 * float(np.mean(rec["plan"])),
        "table_build_ms": first_plan_ms - 1e3 * float(np.mean(rec["plan"])),
        "p2p_tflops": p2p_tflops,
        "p2p_interactions_per_s": st["p2p_interactions"] / (p2p_ms * 1e-3),
        "m2l_tflops": m2l_tflops,
        "p2p_interactions": st["p2p_interactions"],
        "m2l_pairs": st["m2l_pairs"],
        "m2l_keys": st["m2l_keys"],
        "m2l_entries": st["m2l_entries"],
        "m2l_work_items": st["m2l_work_items"],
        "m2l_kept_fraction": st["m2l_kept_fraction"],
        "ncells": st["ncells"],
        "roofline": m2l_roofline(args.precision, m2l_tflops, m2l_traffic(args.workload, p, theta, st)),
        "p2p_roofline": {"kernel": "k_p2p", "bound": "alu", "achieved": p2p_tflops, "peak": VALU_FP32_PEAK_TFLOPS,
                         "unit": "TFLOP/s (20 flop/interaction)", "frac": p2p_tflops / VALU_FP32_PEAK_TFLOPS,
                         "frac_of_packed_peak": p2p_tflops / VALU_FP32_PACKED_PEAK_TFLOPS,
                         "frac_of_issue_peak": p2p_tflops / P2P_ISSUE_PEAK_TFLOPS},
    }

    if not args.skip_accuracy:
        samp = inputs.sample_targets(n, 1000)
        dphi, dgrad = direct_reference(xt, qt, samp)
        dpsi, _ = direct_reference(xt, wt, samp)
        ph_np, g_np, dq_np = phi.cpu().numpy()[samp], grad.cpu().numpy()[samp], dq.cpu().numpy()[samp]
        err = {"phi": rel_l2(ph_np, dphi), "grad": rel_l2(g_np, dgrad), "dL_dq": rel_l2(dq_np, dpsi)}
        result["rel_err_vs_direct_1000"] = err
        result["accuracy_ok"] = bool(max(err.values()) <= 1e-4)

    if not args.skip_cpu_baseline:
        # the FP64 oracle runs the same step: plan + forward FMM + plan + adjoint FMM (the FMM
        # with charges w, whose potential and gradient give dL/dq and dL/dx); the full plan
        # and upward passes are timed, M2L/L2L/L2P/P2P are timed on the targets of 2048
        # random leaves and scaled by the leaf count
        import oracle
        threads = oracle.set_threads(0)
        t0 = time.perf_counter()
        ora = oracle.Plan(x.astype(np.float64), ncrit, theta)
        t_plan = time.perf_counter() - t0
        cells = ora.cells()
        order, _ = ora.order()
        leaves = np.nonzero(cells["leaf"])[0]
        nl_s = min(2048, leaves.shape[0])
        pick = np.sort(np.random.default_rng(4001).choice(leaves, nl_s, replace=False))
        samp = np.concatenate([order[cells["start"][c]:cells["start"][c] + cells["count"][c]] for c in pick])
        scale = leaves.shape[0] / nl_s
        t_up = t_rest = 0.0
        for chg in (q, w):
            t0 = time.perf_counter()
            _, _, tm = ora.eval(chg.astype(np.float64), p, sample=samp)
            t_eval = time.perf_counter() - t0
            t_up += tm[0]
            t_rest += t_eval - tm[0]
        t_step = 2 * t_plan + t_up + t_rest * scale
        result["cpu_baseline"] = {
            "value": n / t_step,
            "unit": "particles/s",
            "cores": threads,
            "kind": "oracle",
            "sample": (f"FP64 oracle, same {n}-point workload and step (plan + forward + plan + adjoint): plan "
                       f"{t_plan:.1f} s (counted twice), upward passes {t_up:.1f} s, M2L/L2L/L2P/P2P for the "
                       f"{samp.shape[0]} targets of {nl_s} random leaves {t_rest:.1f} s scaled by "
                       f"{leaves.shape[0]}/{nl_s}; step {t_step:.0f} s"),
        }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
