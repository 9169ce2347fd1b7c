#!/usr/bin/env python3
"""Benchmark of the MI355X FMM hot path on one GPU.

One step = the whole path on one synthetic point set: plan (root cube, keys, sort,
octree, dual traversal, operator grouping), forward evaluation (P2M, M2M, M2L, L2L,
L2P, P2P, un-permute), a rebuilt plan and the adjoint (the same FMM with charges
w = dL/dphi, plus dL/dx = w grad phi + q grad psi).  `value` is whole-step
particles/s (forward + adjoint) of the FP32 form on the largest workload (2^24 points
uniform in the unit cube, p = 12, ncrit = 64, theta = 0.4); the forward-only and
evaluation-only rates are reported beside it.  Inputs are resident in device memory
before timing starts.

Beside the headline the same run reports: the mixed-precision form and the
SVD-compressed M2L (tolerance 1e-5) on the same workload, the throughput at the smallest
order p whose result still meets 1e-4, the
uniform 2^20-point workload at p = 10, and the FP64 oracle timed on the host cores on a
bounded sample.  Accuracy is checked against the exact FP64 direct sum on 1000
sampled targets (phi, grad phi, dL/dq, dL/dx); `value` is null unless all four are
within 1e-4.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

MFMA_FP32_PEAK_TFLOPS = 157.3      # MI355X dense FP32 MFMA
MFMA_FP16_PEAK_TFLOPS = 2500.0     # MI355X dense FP16 MFMA
VALU_FP32_PACKED_PEAK_TFLOPS = 157.3   # MI355X FP32 vector with packed (2-wide) FMA
VALU_FP32_PEAK_TFLOPS = 78.6           # 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz, packed FP32 not used
ACC_TOL = 1e-4
# Bytes that one M2L step (GEMM + slot sums) moves between L2 and the memory fabric
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, factors from a plain 1 GiB copy), read from the
# rocprofv3 summary named in "source".  Reported only while the M2L kernel's source text (sha256 prefix of
# the k_gemm template in eval.hip) and the plan's grouping (entry and work-item counts)
# are the ones the counters were taken on; else null.
M2L_TRAFFIC = {"kernel_sha256": "6a28cdac88939087", "workload": "uniform-16M", "p": 12, "theta": 0.4,
               "entries": 7271803, "work_items": 1040804, "bytes": 796.8e9,
               "source": "profiles/m2l_uniform-16M_hbm_bytes.md"}
# The same for the split-FP16 M2L step (k_m2l_f16 + sums), keyed to that kernel's source.
M2L_TRAFFIC_MIXED = {"kernel_sha256": "89e4136b21d141bc", "workload": "uniform-16M", "p": 12, "theta": 0.4,
                     "entries": 7275201, "work_items": 1040638, "bytes": 679.9e9,
                     "source": "profiles/m2l_mixed_uniform-16M_hbm_bytes.md"}


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform-16M")
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "mixed"])
    ap.add_argument("--m2l-tol", type=float, default=0.0,
                    help="variable-order M2L tolerance (0: dense operators, the configuration's method)")
    ap.add_argument("--svd-tol", type=float, default=0.0,
                    help="SVD-compressed M2L tolerance (0: dense operators, the configuration's method)")
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--skip-accuracy", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed configuration (no mixed form, no 1e-4 order, no 2^20 workload)")
    ap.add_argument("--accuracy-sweep", default=None, metavar="P_LIST",
                    help="instead of the benchmark line: error against the direct sum and throughput for each "
                         "order in P_LIST (e.g. 2,4,6,8,10,12) at theta 0.4 and 0.5, one JSON line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    return ap.parse_args(argv)


def m2l_kernel_sha(mixed=False):
    """sha256 prefix of the M2L kernel's source text in eval.hip: the k_gemm template, or
    with `mixed` the k_m2l_f16 template."""
    src = open(os.path.join(ROOT, "paper_1602_02244_amd", "csrc", "eval.hip")).read()
    if mixed:
        a = src.index("template <int P, int NW = f16_waves<P>()>")
        b = src.index("constexpr int kReduceChunks", a)
    else:
        a = src.index("template <int P, bool ADD, bool MASKED")
        b = src.index("// ---", a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def m2l_roofline(precision, m2l_tflops, traffic, form="dense"):
    """The M2L step (grouped GEMM + the fixed-order sum of split tiles) against the MFMA
    peak of the type it computes in.  The split-FP16 form runs three FP16 products (hi hi,
    hi lo, lo hi) per algorithmic one.  The compressed forms count the flops they apply
    (two rank-r products per pair for the SVD, the kept 16 x 16 blocks for block
    dropping) and report no traffic: the recorded counters belong to the dense FP32 and
    split-FP16 kernels."""
    if form == "svd":
        return {"kernel": "k_gemm_svd (two FP32 MFMA products of rank r per entry) + sums", "bound": "mfma",
                "achieved": m2l_tflops, "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s (factored flops)",
                "frac": m2l_tflops / MFMA_FP32_PEAK_TFLOPS, "traffic": None}
    if form == "blocks":
        return {"kernel": "k_gemm with dropped 16x16 operator blocks + sums", "bound": "mfma",
                "achieved": m2l_tflops, "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s (applied blocks)",
                "frac": m2l_tflops / MFMA_FP32_PEAK_TFLOPS, "traffic": None}
    if precision == "mixed":
        achieved = 3.0 * m2l_tflops
        return {"kernel": "k_m2l_f16 + k_m2l_reduce (split-FP16 MFMA grouped GEMM, 3 products)", "bound": "mfma",
                "achieved": achieved, "peak": MFMA_FP16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / MFMA_FP16_PEAK_TFLOPS, "fp32_equivalent": m2l_tflops, "traffic": traffic,
                "traffic_kind": "L2-to-fabric bytes per launch (FETCH_SIZE/WRITE_SIZE, copy-scaled)",
                "traffic_source": M2L_TRAFFIC_MIXED["source"] if traffic is not None else None}
    return {"kernel": "k_gemm (FP32 MFMA grouped GEMM) + k_m2l_reduce", "bound": "mfma", "achieved": m2l_tflops,
            "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": m2l_tflops / MFMA_FP32_PEAK_TFLOPS,
            "traffic": traffic, "traffic_kind": "L2-to-fabric bytes per launch (FETCH_SIZE/WRITE_SIZE, copy-scaled)",
            "traffic_source": M2L_TRAFFIC["source"] if traffic is not None else None}


def p2p_roofline(p2p_tflops):
    return {"kernel": "k_p2p", "bound": "alu", "achieved": p2p_tflops, "peak": VALU_FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s (20 flop/interaction)", "frac": p2p_tflops / VALU_FP32_PEAK_TFLOPS,
            "frac_of_packed_peak": p2p_tflops / VALU_FP32_PACKED_PEAK_TFLOPS}


def m2l_traffic(workload, p, theta, st, mixed=False):
    t = M2L_TRAFFIC_MIXED if mixed else M2L_TRAFFIC
    if t["bytes"] is None:
        return None
    if (m2l_kernel_sha(mixed) == t["kernel_sha256"] and (workload, p, theta) == (t["workload"], t["p"], t["theta"])
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


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


class Refs:
    """Exact FP64 values at the sampled targets: phi, grad phi (charges q), psi, grad psi
    (charges w), and dL/dx = w grad phi + q grad psi."""

    def __init__(self, x, q, w, xt, qt, wt, samp):
        self.samp = samp
        self.phi, self.grad = direct_reference(xt, qt, samp)
        self.psi, self.gpsi = direct_reference(xt, wt, samp)
        self.dx = (w.astype(np.float64)[samp, None] * self.grad + q.astype(np.float64)[samp, None] * self.gpsi)

    def errors(self, phi, grad, dq, dx):
        s = self.samp
        out = {"phi": rel_l2(phi.cpu().numpy()[s], self.phi), "grad": rel_l2(grad.cpu().numpy()[s], self.grad)}
        if dq is not None:
            out["dL_dq"] = rel_l2(dq.cpu().numpy()[s], self.psi)
        if dx is not None:
            out["dL_dx"] = rel_l2(dx.cpu().numpy()[s], self.dx)
        return out


def run_steps(xt, qt, wt, ncrit, p, theta, precision, steps, warmup, m2l_tol=0.0, svd_tol=0.0):
    """Times `steps` whole steps (plan + eval + plan + adjoint) after `warmup` untimed
    ones; per-phase HIP-event times and plan statistics from the timed steps."""
    import torch
    from paper_1602_02244_amd import FMM
    n = xt.shape[0]

    def step(record):
        t0 = time.perf_counter()
        plan = FMM(xt, ncrit, p, theta, precision, m2l_tol=m2l_tol, svd_tol=svd_tol)
        if record is not None:
            torch.cuda.synchronize()
            record["plan"].append(time.perf_counter() - t0)
            plan.set_timing(True)
        phi, grad = plan.eval(qt)
        if record is not None:
            torch.cuda.synchronize()
            record["fwd"].append(time.perf_counter() - t0)
            record["eval_phases"].append(plan.phase_times())
            record["stats"] = plan.stats()
        plan.close()
        plan2 = FMM(xt, ncrit, p, theta, precision, m2l_tol=m2l_tol, svd_tol=svd_tol)
        if record is not None:
            plan2.set_timing(True)
        dq, dx = plan2.adjoint(qt, wt, gradient_fwd=grad)
        if record is not None:
            record["adj_phases"].append(plan2.phase_times())
        plan2.close()
        return phi, grad, dq, dx

    # the first plan of a process (per order) also builds the operator tables, a cached constant
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    FMM(xt, ncrit, p, theta, precision, m2l_tol=m2l_tol, svd_tol=svd_tol).close()
    torch.cuda.synchronize()
    first_plan_ms = 1e3 * (time.perf_counter() - t0)
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    rec = {"fwd": [], "plan": [], "eval_phases": [], "adj_phases": []}
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step(rec)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_step = 1e3 * total / steps
    st = rec["stats"]
    phases = rec["eval_phases"] + rec["adj_phases"]
    ph = {k: float(np.mean([d[k] for d in phases])) for k in phases[0]}
    eval_ms = float(np.mean([d["total"] for d in rec["eval_phases"]]))
    # the M2L phase spans the grouped GEMM and the fixed-order sums of split tiles and slots;
    # with a variable-order or SVD-compressed M2L only the applied work counts
    m2l_tflops = st["m2l_flops"] * st["m2l_kept_fraction"] / (ph["m2l"] * 1e-3) / 1e12
    p2p_tflops = st["p2p_flops"] / (ph["p2p"] * 1e-3) / 1e12
    plan_ms = 1e3 * float(np.mean(rec["plan"]))
    return {
        "particles_per_s": n / (ms_step * 1e-3),
        "ms_per_step": ms_step,
        "fwd_particles_per_s": n / float(np.mean(rec["fwd"])),
        "eval_particles_per_s": n / (eval_ms * 1e-3),
        "phase_ms": ph,
        "plan_ms": plan_ms,
        "table_build_ms": first_plan_ms - plan_ms,
        "m2l_tflops": m2l_tflops,
        "p2p_tflops": p2p_tflops,
        "p2p_interactions_per_s": st["p2p_interactions"] / (ph["p2p"] * 1e-3),
        "stats": st,
    }, out


def stats_keys(st):
    return {k: st[k] for k in ("ncells", "m2l_pairs", "m2l_keys", "m2l_entries", "m2l_work_items", "p2p_interactions",
                               "m2l_kept_fraction", "m2l_svd_rank_mean", "m2l_slots", "workspace_bytes")}


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
        ok = [r for r in rows if r["theta"] == th and max(r["err_phi"], r["err_grad"]) <= ACC_TOL]
        if ok:
            best[str(th)] = min(ok, key=lambda r: r["p"])["p"]
    return {"sweep": rows, "smallest_p_at_1e-4": best, "workload": args.workload, "precision": args.precision}


def smallest_order(xt, qt, wt, ncrit, theta, refs, p_max):
    """Smallest p whose forward and adjoint outputs all meet 1e-4 against the direct sum
    (one plan + eval + adjoint per order, FP32), with the errors of every order tried."""
    from paper_1602_02244_amd import FMM
    tried = {}
    for p in range(1, p_max + 1):
        plan = FMM(xt, ncrit, p, theta, "fp32")
        phi, grad = plan.eval(qt)
        dq, dx = plan.adjoint(qt, wt, gradient_fwd=grad)
        plan.close()
        e = refs.errors(phi, grad, dq, dx)
        tried[p] = e
        print(f"[bench] order sweep p={p}: {e}", file=sys.stderr, flush=True)
        if max(e.values()) <= ACC_TOL:
            return p, tried
    return None, tried


def cpu_baseline(x, q, w, ncrit, p, theta, dist):
    """The FP64 oracle timed on this host's cores for the same step (plan + forward + plan
    + adjoint, the adjoint being the FMM with charges w), on a bounded sample: the plan and
    the upward pass are timed in full, M2L/L2L/L2P/P2P on the targets of random leaves and
    scaled by the leaf count.  For more than 2^22 points uniform in the unit cube the
    sample is the octant [0, 1/2)^3 (an eighth of the points, whose tree is the full tree's
    octant subtree), and the plan and upward times are scaled by 8."""
    import oracle
    threads = oracle.set_threads(0)
    n = x.shape[0]
    scale_all = 1.0
    note = ""
    if n > (1 << 22) and dist == "cube":
        sel = np.all(x < 0.5, axis=1)
        x, q, w = x[sel], q[sel], w[sel]
        scale_all = n / x.shape[0]
        note = f"octant [0,1/2)^3 of the workload ({x.shape[0]} of {n} points) scaled by {scale_all:.3f}; "
    t0 = time.perf_counter()
    ora = oracle.Plan(x.astype(np.float64), ncrit, theta)
    t_plan = time.perf_counter() - t0
    cells = ora.cells()
    order, _ = ora.order()
    leaves = np.nonzero(cells["leaf"])[0]
    nl_s = min(256 if scale_all > 1 else 2048, leaves.shape[0])
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
    ora.close()
    t_step = scale_all * (2 * t_plan + t_up + t_rest * scale)
    return {
        "value": n / t_step,
        "unit": "particles/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"FP64 oracle, same workload and step (plan + forward + plan + adjoint): {note}plan "
                   f"{t_plan:.1f} s (counted twice), upward passes {t_up:.1f} s, M2L/L2L/L2P/P2P for the "
                   f"{samp.shape[0]} targets of {nl_s} random leaves {t_rest:.1f} s scaled by "
                   f"{leaves.shape[0]}/{nl_s}; step {t_step:.0f} s"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1602_02244_amd import inputs

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

    print(f"[bench] {args.workload} n={n} p={p} {args.precision}: {args.steps} steps after {args.warmup}",
          file=sys.stderr, flush=True)
    run, (phi, grad, dq, dx) = run_steps(xt, qt, wt, ncrit, p, theta, args.precision, args.steps, args.warmup,
                                         args.m2l_tol, args.svd_tol)
    st = run.pop("stats")
    result = {
        "metric": "Laplace FMM particles/s at 1e-4 rel err (fwd, fwd+adjoint); P2P TFLOP/s",
        "value": run["particles_per_s"],
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "mixed(f16x3 MFMA, f32, f64)",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "distribution": dist, "p": p, "ncrit": ncrit, "theta": theta,
                   "precision": args.precision, "m2l_tol": args.m2l_tol, "svd_tol": args.svd_tol,
                   "step": "plan + eval + plan + adjoint"},
    }
    result.update({k: v for k, v in run.items() if k not in ("particles_per_s", "ms_per_step")})
    result.update(stats_keys(st))
    form = "svd" if args.svd_tol > 0 else ("blocks" if args.m2l_tol > 0 else "dense")
    result["roofline"] = m2l_roofline(args.precision, run["m2l_tflops"],
                                      m2l_traffic(args.workload, p, theta, st, args.precision == "mixed")
                                      if form == "dense" else None, form)
    result["p2p_roofline"] = p2p_roofline(run["p2p_tflops"])

    refs = None
    if not args.skip_accuracy:
        samp = inputs.sample_targets(n, 1000)
        refs = Refs(x, q, w, xt, qt, wt, samp)
        err = refs.errors(phi, grad, dq, dx)
        result["rel_err_vs_direct_1000"] = err
        result["accuracy_ok"] = bool(max(err.values()) <= ACC_TOL)
        if not result["accuracy_ok"]:
            result["value"] = None
    del phi, grad, dq, dx

    if not args.headline_only and args.precision == "fp32" and args.m2l_tol == 0.0 and args.svd_tol == 0.0:
        ks, kw = min(args.steps, 5), min(args.warmup, 1)
        # the mixed-precision form on the same workload
        print("[bench] mixed precision", file=sys.stderr, flush=True)
        mr, (mphi, mgrad, mdq, mdx) = run_steps(xt, qt, wt, ncrit, p, theta, "mixed", ks, kw)
        mst = mr.pop("stats")
        mixed = dict(mr, steps=ks, warmup=kw,
                     roofline=m2l_roofline("mixed", mr["m2l_tflops"], m2l_traffic(args.workload, p, theta, mst, True)),
                     p2p_roofline=p2p_roofline(mr["p2p_tflops"]))
        if refs is not None:
            mixed["rel_err_vs_direct_1000"] = refs.errors(mphi, mgrad, mdq, mdx)
            mixed["accuracy_ok"] = bool(max(mixed["rel_err_vs_direct_1000"].values()) <= ACC_TOL)
        mixed["speedup_vs_fp32_step"] = run["ms_per_step"] / mr["ms_per_step"]
        del mphi, mgrad, mdq, mdx, mst
        result["mixed"] = mixed
        # the SVD-compressed M2L at a tolerance that keeps the FP32 accuracy
        print("[bench] SVD-compressed M2L", file=sys.stderr, flush=True)
        sv_tol = 1e-5
        vr, (vphi, vgrad, vdq, vdx) = run_steps(xt, qt, wt, ncrit, p, theta, "fp32", ks, kw, svd_tol=sv_tol)
        vst = vr.pop("stats")
        svd = {k: vr[k] for k in ("particles_per_s", "ms_per_step", "fwd_particles_per_s", "eval_particles_per_s",
                                  "plan_ms", "table_build_ms", "phase_ms")}
        svd.update(svd_tol=sv_tol, steps=ks, warmup=kw, m2l_svd_rank_mean=vst["m2l_svd_rank_mean"],
                   m2l_factored_tflops=vr["m2l_tflops"],
                   m2l_dense_equivalent_tflops=vst["m2l_flops"] / (vr["phase_ms"]["m2l"] * 1e-3) / 1e12,
                   speedup_vs_fp32_step=run["ms_per_step"] / vr["ms_per_step"])
        if refs is not None:
            svd["rel_err_vs_direct_1000"] = refs.errors(vphi, vgrad, vdq, vdx)
        del vphi, vgrad, vdq, vdx
        result["svd"] = svd
        # throughput at the smallest order that still meets 1e-4
        if refs is not None:
            p_star, tried = smallest_order(xt, qt, wt, ncrit, theta, refs, p)
            at = {"p": p_star, "errors_by_p": {str(k): v for k, v in tried.items()}}
            if p_star is not None:
                print(f"[bench] smallest order p={p_star}", file=sys.stderr, flush=True)
                sr, (sphi, sgrad, sdq, sdx) = run_steps(xt, qt, wt, ncrit, p_star, theta, "fp32", ks, kw)
                sr.pop("stats")
                at.update({k: sr[k] for k in ("particles_per_s", "ms_per_step", "fwd_particles_per_s",
                                              "eval_particles_per_s", "plan_ms", "m2l_tflops", "p2p_tflops")})
                at["steps"] = ks
                at["rel_err_vs_direct_1000"] = refs.errors(sphi, sgrad, sdq, sdx)
                del sphi, sgrad, sdq, sdx
            result["at_1e-4"] = at
        # the uniform 2^20-point workload at its own order
        if args.workload != "uniform-1M":
            print("[bench] uniform-1M", file=sys.stderr, flush=True)
            n1, dist1, p1, ncrit1, theta1 = inputs.WORKLOADS["uniform-1M"]
            x1, q1 = inputs.workload("uniform-1M")
            w1 = inputs.adjoint_weights(n1)
            x1t, q1t, w1t = (torch.from_numpy(a).to(dev) for a in (x1, q1, w1))
            r1, (phi1, grad1, dq1, dx1) = run_steps(x1t, q1t, w1t, ncrit1, p1, theta1, "fp32", args.steps,
                                                    args.warmup)
            st1 = r1.pop("stats")
            c2 = dict(r1, config={"workload": "uniform-1M", "n": n1, "p": p1, "ncrit": ncrit1, "theta": theta1},
                      roofline=m2l_roofline("fp32", r1["m2l_tflops"], None), p2p_roofline=p2p_roofline(r1["p2p_tflops"]))
            c2.update(stats_keys(st1))
            if refs is not None:
                refs1 = Refs(x1, q1, w1, x1t, q1t, w1t, inputs.sample_targets(n1, 1000))
                c2["rel_err_vs_direct_1000"] = refs1.errors(phi1, grad1, dq1, dx1)
            result["uniform-1M"] = c2

    if not args.skip_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(x, q, w, ncrit, p, theta, dist)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
