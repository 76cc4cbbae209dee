"""Benchmark of the periodized Coulomb sum on one MI355X.

One step = one periodic solve ("get", every stage of the hot path) of the
uniform-cube workload: N = 100,000 particles in the unit cube, q ~ N(0,1)
minus its mean, p = 16 (L = 496 check points), R_b = 1.5, FP32 pair arithmetic
with FP64 accumulation.  Inputs are resident on the GPU before timing starts.

Prints one JSON line.  value = pair interactions per second over the whole
solve, counting (N + 2L) * N_b pairs per solve (the particle and check-point
near sums).  The roofline entry is the particle pair-sum kernel, its duration
taken from HIP events recorded by the library on the eval stream.  The CPU
baseline times the FP64 oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector (packed), published
FLOP_PER_PAIR = 20         # potential + field: 3 sub, r^2 (mul + 2 FMA), rsqrt, 3 mul, add, 3 FMA


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(precision):
    """HBM bytes per launch of the pair kernel from the committed rocprofv3
    counter record, or None if the kernel source has changed since."""
    import hashlib
    if precision != "fp32":
        return None
    rec = os.path.join(ROOT, "profiles", "p2p_f32_uniform_cube_N100k_hbm_counters.json")
    if not os.path.exists(rec):
        return None
    src = open(os.path.join(ROOT, "paper_1310_4374_amd", "csrc", "ps_kernels.hip")).read()
    a = src.index("template <int BT, bool FIELD>\n__global__ __launch_bounds__(BT) void k_p2p_f32")
    b = src.index("// FP64 reciprocal square root", a)
    h = hashlib.sha256(src[a:b].encode()).hexdigest()[:16]
    d = json.load(open(rec))
    return d["traffic_bytes"] if d.get("source_sha256_16") == h else None


def cpu_baseline(c, ntarget=4000):
    """The FP64 oracle as it stands, on a bounded sample: its full "get" with the
    check points and `ntarget` particles as targets."""
    from oracle.method import Plan as OPlan
    pl = OPlan(c["box"], c["p"], R_b=c["R_b"])
    t = time.perf_counter()
    parts = pl.solve(c["x"], c["q"], targets=c["x"][:ntarget], return_parts=True)
    dt = time.perf_counter() - t
    pairs = (2 * pl.L + ntarget) * parts["n_near"]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": pairs / dt, "unit": "pair interactions/s", "cores": cores, "kind": "oracle",
            "sample": "oracle get (near set, %d check points, Phi0, far field) with %d particle targets: "
                      "%.3g pairs in %.1f s" % (2 * pl.L, ntarget, pairs, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="time without the per-stage events")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this implementation has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1310_4374_amd as ps
    import workloads as W

    c = W.config2()
    n = len(c["q"])
    dev = torch.device("cuda", 0)
    if args.copy_calibration_mib:
        a = torch.ones(args.copy_calibration_mib * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read, %d MiB written" % (args.copy_calibration_mib, args.copy_calibration_mib))
        del a, b
    x = torch.tensor(np.ascontiguousarray(c["x"].T), device=dev)
    q = torch.tensor(c["q"], device=dev)
    plan = ps.Plan(c["box"], c["p"], R_b=c["R_b"], precision=args.precision, n_max=n)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    field = torch.empty(3, n, dtype=torch.float64, device=dev)
    log("plan ready:", plan.info())
    for _ in range(args.warmup):
        plan.eval(x, q, out=(phi, field))
    plan.status()
    info = plan.info()
    nb, L = info["n_near_last"], info["L"]
    pairs_per_step = (n + 2 * L) * nb
    prof = not args.no_profile
    plan.set_profiling(prof)
    stage_sum = None
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        plan.eval(x, q, out=(phi, field))
        if prof:
            st = plan.stage_times()
            stage_sum = st if stage_sum is None else {k: stage_sum[k] + st[k] for k in st}
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end) / args.steps
    log("timed %d steps: %.3f ms/step (host wall %.3f s)" % (args.steps, ms, wall))
    plan.status()

    # accuracy against the stored FP64 oracle values at 2,000 sampled particles
    acc = {}
    ref_path = os.path.join(ROOT, "tests", "golden", "ref_cfg2.npz")
    if os.path.exists(ref_path):
        ref = np.load(ref_path)
        sub = ref["subset"]
        ph = phi.cpu().numpy()[sub]
        fd = field.cpu().numpy().T[sub]
        acc = {"rel_l2_phi": float(np.linalg.norm(ph - ref["phi"]) / np.linalg.norm(ref["phi"])),
               "rel_l2_field": float(np.linalg.norm(fd - ref["field"]) / np.linalg.norm(ref["field"])),
               "accuracy_sample": "2000 particles vs FP64 oracle"}

    roof = None
    stage_ms = None
    if prof:
        stage_ms = {k: v / args.steps for k, v in stage_sum.items()}
        t_pairs = stage_ms["pairs"] * 1e-3
        achieved = FLOP_PER_PAIR * n * nb / t_pairs / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS, "traffic": measured_traffic(args.precision),
                "kernel": "k_p2p_%s<256,field> (particle near sums)" % ("f32" if args.precision == "fp32" else "f64"),
                "flop_per_pair": FLOP_PER_PAIR, "pairs_per_launch": n * nb,
                "pair_rate": n * nb / t_pairs}
    out = {
        "metric": "pair interactions/s and periodic solves/s at rel-L2 <=1e-6 vs FP64 oracle",
        "value": pairs_per_step / (ms * 1e-3),
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "solves_per_s": 1e3 / ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic (seeded uniform positions, Gaussian charges)",
        "config": {"workload": "uniform cube 1x1x1, N=100000, q~N(0,1)-mean, p=16 (L=496), R_b=1.5, "
                               + ("FP32 pairs with FP64 accumulation" if args.precision == "fp32" else "FP64"),
                   "N": n, "p": c["p"], "L": L, "R_b": c["R_b"], "n_near": nb,
                   "pairs_per_solve": pairs_per_step, "parallelism": "single GPU"},
        "roofline": roof,
        "stage_ms": stage_ms,
    }
    out.update(acc)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(c)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
