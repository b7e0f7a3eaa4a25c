#!/usr/bin/env python
"""Throughput of the SCF hot path on one MI355X.

A step is one pass of the whole hot path over the workload: coefficient
accumulation (Eq. sumanlm) with its FP64 cross-block reduction, the field
evaluation (Eq. total_potential and its gradient, plus the host tidal field
when there is a host) and the fused leapfrog kick-drift.  The workload is the
Hernquist sphere N = 1e6 with nmax = 16, lmax = 10 (T = 2057 real
coefficients), inputs resident in HBM.  The metric is particle x basis-term
evaluations per second, N * T * steps / time.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 vector peak
PEAK_FP64_TFLOPS = 78.6
METRIC = "particle×basis-term evals/s per step (FP32 vs FP64); adjoint/forward time ratio"


def algorithmic_flops(nmax, lmax, host_flops=0):
    """Per-particle flops of one step: coefficient pass 2T + 4B + 30 and field
    pass 4T + 8B + host + 12, with B = (nmax+1)(lmax+1) + (lmax+1)(lmax+2)/2."""
    T = (nmax + 1) * (lmax + 1) ** 2
    B = (nmax + 1) * (lmax + 1) + (lmax + 1) * (lmax + 2) // 2
    return {"coef": 2 * T + 4 * B + 30, "field_step": 4 * T + 8 * B + host_flops + 12}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("scf_kernels.hip", "scf_device.h", "host_field.h"):
        with open(os.path.join(ROOT, "paper_2602_13385_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, n_launch):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def run_gpu(dtype, steps, warmup, torch, scf, I, profile):
    w = I.config3()
    p = w.clusters[0]
    td = torch.float32 if dtype == "f32" else torch.float64
    dev = lambda a: torch.as_tensor(a, dtype=td, device="cuda").contiguous()
    st = [dev(p.state()[i]) for i in range(6)]
    m = dev(p.mass)
    plan = scf.Plan(w.nmax, w.lmax, alpha=w.alpha, b=w.b, G=w.G, dtype=dtype)
    n = p.n
    cen, acc = plan.step(st, m, w.dt, 1)  # start-up evaluation of a(x0)
    if warmup:
        cen, acc = plan.step(st, m, w.dt, warmup, centre=cen, acc=acc)
    torch.cuda.synchronize()
    if profile:
        plan.profile(True)
        plan.kernel_times()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    cen, acc = plan.step(st, m, w.dt, steps, centre=cen, acc=acc)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    kt = plan.kernel_times() if profile else {}
    return {"n": n, "T": plan.T, "nmax": w.nmax, "lmax": w.lmax, "ms": ms, "wall_s": wall,
            "kernels": kt, "dt": w.dt, "name": w.name}


def cpu_baseline(nsample=200_000):
    from oracle import pyoracle as O
    from paper_2602_13385_amd import inputs as I
    w = I.config3()
    p = w.clusters[0]
    B = O.basis(w.nmax, w.lmax, alpha=w.alpha, b=w.b, G=w.G)
    pos = p.pos[:, :nsample].copy()
    mass = p.mass[:nsample].copy()
    t0 = time.perf_counter()
    c = O.coeffs(B, *pos, mass)
    O.field(B, c, *pos, pot=False)
    t = time.perf_counter() - t0
    T = O.ncoef(w.nmax, w.lmax)
    return {"value": nsample * T / t, "unit": "particle-terms/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"one coefficient + field pass of the FP64 oracle over the first {nsample} "
                      f"particles of the Hernquist N=1e6 nmax=16 lmax=10 workload ({t:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy (for counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs the hot path on one GPU only; --gpus {args.gpus} is not "
              f"supported (see the sharding notes in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2602_13385_amd import inputs as I
    from paper_2602_13385_amd import scf
    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4}))
        return
    scf.lib()
    r = run_gpu("f32", args.steps, args.warmup, torch, scf, I, profile=True)
    n, T = r["n"], r["T"]
    ms_per_step = r["ms"] / args.steps
    value = n * T * args.steps / (r["ms"] * 1e-3)
    fl = algorithmic_flops(r["nmax"], r["lmax"])
    # dominant kernel: the larger of the coefficient and field passes
    kt = r["kernels"]
    cands = {k: v for k, v in kt.items() if k in ("coef", "field_step")}
    dom = max(cands, key=lambda k: cands[k][1])
    cnt, tot = cands[dom]
    avg_s = tot / cnt * 1e-3
    achieved = fl[dom] * n / avg_s / 1e12
    traffic = measured_traffic(dom, n)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": r["name"], "N": n, "nmax": r["nmax"], "lmax": r["lmax"], "T": T,
                   "alpha": 1.0, "dt": r["dt"], "host": None},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": traffic, "flops_per_launch": fl[dom] * n,
                     "avg_launch_ms": tot / cnt},
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in kt.items()},
        "step_tflops": (fl["coef"] + fl["field_step"]) * n / (ms_per_step * 1e-3) / 1e12,
    }
    if not args.no_f64:
        steps64 = max(1, args.steps // 4)
        r64 = run_gpu("f64", steps64, max(1, args.warmup // 4), torch, scf, I, profile=False)
        out["f64"] = {"value": n * T * steps64 / (r64["ms"] * 1e-3), "ms_per_step": r64["ms"] / steps64,
                      "steps": steps64}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
