#!/usr/bin/env python
"""Throughput of the SCF hot path on one MI355X.

A step is one pass of the whole hot path over the workload: coefficient
accumulation (Eq. sumanlm) with its FP64 cross-block reduction, the field
evaluation (Eq. total_potential and its gradient, plus the host tidal field
when there is a host) and the fused leapfrog kick-drift.  The headline
workload is the Hernquist sphere N = 1e6 with nmax = 16, lmax = 10 (T = 2057
real coefficients), inputs resident in HBM.  The metric is particle x
basis-term evaluations per second, N * T * steps / time, in FP32.

Also reported on the same JSON line: the FP64 path on the same workload, the
batched path (10 Plummer progenitors in a composite host, direct launches and
graph replay, against the summed plain per-cluster steps), the adjoint/forward
time ratio of the checkpointed reverse pass (Plummer N = 1e5 in an NFW host,
2000 steps, checkpoints every 100), whole runs of the isolated Plummer (1e4
particles, 100 steps) and of the Plummer in the logarithmic host (1e5
particles, 1e4 steps) in FP32 and FP64, the FP32 path's relative errors, the
diagnostics and refresh-cadence legs, and the FP64 CPU oracle timed on a
bounded sample.

Prints one JSON line.  --gpus above 1 is refused: the path runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 peak (dense MFMA; vector with packed FP32)
PEAK_FP64_TFLOPS = 78.6
# The vector ALUs without packed FP32 (which every HIP file here turns off):
# one wave64 FMA per SIMD per 4 cycles, 256 CUs x 4 SIMDs x 64 lanes x 2 flop
# / 4 cycles x 2.4 GHz.  The FMA-chain microbenchmark (scf_bench_ceiling)
# measures 75.6 TFLOP/s at 8 waves per SIMD, 73.0 at 4.
PEAK_FP32_SINGLE_ISSUE_TFLOPS = 78.6
METRIC = "particle×basis-term evals/s per step (FP32 vs FP64); adjoint/forward time ratio"
# The paper's own timings: whole 5 Gyr simulations on other hardware, with its
# relaxation, refreshes and diagnostics included, so context for the scale of
# the problem rather than a figure to compare a per-step kernel rate with
# (Sec. Results, opening; Appendix "Comparisons to N-body Simulations",
# Technical Details).
PAPER_CONTEXT = {
    "krios_wall_clock_hr": [6.6, 6.6, 21.1],
    "krios_hardware": "128 CPU cores",
    "krios_workload": "N = 5e4 King W0 = 5 cluster, M = 1e5 Msun, r_hm = 10 pc, MWPotential2014, "
                      "three orbits (20 kpc circular, eccentric, 5 kpc circular), 5 Gyr",
    "nbody6pp_gpu_wall_clock_hr": [29, 38, 56],
    "nbody6pp_gpu_hardware": "40-core node with one NVIDIA V100",
    "krios_n2e5_wall_clock_hr": {"min": 5.9, "median": 11, "max": 22.1},
    "krios_n2e5_hardware": "192 CPU cores",
    "note": "whole-simulation wall clock on other hardware; not comparable to a per-step rate",
}
KERNEL_FILES = ("scf_kernels.h", "scf_device.h", "scf_dual.h", "host_field.h")


def algorithmic_flops(nmax, lmax, host_flops=0):
    """Per-particle flops of one step: coefficient pass 2T + 4B + 30 and field
    pass 4T + 8B + host + 12, with B = (nmax+1)(lmax+1) + (lmax+1)(lmax+2)/2."""
    T = (nmax + 1) * (lmax + 1) ** 2
    B = (nmax + 1) * (lmax + 1) + (lmax + 1) * (lmax + 2) // 2
    return {"coef": 2 * T + 4 * B + 30, "field_step": 4 * T + 8 * B + host_flops + 12}


def roofline_entry(kernel, achieved, field_variant, traffic, flops, avg_ms):
    """A kernel against the published FP32 peak, 157.3 TFLOP/s (`frac`).  The
    field pass in variants 2 and 3 does its radial sums on the matrix cores
    (dense FP32 MFMA, 157.3) and the rest on the vector ALUs; the other kernels
    run on the vector ALUs alone, whose published 157.3 counts packed FP32.
    Packed FP32 is off in every HIP file here, so a vector-ALU kernel's own
    ceiling is the single-issue 78.6 TFLOP/s (`frac_single_issue_valu`, given
    for the vector-ALU kernels; measured FMA chains reach 75.6)."""
    mfma = kernel == "field_step" and field_variant in (2, 3)
    e = {"bound": "mfma" if mfma else "alu", "kernel": kernel, "achieved": achieved,
         "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
         "traffic": traffic, "flops_per_launch": flops, "avg_launch_ms": avg_ms}
    if not mfma:
        e["frac_single_issue_valu"] = achieved / PEAK_FP32_SINGLE_ISSUE_TFLOPS
    return e


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_FILES:
        with open(os.path.join(ROOT, "paper_2602_13385_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def _timed(torch, fn):
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    out = fn()
    e1.record(s)
    torch.cuda.synchronize()
    return out, e0.elapsed_time(e1)


def run_main(dtype, steps, warmup, torch, scf, I, profile, variants=None):
    """Hernquist N = 1e6, nmax 16, lmax 10: `steps` timed steps.  variants =
    (coefficient variant, field variant) pins the kernels instead of the
    autotuner's choice (for profiles of one fixed kernel pair)."""
    w = I.config3()
    p = w.clusters[0]
    td = torch.float32 if dtype == "f32" else torch.float64
    dev = lambda a: torch.as_tensor(a, dtype=td, device="cuda").contiguous()
    st = [dev(p.state()[i]) for i in range(6)]
    m = dev(p.mass)
    plan = scf.Plan(w.nmax, w.lmax, alpha=w.alpha, b=w.b, G=w.G, dtype=dtype)
    if variants is None:
        variant, _ = plan.autotune(st[0], st[1], st[2], m)
    else:
        variant, plan.variant = variants[0], variants[0]
        plan.field_variant = variants[1]
    n = p.n
    cen, acc = plan.step(st, m, w.dt, 1)  # start-up evaluation of a(x0)
    if warmup:
        cen, acc = plan.step(st, m, w.dt, warmup, centre=cen, acc=acc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    (cen, acc), ms = _timed(torch, lambda: plan.step(st, m, w.dt, steps, centre=cen, acc=acc))
    wall = time.perf_counter() - t0
    kt = {}
    if profile:
        # per-kernel durations from HIP events around every launch, in a
        # second run of the same length (the events are not in the timed run)
        plan.profile(True)
        plan.kernel_times()
        cen, acc = plan.step(st, m, w.dt, steps, centre=cen, acc=acc)
        kt = plan.kernel_times()
        plan.profile(False)
    return {"n": n, "T": plan.T, "nmax": w.nmax, "lmax": w.lmax, "ms": ms, "wall_s": wall,
            "kernels": kt, "dt": w.dt, "name": w.name, "variant": variant,
            "field_variant": plan.field_variant, "coef_units_div": plan.coef_units_div,
            "plan": plan, "describe": plan.describe()}


def accuracy_main(torch, scf, I):
    """FP32 vs FP64 coefficients and forces on the headline workload, and the
    FP64 potential against the closed-form Hernquist potential -1/(1+r)."""
    import numpy as np
    w = I.config3()
    p = w.clusters[0]
    out = {}
    res = {}
    for dtype, td in (("f32", torch.float32), ("f64", torch.float64)):
        pos = np.asarray(p.pos, dtype=np.float32).astype(np.float64)
        mass = np.asarray(p.mass, dtype=np.float32).astype(np.float64)
        x, y, z = (torch.as_tensor(pos[i], dtype=td, device="cuda") for i in range(3))
        m = torch.as_tensor(mass, dtype=td, device="cuda")
        plan = scf.Plan(w.nmax, w.lmax, dtype=dtype)
        c = plan.coeffs(x, y, z, m)
        # forces from every field variant (FP32: 0, 1 vector ALU; 2, 3 matrix cores)
        gs = []
        for fv in range(plan.num_field_variants):
            plan.field_variant = fv
            ax, ay, az, pot = plan.forces(x, y, z, c, pot=True)
            torch.cuda.synchronize()
            gs.append(np.stack([t.double().cpu().numpy() for t in (ax, ay, az)]))
        res[dtype] = (c.cpu().numpy(), gs, pot.double().cpu().numpy())
    c32, g32, _ = res["f32"]
    c64, g64, p64 = res["f64"]
    g64 = g64[0]
    out["coef_relerr_f32_vs_f64"] = float(np.abs(c32 - c64).max() / np.abs(c64).max())
    mag = np.sqrt((g64 ** 2).sum(0))
    errs = [float((np.sqrt(((g - g64) ** 2).sum(0)) / (mag + np.median(mag))).max()) for g in g32]
    out["force_relerr_f32_vs_f64"] = max(errs)
    out["force_relerr_f32_vs_f64_per_field_variant"] = errs
    r = np.sqrt((np.asarray(p.pos) ** 2).sum(0))
    ref = -1.0 / (1.0 + r)
    out["pot_relerr_f64_vs_closed_form_median"] = float(np.median(np.abs(p64 - ref) / np.abs(ref)))
    out["note"] = ("f32 vs f64: same FP32-representable inputs; closed form: N = 1e6 Monte-Carlo "
                   "sample, so the difference is sampling noise of the truncated expansion")
    return out


def run_batched(torch, scf, I, steps):
    """10 Plummer progenitors (N log-uniform in [2e4, 5e5]) on eccentric orbits
    in the composite host: batched launches (direct, and replayed from HIP
    graphs) vs the summed plain steps."""
    import numpy as np
    w = I.config4()
    sizes = [c.n for c in w.clusters]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    state = np.concatenate([c.state() for c in w.clusters], axis=1)
    mass = np.concatenate([c.mass for c in w.clusters])
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    st = [dev(state[i]) for i in range(6)]
    m = dev(mass)
    cens = np.array(w.centres)
    plan = scf.Plan(w.nmax, w.lmax, dtype="f32")
    plan.autotune(st[0], st[1], st[2], m)
    host = (w.host, w.G)
    cen, acc = plan.step_batched(off, st, m, w.dt, 3, host=host, centres=cens)
    # warm both launch modes up (the graph is captured here), then alternate
    # the timed runs and keep the best of each, so that neither mode pays for
    # the GPU's clock ramp
    for g in (False, True, False, True):
        cen, acc = plan.step_batched(off, st, m, w.dt, steps, host=host, centres=cen, acc=acc,
                                     graph=g)
    ms, ms_graph = float("inf"), float("inf")
    for _ in range(3):
        for g in (False, True):
            (cen, acc), t = _timed(torch, lambda: plan.step_batched(off, st, m, w.dt, steps,
                                                                    host=host, centres=cen,
                                                                    acc=acc, graph=g))
            if g:
                ms_graph = min(ms_graph, t)
            else:
                ms = min(ms, t)
    # per-kernel times of the direct launches (HIP events around each launch,
    # in a separate run of the same length)
    plan.profile(True)
    plan.kernel_times()
    cen, acc = plan.step_batched(off, st, m, w.dt, steps, host=host, centres=cen, acc=acc)
    kt = {k: v[1] / steps for k, v in plan.kernel_times().items()}
    plan.profile(False)
    # plain per-cluster steps on the same GPU, same particles
    parts = []
    for c in range(len(sizes)):
        sl = slice(off[c], off[c + 1])
        parts.append(([dev(state[i, sl]) for i in range(6)], dev(mass[sl]), cens[c]))
    accs = []
    cs = []
    for stc, mc, cc in parts:
        c1, a1 = plan.step(stc, mc, w.dt, 3, host=host, centre=cc)
        accs.append(a1)
        cs.append(c1)

    def plain():
        for k, (stc, mc, _) in enumerate(parts):
            cs[k], accs[k] = plan.step(stc, mc, w.dt, steps, host=host, centre=cs[k], acc=accs[k])
    _, ms_plain = _timed(torch, plain)
    N = int(off[-1])
    T = plan.T
    return {"workload": w.name, "N_total": N, "clusters": len(sizes), "steps": steps,
            "value": N * T * steps / (ms * 1e-3), "ms_per_step": ms / steps,
            "graph_ms_per_step": ms_graph / steps,
            "plain_per_cluster_value": N * T * steps / (ms_plain * 1e-3),
            "plain_per_cluster_ms_per_step": ms_plain / steps,
            "speedup_vs_plain": ms_plain / ms, "graph_captures": plan.graph_captures,
            "kernels_ms_per_step": kt}


def _energy(torch, plan, st, m):
    """K + W in the cluster frame, W = 1/2 sum m psi_SCF (isolated cluster)."""
    coef = plan.coeffs(st[0], st[1], st[2], m)
    _, _, _, pot = plan.forces(st[0], st[1], st[2], coef, pot=True)
    v2 = st[3].double() ** 2 + st[4].double() ** 2 + st[5].double() ** 2
    md = m.double()
    return float((0.5 * md * v2).sum() + 0.5 * (md * pot.double()).sum())


def _lagrange_radii(torch, st, m, fracs=(0.1, 0.5, 0.9)):
    r = (st[0].double() ** 2 + st[1].double() ** 2 + st[2].double() ** 2).sqrt()
    order = torch.argsort(r)
    cm = torch.cumsum(m.double()[order], 0)
    cm = cm / cm[-1]
    return [float(r[order][torch.searchsorted(cm, torch.tensor(f, dtype=torch.float64,
                                                                   device=cm.device))])
            for f in fracs]


def run_long(torch, scf, I):
    """The isolated Plummer (N = 1e4, 100 steps) and the Plummer in the log
    host (N = 1e5, 1e4 steps): FP32 and FP64 step rates over the whole run,
    energy conservation of the isolated cluster, and FP32-vs-FP64 agreement
    of the final Lagrange radii (trajectories diverge particle by particle,
    so the comparison is statistical)."""
    out = {}
    for w in (I.config1(), I.config2()):
        p = w.clusters[0]
        res = {}
        for dtype in ("f32", "f64"):
            td = torch.float32 if dtype == "f32" else torch.float64
            st = [torch.as_tensor(p.state()[i], dtype=td, device="cuda").contiguous()
                  for i in range(6)]
            m = torch.as_tensor(p.mass, dtype=td, device="cuda")
            plan = scf.Plan(w.nmax, w.lmax, dtype=dtype)
            plan.autotune(st[0], st[1], st[2], m)
            host = (w.host, w.G) if w.host else None
            e0 = _energy(torch, plan, st, m) if not w.host else None
            cen, acc = plan.step([t.clone() for t in st], m, w.dt, 2, host=host,
                                 centre=w.centres[0])  # warm-up
            (cen, acc), ms = _timed(torch, lambda: plan.step(st, m, w.dt, w.nsteps, host=host,
                                                             centre=w.centres[0]))
            r = {"ms_per_step": ms / w.nsteps,
                 "value": p.n * plan.T * w.nsteps / (ms * 1e-3),
                 "lagrange_radii_10_50_90": _lagrange_radii(torch, st, m)}
            if e0 is not None:
                e1 = _energy(torch, plan, st, m)
                r["energy_rel_drift"] = (e1 - e0) / abs(e0)
            res[dtype] = r
        lr32 = res["f32"]["lagrange_radii_10_50_90"]
        lr64 = res["f64"]["lagrange_radii_10_50_90"]
        res["lagrange_radii_rel_diff_f32_vs_f64"] = [abs(a - b) / b for a, b in zip(lr32, lr64)]
        res["steps"] = w.nsteps
        res["N"] = p.n
        out[w.name] = res
    return out


def run_n_scaling(torch, scf, I, sizes=(100_000, 1_000_000, 10_000_000), steps=10):
    """The headline step (Hernquist, nmax 16, lmax 10, FP32, autotuned
    kernels) at several particle counts on the one GPU: throughput as N
    grows, with the field variant the autotuner picks at each size."""
    import numpy as np
    out = []
    for n in sizes:
        p = I.hernquist(n, 13385 + 3)
        st = [torch.as_tensor(np.ascontiguousarray(p.state()[i]), dtype=torch.float32,
                              device="cuda") for i in range(6)]
        m = torch.as_tensor(p.mass, dtype=torch.float32, device="cuda")
        plan = scf.Plan(16, 10, dtype="f32")
        plan.autotune(st[0], st[1], st[2], m)
        # compensated single-precision coefficients against the double-precision
        # path on the same inputs, before the steps move the particles
        c32 = plan.coeffs(st[0], st[1], st[2], m).cpu().numpy()
        p64 = scf.Plan(16, 10, dtype="f64")
        c64 = p64.coeffs(st[0].double(), st[1].double(), st[2].double(), m.double()).cpu().numpy()
        cerr = float(np.abs(c32 - c64).max() / np.abs(c64).max())
        del p64
        cen, acc = plan.step(st, m, 0.005, 2)
        (cen, acc), ms = _timed(torch, lambda: plan.step(st, m, 0.005, steps, centre=cen, acc=acc))
        out.append({"N": n, "ms_per_step": ms / steps, "value": n * plan.T * steps / (ms * 1e-3),
                    "coef_variant": plan.variant, "field_variant": plan.field_variant,
                    "coef_relerr_f32_vs_f64": cerr})
        del st, m, plan, acc
        torch.cuda.empty_cache()
    return {"workload": "hernquist-n16l10 at several N (FP32 step, autotuned)", "steps": steps,
            "sizes": out}


def run_cadence(torch, scf, I, nint=10):
    """Refresh cadence (Sec. 2.2) on the log-host workload (Plummer N = 1e5
    at R = 20, nmax 10, lmax 6, FP32): integration intervals from the tidal
    timestep (eta = 1/400) covered by substeps of at most the workload's dt,
    complete refresh every 5 intervals, r <= r_99.9 selection, one orbit
    sample per t_dyn.  Reports the whole-run time, the per-kind kernel time
    (from a second, event-bracketed run), the plain step over the same
    simulated time for comparison, and the selection at N = 1e6 with its
    algorithmic HBM bytes."""
    w = I.config2()
    p = w.clusters[0]
    host = (w.host, w.G)
    cad = scf.Cadence(eta=1.0 / 400.0, dt_max=w.dt, frac=0.999, refresh_every=5, n_samples_tdyn=1,
                      ns_max=8)
    plan = scf.Plan(w.nmax, w.lmax, dtype="f32")
    st0 = [torch.as_tensor(p.state()[i], dtype=torch.float32, device="cuda").contiguous()
           for i in range(6)]
    m = torch.as_tensor(p.mass, dtype=torch.float32, device="cuda")
    plan.autotune(st0[0], st0[1], st0[2], m)

    def fresh():
        st = [t.clone() for t in st0]
        coef, wts, state = plan.cadence_init(st, m, cad.frac)
        return st, coef, wts, state

    st, coef, wts, state = fresh()
    plan.evolve(st, m, 1, cad, host, w.centres[0], coef, wts, state)  # warm-up
    st, coef, wts, state = fresh()
    torch.cuda.synchronize()
    (cen, state1, log), ms = _timed(torch, lambda: plan.evolve(st, m, nint, cad, host, w.centres[0],
                                                                coef, wts, state))
    st, coef, wts, state = fresh()
    plan.profile(True)
    plan.kernel_times()
    plan.evolve(st, m, nint, cad, host, w.centres[0], coef, wts, state)
    kt = plan.kernel_times()
    plan.profile(False)
    substeps = sum(e["nsub"] for e in log)
    t_sim = sum(e["dt_int"] for e in log)
    # the same run with the frame moved at complete refreshes (Sec. 2.1)
    cad_r = scf.Cadence(eta=cad.eta, dt_max=cad.dt_max, frac=cad.frac,
                        refresh_every=cad.refresh_every, n_samples_tdyn=cad.n_samples_tdyn,
                        ns_max=cad.ns_max, recentre=True)
    st, coef, wts, state = fresh()
    torch.cuda.synchronize()
    (cen_r, _, log_r), ms_r = _timed(torch, lambda: plan.evolve(st, m, nint, cad_r, host,
                                                                 w.centres[0], coef, wts, state))
    # the plain step (coefficients every step) over the same simulated time
    stp = [t.clone() for t in st0]
    nplain = int(round(t_sim / w.dt))
    plan.step([t.clone() for t in st0], m, w.dt, 2, host=host, centre=w.centres[0])
    _, ms_plain = _timed(torch, lambda: plan.step(stp, m, w.dt, nplain, host=host,
                                                   centre=w.centres[0]))
    # the selection alone at N = 1e6 (HBM-bound kernels)
    big = I.plummer(1_000_000, 9001)
    sb = [torch.as_tensor(big.state()[i], dtype=torch.float32, device="cuda").contiguous()
          for i in range(6)]
    mb = torch.as_tensor(big.mass, dtype=torch.float32, device="cuda")
    cb = plan.coeffs(sb[0], sb[1], sb[2], mb)
    plan.select(sb, mb, cb, 0.999)
    plan.profile(True)
    plan.kernel_times()
    for _ in range(5):
        plan.select(sb, mb, cb, 0.999)
    ks = plan.kernel_times()
    plan.profile(False)
    sel_ms = ks["select"][1] / 5 if "select" in ks else None
    # energy + keys: x, y, z, v (6 x 4 B) + psi (4 B) in, key (4 B) + flag (1 B)
    # out; four 8-bit digit passes over the keys (4 x 4 B); weights: key, m in,
    # w out (12 B)
    sel_bytes = 1_000_000 * (28 + 5 + 16 + 12)
    return {
        "workload": f"{w.name} (N = {p.n}), cadence eta = 1/400, dt_max = {w.dt}, "
                    "complete refresh every 5, r <= r_99.9, 1 sample per t_dyn",
        "intervals": nint, "substeps": substeps, "t_simulated": t_sim,
        "ms_total": ms, "ms_per_interval": ms / nint, "us_per_substep": ms * 1e3 / substeps,
        "plain_step_us": ms_plain * 1e3 / nplain, "plain_steps_same_time": nplain,
        "speedup_vs_plain_same_time": ms_plain / ms,
        "kernel_ms_total": {k: v[1] for k, v in kt.items()},
        "intervals_log": [{k: e[k] for k in ("dt_int", "nsub", "nsamples", "kind", "nbound",
                                             "nchanged", "rx", "rhm")} for e in log],
        "recentre": {"ms_total": ms_r, "ms_per_interval": ms_r / nint,
                     "frame_shifts": [{"interval": i, "dx": [float(v) for v in e["dx"]],
                                       "dv": [float(v) for v in e["dv"]]}
                                      for i, e in enumerate(log_r) if e["kind"] == "complete"]},
        "select_N1e6": {"ms": sel_ms, "algorithmic_bytes": sel_bytes,
                        "GB_per_s": sel_bytes / (sel_ms * 1e-3) / 1e9 if sel_ms else None,
                        "note": "energy/key, 4 radix-digit passes and weights kernels; "
                                "the potential evaluation before them is not included"},
    }


def run_adjoint(torch, scf, I, nsteps=None):
    """Plummer N = 1e5 in an NFW host, 2000 steps with checkpoints every 100:
    forward and backward times of the checkpointed autograd trajectory."""
    import numpy as np
    from paper_2602_13385_amd import adjoint as A
    w = I.config5()
    p = w.clusters[0]
    nsteps = nsteps or w.nsteps
    ck = w.extra["checkpoint"]
    track = w.extra["track"]
    plan = scf.Plan(w.nmax, w.lmax, dtype="f32")
    m = torch.as_tensor(p.mass, dtype=torch.float32, device="cuda")
    s0 = torch.as_tensor(p.state(), dtype=torch.float32, device="cuda").contiguous()
    theta = torch.tensor([list(w.host[0][1])], dtype=torch.float64, requires_grad=True)
    cen0 = torch.tensor(w.centres[0], dtype=torch.float64, requires_grad=True)
    plan.autotune(s0[0].contiguous(), s0[1].contiguous(), s0[2].contiguous(), m)
    kinds = [w.host[0][0]]
    # base trajectory: frozen escaper set and nearest track points
    with torch.no_grad():
        sT, cT = A.trajectory(plan, s0, m, theta.detach(), cen0.detach(), kinds, w.dt, nsteps, ck)
        mask = A.escaped_mask(plan, sT, m)
        idx = A.nearest_track_points(sT, cT.numpy(), track, mask)
    # warm-up: one untimed forward and backward of the same trajectory
    # (workspace, checkpoint buffers and kernel loading)
    th_w = theta.detach().clone().requires_grad_(True)
    sw, cw = A.trajectory(plan, s0.clone().requires_grad_(True), m, th_w, cen0.detach(), kinds,
                          w.dt, nsteps, ck)
    A.track_loss(sw, cw, track, mask, idx).backward()
    s0g = s0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sT, cT = A.trajectory(plan, s0g, m, theta, cen0, kinds, w.dt, nsteps, ck)
    L = A.track_loss(sT, cT, track, mask, idx)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    g = theta.grad.numpy()[0]
    return {"workload": w.name, "N": p.n, "steps": nsteps, "checkpoint": ck,
            "forward_s": t_fwd, "backward_s": t_bwd, "adjoint_forward_ratio": t_bwd / t_fwd,
            "escapers": int(mask.sum().item()), "loss": float(L.item()),
            "dL_dM_s": float(g[0]), "dL_dr_s": float(g[1]),
            "dL_dcentre0": [float(v) for v in cen0.grad.numpy()],
            "timing": "wall clock around the autograd forward (checkpointed scf_step segments + "
                      "loss) and backward (scf_step_adjoint per segment, recompute included)",
            "accuracy_vs_horizon": adjoint_horizons(torch, scf, I)}


def adjoint_horizons(torch, scf, I, horizons=(100, 500, 1000, 2000), h_rel=1e-5):
    """The adjoint workload's gradient of the track loss with respect to
    (M_s, r_s, R0, V0) at several horizons: the FP64 adjoint against FP64
    central differences of the same loss (step h_rel of the parameter, or of
    max(1, |coordinate|)), and the FP32 adjoint against the FP64 one,
    componentwise; escaper set and nearest track points frozen at the FP64
    base trajectory of each horizon."""
    import numpy as np
    from paper_2602_13385_amd import adjoint as A
    w = I.config5()
    p = w.clusters[0]
    ck, track = w.extra["checkpoint"], w.extra["track"]
    kinds = [w.host[0][0]]
    theta0 = np.array([list(w.host[0][1])])
    cen0 = np.array(w.centres[0])

    def setup(dtype):
        td = torch.float32 if dtype == "f32" else torch.float64
        return (scf.Plan(w.nmax, w.lmax, dtype=dtype),
                torch.as_tensor(p.mass, dtype=td, device="cuda"),
                torch.as_tensor(p.state(), dtype=td, device="cuda").contiguous())

    def grad(plan, m, s0, H, mask, idx):
        th = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
        c = torch.tensor(cen0, dtype=torch.float64, requires_grad=True)
        sT, cT = A.trajectory(plan, s0.clone(), m, th, c, kinds, w.dt, H, ck)
        A.track_loss(sT, cT, track, mask, idx).backward()
        return np.concatenate([th.grad.numpy()[0][:2], c.grad.numpy()]), sT

    (p64, m64, s64), (p32, m32, s32) = setup("f64"), setup("f32")
    rows = []
    for H in horizons:
        with torch.no_grad():
            sT, cT = A.trajectory(p64, s64, m64, torch.as_tensor(theta0), torch.as_tensor(cen0),
                                  kinds, w.dt, H, ck)
            mask = A.escaped_mask(p64, sT, m64)
            idx = A.nearest_track_points(sT, cT.numpy(), track, mask)
        g64, sT64 = grad(p64, m64, s64, H, mask, idx)

        def loss(theta, cen):
            with torch.no_grad():
                a, b = A.trajectory(p64, s64, m64, torch.as_tensor(theta), torch.as_tensor(cen),
                                    kinds, w.dt, H, ck)
                return float(A.track_loss(a, b, track, mask, idx).item())
        fd = np.zeros(8)
        for q in range(8):
            th, c = theta0.copy(), cen0.copy()
            arr, k = (th[0], q) if q < 2 else (c, q - 2)
            h = h_rel * (abs(arr[k]) if q < 2 else max(1.0, abs(arr[k])))
            arr[k] += h
            lp = loss(th, c)
            arr[k] -= 2 * h
            fd[q] = (lp - loss(th, c)) / (2 * h)
        g32, sT32 = grad(p32, m32, s32, H, mask, idx)
        rows.append({"steps": H, "escapers": int(mask.sum().item()),
                     "grad_f64": [float(v) for v in g64],
                     "relerr_f64_adjoint_vs_f64_fd": [float(v) for v in np.abs(g64 - fd) / np.abs(g64)],
                     "relerr_f32_vs_f64_adjoint": [float(v) for v in np.abs(g32 - g64) / np.abs(g64)],
                     "forward_pos_relerr_f32_vs_f64": float(
                         ((sT32[:3].double() - sT64[:3]).abs().max() / sT64[:3].abs().max()).item())})
    return {"parameters": ["M_s", "r_s", "X0", "Y0", "Z0", "VX0", "VY0", "VZ0"],
            "fd_step": h_rel, "horizons": rows}


def run_diagnostics(torch, scf, I, chunks=10, per_chunk=200):
    """Power per degree E_l(t) and the tidal-tensor norm ||T||(t) along the
    eccentric orbit of the first progenitor of the batched workload, each
    normalised by its initial value (the paper's power-spectrum time series)."""
    w = I.config4()
    p = w.clusters[0]
    st = [torch.as_tensor(p.state()[i], dtype=torch.float32, device="cuda").contiguous()
          for i in range(6)]
    m = torch.as_tensor(p.mass, dtype=torch.float32, device="cuda")
    plan = scf.Plan(w.nmax, w.lmax, dtype="f32")
    host = (w.host, w.G)
    coef = torch.empty(plan.T, dtype=torch.float64, device="cuda")
    cen, acc = plan.step(st, m, w.dt, 0, host=host, centre=w.centres[0], coef_last=coef)
    rows = []
    for k in range(chunks + 1):
        E = plan.power(coef).cpu().numpy()
        rows.append({"t": k * per_chunk * w.dt, "E_l": [float(v) for v in E],
                     "tidal_norm": scf.tidal_norm(host, cen[:3]), "R": float(sum(cen[:3] ** 2) ** 0.5)})
        if k < chunks:
            cen, acc = plan.step(st, m, w.dt, per_chunk, host=host, centre=cen, acc=acc,
                                 coef_last=coef)
    E0 = rows[0]["E_l"]
    T0 = rows[0]["tidal_norm"]
    return {"workload": f"{w.name} (cluster 0, N = {p.n})", "dt": w.dt,
            "t": [r["t"] for r in rows], "R": [r["R"] for r in rows],
            "E_l_over_initial": [[e / e0 for e, e0 in zip(r["E_l"], E0)] for r in rows],
            "tidal_norm_over_initial": [r["tidal_norm"] / T0 for r in rows]}


def run_ceilings(scf):
    """Issue-rate ceilings (scf_bench_ceiling): single-precision FMA chains
    without packed FP32, and FP32 MFMA chains, at 1, 2, 4 and 8 waves per
    SIMD, in TFLOP/s."""
    names = {0: "fma_f32_16_chains", 1: "fma_f32_32_chains", 2: "mfma_f32_4x4x1",
             3: "mfma_f32_16x16x4", 4: "mfma_f32_32x32x2"}
    out = {}
    for kind, name in names.items():
        out[name] = {str(wv): scf.bench_ceiling(kind, wv, 4000 if kind < 2 else 2000)[0]
                     for wv in (1, 2, 4, 8)}
    out["note"] = "waves per SIMD -> TFLOP/s; the kernels' roofline fractions are read against these"
    # overlap check: kinds 0 and 2 together in every wave against the sum of
    # their separate times (same iters and waves)
    ov = {}
    for wv in (2, 4, 8):
        t_fma = scf.bench_ceiling(0, wv, 4000)[1]
        t_mfma = scf.bench_ceiling(2, wv, 4000)[1]
        t_mix = scf.bench_ceiling(5, wv, 4000)[1]
        ov[str(wv)] = {"fma_ms": t_fma, "mfma_ms": t_mfma, "both_ms": t_mix,
                       "both_over_sum": t_mix / (t_fma + t_mfma),
                       "both_over_max": t_mix / max(t_fma, t_mfma)}
    out["fma_mfma_overlap"] = ov
    return out


def device_info(torch):
    """Device name and the shader-clock level the driver marks active in sysfs
    at the time of the call (read as a file; no helper program runs)."""
    import glob
    info = {"name": torch.cuda.get_device_name(0)}
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            with open(path) as f:
                levels = [ln.strip() for ln in f if ln.strip()]
        except OSError:
            continue
        active = [ln for ln in levels if ln.endswith("*")]
        # the level the driver reports at the moment of the read (the clock
        # drops within milliseconds of the GPU going idle)
        info["sclk_level_at_read"] = active[0] if active else (levels[-1] if levels else None)
        break
    return info


def cpu_baseline(nsample=1_000_000, reps=2):
    """The FP64 oracle (OpenMP over the host's cores) on `reps` coefficient +
    field passes over the headline workload's particles."""
    from oracle import pyoracle as O
    from paper_2602_13385_amd import inputs as I
    w = I.config3()
    p = w.clusters[0]
    B = O.basis(w.nmax, w.lmax, alpha=w.alpha, b=w.b, G=w.G)
    pos = p.pos[:, :nsample].copy()
    mass = p.mass[:nsample].copy()
    t0 = time.perf_counter()
    for _ in range(reps):
        c = O.coeffs(B, *pos, mass)
        O.field(B, c, *pos, pot=False)
    t = time.perf_counter() - t0
    T = O.ncoef(w.nmax, w.lmax)
    cores = O.num_threads()
    # the same passes on one core, over a 2e4-particle slice
    n1 = 20_000
    O.set_threads(1)
    t1 = time.perf_counter()
    c1 = O.coeffs(B, *pos[:, :n1], mass[:n1])
    O.field(B, c1, *pos[:, :n1], pot=False)
    t1 = time.perf_counter() - t1
    O.set_threads(cores)
    return {"value": reps * nsample * T / t, "unit": "particle-terms/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{reps} coefficient + field passes of the FP64 oracle over the {nsample} "
                      f"particles of the Hernquist N=1e6 nmax=16 lmax=10 workload ({t:.1f} s)",
            "single_core_value": n1 * T / t1,
            "single_core_sample": f"one coefficient + field pass over the first {n1} of those "
                                  f"particles on 1 thread ({t1:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default=None, metavar="COEF,FIELD",
                    help="pin the headline run's coefficient and field kernel variants "
                         "instead of autotuning them (profiling runs)")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--legs", default="all",
                    help="comma list of extra legs (f64, accuracy, batched, adjoint, long, "
                         "diagnostics, cadence, nscaling, ceilings) or 'all'")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline FP32 workload only (no FP64, batched, adjoint, accuracy)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy (for counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the hot path runs on one GPU only; --gpus {args.gpus} is not "
              f"supported (the multi-GPU sharding is a design note, not built)", file=sys.stderr)
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
    print("[bench] headline FP32", file=sys.stderr, flush=True)
    pinned = tuple(int(v) for v in args.variants.split(",")) if args.variants else None
    r = run_main("f32", args.steps, args.warmup, torch, scf, I, profile=True, variants=pinned)
    dev = device_info(torch)  # the clock level right after the headline runs
    n, T = r["n"], r["T"]
    ms_per_step = r["ms"] / args.steps
    value = n * T * args.steps / (r["ms"] * 1e-3)
    fl = algorithmic_flops(r["nmax"], r["lmax"])
    kt = r["kernels"]
    per_kernel = {}
    for k in ("coef", "field_step"):
        if k in kt:
            cnt, tot = kt[k]
            avg_s = tot / cnt * 1e-3
            tf = fl[k] * n / avg_s / 1e12
            e = roofline_entry(k, tf, r["field_variant"], None, fl[k] * n, tot / cnt)
            per_kernel[k] = {"avg_launch_ms": tot / cnt, "tflops": tf, "bound": e["bound"],
                             "frac": e["frac"]}
            if "frac_single_issue_valu" in e:
                per_kernel[k]["frac_single_issue_valu"] = e["frac_single_issue_valu"]
    dom = max(per_kernel, key=lambda k: per_kernel[k]["avg_launch_ms"])
    achieved = per_kernel[dom]["tflops"]
    step_tf = (fl["coef"] + fl["field_step"]) * n / (ms_per_step * 1e-3) / 1e12
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
                   "alpha": 1.0, "dt": r["dt"], "host": None, "coef_variant": r["variant"],
                   "field_variant": r["field_variant"], "coef_units_div": r["coef_units_div"]},
        "roofline": roofline_entry(dom, achieved, r["field_variant"], measured_traffic(dom),
                                   fl[dom] * n, per_kernel[dom]["avg_launch_ms"]),
        "kernels": per_kernel,
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in kt.items()},
        "step_tflops": step_tf,
        "step_frac": step_tf / PEAK_FP32_TFLOPS,
    }
    del r["plan"]
    legs = set(("f64", "accuracy", "batched", "adjoint", "long", "diagnostics", "cadence",
                "nscaling", "ceilings")
               if args.legs == "all" else args.legs.split(","))
    if args.no_f64:
        legs.discard("f64")
    if not args.no_extras:
        if "f64" in legs:
            print("[bench] FP64", file=sys.stderr, flush=True)
            steps64 = max(1, args.steps // 4)
            r64 = run_main("f64", steps64, max(1, args.warmup // 4), torch, scf, I, profile=True)
            tf64 = (fl["coef"] + fl["field_step"]) * n / (r64["ms"] / steps64 * 1e-3) / 1e12
            k64 = {}
            for k in ("coef", "field_step"):
                if k in r64["kernels"]:
                    cnt, tot = r64["kernels"][k]
                    tfk = fl[k] * n / (tot / cnt * 1e-3) / 1e12
                    k64[k] = {"avg_launch_ms": tot / cnt, "tflops": tfk,
                              "frac_fp64_peak": tfk / PEAK_FP64_TFLOPS}
            out["f64"] = {"value": n * T * steps64 / (r64["ms"] * 1e-3),
                          "ms_per_step": r64["ms"] / steps64, "steps": steps64,
                          "step_tflops": tf64, "frac_fp64_peak": tf64 / PEAK_FP64_TFLOPS,
                          "f32_over_f64_speed": (r64["ms"] / steps64) / ms_per_step,
                          "config": {"coef_variant": r64["variant"],
                                     "field_variant": r64["field_variant"],
                                     "coef_units_div": r64["coef_units_div"]},
                          "kernels": k64,
                          "kernels_ms_per_step": {k: v[1] / steps64
                                                  for k, v in r64["kernels"].items()}}
            del r64["plan"]
        legs_fn = [("accuracy", "accuracy", lambda: accuracy_main(torch, scf, I)),
                   ("batched", "batched", lambda: run_batched(torch, scf, I, steps=1000)),
                   ("ceilings", "throughput ceilings", lambda: run_ceilings(scf)),
                   ("adjoint", "adjoint", lambda: run_adjoint(torch, scf, I)),
                   ("long", "long runs", lambda: run_long(torch, scf, I)),
                   ("diagnostics", "diagnostics", lambda: run_diagnostics(torch, scf, I)),
                   ("cadence", "cadence", lambda: run_cadence(torch, scf, I)),
                   ("nscaling", "N scaling", lambda: run_n_scaling(torch, scf, I))]
        for key, label, fn in legs_fn:
            if key in legs:
                print(f"[bench] {label}", file=sys.stderr, flush=True)
                out["long_runs" if key == "long" else key] = fn()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    else:
        out["cpu_baseline"] = None
    out["paper_context"] = PAPER_CONTEXT
    out["device"] = dev
    print(json.dumps(out))


if __name__ == "__main__":
    main()
