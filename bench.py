#!/usr/bin/env python3
"""Throughput of the NUFFT forward+adjoint pair (PyNUFFT, arXiv 1710.03197,
Section 2.1: A = V F S, A^H = S^H F^H V^H) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one forward + adjoint pair on the 2D 256x256 golden-angle radial
workload (grid 512x512, J = 6, M = 131072, complex64, synthetic seeded data,
inputs resident in HBM).  Before timing, the pair is checked against the FP64
oracle at relative L2 <= 1e-5.  Prints one JSON line with pairs/s, the
roofline of the dominant kernel (per-kernel HIP events recorded by the
library on the launch stream, in a second loop identical to the timed one),
the FP64 oracle timed on the host cores, and extra fields for the 3D 128^3
koosh-ball pair, for the uneven multi-problem batch (24 spiral problems x 8
coils, one launch per stage) versus looped single transforms, for the
achievable device-to-device copy bandwidth, for the dispatch floor of a
six-kernel sequence (eager and graph-replayed), and for the method's own
NUFFT-versus-NUDFT error (the FP64 oracle against the direct sum at the
64x64 / 4096-sample configuration).

The oracle (test infrastructure) is used only in the CPU-baseline leg: its
timing, and its reference outputs for the parity gates and the NUDFT error.
`--workloads` picks the parts to run (profiling runs use one at a time).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "NUFFT fwd+adj pairs/s, 2D 256² & 3D 128³ at rel err≤1e-5; batched vs looped"
TOL = 1e-5

# HBM traffic per launch of the dominant kernel, from two rocprofv3 --pmc runs
# of this benchmark: read bytes = 128 TCC_EA0_RDREQ_128B + 64 TCC_EA0_RDREQ_64B
# + 32 TCC_EA0_RDREQ_32B, write bytes = 64 TCC_EA0_WRREQ_64B + 32 (the rest of
# TCC_EA0_WRREQ); the 1 GiB device copy this benchmark times reads and writes
# exactly its size by the same formulas (profiles/traffic_2d_256_radial.md,
# profiles/traffic_3d_128_koosh.md).  An entry applies only while kernels.hip
# has the recorded sha256 prefix and the plan uses the recorded options;
# otherwise traffic is reported as null.
MEASURED_TRAFFIC: dict = {
    ("k_grid", "2d_256_golden_radial"): {
        "kernels_sha": "40e87707b14d1007",
        "options": {"fft_groups": 512, "grid_chunk": 512, "interp_merge": 2, "tile": [16, 16], "weight_table": 1},
        "read_bytes": 18463296, "write_bytes": 2308096, "bytes_per_launch": 20771392},
    ("k_grid", "3d_128_koosh"): {
        "kernels_sha": "40e87707b14d1007",
        "options": {"fft_groups": 1024, "grid_chunk": 1536, "grid_waves": 1, "interp_merge": 4, "presort": 2,
                    "tile": [8, 8, 16], "weight_table": 1},
        "read_bytes": 798889184, "write_bytes": 149938176, "bytes_per_launch": 948827360},
}


def kernels_hash() -> str:
    with open(os.path.join(ROOT, "paper_1710_03197_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def prod(v):
    p = 1
    for a in v:
        p *= int(a)
    return p


def algorithmic_bytes(N, K, M, J):
    """Bytes each kernel must move per forward+adjoint pair if every stage
    reads and writes its arrays exactly once (complex64 = 8 B, float32 om):
    the FFT passes read the previous stage's array and write theirs (pruned to
    the non-zero rows), V reads the grid (at most once), om and writes y, V^H
    reads y and om and writes the grid.  Returns {kernel: bytes per pair}."""
    d = len(N)
    out = {}

    def add(name, b):
        out[name] = out.get(name, 0) + b

    for p in range(d):  # forward passes, last axis first: N_ax rows in, K_ax rows out
        ax = d - 1 - p
        lead, tail = prod(N[:ax]), prod(K[ax + 1:])
        add("k_first_pass" if p == 0 else "k_strided_pass<fwd>", 8 * lead * tail * (N[ax] + K[ax]))
    for ax in range(d):  # adjoint passes, first axis first: K_ax rows in, N_ax rows out
        lead, tail = prod(N[:ax]), prod(K[ax + 1:])
        add("k_last_pass" if ax == d - 1 else "k_strided_pass<inv>", 8 * lead * tail * (K[ax] + N[ax]))
    add("k_interp", 8 * min(prod(K), M * J ** d) + 4 * d * M + 8 * M)
    add("k_grid", 8 * M + 4 * d * M + 8 * prod(K))
    return out


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def time_pairs(plan, x, y, xa, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.forward(x, out=y)
        plan.adjoint(y, out=xa)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forward(x, out=y)
        plan.adjoint(y, out=xa)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_graph_pairs(plan, x, y, xa, steps, warmup):
    """The same pair captured once into a HIP graph (torch.cuda.CUDAGraph) and
    replayed: launch overhead removed, same kernels and work."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.forward(x, out=y)
        plan.adjoint(y, out=xa)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.forward(x, out=y)
        plan.adjoint(y, out=xa)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_toeplitz(plan, x, xa, steps, warmup, sec_pair):
    """The Toeplitz normal operator A^H A of the same plan (two 2N-grid FFTs
    and a product per application) against the pair A^H (A x): time per
    application, and its difference to the pair (both approximate A^H A; the
    oracle parity of the operator is in the tests)."""
    import time
    import torch
    t0 = time.perf_counter()
    T = plan.toeplitz()
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    out = torch.empty_like(xa)
    y = plan.forward(x)
    ref = plan.adjoint(y)
    T(x, out=out)
    torch.cuda.synchronize()
    diff = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(ref))
    for _ in range(warmup):
        T(x, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        T(x, out=out)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / steps
    T.close()
    return {"applications_per_s": round(1.0 / sec, 2), "ms_per_application": round(sec * 1e3, 4),
            "speedup_vs_pair": round(sec_pair / sec, 3), "rel_diff_vs_pair": diff,
            "plan_ms": round(plan_ms, 2)}


def kernel_times(plan, x, y, xa, steps):
    """Per-kernel launches and mean duration (ms) over `steps` pairs, from the
    library's HIP events on the launch stream."""
    import torch
    torch.cuda.synchronize()
    plan.timing(True)
    for _ in range(steps):
        plan.forward(x, out=y)
        plan.adjoint(y, out=xa)
    torch.cuda.synchronize()
    rep = plan.timing_report()
    plan.timing(False)
    return {k: (n / steps, ms / n) for k, (n, ms) in rep.items()}


def roofline_entry(ktimes, alg, steps_hash, workload=None, options=None):
    """Roofline of the kernel with the largest share of the pair's time among
    the stages of the byte model (the partial-tile sums and the sample
    permutation are artefacts of the gridding's work split, not stages)."""
    dom = max((k for k in ktimes if k in alg), key=lambda k: ktimes[k][0] * ktimes[k][1])
    launches_per_pair, avg_ms = ktimes[dom]
    bytes_per_launch = alg[dom] / launches_per_pair
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    m = MEASURED_TRAFFIC.get((dom, workload))
    if m and m.get("kernels_sha") == steps_hash and m.get("options") == options:
        traffic = m["bytes_per_launch"]
    return dom, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                 "kernel": dom, "algorithmic_bytes_per_launch": int(bytes_per_launch),
                 "avg_launch_us": round(avg_ms * 1e3, 2)}


def make_plan(om_t, N, K, J, tune):
    """The plan bench.py times.  tune="cache": the options the autotuner stored
    for this workload in paper_1710_03197_amd/tuning_gfx950.json (defaults if
    absent); "now": tune here (every candidate parity-checked against the
    default plan); "off": built-in defaults."""
    from paper_1710_03197_amd import Plan, autotune
    if tune == "off":
        return Plan(om_t, N, K, J), None
    if tune == "now":
        res = autotune.tune(om_t, N, K, J, reps=10, save=False)
        print(f"[bench] tuned {res['options']}: {res['ms_pair']:.4f} ms/pair (defaults {res['default_ms_pair']:.4f})",
              flush=True)
        return Plan(om_t, N, K, J, options=res["options"]), dict(res, source="tuned in this run")
    opts = autotune.cached_options(N, K, J, int(om_t.shape[0]), autotune.SHIPPED_CACHE, om_t.device)
    print(f"[bench] options from the tuning cache: {opts}", flush=True)
    return Plan(om_t, N, K, J, options=opts), {"options": opts, "source": "paper_1710_03197_amd/tuning_gfx950.json"}


def bench_2d(dev, steps, warmup, orc_mod, tune="cache", no_graph=False):
    import numpy as np
    import torch
    from paper_1710_03197_amd import Plan, data
    c = data.config2()
    N, K, J, om = c["N"], c["K"], c["J"], c["om"]
    M = om.shape[0]
    print(f"[bench] 2D workload N={N} K={K} J={J} M={M}", flush=True)
    plan, tuned = make_plan(torch.from_numpy(om).to(dev), N, K, J, tune)
    x = torch.from_numpy(c["x"]).to(dev)
    y = torch.empty(M, dtype=torch.complex64, device=dev)
    xa = torch.empty(N, dtype=torch.complex64, device=dev)
    # parity gate at the benchmarked configuration
    plan.forward(x, out=y)
    plan.adjoint(y, out=xa)
    torch.cuda.synchronize()
    y_np = y.cpu().numpy()
    err_f = rel_l2(y_np, orc_mod.forward(c["x"], om, N, K, J))
    err_a = rel_l2(xa.cpu().numpy(), orc_mod.adjoint(y_np, om, N, K, J))
    print(f"[bench] 2D parity: forward {err_f:.2e}, adjoint {err_a:.2e}", flush=True)
    if not (err_f <= TOL and err_a <= TOL):
        raise SystemExit(f"parity gate failed: forward {err_f:.2e}, adjoint {err_a:.2e}")
    sec = time_pairs(plan, x, y, xa, steps, warmup)
    ktimes = kernel_times(plan, x, y, xa, steps)
    sec_graph = None if no_graph else time_graph_pairs(plan, x, y, xa, steps, warmup)
    toep = time_toeplitz(plan, x, xa, steps, warmup, sec)
    alg = algorithmic_bytes(N, K, M, J)
    info = plan.info()
    opts = dict((tuned or {}).get("options") or {})
    plan.close()
    # the paper's default interpolator (min-max) on the same workload: parity
    # on 2048 sampled outputs against the oracle's direct definition, then time
    # (the window table holds Kaiser-Bessel weights only: min-max plans
    # evaluate their coefficients on the fly)
    mm_opts = {k: v for k, v in opts.items() if k != "weight_table"}
    pm = Plan(torch.from_numpy(om).to(dev), N, K, J, options=dict(mm_opts, interpolator="minmax"))
    pm.forward(x, out=y)
    torch.cuda.synchronize()
    pick = np.random.default_rng(0).choice(M, 2048, replace=False)
    err_mm = rel_l2(y.cpu().numpy()[pick], orc_mod.minmax_forward(c["x"], om[pick], N, K, J))
    if not err_mm <= TOL:
        raise SystemExit(f"min-max parity gate failed: {err_mm:.2e}")
    sec_mm = time_pairs(pm, x, y, xa, steps, warmup)
    pm.close()
    minmax = {"pairs_per_s": round(1.0 / sec_mm, 2), "ms_per_pair": round(sec_mm * 1e3, 4),
              "rel_err_forward_sampled": err_mm}
    return dict(sec=sec, sec_graph=sec_graph, ktimes=ktimes, alg=alg, err_f=err_f, err_a=err_a, N=N, K=K, M=M,
                J=J, info=info, tuned=tuned, toeplitz=toep, minmax=minmax)


def bench_3d(dev, steps, warmup, orc_mod, tune="cache"):
    import torch
    from paper_1710_03197_amd import Plan, data
    c = data.config3()
    N, K, J, om = c["N"], c["K"], c["J"], c["om"]
    M = om.shape[0]
    print(f"[bench] 3D workload N={N} K={K} J={J} M={M}", flush=True)
    plan, tuned = make_plan(torch.from_numpy(om).to(dev), N, K, J, tune)
    x = torch.from_numpy(c["x"]).to(dev)
    y = torch.empty(M, dtype=torch.complex64, device=dev)
    xa = torch.empty(N, dtype=torch.complex64, device=dev)
    plan.forward(x, out=y)
    torch.cuda.synchronize()
    err_f = rel_l2(y.cpu().numpy(), orc_mod.forward(c["x"], om, N, K, J))
    print(f"[bench] 3D parity: forward {err_f:.2e}", flush=True)
    if not err_f <= TOL:
        raise SystemExit(f"3D parity gate failed: forward {err_f:.2e}")
    sec = time_pairs(plan, x, y, xa, steps, warmup)
    ktimes = kernel_times(plan, x, y, xa, max(2, steps // 2))
    toep = time_toeplitz(plan, x, xa, steps, warmup, sec)
    alg = algorithmic_bytes(N, K, M, J)
    plan.close()
    return dict(sec=sec, ktimes=ktimes, alg=alg, err_f=err_f, tuned=tuned, toeplitz=toep)


def bench_batched(dev, steps, warmup, orc_mod, n_problems=24):
    """Config 4: 24 uneven 2D spiral problems x 8 coils.  Batched: one
    multi-plan (coil maps fused into each problem's launches, all problems in
    one captured HIP graph).  Looped: a single-coil plan per problem, called
    once per (problem, coil) with the pre-multiplied image c_i x."""
    import numpy as np
    import torch
    from paper_1710_03197_amd import Plan, data
    from paper_1710_03197_amd.plan import MultiPlan
    probs = data.config4(n_problems=n_problems)
    C = probs[0]["coils"].shape[0]
    print(f"[bench] batched: {len(probs)} spiral problems x {C} coils, "
          f"M {min(p['om'].shape[0] for p in probs)}..{max(p['om'].shape[0] for p in probs)}", flush=True)
    oms = [torch.from_numpy(p["om"]).to(dev) for p in probs]
    coils = [torch.from_numpy(p["coils"]).to(dev) for p in probs]
    xs = [torch.from_numpy(p["x"]).to(dev) for p in probs]
    # both sides take each problem's options from the shipped tuning cache
    # (tuned in coil mode for these sizes), defaults where it has none
    mp = MultiPlan([dict(om=o, N=p["N"], coils=c) for o, p, c in zip(oms, probs, coils)], J=6, tune="cache")
    ys = mp.forward(xs)
    xa = mp.adjoint(ys)
    torch.cuda.synchronize()
    errs = []
    for p in (0, len(probs) - 1):  # parity at the same accuracy before timing
        pr = probs[p]
        yo = orc_mod.forward_coils(pr["x"], pr["coils"], pr["om"], pr["N"], pr["K"], 6)
        errs.append(rel_l2(ys[p].cpu().numpy(), yo))
    print(f"[bench] batched parity: {[f'{e:.2e}' for e in errs]}", flush=True)
    if max(errs) > TOL:
        raise SystemExit("batched parity gate failed")
    from paper_1710_03197_amd import autotune
    singles = [Plan(o, p["N"], p["K"], 6, options=autotune.cached_options(p["N"], p["K"], 6, int(o.shape[0]),
                                                                           autotune.SHIPPED_CACHE, dev, C))
               for o, p in zip(oms, probs)]
    cxs = [c * x[None] for c, x in zip(coils, xs)]
    ybuf = [torch.empty((C, p["om"].shape[0]), dtype=torch.complex64, device=dev) for p in probs]
    xbuf = [torch.empty_like(cx) for cx in cxs]

    def run_batched():
        mp.forward(xs, ys)
        mp.adjoint(ys, xa)

    def run_looped():
        for sp, cx, yb, xb in zip(singles, cxs, ybuf, xbuf):
            for i in range(C):
                sp.forward(cx[i], out=yb[i])
                sp.adjoint(yb[i], out=xb[i])

    res = {}
    for name, fn in (("batched", run_batched), ("looped", run_looped)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / steps
    n_pairs = C * len(probs)
    mp.close()
    for sp in singles:
        sp.close()
    return dict(pairs_per_s_batched=round(n_pairs / res["batched"], 1),
                pairs_per_s_looped=round(n_pairs / res["looped"], 1),
                speedup=round(res["looped"] / res["batched"], 3), problems=len(probs), coils=C,
                ms_per_batch_batched=round(res["batched"] * 1e3, 3), rel_err=max(errs))


def stream_copy(dev, mib=1024, reps=20):
    """Achievable HBM bandwidth: a device-to-device copy of `mib` MiB (read
    and write counted), best of `reps` event-timed copies."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    best = None
    for _ in range(reps + 2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    gbs = 2 * n * 4 / (best * 1e-3) / 1e9
    del src, dst
    return {"gb_per_s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes_moved": 2 * n * 4,
            "kind": "torch device-to-device copy, best of %d" % reps}


def dispatch_floor(dev, n_launch=6, steps=2000):
    """Time of a sequence of `n_launch` one-workgroup kernels (the pair's
    launch count in 2D), back to back on one stream, eager and as a replayed
    HIP graph: the floor under which the 2D pair cannot go."""
    import torch
    bufs = [torch.zeros(64, device=dev) for _ in range(n_launch)]

    def seq():
        for b in bufs:
            b.add_(1.0)

    out = {}
    for _ in range(20):
        seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        seq()
    torch.cuda.synchronize()
    out["eager_us"] = round((time.perf_counter() - t0) / steps * 1e6, 2)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        seq()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        seq()
    for _ in range(20):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    out["graph_us"] = round((time.perf_counter() - t0) / steps * 1e6, 2)
    out["launches"] = n_launch
    return out


def nudft_error(orc_mod):
    """The method's approximation error at J = 6, sigma = 2: the FP64 oracle
    (which follows the NUFFT pipeline) against the direct non-uniform DFT
    y_m = sum_n x_n exp(-i omega_m . n), n centred, on the 64x64 image with 32
    radial spokes x 128 readout points."""
    import numpy as np
    from paper_1710_03197_amd import data
    c = data.config1()
    N, K, J, om, x = c["N"], c["K"], c["J"], c["om"], c["x"]
    grids = np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij")
    pts = np.stack([g.ravel() for g in grids], 1).astype(np.float64)
    y = np.exp(-1j * (om.astype(np.float64) @ pts.T)) @ x.astype(np.complex128).ravel()
    return {"rel_l2": rel_l2(orc_mod.forward(x, om, N, K, J), y), "workload": "64x64, grid 128x128, J=6, M=4096"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(orc_mod, budget_s=12.0):
    """The FP64 oracle pair on the 2D workload, repeated for about budget_s."""
    from paper_1710_03197_amd import data
    c = data.config2()
    N, K, J, om, x = c["N"], c["K"], c["J"], c["om"], c["x"]
    reps = 0
    t0 = time.perf_counter()
    while True:
        y = orc_mod.forward(x, om, N, K, J)
        orc_mod.adjoint(y, om, N, K, J)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    sec = (time.perf_counter() - t0) / reps
    return {"value": round(1.0 / sec, 3), "unit": "pairs/s", "cores": orc_mod.num_threads(), "kind": "oracle",
            "sample": f"{reps} full FP64 forward+adjoint pairs of the 2D 256^2 workload (M=131072), "
                      f"{sec * 1e3:.1f} ms each",
            "cpu_model": cpu_model(), "omp_proc_bind": os.environ.get("OMP_PROC_BIND")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workloads", default="2d,3d,batched",
                    help="comma-separated parts to run: 2d (the headline value), 3d, batched")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--tune", choices=["cache", "now", "off"], default="cache",
                    help="plan options: the shipped tuning cache, tune in this run, or built-in defaults")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--calibration-copy-mb", type=int, default=0,
                    help="after timing, copy this many MiB device to device (a plain copy of known size "
                         "for scaling FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        raise SystemExit(2)

    parts = {w.strip() for w in args.workloads.split(",") if w.strip()}
    if args.no_3d:
        parts.discard("3d")
    if args.no_batched:
        parts.discard("batched")
    # the FP64 oracle's OpenMP threads stay on adjacent cores (set before the
    # oracle library starts its runtime)
    os.environ.setdefault("OMP_PROC_BIND", "close")
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    import oracle as orc_mod
    dev = torch.device("cuda:0")
    khash = kernels_hash()

    r2, roof = None, None
    extra = {"kernels_sha": khash}
    if "2d" in parts:
        r2 = bench_2d(dev, args.steps, args.warmup, orc_mod, tune=args.tune, no_graph=args.no_graph)
        dom, roof = roofline_entry(r2["ktimes"], r2["alg"], khash, "2d_256_golden_radial",
                                   (r2["tuned"] or {}).get("options"))
        extra.update({
            "rel_err_forward": r2["err_f"], "rel_err_adjoint": r2["err_a"],
            "kernels_us_per_pair": {k: round(n * ms * 1e3, 2) for k, (n, ms) in r2["ktimes"].items()},
            "graph_replay_pairs_per_s": None if r2["sec_graph"] is None else round(1.0 / r2["sec_graph"], 2),
            "pair_bytes_model": int(sum(r2["alg"].values())),
            "pair_model_frac": round(sum(r2["alg"].values()) / r2["sec"] / 1e9 / HBM_PEAK_GBS, 4),
            "plan": r2["info"], "tuning": r2["tuned"],
            "toeplitz_normal_2d": r2["toeplitz"],
            "minmax_interpolator_2d": r2["minmax"],
            "dispatch_floor_6_launches": dispatch_floor(dev, steps=max(20, min(2000, args.steps))),
        })
    if "3d" in parts:
        r3 = bench_3d(dev, max(5, args.steps // 10), max(2, args.warmup // 4), orc_mod, tune=args.tune)
        _, roof3 = roofline_entry(r3["ktimes"], r3["alg"], khash, "3d_128_koosh", (r3["tuned"] or {}).get("options"))
        extra["3d_128"] = {
            "pairs_per_s": round(1.0 / r3["sec"], 2), "ms_per_pair": round(r3["sec"] * 1e3, 4),
            "rel_err_forward": r3["err_f"],
            "pair_bytes_model": int(sum(r3["alg"].values())),
            "pair_model_frac": round(sum(r3["alg"].values()) / r3["sec"] / 1e9 / HBM_PEAK_GBS, 4),
            "kernels_us_per_pair": {k: round(n * ms * 1e3, 2) for k, (n, ms) in r3["ktimes"].items()},
            "roofline": roof3,
            "tuning": r3["tuned"],
            "toeplitz_normal": r3["toeplitz"],
        }
    if "batched" in parts:
        extra["batched_vs_looped"] = bench_batched(dev, max(3, args.steps // 40), 2, orc_mod)
    print("[bench] device-to-device copy bandwidth", flush=True)
    extra["stream_copy"] = stream_copy(dev, reps=20 if args.steps >= 100 else 3)
    cpu = None
    if not args.no_cpu and r2 is not None:
        cpu = cpu_baseline(orc_mod, args.cpu_seconds)
        extra["nufft_vs_nudft"] = nudft_error(orc_mod)
    if args.calibration_copy_mb > 0:
        n = args.calibration_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        extra["calibration_copy_bytes"] = n * 4

    result = {
        "metric": METRIC,
        "value": None if r2 is None else round(1.0 / r2["sec"], 2),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None if r2 is None else round(r2["sec"] * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2d_256_golden_radial: image 256x256 complex64 ellipse phantom, grid 512x512 "
                               "(sigma=2), Kaiser-Bessel J=6, M=131072 golden-angle radial (256 spokes x 512)",
                   "global_batch": 1, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
