"""Autotuner for the NUFFT plan's launch parameters.

Chooses, per workload, the grid tile shape used for binning, gathering and
gridding, the number of samples per gridding work item, whether the gather
stages tiles in LDS or reads the grid directly, whether the gridding reads the
samples pre-permuted into sorted order, whether the sample kernels read a
precomputed window table or evaluate the kernel per sample, how many
workgroups the FFT passes aim for (lines or columns per workgroup), the FFT's
radix schedule, and whether the first inverse FFT pass sums the partial tiles
of split gridding tiles.  A workload with coil maps is tuned in coil mode.
These
change only speed: every candidate's forward and adjoint outputs must agree
with the default plan's to 1e-5 (relative L2) before it may win, and the
default plan is the one the parity tests hold to the FP64 oracle.

Results are cached in JSON, keyed by GPU architecture, d, N, K, J and M
rounded to a power of two, at $NUFFT_TUNE_CACHE or
~/.cache/nufft_mi355x/tune.json.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from .plan import Plan as _Plan

TOL = 1e-5

TILE_CANDIDATES = {
    1: [(32,), (64,), (16,)],
    2: [(32, 16), (64, 16), (16, 16), (32, 32), (16, 32), (64, 8)],
    3: [(8, 8, 16), (16, 8, 16), (8, 16, 16), (8, 8, 8), (4, 8, 16), (4, 4, 16), (16, 8, 8)],
}
CHUNK_CANDIDATES = [256, 512, 1024, 1536, 2048]
FFT_GROUP_CANDIDATES = [256, 512, 1024, 2048, 4096]
RADIX_CANDIDATES = [1, 2, 3]  # fft_radix schedules besides the default 0


def cache_path(path: str | None = None) -> str:
    if path:
        return path
    env = os.environ.get("NUFFT_TUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "nufft_mi355x", "tune.json")


def workload_key(N, K, J, M, device=None, C: int = 0) -> str:
    arch = torch.cuda.get_device_properties(device or 0).gcnArchName.split(":")[0]
    mb = 1 << max(0, int(round(math.log2(max(M, 1)))))
    key = f"{arch}|d{len(N)}|N{'x'.join(map(str, N))}|K{'x'.join(map(str, K))}|J{J}|M~{mb}"
    return key + (f"|C{C}" if C else "")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _rel(a, b):
    return float(torch.linalg.vector_norm((a - b).flatten()) / torch.linalg.vector_norm(b.flatten()))


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(om: torch.Tensor, N, K=None, J: int = 6, reps: int = 10, path: str | None = None,
         save: bool = True, verbose: bool = False, coils: torch.Tensor | None = None) -> dict:
    """Tune the plan options for trajectory `om` (float32 [M, d] on the GPU),
    in coil mode when `coils` (complex64 [C, *N]) is given.
    Returns {"options": ..., "ms_pair": ..., "default_ms_pair": ..., "tried": n}."""
    N = tuple(int(n) for n in N)
    K = tuple(2 * n for n in N) if K is None else tuple(int(k) for k in K)
    d, M = len(N), int(om.shape[0])
    C = 0 if coils is None else int(coils.shape[0])
    dev = om.device
    g = torch.Generator(device="cpu").manual_seed(1234)
    x = torch.complex(torch.randn(N, generator=g), torch.randn(N, generator=g)).to(dev)
    ys = (max(C, 1), M) if C else (M,)
    yin = torch.complex(torch.randn(ys, generator=g), torch.randn(ys, generator=g)).to(dev)

    def Plan(om_, N_, K_, J_, options=None):  # noqa: N802 - every candidate in the workload's coil mode
        return _Plan(om_, N_, K_, J_, coils=coils, options=options)

    ref = Plan(om, N, K, J)
    y_ref, x_ref = ref.forward(x), ref.adjoint(yin)

    def pair_time(p):
        y = torch.empty(ys, dtype=torch.complex64, device=dev)
        xa = torch.empty(N, dtype=torch.complex64, device=dev)
        return _time(lambda: (p.forward(x, out=y), p.adjoint(yin, out=xa)), reps)

    def sample_stage_time(p):
        if C:  # coil mode: the stage calls take single grids, so time the pair
            return pair_time(p)
        G = torch.empty(K, dtype=torch.complex64, device=dev)
        return _time(lambda: (p.stage_v(G), p.stage_vh(yin)), reps)

    def valid(p):
        return _rel(p.forward(x), y_ref) <= TOL and _rel(p.adjoint(yin), x_ref) <= TOL

    default_ms = pair_time(ref)
    ref.close()
    tried = 0
    # 1) tile shape and gridding chunk, timed on the two sample stages
    best, best_t = {}, float("inf")
    # 3D tiles that the gridding by 4 x 4 blocks takes are also tried with one
    # wavefront per work item
    blk = [(8, 8, 16), (16, 8, 16), (8, 16, 16)]
    for tile, waves in [(t, 4) for t in TILE_CANDIDATES[d]] + [(t, 1) for t in TILE_CANDIDATES[d] if t in blk]:
        for chunk in CHUNK_CANDIDATES:
            opts = dict(tile=tile, grid_chunk=chunk)
            if waves == 1:
                opts["grid_waves"] = 1
            try:
                p = Plan(om, N, K, J, options=opts)
            except RuntimeError:
                continue
            tried += 1
            if not valid(p):
                p.close()
                continue
            t = sample_stage_time(p)
            p.close()
            if verbose:
                print(f"[tune] {opts}: sample stages {t:.4f} ms", flush=True)
            if t < best_t:
                best, best_t = opts, t
    # 2) the gather reading the grid directly instead of staging tiles in LDS,
    #    the gridding's samples pre-permuted into sorted order or read through
    #    the permutation, and runs of sparse tiles per gather item
    for extra in (dict(interp_direct=1), dict(presort=1), dict(presort=2), dict(interp_merge=1),
                  dict(interp_merge=2), dict(interp_merge=4), dict(weight_table=1)):
        opts = dict(best, **extra)
        p = Plan(om, N, K, J, options=opts)
        tried += 1
        if valid(p):
            t = sample_stage_time(p)
            if verbose:
                print(f"[tune] {opts}: sample stages {t:.4f} ms", flush=True)
            if t < best_t:
                best, best_t = opts, t
        p.close()
    # 3) FFT workgroup target with that tiling, timed on the whole pair
    best_pair, best_pt = dict(best), float("inf")
    for groups in FFT_GROUP_CANDIDATES:
        opts = dict(best, fft_groups=groups)
        p = Plan(om, N, K, J, options=opts)
        tried += 1
        if not valid(p):
            p.close()
            continue
        t = pair_time(p)
        p.close()
        if verbose:
            print(f"[tune] {opts}: pair {t:.4f} ms", flush=True)
        if t < best_pt:
            best_pair, best_pt = opts, t
    # 4) the FFT radix schedule, timed on the whole pair
    for radix in RADIX_CANDIDATES:
        opts = dict(best_pair, fft_radix=radix)
        try:
            p = Plan(om, N, K, J, options=opts)
        except RuntimeError:
            continue
        tried += 1
        if valid(p):
            t = pair_time(p)
            if verbose:
                print(f"[tune] {opts}: pair {t:.4f} ms", flush=True)
            if t < best_pt:
                best_pair, best_pt = opts, t
        p.close()
    # 5) split tiles' partial sums in the first inverse FFT pass or apart
    if d >= 2:
        for fuse in (1, 2):
            opts = dict(best_pair, fuse_reduce=fuse)
            p = Plan(om, N, K, J, options=opts)
            tried += 1
            if valid(p):
                t = pair_time(p)
                if verbose:
                    print(f"[tune] {opts}: pair {t:.4f} ms", flush=True)
                if t < best_pt:
                    best_pair, best_pt = opts, t
            p.close()
    result = {"options": {k: list(v) if isinstance(v, tuple) else v for k, v in best_pair.items()},
              "ms_pair": best_pt, "default_ms_pair": default_ms, "tried": tried}
    if save:
        cp = cache_path(path)
        os.makedirs(os.path.dirname(cp), exist_ok=True)
        db = _load(cp)
        db[workload_key(N, K, J, M, dev, C)] = result
        tmp = cp + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, cp)
    return result


def cached_options(N, K, J, M, path: str | None = None, device=None, C: int = 0) -> dict | None:
    """The cached options of a workload (C: coils; a coil-mode entry falls
    back to the single-coil one)."""
    N = tuple(int(n) for n in N)
    K = tuple(2 * n for n in N) if K is None else tuple(int(k) for k in K)
    db = _load(cache_path(path))
    entry = db.get(workload_key(N, K, J, M, device, C)) if C else None
    if entry is None:
        entry = db.get(workload_key(N, K, J, M, device))
    return None if entry is None else entry["options"]


def tuned_plan(om: torch.Tensor, N, K=None, J: int = 6, coils=None, path: str | None = None,
               tune_if_missing: bool = False) -> Plan:
    """A Plan with the cached tuned options for this workload (tuning first if
    asked and nothing is cached; defaults otherwise)."""
    C = 0 if coils is None else int(coils.shape[0])
    opts = cached_options(N, K, J, int(om.shape[0]), path, om.device, C)
    if opts is None and tune_if_missing:
        opts = tune(om, N, K, J, path=path, coils=coils)["options"]
    return _Plan(om, N, K, J, coils=coils, options=opts)


SHIPPED_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def _main():
    """Tune the benchmark workloads and write the cache:
    python -m paper_1710_03197_amd.autotune --out FILE [--configs 1 2 3 4]
    (4: one problem per distinct image size and sample-count bucket of the
    uneven spiral batch, in coil mode)"""
    import argparse
    from . import data
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--configs", nargs="*", type=int, default=[1, 2, 3, 4])
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    makers = {1: data.config1, 2: data.config2, 3: data.config3}
    dev = torch.device("cuda:0")
    for k in args.configs:
        if k == 4:
            seen = set()
            for pr in data.config4():
                om = torch.from_numpy(pr["om"]).to(dev)
                key = workload_key(pr["N"], pr["K"], 6, om.shape[0], dev, pr["coils"].shape[0])
                if key in seen:
                    continue
                seen.add(key)
                coils = torch.from_numpy(pr["coils"]).to(dev)
                res = tune(om, pr["N"], pr["K"], 6, reps=max(3, args.reps // 4), path=args.out, verbose=False,
                           coils=coils)
                print(f"config 4 {key}: {res}", flush=True)
            continue
        c = makers[k]()
        om = torch.from_numpy(c["om"]).to(dev)
        res = tune(om, c["N"], c["K"], c["J"], reps=args.reps, path=args.out, verbose=True)
        print(f"config {k}: {res}", flush=True)


if __name__ == "__main__":
    _main()
