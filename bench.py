"""Throughput of the cell-by-cell Voronoi path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cluster-16m-f32]

A step is one whole tessellation of the workload (grid sort, k-NN, clipping
with the GPU retry ladder and stream phase, host fallback if any, CSR
assembly) with the points already resident in HBM.  Prints one JSON line:
cells/s for the headline configuration (learned-k, FP32 clipping with FP64
rechecks, when a trained k-model is available; otherwise fixed-k FP32), the
speedup over fixed-k FP64 on the same input, a roofline entry for the
dominant kernel, the step with face areas and centroids, and the CPU oracle
timed on a bounded sample of the same workload on this machine's host cores.
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

# Algorithmic work per cell of the method on the workload (nearest-first
# clipping until the security radius certifies), measured by the oracle on a
# 20000-cell sample with `python -m oracle.work_figures <workload> 20000`:
# 7 flops per vertex-plane evaluation, 40 per created vertex, 5 per vertex
# norm of an R^2 update (5288.5 evaluations, 71.3 vertices created and 266.5
# R^2 vertex norms per cell on cluster-16m-f32).
ALGO_FLOPS_PER_CELL = {"cluster-16m-f32": 41204.79}
FLOP_WEIGHTS = "7 per vertex-plane evaluation + 40 per created vertex + 5 per R^2 vertex norm"

PEAK = {"hbm_gbs": 8000.0, "fp32_tflops": 157.3, "fp64_tflops": 78.6}


def sort_bytes_per_point(dtype, n: int, ncells: int) -> float:
    """Grid sort: read the points, write the 4-field records and perm, write
    cell_start."""
    e = 4 if dtype == np.float32 else 8
    return 3 * e + 4 * e + 4 + 4.0 * (ncells + 1) / max(n, 1)


def knn_bytes_per_query(k: int) -> int:
    return 16 + 4 * k  # read the query's record, write k indices


CLIP_SOURCES = ("clip.hip", "device_common.h", "internal.h")


def clip_sources_sha256() -> str:
    """SHA-256 over the clip kernel's sources, in the order of CLIP_SOURCES."""
    import hashlib
    h = hashlib.sha256()
    for name in CLIP_SOURCES:
        with open(os.path.join(ROOT, "paper_2412_04514_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def clip_traffic_profile(workload: str) -> str:
    """Path of the committed counter summary of a workload's clip traffic
    (cluster-16m-f32 -> profiles/clip_traffic_cluster16m_f32.md)."""
    return os.path.join(ROOT, "profiles", f"clip_traffic_{workload.replace('-', '', 1).replace('-', '_')}.md")


def clip_traffic_fields(workload: str) -> dict:
    """The '- key: value' lines of that summary (empty if it is missing)."""
    try:
        text = open(clip_traffic_profile(workload)).read()
    except OSError:
        return {}
    vals = {}
    for ln in text.splitlines():
        if ":" in ln and ln.strip().startswith("- "):
            k, v = ln.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    return vals


def clip_traffic(workload: str):
    """HBM bytes per step of all k_clip launches from the committed counter
    summary, only while it was taken on the clip kernel as it stands (the
    summary records the SHA-256 of the sources the kernel is compiled from);
    None otherwise."""
    vals = clip_traffic_fields(workload)
    if vals.get("clip sources sha256") != clip_sources_sha256():
        return None
    try:
        return float(vals["bytes per step"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cluster-16m-f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-baseline-f64", action="store_true")
    ap.add_argument("--mode", choices=["auto", "fixed", "learned"], default="auto")
    ap.add_argument("--k0", type=int, default=32)
    ap.add_argument("--retries", type=int, default=0,
                    help="doublings of k after the learned pass (64 -> 128 -> 256) before the stream phase; "
                         "0: the learned pass streams its uncertified cells directly")
    ap.add_argument("--no-faces", action="store_true", help="skip the run with face areas and centroids")
    ap.add_argument("--profile-step", action="store_true", help="one headline step only (for rocprofv3)")
    ap.add_argument("--kmodel-blob", default="",
                    help="k-model blob file: loaded if it exists (no training), else written after training")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB on the device (calibrates rocprofv3 byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the tessellation has no multi-GPU path here.",
              file=sys.stderr)
        return 2

    import torch
    import paper_2412_04514_amd as vt
    from paper_2412_04514_amd import gen

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    P = gen.make(args.workload, seed=0)
    n = P.shape[0]
    log(f"[bench] {args.workload}: {n} points generated in {time.time() - t0:.1f}s")
    pts = torch.from_numpy(P).to(dev)
    torch.cuda.synchronize()
    if args.copy_probe_mib > 0:  # one plain device-to-device copy of known size
        src = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst

    kmodel = None
    if args.mode in ("auto", "learned"):
        try:
            from paper_2412_04514_amd import kmodel as km
            if args.kmodel_blob and os.path.exists(args.kmodel_blob):
                with open(args.kmodel_blob, "rb") as fh:
                    kmodel = km.KModel.load(fh.read())
                log(f"[bench] k-model loaded from {args.kmodel_blob} (tau {kmodel.tau})")
            else:
                kmodel = km.load_default(args.workload, max_gpu_retries=args.retries)
                if args.kmodel_blob:
                    with open(args.kmodel_blob, "wb") as fh:
                        fh.write(kmodel.save())
        except Exception as e:  # no trained model shipped for this workload
            if args.mode == "learned":
                raise
            log(f"[bench] no learned-k model ({e}); timing fixed-k FP32")
    headline = dict(precision="f32", k0=args.k0, max_gpu_retries=1)
    label = "fixed-k FP32"
    if kmodel is not None:
        headline = dict(precision="f32", kmodel=kmodel, tau=kmodel.tau, max_gpu_retries=args.retries)
        label = "learned-k FP32"

    # The Infinity Cache (256 MB) would otherwise keep part of the sorted
    # records from one step to the next: every timed step is preceded by a
    # 1 GiB streaming pass, outside the step's own interval.
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)

    def run(cfg, steps, warmup, tag):
        for i in range(warmup):
            vt.tessellate(pts, **cfg)
            log(f"[bench] {tag} warmup {i + 1}/{warmup}")
        torch.cuda.synchronize()
        stats, per = [], []
        for i in range(steps):
            flush.fill_(float(i))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = vt.tessellate(pts, **cfg)
            torch.cuda.synchronize()
            per.append((time.perf_counter() - t1) * 1e3)
            stats.append(r.stats)
            del r
        ms = float(np.sum(per)) / steps
        log(f"[bench] {tag}: {ms:.2f} ms/step (median {np.median(per):.2f}, min {min(per):.2f})")
        stats[-1]["_ms_median"] = float(np.median(per))
        stats[-1]["_ms_min"] = float(min(per))
        return ms, stats

    ms, stats = run(headline, args.steps, args.warmup, label)
    if args.profile_step:
        log(f"[bench] profile step done: {stats[-1]}")
        return 0
    mean = lambda key: float(np.mean([s[key] for s in stats]))  # noqa: E731
    st0 = stats[-1]
    ms_sort, ms_knn, ms_clip = mean("ms_sort"), mean("ms_knn"), mean("ms_clip")
    ms_feat, ms_mlp = mean("ms_features"), mean("ms_mlp")

    base = None
    if not args.no_baseline_f64:
        ms64, stats64 = run(dict(precision="f64", k0=32, max_gpu_retries=1), max(1, args.steps // 2), 1,
                            "fixed-k FP64")
        base = dict(ms_per_step=ms64, cells_per_s=n / (ms64 / 1e3), knn_clip_ms=float(
            np.mean([s["ms_knn"] + s["ms_clip"] for s in stats64])), last_stats=stats64[-1])
        # the same at fixed k = 64 (no retry), so that the gain is not measured against k = 32 alone
        ms64b, stats64b = run(dict(precision="f64", k0=64, max_gpu_retries=0), max(1, args.steps // 2), 1,
                              "fixed-k64 FP64")
        base["k64_ms_per_step"] = ms64b
    # ablation of the network: the FP32 form at fixed k = 64, streaming after the list
    abl = None
    if kmodel is not None and not args.no_baseline_f64:
        msa, statsa = run(dict(precision="f32", k0=64, max_gpu_retries=0), 2, 1, "fixed-k64 FP32")
        abl = dict(ms_per_step=msa, cells_per_s=n / (msa / 1e3),
                   knn_ms=float(np.mean([s["ms_knn"] for s in statsa])),
                   clip_ms=float(np.mean([s["ms_clip"] for s in statsa])))

    # the headline configuration with the per-face outputs (face areas and
    # centroids): their cost on top of the step
    faces = None
    if not args.no_faces:
        msf, statsf = run(dict(headline, faces=True), 2, 1, label + " + faces")
        faces = dict(ms_per_step=msf, cells_per_s=n / (msf / 1e3),
                     clip_ms=float(np.mean([s["ms_clip"] for s in statsf])),
                     assemble_ms=float(np.mean([s["ms_assemble"] for s in statsf])))

    # Rooflines of the three stages, from their HIP-event times inside the
    # library (on the stream the kernels run on); the dominant one (largest
    # share of the step) is the line's `roofline`.
    ncells = vt.grid_plan(n).ncells
    sbpp = sort_bytes_per_point(P.dtype.type, n, ncells)
    sort_gbs = sbpp * n / (ms_sort / 1e3) / 1e9
    if kmodel is not None:
        # the learned form runs one k-NN at the largest bucket over every cell
        # (its rows' prefixes serve the features and the smaller buckets),
        # then retries of their own above it
        kl = max(vt.BUCKETS)
        knn_q = n + sum(p["cells"] for p in st0["passes"] if p["k"] > kl)
        knn_bytes = n * knn_bytes_per_query(kl) + sum(p["cells"] * knn_bytes_per_query(p["k"])
                                                      for p in st0["passes"] if p["k"] > kl)
    else:
        knn_q = sum(p["cells"] for p in st0["passes"] if p["k"] > 0)
        knn_bytes = sum(p["cells"] * knn_bytes_per_query(p["k"]) for p in st0["passes"] if p["k"] > 0)
    # (the fused form, k0 = 0, has no k-NN pass)
    knn_gbs = knn_bytes / ((ms_knn + ms_feat) / 1e3) / 1e9 if ms_knn + ms_feat > 0 else None
    flops = ALGO_FLOPS_PER_CELL.get(args.workload)
    clip_tf = flops * n / (ms_clip / 1e3) / 1e12 if flops else None
    stages = {
        "sort": dict(bound="hbm", achieved=sort_gbs, peak=PEAK["hbm_gbs"], unit="GB/s",
                     frac=sort_gbs / PEAK["hbm_gbs"], ms=ms_sort,
                     per_unit=f"{sbpp:.2f} bytes per point (points read, records and perm written, cell starts)"),
        "knn": dict(bound="hbm", achieved=knn_gbs, peak=PEAK["hbm_gbs"], unit="GB/s",
                    frac=knn_gbs / PEAK["hbm_gbs"] if knn_gbs is not None else None, ms=ms_knn + ms_feat,
                    queries=knn_q,
                    per_unit="16 + 4k bytes per query (record read, k indices written)"),
        "clip": dict(bound="alu", achieved=clip_tf, peak=PEAK["fp32_tflops"], unit="TFLOP/s",
                     frac=(clip_tf / PEAK["fp32_tflops"]) if clip_tf else None, ms=ms_clip,
                     per_unit=f"{flops} algorithmic flops per cell ({FLOP_WEIGHTS}; oracle work count)"),
    }
    work = {"sort": ms_sort, "knn": ms_knn + ms_feat, "clip": ms_clip}
    dom = max(work, key=work.get)
    roof = dict(stages[dom])
    roof.pop("ms", None)
    roof["kernel"] = {"clip": "k_clip (all launches of a step)", "knn": "k_knn (all launches of a step)",
                      "sort": "grid sort kernels"}[dom]
    roof["traffic"] = clip_traffic(args.workload) if (dom == "clip" and kmodel is not None) else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(P)

    knn_clip_ms = ms_knn + ms_clip + ms_feat + ms_mlp
    gpu_ms = knn_clip_ms + ms_sort + mean("ms_assemble")
    out = {
        "metric": "Voronoi cells/sec at 16M pts (kNN+clip); learned-k FP32 vs fixed-k FP64 speedup",
        "value": n / (ms / 1e3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "points": n, "method": label, "box": "unit cube",
                   "parallelism": "single GPU"},
        "cells_per_s_knn_clip": n / (knn_clip_ms / 1e3),
        "cells_per_s_gpu": n / (gpu_ms / 1e3),
        "ms_step_median": st0.get("_ms_median"), "ms_step_min": st0.get("_ms_min"),
        "speedup_vs_fixed_k_f64": (base["ms_per_step"] / ms) if base else None,
        "fixed_k_f64": {"ms_per_step": base["ms_per_step"], "cells_per_s": base["cells_per_s"],
                        "knn_clip_ms": base["knn_clip_ms"]} if base else None,
        "speedup_vs_fixed_k64_f64": (base["k64_ms_per_step"] / ms) if base else None,
        "fixed_k64_f32": abl,
        "with_faces": faces,
        "stage_ms": {"sort": ms_sort, "knn": ms_knn, "features": ms_feat, "mlp": ms_mlp, "clip": ms_clip,
                     "assemble": mean("ms_assemble"), "fallback": mean("ms_fallback")},
        "stages": stages,
        "mall_flush": "1 GiB streamed between timed steps (outside each step's interval)",
        "passes": st0["passes"],
        "streamed_cells": st0["streamed_cells"], "fallback_cells": st0["fallback_cells"],
        "capacity_cells": st0["capacity_cells"], "rechecks": st0["rechecks"],
        "refined_cells": st0["refined_cells"], "unresolved_cells": st0["unresolved_cells"],
        "bucket_cells": st0["bucket_cells"],
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if kmodel is not None:
        out["kmodel"] = {"tau": kmodel.tau, "train_loss_per_epoch": [round(x, 5) for x in kmodel.history],
                         "label_hist": getattr(kmodel, "label_hist", None),
                         "train_s": round(getattr(kmodel, "train_seconds", 0.0), 2),
                         "label_s": round(getattr(kmodel, "prep_seconds", 0.0), 2)}
    print(json.dumps(out), flush=True)
    return 0


def cpu_baseline(P: np.ndarray) -> dict:
    """The FP64 oracle on the points of the workload inside [0, 0.5)^3 (a
    bounded sample, tessellated within that sub-box) on the host cores."""
    import oracle
    lo, hi = (0.0, 0.0, 0.0), (0.5, 0.5, 0.5)
    sel = np.all(P < 0.5, axis=1)
    S = P[sel].astype(np.float64)
    threads = os.cpu_count() or 1
    t = time.perf_counter()
    oracle.tessellate(S, lo, hi, threads=threads)
    dt = time.perf_counter() - t
    # one thread, on 2^15 seeded cells of the same sample
    cells = np.sort(np.random.default_rng(0).choice(len(S), min(len(S), 1 << 15), replace=False))
    t = time.perf_counter()
    oracle.tessellate(S, lo, hi, threads=1, cells=cells)
    dt1 = time.perf_counter() - t
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": len(S) / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(S)} points of the workload inside [0,0.5)^3, tessellated in that sub-box "
                      f"(FP64 C++ OpenMP oracle, {dt:.1f} s)",
            "one_thread": {"value": len(cells) / dt1, "unit": "cells/s",
                           "sample": f"{len(cells)} seeded cells of the same sub-box ({dt1:.1f} s)"},
            "cpu_model": model}


if __name__ == "__main__":
    sys.exit(main())
