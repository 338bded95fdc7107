"""Command-line front end: points file in, tessellation file out (the paper,
Features section, names a command-line interface beside the library and the
Python wrapper).

    python -m paper_2412_04514_amd.cli POINTS -o OUT [options]

POINTS is a ``.npy`` array [n,3] (float32 or float64) or a text file with
three numbers per line (whitespace or commas; ``#`` starts a comment).  OUT
is a ``.npz`` file (``row_ptr``, ``col``, ``volume``, and with the options
``area``, ``centroid``, ``vxyz``, ``vrow_ptr``, ``vplanes``) or a text file
with one line per cell holding its neighbours' indices (the jagged array).
The run's statistics are printed as one JSON line.  The tessellation runs on
the GPU (``--device``); there is no CPU path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np


def load_points(path: str) -> np.ndarray:
    """Points [n,3] from a .npy file or a text file of three numbers per line."""
    if path.endswith(".npy"):
        P = np.load(path, allow_pickle=False)
    else:
        rows = []
        with open(path) as fh:
            for ln, line in enumerate(fh, 1):
                line = line.split("#", 1)[0].replace(",", " ").split()
                if not line:
                    continue
                if len(line) != 3:
                    raise ValueError(f"{path}:{ln}: expected 3 numbers, got {len(line)}")
                rows.append([float(x) for x in line])
        P = np.array(rows, dtype=np.float64).reshape(-1, 3)
    P = np.asarray(P)
    if P.ndim != 2 or P.shape[1] != 3:
        raise ValueError(f"{path}: expected an array of shape [n, 3], got {P.shape}")
    if P.dtype not in (np.float32, np.float64):
        P = P.astype(np.float64)
    return np.ascontiguousarray(P)


def write_result(path: str, res) -> None:
    """Writes a tessellation result (numpy arrays by name) to .npz or text."""
    arrs = {k: v for k, v in res.items() if v is not None}
    if path.endswith(".npz"):
        np.savez(path, **arrs)
        return
    rp, col = arrs["row_ptr"], arrs["col"]
    with open(path, "w") as fh:
        for i in range(len(rp) - 1):
            fh.write(" ".join(str(int(c)) for c in col[rp[i]:rp[i + 1]]) + "\n")


def build_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser(prog="python -m paper_2412_04514_amd.cli",
                                 description="3D Voronoi tessellation of a point file on the GPU.")
    ap.add_argument("points", help=".npy [n,3] or a text file of x y z lines")
    ap.add_argument("-o", "--out", required=True, help=".npz (all arrays) or text (one neighbour row per line)")
    ap.add_argument("--box", type=float, nargs=6, metavar=("X0", "Y0", "Z0", "X1", "Y1", "Z1"),
                    default=[0.0, 0.0, 0.0, 1.0, 1.0, 1.0], help="closed clip box (default: unit cube)")
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64",
                    help="clip arithmetic; f32 rechecks marginal tests in f64 (the points are rounded to float32)")
    ap.add_argument("--k0", type=int, default=32, help="first neighbour-list size")
    ap.add_argument("--retries", type=int, default=1, help="doublings of k on the GPU before the stream phase")
    ap.add_argument("--no-stream", action="store_true", help="leave cells no list certifies to the host fallback")
    ap.add_argument("--no-fallback", action="store_true", help="fail instead of using the host fallback")
    ap.add_argument("--faces", action="store_true", help="also face areas and cell centroids")
    ap.add_argument("--vertices", action="store_true", help="also cell vertices")
    ap.add_argument("--index-space", choices=["original", "sorted"], default="original")
    ap.add_argument("--device", type=int, default=0, help="GPU ordinal")
    return ap


def main(argv=None) -> int:
    args = build_parser().parse_args(argv)
    P = load_points(args.points)
    if args.precision == "f32":
        P = P.astype(np.float32)
    import torch

    from . import tessellate
    dev = torch.device("cuda", args.device)
    pts = torch.from_numpy(P).to(dev)
    box = (tuple(args.box[:3]), tuple(args.box[3:]))
    r = tessellate(pts, box=box, k0=args.k0, max_gpu_retries=args.retries, precision=args.precision,
                   vertices=args.vertices, faces=args.faces, index_space=args.index_space,
                   host_fallback=not args.no_fallback, gpu_stream=not args.no_stream)
    torch.cuda.synchronize(dev)
    cpu = lambda t: None if t is None else t.cpu().numpy()  # noqa: E731
    out = dict(row_ptr=cpu(r.row_ptr), col=cpu(r.col), volume=cpu(r.volume), area=cpu(r.area),
               centroid=cpu(r.centroid), vrow_ptr=cpu(r.vrow_ptr), vxyz=cpu(r.vxyz), vplanes=cpu(r.vplanes))
    d = os.path.dirname(os.path.abspath(args.out))
    os.makedirs(d, exist_ok=True)
    write_result(args.out, out)
    stats = {k: v for k, v in r.stats.items()}
    print(json.dumps({"points": int(P.shape[0]), "nnz": int(out["col"].shape[0]), "out": args.out,
                      "stats": stats}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
