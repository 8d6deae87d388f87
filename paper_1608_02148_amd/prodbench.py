"""Time the library's large products on their own (for profiling runs).

``python -m paper_1608_02148_amd.prodbench --shape c3 --arith bf16 --mode nn``
runs Y = A X (nn) or Z = A^T Q (tn) through rsvd_gemm_nn / rsvd_gemm_tn on
seeded Gaussian data at the benchmark shapes and prints the mean time per
product (HIP events).  Shapes: c2 = 100000 x 5000 f32 with 120 columns, c3 =
200000 x 20000 bf16 with 220 columns (--m, --n, --c override them).
"""
import argparse
import json

import torch

from . import api

SHAPES = {"c2": (100000, 5000, 120, torch.float32), "c3": (200000, 20000, 220, torch.bfloat16)}


def run(shape, arith, mode, reps, warmup=1, splits=0, m=None, n=None, c=None):
    m0, n0, c0, dt = SHAPES[shape]
    m, n, c = m or m0, n or n0, c or c0
    dev = torch.device("cuda", 0)
    g = torch.Generator(device=dev)
    g.manual_seed(2148)
    A = torch.randn(m, n, generator=g, device=dev, dtype=torch.float32).to(dt)
    if mode == "nn":
        X = torch.randn(n, c, generator=g, device=dev)
        call = lambda: api.gemm_nn(A, X, arith, splits=splits)   # noqa: E731
    else:
        X = torch.randn(m, c, generator=g, device=dev)
        call = lambda: api.gemm_tn(A, X, arith)                   # noqa: E731
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 2.0 * m * n * c
    return {"shape": shape, "mode": mode, "arith": arith, "m": m, "n": n, "c": c, "ms_per_product": round(ms, 4),
            "tflops": round(flops / ms / 1e9, 2), "a_gbs": round(m * n * A.element_size() / ms / 1e6, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", choices=sorted(SHAPES), default="c3")
    ap.add_argument("--arith", choices=["storage", "bf16", "split"], default="bf16")
    ap.add_argument("--mode", choices=["nn", "tn"], default="nn")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--m", type=int, default=None, help="rows of A (default: the shape's)")
    ap.add_argument("--n", type=int, default=None, help="columns of A")
    ap.add_argument("--c", type=int, default=None, help="columns of X")
    ap.add_argument("--splits", type=int, default=0, help="A X: chunks of the reduction (0: the library's choice)")
    args = ap.parse_args()
    print(json.dumps(run(args.shape, args.arith, args.mode, args.reps, splits=args.splits, m=args.m, n=args.n,
                         c=args.c)), flush=True)


if __name__ == "__main__":
    main()
