"""Autotuner of the f32 product tile variants (rsvd_set_tile_variants).

For every (mode, column class) the products come in up to three variants
(4, 8 or 16 waves over the same output tile).  The tuner times real
workloads with each variant of one (mode, class) while every other entry
stays at its best so far, and keeps the fastest (coordinate descent, one
pass):

* classes 32..80: the 4096-matrix ragged batch (graph replays), whose sketch
  widths l = k + 10 in [18, 74] fall in those classes;
* class 128: single solves of a 100000 x 5000 f32 matrix with l = 120.

Class 96 occurs in neither workload and keeps its default.  The result is a
JSON cache keyed by GPU architecture, applied by api.handle() to every new
handle:  {"gfx950": {"f32": [12 ints: NN classes 32..128, then TN]}}.

Usage: python -m paper_1608_02148_amd.autotune [--out PATH] [--reps 3]
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np
import torch

from . import api
from . import lib as L

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tile_variants.json")
CLASSES = (32, 48, 64, 80, 96, 128)
N_VARIANTS = {32: 3, 48: 2, 64: 3, 80: 2, 96: 3, 128: 3}


def get_variants(device=None):
    v = (ctypes.c_int32 * 12)()
    L.check(L.load().rsvd_get_tile_variants(api.handle(device), v), "rsvd_get_tile_variants")
    return list(v)


def set_variants(variants, device=None):
    v = (ctypes.c_int32 * 12)(*[int(x) for x in variants])
    L.check(L.load().rsvd_set_tile_variants(api.handle(device), v), "rsvd_set_tile_variants")


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune(reps=3, log=print):
    from synth import matrices as syn
    dev = torch.device("cuda", torch.cuda.current_device())
    best = get_variants(dev)
    c = syn.CONFIGS["ragged_4096"]
    data = syn.ragged_torch(device=dev, batch=c["batch"], seed=c["gen_seed"])
    ks = [int(x) for x in data["k"]]

    def batch_time():
        bt = api.Batch(data["A"], ks, p=c["p"], q=c["q"], seed=c["omega_seed"], graph=True)
        t = _time(bt.run, reps)
        bt.close()
        return t

    for mode in (0, 1):
        for ci, cls in enumerate(CLASSES[:4]):
            slot = 6 * mode + ci
            times = {}
            for v in range(N_VARIANTS[cls]):
                trial = list(best)
                trial[slot] = v
                set_variants(trial, dev)
                times[v] = batch_time()
            best[slot] = min(times, key=times.get)
            log(f"[autotune] batch {'NN' if mode == 0 else 'TN'} class {cls}: "
                f"{ {v: round(t * 1e3, 3) for v, t in times.items()} } ms -> variant {best[slot]}")
    del data
    torch.cuda.empty_cache()
    A = torch.randn(100000, 5000, device=dev, dtype=torch.float32)
    work = None
    for mode in (0, 1):
        slot = 6 * mode + 5
        times = {}
        for v in range(N_VARIANTS[128]):
            trial = list(best)
            trial[slot] = v
            set_variants(trial, dev)
            prm = api.make_params(20, 2, 1)
            if work is None:
                work = api.workspace(api.workspace_size(A, 100, prm), dev)
            out = (torch.empty(100000, 100, device=dev), torch.empty(100, dtype=torch.float64, device=dev),
                   torch.empty(5000, 100, device=dev))
            times[v] = _time(lambda: api.rsvd(A, 100, p=20, q=2, seed=1, work=work, out=out), reps)
        best[slot] = min(times, key=times.get)
        log(f"[autotune] single {'NN' if mode == 0 else 'TN'} class 128: "
            f"{ {v: round(t * 1e3, 3) for v, t in times.items()} } ms -> variant {best[slot]}")
    set_variants(best, dev)
    return best


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    best = tune(args.reps, log=lambda m: print(m, file=sys.stderr, flush=True))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = {}
    if os.path.exists(args.out):
        cache = json.load(open(args.out))
    cache[arch] = {"f32": best}
    json.dump(cache, open(args.out, "w"), indent=1)
    print(json.dumps(cache), flush=True)


if __name__ == "__main__":
    main()
