"""Command-line autotuner: time every runnable walk plan per n on this GPU.

    python -m paper_2607_04857_amd.tune N_MIN N_MAX [--dtype int32|fp32] [--reps R]
                                        [--cache FILE] [--batch]

Prints one JSON line per n with the winning plan (B, L, tier, vgpr_levels)
and its walk time; with --cache the winners are merged into FILE, which the
library loads when the QUBO_TUNE_CACHE environment variable names it.  Large
n are tuned one at a time so that progress shows as it goes.  --batch tunes
the plans of instances inside batches and the server instead (timed by the
replay of a batch of copies that fills the GPU; n <= 44).
"""
import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("n_min", type=int)
    ap.add_argument("n_max", type=int)
    ap.add_argument("--dtype", default="int32", choices=["int32", "fp32"])
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--cache", default=None)
    ap.add_argument("--batch", action="store_true")
    args = ap.parse_args(argv)
    from . import autotune, device_key
    print(json.dumps({"device": device_key()}), flush=True)
    t0 = time.perf_counter()
    n = args.n_min
    while n <= args.n_max:
        hi = n if n >= 36 else min(args.n_max, 35)     # small n together, large n singly
        if args.batch:
            hi = n                                      # one n per call: progress lines
        for e in autotune(n, hi, args.dtype, args.reps, args.cache, batch=args.batch):
            states = 2.0 ** e["n"]
            if args.batch:
                e["copies"] = min(4096, 2 ** (39 - e["n"])) if e["n"] < 39 else 1
                states *= e["copies"]
            e["states_per_s"] = states / (e["walk_ms"] * 1e-3)
            print(json.dumps(e), flush=True)
        print(json.dumps({"done_through": hi, "elapsed_s": round(time.perf_counter() - t0, 1)}),
              flush=True)
        n = hi + 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
