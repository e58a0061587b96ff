"""Write ``oracle_results.json``: oracle answers for instances too large to solve inside a test.

Calls only the CPU oracle (``oracle/``) and the seeded generators; nothing here
touches the GPU solver.  Each entry records the generator call that rebuilds
its Q, the oracle method (O1 direct evaluation or O2 local-field Gray walk),
the answer (E*, lowest index, optionally the k smallest pairs), and the
wall time and thread count it took.

    python tests/golden/make_oracle_goldens.py [--only NAME ...]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2607_04857_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "oracle_results.json")

# name -> (generator, kwargs, method, k)
ENTRIES = {
    "n24_int_u100_s1": ("uniform_int", dict(n=24, lo=-100, hi=100, seed=1), "O1", 16),
    "n36_int_u1000_s2": ("uniform_int", dict(n=36, lo=-1000, hi=1000, seed=2), "O2", 1),
    "n36_planted_u1000_s3": ("planted", dict(n=36, lo=-1000, hi=1000, seed=3), "O2", 1),
    "n30_int_u1000_s10": ("uniform_int", dict(n=30, lo=-1000, hi=1000, seed=10), "O1", 4),
    "n31_int_u10000_s11": ("uniform_int", dict(n=31, lo=-10000, hi=10000, seed=11), "O2", 1),
    "n33_int_u100_s12": ("uniform_int", dict(n=33, lo=-100, hi=100, seed=12), "O2", 1),
    "n28_fp32_s6": ("normal_fp32", dict(n=28, seed=6), "O1", 4),
    "n32_fp32_s13": ("normal_fp32", dict(n=32, seed=13), "O2", 1),
}


def make_Q(gen, kw):
    out = getattr(inputs, gen)(**kw)
    return out[0] if gen == "planted" else out


def run(name):
    gen, kw, method, k = ENTRIES[name]
    Q = make_Q(gen, kw)
    t0 = time.time()
    if method == "O1":
        pairs = oracle.solve(Q, k=k)
    else:
        pairs = [oracle.gray_solve(Q)]
    dt = time.time() - t0
    return {
        "generator": gen, "kwargs": kw, "dtype": "fp32" if Q.dtype.kind == "f" else "int32",
        "method": method, "best": list(pairs[0]), "topk": [list(p) for p in pairs],
        "seconds": round(dt, 2), "threads": oracle.default_threads(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*")
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in (args.only or list(ENTRIES)):
        res = run(name)
        data[name] = res
        print(name, res["best"], f"{res['seconds']}s", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
