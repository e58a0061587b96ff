"""Write ``oracle_results.json``: oracle answers for instances too large to solve inside a test.

Calls only the CPU oracle (``oracle/``) and the seeded generators; nothing here
touches the GPU solver.  Each entry records the generator call that rebuilds
its Q, the oracle method (O1 direct evaluation or O2 local-field Gray walk),
the answer (E*, lowest index, optionally the k smallest pairs), and the
wall time and thread count it took.

Entries with a shard count are walked by O2 in that many equal ranges of the
Gray index; each finished shard is recorded at once in
``shards_<name>.json`` beside this script, so an interrupted run resumes
where it stopped, and the entry is written when the last shard is done (its
seconds are the sum over shards).

    python tests/golden/make_oracle_goldens.py [--only NAME ...] [--threads T]
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

# name -> (generator, kwargs, method, k[, shards])
ENTRIES = {
    # the n = 44 single-instance configuration (2^44 states): ~4 h of O2 on 8 threads
    "n44_int_u10000_s4": ("uniform_int", dict(n=44, lo=-10000, hi=10000, seed=4), "O2", 1, 1024),
    "n24_int_u100_s1": ("uniform_int", dict(n=24, lo=-100, hi=100, seed=1), "O1", 16),
    "n36_int_u1000_s2": ("uniform_int", dict(n=36, lo=-1000, hi=1000, seed=2), "O2", 1),
    "n36_planted_u1000_s3": ("planted", dict(n=36, lo=-1000, hi=1000, seed=3), "O2", 1),
    "n30_int_u1000_s10": ("uniform_int", dict(n=30, lo=-1000, hi=1000, seed=10), "O1", 1024),
    "n32_int_u1000_s14": ("uniform_int", dict(n=32, lo=-1000, hi=1000, seed=14), "O1", 1024),
    "n31_int_u10000_s11": ("uniform_int", dict(n=31, lo=-10000, hi=10000, seed=11), "O2", 1),
    "n33_int_u100_s12": ("uniform_int", dict(n=33, lo=-100, hi=100, seed=12), "O2", 1),
    "n28_fp32_s6": ("normal_fp32", dict(n=28, seed=6), "O1", 1024),
    "n32_fp32_s13": ("normal_fp32", dict(n=32, seed=13), "O2", 1),
}


# The serving mix (Poisson arrivals, n ~ U{16..40}, 80% int32 U[-100,100] /
# 20% float32 N(0,1), seed 7): oracle answers of every request with n <= 36.
# int32: O1 for n <= 24, else O2.  float32: the O2 argmin, with its energy
# recomputed directly by the oracle's energy() (O2 accumulates its float64
# energy over up to 2^36 steps; the direct sum does not drift).
SERVE = {"serve_s7_r340_c100": dict(count=100, rate_hz=340.0, n_lo=16, n_hi=40, seed=7,
                                      n_max=36)}


def run_serve(name, threads=0):
    kw = dict(SERVE[name])
    n_max = kw.pop("n_max")
    reqs = inputs.poisson_requests(**kw)
    t0 = time.time()
    out = {}
    for i, (_, Q) in enumerate(reqs):
        n = Q.shape[0]
        if n > n_max:
            continue
        if Q.dtype.kind == "f":
            _, idx = oracle.gray_solve(Q, threads=threads)
            best = [oracle.energy(Q, idx), idx]
            method = "O2"
        elif n <= 24:
            best = list(oracle.solve(Q, k=1, threads=threads)[0])
            method = "O1"
        else:
            best = list(oracle.gray_solve(Q, threads=threads))
            method = "O2"
        out[str(i)] = {"n": n, "dtype": "fp32" if Q.dtype.kind == "f" else "int32",
                       "method": method, "best": best}
        print(f"{name} request {i} n={n}: {best}", flush=True)
    return {"generator": "poisson_requests", "kwargs": kw, "n_max": n_max, "requests": out,
            "seconds": round(time.time() - t0, 2), "threads": threads or oracle.default_threads()}


def make_Q(gen, kw):
    out = getattr(inputs, gen)(**kw)
    return out[0] if gen == "planted" else out


def run_shards(name, Q, shards, threads):
    """O2 over ``shards`` equal Gray-index ranges, resumable; returns (best pair, seconds)."""
    path = os.path.join(HERE, f"shards_{name}.json")
    rec = {"name": name, "shards": shards, "done": {}}
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        if rec["shards"] != shards:
            raise SystemExit(f"{path} holds {rec['shards']} shards, not {shards}")
    total = 1 << Q.shape[0]
    for s in range(shards):
        if str(s) in rec["done"]:
            continue
        i0, i1 = s * total // shards, (s + 1) * total // shards
        t0 = time.time()
        e, idx = oracle.gray_solve_range(Q, i0, i1, threads=threads)
        rec["done"][str(s)] = {"best": [e, idx], "seconds": round(time.time() - t0, 2),
                               "threads": threads or oracle.default_threads()}
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(rec, f, indent=0, sort_keys=True)
        os.replace(tmp, path)
        print(f"{name} shard {s + 1}/{shards}: {e} at {idx} "
              f"({rec['done'][str(s)]['seconds']} s)", flush=True)
    best = min(tuple(d["best"]) for d in rec["done"].values())
    return best, sum(d["seconds"] for d in rec["done"].values())


def run(name, threads=0):
    gen, kw, method, k = ENTRIES[name][:4]
    shards = ENTRIES[name][4] if len(ENTRIES[name]) > 4 else 0
    Q = make_Q(gen, kw)
    t0 = time.time()
    if shards:
        best, dt = run_shards(name, Q, shards, threads)
        pairs = [best]
    elif method == "O1":
        pairs = oracle.solve(Q, k=k, threads=threads)
    else:
        pairs = [oracle.gray_solve(Q, threads=threads)]
    if not shards:
        dt = time.time() - t0
    out = {
        "generator": gen, "kwargs": kw, "dtype": "fp32" if Q.dtype.kind == "f" else "int32",
        "method": method, "best": list(pairs[0]), "topk": [list(p) for p in pairs],
        "seconds": round(dt, 2), "threads": threads or oracle.default_threads(),
    }
    if shards:
        out["shards"] = shards
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*")
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (0: every core)")
    args = ap.parse_args()
    for name in (args.only or list(ENTRIES) + list(SERVE)):
        res = run_serve(name, args.threads) if name in SERVE else run(name, args.threads)
        print(name, res.get("best", ""), f"{res['seconds']}s", flush=True)
        # re-read just before writing: another run may have stored entries meanwhile
        data = {}
        if os.path.exists(OUT):
            with open(OUT) as f:
                data = json.load(f)
        data[name] = res
        tmp = OUT + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, OUT)


if __name__ == "__main__":
    main()
