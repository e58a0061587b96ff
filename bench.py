"""Benchmark: exhaustive dense-QUBO minimisation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batch] [--no-serve]

One step = one complete solve (plan, table build, Gray walk, finish, result
copy) of the headline workload: a dense n=44 int32 QUBO, entries i.i.d.
uniform in [-10000, 10000], seed 4, held in device memory (a torch tensor)
before the timed region starts.  Prints ONE JSON line.

value            = 2^44 * K / (timed seconds)  [states/s, whole job]
roofline         = the walk kernel (dominant kernel) against the int32 VALU
                   peak of MI355X: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz
                   = 78.64 T int32 lane-ops/s (the published 157.3 TFLOP/s fp32
                   vector rate counts an FMA lane-op as 2 flops; v_add_u32
                   issues a wave64 in 2 cycles, as the VALU probe confirms);
                   algorithmic work = 1 int32 add per state (the Gray update of
                   Sec. III-B); duration = HIP events around the walk kernel on
                   its own stream.
cpu_baseline     = the CPU oracle (direct evaluation) timed on this host over a
                   bounded contiguous index range of the same instance.
batched          = 4096 instances, n ~ U{20..34}, int32 U[-100,100] (seed 5):
                   aggregate states/s of one graph replay; batched_fp32 the
                   same with float32 N(0,1) entries (seed 6).  Instances whose
                   chunk energies fit 16 bits run the packed walk (tier 4, two
                   states per int32 add); frac_of_valu_peak compares the rate
                   with the peak of the batch's own mix of tiers (78.64 T
                   states/s for an int32 walk, twice that packed).
single_packed    = one lone solve of a dense n=44 int32 QUBO with entries
                   U[-20,20] (seed 4), small enough for the packed walk: the
                   same kernel template as the headline with two 16-bit chunk
                   energies per word, against twice the int32 add peak.
topk             = the k = 1024 lowest-energy states of a dense n = 40 int32
                   instance (U[-10000,10000], seed 3): walk (tier 3) and
                   end-to-end time; "packed" the same for entries U[-100,100]
                   (tier 5, the packed layout).
serving          = Poisson arrivals at a fixed rate (seed 7), n ~ U{16..40},
                   80% int32 U[-100,100] / 20% float32 N(0,1): p50/p99 latency
                   (arrival -> result) and aggregate states/s through the
                   continuous-batching server; the same requests submitted
                   at once (saturation throughput and capacity in requests/s);
                   and Poisson arrivals at half that capacity (half_load).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9        # int32 lane-ops/s
METRIC = ("states/sec on 1 MI355X (single n=44; batched mixed-n) vs VALU peak; "
          "p50/p99 solve latency")
HEADLINE = dict(n=44, lo=-10000, hi=10000, seed=4)
PMC_FILE = os.path.join(ROOT, "profiles", "walk_n44_pmc.md")
# sources of the walk kernel (its template, helpers, layout and the unit of
# the headline variant); a PMC summary taken with other sources is stale
KERNEL_SRCS = [os.path.join(ROOT, "paper_2607_04857_amd", "csrc", f)
               for f in ("kernels.h", "kcommon.h", "walk.h", "walk_g6.hip")]


def kernel_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_name(r):
    """Template instance of the walk kernel a plan runs (row caches "4" and
    "3" are G = 6 and G = 5 with the rows of levels 3 and 4 in LDS)."""
    mc = 2 ** (r.B - 7 if r.tier >= 4 else r.B - 6)    # words per lane
    if r.vgpr_levels in (3, 4):
        return "walk_kernel<%d,%d,%d,true>" % (mc, r.vgpr_levels + 2, r.tier)
    return "walk_kernel<%d,%d,%d>" % (mc, r.vgpr_levels, r.tier)


def traffic_from_profile():
    """HBM bytes per walk launch from the committed PMC summary, if still valid."""
    if not os.path.exists(PMC_FILE):
        return None
    txt = open(PMC_FILE).read()
    m_h = re.search(r"walk sources sha256\[:16\]:\s*`?([0-9a-f]{16})", txt)
    m_b = re.search(r"HBM bytes per walk launch:\s*([0-9.eE+]+)", txt)
    if not m_h or not m_b or m_h.group(1) != kernel_hash():
        return None
    return float(m_b.group(1))


def host_cpus():
    """CPUs this process may run on: the affinity mask, capped by a cgroup CPU
    quota when one is set; with the counts it came from and the CPU model."""
    nproc = os.cpu_count() or 1
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else nproc
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, period = f.read().split()[:2]
        if q != "max":
            quota = -(-int(q) // int(period))
    except (OSError, ValueError):
        pass
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = min(affinity, quota) if quota else affinity
    return usable, {"nproc": nproc, "affinity": affinity, "cgroup_quota_cpus": quota,
                    "cpu_model": model}


def cpu_baseline(Q, budget_s=20.0):
    import oracle
    threads, info = host_cpus()
    n = Q.shape[0]
    first = 0x5A5A5A5 << 17          # a fixed contiguous slice of the 2^44 index space
    probe = 1 << 22
    t0 = time.perf_counter()
    oracle.solve_range(Q, first, probe, k=1, threads=threads)
    rate0 = probe / max(time.perf_counter() - t0, 1e-6)
    count = int(min(max(rate0 * budget_s, probe), 1 << 34))
    t0 = time.perf_counter()
    oracle.solve_range(Q, first, count, k=1, threads=threads)
    dt = time.perf_counter() - t0
    out = {"value": count / dt, "unit": "states/s", "cores": threads, "kind": "oracle",
           "sample": f"direct evaluation of {count} consecutive states (indices "
                     f"[{first}, {first + count})) of the n={n} instance, {dt:.1f} s, "
                     f"one thread per usable host CPU"}
    out.update(info)
    return out


TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2607_04857_amd",
                          "tuning", "gfx950_256cu.json")


def batched(q, steps=2, kind="int"):
    """One graph replay of the 4096-instance batch, with the plans the shipped
    autotuner cache holds for batch instances on this device (built-in plans
    where the cache was made on another device)."""
    from paper_2607_04857_amd import inputs
    seed = 5 if kind == "int" else 6
    Qs = inputs.batch(4096, 20, 34, seed=seed, kind=kind, lo=-100, hi=100)
    tuned = False
    try:
        tuned = q.tune_load(TUNE_CACHE) > 0
    except q.QuboError:
        pass
    b = q.Batch(Qs)
    q.tune_clear()
    b.run()                                   # warm-up replay
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run()
    dt = (time.perf_counter() - t0) / steps
    states, kms = b.stats()
    res = b.results()
    b.close()
    # states by walk tier; the peak of this mix: int32 walks at one state per
    # lane-op, packed (tier 4) at two, direct evaluation counted as int32
    by_tier = {}
    for r in res:
        by_tier[str(r.tier)] = by_tier.get(str(r.tier), 0.0) + float(r.states)
    peak_s = sum(st / (VALU_PEAK_OPS * (2 if t == "4" else 1)) for t, st in by_tier.items())
    what = "int32 U[-100,100], seed 5" if kind == "int" else "float32 N(0,1), seed 6"
    return {"workload": f"4096 dense QUBOs, n~U{{20..34}}, {what}",
            "plans": "autotuned (batch scope)" if tuned else "built-in",
            "states_per_s": states / dt, "ms_per_replay": dt * 1e3,
            "states": states, "graph_ms": kms,
            "states_by_tier": by_tier,
            "mix_peak_states_per_s": states / peak_s,
            "frac_of_valu_peak": (states / dt) / (states / peak_s)}


def single_packed(q, steps=3):
    """Lone solves of an n = 44 instance whose chunk energies fit 16 bits."""
    from paper_2607_04857_amd import inputs
    Q = inputs.uniform_int(44, -20, 20, 4)
    r = q.solve(Q)                            # warm-up
    kms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = q.solve(Q)
        kms.append(r.kernel_ms)
    dt = (time.perf_counter() - t0) / steps
    walk_ms = sum(kms) / len(kms)
    walk_rate = 2.0 ** 44 / (walk_ms / 1e3)
    return {"workload": "single dense QUBO n=44, int32 U[-20,20], seed 4 (host input)",
            "tier": r.tier, "A": r.A, "B": r.B, "L": r.L, "vgpr_levels": r.vgpr_levels,
            "kernel": kernel_name(r), "result": [r.energy_i, r.index],
            "ms_per_solve": dt * 1e3, "states_per_s": 2.0 ** 44 / dt, "walk_ms": walk_ms,
            "walk_states_per_s": walk_rate, "peak_states_per_s": 2 * VALU_PEAK_OPS,
            "frac": walk_rate / (2 * VALU_PEAK_OPS)}


def topk(q, torch, n=40, k=1024, steps=2):
    from paper_2607_04857_amd import inputs
    Q = inputs.uniform_int(n, -10000, 10000, 3)
    dQ = torch.from_numpy(Q).to("cuda:0")
    stream = torch.cuda.current_stream()
    q.solve_device(dQ, k=k, stream=stream)            # warm-up
    best = None
    for _ in range(steps):
        r, pairs = q.solve_device(dQ, k=k, stream=stream)
        if best is None or r.total_ms < best[0].total_ms:
            best = (r, pairs)
    r, pairs = best
    one = q.solve_device(dQ, stream=stream)
    # the same k on an instance whose chunk energies fit 16 bits: the packed
    # top-k walk (tier 5), from host memory, against its own k = 1 walk
    P = inputs.uniform_int(n, -100, 100, 3)
    rp, pp = q.solve(P, k=k)
    rp, pp = q.solve(P, k=k)
    one_p = q.solve(P)
    return {"workload": f"k={k} lowest states of a dense n={n} int32 QUBO, U[-10000,10000], seed 3",
            "walk_ms": r.kernel_ms, "total_ms": r.total_ms,
            "states_per_s": 2.0 ** n / (r.total_ms / 1e3),
            "k1_walk_ms": one.kernel_ms, "kth_energy": pairs[-1][0], "best": list(pairs[0]),
            "packed": {"workload": f"k={k}, n={n}, int32 U[-100,100], seed 3 (host input)",
                       "tier": rp.tier, "walk_ms": rp.kernel_ms, "total_ms": rp.total_ms,
                       "k1_tier": one_p.tier, "k1_walk_ms": one_p.kernel_ms,
                       "kth_energy": pp[-1][0]}}


def serving(q, count=600, rate_hz=150.0):
    """The served mix at a light fixed rate, at saturation (every request
    submitted at once), and at half the saturation capacity measured here
    (requests/s), where requests overlap on the device."""
    import threading
    from paper_2607_04857_amd import inputs

    def mix(rate):
        # the same instances at any rate (the arrival gaps scale, the draws do not change)
        return inputs.poisson_requests(count, rate, 16, 40, seed=7, int_fraction=0.8)

    def run(reqs, paced):
        srv = q.Server(mem_budget_bytes=8 << 30, max_slots=512)
        tickets = [None] * len(reqs)

        def submitter():
            t0 = time.perf_counter()
            for k, (arrival, Q) in enumerate(reqs):
                if paced:
                    while time.perf_counter() - t0 < arrival:
                        time.sleep(0.0001)
                tickets[k] = srv.submit(Q)

        t0 = time.perf_counter()
        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        res = []
        for t in tickets:
            res.append(srv.wait(t, timeout_ms=600000))
            assert res[-1] is not None
        wall = time.perf_counter() - t0
        st = srv.stats()
        info = srv.info()
        info["results"] = res
        srv.close()
        return st, info, wall

    reqs = mix(rate_hz)
    states = sum(2.0 ** Q.shape[0] for _, Q in reqs)
    st, info, wall = run(reqs, True)
    sat, sinfo, sat_wall = run(reqs, False)
    capacity = count / sat_wall                      # requests/s at saturation
    # the served mix's own peak: packed (tier 4) requests at two states per
    # int32 lane-op, the others at one
    by_tier = {}
    for r in sinfo["results"]:
        by_tier[str(r.tier)] = by_tier.get(str(r.tier), 0.0) + float(r.states)
    peak_s = sum(v / (VALU_PEAK_OPS * (2 if t == "4" else 1)) for t, v in by_tier.items())
    half_rate = 0.5 * capacity
    reqs_h = mix(half_rate)
    hst, hinfo, hwall = run(reqs_h, True)
    return {"workload": f"{count} requests, Poisson {rate_hz:g}/s, n~U{{16..40}}, 80% int32 "
                        "U[-100,100] / 20% fp32 N(0,1), seed 7",
            "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "states_per_s": states / wall,
            "offered_states_per_s": states / reqs[-1][0], "ticks": info["ticks"],
            "mem_peak_bytes": info["mem_peak"],
            "saturation_states_per_s": states / sat_wall,
            "states_by_tier": by_tier, "mix_peak_states_per_s": states / peak_s,
            "saturation_frac_of_mix_peak": (states / sat_wall) / (states / peak_s),
            "saturation_p50_ms": sat["p50_ms"], "saturation_p99_ms": sat["p99_ms"],
            "capacity_req_per_s": capacity,
            "half_load": {"rate_req_per_s": half_rate, "p50_ms": hst["p50_ms"],
                          "p99_ms": hst["p99_ms"], "states_per_s": states / hwall,
                          "offered_states_per_s": states / reqs_h[-1][0],
                          "ticks": hinfo["ticks"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-topk", action="store_true")
    ap.add_argument("--no-packed", action="store_true")
    ap.add_argument("--only-packed", action="store_true",
                    help="only the packed n=44 lone solves (profiling the packed walk alone)")
    ap.add_argument("--only-topk", action="store_true",
                    help="only the n=40 top-k instance: two k=1024 solves, then two k=1 solves "
                         "(profiling the top-k walk against the k=1 walk)")
    ap.add_argument("--skip-single", action="store_true",
                    help="skip the n=44 solves (profiling the batched or served kernels alone)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run one plain device copy of BYTES (HBM counter calibration)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only sweep the VALU probe (every op at 1..8 waves per SIMD) and "
                         "print one JSON line per measurement")
    args = ap.parse_args()
    if args.valu_probe:
        import paper_2607_04857_amd as q
        for op in ("add", "min3", "add+salu", "add+branch", "pk_add16", "pk_min16", "add_3w",
                   "add_f32"):
            for w in range(1, 9):
                rate, ms = q.probe_valu(op, w, 4096)
                print(json.dumps({"op": op, "waves_per_simd": w, "lane_ops_per_s": rate,
                                  "ms": ms}), flush=True)
        return
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the solve would shard "
              "by Gray-index range across GPUs with one MIN reduction of an (energy, row) "
              "pair, which is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2607_04857_amd as q
    from paper_2607_04857_amd import inputs

    torch.cuda.set_device(0)
    Q = inputs.uniform_int(HEADLINE["n"], HEADLINE["lo"], HEADLINE["hi"], HEADLINE["seed"])
    dQ = torch.from_numpy(Q).to("cuda:0")
    stream = torch.cuda.current_stream()
    n = Q.shape[0]

    if args.only_packed:
        print(json.dumps({"single_packed": single_packed(q)}), flush=True)
        return
    if args.only_topk:
        T = inputs.uniform_int(40, -10000, 10000, 3)
        out = []
        for k in (1024, 1024, 1, 1):
            r = q.solve(T, k=k)
            r = r[0] if k > 1 else r
            out.append({"k": k, "tier": r.tier, "walk_ms": r.kernel_ms})
        print(json.dumps({"topk_profile": out}), flush=True)
        return
    if args.skip_single:
        out = {}
        if not args.no_batch:
            out["batched"] = batched(q)
            out["batched_fp32"] = batched(q, kind="fp32")
        if not args.no_serve:
            out["serving"] = serving(q)
        print(json.dumps(out), flush=True)
        return

    for _ in range(args.warmup):
        q.solve_device(dQ, stream=stream)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = q.solve_device(dQ, stream=stream)
        kms.append(r.kernel_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    states = float(2 ** n) * args.steps
    value = states / dt
    walk_ms = sum(kms) / len(kms)
    achieved = (2.0 ** n) / (walk_ms / 1e3)          # int32 adds per second in the walk
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": "single dense QUBO n=44, int32 Q upper-triangular, entries "
                               "U[-10000,10000], seed 4", "n": n, "states_per_step": 2 ** n,
                   "tier": r.tier, "A": r.A, "B": r.B, "L": r.L, "vgpr_levels": r.vgpr_levels},
        "result": {"energy": r.energy_i, "index": r.index},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": traffic_from_profile(),
                     "kernel": kernel_name(r),
                     "walk_ms": walk_ms},
        "paper_context": {"states_per_s": 7.42e12, "hardware": "NVIDIA H100 80GB",
                          "precision": "int16", "n": 44},
    }
    probe, _ = q.probe_valu("add", 8, 2048)
    line["roofline"]["probe_peak"] = probe / 1e12       # measured v_add_u32 lane-ops/s
    line["roofline"]["frac_of_probe"] = achieved / probe
    if not args.no_packed:
        line["single_packed"] = single_packed(q)
    if not args.no_batch:
        line["batched"] = batched(q)
        line["batched_fp32"] = batched(q, kind="fp32")
    if not args.no_topk:
        line["topk"] = topk(q, torch)
    if not args.no_serve:
        line["serving"] = serving(q)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(Q)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
