#!/usr/bin/env python3
"""Throughput of sampled-compression-ratio structure prediction on one MI355X.

A step is one whole prediction, ssp_predict_structure, on device-resident
inputs: row sampling, per-row products of the sample, exact distinct counts of
the sampled rows, the sampled ratio, and the streaming pass that writes the
predicted nnz of every row.  The default workload is C = A.A with A the
2^20 x 2^20 R-MAT (0.57, 0.19, 0.19, 0.05) matrix of 16 edges per row,
duplicates merged, sampled at 0.5%.

Prints one JSON line.  `value` is predicted rows per second.  Beside it:
algorithmic HBM GB/s of the step, the device time of 100 single calls (p50,
p99, mean), the roofline of the dominant phase (its
duration from HIP events recorded on the launch stream over a second timed
region of the same steps: the events hold the queue at each phase boundary,
so the headline region runs without them), the reference design and exact
structure timed on the same input,
the accuracy of the prediction against the exact structure, and the CPU
oracle timed on the host (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
WORKLOADS = ("rmat20", "uniform4096", "stencil128", "stencil128_x_uniform", "sweep", "serve",
             "accuracy", "spgemm", "spgemm_rmat18")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="rmat20", choices=WORKLOADS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the reference/exact timings and the accuracy figures")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0,
                    help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--margin", type=int, default=10,
                    help="spgemm workloads: percent added to each predicted row capacity")
    ap.add_argument("--spill", type=int, default=25,
                    help="spgemm workloads: overflow area shared by the rows, percent of the slots")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES three times (the reference "
                         "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE) and exit")
    return ap.parse_args()


def progress(msg: str):
    """A progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_calibration(nbytes: int):
    import torch
    n = nbytes // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 4 * n, "launches": 3}), flush=True)


# Sources of the prediction path's kernels and their launches (the numeric
# product's and the sketch's files add kernels and entry points of their own).
PREDICT_SOURCES = ("ssp_device.hpp", "ssp_internal.hpp", "ssp_kernels.hpp", "ssp_lib.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2207_13848_amd", "csrc")
    for f in PREDICT_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_phase: str, workload: str, src_hash: str):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if they
    were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel_phase}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != src_hash:
        return None
    return d.get("hbm_bytes_per_launch")


KERNEL_OF_PHASE = {"flop": "k_flop", "sym_long": "k_sym_big", "sym_merge": "k_sym_merge",
                   "pred_rows": "k_pred_rows"}


def bernoulli_sample(M: int, rate: float, seed: int):
    """Indices of the rows the Bernoulli sampler keeps: the top 53 bits of
    splitmix64(seed, i) below floor(rate 2^53) (splitmix64: Steele, Lea &
    Flood 2014), the rule the library documents.  Used here only to split the
    byte count over kernels."""
    import numpy as np
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.arange(M, dtype=np.uint64) + np.uint64(1)) * \
            np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    thresh = 0 if rate <= 0 else (1 << 53) if rate >= 1 else int(rate * 9007199254740992.0)
    return np.nonzero((z >> np.uint64(11)) < np.uint64(thresh))[0]


def long_row_mask(rf_s, ncols: int):
    """Sampled rows the long-row kernel serves: above 8192 products, or above
    1024 when all columns fit one 2^20-column bitmap window but not a
    16384-word table."""
    lim = 1024 if (2 ** 19 < ncols <= 2 ** 20) else 8192
    return rf_s > lim


def eps_from_stats(s: dict, Z: int) -> dict:
    """The errors of Sec. VI-A from one prediction's integer statistics and
    the exact total Z: eps1 = Z1*/Z - 1 with Z1* = z* M / n_s (Eq. (2)),
    epsf = F*/F - 1 with F* = f* M / n_s (Eq. (3)), eps2 = Z2*/Z - 1 with
    Z2* = F z* / f* (Eq. (4)), eps2_alloc = (sum of the per-row ceilings)/Z - 1.
    Each is the exact rational's nearest double (Python's int / int rounds
    correctly); None where an estimate or the truth is zero."""
    M, F = s["nrows"], s["total_flop"]
    ns, fs, zs = s["n_sampled"], s["sample_flop"], s["sample_nnz"]
    out = {"eps1": None, "epsf": None, "eps2": None, "eps2_alloc": None}
    if Z > 0 and ns > 0:
        out["eps1"] = (zs * M - ns * Z) / (ns * Z)
    if F > 0 and ns > 0:
        out["epsf"] = (fs * M - ns * F) / (ns * F)
    if Z > 0 and fs > 0:
        out["eps2"] = (F * zs - fs * Z) / (fs * Z)
    if Z > 0:
        out["eps2_alloc"] = (s["out_sum"] - Z) / Z
    return out


def summarise_eps(recs) -> dict:
    """Mean and worst |eps| over cases (Sec. VI-A's statistics) from
    (structure, eps dict) records; cases with an undefined eps are counted
    as excluded."""
    import numpy as np
    keep = [(st, e) for st, e in recs if None not in (e["eps1"], e["epsf"], e["eps2"])]
    out = {"cases": len(keep), "excluded": len(recs) - len(keep)}
    if not keep:
        return out
    arr = {k: np.array([e[k] for _, e in keep]) for k in ("eps1", "epsf", "eps2", "eps2_alloc")}
    for k, v in arr.items():
        out[f"mean_abs_{k}"] = float(np.mean(np.abs(v)))
        out[f"worst_abs_{k}"] = float(np.max(np.abs(v)))
    out["frac_abs_eps2_lt_abs_eps1"] = float(np.mean(np.abs(arr["eps2"]) < np.abs(arr["eps1"])))
    out["by_structure"] = {}
    sts = np.array([st for st, _ in keep])
    for name in sorted(set(sts.tolist())):
        m = sts == name
        out["by_structure"][name] = {"mean_abs_eps1": float(np.mean(np.abs(arr["eps1"][m]))),
                                     "mean_abs_eps2": float(np.mean(np.abs(arr["eps2"][m]))),
                                     "worst_abs_eps2": float(np.max(np.abs(arr["eps2"][m])))}
    return out


def sweep_compare(ssp, params, reps: int = 3, accuracy: bool = False):
    """Plain (one call per matrix, back to back on one stream) vs batched (one
    ssp_predict_batch) vs graph (one launch of a captured batch) over the given
    sweep cases; the three outputs are checked equal.  Times in ms: minimum
    over `reps` timed runs after one warm-up.  With `accuracy`, every case's
    exact structure (ssp_exact_structure) judges the batch's prediction:
    mean and worst |eps1|, |eps2|, |epsf| over the cases."""
    import torch
    import workloads
    t0 = time.time()
    hosts = []
    for k, p in enumerate(params):
        hosts.append(workloads.sweep_workload(p))
        if k % 125 == 124:
            progress(f"generated {k + 1}/{len(params)} cases")
    t_gen = time.time() - t0
    dev = "cuda:0"
    h = ssp.default_handle(dev)
    devA = [ssp.DeviceCSR.from_csr(w.A, dev) for w in hosts]
    mk = lambda: [ssp.Case(A, A, w.rate, w.seed) for A, w in zip(devA, hosts)]  # noqa: E731
    plain, batch, graphc = mk(), mk(), mk()
    g = ssp.BatchGraph(graphc, handle=h)

    def run_plain():
        for c in plain:
            ssp.predict_structure(c.A, c.B, c.sample_rate, c.seed, handle=h, out=c.pred,
                                  stats=c.stats)

    runs = {"plain": run_plain, "batched": lambda: ssp.predict_batch(batch, handle=h),
            "graph": g.launch}
    ms = {}
    for name, fn in runs.items():
        progress(f"timing {name}")
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            ta = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - ta) * 1e3
            best = dt if best is None else min(best, dt)
        ms[name] = best
    same = all(torch.equal(a.pred, b.pred) and torch.equal(a.pred, c.pred) and
               torch.equal(a.stats, b.stats) and torch.equal(a.stats, c.stats)
               for a, b, c in zip(plain, batch, graphc))
    rows = sum(w.A.nrows for w in hosts)
    nnz = sum(w.A.nnz for w in hosts)
    stream_bytes = sum(4 * (w.A.nrows + 1) + 4 * w.A.nnz + 8 * w.A.nrows for w in hosts)
    sym_bytes = 0
    for c in batch:
        st = ssp.read_stats(c.stats)
        sym_bytes += 8 * st["n_sampled"] + 12 * st["a_sample_nnz"] + 4 * st["sample_flop"]
    out = {"cases": len(hosts), "rows": rows, "nnz": nnz, "generate_s": round(t_gen, 1),
           "graph_workspace_bytes": g.workspace_bytes, "outputs_identical": bool(same),
           "algorithmic_bytes": stream_bytes + sym_bytes}
    for name, t in ms.items():
        out[f"{name}_ms"] = round(t, 3)
        out[f"{name}_rows_per_s"] = round(rows / (t * 1e-3), 1)
    out["speedup_batched_vs_plain"] = round(ms["plain"] / ms["batched"], 2)
    out["speedup_graph_vs_plain"] = round(ms["plain"] / ms["graph"], 2)
    out["graph_gbps_algorithmic"] = round(out["algorithmic_bytes"] / (ms["graph"] * 1e-3) / 1e9, 1)
    g.close()
    if accuracy:
        ta = time.time()
        maxM = max(w.A.nrows for w in hosts)
        ex = torch.empty(maxM, dtype=torch.int64, device=dev)
        est = torch.zeros(8, dtype=torch.int64, device=dev)
        recs = []
        for p, A, c in zip(params, devA, batch):
            ssp.exact_structure(A, A, handle=h, out=ex[:A.nrows], stats=est)
            Z = ssp.read_stats(est)["out_sum"]
            recs.append((p[0], eps_from_stats(ssp.read_stats(c.stats), Z)))
        out["accuracy"] = summarise_eps(recs)
        out["accuracy"]["sampler"] = "bernoulli-splitmix64, rate 1%"
        out["accuracy"]["exact_s"] = round(time.time() - ta, 1)
    return out


def main_sweep(args):
    import torch
    import paper_2207_13848_amd as ssp
    import workloads
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    r = sweep_compare(ssp, workloads.sweep_cases(), reps=max(1, min(args.steps, 5)))
    t = r["graph_ms"]
    print(json.dumps({
        "metric": "predicted rows/s (625-case sweep, one batched graph launch)",
        "value": r["graph_rows_per_s"], "unit": "rows/s", "n_gpus": 1,
        "steps": max(1, min(args.steps, 5)), "warmup": 1, "ms_per_step": t,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "sweep625", "sizes": list(workloads.SWEEP_SIZES),
                   "degrees": list(workloads.SWEEP_DEGREES), "structures": list(workloads.STRUCTURES),
                   "seeds": list(workloads.SWEEP_SEEDS), "sample_rate": 0.01},
        "sweep": r}), flush=True)


def serve_run(ssp) -> dict:
    """Serving: Poisson arrivals (2000/s) of A.A predictions over a
    device-resident pool of 64 matrices (rows 2^U, U ~ Uniform[10, 21],
    structure uniform over the five generators, d uniform over 2..32, rate 1%),
    through the continuous-batching server; then a closed-loop burst for the
    saturation throughput.  A sample of results is checked against the same
    prediction made alone."""
    import numpy as np
    import torch
    import workloads
    rng = np.random.default_rng(8)
    t0 = time.time()
    pool = []
    for k in range(64):
        n = int(2.0 ** rng.uniform(10, 21))
        s = workloads.STRUCTURES[int(rng.integers(5))]
        d = int(rng.integers(2, 33))
        pool.append(workloads.make(s, n, d, 100 + k))
    t_gen = time.time() - t0
    dev = "cuda:0"
    devs = [ssp.DeviceCSR.from_csr(m, dev) for m in pool]
    srv = ssp.Server(slots=4, slot_bytes=2 << 30, max_batch=64)
    ids = [srv.register(d) for d in devs]
    ring = 256
    maxrows = max(m.nrows for m in pool)
    outs = [torch.empty(maxrows, dtype=torch.int64, device=dev) for _ in range(ring)]
    stats = [torch.zeros(8, dtype=torch.int64, device=dev) for _ in range(ring)]
    torch.cuda.synchronize()

    def run(n_req, lam):
        """Submit n_req requests (Poisson at lam/s, or all at once if lam is
        None); returns the requests and the wall time to the last completion."""
        arr = np.cumsum(rng.exponential(1.0 / lam, n_req)) if lam else np.zeros(n_req)
        pick = rng.integers(len(pool), size=n_req)
        reqs = []
        srv.reset_stats()
        start = time.perf_counter()
        for i in range(n_req):
            if i >= ring:
                srv.wait(reqs[i - ring][0], 600.0)  # the ring slot is reused
            while time.perf_counter() - start < arr[i]:
                pass
            j = int(pick[i])
            o = outs[i % ring][:pool[j].nrows]
            t = srv.submit(ids[j], ids[j], 0.01, 5000 + i, o, stats[i % ring])
            reqs.append((t, j, 5000 + i, i % ring))
        for r in reqs:
            srv.wait(r[0], 600.0)
        wall = time.perf_counter() - start
        return reqs, wall, srv.info()

    def check(reqs):
        ok = 0
        for t, j, seed, slot in reqs[-min(len(reqs), 24):]:
            p, _, st = ssp.predict_structure(devs[j], devs[j], 0.01, seed)
            torch.cuda.synchronize()
            ok += int(torch.equal(p, outs[slot][:pool[j].nrows]) and torch.equal(st, stats[slot]))
        return ok, min(len(reqs), 24)

    warm, _, _ = run(200, None)
    duration = 5.0
    lam = 2000.0
    reqs, wall, info = run(int(lam * duration), lam)
    ok, nchk = check(reqs)
    rows = sum(pool[r[1]].nrows for r in reqs)
    sat_reqs, sat_wall, sat_info = run(4000, None)
    sat_rows = sum(pool[r[1]].nrows for r in sat_reqs)
    srv.close()
    return {
        "requests_per_s": round(len(reqs) / wall, 1), "requests": len(reqs),
        "warmup": len(warm), "config": {"workload": "serve_poisson2000", "pool": len(pool),
                   "pool_rows_mean": float(np.mean([m.nrows for m in pool])),
                   "pool_nnz_total": int(sum(m.nnz for m in pool)), "sample_rate": 0.01,
                   "slots": 4, "slot_bytes": 2 << 30, "max_batch": 64, "duration_s": duration},
        "open_loop": {"offered_per_s": lam, "requests": len(reqs), "wall_s": round(wall, 3),
                      "rows_per_s": round(rows / wall, 1),
                      "latency_p50_ms": round(info["latency_p50_ms"], 3),
                      "latency_p99_ms": round(info["latency_p99_ms"], 3),
                      "latency_mean_ms": round(info["latency_mean_ms"], 3),
                      "latency_max_ms": round(info["latency_max_ms"], 3),
                      "batches": info["batches"], "max_batch_seen": info["max_batch_seen"],
                      "max_slots_busy": info["max_slots_busy"]},
        "saturation": {"requests": len(sat_reqs), "wall_s": round(sat_wall, 3),
                       "requests_per_s": round(len(sat_reqs) / sat_wall, 1),
                       "rows_per_s": round(sat_rows / sat_wall, 1),
                       "latency_p50_ms": round(sat_info["latency_p50_ms"], 3),
                       "latency_p99_ms": round(sat_info["latency_p99_ms"], 3),
                       "batches": sat_info["batches"],
                       "max_batch_seen": sat_info["max_batch_seen"],
                       "max_slots_busy": sat_info["max_slots_busy"]},
        "results_equal_alone": f"{ok}/{nchk}", "generate_s": round(t_gen, 1)}


def main_serve(args):
    import torch
    import paper_2207_13848_amd as ssp
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    r = serve_run(ssp)
    print(json.dumps({
        "metric": "served requests/s with p50/p99 latency (Poisson 2000/s, continuous batching)",
        "value": r["requests_per_s"], "unit": "requests/s", "n_gpus": 1,
        "steps": r["requests"], "warmup": r["warmup"],
        "ms_per_step": round(1e3 / r["requests_per_s"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic", **{k: v for k, v in r.items() if k not in ("requests_per_s",)}}),
        flush=True)


def main_accuracy(args):
    """Accuracy over the 625-case sweep (Sec. VI-A's analysis): per case the
    proposed prediction (Z2* = F z*/f*), the reference design (Z1* = z* M/n_s)
    and the exact total Z, all on the GPU, with the Bernoulli sampler at 1% and
    the paper's fixed-count sampler; errors eps = estimate / Z - 1, with
    eps_f = F*/F - 1 for F* = f* M / n_s (Eq. (5): (1+eps2)(1+epsf) = 1+eps1).
    Beside them the existing estimator of related work (Sec. III): Amossen's
    k minimum values (k = 1024) with BHash's row and column sampling at
    p = 1/10 (1% of the products, as the 1% row sample)."""
    import numpy as np
    import torch
    import paper_2207_13848_amd as ssp
    import workloads
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = "cuda:0"
    rows = []
    t0 = time.time()
    for p in workloads.sweep_cases():
        w = workloads.sweep_workload(p)
        A = ssp.DeviceCSR.from_csr(w.A, dev)
        ex, exs = ssp.exact_structure(A, A)
        out = {"structure": p[0], "n": p[1], "d": p[2], "seed": p[3]}
        for smp in ("bernoulli", "paper"):
            _, _, st = ssp.predict_structure(A, A, w.rate, w.seed, sampler=smp)
            _, rst = ssp.reference_estimate(A, A, w.rate, w.seed, sampler=smp)
            s_, r_ = ssp.read_stats(st), ssp.read_stats(rst)
            out[smp] = (s_, r_)
        out["kmv"] = ssp.kmv_estimate(A, A, 0.1, 1024, w.seed)["nnz_estimate"]
        e = ssp.read_stats(exs)
        out["Z"], out["F"] = e["out_sum"], e["total_flop"]
        rows.append(out)
        del A
    torch.cuda.synchronize()
    t_run = time.time() - t0

    def summarise(smp):
        recs, excluded = [], 0
        for r in rows:
            s_ = r[smp][0]
            Z, F, M = r["Z"], r["F"], r["n"]
            ns, fs, zs = s_["n_sampled"], s_["sample_flop"], s_["sample_nnz"]
            if Z == 0 or ns == 0 or fs == 0:
                excluded += 1
                continue
            recs.append((r["structure"], zs * M / ns / Z - 1, F * zs / fs / Z - 1,
                         fs * M / ns / F - 1, s_["out_sum"] / Z - 1))
        st = np.array([x[0] for x in recs])
        e1, e2, ef, ea = (np.array([x[k] for x in recs]) for k in (1, 2, 3, 4))
        out = {"cases": int(len(recs)), "excluded": excluded,
               "mean_abs_eps1": float(np.mean(np.abs(e1))), "worst_abs_eps1": float(np.max(np.abs(e1))),
               "mean_abs_eps2": float(np.mean(np.abs(e2))), "worst_abs_eps2": float(np.max(np.abs(e2))),
               "mean_abs_epsf": float(np.mean(np.abs(ef))), "worst_abs_epsf": float(np.max(np.abs(ef))),
               "mean_abs_eps2_alloc": float(np.mean(np.abs(ea))),
               "corr_eps1_epsf": float(np.corrcoef(e1, ef)[0, 1]),
               "frac_abs_eps2_lt_abs_eps1": float(np.mean(np.abs(e2) < np.abs(e1))),
               "frac_same_sign_eps1_epsf": float(np.mean(np.sign(e1) == np.sign(ef))),
               "by_structure": {}}
        for sname in workloads.STRUCTURES:
            m = st == sname
            if m.any():
                out["by_structure"][sname] = {
                    "mean_abs_eps1": float(np.mean(np.abs(e1[m]))),
                    "mean_abs_eps2": float(np.mean(np.abs(e2[m]))),
                    "worst_abs_eps2": float(np.max(np.abs(e2[m])))}
        return out

    def summarise_kmv():
        recs = [(r["structure"], r["kmv"] / r["Z"] - 1) for r in rows
                if r["Z"] and r["kmv"] is not None]
        st = np.array([x[0] for x in recs])
        e = np.array([x[1] for x in recs])
        out = {"cases": int(len(recs)), "mean_abs_eps": float(np.mean(np.abs(e))),
               "worst_abs_eps": float(np.max(np.abs(e))), "by_structure": {}}
        for sname in workloads.STRUCTURES:
            m = st == sname
            if m.any():
                out["by_structure"][sname] = {"mean_abs_eps": float(np.mean(np.abs(e[m]))),
                                              "worst_abs_eps": float(np.max(np.abs(e[m])))}
        return out

    print(json.dumps({"study": "accuracy over the 625-case sweep", "run_s": round(t_run, 1),
                      "bernoulli_1pct": summarise("bernoulli"),
                      "paper_sampler": summarise("paper"),
                      "kmv_p10_k1024": summarise_kmv(),
                      "paper_reports": {"mean_abs_eps1": 0.0812, "mean_abs_eps2": 0.0156,
                                        "worst_abs_eps1": 1.58, "worst_abs_eps2": 0.25}}),
          flush=True)


def main_spgemm(args):
    """The consumer of the prediction: numeric C = A.A (float64 values in
    U[-1, 1)) whose memory is sized by the predicted structure.  A step is the
    whole pipeline: ssp_predict_structure, ssp_spgemm_compute with the
    prediction plus a margin as row capacities and an overflow area shared by
    the rows, ssp_spgemm_copy.  Beside it, other margins and areas,
    the same numeric product sized by the precise method (ssp_exact_structure
    first: the symbolic phase the prediction avoids) and by the upper bound
    (row FLOP: no structure step, the largest slot area).  Sampled rows of C
    are checked against the CPU oracle."""
    import numpy as np
    import torch
    import paper_2207_13848_amd as ssp
    import workloads
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = "cuda:0"
    tg = time.time()
    if args.workload == "spgemm":
        A = workloads.stencil27(128)
        name, rate = "spgemm_stencil27_128", 0.005
    else:
        A = workloads.rmat(1 << 18, 16, 1)
        name, rate = "spgemm_rmat18_d16", 0.005
    seed = 1001
    av = workloads.values(A.nnz, 77)
    Ad = ssp.DeviceCSR.from_csr(A, dev)
    tav = torch.from_numpy(av).to(dev)
    t_gen = time.time() - tg
    M = A.nrows
    h = ssp.default_handle(dev)
    pred = torch.empty(M, dtype=torch.int64, device=dev)
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    margin, spill = int(args.margin), int(args.spill)

    def step():
        ssp.predict_structure(Ad, Ad, rate, seed, handle=h, out=pred, stats=st)
        return ssp.spgemm(Ad, tav, Ad, tav, pred, margin_pct=margin, spill_pct=spill, handle=h)

    steps = max(1, min(args.steps, 10))
    for _ in range(max(1, min(args.warmup, 2))):
        out = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    C_rpt, C_col, C_val, info = out
    F = info["total_flop"]
    # phase-timed region
    h._lib.ssp_timing_enable(h.ptr, 1)
    phase_times(ssp, h)
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    phases = phase_times(ssp, h)
    h._lib.ssp_timing_enable(h.ptr, 0)
    C_rpt, C_col, C_val, info = out

    # algorithmic bytes of the numeric pass: A.rpt pair per row, A.col + A.val
    # + B.rpt pair per A entry, B.col + B.val per product, the row written
    # (column + value) and its count
    rpt64 = A.rpt.astype(np.int64)
    alen = np.diff(rpt64)
    _, rf_t, _ = ssp.predict_structure(Ad, Ad, rate, seed, handle=h, return_row_flop=True)
    rf = rf_t.cpu().numpy()
    cnt = np.diff(C_rpt.cpu().numpy())
    dense = rf > 2048

    def pass_bytes(mask):
        return int(np.sum(8 + 20 * alen[mask] + 12 * rf[mask] + 12 * cnt[mask] + 8))

    phase_bytes = {"num_hash": pass_bytes(~dense & (rf > 0)), "num_dense": pass_bytes(dense),
                   "num_copy": int(24 * cnt.sum() + 24 * M)}
    per_phase = {}
    for pname, (n, tms) in phases.items():
        r = {"launches": n, "avg_us": round(1e3 * tms / max(n, 1), 2)}
        if phase_bytes.get(pname):
            r["algorithmic_bytes"] = phase_bytes[pname] // max(1, n // steps)
            r["gbps"] = round(phase_bytes[pname] * (n // steps) / max(n, 1) /
                              (1e-6 * r["avg_us"]) / 1e9, 1) if r["avg_us"] else None
        per_phase[pname] = r
    cand = [p for p in ("num_hash", "num_dense", "num_copy") if p in per_phase]
    dom = max(cand, key=lambda p: per_phase[p]["avg_us"] * per_phase[p]["launches"])
    dom_us = per_phase[dom]["avg_us"]
    dom_bytes = per_phase[dom].get("algorithmic_bytes", 0)
    achieved = dom_bytes / (dom_us * 1e-6) / 1e9 if dom_us else 0.0
    roofline = {"bound": "hbm", "kernel": {"num_hash": "k_num_hash", "num_dense": "k_num_dense",
                                           "num_copy": "k_num_copy"}[dom],
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "algorithmic_bytes": dom_bytes, "avg_launch_us": dom_us}

    # the precise method and the upper bound as capacities
    info_keys = ("slot_entries", "slot_bytes", "overflow_rows", "overflow_nnz", "spill_rows",
                 "spill_nnz", "spill_bytes")
    variants = {f"predicted_m{margin}_s{spill}": {
        "ms": round(ms, 3), "margin_pct": margin, "spill_pct": spill, "headline": True,
        **{k: info[k] for k in info_keys}}}
    ex = torch.empty(M, dtype=torch.int64, device=dev)
    # other margins and overflow areas on the prediction (memory against
    # recomputed rows), the precise method and the upper bound
    other = [(m, sp) for m, sp in ((0, 0), (10, 0), (30, 0), (100, 0), (0, 25), (0, 50), (10, 50))
             if (m, sp) != (margin, spill)]
    for vname in [f"predicted_m{m}_s{sp}" for m, sp in other] + ["precise", "upper_bound"]:
        for i in range(steps + 1):
            if i == 1:
                torch.cuda.synchronize()
                ta = time.perf_counter()
            if vname == "precise":
                ssp.exact_structure(Ad, Ad, handle=h, out=ex)
                r = ssp.spgemm(Ad, tav, Ad, tav, ex, handle=h)
            elif vname == "upper_bound":
                r = ssp.spgemm(Ad, tav, Ad, tav, rf_t, handle=h)
            else:
                m, sp = (int(x) for x in vname[len("predicted_m"):].split("_s"))
                ssp.predict_structure(Ad, Ad, rate, seed, handle=h, out=pred, stats=st)
                r = ssp.spgemm(Ad, tav, Ad, tav, pred, margin_pct=m, spill_pct=sp, handle=h)
        torch.cuda.synchronize()
        vi = r[3]
        vr = {"ms": round((time.perf_counter() - ta) * 1e3 / steps, 3)}
        if vname.startswith("predicted"):
            vr["margin_pct"], vr["spill_pct"] = m, sp
        variants[vname] = {**vr, **{k: vi[k] for k in info_keys}}
        assert vi["nnz"] == info["nnz"]
        del r
    torch.cuda.synchronize()

    # parity spot check: sampled rows against the oracle
    import oracle
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(M, size=min(M, 2000), replace=False))
    idx = np.concatenate([np.arange(rpt64[i], rpt64[i + 1]) for i in rows])
    srpt = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(alen[rows], out=srpt[1:])
    As = workloads.CSR(len(rows), A.ncols, srpt.astype(np.int32), A.col[idx].copy(), "rows")
    sub_vals = av[idx]
    orpt, ocol, oval, oabs, oterms = oracle.spgemm(As, sub_vals, A, av)
    crpt = C_rpt.cpu().numpy()
    gidx = np.concatenate([np.arange(crpt[i], crpt[i + 1]) for i in rows])
    gsel = torch.from_numpy(gidx).to(dev)
    gc = C_col.index_select(0, gsel).cpu().numpy()
    gv = C_val.index_select(0, gsel).cpu().numpy()
    bound = 2.0 * (oterms + 1.0) * 2.0 ** -53 * oabs * (1 + 1e-9)
    ok = bool(np.array_equal(np.diff(crpt)[rows], np.diff(orpt)) and np.array_equal(gc, ocol)
              and np.all(np.abs(gv - oval) <= bound))

    result = {
        "metric": "intermediate products/s of the numeric SpGEMM sized by the prediction",
        "value": round(F / (ms * 1e-3), 1), "unit": "products/s", "n_gpus": 1, "steps": steps,
        "warmup": max(1, min(args.warmup, 2)), "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "rows": M, "nnz_A": A.nnz, "sample_rate": rate, "seed": seed,
                   "margin_pct": margin, "spill_pct": spill, "values": "U[-1,1) float64"},
        "gflops": round(2.0 * F / (ms * 1e-3) / 1e9, 1),
        "nnz_C": info["nnz"], "F": F, "roofline": roofline, "phases": per_phase,
        "variants": variants,
        "parity_spot_check": {"rows": int(len(rows)), "ok": bool(ok)},
        "kernel_source_hash": kernel_source_hash(), "generate_s": round(t_gen, 2),
    }
    if not args.no_cpu_baseline:
        # the oracle on a bounded sample of rows, scaled to products/s
        sample_F = int(oterms.sum())
        tc0 = time.perf_counter()
        runs = 0
        while True:
            oracle.spgemm(As, sub_vals, A, av)
            runs += 1
            if time.perf_counter() - tc0 >= min(args.cpu_budget_s, 10.0) or runs >= 20:
                break
        t_cpu = (time.perf_counter() - tc0) / runs
        result["cpu_baseline"] = {"value": round(sample_F / t_cpu, 1), "unit": "products/s",
                                  "cores": 1, "kind": "oracle",
                                  "sample": f"{len(rows)} random rows of C ({sample_F} products), "
                                            f"serial C oracle, {runs} runs"}
    print(json.dumps(result), flush=True)


def get_workload(name: str):
    import workloads
    return getattr(workloads, name)()


def phase_times(ssp, handle):
    from paper_2207_13848_amd import _native
    buf = (_native.SspPhaseTime * 16)()
    n = handle._lib.ssp_timing_read(handle.ptr, buf, 16)
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(n)}


def measure(ssp, w, args, *, extras: bool, cpu: bool) -> dict:
    """One workload's line: K timed predictions on device-resident inputs,
    100 single-call device times, the phase-timed region and the roofline of
    its dominant kernel; with `extras` the reference design, the exact
    structure, the accuracy and the sketch on the same input; with `cpu` the
    oracle timed on the host."""
    import numpy as np
    import torch
    dev = "cuda:0"
    t_gen = time.time()
    A, B = w.A, w.B
    aliased = B is A
    Ad = ssp.DeviceCSR.from_csr(A, dev)
    Bd = Ad if aliased else ssp.DeviceCSR.from_csr(B, dev)
    t_gen = time.time() - t_gen
    M = A.nrows
    h = ssp.default_handle(dev)
    out = torch.empty(M, dtype=torch.int64, device=dev)
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        ssp.predict_structure(Ad, Bd, w.rate, w.seed, handle=h, out=out, stats=st)
    torch.cuda.synchronize()
    # The headline timed region runs without the library's phase timers: their
    # HIP events on the stream hold the queue at every phase boundary.
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ssp.predict_structure(Ad, Bd, w.rate, w.seed, handle=h, out=out, stats=st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # Per-call device time over 100 calls: HIP events on the call's stream
    # before and after each call, all calls queued back to back.
    nlat = 100
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(nlat)]
    for a, b in ev:
        a.record(stream)
        ssp.predict_structure(Ad, Bd, w.rate, w.seed, handle=h, out=out, stats=st)
        b.record(stream)
    torch.cuda.synchronize()
    lat = np.sort(np.array([a.elapsed_time(b) for a, b in ev]))
    call_ms = {"runs": nlat, "p50": round(float(np.percentile(lat, 50)), 4),
               "p99": round(float(np.percentile(lat, 99)), 4), "mean": round(float(lat.mean()), 4)}
    # The phase-timed region: the same steps, HIP events around every phase
    # on the call's stream; the kernel durations of the roofline come from it.
    h._lib.ssp_timing_enable(h.ptr, 1)
    phase_times(ssp, h)  # clear
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        ssp.predict_structure(Ad, Bd, w.rate, w.seed, handle=h, out=out, stats=st)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    phases = phase_times(ssp, h)
    h._lib.ssp_timing_enable(h.ptr, 0)
    ms_per_step_timed = (t3 - t2) * 1e3 / args.steps
    stats = ssp.read_stats(st)

    # ---- algorithmic bytes (integers of the CSR format: 4-byte indices)
    # Per-row products and the sampled set, to split the symbolic bytes over
    # the kernels that serve each row (one call outside the timed region).
    _, rf_t, _ = ssp.predict_structure(Ad, Bd, w.rate, w.seed, handle=h, return_row_flop=True)
    rf_np = rf_t.cpu().numpy().astype(np.uint64)
    sampled = bernoulli_sample(M, w.rate, w.seed)
    alen = np.diff(A.rpt.astype(np.int64))[sampled]
    rf_s = rf_np[sampled].astype(np.int64)
    long_rows = long_row_mask(rf_s, B.ncols)
    nnzA, K = A.nnz, A.ncols
    n_s, a_s, f_s = stats["n_sampled"], stats["a_sample_nnz"], stats["sample_flop"]
    assert n_s == len(rf_s) and f_s == int(rf_s.sum()) and a_s == int(alen.sum())

    def sym(mask):  # A.rpt pair + A.col and B.rpt pair per entry + B.col per product
        return int(np.sum(8 + 12 * alen[mask] + 4 * rf_s[mask]))

    flop_bytes = 4 * (M + 1) + 4 * nnzA + (0 if aliased else 4 * (K + 1)) + 8 * M
    phase_bytes = {"flop": flop_bytes, "sym_long": sym(long_rows), "sym_bins": sym(~long_rows),
                   "sample_bin": 16 * n_s, "pred_rows": 16 * M, "tiles": 4 * (M + 1)}
    # the whole call: the stream, the sampled rows, the nnz_pred output
    step_bytes = flop_bytes + sym(np.ones_like(long_rows))
    per_phase = {}
    for name, (n, ms) in phases.items():
        per_phase[name] = {"launches": n, "avg_us": 1e3 * ms / max(n, 1)}
    # the dominant kernel: each of these phases times one kernel
    single = [p for p in ("flop", "sym_long", "sym_merge", "pred_rows") if p in per_phase]
    dom = max(single, key=lambda p: per_phase[p]["avg_us"])
    dom_us = per_phase[dom]["avg_us"]
    dom_bytes = phase_bytes.get(dom, 0)
    achieved = dom_bytes / (dom_us * 1e-6) / 1e9
    src_hash = kernel_source_hash()
    traffic = load_traffic(dom, w.name, src_hash)
    roofline = {"bound": "hbm", "kernel": KERNEL_OF_PHASE[dom], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes": dom_bytes,
                "avg_launch_us": round(dom_us, 2)}
    phase_report = {}
    for p, d in per_phase.items():
        r = dict(d)
        r["avg_us"] = round(r["avg_us"], 2)
        if phase_bytes.get(p):
            r["algorithmic_bytes"] = phase_bytes[p]
            r["gbps"] = round(phase_bytes[p] / (d["avg_us"] * 1e-6) / 1e9, 1)
            r["frac_of_hbm_peak"] = round(r["gbps"] / HBM_PEAK_GBS, 4)
        phase_report[p] = r
    products_long = int(rf_s[long_rows].sum())
    if "sym_long" in per_phase:
        phase_report["sym_long"]["products_per_s"] = round(
            products_long / (per_phase["sym_long"]["avg_us"] * 1e-6), 1)
        phase_report["sym_long"]["rows"] = int(long_rows.sum())

    result = {
        "metric": "predicted rows/s (sampled-CR SpGEMM structure prediction)",
        "value": round(M / (ms_per_step * 1e-3), 1),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": w.name, "rows": M, "cols": B.ncols, "nnz_A": nnzA,
                   "nnz_B": B.nnz, "sample_rate": w.rate, "seed": w.seed,
                   "sampler": "bernoulli-splitmix64"},
        "hbm_gbps_algorithmic": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "nnz_A_per_s": round(nnzA / (ms_per_step * 1e-3), 1),
        "step_algorithmic_bytes": step_bytes,
        "roofline": roofline,
        "phases": phase_report,
        "phase_timing": {"steps": args.steps, "ms_per_step_with_phase_events":
                         round(ms_per_step_timed, 4)},
        "call_ms": call_ms,
        "stats": stats,
        "kernel_source_hash": src_hash,
        "generate_s": round(t_gen, 2),
    }

    if extras:
        # reference design and exact structure on the same input
        ref_out = torch.empty(M, dtype=torch.int64, device=dev)
        ref_st = torch.zeros(8, dtype=torch.int64, device=dev)
        ex_out = torch.empty(M, dtype=torch.int64, device=dev)
        ex_st = torch.zeros(8, dtype=torch.int64, device=dev)
        for fn in ("ref", "exact"):
            reps = 5
            for i in range(reps + 1):
                if i == 1:
                    torch.cuda.synchronize()
                    ta = time.perf_counter()
                if fn == "ref":
                    ssp.reference_estimate(Ad, Bd, w.rate, w.seed, handle=h, out=ref_out,
                                           stats=ref_st)
                else:
                    ssp.exact_structure(Ad, Bd, handle=h, out=ex_out, stats=ex_st)
            torch.cuda.synchronize()
            result[f"{fn}_ms"] = round((time.perf_counter() - ta) * 1e3 / reps, 4)
        Z = ssp.read_stats(ex_st)["out_sum"]
        F = stats["total_flop"]
        z1 = stats["sample_nnz"] * M / n_s if n_s else None
        fstar = f_s * M / n_s if n_s else None
        z2 = F * stats["sample_nnz"] / f_s if f_s else None
        exact_np = ex_out.cpu().numpy()
        pred_np = out.cpu().numpy()
        nz = exact_np > 0
        result["accuracy"] = {
            "Z": Z, "F": F, "CR": round(F / Z, 4) if Z else None,
            "eps1": (z1 / Z - 1) if (Z and z1 is not None) else None,
            "epsf": (fstar / F - 1) if (F and fstar is not None) else None,
            "eps2": (z2 / Z - 1) if (Z and z2 is not None) else None,
            "eps2_alloc": stats["out_sum"] / Z - 1 if Z else None,
            "rows_under_predicted": int(np.sum(pred_np < exact_np)),
            "mean_abs_row_rel_err": float(np.mean(np.abs(pred_np[nz] - exact_np[nz]) /
                                                  exact_np[nz])) if nz.any() else None,
        }
        result["predict_vs_exact_time"] = round(ms_per_step / result["exact_ms"], 4)
        # the existing estimator of related work (Sec. III): k minimum values, p = 1/10
        ssp.kmv_estimate(Ad, Bd, 0.1, 1024, w.seed, handle=h)
        torch.cuda.synchronize()
        tk = time.perf_counter()
        for _ in range(3):
            kmv = ssp.kmv_estimate(Ad, Bd, 0.1, 1024, w.seed, handle=h)
        result["kmv_ms"] = round((time.perf_counter() - tk) * 1e3 / 3, 4)
        result["accuracy"]["eps_kmv_p10_k1024"] = (kmv["nnz_estimate"] / Z - 1) if Z and \
            kmv["nnz_estimate"] is not None else None

    if cpu:
        import oracle
        cores = 1
        oracle.predict(A, B, w.rate, w.seed)  # warm-up (page-in)
        runs, tc0 = 0, time.perf_counter()
        while True:
            oracle.predict(A, B, w.rate, w.seed)
            runs += 1
            if time.perf_counter() - tc0 >= args.cpu_budget_s or runs >= 10:
                break
        t_cpu = (time.perf_counter() - tc0) / runs
        cpu_model = ""
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        result["cpu_baseline"] = {
            "value": round(M / t_cpu, 1), "unit": "rows/s", "cores": cores, "kind": "oracle",
            "sample": f"the whole {w.name} prediction (all {M} rows), serial C oracle, "
                      f"1 warm-up + {runs} timed runs, {t_cpu:.2f} s each",
            "host_cpu": cpu_model, "host_nproc": os.cpu_count()}
    return result


# The other configurations measured beside the headline R-MAT line: the
# uniform 4096^2 product (1%), the 27-point stencil 128^3 squared and the
# stencil times a 2,097,152 x 65,536 uniform B (0.5%).
OTHER_CONFIGS = ("uniform4096", "stencil128", "stencil128_x_uniform")
CONFIG_KEYS = ("value", "unit", "ms_per_step", "config", "hbm_gbps_algorithmic", "nnz_A_per_s",
               "step_algorithmic_bytes", "roofline", "phases", "call_ms", "stats")


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only: bench.py --gpus 1 "
                                   "(the multi-GPU sharding is a design note, not built)"}))
        sys.exit(2)

    if args.workload == "sweep":
        main_sweep(args)
        return
    if args.workload == "serve":
        main_serve(args)
        return
    if args.workload == "accuracy":
        main_accuracy(args)
        return
    if args.workload in ("spgemm", "spgemm_rmat18"):
        main_spgemm(args)
        return

    import torch
    import paper_2207_13848_amd as ssp

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    progress(f"workload {args.workload}")
    result = measure(ssp, get_workload(args.workload), args, extras=not args.no_extras,
                     cpu=not args.no_cpu_baseline)
    if not args.no_extras and args.workload == "rmat20":
        # every other configuration of the benchmark, each with its roofline
        result["configs"] = {}
        for name in OTHER_CONFIGS:
            progress(f"workload {name}")
            r = measure(ssp, get_workload(name), args, extras=False, cpu=False)
            result["configs"][r["config"]["workload"]] = {k: r[k] for k in CONFIG_KEYS}
            torch.cuda.empty_cache()
        # the 625-case sweep: plain vs batched vs graph, accuracy against the
        # exact structure
        import workloads
        progress("625-case sweep")
        result["sweep"] = sweep_compare(ssp, workloads.sweep_cases(), accuracy=True)
        torch.cuda.empty_cache()
        # serving: Poisson arrivals at 2000/s with continuous batching
        progress("serving")
        result["serve"] = serve_run(ssp)
    progress("done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
