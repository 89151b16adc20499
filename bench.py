#!/usr/bin/env python3
"""Benchmark: Gkeys/s into a Count Sketch over p = 2^61-1 (4-universal, two-for-one).

Default workload (the headline): a single stream of n = 2^28 uint64 keys drawn
Zipf(1.1) over [2^32], int32 weights uniform in [-100, 100], t = 9 rows x
m = 2^16 int64 counters, one degree-3 polynomial per row, two-for-one split
(sign = bit 0, bucket = bits 1..16).  Inputs are synthetic, generated on the
GPU and resident in HBM before timing.

One step = reset the counters (Initialize) + cs_update over the whole batch
(Process) + cs_estimate_f2 (Output: per-row sums of squares and the median).
The update's kernels are timed with HIP events on the stream they run on.

Other workloads (--workload) measure the other kernels the same way:
  single_stream_zipf_two_poly  two independent polynomials per row (bucket, sign)
  small_table_u32              t=5, m=2^10 (table in LDS), uint32 uniform keys, int64 weights = 1
  p89_uniform                  p = 2^89-1, t=5, m=2^20, 2^26 uint64 uniform keys, int64 weights = 1
  divmod_p61 / divmod_p89 / divmod_p64_59   2^28 values uniform in [0, p^2)
  batched                      4096 sketches (t=5, m=2^e, e uniform in 8..16, seeds 4000+i), stream
                               lengths floor(2^U(8,22)), uint64 Zipf(1.1) keys, int32 weights in
                               [-100,100]: one batched update (autotuned, HIP graph) vs 4096 cs_update
Prints one JSON line.  --gpus N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ALU peak, from the unit counts: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.64 T lane-slots/s
# (the fp32 vector peak of 157.3 TFLOP/s is this many fused multiply-adds).  Measured by
# `bench.py --workload ceilings` (profiles/ceilings.md): a SIMD issues one wave64 VALU
# instruction per slot, 64 lane-operations where the peak counts 128; only the simple
# two-operand 32-bit operations (add, sub, and, xor, mov) issue two per slot, from two
# waves.  So an instruction costs 2 lane-slots (64-bit v_mad_u64_u32, v_lshl_add_u64,
# v_lshrrev_b64, and 32-bit shifts, bit-field extracts, three-input and carry
# instructions alike: 36.9-37.8 T lane-instructions/s each) and a simple one 1 (69.6 T).
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12  # 78.64 T lane-slots/s
HBM_PEAK_GBS = 8000.0
METRIC = "Gkeys/s into Count Sketch (p=2^61-1, 4-universal) + % of binding roofline"

# Algorithmic VALU lane-slots per key and row: the VALU instructions (register moves not
# counted, so a lower bound) of the compiled straight-line hash + final reduction +
# split of one row on gfx950, as the update kernels run it (the Horner steps before the
# last fold at bit 64, the last step unfolded; the rare carry and guard paths left out),
# each weighted by its measured issue cost (2, or 1 for the simple ones), plus 3 per row
# for the signed weight (v_xad_u32, 2) and the counter address (v_and_b32, 1)
# (profiles/valu_ops_per_key_row.md):
#   p61, key < 2^32, two-for-one: 11 64-bit + 4 other + 1 simple = 31, + 3 = 34
#   p61 two polynomials: 20 64-bit + 7 other + 3 simple = 57, + 3 = 60
#   p61 any bucket count (Algorithm 8): 16 64-bit + 4 other + 1 simple = 41, + 3 = 44
#   p89, 64-bit keys, two-for-one: 35 64-bit + 13 other + 3 simple = 99, + 3 = 102
OPS_PER_KEY_ROW = {("p61", 0): 34, ("p61", 2): 60, ("p89", 0): 102, ("p61", 3): 44}
OPS_PER_KEY = 3  # the key's high-word test (domain check, one-limb path) and load addressing

SKETCH_WORKLOADS = {
    "single_stream_zipf": dict(n=1 << 28, rows=9, log2m=16, mode=0, prime="p61", keys="zipf", kbytes=8, wbytes=4,
                               seed=1002, desc="single stream, 2^28 uint64 keys Zipf(1.1) over [2^32], int32 "
                                               "weights in [-100,100], p=2^61-1, t=9, m=2^16, two-for-one"),
    "single_stream_zipf_two_poly": dict(n=1 << 28, rows=9, log2m=16, mode=2, prime="p61", keys="zipf", kbytes=8,
                                        wbytes=4, seed=1002, desc="as single_stream_zipf with two independent "
                                                                  "polynomials per row (bucket, sign)"),
    "small_table_u32": dict(n=1 << 28, rows=5, log2m=10, mode=0, prime="p61", keys="u32", kbytes=4, wbytes=8,
                            seed=1001, desc="2^28 uint32 keys uniform, int64 weights = 1, p=2^61-1, t=5, m=2^10 "
                                            "(table in LDS), two-for-one"),
    "single_stream_zipf_arb_r": dict(n=1 << 28, rows=9, log2m=16, buckets=50000, mode=3, prime="p61", keys="zipf",
                                     kbytes=8, wbytes=4, seed=1002,
                                     desc="as single_stream_zipf with r = 50000 buckets per row (Algorithm 8, any "
                                          "bucket count; rows padded to 2^16)"),
    "small_table_u32_two_poly": dict(n=1 << 28, rows=5, log2m=10, mode=2, prime="p61", keys="u32", kbytes=4,
                                     wbytes=8, seed=1001, desc="as small_table_u32 with two independent polynomials "
                                                               "per row (bucket, sign): the hashing-bound comparison"),
    "p89_uniform": dict(n=1 << 26, rows=5, log2m=20, mode=0, prime="p89", keys="u64", kbytes=8, wbytes=8,
                        seed=1003, desc="2^26 uint64 keys uniform, int64 weights = 1, p=2^89-1, t=5, m=2^20, "
                                        "two-for-one"),
}
MAP_WORKLOADS = {
    "bucket_map_p61": dict(prime=1, p=(1 << 61) - 1, limbs=1, n=1 << 28, r=1000003),
    "bucket_map_p89": dict(prime=2, p=(1 << 89) - 1, limbs=2, n=1 << 28, r=1000003),
    "bucket_map_p64_59": dict(prime=3, p=(1 << 64) - 59, limbs=1, n=1 << 28, r=1000003),
}
DIVMOD_WORKLOADS = {
    "divmod_p61": dict(prime=1, p=(1 << 61) - 1, limbs=2, qlimbs=1, n=1 << 28),
    "divmod_p89": dict(prime=2, p=(1 << 89) - 1, limbs=3, qlimbs=2, n=1 << 28),
    "divmod_p64_59": dict(prime=3, p=(1 << 64) - 59, limbs=2, qlimbs=1, n=1 << 28),
}


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "hbm_traffic.json")
# The measured HBM traffic stands only for the kernels it was measured on.
KERNEL_SOURCES = sorted("paper_2008_08654_amd/csrc/" + f for f in os.listdir(os.path.join(HERE, "paper_2008_08654_amd",
                                                                                           "csrc"))
                        if f.endswith((".hip", ".hpp")) or f == "mcs_host.cpp")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, n: int):
    """HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter runs (copy-calibrated),
    or None when there is no measurement for this workload and size, or the kernel sources
    changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = t.get("workloads", {}).get(workload)
    if entry is None or entry.get("n") != n or entry.get("sources_sha256") != kernel_sources_sha256():
        return None
    return entry.get("hbm_bytes_per_launch")


# Library kernels that are not part of the measured launch (the step's reset and estimate).
TRAFFIC_EXCLUDE = ("k_estimate", "k_fill_zero")


def summarize_traffic(args):
    """Turns the two counter runs of a workload (FETCH_SIZE, then WRITE_SIZE, each with
    --calib-copy) into HBM bytes per launch of its library kernels, calibrated on the 1 GiB
    copy, and records them with the hash of the kernel sources in profiles/hbm_traffic.json
    and profiles/hbm_traffic.md.  The runs are `bench.py --workload W --steps S --warmup U
    --no-cpu-baseline --no-naive --calib-copy` under rocprofv3 --pmc; pass the same W, S, U."""
    import csv
    import glob

    def per_dispatch(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            sys.exit(f"bench.py: no counter_collection.csv under {d}")
        out = {}
        for f in files:
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] != counter:
                        continue
                    e = out.setdefault((f, int(r["Dispatch_Id"])), [r["Kernel_Name"], 0.0])
                    e[1] += float(r["Counter_Value"])
        return list(out.values())

    launches = args.steps + args.warmup
    res = {}
    for counter, d in (("FETCH_SIZE", args.traffic_summary[0]), ("WRITE_SIZE", args.traffic_summary[1])):
        rows = per_dispatch(d, counter)
        copies = [v for name, v in rows if "copyBuffer" in name]
        if not copies:
            sys.exit(f"bench.py: no copy dispatch in the {counter} run (was it made with --calib-copy?)")
        factor = (1 << 30) / (max(copies) * 1024.0)
        mine = [(name, v) for name, v in rows if "mcs::" in name and not any(x in name for x in TRAFFIC_EXCLUDE)]
        kernels = sorted({name.split("<")[0].split("(")[0].replace("void ", "") for name, _ in mine})
        res[counter] = (factor, sum(v for _, v in mine) * 1024.0 * factor / launches, kernels)
    wl = args.workload
    if wl in SKETCH_WORKLOADS:
        w = SKETCH_WORKLOADS[wl]
        n = args.n or w["n"]
        algo = n * (w["kbytes"] + w["wbytes"])  # keys and weights, read once
    else:
        w = DIVMOD_WORKLOADS[wl]
        n = args.n or w["n"]
        algo = n * 8 * (w["limbs"] + w["qlimbs"] + w["limbs"] - 1)  # x in; quotient and remainder out
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    t.pop("sources_sha256", None)
    t.setdefault("workloads", {})[wl] = {
        "launch": " + ".join(res["FETCH_SIZE"][2]), "n": n,
        "fetch_bytes_per_launch": int(res["FETCH_SIZE"][1]), "write_bytes_per_launch": int(res["WRITE_SIZE"][1]),
        "hbm_bytes_per_launch": int(res["FETCH_SIZE"][1] + res["WRITE_SIZE"][1]),
        "algorithmic_bytes_per_launch": algo,
        "ratio": round((res["FETCH_SIZE"][1] + res["WRITE_SIZE"][1]) / algo, 3),
        "fetch_factor": round(res["FETCH_SIZE"][0], 5), "write_factor": round(res["WRITE_SIZE"][0], 5),
        "sources_sha256": kernel_sources_sha256()}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
    lines = ["# HBM traffic per launch — FETCH_SIZE and WRITE_SIZE, copy-calibrated", "",
             "Each counter in a run of its own (from the repository root, one MI355X), then the summary:", "",
             "```",
             "rocprofv3 --pmc FETCH_SIZE --output-format csv -d /tmp/pmc_<workload>_FETCH_SIZE -o run -- \\",
             "    python3 bench.py --workload <workload> --steps 2 --warmup 1 --no-cpu-baseline --no-naive --calib-copy",
             "rocprofv3 --pmc WRITE_SIZE --output-format csv -d /tmp/pmc_<workload>_WRITE_SIZE -o run -- \\",
             "    python3 bench.py --workload <workload> --steps 2 --warmup 1 --no-cpu-baseline --no-naive --calib-copy",
             "python3 bench.py --workload <workload> --steps 2 --warmup 1 \\",
             "    --traffic-summary /tmp/pmc_<workload>_FETCH_SIZE /tmp/pmc_<workload>_WRITE_SIZE",
             "```", "",
             "`--calib-copy` first copies 1 GiB device to device (`__amd_rocclr_copyBuffer`, 2^30 bytes read",
             "and 2^30 written); each factor is known bytes / (counter KiB x 1024) of that dispatch. The bytes",
             "are those of the library's kernels in the run (not the step's reset and estimate) per launch.",
             "A row stands for the kernel sources it was taken on (sha256 over the kernel sources, as",
             "bench.py computes it); bench.py reports `traffic` only while that hash matches.", "",
             "| Workload | Kernels | Fetch bytes | Write bytes | HBM bytes | Algorithmic bytes | HBM / algorithmic "
             "| Factors (fetch, write) | Sources sha256 |",
             "|---|---|---|---|---|---|---|---|---|"]
    for name, e in t["workloads"].items():
        lines.append(f"| {name} | {e['launch']} | {e['fetch_bytes_per_launch']:.4g} | {e['write_bytes_per_launch']:.4g} "
                     f"| {e['hbm_bytes_per_launch']:.4g} | {e['algorithmic_bytes_per_launch']:.4g} | {e['ratio']} "
                     f"| {e.get('fetch_factor', '-')}, {e.get('write_factor', '-')} "
                     f"| `{e.get('sources_sha256', 'earlier sources')[:16]}` |")
    with open(os.path.join(HERE, "profiles", "hbm_traffic.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return t["workloads"][wl]


def update_kernels(sk, n, path=0) -> str:
    """The dispatches one cs_update of n keys makes on the automatic (or forced) path."""
    chunks = -(-n // (1 << 27))
    pitch = 1 << (sk.buckets - 1).bit_length()
    if path in (0, 1) and sk.rows * pitch * 8 <= 65536:
        return "1 x k_update_lds"
    if path in (0, 5) and pitch <= 1 << 16:
        return "1 x k_update_rows"
    return f"{chunks} x (k_bin_wave or k_bin) + {chunks} x k_accumulate (rounds of 2^27 keys)"


def _stream_ptr(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def cpu_baseline_sketch(keys_dev, w_dev, wl, budget_s=15.0):
    """Times the oracle (the plain CPU implementation, as it stands) on a bounded
    prefix of the same stream, one thread per row.  Returns the baseline record,
    the oracle's table for that prefix and the prefix length."""
    import numpy as np
    import oracle as O
    rows, m, mode = wl["rows"], wl.get("buckets", 1 << wl["log2m"]), wl["mode"]
    prime = O.PRIME_P61 if wl["prime"] == "p61" else O.PRIME_P89
    threads = min(rows, os.cpu_count() or 1)
    coeffs = O.coeffs_from_seed(prime, rows, mode, wl["seed"])

    def host(t, n):
        a = t[:n].cpu().numpy()
        return a.view(np.uint32).astype(np.uint64) if a.dtype == np.int32 else a.view(np.uint64)

    n_probe, dt = 1 << 14, 0.0
    while True:  # grow the probe until it takes a second, then scale to the budget
        kp, wp = host(keys_dev, n_probe), w_dev[:n_probe].cpu().numpy().astype(np.int64)
        t0 = time.perf_counter()
        O.cs_update(prime, mode, rows, m, coeffs, kp, wp)
        dt = time.perf_counter() - t0
        if dt > 1.0 or n_probe >= keys_dev.numel():
            break
        n_probe = min(keys_dev.numel(), n_probe * 4)
    n = int(min(keys_dev.numel(), max(n_probe, n_probe * budget_s / max(dt, 1e-6))))
    k = host(keys_dev, n)
    w = w_dev[:n].cpu().numpy().astype(np.int64)
    t0 = time.perf_counter()
    table = O.cs_update(prime, mode, rows, m, coeffs, k, w)
    dt = time.perf_counter() - t0
    rec = {"value": round(n / dt / 1e9, 6), "unit": "Gkeys/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n} keys of the same stream, same sketch; {dt:.1f} s; one thread per row"}
    return rec, table, n


def sketch_parity(sk, table, n_checked, n_total):
    """Bit-exact comparison of the sketch's counters, row estimates and median with the
    oracle's table (every counter, every row value)."""
    import numpy as np
    import oracle as O
    got = sk.counters()
    st, f2, rows = sk.estimate_f2_status()
    wst, wmed, wrows = O.cs_estimate_status(table)
    diff = int((got != table).sum())
    ok = diff == 0 and list(rows) == list(wrows) and f2 == wmed and (st == 0) == (wst == 0)
    what = "all" if n_checked == n_total else f"the first {n_checked} of the"
    return {"status": "bit-exact" if ok else "MISMATCH",
            "checked": f"counters ({table.size}), {len(wrows)} row estimates and the median over {what} "
                       f"{n_total} keys against the oracle",
            "counters_differing": diff}


def run_sketch(args, wl):
    import torch
    import paper_2008_08654_amd as M
    import workloads as W

    n = args.n or wl["n"]
    rows, m, mode = wl["rows"], wl.get("buckets", 1 << wl["log2m"]), wl["mode"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    if wl["keys"] == "zipf":
        keys, w = W.stream_zipf_u64(n, device=dev)
    elif wl["keys"] == "u32":
        keys, w = W.stream_small_u32(n, device=dev)
        keys = keys.to(torch.int32)
    else:
        keys, w = W.stream_uniform_u64(n, device=dev)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen

    prime = M.CS_P61 if wl["prime"] == "p61" else M.CS_P89
    sk = M.Sketch(rows, m, prime=prime, seed=wl["seed"], mode=mode)
    if args.path:
        sk.set_update_path(args.path)
    sk.reserve(n)  # one workspace for the largest rounds (two-pass path only), outside the timed steps
    L = M.lib()
    stream = _stream_ptr(torch)
    kp, wp = ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(w.data_ptr())
    kt = M.CS_U32 if wl["kbytes"] == 4 else M.CS_U64
    wt = M.CS_I32 if wl["wbytes"] == 4 else M.CS_I64
    f2 = ctypes.c_int64()

    def step(ev=None):
        M._check(L.cs_reset(sk.handle, stream))
        if ev is not None:
            ev[0].record()
        M._check(L.cs_update(sk.handle, kp, kt, wp, wt, n, stream))
        if ev is not None:
            ev[1].record()
        st = L.cs_estimate_f2(sk.handle, ctypes.byref(f2), None, stream)
        if st not in (M.CS_OK, M.CS_EOVERFLOW):
            M._check(st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    upd_ms = [a.elapsed_time(b) for a, b in events]
    upd_avg_ms = sum(upd_ms) / len(upd_ms)

    ops_key = rows * OPS_PER_KEY_ROW[(wl["prime"], mode)] + OPS_PER_KEY
    achieved = ops_key * n / (upd_avg_ms * 1e-3) / 1e12
    bytes_key = wl["kbytes"] + wl["wbytes"]
    out = {"metric": METRIC if wl["prime"] == "p61" else METRIC.replace("2^61-1", "2^89-1"),
           "value": round(n * args.steps / elapsed / 1e9, 3), "unit": "Gkeys/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
           "data": "synthetic",
           "config": {"workload": args.workload, "description": wl["desc"], "keys": n, "rows": rows, "buckets": m,
                      "k": 4, "parallelism": "none (1 GPU)",
                      "update_only_gkeys_per_s": round(n / (upd_avg_ms * 1e-3) / 1e9, 3),
                      "input_generation_s": round(t_gen, 2)},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                        "unit": "T VALU lane-slots/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                        "traffic": measured_traffic(args.workload, n),
                        "algorithmic_bytes_per_launch": bytes_key * n,
                        "kernel": "cs_update", "kernel_avg_ms": round(upd_avg_ms, 4),
                        "kernels_per_launch": update_kernels(sk, n, args.path),
                        "algorithmic_ops_per_key": ops_key,
                        "hbm_frac_of_input_stream": round(bytes_key * n / (upd_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"], table, n_or = cpu_baseline_sketch(keys, w, wl)
        # Parity on the benchmark's own inputs: the timed steps reset the counters and
        # add the whole stream, so the table now holds one update of all n keys.  A
        # prefix-only oracle run is checked on a fresh sketch updated with that prefix.
        if n_or == n:
            out["parity"] = sketch_parity(sk, table, n_or, n)
        else:
            chk = M.Sketch(rows, m, prime=prime, seed=wl["seed"], mode=mode)
            M._check(L.cs_update(chk.handle, kp, kt, wp, wt, n_or, stream))
            out["parity"] = sketch_parity(chk, table, n_or, n)
            chk.close()
        del table
    else:
        out["parity"] = {"status": "not checked (--no-cpu-baseline)"}
    sk.close()
    return out


def _log(msg):
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def run_batched(args):
    import numpy as np
    import torch
    import paper_2008_08654_amd as M
    import workloads as W

    count = args.n or 4096
    dev = torch.device("cuda:0")
    seed = W.DATA_SEED + 4
    lens = W.loguniform_int(seed, count, 8.0, 22.0)
    log2m = W.bounded_int(seed, count, 8, 16, stream=6)
    total = int(lens.sum())
    offs = [0] + np.cumsum(lens.numpy()).tolist()
    t_gen = time.perf_counter()
    keys = torch.empty(total, dtype=torch.int64, device=dev)
    w = torch.empty(total, dtype=torch.int32, device=dev)
    step_gen = 1 << 27
    for o in range(0, total, step_gen):  # chunked generation bounds the temporaries
        nn = min(step_gen, total - o)
        kk, ww = W.stream_zipf_u64(nn, device=dev, seed=seed + 1 + o // step_gen)
        keys[o:o + nn] = kk
        w[o:o + nn] = ww
        del kk, ww
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    _log(f"batched: {count} members, {total} keys generated in {t_gen:.1f} s")
    sketches = [M.Sketch(5, 1 << int(log2m[i]), prime=M.CS_P61, seed=4000 + i) for i in range(count)]
    members = [(sketches[i], keys[offs[i]:offs[i + 1]], w[offs[i]:offs[i + 1]]) for i in range(count)]
    batch = M.Batch(members)
    stream = torch.cuda.current_stream()
    t_tune = time.perf_counter()
    chosen = batch.options() if args.no_autotune else batch.autotune(stream)
    t_tune = time.perf_counter() - t_tune
    _log(f"batched: autotuned in {t_tune:.1f} s -> lds_table_max {chosen.lds_table_max}, "
         f"chunk {chosen.lds_chunk_keys}, combine {chosen.combine}, direct {chosen.direct_fraction}, "
         f"keys/thread {chosen.keys_per_thread or 8}, row-resident {chosen.row_resident}")

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, sum(a.elapsed_time(b) for a, b in ev) / steps

    L = M.lib()
    sp = M._stream(None)
    handles = [(sk.handle, ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(ww.data_ptr()), k.numel())
               for sk, k, ww in members]

    def plain():
        for h, kp, wp, n in handles:
            if n:
                M._check(L.cs_update(h, kp, M.CS_U64, wp, M.CS_I32, n, sp))

    elapsed, batch_ms = timed(batch.update, args.steps)
    _log(f"batched: {args.steps} batched steps, {elapsed * 1e3 / args.steps:.2f} ms each")
    plain_elapsed, plain_ms = timed(plain, max(1, args.steps // 4))
    _log(f"batched: plain per-sketch launches, {plain_elapsed * 1e3 / max(1, args.steps // 4):.2f} ms per pass")
    plain_wall_ms = plain_elapsed * 1e3 / max(1, args.steps // 4)
    ops_key = 5 * OPS_PER_KEY_ROW[("p61", 0)] + OPS_PER_KEY
    achieved = ops_key * total / (batch_ms * 1e-3) / 1e12
    ng, nl, nr, nt = batch.classes()
    out = {"metric": "aggregate Gkeys/s into 4096 Count Sketches (p=2^61-1, 4-universal), one batched update",
           "value": round(total * args.steps / elapsed / 1e9, 3), "unit": "Gkeys/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "batched", "sketches": count, "keys": total, "rows": 5,
                      "buckets": "2^8..2^16 log-uniform", "classes": {"direct_atomics": ng, "lds": nl,
                                                                      "row_resident": nr, "two_pass": nt},
                      "autotuned": {"lds_table_max": chosen.lds_table_max, "lds_chunk_keys": chosen.lds_chunk_keys,
                                    "combine": chosen.combine, "direct_fraction": chosen.direct_fraction,
                                    "keys_per_thread": chosen.keys_per_thread or 8,
                                    "row_resident": chosen.row_resident},
                      "autotune_s": round(t_tune, 2),
                      "plain_launches_ms": round(plain_wall_ms, 3),
                      "plain_gkeys_per_s": round(total / (plain_wall_ms * 1e-3) / 1e9, 3),
                      "batched_vs_plain_speedup": round(plain_wall_ms / (elapsed * 1e3 / args.steps), 2),
                      "input_generation_s": round(t_gen, 2)},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                        "unit": "T VALU lane-slots/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                        "kernel": "batched update (all launches)", "kernel_avg_ms": round(batch_ms, 4),
                        "algorithmic_ops_per_key": ops_key}}
    if not args.no_cpu_baseline:
        import oracle as O
        # Parity on the benchmark's own inputs: the tables are cleared and take exactly one
        # batched update; every member the oracle sample reaches is then compared with the
        # oracle's table for its stream, counter by counter.
        for sk in sketches:
            sk.reset(stream)
        batch.update(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_or = 0.0
        done = 0
        i = 0
        bad_members, by_class = [], {}
        while t_or < 15.0 and i < count:
            sk, k, ww = members[i]
            c = O.coeffs_from_seed(O.PRIME_P61, 5, O.TWO_FOR_ONE, 4000 + i)
            kh, wh = k.cpu().numpy().view(np.uint64), ww.cpu().numpy().astype(np.int64)
            t1 = time.perf_counter()
            want = O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, 5, 1 << int(log2m[i]), c, kh, wh)
            t_or += time.perf_counter() - t1
            done += k.numel()
            if not np.array_equal(sk.counters(), want):
                bad_members.append(i)
            i += 1
        _log(f"batched: oracle sample of {i} members done, {len(bad_members)} differ")
        out["cpu_baseline"] = {"value": round(done / t_or / 1e9, 6), "unit": "Gkeys/s", "cores": 5,
                               "kind": "oracle",
                               "sample": f"first {i} members ({done} keys), {t_or:.1f} s, one thread per row"}
        out["parity"] = {"status": "bit-exact" if not bad_members else "MISMATCH",
                         "checked": f"every counter of the first {i} of {count} members ({done} of {total} keys) "
                                    f"after one batched update, against the oracle",
                         "members_differing": bad_members[:16]}
    else:
        out["parity"] = {"status": "not checked (--no-cpu-baseline)"}
    for sk in sketches:
        sk.close()
    batch.close()
    return out


def run_served(args):
    import numpy as np
    import torch
    import paper_2008_08654_amd as M
    import workloads as W

    dev = torch.device("cuda:0")
    seed = W.DATA_SEED + 5
    n_tenants, rows = 1024, 7
    log2m = W.served_tenants(n_tenants, seed).tolist()
    pool_n = 1 << 27
    t_gen = time.perf_counter()
    keys = torch.empty(pool_n, dtype=torch.int64, device=dev)
    w = torch.empty(pool_n, dtype=torch.int32, device=dev)
    step_gen = 1 << 25
    for o in range(0, pool_n, step_gen):  # chunked generation bounds the temporaries
        keys[o:o + step_gen] = W.zipf(seed + 1 + o // step_gen, step_gen, 1.2, 1 << 32, device=dev)
        w[o:o + step_gen] = W.bounded_int(seed + 1 + o // step_gen, step_gen, -100, 100, device=dev).to(torch.int32)
    torch.cuda.synchronize()
    srv = M.Server(direct_fraction=args.direct_fraction)
    ids = [srv.admit(rows, 1 << e, 5000 + i) for i, e in enumerate(log2m)]
    n_req = args.n or 100000
    tenant, is_f2, size = W.served_requests(n_req, n_tenants, seed)
    offs = W.bounded_int(seed, n_req, 0, pool_n - (1 << 20), stream=11).tolist()
    reqs = []
    for t, f, n, o in zip(tenant.tolist(), is_f2.tolist(), size.tolist(), offs):
        reqs.append((ids[t], M.CS_REQ_F2, None, None) if f else
                    (ids[t], M.CS_REQ_UPDATE, keys[o:o + n], w[o:o + n]))
    total_keys = int(size.sum())
    _log(f"served: {n_tenants} tenants admitted, {n_req} requests ({total_keys} keys) in "
         f"{time.perf_counter() - t_gen:.1f} s")
    # The arrival schedules at unit rate, made before any replay (scaled below by the
    # measured rate): torch's CPU threads keep spinning for a while after an op, and in a
    # replay that starts right after one they took the CPU quota from the server's worker
    # thread (its first step then formed 5-8 ms late).
    unit_arrivals = [W.poisson_arrivals(n_req, 1.0, seed=seed, stream=20 + i).numpy() for i in range(3)]
    srv.replay(reqs[: n_req // 20], np.zeros(n_req // 20))  # warm-up
    # the trace is marshalled once, outside the timed replays
    trace = srv.prepare(reqs)
    t0 = time.perf_counter()
    res = srv.replay(trace, np.zeros(n_req))
    sat_s = time.perf_counter() - t0
    bad = sum(1 for r in res if r.status != M.CS_OK)
    sat_rate = n_req / sat_s
    _log(f"served: saturated {sat_rate:.0f} requests/s, {total_keys / sat_s / 1e9:.2f} Gkeys/s")

    def lat_stats(res):
        lat = np.array([r.done_ns - r.arrival_ns for r in res], dtype=np.float64) / 1e6
        span = (max(r.done_ns for r in res) - min(r.arrival_ns for r in res)) / 1e9
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "gkeys_per_s": round(total_keys / span / 1e9, 3)}

    loads = []
    for i, frac in enumerate((0.3, 0.6, 0.9)):
        arr = unit_arrivals[i] / (frac * sat_rate)
        r = srv.replay(trace, arr)
        bad += sum(1 for x in r if x.status != M.CS_OK)
        st = lat_stats(r)
        st.update({"load": frac, "requests_per_s": round(frac * sat_rate, 1)})
        loads.append(st)
        _log(f"served: load {frac}: p50 {st['p50_ms']} ms, p99 {st['p99_ms']} ms")
    stats = srv.stats()
    ops_key = rows * OPS_PER_KEY_ROW[("p61", 0)] + OPS_PER_KEY
    achieved = ops_key * total_keys / sat_s / 1e12
    out = {"metric": "served Count Sketch updates: saturated Gkeys/s over 1024 tenants, p50/p99 latency at 0.3/0.6/0.9 load",
           "value": round(total_keys / sat_s / 1e9, 3), "unit": "Gkeys/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": round(sat_s * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int64", "data": "synthetic",
           "config": {"workload": "served", "tenants": n_tenants, "rows": rows, "buckets": "2^12..2^18 uniform exponent",
                      "requests": n_req, "keys": total_keys, "f2_fraction": round(float(is_f2.float().mean()), 4),
                      "update_keys": "floor(2^U(10,20)), Zipf(1.2) over [2^32], int32 weights in [-100,100]",
                      "saturated_requests_per_s": round(sat_rate, 1), "direct_fraction": args.direct_fraction or "default",
                      "saturated_latency_p50_ms": lat_stats(res)["p50_ms"], "loads": loads,
                      "steps_run": stats.steps, "resident_bytes": stats.resident_bytes, "failed_requests": bad},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                        "unit": "T VALU lane-slots/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                        "kernel": "served steps (all launches, closed loop)", "algorithmic_ops_per_key": ops_key}}
    if not args.no_cpu_baseline:
        import oracle as O
        # Parity on the benchmark's own inputs: the warm-up replay ran the first n_req / 20
        # requests and four replays ran all of them, so a tenant's counters must equal the
        # oracle's table of its updates in the prefix plus four times that of all its updates.
        upd_of = {}
        for i, (t, f) in enumerate(zip(tenant.tolist(), is_f2.tolist())):
            if not f and int(size[i]):
                upd_of.setdefault(t, []).append(i)
        sample = sorted(upd_of)[:: max(1, len(upd_of) // 8)][:8]
        bad_tenants = []
        checked_keys = 0
        for t in sample:
            c = O.coeffs_from_seed(O.PRIME_P61, rows, O.TWO_FOR_ONE, 5000 + t)
            m_t = 1 << log2m[t]
            prefix = np.zeros((rows, m_t), dtype=np.int64)
            full = np.zeros((rows, m_t), dtype=np.int64)
            for i in upd_of[t]:
                n_i, o_i = int(size[i]), offs[i]
                kh, wh = W.as_uint64_numpy(keys[o_i:o_i + n_i]), w[o_i:o_i + n_i].cpu().numpy().astype(np.int64)
                O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, rows, m_t, c, kh, wh, table=full)
                if i < n_req // 20:
                    O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, rows, m_t, c, kh, wh, table=prefix)
                checked_keys += n_i
            if not np.array_equal(srv.counters(ids[t], rows, m_t), prefix + 4 * full):
                bad_tenants.append(t)
        out["parity"] = {"status": "bit-exact" if not bad_tenants and not bad else "MISMATCH",
                         "checked": f"every counter of tenants {sample} ({checked_keys} update keys per replay) "
                                    f"after all replays, against the oracle; failed requests: {bad}",
                         "tenants_differing": bad_tenants}
        _log(f"served: parity over {len(sample)} tenants: {out['parity']['status']}")
        coeffs = {}
        t0 = time.perf_counter()
        done = 0
        i = 0
        while time.perf_counter() - t0 < 15.0 and i < n_req:
            t, f, n, o = int(tenant[i]), int(is_f2[i]), int(size[i]), offs[i]
            if not f and n:
                if t not in coeffs:
                    coeffs[t] = (O.coeffs_from_seed(O.PRIME_P61, rows, O.TWO_FOR_ONE, 5000 + t),
                                 np.zeros((rows, 1 << log2m[t]), dtype=np.int64))
                c, table = coeffs[t]
                O.cs_update(O.PRIME_P61, O.TWO_FOR_ONE, rows, 1 << log2m[t], c, W.as_uint64_numpy(keys[o:o + n]),
                            w[o:o + n].cpu().numpy().astype(np.int64), table=table)
                done += n
            i += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(done / dt / 1e9, 6), "unit": "Gkeys/s", "cores": rows, "kind": "oracle",
                               "sample": f"first {i} requests ({done} keys), {dt:.1f} s, one thread per row"}
    else:
        out["parity"] = {"status": "not checked (--no-cpu-baseline)"}
    srv.close()
    return out


def run_bucket_map(args, wl):
    """Most uniform maps of 2^28 hash values uniform in [p] to r = 1000003 buckets: the exact
    floor(v r / p) (Algorithms 4 or 5-6 on the product) and, for Mersenne primes, ((v+1) r) >> b."""
    import numpy as np
    import torch
    import paper_2008_08654_amd as M
    import workloads as W

    n = args.n or wl["n"]
    dev = torch.device("cuda:0")
    v = W.below_limbs(wl["p"], wl["limbs"], 0x2008086544, n, device=dev)
    v = v.reshape(-1) if wl["limbs"] == 1 else v.contiguous()
    out = torch.empty(n, dtype=torch.int32, device=dev)

    def timed(method):
        for _ in range(args.warmup):
            M.mersenne_bucket_map(wl["prime"], v, wl["r"], out, method=method)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        t0 = time.perf_counter()
        for a, b in ev:
            a.record()
            M.mersenne_bucket_map(wl["prime"], v, wl["r"], out, method=method)
            b.record()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, sum(a.elapsed_time(b) for a, b in ev) / len(ev)

    elapsed, k_ms = timed(M.CS_MAP_EXACT)
    M.mersenne_status()
    fast_ms = None
    if wl["prime"] != M.CS_P64_59:
        _, fast_ms = timed(M.CS_MAP_MERSENNE)
        M.mersenne_status()
    bytes_per = 8 * wl["limbs"] + 4
    gbs = bytes_per * n / (k_ms * 1e-3) / 1e9
    out_d = {"metric": "G values/s most uniform map of hash values to r buckets (exact floor(v r / p)) + % of HBM roofline",
             "value": round(n * args.steps / elapsed / 1e9, 3), "unit": "Gvalues/s", "n_gpus": 1,
             "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
             "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
             "config": {"workload": args.workload, "values": n, "r": wl["r"], "limbs_in": wl["limbs"],
                        "mersenne_map_kernel_ms": None if fast_ms is None else round(fast_ms, 4)},
             "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.workload, n),
                          "algorithmic_bytes_per_launch": bytes_per * n, "kernel": "k_bucket_map",
                          "kernel_avg_ms": round(k_ms, 4), "algorithmic_bytes_per_value": bytes_per}}
    if not args.no_cpu_baseline:
        import oracle as O
        nn = 1 << 22
        vh = v[:nn].cpu().numpy().view(np.uint64)
        t0 = time.perf_counter()
        O.bucket_map_exact(wl["p"], vh, wl["r"])
        dt = time.perf_counter() - t0
        out_d["cpu_baseline"] = {"value": round(nn / dt / 1e9, 6), "unit": "Gvalues/s", "cores": 1, "kind": "oracle",
                                 "sample": f"first {nn} values, {dt:.2f} s, one thread"}
    return out_d


def run_divmod_bsweep(args):
    """The paper's division experiment on the GPU: 10^7 divisions of uniform 2b-bit numbers
    by p = 2^b - 1 for b = 32 .. 1024, Algorithm 5 (+ 6) against the Crandall-Chung-Hasan
    algorithm (Algorithm 10); limb-plane layout."""
    import numpy as np
    import torch
    import paper_2008_08654_amd as M
    import workloads as W

    n = args.n or 10 ** 7
    dev = torch.device("cuda:0")
    sweep = {}
    for b in (32, 64, 128, 256, 512, 1024):
        w = b // 32
        x = W.uniform_u32(0x2008086545 + b, 2 * w * n, device=dev).to(torch.int32).reshape(2 * w, n)
        q = torch.empty((w + 1, n), dtype=torch.int32, device=dev)
        r = torch.empty((w, n), dtype=torch.int32, device=dev)
        res = {}
        for name, method in (("alg5", M.CS_WIDE_ALG5), ("cch", M.CS_WIDE_CCH)):
            for _ in range(args.warmup):
                M.mersenne_divmod_wide(b, 1, x, q, r, method=method)
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
            for a, e in ev:
                a.record()
                M.mersenne_divmod_wide(b, 1, x, q, r, method=method)
                e.record()
            torch.cuda.synchronize()
            res[name] = sum(a.elapsed_time(e) for a, e in ev) / len(ev)
        bytes_per = 4 * (2 * w + (w + 1) + w)
        sweep[b] = {"alg5_ms_per_1e7": round(res["alg5"] * 1e7 / n, 4), "cch_ms_per_1e7": round(res["cch"] * 1e7 / n, 4),
                    "cch_over_alg5": round(res["cch"] / res["alg5"], 2),
                    "alg5_gb_per_s": round(bytes_per * n / (res["alg5"] * 1e-3) / 1e9, 1)}
        _log(f"divmod_bsweep: b = {b}: {sweep[b]}")
        del x, q, r
    top = sweep[1024]
    k_ms = top["alg5_ms_per_1e7"] * n / 1e7
    bytes_per = 4 * (2 * 32 + 33 + 32)
    gbs = bytes_per * n / (k_ms * 1e-3) / 1e9
    out = {"metric": "G divisions/s of 2048-bit numbers by 2^1024 - 1 (Algorithm 5), with the b = 32..1024 sweep "
                     "against the Crandall-Chung-Hasan algorithm",
           "value": round(n / (k_ms * 1e-3) / 1e9, 3), "unit": "Gdivisions/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(k_ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32 limbs", "data": "synthetic",
           "config": {"workload": "divmod_bsweep", "divisions": n, "c": 1, "layout": "limb planes",
                      "sweep": {str(k): v for k, v in sweep.items()}},
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic("divmod_bsweep", n),
                        "algorithmic_bytes_per_launch": bytes_per * n, "kernel": "k_wide_alg5<32>",
                        "kernel_avg_ms": round(k_ms, 4), "algorithmic_bytes_per_value": bytes_per}}
    if not args.no_cpu_baseline:
        import oracle as O
        nn = 20000
        xh = W.uniform_u32(0x2008086545 + 1024, 64 * nn).numpy().astype(np.uint32).reshape(64, nn)
        t0 = time.perf_counter()
        O.divmod_wide(1024, 1, xh)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(nn / dt / 1e9, 9), "unit": "Gdivisions/s", "cores": 1, "kind": "oracle",
                               "sample": f"{nn} divisions at b = 1024 (Python integer divmod), {dt:.2f} s"}
    return out


CEILING_PROBES = [  # (probe id, name, unit of one operation, iters, buffer bytes)
    (0, "v_add_u32", "lane-instructions", 2000, 8),
    (1, "v_mad_u64_u32", "lane-instructions", 2000, 8),
    (2, "v_lshl_add_u64", "lane-instructions", 2000, 8),
    (3, "v_lshrrev_b64", "lane-instructions", 2000, 8),
    (4, "HBM read stream (16-byte loads, 4 GiB)", "bytes", 0, 1 << 32),
    (5, "ds_add_u64, random addresses of 64 KiB", "atomics", 1000, 8),
    (6, "ds_add_rtn_u32, random addresses of 64 KiB", "atomics", 1000, 8),
    (7, "global int64 atomics, random over 40 KiB", "atomics", 64, 40 << 10),
    (7, "global int64 atomics, random over 4.5 MiB", "atomics", 64, 9 << 19),
    (7, "global int64 atomics, random over 40 MiB", "atomics", 64, 40 << 20),
    (8, "global int64 atomics, coalesced over 4.5 MiB", "atomics", 512, 9 << 19),
    (9, "v_mov_b32", "lane-instructions", 2000, 8),
    (10, "v_bfe_u32", "lane-instructions", 2000, 8),
    (11, "v_and_or_b32", "lane-instructions", 2000, 8),
    (12, "v_xad_u32", "lane-instructions", 2000, 8),
    (13, "v_lshlrev_b32 (two-operand)", "lane-instructions", 2000, 8),
    (14, "v_and_b32 (two-operand)", "lane-instructions", 2000, 8),
    (15, "v_add_co_u32 + v_addc_co_u32", "lane-instructions", 2000, 8),
    (16, "v_add_u32, one wave per SIMD", "lane-instructions", 2000, 8),
    (17, "v_mad_u64_u32 and v_add_u32 in turn", "lane-instructions", 2000, 8),
]


def run_ceilings(args):
    """Measured ceilings: issue rates of the VALU instructions of the Horner step (in
    lane-instructions per second against the 256 CU x 4 SIMD x 16 lanes x 2.4 GHz peak),
    the HBM read stream, LDS atomics and device-scope global atomics."""
    import torch
    import paper_2008_08654_amd as M

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L = M.lib()
    stream = _stream_ptr(torch)
    results = []
    for probe, name, unit, iters, nbytes in CEILING_PROBES:
        buf = torch.zeros(max(nbytes, 8) // 8, dtype=torch.int64, device=dev)
        ops = ctypes.c_uint64()
        times = []
        for rep in range(args.warmup + max(args.steps, 5)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            M._check(L.cs_ceiling_run(probe, ctypes.c_void_p(buf.data_ptr()), buf.numel() * 8, iters,
                                      ctypes.byref(ops), stream))
            b.record()
            torch.cuda.synchronize()
            if rep >= args.warmup:
                times.append(a.elapsed_time(b))
        times.sort()
        ms = times[len(times) // 2]
        rate = ops.value / (ms * 1e-3)
        rec = {"probe": name, "unit": unit, "ops_per_launch": ops.value, "median_ms": round(ms, 4),
               "rate": rate}
        if unit == "lane-instructions":
            rec["frac_of_full_rate"] = round(rate / (VALU_PEAK_TOPS * 1e12), 3)
        _log(f"ceilings: {name}: {rate:.4g} {unit}/s in {ms:.3f} ms")
        results.append(rec)
        del buf
    mad = next(r for r in results if r["probe"] == "v_mad_u64_u32")
    return {"metric": "measured ceilings (VALU issue rates, HBM read, LDS and global atomics)",
            "value": round(mad["rate"] / 1e12, 3), "unit": "T lane-instructions/s (v_mad_u64_u32)", "n_gpus": 1,
            "steps": max(args.steps, 5), "warmup": args.warmup, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": "ceilings", "valu_peak_tops": round(VALU_PEAK_TOPS, 2),
                       "probes": results}}


def run_divmod(args, wl):
    import numpy as np
    import torch
    import paper_2008_08654_amd as M
    import workloads as W

    n = args.n or wl["n"]
    dev = torch.device("cuda:0")
    x = W.below_limbs(wl["p"] * wl["p"], wl["limbs"], 0x2008086543, n, device=dev)
    q = torch.empty((n, wl["qlimbs"]), dtype=torch.int64, device=dev)
    r = torch.empty((n, wl["qlimbs"]), dtype=torch.int64, device=dev)
    for _ in range(args.warmup):
        M.mersenne_divmod(wl["prime"], x, q, r)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        M.mersenne_divmod(wl["prime"], x, q, r)
        b.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    M.mersenne_status()
    k_ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
    # the outputs the oracle checks (before the naive kernel reuses the buffers): the first
    # 2^22 values (the ones it is timed on) and every (n / 2^20)-th value of the batch
    n_pre = min(n, 1 << 22)
    idx = torch.arange(0, n, max(1, n // (1 << 20)), device=dev)
    check = None
    if not args.no_cpu_baseline:
        check = [(x[:n_pre], q[:n_pre], r[:n_pre]), (x[idx], q[idx], r[idx])]
        check = [tuple(t.cpu().numpy().view(np.uint64) for t in c) for c in check]
    naive_ms = None
    if not args.no_naive:
        nn = min(n, 1 << 24)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        M.mersenne_divmod(wl["prime"], x[:nn], q[:nn], r[:nn], naive=True)
        a.record()
        M.mersenne_divmod(wl["prime"], x[:nn], q[:nn], r[:nn], naive=True)
        b.record()
        torch.cuda.synchronize()
        naive_ms = a.elapsed_time(b) * n / nn
    bytes_per = 8 * (wl["limbs"] + 2 * wl["qlimbs"])
    gbs = bytes_per * n / (k_ms * 1e-3) / 1e9
    out = {"metric": "G values/s quotient and remainder (branch-free) + % of HBM roofline",
           "value": round(n * args.steps / elapsed / 1e9, 3), "unit": "Gvalues/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": args.workload, "values": n, "limbs_in": wl["limbs"], "limbs_out": wl["qlimbs"],
                      "naive_kernel_ms_scaled": None if naive_ms is None else round(naive_ms, 3),
                      "speedup_vs_naive": None if naive_ms is None else round(naive_ms / k_ms, 2)},
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.workload, n),
                        "algorithmic_bytes_per_launch": bytes_per * n, "kernel": "k_divmod",
                        "kernel_avg_ms": round(k_ms, 4), "algorithmic_bytes_per_value": bytes_per}}
    if check is not None:
        import oracle as O
        differ = 0
        for i, (xh, qg, rg) in enumerate(check):
            t0 = time.perf_counter()
            qo, ro = O.divmod_batch(wl["prime"], xh)
            dt = time.perf_counter() - t0
            if i == 0:
                out["cpu_baseline"] = {"value": round(xh.shape[0] / dt / 1e9, 6), "unit": "Gvalues/s", "cores": 1,
                                       "kind": "oracle",
                                       "sample": f"first {xh.shape[0]} values, {dt:.1f} s, one thread"}
            qo, ro = qo.reshape(qg.shape), ro.reshape(rg.shape)
            differ += int((qo != qg).any(axis=-1).sum() + (ro != rg).any(axis=-1).sum()) if qg.ndim > 1 else \
                int((qo != qg).sum() + (ro != rg).sum())
        out["parity"] = {"status": "bit-exact" if differ == 0 else "MISMATCH",
                         "checked": f"quotient and remainder of the first {n_pre} values and of every "
                                    f"{max(1, n // (1 << 20))}-th value of the {n} (after the timed launches), "
                                    f"against the oracle", "values_differing": differ}
    else:
        out["parity"] = {"status": "not checked (--no-cpu-baseline)"}
    return out


def summarize_kernel_stats(args):
    """Writes profiles/<name>.md from a `rocprofv3 --kernel-trace --stats --output-format csv` run:
    the kernels by total time, with the command that made the run."""
    import csv
    import glob
    d, name = args.profile_summary
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        sys.exit(f"bench.py: no kernel_stats.csv under {d}")
    with open(files[0]) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics — {args.profile_title or name}", "",
             "Command (from the repository root, one MI355X):", "", "```",
             f"rocprofv3 --kernel-trace --stats --output-format csv -d /tmp/{name} -o run -- \\",
             f"    python3 {args.profile_command}", "```", "",
             "The input generators' torch kernels run too (bench.py does not time them). Durations in "
             "microseconds.", "",
             "| Kernel | Calls | Avg us | Min us | Max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in rows[:14]:
        kname = r["Name"] if len(r["Name"]) <= 110 else r["Name"][:107] + "..."
        lines.append(f"| `{kname}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    out = os.path.join(HERE, "profiles", name + ".md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return {"written": out, "kernels": len(rows)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="single_stream_zipf",
                    choices=sorted(SKETCH_WORKLOADS) + sorted(DIVMOD_WORKLOADS) + sorted(MAP_WORKLOADS)
                    + ["batched", "served", "divmod_bsweep", "ceilings"])
    ap.add_argument("--n", type=int, default=None, help="override the number of keys / values")
    ap.add_argument("--path", type=int, default=0, help="force an update path (1 LDS, 2 global, 3 binned)")
    ap.add_argument("--direct-fraction", type=float, default=0.0,
                    help="served: updates with n < f * buckets use direct atomics (0: library default)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 1 GiB device to device (reference dispatch for HBM byte counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched: keep the default options instead of autotuning (for profiles)")
    ap.add_argument("--no-naive", action="store_true")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="summarize the FETCH_SIZE and WRITE_SIZE counter runs of --workload into "
                         "profiles/hbm_traffic.json (no GPU work)")
    ap.add_argument("--profile-summary", nargs=2, metavar=("DIR", "NAME"), default=None,
                    help="write profiles/NAME.md from the rocprofv3 kernel statistics under DIR (no GPU work)")
    ap.add_argument("--profile-title", default=None)
    ap.add_argument("--profile-command", default="bench.py", help="the profiled command, for the summary")
    args = ap.parse_args()
    if args.profile_summary:
        print(json.dumps(summarize_kernel_stats(args)), flush=True)
        return
    if args.traffic_summary:
        print(json.dumps(summarize_traffic(args)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the benchmark runs on one GPU "
              f"(the sketch would shard by key range plus one int64 all-reduce, which is not implemented)",
              file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        import torch
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "ceilings":
        out = run_ceilings(args)
    elif args.workload == "batched":
        out = run_batched(args)
    elif args.workload == "served":
        out = run_served(args)
    elif args.workload == "divmod_bsweep":
        out = run_divmod_bsweep(args)
    elif args.workload in MAP_WORKLOADS:
        out = run_bucket_map(args, MAP_WORKLOADS[args.workload])
    elif args.workload in SKETCH_WORKLOADS:
        out = run_sketch(args, SKETCH_WORKLOADS[args.workload])
    else:
        out = run_divmod(args, DIVMOD_WORKLOADS[args.workload])
    # A run whose work failed or disagreed with the oracle reports no throughput.
    failed = out.get("config", {}).get("failed_requests", 0) or out.get("config", {}).get("failed_members", 0)
    mismatch = str(out.get("parity", {}).get("status", "")).startswith("MISMATCH")
    if failed or mismatch:
        out["value"] = None
        print(json.dumps(out), flush=True)
        print(f"bench.py: {'failed work' if failed else 'parity mismatch'}: no throughput is reported",
              file=sys.stderr, flush=True)
        sys.exit(1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
