"""Throughput benchmark: batched CKKS encryption on one MI355X, Zinc
(Algorithm 1) against vanilla public-key encryption (Eq. 8) on the same GPU.

One step = one fused launch (FP64 encode + sampling + every limb's NTTs + the
cached-Enc(0) / pk*u epilogue) over the whole batch of the workload, inputs
resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload n8192_b1024]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CKKS encryptions/sec (Zinc vs vanilla, same GPU) at N=8192; p99 latency served"

# ALU roofline of the NTT butterflies (the dominant work of the fused launch).
# Measured peak: zinc_butterfly_rate runs the kernels' own butterfly in a
# register-resident loop over a full-occupancy grid (no memory traffic) and
# returns butterflies per second, per arithmetic: 64-bit integer Shoup with
# the lazy reduction every fourth stage (moduli >= 2^50) or exact FP64
# (moduli < 2^50).  A launch's limbs have equal butterfly counts, so its peak
# is the harmonic mean of its limbs' rates.
# Model beside it, from the chip's unit counts and clock: VALU issue of
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 lane-instructions/s over
# the butterfly's instruction count in the gfx950 code (23.25 integer, 8 FP64;
# one instruction per lane-cycle).
VALU_LANE_CYCLES_PER_S = 256 * 4 * 16 * 2.4e9
BFLY_COST_INT = 23.25
BFLY_COST_FP64 = 8


def model_peak_bfly_per_s(limbs: int, fp64_mask: int) -> float:
    cost = sum(BFLY_COST_FP64 if (fp64_mask >> l) & 1 else BFLY_COST_INT for l in range(limbs)) / limbs
    return VALU_LANE_CYCLES_PER_S / cost


_RATES = {}


def measured_rates(moduli, limbs: int, fp64_mask: int) -> list:
    """Measured butterflies/s of each data limb's arithmetic (one measurement
    per arithmetic, with the first such limb's modulus)."""
    import paper_2408_07304_amd as zinc

    out = []
    for l in range(limbs):
        arith = (fp64_mask >> l) & 1
        if arith not in _RATES:
            _RATES[arith] = (zinc.butterfly_rate(arith, moduli[l]), moduli[l])
            print(f"[bench] butterfly rate ({'FP64' if arith else 'integer'}, q = {moduli[l]}): "
                  f"{_RATES[arith][0] / 1e12:.3f} T/s", file=sys.stderr, flush=True)
        out.append(_RATES[arith][0])
    return out


def measured_peak_bfly_per_s(moduli, limbs: int, fp64_mask: int) -> float:
    rates = measured_rates(moduli, limbs, fp64_mask)
    return limbs / sum(1.0 / r for r in rates)


HBM_PEAK_BYTES_PER_S = 8.0e12
# results of zinc_autotune on MI355X, keyed by device, ring degree, moduli and batch
TUNE_CACHE = os.path.join(ROOT, "paper_2408_07304_amd", "tuning_cache.txt")
KERNEL_SOURCES = ("paper_2408_07304_amd/csrc/kernels.hip", "paper_2408_07304_amd/csrc/kernels_common.h",
                  "paper_2408_07304_amd/csrc/kernels_tiles.h",
                  "paper_2408_07304_amd/csrc/kernels_elementwise.hip", "paper_2408_07304_amd/csrc/device.h")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


SETTLE_MS = 250.0


def settle(fn):
    """Run fn for about SETTLE_MS of wall time before the warmup steps: the
    GPU's clocks rise over the first tens of milliseconds under load, and the
    timed steps should see the clocks a sustained workload runs at."""
    import torch
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < SETTLE_MS:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()


def butterflies(n: int, limbs: int, scheme: int) -> int:
    ntts = (2 if scheme == 1 else 3) * limbs
    return ntts * (n // 2) * int(math.log2(n))


def algorithmic_bytes(n: int, limbs: int, n_slots: int) -> int:
    """HBM bytes one encryption must move: slots in, ciphertext out."""
    return 8 * n_slots + 16 * limbs * n


def traffic_from_profile(workload: str, scheme_name: str):
    """Measured HBM bytes per launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_encrypt_{scheme_name}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def elementwise_traffic(workload: str, scheme_name: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-kernel scaled) of a
    standalone element-wise kernel, from the committed PMC summary when it was
    taken with the current kernel sources, else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_elementwise_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash() or scheme_name not in d.get("kernels", {}):
        return None
    k = d["kernels"][scheme_name]
    return k["read_bytes_per_launch"] + k["write_bytes_per_launch"]


def cpu_model() -> str:
    """The host CPU's model name (what lscpu reports), from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ws, scheme: int, budget_s: float):
    """The CPU oracle (plain C, -O2, scalar) on a bounded sample of the same
    workload: encode + encrypt of the first plaintexts, one per thread, on all
    host threads (up to 16) for most of the budget and on one thread for the
    rest (the like-for-like analogue of the paper's single-threaded setup)."""
    import concurrent.futures as cf

    import oracle
    from paper_2408_07304_amd.workloads import make_slots

    ps = ws.params[0]
    P = oracle.Params(ps.log_n, ps.bits, ps.scale, ps.seed)
    _, pk = oracle.keygen(P)
    key = oracle.zinc_precompute(P, pk) if scheme == 1 else pk
    threads = max(1, min(os.cpu_count() or 1, 16))
    z1 = make_slots(ws, 1)
    t0 = time.perf_counter()
    oracle.encrypt_slots(P, scheme, key, z1[0], 0)
    one = time.perf_counter() - t0
    count = int(min(ws.batch, max(threads, threads * 0.75 * budget_s / max(one, 1e-6))))
    z = make_slots(ws, count)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda i: oracle.encrypt_slots(P, scheme, key, z[i], i), range(count)))
    dt = time.perf_counter() - t0
    count1 = int(max(1, min(count, 0.25 * budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    for i in range(count1):
        oracle.encrypt_slots(P, scheme, key, z[i], i)
    dt1 = time.perf_counter() - t0
    return {"value": count / dt, "unit": "enc/s", "cores": threads, "kind": "oracle",
            "sample": f"{count} of {ws.batch} plaintexts of {ws.name} (encode + "
                      f"{'Zinc' if scheme == 1 else 'vanilla'} encrypt), {threads} threads, {dt:.1f} s; "
                      f"{count1} of them on 1 thread, {dt1:.1f} s",
            "one_thread": {"value": count1 / dt1, "unit": "enc/s", "cores": 1},
            "cpu_model": cpu_model(), "host_threads": os.cpu_count()}


_ORACLE_KEYS = {}


def _oracle_key(ps, scheme: int):
    import oracle

    if ps.name not in _ORACLE_KEYS:
        P = oracle.Params(ps.log_n, ps.bits, ps.scale, ps.seed)
        _, pk = oracle.keygen(P)
        _ORACLE_KEYS[ps.name] = (P, pk, oracle.zinc_precompute(P, pk))
    P, pk, zero = _ORACLE_KEYS[ps.name]
    return P, (zero if scheme == 1 else pk)


def oracle_rate(items, scheme: int, threads: int, budget_s: float) -> dict:
    """Oracle encode + encrypt throughput over a bounded prefix of `items`
    ((ParamSet, slot vector) pairs), `threads` plaintexts at a time."""
    import concurrent.futures as cf

    import oracle

    keys = {}
    for ps, _ in items:
        if ps.name not in keys:
            keys[ps.name] = _oracle_key(ps, scheme)
    t0 = time.perf_counter()
    P, key = keys[items[0][0].name]
    oracle.encrypt_slots(P, scheme, key, items[0][1], 0)
    one = time.perf_counter() - t0
    count = int(min(len(items), max(threads, threads * budget_s / max(one, 1e-6))))

    def enc(i):
        P, key = keys[items[i][0].name]
        return oracle.encrypt_slots(P, scheme, key, items[i][1], i)

    t0 = time.perf_counter()
    if threads == 1:
        for i in range(count):
            enc(i)
    else:
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(enc, range(count)))
    dt = time.perf_counter() - t0
    return {"enc_per_s": count / dt, "plaintexts": count, "threads": threads, "seconds": dt}


def bench_config_table(steps: int, warmup: int, budget_s: float) -> list:
    """Every benchmark configuration (N = 4096, 8192, 16384 batches and the
    mixed batch), both schemes: GPU enc/s (autotuned fused launch, or the
    mixed plan) beside the oracle on one thread and on all host threads (up
    to 16), each timed on a bounded prefix of the same plaintexts."""
    import torch

    import paper_2408_07304_amd as zinc
    from paper_2408_07304_amd.workloads import W_LARGE, W_MAIN, W_MIXED, W_SMALL, make_mixed, make_slots

    threads = max(1, min(os.cpu_count() or 1, 16))
    rows = []
    for ws in (W_SMALL, W_MAIN, W_LARGE):
        ps = ws.params[0]
        ctx = zinc.context_for(ps)
        ctx.keygen()
        ctx.precompute()
        ctx.autotune(batch=ws.batch, cache_path=TUNE_CACHE)
        zh = make_slots(ws)
        z = torch.from_numpy(zh).to("cuda")
        ids = torch.arange(ws.batch, dtype=torch.int64, device="cuda")
        ct = torch.empty((ws.batch, 2, ps.limbs, ps.n), dtype=torch.int64, device="cuda")
        items = [(ps, zh[i]) for i in range(ws.batch)]
        for name, sch in (("zinc", 1), ("vanilla", 0)):
            settle(lambda: ctx.encrypt_slots(sch, z, ids, ct))
            for _ in range(max(1, warmup)):
                ctx.encrypt_slots(sch, z, ids, ct)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                ctx.encrypt_slots(sch, z, ids, ct)
            b.record()
            torch.cuda.synchronize()
            gpu = ws.batch / (a.elapsed_time(b) / steps / 1e3)
            row = {"workload": ws.name, "scheme": name, "gpu_enc_per_s": gpu,
                   "oracle_1_thread": oracle_rate(items, sch, 1, budget_s),
                   "oracle_all_threads": oracle_rate(items, sch, threads, budget_s)}
            rows.append(row)
            print(f"[bench] config table: {row}", file=sys.stderr, flush=True)
        del z, ct, ids
        ctx.close()
        torch.cuda.empty_cache()
    mb = make_mixed(W_MIXED)
    items = [(W_MIXED.params[int(mb.ctx_idx[i])],
              mb.slots[int(mb.slot_off[i]): int(mb.slot_off[i]) + W_MIXED.params[int(mb.ctx_idx[i])].slots])
             for i in range(len(mb.ct_id))]
    mctx = mixed_contexts()
    mixed = bench_mixed(mctx, steps, warmup)
    for c in mctx:
        c.close()
    for name, sch in (("zinc", 1), ("vanilla", 0)):
        row = {"workload": W_MIXED.name, "scheme": name, "gpu_enc_per_s": mixed[f"{name}_enc_per_s"],
               "oracle_1_thread": oracle_rate(items, sch, 1, budget_s),
               "oracle_all_threads": oracle_rate(items, sch, threads, budget_s)}
        rows.append(row)
        print(f"[bench] config table: {row}", file=sys.stderr, flush=True)
    return rows


def bench_configs(steps: int, warmup: int, tune_cache) -> dict:
    """The other single-parameter configurations (N = 4096 with 64 plaintexts,
    N = 16384 with 4096 plaintexts), both schemes: the autotuned fused launch,
    timed with HIP events on the launch stream, with the measured-peak ALU
    roofline of each."""
    import torch

    import paper_2408_07304_amd as zinc
    from paper_2408_07304_amd.workloads import W_LARGE, W_SMALL, make_slots

    out = {}
    for ws in (W_SMALL, W_LARGE):
        ps = ws.params[0]
        ctx = zinc.context_for(ps)
        ctx.keygen()
        ctx.precompute()
        ctx.autotune(batch=ws.batch, cache_path=tune_cache or None)
        z = torch.from_numpy(make_slots(ws)).to("cuda")
        ids = torch.arange(ws.batch, dtype=torch.int64, device="cuda")
        ct = torch.empty((ws.batch, 2, ps.limbs, ps.n), dtype=torch.int64, device="cuda")
        mask = ctx.info()["ntt_fp64_mask"]
        peak = measured_peak_bfly_per_s(ctx.moduli, ps.limbs, mask)
        r = {"N": ps.n, "batch": ws.batch, "data_limbs": ps.limbs, "slot_values": ws.dist,
             "tuning": ctx.get_tuning()}
        for name, sch in (("zinc", 1), ("vanilla", 0)):
            settle(lambda: ctx.encrypt_slots(sch, z, ids, ct))
            for _ in range(max(1, warmup)):
                ctx.encrypt_slots(sch, z, ids, ct)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                ctx.encrypt_slots(sch, z, ids, ct)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / steps
            ach = ws.batch * butterflies(ps.n, ps.limbs, sch) / (ms / 1e3)
            r[name] = {"kernel_ms": ms, "enc_per_s": ws.batch / (ms / 1e3), "alu_frac": ach / peak,
                       "hbm_frac": ws.batch * algorithmic_bytes(ps.n, ps.limbs, ps.slots) / (ms / 1e3)
                       / HBM_PEAK_BYTES_PER_S}
        r["zinc_over_vanilla"] = r["vanilla"]["kernel_ms"] / r["zinc"]["kernel_ms"]
        r["peak_gbutterfly_per_s"] = peak / 1e9
        out[ws.name] = r
        print(f"[bench] config {ws.name}: {r}", file=sys.stderr, flush=True)
        if ctx.device_errors():
            raise SystemExit("device error flag set during the benchmark")
        del z, ct, ids
        ctx.close()
        torch.cuda.empty_cache()
    return out


def bench_encrypt_only(ctx, z, ids, ct, steps: int, warmup: int) -> dict:
    """Encryption alone from plaintexts encoded beforehand (zinc_encode), the
    figure reported beside the fused encode + encrypt throughput."""
    import torch

    b, L, n = ct.shape[0], ct.shape[2], ct.shape[3]
    pt = torch.empty((b, L, n), dtype=torch.int64, device="cuda")
    ctx.encode(z, pt)
    out = {}
    for name, fn in (("zinc", lambda: ctx.encrypt(pt, ids, ct)), ("vanilla", lambda: ctx.encrypt_vanilla(pt, ids, ct))):
        settle(fn)
        for _ in range(max(1, warmup)):
            fn()
        torch.cuda.synchronize()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        e.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(e) / steps
        out[name] = {"kernel_ms": ms, "enc_per_s": b / (ms / 1e3)}
        print(f"[bench] encrypt only (pre-encoded) {name}: {out[name]}", file=sys.stderr, flush=True)
    out["zinc_over_vanilla"] = out["vanilla"]["kernel_ms"] / out["zinc"]["kernel_ms"]
    del pt
    return out


def bench_elementwise(ctx, ps, batch: int, steps: int, warmup: int) -> dict:
    """The element-wise steps alone (Algorithm 1's additions, Eq. 8's products
    and additions) on `batch` ciphertexts of transform outputs: HBM-bound
    streams.  Algorithmic bytes per ciphertext: Zinc 32 L N (read the two
    transforms, write the ciphertext), vanilla 40 L N (plus NTT(u)); the cached
    Enc(0) and the public key are shared by the batch."""
    import torch

    L, n = ps.limbs, ps.n
    hat = torch.randint(0, 2 ** 20, (batch, 2, L, n), dtype=torch.int64, device="cuda")
    uhat = torch.randint(0, 2 ** 20, (batch, L, n), dtype=torch.int64, device="cuda")
    out = torch.empty_like(hat)
    out_d = {}
    for name, fn, per_ct in (("zinc", lambda: ctx.elementwise_zinc(hat, out), 32 * L * n),
                             ("vanilla", lambda: ctx.elementwise_vanilla(uhat, hat, out), 40 * L * n)):
        settle(fn)
        for _ in range(max(1, warmup)):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        gbps = batch * per_ct / (ms / 1e3) / 1e9
        out_d[name] = {"us": ms * 1e3, "algorithmic_bytes": batch * per_ct, "GB_per_s": gbps,
                       "hbm_frac": gbps * 1e9 / HBM_PEAK_BYTES_PER_S,
                       "traffic": elementwise_traffic(f"n{ps.n}_b{batch}", name)}
        print(f"[bench] element-wise {name}: {out_d[name]}", file=sys.stderr, flush=True)
    del hat, uhat, out
    return out_d


# Total encryption times the paper reports for its datasets (Table 2; SEAL,
# one thread of an EPYC 7302P, N = 32768): context, not a target.
PAPER_TABLE2_S = {"covid19": {"ckks": 19.2, "zinc": 8.2}, "bitcoin": {"ckks": 62.2, "zinc": 24.8},
                  "hg38": {"ckks": 1983.6, "zinc": 812.6}}


def bench_table2(chunk: int = 1024, reps: int = 2) -> dict:
    """The paper's parameters (N = 32768, 16 primes, Delta = 2^55) on
    synthetic rows shaped like its three datasets: one ciphertext per row,
    fused encode + encrypt in launches of `chunk` rows into one reused output
    buffer; total time for the whole dataset, for Zinc, Eq. 8 vanilla and the
    special-prime vanilla (the form of the paper's CKKS baseline)."""
    import torch

    import paper_2408_07304_amd as zinc
    from paper_2408_07304_amd.workloads import P32768_Q16, TABLE2, dataset_rows

    ps = P32768_Q16
    ctx = zinc.context_for(ps)
    ctx.keygen()
    ctx.precompute()
    ct = torch.empty((chunk, 2, ps.limbs, ps.n), dtype=torch.int64, device="cuda")
    out = {"params": {"N": ps.n, "moduli_bits": list(ps.bits), "scale_log2": 55}, "chunk": chunk, "reps": reps}
    for d in TABLE2:
        z = torch.from_numpy(dataset_rows(d, 0, d.rows)).to("cuda")
        ids = torch.arange(d.rows, dtype=torch.int64, device="cuda")
        r = {"rows": d.rows, "slots_per_row": d.slots}
        for name, sch in (("zinc", zinc.ZINC_SCHEME_ZINC), ("vanilla", zinc.ZINC_SCHEME_VANILLA),
                          ("vanilla_sp", zinc.ZINC_SCHEME_VANILLA_SP)):
            def run():
                for s0 in range(0, d.rows, chunk):
                    n = min(chunk, d.rows - s0)
                    ctx.encrypt_slots(sch, z[s0:s0 + n], ids[s0:s0 + n], ct[:n])
            m = min(chunk, d.rows)
            settle(lambda: ctx.encrypt_slots(sch, z[:m], ids[:m], ct[:m]))
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                run()
            b.record()
            torch.cuda.synchronize()
            r[f"{name}_s"] = a.elapsed_time(b) / reps / 1e3
        r["zinc_over_vanilla"] = r["vanilla_s"] / r["zinc_s"]
        r["zinc_over_vanilla_sp"] = r["vanilla_sp_s"] / r["zinc_s"]
        r["paper_seal_cpu_s"] = PAPER_TABLE2_S[d.name]
        out[d.name] = r
        print(f"[bench] table-2 shape {d.name}: {r}", file=sys.stderr, flush=True)
        del z, ids
    ctx.close()
    del ct
    torch.cuda.empty_cache()
    return out


def mixed_contexts():
    """Keyed and precomputed contexts of the four mixed-workload parameter sets."""
    import paper_2408_07304_amd as zinc
    from paper_2408_07304_amd.workloads import W_MIXED

    ctxs = []
    for ps in W_MIXED.params:
        c = zinc.context_for(ps)
        c.keygen()
        c.precompute()
        ctxs.append(c)
    return ctxs


def bench_mixed(ctxs, steps: int, warmup: int) -> dict:
    """The mixed batch: 2048 plaintexts, ring degree drawn per plaintext from
    {4096, 8192, 16384, 32768}, encrypted by one persistent plan launch
    (captured as a HIP graph on the first launch, replayed after)."""
    import torch

    import paper_2408_07304_amd as zinc
    from paper_2408_07304_amd.workloads import W_MIXED, make_mixed

    mb = make_mixed(W_MIXED)
    items = list(zip(mb.ctx_idx.tolist(), mb.slot_off.tolist(), mb.ct_off.tolist(), mb.ct_id.tolist()))
    d_slots = torch.from_numpy(mb.slots).to("cuda")
    d_ct = torch.empty(mb.ct_words, dtype=torch.int64, device="cuda")
    out = {"batch": int(len(mb.ct_id)), "ring_degrees": [ps.n for ps in W_MIXED.params],
           "per_degree": [int((mb.ctx_idx == k).sum()) for k in range(len(W_MIXED.params))],
           "ciphertext_gib": mb.ct_words * 8 / 2 ** 30}
    for name, sch in (("zinc", 1), ("vanilla", 0)):
        plan = zinc.Plan(ctxs, items, sch)
        settle(lambda: plan.launch(d_slots, d_ct))
        for _ in range(max(1, warmup)):
            plan.launch(d_slots, d_ct)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            plan.launch(d_slots, d_ct)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        out[f"{name}_ms"] = ms
        out[f"{name}_enc_per_s"] = len(mb.ct_id) / (ms / 1e3)
        plan.close()
        print(f"[bench] mixed {name}: {ms:.3f} ms", file=sys.stderr, flush=True)
    out["zinc_over_vanilla"] = out["vanilla_ms"] / out["zinc_ms"]
    del d_ct, d_slots
    torch.cuda.empty_cache()
    return out


def bench_serving(ctxs, saturated_enc_per_s: float, n_requests: int, warm: int, n_streams: int,
                  max_batch: int, budget_gib: float) -> dict:
    """Open-loop serving: Poisson arrivals at 0.7 x the vanilla mixed-batch
    throughput (in requests/s, requests of 1..64 plaintexts of one parameter
    set each), the same trace replayed for both schemes; latency = completion
    observed on the host - scheduled arrival, over the requests after the
    first `warm`."""
    import numpy as np
    import torch

    import paper_2408_07304_amd as zinc
    from paper_2408_07304_amd.workloads import W_MIXED, make_trace, trace_requests

    mean_pt = 32.5
    rate = 0.7 * saturated_enc_per_s / mean_pt
    tr = make_trace(n_requests + warm, rate, W_MIXED.params, seed=5, pool=256)
    req = trace_requests(tr)
    d_slots = torch.from_numpy(tr.slots).to("cuda")
    torch.cuda.synchronize()
    out = {"requests": n_requests, "warmup_requests": warm, "offered_req_per_s": rate,
           "offered_enc_per_s": rate * mean_pt, "load_vs_vanilla_saturated": 0.7, "streams": n_streams,
           "max_batch": max_batch, "hbm_budget_gib": budget_gib, "outputs": "server arena, discarded"}
    for name, sch in (("zinc", 1), ("vanilla", 0)):
        t0 = time.perf_counter()
        times = zinc.serve_trace(ctxs, sch, req, tr.arrival_ns, d_slots, None, n_streams=n_streams,
                                 max_batch=max_batch, hbm_budget=int(budget_gib * 2 ** 30))
        wall = time.perf_counter() - t0
        m = slice(warm, None)
        lat = (times["done_ns"][m] - times["submit_ns"][m]).astype(np.float64) / 1e6
        span = (times["done_ns"][m].max() - times["submit_ns"][m].min()) / 1e9
        nb = len(np.unique(times["batch"]))
        out[name] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                     "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                     "enc_per_s": float(tr.n_pt[m].sum() / span), "batches": nb,
                     "mean_batch_plaintexts": float(tr.n_pt.sum() / nb), "replay_s": wall}
        print(f"[bench] serving {name}: {out[name]}", file=sys.stderr, flush=True)
    out["p99_vanilla_over_zinc"] = out["vanilla"]["p99_ms"] / out["zinc"]["p99_ms"]
    return out


def main():
    global SETTLE_MS
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--settle-ms", type=float, default=SETTLE_MS,
                    help="untimed launches before the warmup steps, in ms of wall time (clock ramp)")
    ap.add_argument("--workload", default="n8192_b1024")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scheme", choices=["both", "zinc", "vanilla", "vanilla_sp"], default="both",
                    help="'both' runs Zinc, vanilla and the special-prime vanilla")
    ap.add_argument("--no-tune", action="store_true", help="keep the default kernel configuration")
    ap.add_argument("--config-table", action="store_true",
                    help="also measure every configuration, both schemes, GPU and oracle (1 and all threads)")
    ap.add_argument("--no-table2", action="store_true",
                    help="skip the paper-parameter runs on rows shaped like its datasets")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuning cache file ('' to time every candidate afresh)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-degree plan and serving measurements")
    ap.add_argument("--no-configs", action="store_true", help="skip the N = 4096 and N = 16384 configurations")
    ap.add_argument("--serve-requests", type=int, default=10000, help="measured requests of the serving replay")
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-max-batch", type=int, default=512)
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="also run one torch copy of this many MiB (reference kernel for HBM byte counters)")
    args = ap.parse_args()

    SETTLE_MS = args.settle_ms
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              "ciphertexts are independent, so N GPUs would each run this benchmark on 1/N of the batch.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2408_07304_amd as zinc
    from paper_2408_07304_amd.workloads import WORKLOADS, make_slots

    ws = WORKLOADS[args.workload]
    if len(ws.params) != 1:
        raise SystemExit("the throughput benchmark runs single-parameter workloads")
    ps = ws.params[0]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    ctx = zinc.context_for(ps)
    ctx.keygen()
    ctx.precompute()
    tune = None
    if not args.no_tune:
        # kernel form and NTT arithmetic, outside the timed region; the tuning
        # cache holds earlier results for this device and parameter set
        tune = ctx.autotune(batch=ws.batch, cache_path=args.tune_cache or None)
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    z = torch.from_numpy(make_slots(ws)).to(dev)
    ids = torch.arange(ws.batch, dtype=torch.int64, device=dev)
    ct = torch.empty((ws.batch, 2, ps.limbs, ps.n), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()

    schemes = {"zinc": 1, "vanilla": 0, "vanilla_sp": 2}
    run = [s for s in ("zinc", "vanilla", "vanilla_sp") if args.scheme in ("both", s)]
    res = {}
    for name in run:
        sch = schemes[name]
        settle(lambda: ctx.encrypt_slots(sch, z, ids, ct))
        for _ in range(args.warmup):
            ctx.encrypt_slots(sch, z, ids, ct)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t0 = time.perf_counter()
        for a, b in ev:
            a.record()
            ctx.encrypt_slots(sch, z, ids, ct)
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = [a.elapsed_time(b) for a, b in ev]
        res[name] = {"ms_per_step": wall * 1e3 / args.steps, "kernel_ms": sum(kms) / len(kms),
                     "kernel_ms_min": min(kms)}
        print(f"[bench] {name}: {res[name]}", file=sys.stderr, flush=True)
    if ctx.device_errors():
        raise SystemExit("device error flag set during the benchmark")
    if args.copy_ref_mib:
        src = torch.empty(args.copy_ref_mib << 17, dtype=torch.int64, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy reference: {args.copy_ref_mib} MiB read + {args.copy_ref_mib} MiB written",
              file=sys.stderr, flush=True)

    main_name = run[0]
    sch = schemes[main_name]
    r = res[main_name]
    value = ws.batch / (r["ms_per_step"] / 1e3)
    bfly = ws.batch * butterflies(ps.n, ps.limbs, sch)
    achieved = bfly / (r["kernel_ms"] / 1e3)
    mask = ctx.info()["ntt_fp64_mask"]
    peak = measured_peak_bfly_per_s(ctx.moduli, ps.limbs, mask)
    peak_model = model_peak_bfly_per_s(ps.limbs, mask)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "enc/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": ws.name, "N": ps.n, "moduli_bits": list(ps.bits), "data_limbs": ps.limbs,
                   "scale_log2": int(math.log2(ps.scale)), "batch": ws.batch, "slots": ps.slots,
                   "slot_values": ws.dist, "scheme": main_name, "fused_encode": True,
                   "tuning": ctx.get_tuning(), "autotuned": tune is not None,
                   "tuning_from_cache": bool(tune and tune["from_cache"])},
        "roofline": {"bound": "alu", "achieved": achieved / 1e9, "peak": peak / 1e9,
                     "unit": "Gbutterfly/s", "frac": achieved / peak,
                     "peak_source": "measured: zinc_butterfly_rate, the kernels' butterflies in registers, "
                                    "harmonic mean over the data limbs' arithmetic",
                     "peak_rates_gbutterfly_per_s": {("fp64" if a else "integer"): v[0] / 1e9
                                                     for a, v in sorted(_RATES.items())},
                     "peak_model": peak_model / 1e9, "frac_model": achieved / peak_model,
                     "ntt_fp64_limbs": [l for l in range(ps.limbs) if (mask >> l) & 1],
                     "traffic": traffic_from_profile(ws.name, main_name),
                     "kernel": ("k_encrypt" if ctx.get_tuning()["tile"][sch] == 16
                                and not (ctx.get_tuning()["reg_epilogue"] >> sch) & 1 else "k_encrypt_tile")
                     + " (fused encode + sample + NTT + add)",
                     "kernel_ms": r["kernel_ms"], "butterflies_per_launch": bfly,
                     "hbm_algorithmic_bytes_per_launch": ws.batch * algorithmic_bytes(ps.n, ps.limbs, ps.slots),
                     "hbm_frac": ws.batch * algorithmic_bytes(ps.n, ps.limbs, ps.slots)
                     / (r["kernel_ms"] / 1e3) / HBM_PEAK_BYTES_PER_S},
    }
    for name in run:
        line[f"{name}_enc_per_s"] = ws.batch / (res[name]["ms_per_step"] / 1e3)
        line[f"{name}_kernel_ms"] = res[name]["kernel_ms"]
    if "vanilla" in res and "zinc" in res:
        line["zinc_over_vanilla"] = res["vanilla"]["ms_per_step"] / res["zinc"]["ms_per_step"]
    if "vanilla_sp" in res and "zinc" in res:
        # vanilla as a library with a special prime computes it (division by
        # the prime with rounding), the form of the paper's CPU baseline
        line["zinc_over_vanilla_sp"] = res["vanilla_sp"]["ms_per_step"] / res["zinc"]["ms_per_step"]
    line["encrypt_only"] = bench_encrypt_only(ctx, z, ids, ct, args.steps, args.warmup)
    if not args.no_configs:
        line["configs"] = bench_configs(args.steps, args.warmup, args.tune_cache)
    line["elementwise"] = bench_elementwise(ctx, ps, ws.batch, args.steps, args.warmup)
    if not args.no_mixed:
        del ct, z
        torch.cuda.empty_cache()
        mctx = mixed_contexts()
        line["mixed_b2048"] = bench_mixed(mctx, args.steps, args.warmup)
        if args.serve_requests > 0:
            line["serving"] = bench_serving(mctx, line["mixed_b2048"]["vanilla_enc_per_s"], args.serve_requests,
                                            args.serve_warmup, args.serve_streams, args.serve_max_batch,
                                            args.serve_budget_gib)
        for c in mctx:
            c.close()
    if not args.no_table2:
        line["table2_shapes"] = bench_table2()
    if args.config_table:
        line["config_table"] = bench_config_table(args.steps, args.warmup, args.cpu_budget / 4)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(ws, sch, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
