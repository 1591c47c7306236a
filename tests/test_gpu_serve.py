"""Serving (zinc_server_*, zinc_serve_trace): requests admitted against an HBM
budget and encrypted by continuous batching on several streams.  Served
ciphertexts must be bit-identical to separate launches with the same ct_ids,
and sampled requests of every ring degree equal the oracle's encryption
(Algorithm 1 / Eq. 8); the scheduler's records must show submission-order
admission, the budget never exceeded, batches within max_batch, and batches
of different streams overlapping on the device."""
import numpy as np
import pytest

import paper_2408_07304_amd as zinc
from gpu_util import check_fused, empty_u64, from_dev, gpu_ctx, ids, oracle_keys, to_dev, torch_cuda
from paper_2408_07304_amd.workloads import W_MIXED, make_trace, trace_requests

pytestmark = pytest.mark.gpu

NAMES = ["n4096", "n8192", "n16384", "n32768"]      # order of W_MIXED.params


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def _granted(tr, r):
    p = W_MIXED.params[int(tr.ctx_idx[r])]
    b = int(tr.n_pt[r]) * 2 * p.limbs * p.n * 8
    return (b + 255) // 256 * 256


def _check_schedule(tr, times, budget, max_batch, n_streams):
    n = len(tr)
    assert np.all(times["submit_ns"] <= times["admit_ns"])
    assert np.all(times["admit_ns"] <= times["launch_ns"])
    assert np.all(times["launch_ns"] <= times["done_ns"])
    # submission order: admissions (and arrivals) are non-decreasing by request
    assert np.all(np.diff(times["admit_ns"].astype(np.int64)) >= 0)
    assert np.all(times["stream"] < n_streams)
    # batches: whole requests, at most max_batch plaintexts, one stream each
    for b in np.unique(times["batch"]):
        sel = times["batch"] == b
        assert int(tr.n_pt[sel].sum()) <= max_batch
        assert len(np.unique(times["stream"][sel])) == 1
        assert len(np.unique(times["launch_ns"][sel])) == 1
    # budget: bytes held between admission and completion never exceed it
    ev = [(int(times["done_ns"][r]), 0, -_granted(tr, r)) for r in range(n)]
    ev += [(int(times["admit_ns"][r]), 1, _granted(tr, r)) for r in range(n)]
    held = 0
    for _, _, d in sorted(ev):
        held += d
        assert held <= budget


def _device_overlaps(times):
    """Pairs of batches on different streams whose device intervals (HIP
    events before and after each launch) intersect."""
    b = {}
    for r in range(len(times)):
        b[int(times["batch"][r])] = (int(times["stream"][r]), int(times["dev_start_ns"][r]),
                                     int(times["dev_end_ns"][r]))
    items = sorted(b.values(), key=lambda x: x[1])
    pairs = 0
    for i, (s1, a1, e1) in enumerate(items):
        for s2, a2, e2 in items[i + 1:]:
            if a2 >= e1:
                break
            if s2 != s1:
                pairs += 1
    return pairs


def _oracle_check_request(tr, r, scheme, got_req):
    """Plaintext 0 of request r (its ciphertexts `got_req`, flat) against the
    oracle's encryption of its slot vector."""
    name = NAMES[int(tr.ctx_idx[r])]
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    so = int(tr.slot_off[r])
    z = np.asarray(tr.slots[so: so + P.n // 2])
    key = zero if scheme == zinc.ZINC_SCHEME_ZINC else pk
    ct0 = np.asarray(got_req[: 2 * P.L * P.n]).reshape(2, P.L, P.n)
    check_fused(c, P, scheme, key, z, int(tr.ct_id[r]), ct0, ("request", r))


def _separate(ctxs, tr, r, scheme):
    """Request r encrypted alone by its context's batch entry point."""
    c = ctxs[int(tr.ctx_idx[r])]
    k, so = int(tr.n_pt[r]), int(tr.slot_off[r])
    z = np.ascontiguousarray(tr.slots[so: so + k * (c.n // 2)]).reshape(k, c.n // 2)
    out = empty_u64(k, 2, c.L, c.n)
    c.encrypt_slots(scheme, to_dev(z), ids(np.arange(int(tr.ct_id[r]), int(tr.ct_id[r]) + k, dtype=np.uint64)),
                    out)
    return from_dev(out).reshape(-1)


@pytest.mark.parametrize("scheme", [zinc.ZINC_SCHEME_VANILLA, zinc.ZINC_SCHEME_ZINC])
def test_served_equals_separate_launches(scheme):
    torch = torch_cuda()
    ctxs = [gpu_ctx(n) for n in NAMES]
    tr = make_trace(48, 20000.0, W_MIXED.params, seed=11, max_count=8)
    assert len(set(tr.ctx_idx.tolist())) == 4
    d_slots = to_dev(tr.slots)
    d_ct = torch.zeros(tr.ct_words, dtype=torch.int64, device="cuda")
    budget, max_batch, streams = 96 << 20, 24, 3          # small budget: requests wait for admission
    torch.cuda.synchronize()
    say(f"serve_trace scheme={scheme}: {len(tr)} requests, {tr.plaintexts} plaintexts, caller output")
    times = zinc.serve_trace(ctxs, scheme, trace_requests(tr), tr.arrival_ns, d_slots, d_ct,
                             n_streams=streams, max_batch=max_batch, hbm_budget=budget)
    _check_schedule(tr, times, budget, max_batch, streams)
    got = from_dev(d_ct)
    seen = set()
    for r in range(len(tr)):
        off = int(tr.ct_off[r])
        ref = _separate(ctxs, tr, r, scheme)
        assert np.array_equal(got[off: off + len(ref)], ref), r
        if int(tr.ctx_idx[r]) not in seen:              # first request of each ring degree vs the oracle
            seen.add(int(tr.ctx_idx[r]))
            say(f"served request {r} (N = {ctxs[int(tr.ctx_idx[r])].n}) vs the oracle")
            _oracle_check_request(tr, r, scheme, got[off: off + len(ref)])
    assert len(seen) == 4


def test_server_object_and_errors():
    torch = torch_cuda()
    ctxs = [gpu_ctx(n) for n in NAMES]
    tr = make_trace(6, 1000.0, W_MIXED.params, seed=12, max_count=4)
    d_slots = to_dev(tr.slots)
    d_ct = torch.zeros(tr.ct_words, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    srv = zinc.Server(ctxs, zinc.ZINC_SCHEME_ZINC, d_slots, d_ct, n_streams=2, max_batch=8, hbm_budget=48 << 20)
    tickets = [srv.submit(int(tr.ctx_idx[r]), int(tr.n_pt[r]), int(tr.slot_off[r]), int(tr.ct_id[r]),
                          int(tr.ct_off[r])) for r in range(len(tr))]
    assert tickets == list(range(len(tr)))
    say("server: submit/progress/query")
    while any(srv.query(t) is None for t in tickets):
        srv.progress()
    srv.drain()
    got = from_dev(d_ct)
    for r in range(len(tr)):
        off = int(tr.ct_off[r])
        ref = _separate(ctxs, tr, r, zinc.ZINC_SCHEME_ZINC)
        assert np.array_equal(got[off: off + len(ref)], ref), r
    # argument errors are reported synchronously
    n_slots, n_ct = d_slots.numel(), d_ct.numel()
    for args, status in [((4, 1, 0, 0), zinc.ZINC_E_INVAL),           # context out of range
                         ((0, 9, 0, 0), zinc.ZINC_E_RANGE),           # above max_batch
                         ((0, 0, 0, 0), zinc.ZINC_E_INVAL),           # empty request
                         ((0, 1, 0, 2 ** 63), zinc.ZINC_E_INVAL),           # ct_id range
                         ((3, 8, 0, 0), zinc.ZINC_E_RANGE),           # 8 x 7 MiB > 48 MiB budget
                         ((0, 1, n_slots - 1, 0), zinc.ZINC_E_INVAL),       # slots past the buffer
                         ((0, 1, 0, 0, n_ct - 1), zinc.ZINC_E_INVAL),       # output past the buffer
                         ((0, 1, 2 ** 64 - 1, 0), zinc.ZINC_E_INVAL)]:      # offset overflow
        with pytest.raises(zinc.ZincError) as e:
            srv.submit(*args)
        assert e.value.status == status, args
    with pytest.raises(zinc.ZincError) as e:
        srv.query(99)
    assert e.value.status == zinc.ZINC_E_INVAL
    srv.close()
    with pytest.raises(zinc.ZincError) as e:
        zinc.Server(ctxs, zinc.ZINC_SCHEME_ZINC, d_slots, d_ct, n_streams=0)
    assert e.value.status == zinc.ZINC_E_INVAL
    with pytest.raises(zinc.ZincError) as e:
        zinc.Server(ctxs, zinc.ZINC_SCHEME_ZINC, d_slots, d_ct, max_batch=0)
    assert e.value.status == zinc.ZINC_E_INVAL
    with pytest.raises(zinc.ZincError) as e:                             # retention needs the arena
        zinc.Server(ctxs, zinc.ZINC_SCHEME_ZINC, d_slots, d_ct, retain_outputs=True)
    assert e.value.status == zinc.ZINC_E_INVAL
    fresh = zinc.context_for(W_MIXED.params[0])
    with pytest.raises(zinc.ZincError) as e:
        zinc.Server([fresh], zinc.ZINC_SCHEME_VANILLA, d_slots, d_ct)      # no keys
    assert e.value.status == zinc.ZINC_E_STATE
    fresh.keygen()
    with pytest.raises(zinc.ZincError) as e:
        zinc.Server([fresh], zinc.ZINC_SCHEME_ZINC, d_slots, d_ct)         # no cached Enc(0)
    assert e.value.status == zinc.ZINC_E_STATE
    fresh.close()


@pytest.mark.parametrize("scheme", [zinc.ZINC_SCHEME_VANILLA, zinc.ZINC_SCHEME_ZINC])
def test_arena_replay_schedule(scheme):
    """Load-generation mode: outputs in the server's arena; a Poisson trace of
    the serving workload's shape completes with a valid schedule."""
    torch = torch_cuda()
    ctxs = [gpu_ctx(n) for n in NAMES]
    tr = make_trace(400, 2000.0, W_MIXED.params, seed=13, pool=64)
    d_slots = to_dev(tr.slots)
    torch.cuda.synchronize()
    budget, max_batch, streams = 1 << 30, 256, 4
    say(f"arena replay scheme={scheme}: {len(tr)} requests, {tr.plaintexts} plaintexts")
    times = zinc.serve_trace(ctxs, scheme, trace_requests(tr), tr.arrival_ns, d_slots, None,
                             n_streams=streams, max_batch=max_batch, hbm_budget=budget)
    _check_schedule(tr, times, budget, max_batch, streams)
    assert np.array_equal(times["submit_ns"], tr.arrival_ns)
    lat = (times["done_ns"] - times["submit_ns"]) / 1e6
    say(f"latency ms p50 {np.percentile(lat, 50):.3f} p99 {np.percentile(lat, 99):.3f}")
    # continuous batching: batches of different streams run at the same time
    assert np.all(times["dev_start_ns"] <= times["dev_end_ns"])
    pairs = _device_overlaps(times)
    say(f"{len(np.unique(times['batch']))} batches, {pairs} pairs overlapping on the device")
    assert pairs >= 1


def test_retained_outputs_in_the_arena():
    """Arena mode with retained outputs: completed requests keep their
    ciphertexts in the server's memory until released, where the caller reads
    them (equal to separate launches and, sampled, to the oracle); held
    outputs count against the budget, so a request that needs their memory
    is admitted only after a release."""
    torch = torch_cuda()
    ctxs = [gpu_ctx(n) for n in NAMES]
    tr = make_trace(6, 1000.0, W_MIXED.params, seed=14, max_count=4)
    d_slots = to_dev(tr.slots)
    torch.cuda.synchronize()
    sizes = [int(tr.n_pt[r]) * 2 * ctxs[int(tr.ctx_idx[r])].L * ctxs[int(tr.ctx_idx[r])].n for r in range(len(tr))]
    held = [(s * 8 + 255) // 256 * 256 for s in sizes]     # bytes each request holds
    budget = max(held)                                      # the largest request fits alone
    srv = zinc.Server(ctxs, zinc.ZINC_SCHEME_ZINC, d_slots, None, n_streams=2, max_batch=8, hbm_budget=budget,
                      retain_outputs=True)
    say("retained outputs: submit, read, release")
    tickets = [srv.submit(int(tr.ctx_idx[r]), int(tr.n_pt[r]), int(tr.slot_off[r]), int(tr.ct_id[r]))
               for r in range(len(tr))]
    for r, tk in enumerate(tickets):
        while srv.query(tk) is None:
            srv.progress()
        if r + 1 < len(tr) and held[r] + held[r + 1] > budget:   # the next one waits for this one's memory
            for _ in range(50):
                srv.progress()
            assert srv.query(tickets[r + 1]) is None
        out = torch.empty(sizes[r], dtype=torch.int64, device="cuda")
        srv.read_output(tk, out)
        got = from_dev(out)
        assert np.array_equal(got, _separate(ctxs, tr, r, zinc.ZINC_SCHEME_ZINC)), r
        if r < 2:
            _oracle_check_request(tr, r, zinc.ZINC_SCHEME_ZINC, got)
        srv.release(tk)
        with pytest.raises(zinc.ZincError) as e:
            srv.release(tk)
        assert e.value.status == zinc.ZINC_E_STATE
    srv.drain()
    srv.close()
