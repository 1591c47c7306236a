"""Serving (zinc_server_*, zinc_serve_trace): requests admitted against an HBM
budget and encrypted by continuous batching on several streams.  Served
ciphertexts must be bit-identical to separate launches with the same ct_ids
(which the parity tests tie to the oracle); the scheduler's records must show
submission-order admission, the budget never exceeded and batches within
max_batch."""
import numpy as np
import pytest

import paper_2408_07304_amd as zinc
from gpu_util import empty_u64, from_dev, gpu_ctx, ids, to_dev, torch_cuda
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
    for r in range(len(tr)):
        off = int(tr.ct_off[r])
        ref = _separate(ctxs, tr, r, scheme)
        assert np.array_equal(got[off: off + len(ref)], ref), r


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
    for args, status in [((4, 1, 0, 0), zinc.ZINC_E_INVAL),           # context out of range
                         ((0, 9, 0, 0), zinc.ZINC_E_RANGE),           # above max_batch
                         ((0, 0, 0, 0), zinc.ZINC_E_INVAL),           # empty request
                         ((0, 1, 0, 2 ** 63), zinc.ZINC_E_INVAL),           # ct_id range
                         ((3, 8, 0, 0), zinc.ZINC_E_RANGE)]:          # 8 x 7 MiB > 48 MiB budget
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
