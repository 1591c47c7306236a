"""Mixed-shape plans: one persistent, graph-captured launch over ciphertexts of
several parameter sets (ring degrees 4096..32768).  Every ciphertext must be
bit-identical to the same ciphertext encrypted alone by its own context's
batch launch, on the first launch (graph capture), on replays, and after
re-capture for new buffers; sampled ciphertexts of every ring degree are also
checked against the oracle's Algorithm 1 / Eq. 8 directly."""
import numpy as np
import pytest

import paper_2408_07304_amd as zinc
from gpu_util import check_fused, empty_u64, from_dev, gpu_ctx, ids, oracle_keys, to_dev, torch_cuda
from paper_2408_07304_amd.workloads import W_MIXED, make_mixed

pytestmark = pytest.mark.gpu

NAMES = ["n4096", "n8192", "n16384", "n32768"]      # order of W_MIXED.params


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def _items(mb):
    return list(zip(mb.ctx_idx.tolist(), mb.slot_off.tolist(), mb.ct_off.tolist(), mb.ct_id.tolist()))


def _oracle_check(mb, i, scheme, seg):
    """Plan ciphertext `seg` of item i against the oracle's encryption of its
    slot vector (c2 bit-exact, c1 under the encoding rule)."""
    name = NAMES[int(mb.ctx_idx[i])]
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    so = int(mb.slot_off[i])
    z = np.asarray(mb.slots[so: so + P.n // 2])
    key = zero if scheme == zinc.ZINC_SCHEME_ZINC else pk
    return check_fused(c, P, scheme, key, z, int(mb.ct_id[i]), seg.reshape(2, P.L, P.n), ("plan item", i))


def _alone(ctxs, mb, i, scheme):
    c = ctxs[int(mb.ctx_idx[i])]
    so = int(mb.slot_off[i])
    z = np.ascontiguousarray(mb.slots[so: so + c.n // 2])[None, :]
    out = empty_u64(1, 2, c.L, c.n)
    c.encrypt_slots(scheme, to_dev(z), ids([int(mb.ct_id[i])]), out)
    return from_dev(out).reshape(-1)


@pytest.mark.parametrize("scheme", [zinc.ZINC_SCHEME_VANILLA, zinc.ZINC_SCHEME_ZINC])
def test_plan_equals_separate_launches(scheme):
    torch = torch_cuda()
    ctxs = [gpu_ctx(n) for n in NAMES]
    mb = make_mixed(W_MIXED, 23)          # partial units of every degree
    assert len(set(mb.ctx_idx.tolist())) == 4
    plan = zinc.Plan(ctxs, _items(mb), scheme)
    d_slots = to_dev(mb.slots)
    d_ct = torch.zeros(mb.ct_words, dtype=torch.int64, device="cuda")
    say(f"plan scheme={scheme}: first launch (capture)")
    plan.launch(d_slots, d_ct)
    got = from_dev(d_ct)
    seen = set()
    for i in range(len(mb.ct_id)):
        c = ctxs[int(mb.ctx_idx[i])]
        off = int(mb.ct_off[i])
        seg = got[off: off + 2 * c.L * c.n]
        assert np.array_equal(seg, _alone(ctxs, mb, i, scheme)), i
        if int(mb.ctx_idx[i]) not in seen:              # first item of each ring degree vs the oracle
            seen.add(int(mb.ctx_idx[i]))
            say(f"plan item {i} (N = {c.n}) vs the oracle")
            _oracle_check(mb, i, scheme, seg)
    say("replay")
    d_ct.zero_()
    plan.launch(d_slots, d_ct)
    assert np.array_equal(from_dev(d_ct), got)
    say("new output buffer (re-capture) and replay")
    d_ct2 = torch.zeros(mb.ct_words, dtype=torch.int64, device="cuda")
    plan.launch(d_slots, d_ct2)
    plan.launch(d_slots, d_ct2)
    assert np.array_equal(from_dev(d_ct2), got)
    plan.close()


def test_plan_argument_errors():
    torch_cuda()
    ctxs = [gpu_ctx("n4096")]
    with pytest.raises(zinc.ZincError) as e:
        zinc.Plan(ctxs, [(1, 0, 0, 0)], zinc.ZINC_SCHEME_ZINC)          # context index out of range
    assert e.value.status == zinc.ZINC_E_INVAL
    with pytest.raises(zinc.ZincError) as e:
        zinc.Plan(ctxs, [(0, 0, 0, 2 ** 63)], zinc.ZINC_SCHEME_ZINC)    # reserved identifier range
    assert e.value.status == zinc.ZINC_E_INVAL
    with pytest.raises(zinc.ZincError) as e:
        zinc.Plan(ctxs, [(0, 0, 0, 0)], 5)
    assert e.value.status == zinc.ZINC_E_INVAL
    fresh = zinc.context_for(__import__("paper_2408_07304_amd.workloads", fromlist=["P4096"]).P4096)
    with pytest.raises(zinc.ZincError) as e:
        zinc.Plan([fresh], [(0, 0, 0, 0)], zinc.ZINC_SCHEME_ZINC)       # no keys yet
    assert e.value.status == zinc.ZINC_E_STATE
    fresh.close()
    empty = zinc.Plan(ctxs, [], zinc.ZINC_SCHEME_ZINC)                  # nothing to do
    empty.launch(None, None)
    empty.close()
    # buffers that end before an item's slots or ciphertext are refused
    torch = torch_cuda()
    c = ctxs[0]
    plan = zinc.Plan(ctxs, [(0, 0, 0, 1), (0, c.n // 2, 2 * c.L * c.n, 2)], zinc.ZINC_SCHEME_ZINC)
    slots = torch.zeros(c.n, dtype=torch.float64, device="cuda")
    ct = torch.zeros(4 * c.L * c.n, dtype=torch.int64, device="cuda")
    for s_, o_ in ((slots[:c.n - 1], ct), (slots, ct[:4 * c.L * c.n - 1])):
        with pytest.raises(zinc.ZincError) as e:
            plan.launch(s_, o_)
        assert e.value.status == zinc.ZINC_E_INVAL
    plan.launch(slots, ct)                                               # exact sizes are accepted
    torch.cuda.synchronize()
    plan.close()


@pytest.mark.parametrize("scheme", [zinc.ZINC_SCHEME_VANILLA, zinc.ZINC_SCHEME_ZINC])
def test_full_mixed_batch_sampled(scheme):
    """The 2048-plaintext mixed batch in the benchmark's launch configuration;
    sampled ciphertexts of every degree compared with separate launches and
    with the oracle."""
    torch = torch_cuda()
    ctxs = [gpu_ctx(n) for n in NAMES]
    mb = make_mixed(W_MIXED)
    plan = zinc.Plan(ctxs, _items(mb), scheme)
    d_slots = to_dev(mb.slots)
    d_ct = torch.empty(mb.ct_words, dtype=torch.int64, device="cuda")
    say(f"full mixed batch ({len(mb.ct_id)} plaintexts, {mb.ct_words * 8 / 2**30:.2f} GiB) scheme={scheme}")
    plan.launch(d_slots, d_ct)
    plan.launch(d_slots, d_ct)
    picks = []
    for k in range(4):
        where = np.nonzero(mb.ctx_idx == k)[0]
        picks += [int(where[0]), int(where[len(where) // 2]), int(where[-1])]
    for i in picks:
        c = ctxs[int(mb.ctx_idx[i])]
        off = int(mb.ct_off[i])
        seg = from_dev(d_ct[off: off + 2 * c.L * c.n].contiguous())
        assert np.array_equal(seg, _alone(ctxs, mb, i, scheme)), i
        say(f"mixed item {i} (N = {c.n}) vs the oracle")
        _oracle_check(mb, i, scheme, seg)
    plan.close()
