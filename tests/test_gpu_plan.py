"""Mixed-shape plans: one persistent, graph-captured launch over ciphertexts of
several parameter sets (ring degrees 4096..32768).  Every ciphertext must be
bit-identical to the same ciphertext encrypted alone by its own context's
batch launch (which the parity tests check against the oracle), on the first
launch (graph capture), on replays, and after re-capture for new buffers."""
import numpy as np
import pytest

import paper_2408_07304_amd as zinc
from gpu_util import empty_u64, from_dev, gpu_ctx, ids, to_dev, torch_cuda
from paper_2408_07304_amd.workloads import W_MIXED, make_mixed

pytestmark = pytest.mark.gpu

NAMES = ["n4096", "n8192", "n16384", "n32768"]      # order of W_MIXED.params


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def _items(mb):
    return list(zip(mb.ctx_idx.tolist(), mb.slot_off.tolist(), mb.ct_off.tolist(), mb.ct_id.tolist()))


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
    for i in range(len(mb.ct_id)):
        c = ctxs[int(mb.ctx_idx[i])]
        off = int(mb.ct_off[i])
        assert np.array_equal(got[off: off + 2 * c.L * c.n], _alone(ctxs, mb, i, scheme)), i
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
    empty.launch(0, 0)
    empty.close()


@pytest.mark.parametrize("scheme", [zinc.ZINC_SCHEME_VANILLA, zinc.ZINC_SCHEME_ZINC])
def test_full_mixed_batch_sampled(scheme):
    """The 2048-plaintext mixed batch in the benchmark's launch configuration;
    sampled ciphertexts of every degree compared with separate launches."""
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
    plan.close()
