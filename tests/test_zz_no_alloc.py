"""The allocation-free special-prime entry point (zinc_encrypt_vanilla_sp_noalloc)
against the allocating one (zinc_encrypt_vanilla_sp), through the C ABI: two
calls in a row on one GPU, the second with a smaller batch, each bit-exact;
a call at the static scratch's full capacity; a batch one above it refused.
N = 8192 runs the one-workgroup kernel, N = 32768 the split kernel."""
import numpy as np
import pytest

import paper_2408_07304_amd as zinc
from gpu_util import empty_u64, from_dev, gpu_ctx, ids, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def _pt(c, count, seed):
    rng = np.random.default_rng(seed)
    return np.stack([np.stack([rng.integers(0, q, size=c.n, dtype=np.uint64) for q in c.moduli[:c.L]])
                     for _ in range(count)])


@pytest.mark.parametrize("name", ["n8192", "n32768"])
def test_noalloc_equals_allocating_entry_point(name):
    torch_cuda()
    c = gpu_ctx(name)
    for batch, seed, first in ((6, 1, 100), (3, 2, 900)):          # the second call is smaller
        pt = to_dev(_pt(c, batch, seed))
        d_ids = ids(range(first, first + batch))
        got, want = empty_u64(batch, 2, c.L, c.n), empty_u64(batch, 2, c.L, c.n)
        say(f"{name} no-alloc special-prime vanilla, batch {batch}")
        c.encrypt_vanilla_sp_noalloc(pt, d_ids, got)
        c.encrypt_vanilla_sp(pt, d_ids, want)
        assert np.array_equal(from_dev(got), from_dev(want)), (name, batch)
    assert c.device_errors() == 0


def test_noalloc_full_capacity_and_limit():
    torch = torch_cuda()
    c = gpu_ctx("n32768")
    cap = SCRATCH_BYTES // (3 * c.n * 8)
    assert cap == 85
    pt = to_dev(_pt(c, cap, 3))
    d_ids = ids(range(5000, 5000 + cap))
    got, want = empty_u64(cap, 2, c.L, c.n), empty_u64(cap, 2, c.L, c.n)
    say(f"n32768 no-alloc at capacity ({cap} ciphertexts)")
    c.encrypt_vanilla_sp_noalloc(pt, d_ids, got)
    c.encrypt_vanilla_sp(pt, d_ids, want)
    assert torch.equal(got, want)
    del got, want, pt
    small = gpu_ctx("n4096")
    cap4 = SCRATCH_BYTES // (3 * small.n * 8)
    pt = empty_u64(cap4 + 1, small.L, small.n)
    out = empty_u64(cap4 + 1, 2, small.L, small.n)
    with pytest.raises(zinc.ZincError) as e:
        small.encrypt_vanilla_sp_noalloc(pt, ids(range(cap4 + 1)), out)
    assert e.value.status == zinc.ZINC_E_RANGE
    assert str(cap4) in str(e.value)
