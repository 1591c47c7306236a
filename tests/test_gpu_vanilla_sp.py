"""Vanilla encryption with division by the special prime (the SEAL-style
baseline): bit-exact against the oracle from a shared integer plaintext, the
fused launch equal to encode followed by encrypt, decryption within the noise
bound, and the argument and state errors."""
import numpy as np
import pytest

import oracle
import paper_2408_07304_amd as zinc
from gpu_util import empty_u64, from_dev, gpu_ctx, ids, oracle_keys, to_dev, torch_cuda
from paper_2408_07304_amd.workloads import PARAM_SETS, W_MAIN, make_slots

pytestmark = pytest.mark.gpu

# N = 32768 runs the split-transform kernel; n32768_q16 is the 881-bit chain
NAMES = ["n4096", "n8192", "n16384", "n32768", "n32768_q16"]


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.mark.parametrize("name", NAMES)
def test_vanilla_sp_from_plaintext_bit_exact(name):
    torch_cuda()
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    rng = np.random.default_rng(41)
    B = 3
    pt = np.stack([np.stack([rng.integers(0, q, size=P.n, dtype=np.uint64) for q in P.data_moduli])
                   for _ in range(B)])
    idv = [5, 0, 2 ** 35 + 7]
    out = empty_u64(B, 2, P.L, P.n)
    say(f"{name} special-prime vanilla from plaintext")
    c.encrypt_vanilla_sp(to_dev(pt), ids(idv), out)
    got = from_dev(out)
    for i in range(B):
        assert np.array_equal(got[i], oracle.encrypt_vanilla_sp(P, pk, pt[i], idv[i])), i


@pytest.mark.parametrize("name", NAMES)
def test_vanilla_sp_fused_and_round_trip(name):
    torch_cuda()
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    ps = PARAM_SETS[name]
    z = make_slots(W_MAIN, 4, ps)
    d_ids = ids(range(60, 64))
    f = empty_u64(4, 2, P.L, P.n)
    u = empty_u64(4, 2, P.L, P.n)
    pt = empty_u64(4, P.L, P.n)
    say(f"{name} special-prime vanilla fused vs unfused")
    c.encrypt_slots(zinc.ZINC_SCHEME_VANILLA_SP, to_dev(z), d_ids, f)
    c.encode(to_dev(z), pt)
    c.encrypt_vanilla_sp(pt, d_ids, u)
    assert np.array_equal(from_dev(f), from_dev(u))
    # decrypt + decode recovers the slots; the rounding noise is far below the
    # noise of the plain vanilla encryption
    torch = torch_cuda()
    dec = empty_u64(4, P.L, P.n)
    c.decrypt(f, dec)
    zd = torch.empty((4, P.n // 2), dtype=torch.float64, device="cuda")
    c.decode(dec, zd)
    err = np.abs(from_dev(zd, np.float64) - z).max()
    # rounding noise: at most (1 + |s|_1) / 2 per coefficient, |s|_1 ~ 2N/3
    bound = 8 * np.sqrt(P.n) * (1 + P.n / 3) / ps.scale + 1e-9
    say(f"{name} round trip error {err:.3g} (bound {bound:.3g})")
    assert err < bound, err


def test_vanilla_sp_errors():
    torch_cuda()
    from paper_2408_07304_amd.workloads import P4096
    fresh = zinc.context_for(P4096)
    with pytest.raises(zinc.ZincError) as e:
        fresh.encrypt_vanilla_sp(empty_u64(1, P4096.limbs, P4096.n), ids([0]), empty_u64(1, 2, P4096.limbs, P4096.n))
    assert e.value.status == zinc.ZINC_E_STATE
    fresh.close()
