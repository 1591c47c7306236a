"""BFV on the GPU contexts (Scheme Flexibility section, Eq. 12): the scaled
encoding bit-exact against the oracle, the RNS scale-and-round decoding equal
to the oracle's exact big-integer rounding, and Zinc and vanilla encryptions
of BFV plaintexts decrypting and decoding to the message."""
import numpy as np
import pytest

import oracle
import paper_2408_07304_amd as zinc
from gpu_util import empty_u64, from_dev, gpu_ctx, ids, oracle_keys, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

NAMES = ["n4096", "n8192", "n16384", "n32768"]
TS = [257, 65537, (1 << 20) + 7]


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.mark.parametrize("name", NAMES)
def test_bfv_round_trip_and_parity(name):
    torch = torch_cuda()
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    B = 3
    for t in TS:
        rng = np.random.default_rng(t + P.n)
        m = rng.integers(-(t // 2), t // 2 + 1, size=(B, P.n))
        m[0, :5] = [0, 1, -1, t // 2, -(t // 2)]
        say(f"{name} BFV t={t}")
        pt = empty_u64(B, P.L, P.n)
        c.bfv_encode(t, to_dev(m), pt)
        got_pt = from_dev(pt)
        for b in range(B):
            assert np.array_equal(got_pt[b], oracle.bfv_encode(P, t, m[b])), (t, b)
        for scheme in (zinc.ZINC_SCHEME_ZINC, zinc.ZINC_SCHEME_VANILLA):
            ct = empty_u64(B, 2, P.L, P.n)
            (c.encrypt if scheme == zinc.ZINC_SCHEME_ZINC else c.encrypt_vanilla)(pt, ids([1, 2, 3]), ct)
            dec = empty_u64(B, P.L, P.n)
            c.decrypt(ct, dec)
            out = torch.empty((B, P.n), dtype=torch.int64, device="cuda")
            c.bfv_decode(t, dec, out)
            got = from_dev(out, np.int64)
            assert np.array_equal(got, m), (t, scheme)
            if scheme == zinc.ZINC_SCHEME_ZINC:          # decoding parity on the same residues
                d0 = from_dev(dec)[0]
                assert np.array_equal(got[0], oracle.bfv_decode(P, t, d0))


def test_bfv_argument_errors():
    torch = torch_cuda()
    c = gpu_ctx("n4096")
    m = torch.zeros((1, c.n), dtype=torch.int64, device="cuda")
    pt = empty_u64(1, c.L, c.n)
    for t in (0, 1, 1 << 32, int(oracle_keys("n4096")[0].data_moduli[0])):
        with pytest.raises(zinc.ZincError) as e:
            c.bfv_encode(t, m, pt)
        assert e.value.status == zinc.ZINC_E_INVAL
        with pytest.raises(zinc.ZincError) as e:
            c.bfv_decode(t, pt, m)
        assert e.value.status == zinc.ZINC_E_INVAL
