"""Batch (slot) encoding of BFV and BGV plaintexts on the GPU: encoding and
decoding bit-exact against the oracle at every ring degree, in place, two
plaintext moduli on one context, and slot vectors carried through BFV and BGV
encryption (Zinc and vanilla) and back."""
import numpy as np
import pytest

import oracle
import paper_2408_07304_amd as zinc
from gpu_util import empty_u64, from_dev, gpu_ctx, ids, to_dev, torch_cuda
from paper_2408_07304_amd.workloads import PARAM_SETS

pytestmark = pytest.mark.gpu

NAMES = ["n4096", "n8192", "n16384", "n32768"]
TS = [65537, 786433]          # 2^16 + 1 and 3 * 2^18 + 1: both 1 mod 2N for every N here


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def _i64(torch, shape):
    return torch.empty(shape, dtype=torch.int64, device="cuda")


def _centred(v, t):
    r = np.mod(v, t)
    return np.where(r > t // 2, r - t, r)


@pytest.mark.parametrize("name", NAMES)
def test_batch_codec_bit_exact(name):
    torch = torch_cuda()
    c = gpu_ctx(name)
    ln, n = c.info()["log_n"], c.n
    B = 3
    for t in TS:
        say(f"{name} batch codec t={t}")
        rng = np.random.default_rng(t + n)
        v = rng.integers(-2 * t, 2 * t, size=(B, n))
        v[0, :4] = [0, 1, -1, t]
        m = _i64(torch, (B, n))
        c.batch_encode(t, to_dev(v), m)
        got_m = from_dev(m, np.int64)
        for b in (0, B - 1):
            assert np.array_equal(got_m[b], oracle.batch_encode(ln, t, v[b])), (t, b)
        back = _i64(torch, (B, n))
        c.batch_decode(t, m, back)
        assert np.array_equal(from_dev(back, np.int64), _centred(v, t)), t
        # decoding from arbitrary representatives of the coefficients
        w = rng.integers(-(1 << 40), 1 << 40, size=(1, n))
        out = _i64(torch, (1, n))
        c.batch_decode(t, to_dev(w), out)
        assert np.array_equal(from_dev(out, np.int64)[0], oracle.batch_decode(ln, t, w[0])), t
        # in place
        x = to_dev(v)
        c.batch_encode(t, x, x)
        assert np.array_equal(from_dev(x, np.int64), got_m), t


@pytest.mark.parametrize("name", ["n8192", "n32768"])
def test_bfv_slots_through_encryption(name):
    torch = torch_cuda()
    c = gpu_ctx(name)
    n, L, t = c.n, c.L, 65537
    B = 2
    v = np.random.default_rng(5).integers(-(t // 2), t // 2 + 1, size=(B, n))
    m = _i64(torch, (B, n))
    c.batch_encode(t, to_dev(v), m)
    pt = empty_u64(B, L, n)
    c.bfv_encode(t, m, pt)
    for scheme in (zinc.ZINC_SCHEME_ZINC, zinc.ZINC_SCHEME_VANILLA):
        say(f"{name} BFV slots scheme={scheme}")
        ct = empty_u64(B, 2, L, n)
        (c.encrypt if scheme == zinc.ZINC_SCHEME_ZINC else c.encrypt_vanilla)(pt, ids([4, 8]), ct)
        dec = empty_u64(B, L, n)
        c.decrypt(ct, dec)
        mm = _i64(torch, (B, n))
        c.bfv_decode(t, dec, mm)
        c.batch_decode(t, mm, mm)
        assert np.array_equal(from_dev(mm, np.int64), v), scheme


@pytest.mark.parametrize("name,t", [("n8192", 65537), ("n32768", 786433)])
def test_bgv_slots_through_encryption(name, t):
    torch = torch_cuda()
    c = zinc.context_for(PARAM_SETS[name])
    c.set_bgv(t)
    c.keygen()
    c.precompute()
    n, L, B = c.n, c.L, 2
    v = np.random.default_rng(6).integers(-(t // 2), t // 2 + 1, size=(B, n))
    m = _i64(torch, (B, n))
    c.batch_encode(t, to_dev(v), m)
    pt = empty_u64(B, L, n)
    c.bgv_encode(m, pt)
    for scheme in (zinc.ZINC_SCHEME_ZINC, zinc.ZINC_SCHEME_VANILLA):
        say(f"{name} BGV slots scheme={scheme}")
        ct = empty_u64(B, 2, L, n)
        (c.encrypt if scheme == zinc.ZINC_SCHEME_ZINC else c.encrypt_vanilla)(pt, ids([4, 8]), ct)
        dec = empty_u64(B, L, n)
        c.decrypt(ct, dec)
        mm = _i64(torch, (B, n))
        c.bgv_decode(dec, mm)
        c.batch_decode(t, mm, mm)
        assert np.array_equal(from_dev(mm, np.int64), v), scheme


def test_batch_rejects_unsuitable_t():
    torch = torch_cuda()
    c = gpu_ctx("n8192")
    x = _i64(torch, (1, c.n))
    for t in (257, 65536, 40961, (1 << 31) + 1):     # 257 and 40961 are primes but not 1 mod 16384
        for call in (c.batch_encode, c.batch_decode):
            with pytest.raises(zinc.ZincError) as e:
                call(t, x, x)
            assert e.value.status == zinc.ZINC_E_INVAL
