"""Edge cases of the batch entry points: empty batches (every entry point, and
a plan with no items) are no-ops; messages whose coefficients exceed 2^52 take
the integer route of the fused kernel and still equal encode-then-encrypt;
the largest allowed ciphertext identifier is bit-exact against the oracle;
reserved identifiers (2^63 and above) are refused by every encryption
entry point without touching their ciphertexts."""
import numpy as np
import pytest

import oracle
import paper_2408_07304_amd as zinc
from gpu_util import empty_u64, from_dev, gpu_ctx, ids, oracle_keys, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def test_empty_batches_are_no_ops():
    torch = torch_cuda()
    c = gpu_ctx("n4096")
    L, n = c.L, c.n
    z0 = torch.empty((0, n // 2), dtype=torch.float64, device="cuda")
    i0 = torch.empty((0,), dtype=torch.int64, device="cuda")
    pt0 = empty_u64(0, L, n)
    ct0 = empty_u64(0, 2, L, n)
    m0 = torch.empty((0, n), dtype=torch.int64, device="cuda")
    sl0 = torch.empty((0, n // 2), dtype=torch.float64, device="cuda")
    say("empty batches")
    c.encode(z0, pt0)
    for s in (zinc.ZINC_SCHEME_VANILLA, zinc.ZINC_SCHEME_ZINC, zinc.ZINC_SCHEME_VANILLA_SP):
        c.encrypt_slots(s, z0, i0, ct0)
    c.encrypt(pt0, i0, ct0)
    c.encrypt_vanilla(pt0, i0, ct0)
    c.encrypt_vanilla_sp(pt0, i0, ct0)
    c.decrypt(ct0, pt0)
    c.decode(pt0, sl0)
    c.add(ct0, ct0, ct0)
    c.elementwise_zinc(ct0, ct0)
    c.elementwise_vanilla(pt0, ct0, ct0)
    c.ntt_forward(0, empty_u64(0, n))
    c.ntt_inverse(0, empty_u64(0, n))
    c.sample(1, 7, 0, i0, empty_u64(0, n))
    c.bfv_encode(257, m0, pt0)
    c.bfv_decode(257, pt0, m0)
    c.batch_encode(65537, m0, m0)
    c.batch_decode(65537, m0, m0)
    plan = zinc.Plan([c], [], zinc.ZINC_SCHEME_ZINC)
    plan.launch(None, None)
    plan.close()
    torch.cuda.synchronize()
    assert c.device_errors() == 0


@pytest.mark.parametrize("scheme", [zinc.ZINC_SCHEME_ZINC, zinc.ZINC_SCHEME_VANILLA])
def test_large_messages_take_the_integer_route(scheme):
    """Delta = 2^25 and slot values up to 2^34: coefficients near 2^54, above
    the 2^52 limit of the FP64 message input and the 2^51 limit of the
    encoder's bias conversion, below the 2^62 range limit (and below
    Q ~ 2^60, so the residues still define the message)."""
    torch_cuda()
    c = gpu_ctx("n4096")
    P = oracle_keys("n4096")[0]
    rng = np.random.default_rng(31)
    B = 4
    z = rng.uniform(-2.0 ** 34, 2.0 ** 34, size=(B, P.n // 2))
    d_ids = ids(range(100, 100 + B))
    f, u = empty_u64(B, 2, P.L, P.n), empty_u64(B, 2, P.L, P.n)
    pt = empty_u64(B, P.L, P.n)
    say(f"large messages scheme={scheme}")
    c.encrypt_slots(scheme, to_dev(z), d_ids, f)
    c.encode(to_dev(z), pt)
    (c.encrypt if scheme == zinc.ZINC_SCHEME_ZINC else c.encrypt_vanilla)(pt, d_ids, u)
    assert np.array_equal(from_dev(f), from_dev(u))
    got = from_dev(pt)
    m, _ = oracle.encode(P, z[0])
    assert np.abs(m).max() > 2 ** 52
    # each coefficient is the oracle's integer within a worst-case bound on
    # the FP64 evaluation error at this size, 8 log2(N) 2^-53 max|x| (about
    # 190 here), and the same integer on every limb
    bound = 8 * np.log2(P.n) * 2.0 ** -53 * float(np.abs(m).max()) + 1
    deltas = []
    for l, q in enumerate(P.data_moduli):
        q = int(q)
        d = [(int(g) - int(x)) % q for g, x in zip(got[0, l], m)]
        d = [x - q if x > q // 2 else x for x in d]
        assert max(abs(x) for x in d) <= bound, l
        deltas.append(d)
    assert all(d == deltas[0] for d in deltas)
    assert c.device_errors() == 0


def test_largest_ct_id_bit_exact():
    torch_cuda()
    c = gpu_ctx("n8192")
    P, sh, pk, zero = oracle_keys("n8192")
    rng = np.random.default_rng(32)
    pt = np.stack([np.stack([rng.integers(0, q, size=P.n, dtype=np.uint64) for q in P.data_moduli])
                   for _ in range(2)])
    idv = [(1 << 63) - 1, 0]
    for scheme in (zinc.ZINC_SCHEME_ZINC, zinc.ZINC_SCHEME_VANILLA):
        out = empty_u64(2, 2, P.L, P.n)
        (c.encrypt if scheme == zinc.ZINC_SCHEME_ZINC else c.encrypt_vanilla)(to_dev(pt), ids(idv), out)
        got = from_dev(out)
        for i, cid in enumerate(idv):
            want = (oracle.encrypt_zinc(P, zero, pt[i], cid) if scheme == zinc.ZINC_SCHEME_ZINC
                    else oracle.encrypt_vanilla(P, pk, pt[i], cid))
            assert np.array_equal(got[i], want), (scheme, cid)


@pytest.mark.parametrize("name", ["n4096", "n32768"])
def test_reserved_identifiers_are_refused(name):
    """An identifier of 2^63 or more (the keys' and the cached Enc(0)'s) in a
    direct encryption call: that ciphertext is left unwritten and bit 2 of
    the device error flags is set; the others in the batch are encrypted as
    usual.  Every entry point, both ring-degree families (N = 32768 runs the
    split kernels)."""
    torch = torch_cuda()
    c = gpu_ctx(name)
    P = oracle_keys(name)[0]
    rng = np.random.default_rng(33)
    z = to_dev(rng.uniform(-1, 1, size=(3, P.n // 2)))
    pt = empty_u64(3, P.L, P.n)
    c.encode(z, pt)
    idv = [5, zinc.ZINC_ZERO_ID, 1 << 63]
    d_ids = ids(idv)
    sentinel = -0x5A5A5A5A5A5A5A5B
    assert c.device_errors() == 0
    calls = [("slots vanilla", lambda o: c.encrypt_slots(zinc.ZINC_SCHEME_VANILLA, z, d_ids, o),
              lambda o: c.encrypt_slots(zinc.ZINC_SCHEME_VANILLA, z[:1], d_ids[:1], o)),
             ("slots zinc", lambda o: c.encrypt_slots(zinc.ZINC_SCHEME_ZINC, z, d_ids, o),
              lambda o: c.encrypt_slots(zinc.ZINC_SCHEME_ZINC, z[:1], d_ids[:1], o)),
             ("slots vanilla_sp", lambda o: c.encrypt_slots(zinc.ZINC_SCHEME_VANILLA_SP, z, d_ids, o),
              lambda o: c.encrypt_slots(zinc.ZINC_SCHEME_VANILLA_SP, z[:1], d_ids[:1], o)),
             ("encrypt", lambda o: c.encrypt(pt, d_ids, o), lambda o: c.encrypt(pt[:1], d_ids[:1], o)),
             ("encrypt_vanilla", lambda o: c.encrypt_vanilla(pt, d_ids, o),
              lambda o: c.encrypt_vanilla(pt[:1], d_ids[:1], o)),
             ("encrypt_vanilla_sp", lambda o: c.encrypt_vanilla_sp(pt, d_ids, o),
              lambda o: c.encrypt_vanilla_sp(pt[:1], d_ids[:1], o))]
    for what, batch_call, one_call in calls:
        out = torch.full((3, 2, P.L, P.n), sentinel, dtype=torch.int64, device="cuda")
        say(f"{name} reserved identifiers: {what}")
        batch_call(out)
        assert c.device_errors() & 4, what
        assert c.device_errors() == 0
        got = from_dev(out)
        assert np.all(got[1:].view(np.int64) == sentinel), what
        one = empty_u64(1, 2, P.L, P.n)
        one_call(one)
        assert np.array_equal(got[0], from_dev(one)[0]), what
        assert c.device_errors() == 0
