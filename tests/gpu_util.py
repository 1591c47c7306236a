"""Helpers shared by the GPU tests: device buffers for uint64 data (carried in
int64 torch tensors), cached contexts / oracle key material per parameter
set, and the parity rule for FP64 encoding (the tie window and the bound on
the share of coefficients that may round the other way)."""
import functools

import numpy as np
import pytest

import paper_2408_07304_amd as zinc
from paper_2408_07304_amd.workloads import PARAM_SETS


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(a):
    torch = torch_cuda()
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a.copy()).to("cuda")


def from_dev(t, dtype=np.uint64):
    torch_cuda().cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(dtype) if a.dtype == np.int64 and dtype == np.uint64 else a


def empty_u64(*shape):
    torch = torch_cuda()
    return torch.empty(shape, dtype=torch.int64, device="cuda")


def ids(values):
    return to_dev(np.asarray(values, dtype=np.uint64))


@functools.lru_cache(maxsize=None)
def gpu_ctx(name):
    ps = PARAM_SETS[name]
    print(f"[gpu] context {name} keygen+precompute", flush=True)
    c = zinc.context_for(ps)
    c.keygen()
    c.precompute()
    torch_cuda().cuda.synchronize()
    return c


@functools.lru_cache(maxsize=None)
def oracle_keys(name):
    import oracle
    ps = PARAM_SETS[name]
    P = oracle.Params(ps.log_n, ps.bits, ps.scale, ps.seed)
    sh, pk = oracle.keygen(P)
    zero = oracle.zinc_precompute(P, pk)
    return P, sh, pk, zero


# ---------------------------------------------------------------------------
# FP64 encoding parity.  The oracle sums the encoding's defining series in x87
# extended precision; the GPU evaluates it with an FP64 FFT.  Write x for the
# exact coefficient before rounding and e for the GPU's FP64 error.  A
# coefficient can round the other way only when frac(x) lies within |e| of
# 1/2, and then by one.  Under the standard rounding model of a radix-2 FFT
# (independent roundings of relative size at most u = 2^-53 per operation,
# correctly rounded twiddles) the error's rms is about u sqrt(log2 n) rms(x);
# the GPU's route has log2(N) - 2 complex stages plus the real-input
# unscrambling, the twist and the conversion.
# ---------------------------------------------------------------------------
U = 2.0 ** -53


def rms(x):
    x = np.asarray(x, dtype=np.float64)
    return float(np.sqrt(np.mean(x * x))) if x.size else 0.0


def tie_tau(n, x):
    """Half-width of the window around x.5 outside which the GPU's integer must
    equal the oracle's: 4 log2(N) u rms(x), several times the modelled rms
    error (the window is a pointwise test, so it must hold the error's tail)."""
    return 4 * np.log2(n) * U * rms(x)


def mismatch_allowance(n, x, count):
    """Largest number of coefficients, out of `count` with values x, that may
    round the other way.  With the fractions of x equidistributed and
    independent of e, coefficient i differs with probability 2|e_i|, so the
    expected share is 2 E|e| <= 2 rms(e).  rms(e) is taken from the model
    with unit constant, u sqrt(log2 N + 2) rms(x) (two stages added for the
    twist and the unscrambling), giving the expected count
    mu = count * 2 u sqrt(log2 N + 2) rms(x); the allowance adds Poisson
    slack, mu + 4 sqrt(mu) + 4, so that small expected counts do not fail by
    chance."""
    mu = count * 2 * U * np.sqrt(np.log2(n) + 2) * rms(x)
    return mu + 4 * np.sqrt(mu) + 4


def centred(pt0, q):
    v = pt0.astype(object)
    return np.array([int(x) - q if int(x) > q // 2 else int(x) for x in v], dtype=np.int64)


def check_encoding(n, m_gpu, m_oracle, frac, where=""):
    """GPU integers m_gpu (centred) against the oracle's rounded m_oracle with
    the fractions frac = x - m_oracle of the exact values: differences of at
    most one, only inside the tie window, and no more of them than the
    allowance.  Returns the number of differences."""
    m_gpu, m_oracle, frac = (np.asarray(a).reshape(-1) for a in (m_gpu, m_oracle, frac))
    d = m_gpu - m_oracle
    x = m_oracle.astype(np.float64) + frac
    assert np.abs(d).max() <= 1, where
    tau = tie_tau(n, x)
    assert np.all(np.abs(np.abs(frac[d != 0]) - 0.5) <= tau), (where, tau)
    mism = int(np.count_nonzero(d))
    allow = mismatch_allowance(n, x, x.size)
    print(f"[gpu]   encoding {where}: {mism} of {x.size} rounded the other way (allowed {allow:.0f}, "
          f"tie window {tau:.3g})", flush=True)
    assert mism <= allow, (where, mism, allow)
    return mism


def check_fused(c, P, scheme, key, z, cid, got, where=""):
    """One fused ciphertext `got` ([2][L][N]) of slot vector z against the
    oracle's encryption (Algorithm 1 or Eq. 8 after the oracle's encoding):
    c2 bit-exact; c1 equal up to NTT(delta), delta the same integer polynomial
    on every limb (taken with the library's inverse NTT, itself checked
    bit-exact), with entries in {-1, 0, 1} subject to check_encoding's rule."""
    import oracle
    want = oracle.encrypt_slots(P, scheme, key, z, cid)
    assert np.array_equal(got[1], want[1]), where
    if np.array_equal(got[0], want[0]):
        return 0
    m, fr = oracle.encode(P, z)
    delta = None
    for l, q in enumerate(P.data_moduli):
        diff = ((got[0, l].astype(object) - want[0, l].astype(object)) % q).astype(np.uint64)
        d = to_dev(diff[None, :])
        c.ntt_inverse(l, d)
        dl = centred(from_dev(d)[0], q)
        if delta is None:
            delta = dl
        else:
            assert np.array_equal(dl, delta), (where, l)
    return check_encoding(P.n, m + delta, m, fr, where)
