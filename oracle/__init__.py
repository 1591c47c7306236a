"""CPU oracle for batched CKKS / Zinc encryption (arXiv 2408.07304).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library: its own C file (``zinc_oracle.c``) and its own discrete
Gaussian table (computed here with mpmath).

Every function cites the passage of the paper it follows:
  * Gen (Eq. 7), vanilla Enc (Eq. 8), Enc_z (Algorithm 1), Dec (the equation
    after Algorithm 1), homomorphic add (Eq. 2);
  * distributions R_q, chi (sigma = 3.2), R_2 (Polynomials and Distributions);
  * the RNS / DFT structure of the Theoretical Analysis section;
  * CKKS encoding, which the paper takes from the CKKS paper (Scheme
    Flexibility section) -- the canonical-embedding definition is used;
  * the BFV (Eq. 12) and BGV (Eq. 13) forms of the same section: BFV's
    Delta = floor(Q / t) scaling with exact rounding on decryption, BGV's
    errors scaled by t with the centred CRT value reduced mod t, and the
    standard batch (slot) encoding mod a prime t = 1 (mod 2N) that both use
    for vector plaintexts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zinc_oracle.c")
_LIB = os.path.join(_HERE, "libzinc_oracle.so")

KEY_ID = (1 << 64) - 1
ZERO_ID = (1 << 64) - 2
TAG_SK, TAG_A, TAG_EPK, TAG_U, TAG_E1, TAG_E2, TAG_E1Z, TAG_E2Z = 1, 2, 3, 4, 5, 6, 7, 8
CDT_LEN = 38
TAIL = 19  # floor(6 sigma) for sigma = 3.2


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f64p = ctypes.POINTER(ctypes.c_double)


class _Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_moduli", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("scale", ctypes.c_double),
                ("q", ctypes.c_uint64 * 32), ("psi", ctypes.c_uint64 * 32),
                ("cdt", ctypes.c_uint64 * CDT_LEN), ("noise_t", ctypes.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)          # (re)compile when missing or older than the C source
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        sigs = {
            "oracle_mulmod": (ctypes.c_uint64, [ctypes.c_uint64] * 3),
            "oracle_powmod": (ctypes.c_uint64, [ctypes.c_uint64] * 3),
            "oracle_is_prime": (ctypes.c_int, [ctypes.c_uint64]),
            "oracle_choose_moduli": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u64p]),
            "oracle_find_psi": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint32]),
            "oracle_ntt_forward": (None, [_u64p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64]),
            "oracle_ntt_inverse": (None, [_u64p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64]),
            "oracle_philox4x32_10": (None, [_u32p, _u32p, _u32p]),
            "oracle_sample_ternary": (None, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                             ctypes.c_uint32, _i64p]),
            "oracle_sample_gaussian": (None, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                              ctypes.c_uint32, _u64p, _i64p]),
            "oracle_sample_uniform": (None, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                             ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, _u64p]),
            "oracle_keygen": (None, [P, _u64p, _u64p]),
            "oracle_encrypt_vanilla": (None, [P, _u64p, _u64p, ctypes.c_uint64, _u64p]),
            "oracle_zinc_precompute": (None, [P, _u64p, _u64p]),
            "oracle_encrypt_zinc": (None, [P, _u64p, _u64p, ctypes.c_uint64, _u64p]),
            "oracle_decrypt": (None, [P, _u64p, _u64p, _u64p]),
            "oracle_add": (None, [P, _u64p, _u64p, _u64p]),
            "oracle_elementwise_zinc": (None, [P, _u64p, _u64p, _u64p]),
            "oracle_encrypt_vanilla_sp": (None, [P, _u64p, _u64p, ctypes.c_uint64, _u64p]),
            "oracle_elementwise_vanilla": (None, [P, _u64p, _u64p, _u64p, _u64p]),
            "oracle_encode": (None, [P, _f64p, ctypes.c_uint32, _i64p, _f64p]),
            "oracle_decode": (None, [P, _i64p, _f64p]),
            "oracle_to_rns": (None, [P, _i64p, ctypes.c_uint32, _u64p]),
            "oracle_encrypt_slots": (None, [P, ctypes.c_int, _u64p, _f64p, ctypes.c_uint32,
                                            ctypes.c_uint64, _u64p]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------------------
# discrete Gaussian table (chi, sigma = 3.2)
# ---------------------------------------------------------------------------

def cdt_table(sigma: float = 3.2, tail: int = TAIL) -> np.ndarray:
    """Cumulative table of chi, the discrete Gaussian of standard deviation
    sigma (Polynomials and Distributions), restricted to |x| <= tail:
    T[i] = floor(2^64 * sum_{x=-tail}^{-tail+i} rho(x) / S), i < 2*tail,
    rho(x) = exp(-x^2 / (2 sigma^2)), S = sum_{|x|<=tail} rho(x).
    Computed with 60-digit mpmath arithmetic."""
    import mpmath
    with mpmath.workdps(60):
        s = mpmath.mpf(str(sigma))
        rho = [mpmath.exp(-(mpmath.mpf(x) ** 2) / (2 * s * s)) for x in range(-tail, tail + 1)]
        total = mpmath.fsum(rho)
        out = []
        acc = mpmath.mpf(0)
        two64 = mpmath.mpf(2) ** 64
        for i in range(2 * tail):
            acc += rho[i]
            out.append(int(mpmath.floor(two64 * acc / total)))
    return np.array(out, dtype=np.uint64)


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

def choose_moduli(log_n: int, bits) -> list[int]:
    """Moduli rule: per bit size, the largest unused prime q < 2^b, q = 1 mod 2N."""
    b = np.array(bits, dtype=np.uint32)
    out = np.zeros(len(bits), dtype=np.uint64)
    rc = lib().oracle_choose_moduli(log_n, len(bits), _p(b, _u32p), _p(out, _u64p))
    if rc != 0:
        raise ValueError(f"oracle_choose_moduli failed ({rc})")
    return [int(x) for x in out]


def find_psi(q: int, log_n: int) -> int:
    return int(lib().oracle_find_psi(q, log_n))


def is_prime(n: int) -> bool:
    return bool(lib().oracle_is_prime(n))


class Params:
    """Parameter set: ring degree N = 2^log_n, moduli (last one special), scale
    Delta, scheme seed.  L = M - 1 data limbs."""

    def __init__(self, log_n: int, bits=None, scale: float = 2.0 ** 40, seed: int = 0,
                 moduli=None, sigma: float = 3.2, bgv_t: int = 1):
        self.log_n = log_n
        self.n = 1 << log_n
        self.moduli = list(moduli) if moduli is not None else choose_moduli(log_n, bits)
        self.M = len(self.moduli)
        self.L = self.M - 1
        self.scale = float(scale)
        self.seed = int(seed)
        self.psi = [find_psi(q, log_n) for q in self.moduli]
        self.cdt = cdt_table(sigma)
        s = _Params()
        s.log_n, s.n_moduli, s.seed, s.scale = log_n, self.M, self.seed, self.scale
        for i, q in enumerate(self.moduli):
            s.q[i] = q
            s.psi[i] = self.psi[i]
        for i in range(CDT_LEN):
            s.cdt[i] = int(self.cdt[i])
        self.noise_t = int(bgv_t)            # BGV: errors scaled by the plaintext modulus t
        s.noise_t = self.noise_t
        self._c = s

    @property
    def data_moduli(self):
        return self.moduli[: self.L]

    def ref(self):
        return ctypes.byref(self._c)


# ---------------------------------------------------------------------------
# primitives
# ---------------------------------------------------------------------------

def philox(ctr, key) -> list[int]:
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(o, _u32p))
    return [int(x) for x in o]


def ntt_forward(a, log_n: int, q: int, psi: int) -> np.ndarray:
    x = np.array(a, dtype=np.uint64).copy()
    lib().oracle_ntt_forward(_p(x, _u64p), log_n, q, psi)
    return x


def ntt_inverse(a, log_n: int, q: int, psi: int) -> np.ndarray:
    x = np.array(a, dtype=np.uint64).copy()
    lib().oracle_ntt_inverse(_p(x, _u64p), log_n, q, psi)
    return x


def sample_ternary(seed: int, ct_id: int, tag: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int64)
    lib().oracle_sample_ternary(seed, ct_id, tag, n, _p(out, _i64p))
    return out


def sample_gaussian(seed: int, ct_id: int, tag: int, n: int, cdt=None) -> np.ndarray:
    t = np.ascontiguousarray(cdt_table() if cdt is None else cdt, dtype=np.uint64)
    out = np.zeros(n, dtype=np.int64)
    lib().oracle_sample_gaussian(seed, ct_id, tag, n, _p(t, _u64p), _p(out, _i64p))
    return out


def sample_uniform(seed: int, ct_id: int, tag: int, limb: int, n: int, q: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    lib().oracle_sample_uniform(seed, ct_id, tag, limb, n, q, _p(out, _u64p))
    return out


# ---------------------------------------------------------------------------
# scheme
# ---------------------------------------------------------------------------

def keygen(P: Params):
    """Gen (Eq. 7).  Returns (s_hat [M][N], pk [2][M][N]) in the NTT domain."""
    sh = np.zeros((P.M, P.n), dtype=np.uint64)
    pk = np.zeros((2, P.M, P.n), dtype=np.uint64)
    lib().oracle_keygen(P.ref(), _p(sh, _u64p), _p(pk, _u64p))
    return sh, pk


def encrypt_vanilla(P: Params, pk, pt, ct_id: int) -> np.ndarray:
    """Eq. 8 on one plaintext pt [L][N] (coefficient-domain residues)."""
    pk = np.ascontiguousarray(pk, dtype=np.uint64)
    pt = np.ascontiguousarray(pt, dtype=np.uint64)
    ct = np.zeros((2, P.L, P.n), dtype=np.uint64)
    lib().oracle_encrypt_vanilla(P.ref(), _p(pk, _u64p), _p(pt, _u64p), ct_id, _p(ct, _u64p))
    return ct


def encrypt_vanilla_sp(P: Params, pk, pt, ct_id: int) -> np.ndarray:
    """Eq. 8 over the whole chain, then division by the special prime with
    rounding down to the L data limbs, then + m (a SEAL-style vanilla)."""
    pk = np.ascontiguousarray(pk, dtype=np.uint64)
    pt = np.ascontiguousarray(pt, dtype=np.uint64)
    ct = np.zeros((2, P.L, P.n), dtype=np.uint64)
    lib().oracle_encrypt_vanilla_sp(P.ref(), _p(pk, _u64p), _p(pt, _u64p), ct_id, _p(ct, _u64p))
    return ct


def zinc_precompute(P: Params, pk) -> np.ndarray:
    """Zinc precomputation: cache one Enc(0) (vanilla, identifier ZERO_ID)."""
    pk = np.ascontiguousarray(pk, dtype=np.uint64)
    z = np.zeros((2, P.L, P.n), dtype=np.uint64)
    lib().oracle_zinc_precompute(P.ref(), _p(pk, _u64p), _p(z, _u64p))
    return z


def encrypt_zinc(P: Params, zero, pt, ct_id: int) -> np.ndarray:
    """Algorithm 1 (Enc_z) on one plaintext."""
    zero = np.ascontiguousarray(zero, dtype=np.uint64)
    pt = np.ascontiguousarray(pt, dtype=np.uint64)
    ct = np.zeros((2, P.L, P.n), dtype=np.uint64)
    lib().oracle_encrypt_zinc(P.ref(), _p(zero, _u64p), _p(pt, _u64p), ct_id, _p(ct, _u64p))
    return ct


def elementwise_zinc(P: Params, zero, hat) -> np.ndarray:
    """Algorithm 1's additions alone, in the NTT domain: [zero + hat]_q, with
    hat = (NTT(m + e1'), NTT(e2')) as [2][L][N] residues."""
    zero = np.ascontiguousarray(zero, dtype=np.uint64)
    hat = np.ascontiguousarray(hat, dtype=np.uint64)
    ct = np.zeros((2, P.L, P.n), dtype=np.uint64)
    lib().oracle_elementwise_zinc(P.ref(), _p(zero, _u64p), _p(hat, _u64p), _p(ct, _u64p))
    return ct


def elementwise_vanilla(P: Params, pk, uhat, hat) -> np.ndarray:
    """Eq. 8's products and additions alone, in the NTT domain:
    (pk1 u_hat + hat1, pk2 u_hat + hat2) mod q_l over the L data limbs."""
    pk = np.ascontiguousarray(pk, dtype=np.uint64)
    uhat = np.ascontiguousarray(uhat, dtype=np.uint64)
    hat = np.ascontiguousarray(hat, dtype=np.uint64)
    ct = np.zeros((2, P.L, P.n), dtype=np.uint64)
    lib().oracle_elementwise_vanilla(P.ref(), _p(pk, _u64p), _p(uhat, _u64p), _p(hat, _u64p), _p(ct, _u64p))
    return ct


def decrypt(P: Params, s_hat, ct) -> np.ndarray:
    """Dec(c) = [c1 + c2 sk]_q, back in the coefficient domain ([L][N] residues)."""
    s_hat = np.ascontiguousarray(s_hat, dtype=np.uint64)
    ct = np.ascontiguousarray(ct, dtype=np.uint64)
    pt = np.zeros((P.L, P.n), dtype=np.uint64)
    lib().oracle_decrypt(P.ref(), _p(s_hat, _u64p), _p(ct, _u64p), _p(pt, _u64p))
    return pt


def add(P: Params, a, b) -> np.ndarray:
    """Homomorphic addition (Eq. 2): component-wise modular addition."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.zeros((2, P.L, P.n), dtype=np.uint64)
    lib().oracle_add(P.ref(), _p(a, _u64p), _p(b, _u64p), _p(out, _u64p))
    return out


def encode(P: Params, z):
    """CKKS encoding by definition.  Returns (m int64 [N], x - m float64 [N])."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    m = np.zeros(P.n, dtype=np.int64)
    fr = np.zeros(P.n, dtype=np.float64)
    lib().oracle_encode(P.ref(), _p(z, _f64p), len(z), _p(m, _i64p), _p(fr, _f64p))
    return m, fr


def decode(P: Params, m) -> np.ndarray:
    """CKKS decoding by definition of a centred integer polynomial m [N]."""
    m = np.ascontiguousarray(m, dtype=np.int64)
    z = np.zeros(P.n // 2, dtype=np.float64)
    lib().oracle_decode(P.ref(), _p(m, _i64p), _p(z, _f64p))
    return z


def to_rns(P: Params, m, n_limbs: int | None = None) -> np.ndarray:
    L = P.L if n_limbs is None else n_limbs
    m = np.ascontiguousarray(m, dtype=np.int64)
    pt = np.zeros((L, P.n), dtype=np.uint64)
    lib().oracle_to_rns(P.ref(), _p(m, _i64p), L, _p(pt, _u64p))
    return pt


def encrypt_slots(P: Params, scheme: int, key, z, ct_id: int) -> np.ndarray:
    """Encode then encrypt one slot vector; scheme 0 = vanilla (key = pk),
    1 = Zinc (key = cached zero), 2 = vanilla with division by the special
    prime (key = pk)."""
    key = np.ascontiguousarray(key, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    ct = np.zeros((2, P.L, P.n), dtype=np.uint64)
    lib().oracle_encrypt_slots(P.ref(), scheme, _p(key, _u64p), _p(z, _f64p), len(z), ct_id,
                               _p(ct, _u64p))
    return ct


def bfv_delta(P: Params, t: int) -> int:
    """BFV's scale Delta = floor(Q / t), Q the product of the data moduli
    (Scheme Flexibility section, Eq. 12)."""
    Q = 1
    for q in P.data_moduli:
        Q *= int(q)
    return Q // t


def bfv_encode(P: Params, t: int, m) -> np.ndarray:
    """BFV plaintext scaling: residues of Delta * (m mod t) per data limb,
    [L][N] (coefficient encoding: one element of Z_t per ring coefficient)."""
    d = bfv_delta(P, t)
    return np.array([[(d * (int(x) % t)) % int(q) for x in m] for q in P.data_moduli], dtype=np.uint64)


def bfv_decode(P: Params, t: int, pt) -> np.ndarray:
    """BFV decoding of decrypted residues [L][N]: x = CRT value in [0, Q),
    m = round(t x / Q) mod t (halves rounded up), centred to (-t/2, t/2]."""
    qs = [int(q) for q in P.data_moduli]
    Q = 1
    for q in qs:
        Q *= q
    basis = [(Q // q) * pow(Q // q, -1, q) for q in qs]
    out = []
    for k in range(P.n):
        x = sum(int(pt[l][k]) * basis[l] for l in range(len(qs))) % Q
        r = ((2 * t * x + Q) // (2 * Q)) % t
        out.append(r - t if r > t // 2 else r)
    return np.array(out, dtype=np.int64)


def bgv_encode(P: Params, t: int, m) -> np.ndarray:
    """BGV plaintext: residues of (m mod t) per data limb, [L][N]."""
    return np.array([[(int(x) % t) % int(q) for x in m] for q in P.data_moduli], dtype=np.uint64)


def bgv_decode(P: Params, t: int, pt) -> np.ndarray:
    """BGV decoding (Eq. 13): the centred CRT value of the decrypted residues,
    reduced mod t and centred to (-t/2, t/2]."""
    out = []
    for x in crt_centered(P, pt):
        r = x % t
        out.append(r - t if r > t // 2 else r)
    return np.array(out, dtype=np.int64)


# ---------------------------------------------------------------------------
# Batch (slot) encoding of BFV and BGV plaintexts.  The paper leaves encoding
# to those schemes' own papers (Scheme Flexibility section); the batch
# encoding used here is the standard one: for a prime t = 1 (mod 2N), Z_t[X] /
# (X^N + 1) splits into N copies of Z_t, one per primitive 2N-th root of unity
# zeta^e (e odd), and a plaintext m carries the slot values m(zeta^e).
# ---------------------------------------------------------------------------
def batch_exponents(log_n: int) -> list[int]:
    """Slot j's evaluation point zeta^(e_j) (mod 2N): e_i = 3^i for i < N/2 and
    e_(N/2 + i) = -3^i.  3 has order N/2 mod 2N and -1 is not a power of 3,
    so the N exponents are the N odd residues, and X -> X^3 rotates each half
    by one slot."""
    n = 1 << log_n
    two_n = 2 * n
    pw = [pow(3, i, two_n) for i in range(n // 2)]
    return pw + [(two_n - e) % two_n for e in pw]


def _brv(x: int, bits: int) -> int:
    return int(format(x, f"0{bits}b")[::-1], 2) if bits else 0


def _batch_index(log_n: int) -> list[int]:
    """Position of each slot in the oracle's NTT output, whose entry k is the
    evaluation at psi^(2 brv(k) + 1) (ntt_forward)."""
    return [_brv((e - 1) // 2, log_n) for e in batch_exponents(log_n)]


def batch_zeta(log_n: int, t: int) -> int:
    """zeta: the smallest primitive 2N-th root of unity mod t (the moduli's rule)."""
    if not is_prime(t) or t % (2 << log_n) != 1:
        raise ValueError("batch encoding needs a prime t = 1 mod 2N")
    return find_psi(t, log_n)


def batch_encode(log_n: int, t: int, slots) -> np.ndarray:
    """Slot values (any integers, taken mod t) -> the coefficients in [0, t) of
    the m in Z_t[X]/(X^N + 1) with m(zeta^(e_j)) = slots[j] mod t."""
    hat = np.zeros(1 << log_n, dtype=np.uint64)
    for j, k in enumerate(_batch_index(log_n)):
        hat[k] = int(slots[j]) % t
    return ntt_inverse(hat, log_n, t, batch_zeta(log_n, t)).astype(np.int64)


def batch_decode(log_n: int, t: int, m) -> np.ndarray:
    """Coefficients (any integers, taken mod t) -> slot values m(zeta^(e_j)) mod
    t, centred to (-t/2, t/2]."""
    a = np.array([int(x) % t for x in m], dtype=np.uint64)
    hat = ntt_forward(a, log_n, t, batch_zeta(log_n, t))
    out = []
    for k in _batch_index(log_n):
        r = int(hat[k])
        out.append(r - t if r > t // 2 else r)
    return np.array(out, dtype=np.int64)


def crt_centered(P: Params, pt, limbs: int | None = None) -> list[int]:
    """Exact centred lift of RNS residues [L][N] to integers in (-Q/2, Q/2]
    (Chinese remaindering with Python integers)."""
    L = P.L if limbs is None else limbs
    qs = [int(q) for q in P.moduli[:L]]
    Q = 1
    for q in qs:
        Q *= q
    basis = []
    for q in qs:
        Qi = Q // q
        basis.append(Qi * pow(Qi, -1, q))
    rows = [[int(v) for v in pt[l]] for l in range(L)]
    out = []
    for k in range(P.n):
        x = sum(rows[l][k] * basis[l] for l in range(L)) % Q
        if x > Q // 2:
            x -= Q
        out.append(x)
    return out
