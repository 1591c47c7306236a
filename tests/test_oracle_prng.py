"""Pins of the oracle's randomness: Philox4x32-10 against the published
zero-input known answer and against rocRAND's independent engine; the three
samplers of the Polynomials and Distributions section (R_2 ternary, chi with
sigma = 3.2, R_q uniform) against their distributions; the cumulative table of
chi against an independent decimal-arithmetic computation."""
import os
import shutil
import subprocess
import tempfile
from decimal import Decimal, getcontext

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_zero_known_answer(orc):
    # Philox4x32-10 at counter 0, key 0 (Salmon et al., SC'11 reference output)
    assert orc.philox([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-I/opt/rocm/include", os.path.join(HERE, "helpers", "philox_ref.cpp"),
                           "-o", exe], stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(11)
    rows = []
    for _ in range(400):
        c = [int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 2 ** 16)),
             int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 2 ** 32))]
        k = [int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 2 ** 32))]
        rows.append((c, k))
    rows.append(([0, 0, 0, 0], [0, 0]))
    rows.append(([5, 7 | (3 << 8), 0xFFFFFFFE, 0xFFFFFFFF], [0, 0]))
    inp = "".join(f"{c[0]} {c[1]} {c[2]} {c[3]} {k[0]} {k[1]}\n" for c, k in rows)
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [[int(v) for v in line.split()] for line in out.strip().splitlines()]
    assert len(ref) == len(rows)
    for (c, k), r in zip(rows, ref):
        assert orc.philox(c, k) == r


def test_cdt_matches_decimal_computation(orc):
    """The table recomputed with Python's decimal module (a different
    arbitrary-precision library) at 70 digits."""
    getcontext().prec = 70
    sigma = Decimal("3.2")
    rho = [(-(Decimal(x) ** 2) / (2 * sigma * sigma)).exp() for x in range(-19, 20)]
    tot = sum(rho)
    acc = Decimal(0)
    want = []
    for i in range(38):
        acc += rho[i]
        want.append(int((acc / tot * (Decimal(2) ** 64)).to_integral_value(rounding="ROUND_FLOOR")))
    got = [int(x) for x in orc.cdt_table()]
    assert got == want
    assert all(a < b for a, b in zip(got, got[1:]))
    # symmetry of chi: CDF(x) + CDF(-x-1) = 1, up to the two floors
    # with T[i] = CDF(-19 + i) and -(-19 + i) - 1 = -19 + (37 - i)
    for i in range(38):
        assert abs(got[i] + got[37 - i] - 2 ** 64) <= 2


def test_ternary_distribution(orc):
    x = orc.sample_ternary(0, 12345, orc.TAG_U, 300000)  # multiple of 4
    assert set(np.unique(x).tolist()) <= {-1, 0, 1}
    counts = np.array([(x == v).sum() for v in (-1, 0, 1)], dtype=float)
    exp = len(x) / 3
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 20.0   # 2 dof; p ~ 5e-5
    # counter addressing: coefficient k of an n-draw uses word k // (n/4) of
    # block k mod (n/4), so the first quarter of a 4n-draw is column 0 of the
    # blocks; each quarter is itself a uniform ternary stream
    q4 = len(x) // 4
    for j in range(4):
        cj = np.array([(x[j * q4:(j + 1) * q4] == v).sum() for v in (-1, 0, 1)], dtype=float)
        assert ((cj - q4 / 3) ** 2 / (q4 / 3)).sum() < 20.0


def _gauss_pmf():
    getcontext().prec = 50
    rho = [(-(Decimal(x) ** 2) / (Decimal("20.48"))).exp() for x in range(-19, 20)]
    t = sum(rho)
    return np.array([float(r / t) for r in rho])


def test_gaussian_distribution(orc):
    n = 2_000_000
    x = orc.sample_gaussian(0, 99, orc.TAG_E1, n)
    assert x.min() >= -19 and x.max() <= 19
    pmf = _gauss_pmf()
    var_exact = float(sum(p * v * v for p, v in zip(pmf, range(-19, 20))))
    assert abs(var_exact - 3.2 ** 2) < 1e-6     # truncation at 6 sigma loses ~1e-7
    assert abs(x.mean()) < 5 * 3.2 / np.sqrt(n)
    assert abs(x.var() - var_exact) < 0.03
    counts = np.bincount(x + 19, minlength=39).astype(float)
    exp = pmf * n
    sel = exp > 20
    chi2 = (((counts - exp) ** 2 / exp)[sel]).sum()
    assert chi2 < sel.sum() + 8 * np.sqrt(2 * sel.sum())
    # halves of one draw share Philox blocks but are separate 64-bit words
    h = n // 2
    assert abs(np.corrcoef(x[:h].astype(float), x[h:].astype(float))[0, 1]) < 0.005


def test_gaussian_extreme_uniforms(orc):
    """Direct check of the inversion rule on the table's edges: the table's
    own end points map to the first and last support points."""
    t = orc.cdt_table()
    # P(x = -19) = T[0] / 2^64 must equal the normalised rho(19) to 1 part in 2^-60
    pmf = _gauss_pmf()
    assert abs(int(t[0]) / 2 ** 64 - pmf[0]) < 1e-18
    assert abs((2 ** 64 - int(t[37])) / 2 ** 64 - pmf[-1]) < 1e-18


def test_streams_are_distinct(orc):
    a = orc.sample_gaussian(0, 5, orc.TAG_E1, 4096)
    b = orc.sample_gaussian(0, 5, orc.TAG_E2, 4096)
    c = orc.sample_gaussian(0, 6, orc.TAG_E1, 4096)
    d = orc.sample_gaussian(1, 5, orc.TAG_E1, 4096)
    assert not np.array_equal(a, b) and not np.array_equal(a, c) and not np.array_equal(a, d)


def test_uniform_distribution(orc):
    q = orc.choose_moduli(13, (60,))[0]
    x = orc.sample_uniform(0, orc.KEY_ID, orc.TAG_A, 0, 200000, q).astype(object)
    assert max(x) < q
    xf = np.array([float(v) / q for v in x])
    assert abs(xf.mean() - 0.5) < 0.005
    hist = np.histogram(xf, bins=16, range=(0, 1))[0].astype(float)
    exp = len(xf) / 16
    assert ((hist - exp) ** 2 / exp).sum() < 50
    y = orc.sample_uniform(0, orc.KEY_ID, orc.TAG_A, 1, 1000, q)
    assert not np.array_equal(y, orc.sample_uniform(0, orc.KEY_ID, orc.TAG_A, 0, 1000, q))
