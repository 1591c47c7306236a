"""CPU check of the lazy reduction schedule of the library's integer forward
NTT (moduli below 2^60): Shoup products lie in [0, 2q) for any 64-bit input,
so a butterfly raises its bound by 2q; from inputs in [0, 4q) the transform
subtracts 8q from the sum operand at stages 6, 10, 14 only.  A Python
emulation with exact integers of every butterfly (the same Cooley-Tukey order
and twiddle table as the kernels) checks that no value reaches 16q (so 64-bit
words never overflow), that each Shoup product is in [0, 2q), and that the
outputs reduce to the oracle's transform."""
import random

import pytest

M64 = (1 << 64) - 1


def fwd_reduce(j):
    """Stages whose sum operand is first brought from [0, 16q) into [0, 8q)."""
    return j >= 6 and (j - 6) % 4 == 0


def brv(x, bits):
    return int(format(x, f"0{bits}b")[::-1], 2)


@pytest.mark.parametrize("log_n,bits", [(12, 60), (13, 60), (14, 60), (14, 55)])
def test_lazy_schedule_stays_below_16q(orc, log_n, bits):
    n = 1 << log_n
    q = orc.choose_moduli(log_n, [bits])[0]
    assert q < 1 << 60
    psi = orc.find_psi(q, log_n)
    tw = [pow(psi, brv(k, log_n), q) for k in range(n)]
    twp = [(w << 64) // q for w in tw]
    rng = random.Random(log_n * 100 + bits)
    a = [rng.randrange(q) for _ in range(n)]
    # inputs anywhere in [0, 4q) with the same residues, extremes included
    v = [x + q * rng.choice((0, 1, 2, 3)) for x in a]
    v[0], v[1] = 4 * q - 1 - (q - 1 - a[0]) % q, a[1]
    assert all(0 <= x < 4 * q and x % q == y for x, y in zip(v, a))
    m, gap, j, top = 1, n // 2, 0, 0
    while m < n:
        for i in range(m):
            w, wp = tw[m + i], twp[m + i]
            for k in range(2 * i * gap, 2 * i * gap + gap):
                x, y = v[k], v[k + gap]
                assert x < 16 * q and y <= M64
                if fwd_reduce(j):
                    x = x - 8 * q if x >= 8 * q else x
                t = (y * w - ((y * wp) >> 64) * q) & M64          # 64-bit wrap-around, as on the GPU
                assert 0 <= t < 2 * q
                v[k], v[k + gap] = x + t, x - t + 2 * q
                top = max(top, v[k], v[k + gap])
        m, gap, j = 2 * m, gap // 2, j + 1
    assert top < 16 * q <= M64
    assert [x % q for x in v] == [int(r) for r in orc.ntt_forward(a, log_n, q, psi)]


@pytest.mark.parametrize("bits", [55, 60])
def test_split_schedule_log15(orc, bits):
    """N = 32768 as the split kernels compute it: the first stage pairs j and
    j + N/2 (sum operand reduced from [0, 4q) to [0, 2q), outputs in [0, 4q)),
    then each half is an independent 16384-point transform whose stage s,
    group g uses twiddle (2 + h) 2^s + g of the full table and whose lazy
    reductions follow the half's own stage count (stages 6 and 10 of 14)."""
    log_n = 15
    n, nh = 1 << log_n, 1 << (log_n - 1)
    q = orc.choose_moduli(log_n, [bits])[0]
    psi = orc.find_psi(q, log_n)
    tw = [pow(psi, brv(k, log_n), q) for k in range(n)]
    twp = [(w << 64) // q for w in tw]
    rng = random.Random(bits)
    a = [rng.randrange(q) for _ in range(n)]
    v = [x + q * rng.choice((0, 1, 2, 3)) for x in a]
    v[0] = a[0] + 3 * q
    v[nh] = a[nh] + 3 * q
    halves = [[0] * nh, [0] * nh]
    w, wp = tw[1], twp[1]
    for j in range(nh):
        xl, xh = v[j], v[j + nh]
        assert xl < 4 * q and xh < 4 * q
        x = xl - 2 * q if xl >= 2 * q else xl
        t = (xh * w - ((xh * wp) >> 64) * q) & M64
        assert 0 <= t < 2 * q
        halves[0][j], halves[1][j] = x + t, x - t + 2 * q
        assert halves[0][j] < 4 * q and halves[1][j] < 4 * q
    top = 0
    for h in (0, 1):
        u = halves[h]
        m, gap, j = 1, nh // 2, 0
        while m < nh:
            for i in range(m):
                idx = (2 + h) * m + i
                w, wp = tw[idx], twp[idx]
                for k in range(2 * i * gap, 2 * i * gap + gap):
                    x, y = u[k], u[k + gap]
                    assert x < 16 * q
                    if fwd_reduce(j):
                        x = x - 8 * q if x >= 8 * q else x
                    t = (y * w - ((y * wp) >> 64) * q) & M64
                    assert 0 <= t < 2 * q
                    u[k], u[k + gap] = x + t, x - t + 2 * q
                    top = max(top, u[k], u[k + gap])
            m, gap, j = 2 * m, gap // 2, j + 1
    assert top < 16 * q <= M64
    out = [x % q for x in halves[0] + halves[1]]
    assert out == [int(r) for r in orc.ntt_forward(a, log_n, q, psi)]
