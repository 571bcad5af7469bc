"""Pins for the oracle's RNG and closed-form pickers.

- Philox4x64-10 against numpy's independent implementation (and the
  published known-answer vectors of the Random123 distribution).
- Eq. (1) uniform: exact uniformity of the integer scaling.
- Eq. (2) linear: against Eq. (2) itself in 60-digit decimal arithmetic and
  against the law P(i) = 2(i+1)/(n(n+1)) summed in exact rationals.
- Eq. (3) exponential (read as the exact inverse CDF): against the law
  P(i) ~ exp(lambda i) summed in 60-digit decimal, with the tie to the
  paper's printed asymptotic form for lambda = 1.
- lambda: the index-based exponential law equals the weight-based law
  w = exp((t - t_min) / tau) whenever timestamp gaps are uniform, which is
  the exactness condition the paper states for the index-based sampler.
"""
import decimal
import math
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle

RNG = np.random.default_rng(12345)


def _rand_u64(n):
    return [int(x) for x in RNG.integers(0, 2**64, size=n, dtype=np.uint64)]


# ----------------------------------------------------------------- Philox

def test_philox_matches_numpy():
    for _ in range(200):
        wid, hop, trial = _rand_u64(1)[0], int(RNG.integers(0, 2**20)), int(RNG.integers(0, 5000))
        seed = _rand_u64(1)[0]
        got = [int(v) for v in oracle.philox([wid, hop, trial, 0], [seed, 0])]
        assert got == brute.philox_numpy(seed, wid, hop, trial)


def test_philox_counter_carry_edge():
    # counter words at their limits exercise numpy's 256-bit increment path
    for wid in (0, 1, 2**64 - 1):
        for hop in (0, 2**64 - 1):
            got = [int(v) for v in oracle.philox([wid, hop, 0, 0], [7, 0])]
            assert got == brute.philox_numpy(7, wid, hop, 0)


KAT = [
    # counter, key, expected output: the philox4x64-10 known-answer vectors
    # of the Random123 distribution
    ([0, 0, 0, 0], [0, 0],
     [0x16554d9eca36314c, 0xdb20fe9d672d0fdc, 0xd7e772cee186176b, 0x7e68b68aec7ba23b]),
    ([2**64 - 1] * 4, [2**64 - 1] * 2,
     [0x87b092c3013fe90b, 0x438c3c67be8d0224, 0x9cc7d7c69cd777b6, 0xa09caebf594f0ba0]),
    ([0x243f6a8885a308d3, 0x13198a2e03707344, 0xa4093822299f31d0, 0x082efa98ec4e6c89],
     [0x452821e638d01377, 0xbe5466cf34e90c6c],
     [0xa528f45403e61d95, 0x38c72dbd566e9788, 0xa5a1610e72fd18b5, 0x57bd43b5e52b7fe6]),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    assert [int(v) for v in oracle.philox(ctr, key)] == want


# ----------------------------------------------------------------- uniform

@pytest.mark.parametrize("n", [1, 2, 3, 7, 1000, 2**31 - 1, 2**40 + 3])
def test_uniform_preimages_are_equal(n):
    # pick(x) = i exactly on [ceil(i 2^64 / n), ceil((i+1) 2^64 / n)): every
    # index owns floor or ceil of 2^64/n inputs, and the map is monotone
    for i in [0, n - 1] + [int(v) for v in RNG.integers(0, n, size=5)]:
        lo = -((-i << 64) // n)
        assert oracle.pick_uniform(n, lo) == i
        if lo > 0:
            assert oracle.pick_uniform(n, lo - 1) == i - 1
        hi = -((-(i + 1) << 64) // n) - 1
        assert oracle.pick_uniform(n, min(hi, 2**64 - 1)) == i


def test_uniform_single_candidate():
    for x in _rand_u64(50):
        assert oracle.pick_uniform(1, x) == 0


# ----------------------------------------------------------------- linear

def _eq2_decimal(n, x):
    """Eq. (2) literally, u = (x>>11)/2^53, in 60-digit decimal arithmetic."""
    with decimal.localcontext() as ctx:
        ctx.prec = 80
        u = decimal.Decimal(x >> 11) / decimal.Decimal(2**53)
        r = (-1 + (1 + 4 * u * n * (n + 1)).sqrt()) / 2
        return int(r.to_integral_value(rounding=decimal.ROUND_FLOOR))


@pytest.mark.parametrize("n", [1, 2, 3, 10, 999, 12345, 2**20 + 7, 2**31 - 1, 2**32 - 1])
def test_linear_matches_eq2_high_precision(n):
    for x in _rand_u64(300):
        assert oracle.pick_linear(n, x) == _eq2_decimal(n, x)


def test_linear_matches_law_exact_rationals():
    # the law implied by Eq. (2): P(i) = 2(i+1) / (n(n+1))
    for n in (1, 2, 5, 17, 60):
        for x in _rand_u64(200):
            assert oracle.pick_linear(n, x) == brute.linear_pick(n, x)


def test_linear_boundaries_exact():
    # draws that land exactly on a CDF boundary F(i) = i(i+1)/(n(n+1)) pick i
    for n in (3, 8, 100):
        for i in range(1, n):
            F = brute.linear_cdf(n, i)
            a = F * 2**53
            if a.denominator == 1:
                x = int(a) << 11
                assert oracle.pick_linear(n, x) == i
                assert oracle.pick_linear(n, x - (1 << 11)) == i - 1


def test_linear_extremes():
    n = 1000
    assert oracle.pick_linear(n, 0) == 0
    assert oracle.pick_linear(n, 2**64 - 1) == n - 1


# ----------------------------------------------------------------- exponential

@pytest.mark.parametrize("n,lam", [(2, 0.3), (5, 1.0), (12, 0.05), (40, 1.0), (40, 0.02),
                                   (33, 2.5), (200, 1e-4), (64, 30.0)])
def test_exponential_matches_law_decimal(n, lam):
    bad = 0
    for x in _rand_u64(150):
        i, margin = oracle.pick_exponential(n, lam, x)
        j, m2 = brute.exp_pick(n, lam, x)
        if i != j:
            assert m2 < 1e-12, (n, lam, x, i, j, m2)
            bad += 1
        else:
            assert margin == pytest.approx(m2, rel=1e-6, abs=1e-12)
    assert bad <= 1


def test_exponential_single_group():
    for x in _rand_u64(20):
        assert oracle.pick_exponential(1, 3.0, x)[0] == 0


def test_exponential_small_lambda_is_uniform():
    n = 97
    for x in _rand_u64(200):
        i, _ = oracle.pick_exponential(n, 1e-13, x)
        u = oracle.unit_open(x)
        assert abs(i - math.floor(u * n)) <= (1 if abs(u * n - round(u * n)) < 1e-6 else 0)


def test_exponential_lambda_one_tail_and_eq3_form():
    # lambda = 1 (the printed form of Eq. (3)): for large n the last index
    # has probability (e - 1)/e and the pick agrees with ceil(n + ln u) - 1
    n = 5000
    xs = [int(v) for v in np.random.default_rng(7).integers(0, 2**64, 40000, dtype=np.uint64)]
    last = 0
    for x in xs:
        i, m = oracle.pick_exponential(n, 1.0, x)
        u = oracle.unit_open(x)
        if m > 1e-9:
            assert i == max(0, math.ceil(n + math.log(u)) - 1)
        last += i == n - 1
    p = (math.e - 1) / math.e
    assert abs(last / len(xs) - p) < 5 * math.sqrt(p * (1 - p) / len(xs))


def test_lambda_uniform_gaps_equal_weight_law():
    # groups at t_j = t0 + j*gap: exp(lambda*i) == exp((t_i - t_min)/tau)
    for t0, gap, n, tau in [(0, 10, 50, 100.0), (12345, 7, 9, 3.5), (-50, 1, 200, 1e3)]:
        lam = oracle.exp_lambda(t0, t0 + gap * (n - 1), n, tau)
        for i in range(n):
            assert lam * i == pytest.approx((gap * i) / tau, rel=1e-12)
    assert oracle.exp_lambda(0, 100, 5, 0.0) == 1.0  # tau <= 0: Eq. (3) literal, lambda = 1


def test_unit_open_range():
    assert 0.0 < oracle.unit_open(0) < 1e-15
    assert 1.0 - 1e-15 < oracle.unit_open(2**64 - 1) < 1.0


# ------------------------------------------------------ weight-based picker

@pytest.mark.parametrize("n,gap,tau", [(2, 3, 2.0), (5, 1, 1.0), (37, 4, 10.0), (200, 7, 50.0)])
def test_weight_equal_gaps_is_the_exponential_law(n, gap, tau):
    # equal gaps make the weights exp(gap i / tau): the law of Eq. (3)'s exact
    # inverse with lambda = gap / tau, evaluated by a different formula
    ts = np.arange(n, dtype=np.int64) * gap
    rng = np.random.default_rng(n)
    for x in rng.integers(0, 2**64, 3000, dtype=np.uint64):
        kw, mw = oracle.pick_weight(ts, tau, int(x))
        ke, me = oracle.pick_exponential(n, gap / tau, int(x))
        assert kw == ke or min(mw, me) < 1e-9, (x, kw, ke, mw, me)


def test_weight_matches_decimal_law():
    # random timestamps with ties against the printed definition summed in
    # 60-digit decimal (weights exp(t_i - t_min), scale tau)
    rng = np.random.default_rng(12)
    for trial in range(40):
        n = int(rng.integers(1, 30))
        ts = np.sort(rng.integers(0, 50, n)).astype(np.int64)
        tau = float(rng.choice([0.0, 0.7, 3.0, 25.0]))
        for x in rng.integers(0, 2**64, 200, dtype=np.uint64):
            k, m = oracle.pick_weight(ts, tau, int(x))
            kb, mb = brute.weight_pick([int(t) for t in ts], tau, int(x))
            assert k == kb or min(m, mb) < 1e-9, (trial, x, k, kb, m, mb)
            if k == kb:
                assert abs(m - mb) < 1e-9 or (m == mb == float("inf"))


def test_weight_large_tau_is_uniform_over_edges():
    # tau far above the span: every weight is 1, so k = ceil(u n) - 1
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 64, 1000):
        ts = np.sort(rng.integers(0, 10**6, n)).astype(np.int64)
        for x in rng.integers(0, 2**64, 500, dtype=np.uint64):
            u = Fraction(2 * (int(x) >> 12) + 1, 1 << 53)
            want = -(-(u * n).numerator // (u * n).denominator) - 1
            k, m = oracle.pick_weight(ts, 1e300, int(x))
            assert k == want or m < 1e-12


def test_weight_single_candidate_and_ties():
    assert oracle.pick_weight([7], 2.0, 12345) == (0, float("inf"))
    # four equal timestamps: equal weights, k = ceil(4u) - 1
    for x, want in [(0, 0), (2**62 - 1, 0), (2**62 + 2**20, 1), (2**64 - 1, 3)]:
        assert oracle.pick_weight([5, 5, 5, 5], 3.0, x)[0] == want
