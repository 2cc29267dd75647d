"""Property-based checks of the oracle (hypothesis, derandomised so every
run draws the same examples): round trips of the transposes and of the
compressed stream over arbitrary data and shapes, the block decoder on
mutated input (it never fails uncontrolled, and whatever liblz4 accepts it
accepts with the same bytes), and the rounding invariants of Section 3.2
(Eq. trunc_error and its footnote) over arbitrary floats and granularities."""
import math
from fractions import Fraction

import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import lz4ref  # noqa: E402

SETTINGS = settings(max_examples=400, deadline=None, derandomize=True,
                    suppress_health_check=list(hypothesis.HealthCheck))

elem_sizes = st.sampled_from([1, 2, 3, 4, 5, 8, 12, 16])
block_sizes = st.sampled_from([0, 8, 16, 24, 64, 2048])


def _data(draw, E, max_elems=3000):
    n = draw(st.integers(0, max_elems))
    kind = draw(st.integers(0, 3))
    seed = draw(st.integers(0, 2**32 - 1))
    rng = np.random.default_rng(seed)
    if kind == 0:
        b = rng.integers(0, 256, n * E, dtype=np.uint8)
    elif kind == 1:
        b = rng.integers(0, 3, n * E, dtype=np.uint8)
    elif kind == 2:
        b = np.resize(rng.integers(0, 256, int(rng.integers(1, 40)), dtype=np.uint8), n * E)
    else:
        b = np.zeros(n * E, np.uint8)
        b[rng.integers(0, max(n * E, 1), size=min(n * E, 5))] = 7 if n * E else 0
    return n, b


@st.composite
def shaped(draw):
    E = draw(elem_sizes)
    B = draw(block_sizes)
    n, b = _data(draw, E)
    return b, n, E, B


@SETTINGS
@given(shaped())
def test_transpose_round_trips(oracle_lib, case):
    b, n, E, B = case
    for fwd, inv in ((oracle_lib.bitshuffle, oracle_lib.bitunshuffle),
                     (oracle_lib.byteshuffle, oracle_lib.byteunshuffle)):
        y = fwd(b, E, B)
        assert y.size == b.size
        assert np.array_equal(inv(y, E, B), b)


@SETTINGS
@given(shaped(), st.sampled_from([0, 1]))
def test_stream_round_trip_and_framing(oracle_lib, case, filt):
    b, n, E, B = case
    s = oracle_lib.compress(b, E, B, filter=filt)
    assert s.size <= oracle_lib.compress_bound(n, E, B)
    assert np.array_equal(oracle_lib.decompress(s, n, E, B, filter=filt), b)
    # a truncated stream and one with a byte appended are refused
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.decompress(s[:-1], n, E, B, filter=filt)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.decompress(np.concatenate([s, np.zeros(1, np.uint8)]), n, E, B, filter=filt)


@st.composite
def mutated_block(draw):
    n = draw(st.integers(13, 1500))
    seed = draw(st.integers(0, 2**32 - 1))
    rng = np.random.default_rng(seed)
    data = np.resize(rng.integers(0, 256, int(rng.integers(1, 60)), dtype=np.uint8), n)
    data[rng.integers(0, n, size=int(rng.integers(0, 8)))] = 0
    muts = draw(st.lists(st.tuples(st.integers(0, 10**6), st.integers(1, 255)), min_size=1,
                         max_size=4))
    return data.tobytes(), muts


@SETTINGS
@given(mutated_block())
def test_block_decoder_on_mutated_input(oracle_lib, case):
    data, muts = case
    comp = bytearray(oracle_lib.lz4_compress_block(np.frombuffer(data, np.uint8)))
    assert oracle_lib.lz4_decompress_block(bytes(comp), len(data)) == data
    for pos, x in muts:
        comp[pos % len(comp)] ^= x
    try:
        got = oracle_lib.lz4_decompress_block(bytes(comp), len(data))
    except oracle_lib.OracleError:
        got = None
    if got is not None:
        assert len(got) == len(data)
    if lz4ref.available():
        ref = lz4ref.decompress_safe(bytes(comp), len(data))
        if ref is not None and len(ref) == len(data):
            assert got == ref


# ---- rounding (Section 3.2) --------------------------------------------------
finite_f32 = st.floats(width=32, allow_nan=False, allow_infinity=False)


@SETTINGS
@given(finite_f32, st.integers(-149, 127))
def test_float_rounding_invariants(oracle_lib, x, k):
    r = oracle_lib.round_to_multiple(x, k)
    if math.isinf(r):  # only when the exact result overflows float32
        assert abs(x) > 3.0e38
        return
    g = Fraction(2) ** k
    fr, fx = Fraction(r), Fraction(x)
    assert (fr / g).denominator == 1  # a multiple of 2^k
    assert abs(fr - fx) <= g / 2
    if abs(fr - fx) == g / 2:  # a tie goes to the even multiple
        assert (fr / g).numerator % 2 == 0
    assert oracle_lib.round_to_multiple(r, k) == r  # idempotent
    assert oracle_lib.round_to_multiple(-x, k) == -r  # odd
    if r == 0.0:
        assert math.copysign(1.0, r) == math.copysign(1.0, x)  # zero keeps the sign


@SETTINGS
@given(st.floats(min_value=1e-300, max_value=1e300, allow_nan=False))
def test_granularity_is_the_largest_power_below(oracle_lib, G2):
    k = oracle_lib.granularity_exponent(G2)
    g2 = Fraction(4) ** k
    assert g2 < Fraction(G2) <= 4 * g2  # 4^k < G2 <= 4^(k+1): g^2 < G2, the largest such g


@SETTINGS
@given(st.integers(-2**31, 2**31 - 1), st.integers(0, 31))
def test_integer_rounding_invariants(oracle_lib, x, k):
    r = oracle_lib.round_int_to_multiple(x, k)
    assert -2**31 <= r <= 2**31 - 1
    assert r % (1 << k) == 0
    if k == 0:
        assert r == x
        return
    exact = Fraction(x, 1 << k)
    q = math.floor(exact + Fraction(1, 2))
    if exact + Fraction(1, 2) == q and q % 2:  # tie: to even
        q -= 1
    want = q << k
    if want > 2**31 - 1:  # saturates to the largest multiple that fits
        want = ((2**31 - 1) >> k) << k
    assert r == want
