"""Pins for the oracle's integer rounding (the paper's own data type,
Section 5: correlator output is integers, so a granularity g <= 1 means no
rounding).  Checks use exact Python integer and Fraction arithmetic, not the
oracle's own formulation."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1503_00638_amd import synth

INT32_MAX, INT32_MIN = 2**31 - 1, -2**31


def exact_int_round(x: int, k: int) -> int:
    """Nearest multiple of 2^k, ties to the even multiple; saturated to the
    largest multiple that fits int32."""
    if k <= 0:
        return x
    g = 2 ** k
    q, rem = divmod(x, g)  # Python: floor division, 0 <= rem < g
    if 2 * rem > g or (2 * rem == g and q % 2 == 1):
        q += 1
    r = q * g
    if r > INT32_MAX:
        r = (INT32_MAX // g) * g
    return r


def exact_k(G2: float) -> int:
    g2 = Fraction(G2)
    k = 0
    while Fraction(4) ** k >= g2:
        k -= 1
    while Fraction(4) ** (k + 1) < g2:
        k += 1
    return k


def test_int_rounding_exact_random():
    rng = np.random.default_rng(0)
    xs = list(rng.integers(INT32_MIN, INT32_MAX, 3000, endpoint=True, dtype=np.int64))
    xs += [0, 1, -1, INT32_MAX, INT32_MIN, INT32_MAX - 1, INT32_MIN + 1]
    for k in list(range(-3, 40)) + [62, 63, 100, 511]:
        for x in xs[: 300 if k not in (1, 2, 3, 30, 31, 32) else len(xs)]:
            assert oracle.round_int_to_multiple(int(x), k) == exact_int_round(int(x), min(k, 62)), (x, k)


def test_int_rounding_ties_and_worked_values():
    # g = 2: 7 = 3.5 g -> 4 g;  5 = 2.5 g -> 2 g;  g = 4: -6 = -1.5 g -> -2 g, -10 = -2.5 g -> -2 g
    assert [oracle.round_int_to_multiple(x, k) for x, k in
            ((7, 1), (5, 1), (-6, 2), (-10, 2), (6, 2), (2, 2), (-2, 2), (3, 0), (-3, -5))] == \
        [8, 4, -8, -8, 8, 0, 0, 3, -3]
    # saturation: 2^31 - 1 rounds up to 2^31 (does not fit) -> largest multiple that fits
    assert oracle.round_int_to_multiple(INT32_MAX, 1) == INT32_MAX - 1
    assert oracle.round_int_to_multiple(INT32_MAX, 31) == 0
    assert oracle.round_int_to_multiple(INT32_MIN, 31) == INT32_MIN
    assert oracle.round_int_to_multiple(INT32_MIN, 32) == 0  # tie at -g/2 goes to the even 0
    assert oracle.round_int_to_multiple(INT32_MIN, 33) == 0


def reference_round_to_noise_i32(vis, autos, N, f):
    """Pure-Python definition on tiny arrays: exact k, exact integer rounding."""
    F, I, T = autos.shape
    pairs = synth.product_pairs(I)
    c = (12.0 * f) / (2.0 * N)
    out = vis.copy()
    for fr in range(F):
        for p, (i, j) in enumerate(pairs):
            for t in range(T):
                a, b = int(autos[fr, i, t]), int(autos[fr, j, t])
                G2 = float(a * b) * (c if i != j else 2.0 * c)
                if not (G2 > 0.0) or G2 == float("inf"):
                    continue
                k = exact_k(G2)
                out[fr, p, t, 0] = exact_int_round(int(vis[fr, p, t, 0]), k)
                if i != j:
                    out[fr, p, t, 1] = exact_int_round(int(vis[fr, p, t, 1]), k)
    return out


@pytest.mark.parametrize("F,I,T,seed,f", [(2, 4, 5, 0, 0.01), (1, 3, 16, 1, 0.1), (3, 2, 3, 2, 1e-3)])
def test_round_to_noise_i32_exact_small(F, I, T, seed, f):
    vis, autos = synth.gen_vis_int(F, I, T, seed)
    got = oracle.round_to_noise_i32(vis, autos, synth.N_SAMPLES_DEFAULT, f)
    assert np.array_equal(got, reference_round_to_noise_i32(vis, autos, synth.N_SAMPLES_DEFAULT, f))


def test_int_invariants():
    N = synth.N_SAMPLES_DEFAULT
    vis, autos = synth.gen_vis_int(4, 6, 32, 3)
    r = oracle.round_to_noise_i32(vis, autos, N, 0.01)
    # something is rounded away (g = 2^k with k >= 1 at this scale), but not everything
    assert (r != vis).any() and (r == vis).any()
    # idempotent with the same autos
    assert np.array_equal(oracle.round_to_noise_i32(r, autos, N, 0.01), r)
    # odd symmetry (away from the int32 limits)
    assert np.array_equal(oracle.round_to_noise_i32(-vis, autos, N, 0.01), -r)
    # scale covariance: vis and autos times 2^m scale G2 by 4^m, k by m
    for m in (1, 3):
        r2 = oracle.round_to_noise_i32(vis * 2**m, autos * 2**m, N, 0.01)
        assert np.array_equal(r2, r * 2**m)
    # error bound |R(x) - x| <= g/2 with g = 2^k of each element
    pairs = synth.product_pairs(6)
    c = 12 * 0.01 / (2 * N)
    for fr in range(4):
        for p, (i, j) in enumerate(pairs):
            G2 = float(int(autos[fr, i, 0]) * int(autos[fr, j, 0])) * (c if i != j else 2 * c)
            g = 2 ** max(exact_k(G2), 0)
            assert abs(int(r[fr, p, 0, 0]) - int(vis[fr, p, 0, 0])) <= g // 2 if g > 1 else \
                r[fr, p, 0, 0] == vis[fr, p, 0, 0]


def test_int_small_noise_is_untouched():
    """G2 <= 4 gives k <= 0: integers are already multiples of g <= 1."""
    N = synth.N_SAMPLES_DEFAULT
    vis, autos = synth.gen_vis_int(2, 4, 8, 4, scale=1.0)  # autos ~ 1e3: G2 ~ 0.03
    assert np.array_equal(oracle.round_to_noise_i32(vis, autos, N, 0.01), vis)
    # zero or opposite-sign autos, and f = 0, leave data unchanged
    a2 = autos.copy()
    a2[0, 0, :] = 0
    r = oracle.round_to_noise_i32(vis * 4096, a2 * 4096, N, 0.01)
    assert np.array_equal(r[0, :4, :, :], (vis * 4096)[0, :4, :, :])  # products (0, j)
    assert np.array_equal(oracle.round_to_noise_i32(vis * 4096, autos * 4096, N, 0.0), vis * 4096)
