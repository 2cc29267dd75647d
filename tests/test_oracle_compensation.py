"""Pins for the compensation of the diagonal noise model (Section 3.2):
f is multiplied, per frequency and time, by the minimum over cross
products of 1 - |V_ij|^2 / (V_ii V_jj).  Checks: closed forms on
constructed data, the paper's point-source limit, exact rational brute
force on small arrays, and how the factor enters the rounding."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1503_00638_amd import synth

N = synth.N_SAMPLES_DEFAULT


def brute_min(vis, autos):
    """Exact rational minimum, its (p) position, per (f, t)."""
    F, I, T = autos.shape
    pairs = synth.product_pairs(I)
    out = np.ones((F, T))
    for fr in range(F):
        for t in range(T):
            best = Fraction(1)
            for p, (i, j) in enumerate(pairs):
                if i == j:
                    continue
                a, b = Fraction(float(autos[fr, i, t])), Fraction(float(autos[fr, j, t]))
                if a * b <= 0:
                    continue
                v = vis[fr, p, t]
                term = 1 - (Fraction(float(v.real)) ** 2 + Fraction(float(v.imag)) ** 2) / (a * b)
                best = min(best, term)
            out[fr, t] = float(best)
    return out


def test_closed_form_equal_crosses():
    """All crosses s (real), all autos A: the factor is 1 - s^2 / A^2."""
    F, I, T = 2, 5, 3
    P = I * (I + 1) // 2
    vis = np.zeros((F, P, T), np.complex64)
    autos = np.full((F, I, T), 1000.0, np.float32)
    pairs = synth.product_pairs(I)
    for p, (i, j) in enumerate(pairs):
        vis[:, p, :] = 1000.0 if i == j else 300.0
    m = oracle.noise_compensation(vis, autos)
    assert np.allclose(m, 1 - 0.3 ** 2, rtol=0, atol=1e-15)
    # an imaginary part counts through |V_ij|^2
    vis[0, 1, 0] = 300 + 400j
    assert oracle.noise_compensation(vis, autos)[0, 0] == pytest.approx(1 - 0.25, abs=1e-15)


def test_point_source_limit_stops_rounding():
    """Section 3.1 example: a single dominant source makes all visibilities
    equal; the factor is 0 and the compensated rounding changes nothing."""
    F, I, T = 2, 6, 4
    vis, autos = synth.gen_vis(F, I, T, 3)
    vis[...] = np.complex64(500.0)
    autos[...] = np.float32(500.0)
    m = oracle.noise_compensation(vis, autos)
    assert np.array_equal(m, np.zeros((F, T)))
    r = oracle.round_to_noise_scaled(vis, autos, N, 0.01, m)
    assert np.array_equal(r.view(np.uint32), vis.view(np.uint32))


@pytest.mark.parametrize("seed,source", [(0, 0.0), (1, 0.4), (2, 2.0)])
def test_brute_force_minimum(seed, source):
    vis, autos = synth.gen_vis_point_source(3, 5, 6, seed, source)
    m = oracle.noise_compensation(vis, autos)
    ref = brute_min(vis, autos)
    assert np.allclose(m, ref, rtol=0, atol=4e-16)
    if source > 0:
        assert (m < 0.99).all()


def test_invalid_products_are_skipped():
    vis, autos = synth.gen_vis_point_source(1, 4, 3, 5, 0.4)
    autos[0, 1, 0] = 0.0       # products with input 1 skipped at t = 0
    autos[0, 2, 1] = -3.0      # negative power: skipped where the product is negative
    autos[0, 3, 2] = np.nan    # NaN: skipped
    m = oracle.noise_compensation(vis, autos)
    assert np.allclose(m, brute_min_skip_nan(vis, autos), rtol=0, atol=4e-16)
    # a single input has no cross products: factor 1
    v1, a1 = synth.gen_vis(2, 1, 4, 0)
    assert np.array_equal(oracle.noise_compensation(v1, a1), np.ones((2, 4)))


def brute_min_skip_nan(vis, autos):
    F, I, T = autos.shape
    pairs = synth.product_pairs(I)
    out = np.ones((F, T))
    for fr in range(F):
        for t in range(T):
            best = 1.0
            for p, (i, j) in enumerate(pairs):
                a, b = float(autos[fr, i, t]), float(autos[fr, j, t])
                if i == j or not (a * b > 0) or np.isinf(a * b):
                    continue
                v = vis[fr, p, t]
                term = float(1 - (Fraction(float(v.real)) ** 2 + Fraction(float(v.imag)) ** 2)
                             / (Fraction(a) * Fraction(b)))
                best = min(best, term)
            out[fr, t] = best
    return out


def test_scale_enters_as_a_factor_on_f():
    vis, autos = synth.gen_vis_point_source(3, 6, 16, 7, 0.4)
    F, T = 3, 16
    ones = np.ones((F, T))
    base = oracle.round_to_noise(vis, autos, N, 0.01)
    assert np.array_equal(oracle.round_to_noise_scaled(vis, autos, N, 0.01, ones).view(np.uint32),
                          base.view(np.uint32))
    # a power-of-two factor is exact: scale 4^-2 equals f / 16
    q = oracle.round_to_noise_scaled(vis, autos, N, 0.01, ones / 16)
    assert np.array_equal(q.view(np.uint32), oracle.round_to_noise(vis, autos, N, 0.01 / 16).view(np.uint32))
    # compensation never coarsens: the error is at most the uncompensated one's bound
    m = oracle.noise_compensation(vis, autos)
    c = oracle.round_to_noise_scaled(vis, autos, N, 0.01, m)
    err_c = np.abs(c.view(np.float32) - vis.view(np.float32))
    err_b = np.abs(base.view(np.float32) - vis.view(np.float32))
    assert err_c.max() <= err_b.max()
    assert (c != base).any()
