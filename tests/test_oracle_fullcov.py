"""Pins for the full-covariance noise of small arrays (Section 3.1, Eqs.
rad_full1-3 and Eq. noise): the oracle's (C^-1)_kk against numpy's
inverse of a covariance built here independently (itself checked against
the paper's special-case formulas), the diagonal limit, the positive
definite inequality (C^-1)_kk C_kk >= 1 and the point-source regime the
paper describes, and the unchanged output when C is not invertible."""
import numpy as np
import pytest

import oracle
from paper_1503_00638_amd import synth

N = synth.N_SAMPLES_DEFAULT


def dofs(I):
    pairs = synth.product_pairs(I)
    out = []
    for p, (i, j) in enumerate(pairs):
        out.append((p, i, j, 0))
        if i != j:
            out.append((p, i, j, 1))
    return out


def hermitian_v(vis, autos, fr, t):
    I = autos.shape[1]
    pairs = synth.product_pairs(I)
    V = np.zeros((I, I), np.complex128)
    for p, (i, j) in enumerate(pairs):
        if i == j:
            V[i, i] = float(autos[fr, i, t])
        else:
            V[i, j] = complex(vis[fr, p, t])
            V[j, i] = np.conj(V[i, j])
    return V


def cov_2n(V):
    """2N C from Eqs. rad_full1-3, written from the equations."""
    I = V.shape[0]
    ds = dofs(I)
    D = len(ds)
    Q = np.zeros((D, D))
    for x, (_, i, j, ax) in enumerate(ds):
        for y, (_, g, h, ay) in enumerate(ds):
            a = V[i, g] * np.conj(V[j, h])
            b = V[i, h] * np.conj(V[j, g])
            if ax == 0 and ay == 0:
                Q[x, y] = (a + b).real
            elif ax == 1 and ay == 1:
                Q[x, y] = (a - b).real
            elif ax == 0 and ay == 1:
                Q[x, y] = (-a + b).imag
            else:  # Im ij, Re gh: the (Re gh, Im ij) element
                a2 = V[g, i] * np.conj(V[h, j])
                b2 = V[g, j] * np.conj(V[h, i])
                Q[x, y] = (-a2 + b2).imag
    return Q


def test_builder_matches_special_cases():
    rng = np.random.default_rng(0)
    I = 3
    A = rng.standard_normal((I, I)) + 1j * rng.standard_normal((I, I))
    V = A @ A.conj().T + 3 * np.eye(I)  # Hermitian positive definite
    V[np.diag_indices(I)] = V.diagonal().real
    Q = cov_2n(V)
    idx = {(d[1], d[2], d[3]): k for k, d in enumerate(dofs(I))}
    i, j = 0, 1
    re_ii, re_ij, im_ij = idx[(i, i, 0)], idx[(i, j, 0)], idx[(i, j, 1)]
    vii, vjj, vij = V[i, i].real, V[j, j].real, V[i, j]
    # the paper's special cases, times 2N
    assert Q[re_ii, re_ii] == pytest.approx(2 * vii ** 2)
    assert Q[re_ii, re_ij] == pytest.approx(2 * vii * vij.real)
    assert Q[re_ij, re_ij] == pytest.approx(vii * vjj + vij.real ** 2 - vij.imag ** 2)
    assert Q[im_ij, im_ij] == pytest.approx(vii * vjj - vij.real ** 2 + vij.imag ** 2)
    assert Q[re_ij, im_ij] == pytest.approx(2 * vij.real * vij.imag)
    assert np.allclose(Q, Q.T)
    assert np.linalg.eigvalsh(Q).min() > 0


@pytest.mark.parametrize("I,seed,source", [(2, 0, 0.0), (3, 1, 0.4), (4, 2, 2.0), (5, 3, 0.4)])
def test_inverse_diagonal_against_numpy(I, seed, source):
    vis, autos = synth.gen_vis_point_source(2, I, 3, seed, source)
    q = oracle.fullcov_inverse_diag(vis, autos)
    for fr in range(2):
        for t in range(3):
            Q = cov_2n(hermitian_v(vis, autos, fr, t))
            ref = np.diag(np.linalg.inv(Q))
            assert np.allclose(q[fr, t], ref, rtol=1e-9, atol=0)
            # positive definite: (Q^-1)_kk Q_kk >= 1
            assert (q[fr, t] * np.diag(Q) >= 1 - 1e-12).all()


def test_diagonal_limit_is_the_diagonal_model():
    vis, autos = synth.gen_vis(3, 5, 8, 4)
    vis[:, [p for p, (i, j) in enumerate(synth.product_pairs(5)) if i != j], :] = 0
    q = oracle.fullcov_inverse_diag(vis, autos)
    for fr in range(3):
        for t in range(8):
            for k, (p, i, j, ax) in enumerate(dofs(5)):
                a, b = float(autos[fr, i, t]), float(autos[fr, j, t])
                expect = 1 / (2 * a * a) if i == j else 1 / (a * b)
                assert q[fr, t, k] == pytest.approx(expect, rel=1e-12)
    # with zero crosses the data rounded is the diagonal model's
    v2, a2 = synth.gen_vis(3, 5, 8, 4)
    v2[:, [p for p, (i, j) in enumerate(synth.product_pairs(5)) if i != j], :] *= 1e-30
    r_full = oracle.round_to_noise_fullcov(v2, a2, N, 0.01)
    r_diag = oracle.round_to_noise(v2, a2, N, 0.01)
    assert np.array_equal(r_full.view(np.uint32), r_diag.view(np.uint32))


def test_point_source_noise_is_much_smaller_than_marginal():
    """Section 3.1: with one dominant source the visibilities are strongly
    correlated; the noise not marginalised over the other products is far
    below the diagonal of C, so the full-covariance rounding is finer."""
    vis, autos = synth.gen_vis_point_source(1, 6, 4, 5, source=20.0)
    q = oracle.fullcov_inverse_diag(vis, autos)
    Q = cov_2n(hermitian_v(vis, autos, 0, 0))
    ratio = q[0, 0] * np.diag(Q)  # (C^-1)_kk C_kk
    assert ratio.max() > 20
    r_full = oracle.round_to_noise_fullcov(vis, autos, N, 0.01)
    r_diag = oracle.round_to_noise(vis, autos, N, 0.01)
    e_full = np.abs(r_full.view(np.float32) - vis.view(np.float32)).max()
    e_diag = np.abs(r_diag.view(np.float32) - vis.view(np.float32)).max()
    assert e_full < e_diag


def test_singular_sample_is_left_unchanged():
    vis, autos = synth.gen_vis(2, 4, 3, 6)
    autos[1, 2, 1] = 0.0  # Q has a zero pivot at (f=1, t=1)
    q = oracle.fullcov_inverse_diag(vis, autos)
    assert np.isnan(q[1, 1]).all() and np.isfinite(q[0]).all()
    r = oracle.round_to_noise_fullcov(vis, autos, N, 0.01)
    assert np.array_equal(np.ascontiguousarray(r[1, :, 1]).view(np.uint32),
                          np.ascontiguousarray(vis[1, :, 1]).view(np.uint32))
    assert not np.array_equal(r[0].view(np.uint32), vis[0].view(np.uint32))
    # Im of autos is copied
    autop = [p for p, (i, j) in enumerate(synth.product_pairs(4)) if i == j]
    assert np.array_equal(r[:, autop, :].imag, vis[:, autop, :].imag)
