"""Pins of the oracle's linear operators against what the paper and mathematics fix.

* eq:ak: A_k(L) vec(X) is the circular convolution L * X, checked against the
  FFT (convolution theorem) and a brute-force nested-loop sum on tiny inputs.
* The adjoint of Section III-D: <A_k(L), X> = <L, A_k^*(X)> and A_k^* A_k = k I.
* eq:convset: every column of A_k(Theta_Omega) holds exactly |Omega| ones.
Each pin is chosen so that a plausible mistake (correlation instead of
convolution, a wrong sign in the shift, a transposed operand, a dropped /k)
fails at least one of them; the mutation tests at the bottom plant such
mistakes in a copy of the oracle and check that the pins catch them.
"""
import itertools

import numpy as np
import pytest

from oracle import icnnm_ref as O

SHAPES = [((6, 5, 4), (3, 2, 2)), ((7, 3), (2, 3)), ((11,), (4,)), ((4, 4, 4), (4, 4, 4)),
          ((5, 6, 3), (1, 1, 1))]


def _fft_conv(L, X):
    Xp = np.zeros_like(L)
    Xp[tuple(slice(0, k) for k in X.shape)] = X
    return np.real(np.fft.ifftn(np.fft.fftn(L) * np.fft.fftn(Xp)))


def _brute_conv(L, X):
    out = np.zeros_like(L)
    for i in itertools.product(*[range(d) for d in L.shape]):
        acc = 0.0
        for s in itertools.product(*[range(k) for k in X.shape]):
            src = tuple((ii - ss) % d for ii, ss, d in zip(i, s, L.shape))
            acc += L[src] * X[s]
        out[i] = acc
    return out


@pytest.mark.parametrize("dims,kdims", SHAPES)
def test_conv_matrix_is_circular_convolution_fft(dims, kdims):
    g = np.random.default_rng(1)
    L, X = g.standard_normal(dims), g.standard_normal(kdims)
    A = O.conv_matrix(L, kdims)
    assert A.shape == (int(np.prod(dims)), int(np.prod(kdims)))
    np.testing.assert_allclose((A @ X.ravel()).reshape(dims), _fft_conv(L, X), atol=1e-12)


@pytest.mark.parametrize("dims,kdims", SHAPES[:3])
def test_conv_matrix_brute_force(dims, kdims):
    g = np.random.default_rng(2)
    L, X = g.standard_normal(dims), g.standard_normal(kdims)
    np.testing.assert_allclose(O.conv(L, X), _brute_conv(L, X), atol=1e-12)


@pytest.mark.parametrize("dims,kdims", SHAPES)
def test_adjoint_identity(dims, kdims):
    g = np.random.default_rng(3)
    m, k = int(np.prod(dims)), int(np.prod(kdims))
    L, X = g.standard_normal(dims), g.standard_normal((m, k))
    lhs = float(np.sum(O.conv_matrix(L, kdims) * X))
    rhs = float(np.sum(L * O.adjoint(X, dims, kdims)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # A_k^* A_k = k I: the source of the 1/k in the L-step and of ||N||_F = ||N_A||_F / sqrt(k)
    np.testing.assert_allclose(O.adjoint(O.conv_matrix(L, kdims), dims, kdims), k * L, atol=1e-12)


def test_adjoint_matches_explicit_transpose():
    g = np.random.default_rng(4)
    dims, kdims = (4, 3, 3), (2, 2, 3)
    m, k = 36, 12
    # the explicit m x (m k) matrix of L -> vec(A_k(L)), built column by column from unit tensors
    big = np.stack([O.conv_matrix(np.eye(m)[j].reshape(dims), kdims).ravel() for j in range(m)], 1)
    X = g.standard_normal((m, k))
    np.testing.assert_allclose(O.adjoint(X, dims, kdims).ravel(), big.T @ X.ravel(), atol=1e-12)


@pytest.mark.parametrize("p", [0.1, 0.5, 0.93])
def test_convolution_sampling_set_column_counts(p):
    g = np.random.default_rng(5)
    dims, kdims = (9, 7, 5), (3, 4, 2)
    mask = (g.random(dims) < p).astype(np.uint8)
    cols = O.conv_matrix(mask, kdims).sum(axis=0)
    assert np.all(cols == mask.sum())


def test_kernel_bounds_rejected():
    with pytest.raises(ValueError):
        O.conv_matrix(np.zeros((4, 4)), (5, 1))


def test_offsets_c_order():
    assert O.kernel_offsets((2, 3))[:4] == [(0, 0), (0, 1), (0, 2), (1, 0)]


# ------------------------------------------------------------------ planted-mistake checks
def _correlation_matrix(L, kdims):
    axes = tuple(range(L.ndim))
    return np.stack([np.roll(L, shift=tuple(-x for x in s), axis=axes).ravel()
                     for s in O.kernel_offsets(kdims)], 1)


def test_pins_catch_correlation_mistake():
    g = np.random.default_rng(6)
    L, X = g.standard_normal((6, 5, 4)), g.standard_normal((3, 2, 2))
    bad = (_correlation_matrix(L, X.shape) @ X.ravel()).reshape(L.shape)
    assert np.abs(bad - _fft_conv(L, X)).max() > 1e-3


def test_pins_catch_unshifted_adjoint():
    g = np.random.default_rng(7)
    dims, kdims = (5, 4, 3), (2, 2, 2)
    L, X = g.standard_normal(dims), g.standard_normal((60, 8))
    bad_adj = X.sum(axis=1).reshape(dims)       # forgot to shift the columns back
    lhs = float(np.sum(O.conv_matrix(L, kdims) * X))
    assert abs(lhs - float(np.sum(L * bad_adj))) > 1e-3


def test_zero_padded_kernel_offsets_change_nothing():
    # Padding the innermost kernel extent (13 -> 16) with offsets whose rows of V are
    # zero leaves A_k(L)V and A_k^*(X V^T) unchanged: the padded offsets' columns of the
    # convolution matrix meet zero rows of V, and the adjoint of a zero column is zero.
    # (The reduced-precision contractions rely on this; the L-step keeps the true k.)
    rng = np.random.default_rng(5)
    dims, kd, kdp = (9, 20), (3, 13), (3, 16)
    L = rng.standard_normal(dims)
    k, kc = 3 * 13, 3 * 16
    V = np.linalg.qr(rng.standard_normal((k, k)))[0]
    Vp = np.zeros((kc, kc))
    for s0 in range(3):
        for s1 in range(13):
            Vp[s0 * 16 + s1, :k] = V[s0 * 13 + s1]
    W = O.conv_matrix(L, kd) @ V
    Wp = O.conv_matrix(L, kdp) @ Vp
    assert np.allclose(Wp[:, :k], W, atol=1e-12) and np.abs(Wp[:, k:]).max() == 0.0
    X = rng.standard_normal((L.size, k))
    Xp = np.zeros((L.size, kc))
    Xp[:, :k] = X
    assert np.allclose(O.adjoint(Xp @ Vp.T, dims, kdp), O.adjoint(X @ V.T, dims, kd), atol=1e-12)
    # but A_k'^* A_k' = k' I: the L-step must divide by the true k
    assert np.allclose(O.adjoint(O.conv_matrix(L, kdp), dims, kdp), kc * L)
