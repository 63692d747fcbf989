"""Pins of the oracle's eigenvector learning (Definition 3, eq:A, eq:cnnorm).

* The Gram matrix sum_j A_k(L_j)^T A_k(L_j) equals the circular
  autocorrelation of the references, G[s, s'] = R(s - s') with
  R = ifftn(|fftn L|^2) (Wiener-Khinchin), and trace G = k sum_j ||L_j||^2.
* Its eigenvectors are the right singular vectors of the stacked matrix of
  eq:A (checked with an SVD of the stack), sorted by descending eigenvalue.
* eq:cnnorm: with K learned from L itself, ||A_k(L)K||_{2,1} = ||A_k(L)||_*.
* For any orthogonal K, ||A_k(L)K||_{2,1} >= ||A_k(L)||_*, and K = I gives k||L||_F.
"""
import math

import numpy as np
import pytest

from oracle import icnnm_ref as O


def _refs(dims, b, seed):
    g = np.random.default_rng(seed)
    return [g.standard_normal(dims) for _ in range(b)]


def _autocorr_gram(refs, kdims):
    offs = O.kernel_offsets(kdims)
    k = len(offs)
    G = np.zeros((k, k))
    for L in refs:
        F = np.fft.fftn(L)
        R = np.real(np.fft.ifftn(np.abs(F) ** 2))
        for a, s in enumerate(offs):
            for b, t in enumerate(offs):
                d = tuple((si - ti) % m for si, ti, m in zip(s, t, L.shape))
                G[a, b] += R[d]
    return G


@pytest.mark.parametrize("dims,kdims", [((6, 5, 4), (3, 2, 2)), ((9, 8), (3, 3)), ((16,), (5,))])
def test_gram_is_autocorrelation(dims, kdims):
    refs = _refs(dims, 3, 10)
    G = O.gram(refs, kdims)
    np.testing.assert_allclose(G, _autocorr_gram(refs, kdims), rtol=0, atol=1e-10 * np.abs(G).max())
    k = int(np.prod(kdims))
    assert abs(np.trace(G) - k * sum(float(np.sum(L ** 2)) for L in refs)) < 1e-9 * np.trace(G)


def test_learn_matches_stacked_svd():
    dims, kdims = (6, 5, 4), (3, 2, 2)
    refs = _refs(dims, 4, 11)
    V, w = O.learn(refs, kdims)
    k = V.shape[0]
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-12)
    assert np.all(np.diff(w) <= 1e-9 * w[0])
    A = np.concatenate([O.conv_matrix(L, kdims) for L in refs], 0)
    _, sv, Vt = np.linalg.svd(A, full_matrices=False)
    np.testing.assert_allclose(w, sv ** 2, rtol=1e-10, atol=1e-10 * w[0])
    # eigenvalues here are simple: each eigenvector equals a right singular vector up to sign
    dots = np.abs(np.sum(V * Vt.T, axis=0))
    np.testing.assert_allclose(dots, 1.0, atol=1e-8)
    G = O.gram(refs, kdims)
    assert np.abs(G @ V - V * w).max() < 1e-10 * w[0]
    # deterministic sign convention: the largest-magnitude entry of each column is positive
    assert np.all(V[np.argmax(np.abs(V), 0), np.arange(k)] > 0)


def test_learn_is_ensemble_maximizer():
    """sigma_1 of Definition 3 is the max of sum_j ||L_j * X||_F^2 over unit X."""
    dims, kdims = (5, 4, 3), (2, 2, 2)
    refs = _refs(dims, 3, 12)
    V, w = O.learn(refs, kdims)
    val = lambda X: sum(float(np.sum(O.conv(L, X.reshape(kdims)) ** 2)) for L in refs)
    assert abs(val(V[:, 0]) - w[0]) < 1e-9 * w[0]
    g = np.random.default_rng(0)
    for _ in range(50):
        X = g.standard_normal(int(np.prod(kdims)))
        X /= np.linalg.norm(X)
        assert val(X) <= w[0] * (1 + 1e-12)


@pytest.mark.parametrize("dims,kdims", [((6, 5, 4), (3, 2, 2)), ((8, 7), (3, 2))])
def test_eigenvector_rewrite_of_nuclear_norm(dims, kdims):
    L = np.random.default_rng(13).standard_normal(dims)
    V, _ = O.learn([L], kdims)
    A = O.conv_matrix(L, kdims)
    nuc = float(np.linalg.svd(A, compute_uv=False).sum())
    assert abs(O.norm21(A @ V) - nuc) < 1e-10 * nuc


def test_objective_bounds():
    dims, kdims = (6, 5, 4), (3, 2, 2)
    g = np.random.default_rng(14)
    L = g.standard_normal(dims)
    A = O.conv_matrix(L, kdims)
    nuc = float(np.linalg.svd(A, compute_uv=False).sum())
    k = A.shape[1]
    for _ in range(5):
        K, _ = np.linalg.qr(g.standard_normal((k, k)))
        assert O.norm21(A @ K) >= nuc * (1 - 1e-12)
    assert abs(O.norm21(A) - k * np.linalg.norm(L)) < 1e-10 * k * np.linalg.norm(L)


def test_ground_truth_eigenvectors_have_unit_alpha():
    """Table 1, ground-truth scheme: K learned from L0 itself gives alpha_K = 1 and
    r_K equal to the convolution rank."""
    dims, kdims = (8, 8, 4), (4, 4, 2)
    x = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    L0 = np.cos(2 * np.pi * (x[0] / 8 + 2 * x[1] / 8 + x[2] / 4) + 0.3) \
        + 0.5 * np.cos(2 * np.pi * (3 * x[0] / 8 + x[1] / 8) + 1.1)
    V, _ = O.learn([L0], kdims)
    assert abs(O.spectral_correlation(L0, V, kdims) - 1.0) < 1e-9
    r0 = int(np.linalg.matrix_rank(O.conv_matrix(L0, kdims), tol=1e-8))
    assert O.relative_rank(L0, V, kdims) == r0 == 4


def _fft_conv(L, X):
    """Circular convolution L * X by the convolution theorem, X zero-padded to L's shape."""
    Xp = np.zeros(L.shape)
    Xp[tuple(slice(0, k) for k in X.shape)] = X
    return np.real(np.fft.ifftn(np.fft.fftn(L) * np.fft.fftn(Xp)))


@pytest.mark.parametrize("dims,kdims", [((8, 6, 5), (3, 2, 2)), ((10, 7), (4, 3))])
def test_relative_eigenvalues_by_fft_convolution(dims, kdims):
    """Definition 2: sigma^K_i = ||L0 * kappa_i||_F, here with the convolution done by
    FFT and kappa_i the i-th column of V reshaped to the kernel."""
    g = np.random.default_rng(15)
    L0 = g.standard_normal(dims)
    V, _ = O.learn(_refs(dims, 3, 16), kdims)
    want = np.array([np.linalg.norm(_fft_conv(L0, V[:, i].reshape(kdims))) for i in range(V.shape[1])])
    np.testing.assert_allclose(O.relative_eigs(L0, V, kdims), want, rtol=1e-11, atol=1e-12 * want.max())


def test_spectral_correlation_by_autocorrelation_gram():
    """eq:alphaK: alpha_K^2 is the largest eigenvalue of D V^T G V D, with G the Gram of
    A_k(L0) built from the FFT autocorrelation and D = diag(1/sigma^K_i) on the support."""
    dims, kdims = (8, 6, 5), (3, 2, 2)
    g = np.random.default_rng(17)
    L0 = g.standard_normal(dims)
    V, _ = O.learn(_refs(dims, 3, 18), kdims)
    C = V.T @ _autocorr_gram([L0], kdims) @ V
    s = np.sqrt(np.diag(C))
    d = 1.0 / s
    alpha = math.sqrt(float(np.linalg.eigvalsh(C * np.outer(d, d)).max()))
    assert abs(O.spectral_correlation(L0, V, kdims) - alpha) < 1e-10 * alpha
    assert O.relative_rank(L0, V, kdims) == V.shape[1]
