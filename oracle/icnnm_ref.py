"""FP64 CPU oracle for Inductive Convolution Nuclear Norm Minimization (ICNNM).

TEST INFRASTRUCTURE ONLY. This module is the slow, explicit reference that the
GPU library is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.

Every operator is formed explicitly in float64 with NumPy, with no blocking,
fusion or reordering beyond what the definitions state:

* circular convolution and the convolution matrix A_k(L) (Section II-B, eq:ak):
  column s of A_k(L) is vec(L) circularly shifted by the kernel offset s, so
  [A_k(L)]_{i,s} = L_{(i-s) mod m} per dimension;
* its Hermitian adjoint A_k^* (Section III-D, L-step): transposed convolutions
  summed back, [A_k^*(X)]_t = sum_s X_{(t+s) mod m, s};
* the ensemble convolution eigenvectors learned from reference tensors
  (Definition 3 and eq:A): eigenvectors of sum_j A_k(L_j)^T A_k(L_j);
* the ADMM iteration for the ICNNM program (eq:InductiveCNNM) and its
  penalized form (eq:admm), in the literal unscaled multiplier form of the
  augmented Lagrangian of Section III-D.

Readings of points the paper leaves open (each listed in the design notes):
vectorisation is C-order for tensors and for kernel offsets; indices are
0-based with offsets s_j in [0, k_j); the Y/theta rule is the standard
inexact-ALM update Y <- Y + theta (Z - A_k(L)K), theta <- min(rho theta,
theta_max); L^0 = P_Omega(M), Y^0 = 0, theta_0 = 1.25 / ||A_k(L^0)K||_{2,inf}
(1.0 when that norm is zero); lambda = +inf selects the exact-constraint
program, for which the L-step is the lambda -> inf limit of the paper's
closed form; a column with zero norm shrinks to zero.
"""
from __future__ import annotations

import math

import numpy as np


# ----------------------------------------------------------------------------- operators

def kernel_offsets(kdims):
    """All kernel offsets s = (s_1..s_n), s_j in [0, k_j), in C order (row s of V)."""
    return [tuple(int(x) for x in s) for s in np.ndindex(*tuple(kdims))]


def _check(dims, kdims):
    dims, kdims = tuple(int(d) for d in dims), tuple(int(d) for d in kdims)
    if len(dims) != len(kdims) or any(k < 1 or k > m for k, m in zip(kdims, dims)):
        raise ValueError(f"kernel {kdims} must satisfy 1 <= k_j <= m_j for tensor {dims}")
    return dims, kdims


def conv_matrix(L, kdims):
    """A_k(L) in R^{m x k} (eq:ak): column s is vec(L) shifted circularly by s.

    ``np.roll(L, s)[i] == L[(i - s) mod m]`` per axis, which is the definition
    [A_k(L)]_{i,s} = L_{i-s} with the paper's wrap-around convention.
    """
    L = np.asarray(L, dtype=np.float64)
    dims, kdims = _check(L.shape, kdims)
    axes = tuple(range(L.ndim))
    cols = [np.roll(L, shift=s, axis=axes).ravel() for s in kernel_offsets(kdims)]
    return np.stack(cols, axis=1)


def conv(L, X):
    """Circular convolution L * X (Section II-B) through the convolution matrix."""
    X = np.asarray(X, dtype=np.float64)
    return (conv_matrix(L, X.shape) @ X.ravel()).reshape(np.shape(L))


def adjoint(X, dims, kdims):
    """A_k^*(X): the adjoint of A_k, [A_k^*(X)]_t = sum_s X_{(t+s) mod m, s}.

    Each column of X is shifted back by its kernel offset and the k tensors are
    summed (transposed convolutions summed back into tensor space).
    """
    X = np.asarray(X, dtype=np.float64)
    dims, kdims = _check(dims, kdims)
    axes = tuple(range(len(dims)))
    T = np.zeros(dims, dtype=np.float64)
    for col, s in enumerate(kernel_offsets(kdims)):
        T += np.roll(X[:, col].reshape(dims), shift=tuple(-x for x in s), axis=axes)
    return T


def project(L, mask):
    """P_Omega: keep observed entries, zero the rest (Section II-A)."""
    return np.where(np.asarray(mask) != 0, np.asarray(L, dtype=np.float64), 0.0)


def norm21(X):
    """||X||_{2,1}: sum of column l2 norms (Section II-A)."""
    return float(np.linalg.norm(X, axis=0).sum())


# ----------------------------------------------------------------------------- learning V

def gram(refs, kdims):
    """sum_j A_k(L_j)^T A_k(L_j), i.e. A^T A for the stacked matrix of eq:A."""
    k = int(np.prod(kdims))
    G = np.zeros((k, k), dtype=np.float64)
    for L in refs:
        A = conv_matrix(L, kdims)
        G += A.T @ A
    return G


def normalize_signs(V):
    """Flip each column so its largest-magnitude entry is positive (first on ties)."""
    V = np.array(V, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(V), axis=0)
    sgn = np.sign(V[idx, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    return V * sgn


def learn(refs, kdims):
    """Ensemble convolution eigenvectors (Definition 3): the right singular vectors
    of the stacked convolution matrix (eq:A), computed as the eigenvectors of its
    Gram matrix, all k of them, sorted by descending eigenvalue.

    Returns (V, eigenvalues): V is k x k, row s = kernel offset (C order),
    column i = i-th convolution eigenvector.
    """
    G = gram(refs, kdims)
    w, V = np.linalg.eigh(G)
    order = np.argsort(-w, kind="stable")
    return normalize_signs(V[:, order]), w[order]


# ----------------------------------------------------------------------------- solver

def prox_l21(Q, tau):
    """argmin_Z tau ||Z||_{2,1} + 1/2 ||Z - Q||_F^2 (the Z-step, Section III-D):
    z_i = max(0, 1 - tau/||q_i||) q_i, and z_i = 0 when ||q_i|| = 0."""
    nrm = np.linalg.norm(Q, axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        shrink = np.where(nrm > 0, np.maximum(0.0, 1.0 - tau / nrm), 0.0)
    return Q * shrink


def l_step(Y, Z, theta, V, M, mask, kdims, lam=math.inf):
    """Closed-form L-step (Section III-D):
    L = (A_k^*((Y + theta Z)K^T)/k + lam P_Omega(M)) / (lam Theta_Omega + theta);
    for lam = inf, L = M on Omega and A_k^*((Y + theta Z)K^T)/(k theta) elsewhere."""
    M = np.asarray(M, dtype=np.float64)
    theta_mask = np.asarray(mask) != 0
    k = int(np.prod(kdims))
    T = adjoint((Y + theta * Z) @ np.asarray(V, dtype=np.float64).T, M.shape, kdims)
    if math.isinf(lam):
        return np.where(theta_mask, M, T / (k * theta))
    return (T / k + lam * np.where(theta_mask, M, 0.0)) / (lam * theta_mask + theta)


def default_theta0(W):
    n = float(np.linalg.norm(W, axis=0).max()) if W.size else 0.0
    return 1.25 / n if n > 0 else 1.0


def solve(M, mask, V, kdims, iters, lam=math.inf, theta0=0.0, rho=1.1,
          theta_max=1e10, tol=0.0, history=False):
    """ADMM for ICNNM (Section III-D) in the literal unscaled form.

    Splitting Z = A_k(L)K with multiplier Y and penalty theta:

    * Z-step: column-wise l2,1 proximal map of Q = A_k(L)K - Y/theta with
      threshold 1/theta, z_i = max(0, 1 - 1/(theta ||q_i||)) q_i;
    * L-step: L = (A_k^*((Y + theta Z)K^T)/k + lam P_Omega(M)) / (lam Theta + theta),
      element-wise; for lam = inf this is P_Omega(M) on Omega and
      A_k^*((Y + theta Z)K^T)/(k theta) elsewhere;
    * Y <- Y + theta (Z - A_k(L)K);  theta <- min(rho theta, theta_max).

    Runs ``iters`` iterations, or stops early when tol > 0 and
    max(r_primal, r_change) <= tol, with r_primal = ||Z - A_k(L)K||_F /
    (sqrt(k) ||P_Omega M||_F) and r_change = ||L^t - L^{t-1}||_F / ||P_Omega M||_F.
    """
    M = np.asarray(M, dtype=np.float64)
    theta_mask = np.asarray(mask) != 0
    V = np.asarray(V, dtype=np.float64)
    dims, kdims = _check(M.shape, kdims)
    k = int(np.prod(kdims))
    if V.shape != (k, k):
        raise ValueError(f"V must be {k}x{k}")
    PM = np.where(theta_mask, M, 0.0)
    denom = float(np.linalg.norm(PM)) or 1.0

    L = PM.copy()
    W = conv_matrix(L, kdims) @ V
    Y = np.zeros_like(W)
    theta = float(theta0) if theta0 and theta0 > 0 else default_theta0(W)
    info = {"theta0": theta, "iters": 0, "converged": False,
            "r_primal": float("nan"), "r_change": float("nan")}
    hist = []
    for t in range(int(iters)):
        Z = prox_l21(W - Y / theta, 1.0 / theta)
        L_new = l_step(Y, Z, theta, V, M, mask, kdims, lam)
        W = conv_matrix(L_new, kdims) @ V
        Y = Y + theta * (Z - W)
        r_primal = float(np.linalg.norm(Z - W)) / (math.sqrt(k) * denom)
        r_change = float(np.linalg.norm(L_new - L)) / denom
        L = L_new
        info.update(iters=t + 1, r_primal=r_primal, r_change=r_change, theta_used=theta)
        if history:
            hist.append(L.copy())
        theta = min(rho * theta, theta_max)
        if tol > 0 and max(r_primal, r_change) <= tol:
            info["converged"] = True
            break
    info["theta_final"] = theta
    info["objective"] = objective(L, V, kdims, M=M, mask=mask, lam=lam)
    info["Y"] = Y
    if history:
        info["history"] = hist
    return L, info


def objective(L, V, kdims, M=None, mask=None, lam=math.inf):
    """||A_k(L)K||_{2,1} (eq:InductiveCNNM), plus (lam k/2)||P_Omega(L-M)||_F^2 (eq:admm)."""
    f = norm21(conv_matrix(L, kdims) @ np.asarray(V, dtype=np.float64))
    if not math.isinf(lam) and M is not None:
        k = int(np.prod(kdims))
        f += 0.5 * lam * k * float(np.sum(project(np.asarray(L) - np.asarray(M), mask) ** 2))
    return f


def kkt(L, Y, V, kdims, mask):
    """Optimality residuals of the exact-constraint program at (L, Y).

    From the Lagrangian of Section III-D at a fixed point Z = A_k(L)K:
    * stationarity: P_Omega^perp A_k^*(Y K^T) = 0;
    * dual feasibility: max_i ||Y_i|| <= 1;
    * alignment on the support: -Y_i = W_i / ||W_i|| for nonzero columns W_i.
    """
    V = np.asarray(V, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    W = conv_matrix(L, kdims) @ V
    stat = adjoint(Y @ V.T, L.shape, kdims)
    stat = np.where(np.asarray(mask) != 0, 0.0, stat)
    wn = np.linalg.norm(W, axis=0)
    yn = np.linalg.norm(Y, axis=0)
    big = wn > 1e-8 * max(wn.max(), 1e-300)
    align = 0.0
    if big.any():
        align = float(np.abs(-Y[:, big] - W[:, big] / wn[big]).max())
    return {"stationarity": float(np.linalg.norm(stat)), "dual_max": float(yn.max()),
            "alignment": align}


# ----------------------------------------------------------------------------- diagnostics

def relative_eigs(L0, V, kdims):
    """Relative convolution eigenvalues sigma^K_i = ||L0 * kappa_i||_F (Definition 2)."""
    return np.linalg.norm(conv_matrix(L0, kdims) @ np.asarray(V, dtype=np.float64), axis=0)


def relative_rank(L0, V, kdims, rtol=1e-10):
    """r_K(L0): number of nonzero relative convolution eigenvalues (eq:rkL0)."""
    s = relative_eigs(L0, V, kdims)
    return int(np.sum(s > rtol * max(s.max(), 1e-300)))


def spectral_correlation(L0, V, kdims, rtol=1e-10):
    """alpha_K(L0) = ||A_k(L0) K D|| (eq:alphaK), D = diag(1/sigma^K_i) on the support."""
    W = conv_matrix(L0, kdims) @ np.asarray(V, dtype=np.float64)
    s = np.linalg.norm(W, axis=0)
    sup = s > rtol * max(s.max(), 1e-300)
    d = np.zeros_like(s)
    d[sup] = 1.0 / s[sup]
    return float(np.linalg.norm(W * d, 2))
