"""Pins of the oracle's ADMM solver (Section III-D) and of the programs it solves.

* Z-step: the l2,1 proximal map satisfies its optimality condition
  q_i - z_i in tau * subdiff ||z_i||.
* L-step: the paper's closed form is a stationary point of the augmented
  Lagrangian in L (checked against finite differences of the Lagrangian
  written out term by term), on Omega^perp for lam = inf and everywhere for
  finite lam.
* Whole solver: K = I gives zero-fill, full sampling returns M bit-exactly,
  empty sampling returns 0, every iterate keeps P_Omega(L) = P_Omega(M)
  bit-exactly, a planted low-convolution-rank tensor is recovered with the
  ground-truth eigenvectors, the KKT residuals of eq:InductiveCNNM vanish,
  and the optimal objective agrees with an independent primal-dual
  (Chambolle-Pock) solver of the same convex program, for lam = inf and for
  the penalized eq:admm.
"""
import math

import numpy as np
import pytest

from oracle import icnnm_ref as O


def _problem(dims=(8, 6, 4), kdims=(3, 3, 2), p_obs=0.6, seed=0, b=6):
    g = np.random.default_rng(seed)
    x = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    M = sum(np.cos(2 * np.pi * sum(int(g.integers(0, d // 2 + 1)) * xi / d
                                   for xi, d in zip(x, dims)) + g.uniform(0, 6.28))
            for _ in range(3)) + 0.01 * g.standard_normal(dims)
    mask = (g.random(dims) < p_obs).astype(np.uint8)
    refs = [g.standard_normal(dims) for _ in range(b)]
    V, _ = O.learn(refs, kdims)
    return M, mask, V, kdims


def test_prox_optimality():
    g = np.random.default_rng(1)
    Q = g.standard_normal((40, 6)) * np.array([0.01, 0.1, 1, 5, 0, 2])
    tau = 0.7
    Z = O.prox_l21(Q, tau)
    for i in range(Q.shape[1]):
        q, z = Q[:, i], Z[:, i]
        nz = np.linalg.norm(z)
        if nz > 0:
            np.testing.assert_allclose(q - z, tau * z / nz, atol=1e-12)
        else:
            assert np.linalg.norm(q) <= tau + 1e-12


def _lagrangian(L, Z, Y, theta, V, M, mask, kdims, lam):
    W = O.conv_matrix(L, kdims) @ V
    k = V.shape[0]
    val = O.norm21(Z) + float(np.sum((Z - W) * Y)) + 0.5 * theta * float(np.sum((Z - W) ** 2))
    if not math.isinf(lam):
        val += 0.5 * lam * k * float(np.sum(O.project(L - M, mask) ** 2))
    return val


@pytest.mark.parametrize("lam", [math.inf, 1000.0, 3.0])
def test_l_step_is_lagrangian_minimizer(lam):
    M, mask, V, kdims = _problem()
    g = np.random.default_rng(2)
    m, k = M.size, V.shape[0]
    Y, Z, theta = g.standard_normal((m, k)), g.standard_normal((m, k)), 0.8
    L = O.l_step(Y, Z, theta, V, M, mask, kdims, lam)
    if math.isinf(lam):
        assert np.array_equal(L[mask != 0], M[mask != 0])
    free = np.flatnonzero(mask.ravel() == 0) if math.isinf(lam) else np.arange(m)
    h = 1e-5
    base = _lagrangian(L, Z, Y, theta, V, M, mask, kdims, lam)
    for j in g.choice(free, size=12, replace=False):
        E = np.zeros(m)
        E[j] = h
        E = E.reshape(M.shape)
        up = _lagrangian(L + E, Z, Y, theta, V, M, mask, kdims, lam)
        dn = _lagrangian(L - E, Z, Y, theta, V, M, mask, kdims, lam)
        grad = (up - dn) / (2 * h)
        curv = (up + dn - 2 * base) / h ** 2
        assert abs(grad) < 1e-5 * max(1.0, curv)
        assert curv > 0


def test_identity_eigenvectors_give_zero_fill():
    M, mask, V, kdims = _problem()
    k = V.shape[0]
    L, _ = O.solve(M, mask, np.eye(k), kdims, 60)
    np.testing.assert_array_equal(L[mask != 0], M[mask != 0])
    assert np.abs(L[mask == 0]).max() < 1e-12 * np.abs(M).max()


def test_full_sampling_returns_M_bitwise():
    M, mask, V, kdims = _problem()
    full = np.ones_like(mask)
    L, _ = O.solve(M.astype(np.float32), full, V, kdims, 10)
    assert np.array_equal(L, M.astype(np.float32).astype(np.float64))


def test_empty_sampling_returns_zero():
    M, mask, V, kdims = _problem()
    L, info = O.solve(M, np.zeros_like(mask), V, kdims, 10)
    assert np.all(L == 0) and info["theta0"] == 1.0


def test_every_iterate_keeps_observed_entries():
    M, mask, V, kdims = _problem()
    M32 = M.astype(np.float32)
    _, info = O.solve(M32, mask, V, kdims, 15, history=True)
    for L in info["history"]:
        assert np.array_equal(L[mask != 0], M32[mask != 0].astype(np.float64))


def test_planted_recovery_with_ground_truth_eigenvectors():
    """Noiseless case of Theorem 1 with K learned from L0 (alpha_K = 1, Table 1 G.T.)."""
    dims, kdims = (16, 16, 8), (4, 4, 2)
    x = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    g = np.random.default_rng(3)
    L0 = sum(np.cos(2 * np.pi * sum(int(g.integers(0, d // 2 + 1)) * xi / d
                                    for xi, d in zip(x, dims)) + g.uniform(0, 6.28))
             for _ in range(3))
    mask = (g.random(dims) < 0.7).astype(np.uint8)
    V, _ = O.learn([L0], kdims)
    L, _ = O.solve(L0, mask, V, kdims, 100)
    assert np.linalg.norm(L - L0) / np.linalg.norm(L0) < 1e-10


def _pdhg(M, mask, V, kdims, lam=math.inf, iters=40000):
    """Chambolle-Pock for min_L ||A_k(L)K||_{2,1} + g(L); g is the indicator of
    P_Omega L = P_Omega M (lam = inf) or (lam k/2)||P_Omega(L - M)||^2.
    Operator norm of L -> A_k(L)K is sqrt(k)."""
    k = V.shape[0]
    obs = mask != 0
    tau = sigma = 0.99 / math.sqrt(k)
    L = np.where(obs, M, 0.0)
    Lbar = L.copy()
    Y = np.zeros((M.size, k))
    for _ in range(iters):
        Y = Y + sigma * (O.conv_matrix(Lbar, kdims) @ V)
        Y = Y / np.maximum(1.0, np.linalg.norm(Y, axis=0))
        Lt = L - tau * O.adjoint(Y @ V.T, M.shape, kdims)
        if math.isinf(lam):
            Ln = np.where(obs, M, Lt)
        else:
            c = tau * lam * k
            Ln = np.where(obs, (Lt + c * M) / (1 + c), Lt)
        Lbar = 2 * Ln - L
        L = Ln
    return L


@pytest.mark.parametrize("lam", [math.inf, 2.0])
def test_optimum_matches_independent_primal_dual_solver(lam):
    dims, kdims = (5, 4, 3), (2, 2, 2)
    M, mask, V, _ = _problem(dims, kdims, 0.5, seed=4, b=4)
    L_admm, info = O.solve(M, mask, V, kdims, 400, lam=lam)
    L_cp = _pdhg(M, mask, V, kdims, lam, iters=30000)
    f_admm = O.objective(L_admm, V, kdims, M, mask, lam)
    f_cp = O.objective(L_cp, V, kdims, M, mask, lam)
    assert abs(f_admm - f_cp) < 2e-6 * f_cp, (f_admm, f_cp)


def test_kkt_residuals_vanish():
    """The L-step makes P_Omega^perp A_k^*(Y K^T) vanish at every iterate (up to rounding
    amplified by theta); convergence shows in the primal residual, dual feasibility
    and the alignment -Y_i = W_i/||W_i|| on the support."""
    M, mask, V, kdims = _problem(seed=5)
    scale = np.linalg.norm(M)
    res = {}
    for n in (4, 100):
        L, info = O.solve(M, mask, V, kdims, n)
        res[n] = (O.kkt(L, info["Y"], V, kdims, mask), info["r_primal"])
    (k4, p4), (k100, p100) = res[4], res[100]
    assert k4["stationarity"] < 1e-10 * scale and k100["stationarity"] < 1e-8 * scale
    assert p100 < 1e-6 * p4
    assert k100["dual_max"] < 1 + 1e-4
    assert k100["alignment"] < 1e-2 * k4["alignment"] and k100["alignment"] < 1e-4


def test_penalized_mode_does_not_pin_observed_entries():
    M, mask, V, kdims = _problem(seed=6)
    L, _ = O.solve(M, mask, V, kdims, 200, lam=1000.0)
    dev = np.abs(L - M)[mask != 0].max()
    assert 0 < dev < 1e-2


def test_stopping_rule():
    M, mask, V, kdims = _problem(seed=7)
    L, info = O.solve(M, mask, V, kdims, 1000, tol=1e-4)
    assert info["converged"] and info["iters"] < 1000
    assert max(info["r_primal"], info["r_change"]) <= 1e-4


def test_penalized_objective_hand_value():
    """eq:admm on a 3 x 2 tensor with a 2 x 1 kernel (k = 2) and K = I, by hand.

    L has a single 1 at (0, 0), so both columns of A_k(L) (L and L shifted by one
    row) have norm 1 and ||A_k(L)I||_{2,1} = 2. Observed entries (0,0), (1,0), (2,1)
    with M values 3, 1, 2 give L - M = -2, -1, -2 there, ||P_Omega(L - M)||^2 = 9,
    and the penalty (lambda k / 2) * 9 = 9 lambda: 9002 for lambda = 1000.
    """
    L = np.array([[1.0, 0.0], [0.0, 0.0], [0.0, 0.0]])
    M = np.array([[3.0, 7.0], [1.0, 7.0], [7.0, 2.0]])
    mask = np.array([[1, 0], [1, 0], [0, 1]], dtype=np.uint8)
    V = np.eye(2)
    assert O.objective(L, V, (2, 1)) == 2.0
    assert O.objective(L, V, (2, 1), M, mask, 1000.0) == 9002.0
    assert O.objective(L, V, (2, 1), M, mask, 0.5) == 2.0 + 4.5


@pytest.mark.parametrize("lam", [2.0, 50.0])
def test_penalized_solution_minimizes_objective(lam):
    """The ADMM limit of the penalized program (whose L-step is the paper's closed
    form) is a minimizer of objective(): no perturbation lowers it. A wrong
    weight of the penalty term in objective() moves its minimizer away."""
    dims, kdims = (5, 4, 3), (2, 2, 2)
    M, mask, V, _ = _problem(dims, kdims, 0.5, seed=8, b=4)
    L, _ = O.solve(M, mask, V, kdims, 600, lam=lam)
    f0 = O.objective(L, V, kdims, M, mask, lam)
    g = np.random.default_rng(9)
    eps = 1e-3 * np.linalg.norm(L) / math.sqrt(L.size)
    for _ in range(20):
        E = g.standard_normal(dims)
        E *= eps / np.linalg.norm(E) * math.sqrt(L.size)
        assert O.objective(L + E, V, kdims, M, mask, lam) >= f0 - 1e-9 * f0
    # the same check fails for a doubled penalty weight (what a dropped 1/2 would give)
    twice = lambda X: O.objective(X, V, kdims) + lam * int(np.prod(kdims)) * float(
        np.sum(O.project(X - M, mask) ** 2))
    lower = 0
    for _ in range(20):
        E = g.standard_normal(dims)
        E *= eps / np.linalg.norm(E) * math.sqrt(L.size)
        lower += twice(L + E) < twice(L) or twice(L - E) < twice(L)
    assert lower > 0
