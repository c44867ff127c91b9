"""Pins of the oracle's normal-equation operator (Sec. 5.1, eq. (19)), prior
(Sec. 3, eq. (13)), modified Jacobi preconditioner (Sec. 5.1) and PCG."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as WL
from tests.dense import assemble
from tests.tiny import tiny_config


def _sigmas(cfg):
    return [0.05 + 0.01 * m for m in range(len(cfg["wfs"]))]


def _blocks(cfg, sysm, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for sen in sysm.sensors:
        S = sen["S"]
        beta = rng.standard_normal((S, 2))
        tau_f2 = 0.8
        sg2 = 0.04
        blk = np.zeros((S, 3))
        for q in range(S):
            C = sg2 * (np.eye(2) + tau_f2 * np.outer(beta[q], beta[q]))   # eq. (16)
            Ci = np.linalg.inv(C)
            blk[q] = Ci[0, 0], Ci[0, 1], Ci[1, 1]
        out.append(blk)
    return out


@pytest.fixture(scope="module")
def tiny():
    cfg = tiny_config()
    A, parts, sysm = assemble(cfg, _sigmas(cfg))
    return cfg, A, sysm


def test_apply_matches_dense_assembly(tiny):
    cfg, A, S = tiny
    rng = np.random.default_rng(1)
    for _ in range(3):
        v = rng.standard_normal(S.n)
        ref = A @ v
        assert np.linalg.norm(S.apply_A(v) - ref) < 1e-12 * np.linalg.norm(ref)


def test_apply_matches_dense_with_elongation_blocks():
    cfg = tiny_config()
    S0 = O.System(cfg, _sigmas(cfg))
    blk = _blocks(cfg, S0)
    A, _, S = assemble(cfg, _sigmas(cfg), blk)
    v = np.random.default_rng(2).standard_normal(S.n)
    assert np.linalg.norm(S.apply_A(v) - A @ v) < 1e-12 * np.linalg.norm(A @ v)


def test_operator_is_spd(tiny):
    cfg, A, S = tiny
    assert np.max(np.abs(A - A.T)) < 1e-12 * np.max(np.abs(A))
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert lam[0] > 0.0
    assert lam[0] >= cfg["alpha"] * S.D.min() * (1 - 1e-9)


def test_matrix_free_symmetry_random_vectors(tiny):
    cfg, A, S = tiny
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(S.n), rng.standard_normal(S.n)
    lhs, rhs = x @ S.apply_A(y), y @ S.apply_A(x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_rhs_is_adjoint_of_forward(tiny):
    cfg, A, S = tiny
    rng = np.random.default_rng(4)
    c = rng.standard_normal(S.n)
    s = rng.standard_normal(S.n_slopes)
    # <W P^T G^T N s, c> = <N s, G P W^-1 c>
    lhs = S.rhs(s) @ c
    rhs = S.weight(s) @ S.forward(c)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_prior_values_c1():
    # values of the reading D = d^2 (L0^-11/3 + nu_k^11/3) / c_rho for the
    # ground layer of the 8 m telescope (w = 0.6, r0 = 0.15 m, L0 = 25 m,
    # d = 0.5 m), computed independently of the oracle.
    S = O.System(WL.config_c1(), [1.0, 1.0, 1.0])
    np.testing.assert_allclose(S.prior_level_values(0),
                               [7.67154679e-01, 6.04149358e-02, 4.76266838e-03, 3.80326924e-04],
                               rtol=1e-8)


def test_prior_matches_inverse_coefficient_variance():
    # Bernstein-Jackson equivalence (Sec. 3, eqs. (11)-(13)): the diagonal
    # prior is equivalent to the von Karman inverse covariance, so D_k times
    # the empirical variance of level-k coefficients of von Karman screens is
    # of order one and nearly scale independent on the fine levels.
    cfg = WL.config_c1()
    S = O.System(cfg, [1.0, 1.0, 1.0])
    lev = O.coefficient_level(64, 4)
    acc = np.zeros(4)
    for f in range(6):
        scr = WL.layer_screens(cfg, 100 + f)
        c = O.fdwt2(scr[0], 4)
        for k in range(1, 5):
            sel = (lev == k) & ~((np.arange(64)[:, None] < 4) & (np.arange(64)[None, :] < 4))
            acc[k - 1] += np.mean(c[sel] ** 2) / 6
    prod = acc * S.prior_level_values(0)
    assert np.all(prod[:3] > 0.1) and np.all(prod[:3] < 10.0)
    assert prod[:3].max() / prod[:3].min() < 3.0


def test_jacobi_three_ways(tiny):
    cfg, A, S = tiny
    Ap, _, _ = assemble(cfg, _sigmas(cfg), precond_only=True)
    dense_diag = np.diag(Ap)
    sep = S.jacobi_separable()
    brute = S.jacobi_bruteforce()
    assert np.max(np.abs(sep - dense_diag) / dense_diag) < 1e-12
    assert np.max(np.abs(brute - dense_diag) / dense_diag) < 1e-12


def test_jacobi_with_blocks_and_aggregated_sensor():
    cfg = tiny_config()
    for w in cfg["wfs"]:
        w["in_precond"] = True              # every sensor, including the 2x2 one
    S0 = O.System(cfg, _sigmas(cfg))
    blk = _blocks(cfg, S0, seed=5)
    Ap, _, S = assemble(cfg, _sigmas(cfg), blk, precond_only=True)
    assert np.max(np.abs(S.jacobi_separable() - np.diag(Ap)) / np.diag(Ap)) < 1e-12


def test_jacobi_separable_vs_brute_c1_sample():
    S = O.System(WL.config_c1(), [0.5, 0.55, 0.6])
    J = S.jacobi_separable()
    idx = np.random.default_rng(0).choice(S.n, 200, replace=False)
    assert np.max(np.abs(S.jacobi_bruteforce(idx) - J[idx]) / J[idx]) < 1e-13


def test_pcg_iterate_matches_krylov_galerkin(tiny):
    # the k-th PCG iterate is x0 + V (V^T A V)^-1 V^T r0 for any basis V of
    # the Krylov space K_k(J^-1 A, J^-1 r0).
    cfg, A, S = tiny
    rng = np.random.default_rng(8)
    b = rng.standard_normal(S.n)
    x0 = rng.standard_normal(S.n)
    Jd = S.jacobi_separable()
    for k in (1, 3, 6):
        x, info = O.pcg(S.apply_A, b, k, x0=x0, jacobi=Jd)
        r0 = b - A @ x0
        v = r0 / Jd
        V = []
        for _ in range(k):
            for u in V:
                v = v - (u @ v) * u
            v = v / np.linalg.norm(v)
            V.append(v)
            v = (A @ v) / Jd
        V = np.array(V).T
        xk = x0 + V @ np.linalg.solve(V.T @ A @ V, V.T @ r0)
        assert np.linalg.norm(x - xk) < 1e-9 * np.linalg.norm(xk)


def test_pcg_converges_to_cholesky():
    # a stronger prior weight keeps cond(J^-1 A) near 240 so that a few
    # hundred iterations reach the direct solution to rounding level
    cfg = tiny_config()
    cfg["alpha"] = 1000.0
    A, _, S = assemble(cfg, _sigmas(cfg))
    b = np.random.default_rng(9).standard_normal(S.n)
    xs = sla.cho_solve(sla.cho_factor(A), b)
    x, info = O.pcg(S.apply_A, b, 300, jacobi=S.jacobi_separable())
    assert np.linalg.norm(x - xs) < 1e-10 * np.linalg.norm(xs)


def test_pcg_energy_norm_decreases_and_plain_cg(tiny):
    cfg, A, S = tiny
    b = np.random.default_rng(10).standard_normal(S.n)
    xs = sla.cho_solve(sla.cho_factor(A), b)
    Jd = S.jacobi_separable()
    errs = []
    for k in range(0, 12):
        x, _ = O.pcg(S.apply_A, b, k, jacobi=Jd)
        e = x - xs
        errs.append(e @ A @ e)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    x, info = O.pcg(S.apply_A, b, 5)                         # plain CG (J = I)
    assert info["iters"] == 5 and info["status"] == O.STATUS_OK


def test_pcg_breakdown_and_zero_rhs():
    cfg = tiny_config()
    S = O.System(cfg, _sigmas(cfg))
    x, info = O.pcg(S.apply_A, np.zeros(S.n), 5, jacobi=S.jacobi_separable())
    assert info["status"] == O.STATUS_CONVERGED and not x.any()
    x, info = O.pcg(lambda v: -v, np.ones(4), 3)
    assert info["status"] == O.STATUS_BREAKDOWN
