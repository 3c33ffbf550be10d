"""Pins for the sweep's and the dictionary step's conditionals.

z and s: one-dimensional quadrature of the joint density over s.
Dictionary: the dense Gaussian posterior of a column d_p (precision
P I + gamma_eps sum_i m_ip w_i w_i^T), built with numpy linear algebra; its
single-coordinate conditionals and its moments must match the oracle's
coordinate-wise step.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import bpfa


def joint_factor(s, e, d, gs, ge):
    """N(s; 0, 1/gs) * exp(-ge/2 |e - d s|^2) / exp(-ge/2 |e|^2), e, d on Obs."""
    return np.sqrt(gs / (2 * np.pi)) * np.exp(-0.5 * gs * s * s + ge * s * (d @ e)
                                              - 0.5 * ge * s * s * (d @ d))


@pytest.mark.parametrize("seed", range(4))
def test_log_odds_and_s_moments_by_quadrature(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = rng.integers(1, 12)
    d = rng.standard_normal(n) * rng.uniform(0.05, 0.6)
    e = rng.standard_normal(n) * rng.uniform(0.05, 0.5)
    gs, ge = rng.uniform(0.3, 3.0), rng.uniform(5.0, 80.0)
    ell = rng.uniform(-4, 1)
    delta, rho = float(d @ d), float(d @ e)
    mean, lam = bpfa.s_posterior(gs, ge, delta, rho)
    lim = abs(mean) + 40 / np.sqrt(lam)
    z1, _ = integrate.quad(joint_factor, -lim, lim, args=(e, d, gs, ge), epsabs=0, epsrel=1e-12,
                           limit=200, points=[mean])
    L, _, _ = bpfa.z_log_odds(ell, gs, ge, delta, rho)
    assert abs(L - (ell + np.log(z1))) < 1e-9 * (1 + abs(L))
    m1, _ = integrate.quad(lambda s: s * joint_factor(s, e, d, gs, ge), -lim, lim, epsabs=0,
                           epsrel=1e-12, limit=200, points=[mean])
    m2, _ = integrate.quad(lambda s: s * s * joint_factor(s, e, d, gs, ge), -lim, lim, epsabs=0,
                           epsrel=1e-12, limit=200, points=[mean])
    assert abs(m1 / z1 - mean) < 1e-9 * (1 + abs(mean))
    assert abs((m2 / z1 - (m1 / z1) ** 2) - 1 / lam) < 1e-9 / lam


def small_problem(seed, N=40, P=5, K=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((N, P))
    Mk = rng.random((N, P)) < 0.6
    Z = rng.random((N, K)) < 0.5
    W = np.where(Z, rng.standard_normal((N, K)), 0.0)
    D = rng.standard_normal((K, P)) / np.sqrt(P)
    st = bpfa.State(D=D, W=W, Z=Z, ell=np.zeros(K), gamma_s=1.0, gamma_eps=rng.uniform(2, 9), t=3)
    return bpfa.Params(K=K, seed=seed + 40), X, Mk, st


def dense_precision(P, ge, Mk, W, X, p):
    m = Mk[:, p].astype(float)
    Lam = P * np.eye(W.shape[1]) + ge * (W * m[:, None]).T @ W
    h = ge * (W * m[:, None]).T @ X[:, p]
    return Lam, h


@pytest.mark.parametrize("seed", range(3))
def test_dictionary_step_matches_dense_conditionals(seed):
    prm, X, Mk, st = small_problem(seed)
    K, P = st.D.shape
    R = bpfa.residual(X, Mk, st.D, st.W)
    D_new, R_new = bpfa.dictionary_update(prm, Mk, st, st.W, R)
    for p in range(P):
        Lam, h = dense_precision(P, st.gamma_eps, Mk, st.W, X, p)
        cur = st.D[:, p].copy()
        for k in range(K):
            others = [j for j in range(K) if j != k]
            mean = (h[k] - Lam[k, others] @ cur[others]) / Lam[k, k]
            n = bpfa.dict_normal(prm, np.array([p], np.uint64), k, st.t)[0]
            cur[k] = mean + n / np.sqrt(Lam[k, k])
        assert np.allclose(D_new[:, p], cur, rtol=1e-12, atol=1e-12)
    assert np.allclose(R_new, bpfa.residual(X, Mk, D_new, st.W), rtol=0, atol=1e-12)


def test_dictionary_chain_is_stationary_at_dense_posterior():
    prm, X, Mk, st = small_problem(9, N=25, P=3, K=3)
    K, P = st.D.shape
    samples = []
    R = bpfa.residual(X, Mk, st.D, st.W)
    for it in range(6000):
        D, R = bpfa.dictionary_update(prm, Mk, st, st.W, R)
        st = bpfa.State(D=D, W=st.W, Z=st.Z, ell=st.ell, gamma_s=st.gamma_s,
                        gamma_eps=st.gamma_eps, t=st.t + 1)
        if it >= 200:
            samples.append(D.copy())
    S = np.array(samples)                                   # T x K x P
    for p in range(P):
        Lam, h = dense_precision(P, st.gamma_eps, Mk, st.W, X, p)
        cov = np.linalg.inv(Lam)
        mu = cov @ h
        sd = np.sqrt(np.diag(cov))
        emp_mu = S[:, :, p].mean(0)
        emp_cov = np.cov(S[:, :, p].T)
        # batch means for the standard error of the chain average
        bm = S[: (S.shape[0] // 50) * 50, :, p].reshape(50, -1, K).mean(1)
        se = bm.std(0, ddof=1) / np.sqrt(50)
        assert np.all(np.abs(emp_mu - mu) < 5 * se + 1e-3 * sd), (emp_mu, mu, se)
        assert np.allclose(emp_cov, cov, atol=0.12 * np.outer(sd, sd).max())


def test_empty_patch_draws_from_prior():
    """A patch with no observed pixel has delta = rho = 0: log-odds = ell_k."""
    L, lam, q = bpfa.z_log_odds(-1.7, 2.0, 50.0, 0.0, 0.0)
    assert L == -1.7 and lam == 2.0 and q == 0.0
