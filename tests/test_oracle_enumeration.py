"""The z/s sweep's stationary law equals the exact posterior over all 2^K z.

For one patch with D, pi, gamma_s, gamma_eps held fixed, the exact marginal
posterior of z is (s integrated out; only observed pixels enter)

    p(z | x) ∝ prod_k pi_k^z_k (1 - pi_k)^(1 - z_k) * N(x_O; 0, I/gamma_eps + D_OA D_OA^T / gamma_s)

with A the active atoms.  Many independent copies of the patch (different
Philox counters) run the oracle's sweep repeatedly; after burn-in their z
configurations must follow that law (chi-square).  A dropped term, a wrong
sign, an index slip or an s draw from the wrong conditional shifts the law.
"""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle import bpfa


def exact_z_posterior(D, x, m, pi, gs, ge):
    K = D.shape[0]
    obs = np.nonzero(m)[0]
    xo = x[obs]
    configs = list(itertools.product([0, 1], repeat=K))
    logp = []
    for z in configs:
        z = np.array(z, bool)
        Do = D[z][:, obs]                                    # |A| x |O|
        cov = np.eye(obs.size) / ge + Do.T @ Do / gs
        lp = stats.multivariate_normal(mean=np.zeros(obs.size), cov=cov).logpdf(xo)
        lp += np.sum(np.where(z, np.log(pi), np.log1p(-pi)))
        logp.append(lp)
    logp = np.array(logp)
    p = np.exp(logp - logp.max())
    return configs, p / p.sum()


def run_chains(D, x, m, pi, gs, ge, copies, sweeps, seed):
    K, P = D.shape
    prm = bpfa.Params(K=K, seed=seed)
    X = np.tile(x, (copies, 1))
    Mk = np.tile(m, (copies, 1))
    st = bpfa.State(D=D.copy(), W=np.zeros((copies, K)), Z=np.zeros((copies, K), bool),
                    ell=np.log(pi) - np.log1p(-pi), gamma_s=gs, gamma_eps=ge, t=1)
    samples = []
    for s in range(sweeps):
        W, Z, _, _ = bpfa.sweep(prm, X, Mk, st)
        st = bpfa.State(D=st.D, W=W, Z=Z, ell=st.ell, gamma_s=gs, gamma_eps=ge, t=st.t + 1)
        if s >= sweeps // 2:
            samples.append(Z.copy())
    return samples


@pytest.mark.parametrize("K,seed", [(2, 11), (3, 12), (4, 13)])
def test_sweep_matches_enumerated_posterior(K, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    P = 6
    D = rng.standard_normal((K, P)) / np.sqrt(P) * 2.0
    m = np.array([1, 1, 0, 1, 1, 0], bool)
    ztrue = np.zeros(K, bool)
    ztrue[0] = True
    x = ztrue.astype(float) @ D * 1.3 + 0.2 * rng.standard_normal(P)
    pi = rng.uniform(0.2, 0.6, size=K)
    gs, ge = 1.5, 12.0
    configs, p = exact_z_posterior(D, x, m, pi, gs, ge)
    # copies are independent chains; the last half of each chain is kept
    samples = run_chains(D, x, m, pi, gs, ge, copies=4000, sweeps=16, seed=seed)
    Z = np.concatenate(samples)
    code = (Z.astype(np.int64) * (1 << np.arange(K - 1, -1, -1))).sum(1)
    counts = np.bincount(code, minlength=2 ** K)
    # samples within a chain are correlated: test one sweep per chain for the
    # chi-square (independent), and the pooled frequencies loosely
    last = samples[-1]
    code1 = (last.astype(np.int64) * (1 << np.arange(K - 1, -1, -1))).sum(1)
    c1 = np.bincount(code1, minlength=2 ** K)
    expect = p * c1.sum()
    keep = expect > 5
    chi2 = (((c1 - expect) ** 2 / expect)[keep]).sum()
    pval = stats.chi2.sf(chi2, keep.sum() - 1)
    assert pval > 1e-3, (pval, c1, expect)
    assert np.max(np.abs(counts / counts.sum() - p)) < 0.02


def test_k1_log_odds_is_exact_posterior():
    """K = 1: sigmoid of the sweep's log-odds equals the closed-form posterior."""
    rng = np.random.Generator(np.random.PCG64(5))
    P = 7
    d = rng.standard_normal(P) * 0.5
    m = np.array([1, 0, 1, 1, 0, 1, 1], bool)
    x = 0.8 * d + 0.1 * rng.standard_normal(P)
    pi, gs, ge = 0.3, 2.0, 25.0
    _, p = exact_z_posterior(d[None, :], x, m, np.array([pi]), gs, ge)
    delta = float((d[m] ** 2).sum())
    rho = float((d[m] * x[m]).sum())
    L, _, _ = bpfa.z_log_odds(np.log(pi / (1 - pi)), gs, ge, delta, rho)
    assert abs(1.0 / (1.0 + np.exp(-L)) - p[1]) < 1e-12
