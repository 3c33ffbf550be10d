"""Geweke's "getting it right" joint-distribution test of the whole sampler.

J. Geweke, "Getting it right: joint distribution tests of posterior
simulators", JASA 99(467), 2004.  A successive-conditional chain alternates
x ~ p(x | theta) and one Gibbs iteration theta ~ K(theta | x); if every
conditional is right, theta's marginal stays the prior.  Means of test
functions along the chain are compared with their prior values, with
batch-means standard errors.  Tiny problem (N = 6, P = 4, K = 3), proper
priors, a partial mask.
"""
import math

import numpy as np
import pytest

from oracle import bpfa


def prior_draw(prm, N, P, rng):
    K = prm.K
    pi = rng.beta(prm.a / K, prm.b * (K - 1) / K, size=K)
    gs = rng.gamma(prm.c, 1 / prm.d)
    ge = rng.gamma(prm.e, 1 / prm.f)
    D = rng.normal(0, 1 / math.sqrt(P), size=(K, P))
    Z = rng.random((N, K)) < pi
    W = np.where(Z, rng.normal(0, 1 / math.sqrt(gs), size=(N, K)), 0.0)
    return bpfa.State(D=D, W=W, Z=Z, ell=np.log(pi) - np.log1p(-pi), gamma_s=gs, gamma_eps=ge, t=1)


def stat_functions(st):
    pi = 1 / (1 + np.exp(-st.ell))
    return np.array([st.gamma_s, st.gamma_eps, pi.mean(), (st.D ** 2).mean(),
                     st.Z.mean(), (st.W ** 2).mean(), st.D[0, 0], st.W[0, 0]])


@pytest.mark.slow
def test_geweke_successive_conditional():
    N, P, K = 6, 4, 3
    prm = bpfa.Params(K=K, a=3.0, b=3.0, c=3.0, d=2.0, e=4.0, f=0.1, seed=2024)
    rng = np.random.Generator(np.random.PCG64(77))
    Mk = rng.random((N, P)) < 0.75
    # prior values of the test functions
    E_pi = (prm.a / K) / (prm.a / K + prm.b * (K - 1) / K)
    E_inv_gs = prm.d / (prm.c - 1)
    prior = np.array([prm.c / prm.d, prm.e / prm.f, E_pi, 1 / P, E_pi, E_pi * E_inv_gs, 0.0, 0.0])
    st = prior_draw(prm, N, P, rng)
    n_iter, burn = 12000, 500
    rec = []
    for it in range(n_iter):
        X = st.W @ st.D + rng.normal(0, 1 / math.sqrt(st.gamma_eps), size=(N, P))
        st, _ = bpfa.iterate(prm, X, Mk, st)
        if it >= burn:
            rec.append(stat_functions(st))
    G = np.array(rec)
    nb = 40
    Gb = G[: (len(G) // nb) * nb].reshape(nb, -1, G.shape[1]).mean(1)
    se = Gb.std(0, ddof=1) / math.sqrt(nb)
    z = (G.mean(0) - prior) / se
    assert np.all(np.abs(z) < 4.0), (z, G.mean(0), prior)
