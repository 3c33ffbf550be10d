"""Learning behaviour, follow-mode bookkeeping and the reconstruction identity."""
import numpy as np
import pytest

from oracle import bpfa, patches


def _known_dictionary_data():
    rng = np.random.Generator(np.random.PCG64(21))
    Kt, P, N, sig = 8, 16, 2000, 0.01
    Dt = rng.standard_normal((Kt, P))
    Dt /= np.linalg.norm(Dt, axis=1, keepdims=True)
    Zt = rng.random((N, Kt)) < 0.05
    X = (Zt * rng.standard_normal((N, Kt))) @ Dt + sig * rng.standard_normal((N, P))
    return Dt, X, np.ones((N, P), bool), sig


def _matched_cos(Dt, D):
    from scipy.optimize import linear_sum_assignment
    Dn = D / np.linalg.norm(D, axis=1, keepdims=True)
    C = np.abs(Dt @ Dn.T)
    r, c = linear_sum_assignment(-C)
    return C[r, c]


def test_fully_sampled_known_dictionary_recovery():
    """8 true atoms (P = 16), 5% usage, noise sigma = 0.01, all pixels observed.

    From a prior draw of D, after 200 iterations the sampler must learn the
    noise precision within 10% of 1/sigma^2 and span every true atom with
    its used atoms (cos of the projection > 0.99).  (One-to-one atom identity
    is slow to reach from a random start: the chain keeps atoms blended for a
    long time, so identity is pinned by the next test instead.)
    """
    Dt, X, Mk, sig = _known_dictionary_data()
    prm = bpfa.Params(K=16, seed=101)
    st = bpfa.init_state(prm, X.shape[0], X.shape[1])
    for _ in range(200):
        st, _ = bpfa.iterate(prm, X, Mk, st)
    assert abs(st.gamma_eps * sig ** 2 - 1) < 0.10
    used = st.Z.mean(0) > 0.01
    Q, _ = np.linalg.qr(st.D[used].T)
    proj = np.linalg.norm(Dt @ Q, axis=1)
    assert np.all(proj > 0.99), proj


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_one_to_one_recovery_from_a_prior_draw(seed):
    """8 true atoms (P = 16), usage pi = 0.2, noise sigma = 0.1, all pixels
    observed, K = 16 from a prior draw of D: after 200 iterations at least
    7 of the 8 true atoms are matched one to one (Hungarian matching) with
    |cos| > 0.95 and gamma_eps is within 10% of 1/sigma^2.  (At sigma = 0.01
    the same chain mixes slowly -- atoms stay blended for hundreds of
    iterations -- so that noise level pins the span above, not identity.)"""
    from scipy.optimize import linear_sum_assignment
    rng = np.random.Generator(np.random.PCG64(21 + seed))
    Kt, P, N, sig = 8, 16, 2000, 0.1
    Dt = rng.standard_normal((Kt, P))
    Dt /= np.linalg.norm(Dt, axis=1, keepdims=True)
    Zt = rng.random((N, Kt)) < 0.2
    X = (Zt * rng.standard_normal((N, Kt))) @ Dt + sig * rng.standard_normal((N, P))
    prm = bpfa.Params(K=16, seed=101 + seed)
    st = bpfa.init_state(prm, N, P)
    for _ in range(200):
        st, _ = bpfa.iterate(prm, X, np.ones((N, P), bool), st)
    cos = _matched_cos(Dt, st.D)
    assert (cos > 0.95).sum() >= 7, cos
    assert abs(st.gamma_eps * sig ** 2 - 1) < 0.10


def test_true_dictionary_is_kept():
    """Started at the true atoms (plus 8 prior atoms), 100 iterations keep at
    least 7 of 8 true atoms matched one to one with |cos| > 0.95."""
    Dt, X, Mk, sig = _known_dictionary_data()
    prm = bpfa.Params(K=16, seed=101)
    st = bpfa.init_state(prm, X.shape[0], X.shape[1])
    st.D[:8] = Dt
    for _ in range(100):
        st, _ = bpfa.iterate(prm, X, Mk, st)
    cos = _matched_cos(Dt, st.D)
    assert (cos > 0.95).sum() >= 7, cos
    assert abs(st.gamma_eps * sig ** 2 - 1) < 0.10


def _problem(seed=3, N=200, P=9, K=6):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.random((N, P))
    Mk = rng.random((N, P)) < 0.5
    prm = bpfa.Params(K=K, seed=seed)
    st = bpfa.init_state(prm, N, P)
    st, _ = bpfa.iterate(prm, X, Mk, st)
    return prm, X, Mk, st


def test_follow_mode_without_mismatch_is_identity():
    prm, X, Mk, st = _problem()
    W, Z, R, rep = bpfa.sweep(prm, X, Mk, st)
    W2, Z2, R2, rep2 = bpfa.sweep(prm, X, Mk, st, follow_z=Z)
    assert rep2.near_ties == 0 and rep2.hard_mismatches == 0
    assert np.array_equal(W, W2) and np.array_equal(Z, Z2)


def test_follow_mode_flags_far_mismatch_as_hard():
    prm, X, Mk, st = _problem()
    W, Z, R, rep = bpfa.sweep(prm, X, Mk, st)
    fz = Z.copy()
    fz[5, 0] = ~fz[5, 0]
    _, Z2, _, rep2 = bpfa.sweep(prm, X, Mk, st, follow_z=fz)
    assert rep2.hard_mismatches >= 1 and (5, 0) in rep2.hard_sites
    assert Z2[5, 0] == Z[5, 0]          # the oracle keeps its own draw at a hard mismatch


def test_follow_mode_adopts_certified_tie():
    prm, X, Mk, st = _problem()
    # find the draw closest to its threshold at atom 0 and widen the band to it
    N, K = st.W.shape
    R = bpfa.residual(X, Mk, st.D, st.W)
    d0 = st.D[0]
    delta = Mk.astype(float) @ (d0 * d0)
    rho = R @ d0 + delta * st.W[:, 0]
    L, lam, q = bpfa.z_log_odds(st.ell[0], st.gamma_s, st.gamma_eps, delta, rho)
    u, _ = bpfa.zs_uniforms(prm, np.arange(N, dtype=np.uint64), 0, st.t)
    gap = np.abs(bpfa.logit_uniform(u) - L)
    i = int(np.argmin(gap))
    scale = 1 + abs(st.ell[0]) + abs(0.5 * np.log(st.gamma_s / lam[i])) + q[i]
    W, Z, _, _ = bpfa.sweep(prm, X, Mk, st)
    fz = Z.copy()
    fz[i, 0] = ~fz[i, 0]
    _, Z2, _, rep = bpfa.sweep(prm, X, Mk, st, follow_z=fz, tie_tol=1.0001 * gap[i] / scale)
    assert (i, 0) in rep.tie_sites
    assert Z2[i, 0] == fz[i, 0]


def test_sparse_code_only_keeps_dictionary():
    prm, X, Mk, st = _problem()
    st2, _ = bpfa.iterate(prm, X, Mk, st, learn_dict=False)
    assert np.array_equal(st2.D, st.D) and st2.t == st.t + 1


def test_reconstruct_identity_dictionary():
    """With D = I (K = P) and w_i the exact patches, the overlap average is the image."""
    rng = np.random.Generator(np.random.PCG64(8))
    shape, patch, stride = (12, 10), (3, 4), (1, 2)
    img = rng.integers(0, 64, size=shape) / 64.0
    X, _ = patches.extract(img, np.ones(shape, np.uint8), patch, stride)
    P = X.shape[1]
    st = bpfa.State(D=np.eye(P), W=X.copy(), Z=X != 0, ell=np.zeros(P), gamma_s=1.0,
                    gamma_eps=1.0, t=1)
    out = bpfa.reconstruct(st, shape, patch, stride)
    assert np.array_equal(out, img)


def test_init_state_prior_scale():
    prm = bpfa.Params(K=64, seed=5)
    st = bpfa.init_state(prm, 10, 100)
    assert abs((st.D ** 2).mean() * 100 - 1) < 0.05
    assert np.allclose(st.ell, np.log(1 / 63))
