"""Pins for the oracle's mini-batch epoch schedule.

Reading (the Time-to-solution section trains "two complete epochs" and gives
no schedule): patch i belongs to batch i mod B; a batch step sweeps only that
batch's patches and draws D, pi, gamma_s and gamma_eps from the conditionals
given the batch with its data statistics scaled by s = N / n_b.  Pinned by:

* one batch (B = 1): the batch step is the full iteration, bit for bit;
* the scaled conditionals equal the unscaled ones on a data set made of r
  copies of the batch (codes and residuals copied with it): the scale enters
  A and b of every d_kp, the counts of every pi_k and both gamma sums, and
  not the priors;
* the partition covers every patch once, batch sizes differ by at most one;
* a batch step leaves the other batches' codes untouched;
* learning: on a fully sampled known-dictionary problem, mini-batch epochs
  learn the noise precision within 10% of 1/sigma^2 and span every true atom.
"""
import numpy as np
import pytest

from oracle import bpfa


def _problem(seed=3, N=150, P=9, K=6):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.random((N, P))
    Mk = rng.random((N, P)) < 0.5
    prm = bpfa.Params(K=K, seed=seed)
    st = bpfa.init_state(prm, N, P)
    st, _ = bpfa.iterate(prm, X, Mk, st)
    return prm, X, Mk, st


def _same(a, b):
    return all(np.array_equal(getattr(a, f), getattr(b, f)) for f in ("D", "W", "Z", "ell")) and \
        (a.gamma_s, a.gamma_eps, a.t) == (b.gamma_s, b.gamma_eps, b.t)


@pytest.mark.parametrize("learn", [True, False])
def test_one_batch_is_the_full_iteration(learn):
    prm, X, Mk, st = _problem()
    full, _ = bpfa.iterate(prm, X, Mk, st, learn_dict=learn)
    mb, _ = bpfa.minibatch_step(prm, X, Mk, st, 1, 0, learn_dict=learn)
    assert _same(full, mb)
    ep = bpfa.epochs(prm, X, Mk, st, 1, 1, learn_dict=learn)
    assert _same(full, ep)


@pytest.mark.parametrize("N,B", [(10, 3), (150, 4), (7, 7), (5, 1)])
def test_partition(N, B):
    rows = [bpfa.batch_rows(N, B, b) for b in range(B)]
    allr = np.sort(np.concatenate(rows))
    assert np.array_equal(allr, np.arange(N))
    sizes = [r.size for r in rows]
    assert max(sizes) - min(sizes) <= 1
    for b, r in enumerate(rows):
        assert np.all(r % B == b)


def test_scaled_conditionals_equal_replicated_batch():
    """Batch statistics scaled by r give the conditionals of r copies of the batch."""
    prm, X, Mk, st = _problem(seed=5, N=40)
    W, Z, R, _ = bpfa.sweep(prm, X, Mk, st)
    rows = bpfa.batch_rows(40, 4, 1)
    r = 7
    sub = bpfa.State(D=st.D, W=st.W[rows], Z=st.Z[rows], ell=st.ell, gamma_s=st.gamma_s,
                     gamma_eps=st.gamma_eps, t=st.t)
    rep = bpfa.State(D=st.D, W=np.tile(st.W[rows], (r, 1)), Z=np.tile(st.Z[rows], (r, 1)),
                     ell=st.ell, gamma_s=st.gamma_s, gamma_eps=st.gamma_eps, t=st.t)
    Wb, Zb, Rb, Mb = W[rows], Z[rows], R[rows], Mk[rows]
    Wr, Zr, Rr, Mr = (np.tile(a, (r, 1)) for a in (Wb, Zb, Rb, Mb))
    Ds, Rs = bpfa.dictionary_update(prm, Mb, sub, Wb, Rb, scale=float(r))
    Dr, Rr2 = bpfa.dictionary_update(prm, Mr, rep, Wr, Rr)
    assert np.allclose(Ds, Dr, rtol=1e-11, atol=1e-13)
    assert np.allclose(np.tile(Rs, (r, 1)), Rr2, rtol=1e-10, atol=1e-12)
    assert np.allclose(bpfa.pi_update(prm, Zb, st.t, scale=float(r)), bpfa.pi_update(prm, Zr, st.t),
                       rtol=1e-11, atol=1e-12)
    assert np.isclose(bpfa.gamma_s_update(prm, Zb, Wb, st.t, scale=float(r)),
                      bpfa.gamma_s_update(prm, Zr, Wr, st.t), rtol=1e-11)
    assert np.isclose(bpfa.gamma_eps_update(prm, Mb, Rs, st.t, scale=float(r)),
                      bpfa.gamma_eps_update(prm, Mr, Rr2, st.t), rtol=1e-11)
    # the scale changes the draws (it is not a no-op), and the prior is not scaled:
    # an unscaled batch gives another dictionary
    D1, _ = bpfa.dictionary_update(prm, Mb, sub, Wb, Rb)
    assert not np.allclose(D1, Ds, rtol=1e-6)


def test_batch_step_touches_only_its_batch():
    prm, X, Mk, st = _problem(seed=7, N=60)
    B = 3
    cur = st
    for b in range(B):
        nxt, _ = bpfa.minibatch_step(prm, X, Mk, cur, B, b)
        rows = bpfa.batch_rows(60, B, b)
        others = np.setdiff1d(np.arange(60), rows)
        assert np.array_equal(nxt.W[others], cur.W[others])
        assert np.array_equal(nxt.Z[others], cur.Z[others])
        # the batch's rows are exactly a sweep of those patches at this step
        sub = bpfa.State(D=cur.D, W=cur.W[rows], Z=cur.Z[rows], ell=cur.ell,
                         gamma_s=cur.gamma_s, gamma_eps=cur.gamma_eps, t=cur.t)
        Ws, Zs, _, _ = bpfa.sweep(prm, X[rows], Mk[rows], sub, patch_ids=rows)
        assert np.array_equal(nxt.W[rows], Ws) and np.array_equal(nxt.Z[rows], Zs)
        assert nxt.t == cur.t + 1
        cur = nxt
    assert np.array_equal(bpfa.epochs(prm, X, Mk, st, 1, B).W, cur.W)


def test_minibatch_epochs_learn_known_dictionary():
    """8 true atoms (P = 16), 5% usage, sigma = 0.01, all pixels observed,
    4 batches of 500 patches, 60 epochs from a prior draw of D."""
    rng = np.random.Generator(np.random.PCG64(21))
    Kt, P, N, sig = 8, 16, 2000, 0.01
    Dt = rng.standard_normal((Kt, P))
    Dt /= np.linalg.norm(Dt, axis=1, keepdims=True)
    Zt = rng.random((N, Kt)) < 0.05
    X = (Zt * rng.standard_normal((N, Kt))) @ Dt + sig * rng.standard_normal((N, P))
    Mk = np.ones((N, P), bool)
    prm = bpfa.Params(K=16, seed=101)
    st = bpfa.init_state(prm, N, P)
    st = bpfa.epochs(prm, X, Mk, st, 60, 4)
    assert st.t == 1 + 60 * 4
    assert abs(st.gamma_eps * sig ** 2 - 1) < 0.10
    used = st.Z.mean(0) > 0.01
    Q, _ = np.linalg.qr(st.D[used].T)
    proj = np.linalg.norm(Dt @ Q, axis=1)
    assert np.all(proj > 0.99), proj
