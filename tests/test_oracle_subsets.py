"""The oracle's sweep on a subset of patches and its dictionary update on a
subset of positions reproduce the rows / columns of the full steps exactly.

Patches are conditionally independent given (D, pi, gamma) in the sweep and
positions are independent given W in the dictionary update (BPFA section), and
every draw comes from counters keyed by the patch or position index; so the
full-size GPU tests may check sampled patches and positions against these
subset calls.
"""
import numpy as np

from oracle import bpfa as ob
from parity_util import case, oracle_problem


def _state_after_one(prm, X, Mk):
    st = ob.init_state(prm, X.shape[0], X.shape[1])
    st, _ = ob.iterate(prm, X, Mk, st)
    return st


def test_sweep_on_patch_subset_equals_rows_of_full_sweep():
    y, m, _ = case((24, 22), (5, 4), (1, 1), 12, 0.3, seed=3)
    prm, X, Mk = oracle_problem(y, m, (5, 4), (1, 1), 12, seed=0x77)
    st = _state_after_one(prm, X, Mk)
    W, Z, R, _ = ob.sweep(prm, X, Mk, st)
    rng = np.random.Generator(np.random.PCG64(1))
    S = np.sort(rng.choice(X.shape[0], size=37, replace=False))
    sub = ob.State(D=st.D, W=st.W[S], Z=st.Z[S], ell=st.ell, gamma_s=st.gamma_s,
                   gamma_eps=st.gamma_eps, t=st.t)
    Ws, Zs, Rs, _ = ob.sweep(prm, X[S], Mk[S], sub, patch_ids=S)
    assert np.array_equal(Ws, W[S]) and np.array_equal(Zs, Z[S]) and np.array_equal(Rs, R[S])
    # the patch index matters: the same rows under other ids draw other numbers
    Wo, _, _, _ = ob.sweep(prm, X[S], Mk[S], sub, patch_ids=S + 1)
    assert not np.array_equal(Wo, W[S])


def test_dictionary_update_on_position_subset_equals_columns():
    y, m, _ = case((24, 22), (5, 4), (1, 1), 12, 0.3, seed=4)
    prm, X, Mk = oracle_problem(y, m, (5, 4), (1, 1), 12, seed=0x78)
    st = _state_after_one(prm, X, Mk)
    W, Z, R, _ = ob.sweep(prm, X, Mk, st)
    D, _ = ob.dictionary_update(prm, Mk, st, W, R)
    P = X.shape[1]
    cols = np.array([0, 3, 7, 19])
    sub = ob.State(D=st.D[:, cols], W=st.W, Z=st.Z, ell=st.ell, gamma_s=st.gamma_s,
                   gamma_eps=st.gamma_eps, t=st.t)
    Ds, _ = ob.dictionary_update(prm, Mk[:, cols], sub, W, R[:, cols], positions=cols, prior_P=P)
    assert np.array_equal(Ds, D[:, cols])
    # the prior precision is the full patch dimension, not the subset's
    Dw, _ = ob.dictionary_update(prm, Mk[:, cols], sub, W, R[:, cols], positions=cols)
    assert not np.allclose(Dw, D[:, cols])
