"""GPU parity of the mini-batch epoch schedule (bpfa_minibatch) against the
oracle's minibatch_step, in follow mode, on the same Philox streams.

Reading (Time-to-solution section, "complete epochs"): patch i in batch
i mod B; a step sweeps its batch and draws D, pi, gamma_s and gamma_eps from
the batch's statistics scaled by N / n_b; one iteration number per step.
Cases: several batch counts with ragged batches (N not a multiple of B),
sparse-coding-only steps, a 3-D frame, a large dictionary (several sweep
tiles and statistics row groups: the binary64 chain streamed from HBM), a
cursor that runs across calls and resets when B changes, B = 1 equal to
bpfa_iterate bit for bit, and a full 512 x 512 frame (one epoch of 4 batches)
checked on sampled patches and positions.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import bpfa as ob  # noqa: E402
from parity_util import FP32_TOL, assert_close, case, oracle_problem  # noqa: E402

from paper_2311_15061_amd import bpfa  # noqa: E402
from test_gpu_parity import compare_state, gpu_problem  # noqa: E402
import synth  # noqa: E402


def run_minibatch_follow(y, m, patch, stride, K, seed, B, steps, flags=bpfa.LEARN_DICT,
                         per_call=1):
    prob = gpu_problem(y, m, patch, stride, K, seed)
    prm, X, Mk = oracle_problem(y, m, patch, stride, K, seed)
    st = ob.init_state(prm, X.shape[0], X.shape[1])
    learn = bool(flags & bpfa.LEARN_DICT)
    done = 0
    ties = 0
    while done < steps:
        n = min(per_call, steps - done)
        prob.minibatch(B, n, flags)
        gs = prob.get_state()
        for j in range(n):
            # follow the GPU's z only for the last step of the call (its state is what we see)
            fz = gs["Z"] if j == n - 1 else None
            st, rep = ob.minibatch_step(prm, X, Mk, st, B, (done + j) % B, learn_dict=learn,
                                        follow_z=fz)
            if fz is not None:
                assert rep.hard_mismatches == 0, "step %d: %d hard z mismatches, e.g. %s" % (
                    done + j, rep.hard_mismatches, rep.hard_sites[:5])
                ties += rep.near_ties
        compare_state(gs, st, FP32_TOL, "after step %d" % (done + n - 1))
        done += n
    return prob, st, ties


@pytest.mark.parametrize("B,steps", [(2, 4), (3, 7), (5, 5)])
def test_minibatch_parity_lattice64(B, steps):
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    prob, st, ties = run_minibatch_follow(y, m, wl.patch, wl.stride, wl.K, wl.method_seed, B, steps)
    xh = prob.reconstruct()
    ref = ob.reconstruct(st, wl.shape, wl.patch, wl.stride)
    e = assert_close(xh, ref, FP32_TOL, "reconstruction")
    print("B=%d steps=%d near-ties %d recon err %.2e" % (B, steps, ties, e), flush=True)
    prob.close()


def test_minibatch_sparse_code_only():
    y, m, g = case((40, 37), (6, 6), (1, 1), 20, 0.25, seed=9)
    prob, st, ties = run_minibatch_follow(y, m, (6, 6), (1, 1), 20, 0x5151, 3, 5,
                                          flags=bpfa.SPARSE_CODE_ONLY)
    prob.close()


def test_minibatch_3d():
    y, m, g = case((14, 13, 8), (4, 4, 2), (1, 1, 2), 12, 0.3, seed=4)
    prob, st, ties = run_minibatch_follow(y, m, (4, 4, 2), (1, 1, 2), 12, 0x5152, 4, 6)
    prob.close()


def test_minibatch_large_dictionary():
    """K = 300: two sweep tiles, several statistics row groups, the chain from HBM."""
    y, m, g = case((30, 30), (5, 5), (1, 1), 300, 0.4, seed=6)
    prob, st, ties = run_minibatch_follow(y, m, (5, 5), (1, 1), 300, 0x5153, 3, 3)
    prob.close()


def test_one_batch_is_iterate_bit_for_bit():
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    a = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    b = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    a.iterate(3)
    b.minibatch(1, 3)
    sa, sb = a.get_state(), b.get_state()
    for k in ("D", "W", "Z", "logit_pi"):
        assert np.array_equal(sa[k], sb[k]), k
    assert (sa["gamma_s"], sa["gamma_eps"], sa["t"]) == (sb["gamma_s"], sb["gamma_eps"], sb["t"])
    assert np.array_equal(a.reconstruct(), b.reconstruct())
    a.close()
    b.close()


def test_cursor_across_calls_and_partition_change():
    """Steps split over calls equal one call; a full iteration in between
    works on the batch-ordered slots; a new B restarts at batch 0."""
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    a = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    b = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    a.minibatch(3, 4)
    for _ in range(4):
        b.minibatch(3, 1)
    a.iterate(1)
    b.iterate(1)
    a.minibatch(2, 2)
    b.minibatch(2, 1)
    b.minibatch(2, 1)
    sa, sb = a.get_state(), b.get_state()
    for k in ("D", "W", "Z", "logit_pi"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["t"] == sb["t"] == 1 + 4 + 1 + 2
    # the same sequence in the oracle (one step per batch, iterate between)
    prm, X, Mk = oracle_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    st = ob.init_state(prm, X.shape[0], X.shape[1])
    for j in range(4):
        st, _ = ob.minibatch_step(prm, X, Mk, st, 3, j % 3)
    st, _ = ob.iterate(prm, X, Mk, st)
    for j in range(2):
        st, _ = ob.minibatch_step(prm, X, Mk, st, 2, j, follow_z=sa["Z"] if j == 1 else None)
    compare_state(sa, st, FP32_TOL, "after the mixed sequence")
    with pytest.raises(bpfa.BpfaError):
        a.minibatch(0, 1)
    with pytest.raises(bpfa.BpfaError):
        a.minibatch(257, 1)
    a.close()
    b.close()


def test_minibatch_full_frame_512_sampled():
    """The 512 x 512 workload, one epoch of 4 batches: after steps 1-3 (from the
    GPU's state), step 4 (batch 3) is checked on 1000 sampled patches of the
    batch and 6 sampled positions of the dictionary, and the pi / gamma draws
    from the batch's whole counts and sums."""
    wl = synth.workload("stem512")
    y, m, g = synth.make_frame(wl)
    B = 4
    prob = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    prm, X, Mk = oracle_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    prob.minibatch(B, 3)
    s0 = prob.get_state()
    prob.minibatch(B, 1)
    s1 = prob.get_state()
    N = X.shape[0]
    rows = ob.batch_rows(N, B, 3)
    scale = N / rows.size
    rng = np.random.Generator(np.random.PCG64(77))
    S = np.sort(rng.choice(rows, size=1000, replace=False))
    st0 = ob.State(D=s0["D"].astype(np.float64), W=s0["W"].astype(np.float64), Z=s0["Z"].astype(bool),
                   ell=s0["logit_pi"], gamma_s=s0["gamma_s"], gamma_eps=s0["gamma_eps"], t=s0["t"])
    sub = ob.State(D=st0.D, W=st0.W[S], Z=st0.Z[S], ell=st0.ell, gamma_s=st0.gamma_s,
                   gamma_eps=st0.gamma_eps, t=st0.t)
    Ws, Zs, _, rep = ob.sweep(prm, X[S], Mk[S], sub, follow_z=s1["Z"][S], patch_ids=S)
    assert rep.hard_mismatches == 0
    assert_close(s1["W"][S], Ws, FP32_TOL, "sampled batch patches W")
    # patches outside the batch are untouched
    other = np.setdiff1d(np.arange(N), rows)[:5000]
    assert np.array_equal(s1["W"][other], s0["W"][other])
    # dictionary positions given the GPU's new codes of the batch
    Wb = s1["W"][rows].astype(np.float64)
    cols = np.sort(rng.choice(X.shape[1], size=6, replace=False))
    Rb = ob.residual(X[rows][:, cols], Mk[rows][:, cols], st0.D[:, cols], Wb)
    subd = ob.State(D=st0.D[:, cols], W=Wb, Z=s1["Z"][rows].astype(bool), ell=st0.ell,
                    gamma_s=st0.gamma_s, gamma_eps=st0.gamma_eps, t=st0.t)
    Dd, _ = ob.dictionary_update(prm, Mk[rows][:, cols], subd, Wb, Rb, positions=cols,
                                 prior_P=X.shape[1], scale=scale)
    assert_close(s1["D"][:, cols], Dd, FP32_TOL, "sampled dictionary positions")
    # pi and gamma_s from the batch's counts and sums
    ell = ob.pi_update(prm, s1["Z"][rows].astype(bool), st0.t, scale=scale)
    assert np.all(np.abs(s1["logit_pi"] - ell) <= FP32_TOL * (1 + np.abs(ell)))
    gs = ob.gamma_s_update(prm, s1["Z"][rows].astype(bool), Wb, st0.t, scale=scale)
    assert abs(s1["gamma_s"] / gs - 1) < FP32_TOL
    assert s1["t"] == s0["t"] + 1
    prob.close()
