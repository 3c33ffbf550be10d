"""GPU parity: the HIP library against the binary64 oracle on the same Philox streams.

Bars: integer work (patch index, Philox words, z decisions away from
near-ties) bit-exact; floating point within the binary32 tolerance 1e-5
(normwise relative, and elementwise against |b| + rms(b)).  z decisions are
compared in follow mode: the oracle adopts the GPU's z only where its own
log-odds sit within 1e-4 (scaled) of the draw's logit; every other mismatch
fails the test.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import bpfa as ob  # noqa: E402
from oracle import patches, philox  # noqa: E402
from parity_util import (FP32_TOL, assert_close, case, oracle_problem, record, rel_err,  # noqa: E402
                         state_errors)

from paper_2311_15061_amd import bpfa  # noqa: E402
import synth  # noqa: E402


def gpu_problem(y, m, patch, stride, K, seed, problem_id=0, **hyper):
    print("case: shape=%s patch=%s stride=%s K=%d seed=%#x" % (np.shape(y), patch, stride, K, seed),
          flush=True)
    return bpfa.Problem(np.asarray(y, np.float32), m, patch, stride, K=K, seed=seed,
                        problem_id=problem_id, **hyper)


def compare_state(gs, st, tol=FP32_TOL, what=""):
    assert np.array_equal(gs["Z"].astype(bool), st.Z), what + ": Z differs after follow mode"
    eD = assert_close(gs["D"], st.D, tol, what + " D")
    eW = assert_close(gs["W"], st.W, tol, what + " W")
    assert abs(gs["gamma_s"] / st.gamma_s - 1) < tol, (what, gs["gamma_s"], st.gamma_s)
    assert abs(gs["gamma_eps"] / st.gamma_eps - 1) < tol, (what, gs["gamma_eps"], st.gamma_eps)
    ell_scale = 1.0 + np.abs(st.ell)
    assert np.all(np.abs(gs["logit_pi"] - st.ell) <= tol * ell_scale), what + " logit pi"
    assert gs["t"] == st.t
    return eD, eW


# ---------------------------------------------------------------- integer work

@pytest.mark.parametrize("tag,c1,t", [(philox.TAG_ZS, 0, 1), (philox.TAG_DICT, 77, 5),
                                      (philox.TAG_GE, 3, 123456)])
def test_philox_blocks_bit_exact(tag, c1, t):
    c0 = np.concatenate([np.arange(1000), [0xFFFFFFFF, 0x80000000, 123456789]]).astype(np.uint32)
    seed, pid = 0xB1FA0002DEADBEEF, 0x123
    dev = bpfa.debug_philox(seed, pid, tag, c0, c1, t)
    ref = philox.block(seed, pid, tag, c0.astype(np.uint64), c1, t)
    for w in range(4):
        assert np.array_equal(dev[:, w], ref[w])


@pytest.mark.parametrize("shape,patch,stride", [
    ((64, 64), (8, 8), (1, 1)),
    ((37, 29), (5, 7), (2, 2)),
    ((12, 10, 9), (4, 3, 3), (1, 1, 2)),
    ((61,), (5,), (1,)),
    ((6, 7, 5, 4), (2, 3, 2, 2), (1, 2, 1, 2)),
])
def test_patch_index_bit_exact(shape, patch, stride):
    rng = np.random.Generator(np.random.PCG64(3))
    y = rng.random(shape).astype(np.float32)
    m = (rng.random(shape) < 0.3).astype(np.uint8)
    prob = gpu_problem(y, m, patch, stride, K=4, seed=1)
    bits, cnt = prob.patch_index()
    _, Mk = patches.extract(y, m, patch, stride)
    P = Mk.shape[1]
    ref_bits = np.zeros((Mk.shape[0], (P + 31) // 32), np.uint32)
    for p in range(P):
        ref_bits[:, p // 32] |= (Mk[:, p].astype(np.uint32) << np.uint32(p % 32))
    assert np.array_equal(cnt, Mk.sum(1))
    assert np.array_equal(bits, ref_bits)
    assert prob.stats()["n_obs"] == int(Mk.sum())
    prob.close()


def test_initial_state_matches_oracle():
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    prob = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    gs = prob.get_state()
    prm, X, Mk = oracle_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    st = ob.init_state(prm, X.shape[0], X.shape[1])
    # binary64 draw rounded once to binary32
    assert np.max(np.abs(gs["D"] - st.D.astype(np.float32))) <= np.spacing(np.float32(1.0))
    assert np.allclose(gs["logit_pi"], st.ell, rtol=1e-15)
    assert gs["t"] == 1 and not gs["Z"].any() and not gs["W"].any()
    prob.close()


# ---------------------------------------------------------- floating point work

def run_follow(y, m, patch, stride, K, seed, iters, flags=bpfa.LEARN_DICT, state=None,
               problem_id=0, tol=FP32_TOL, **hyper):
    prob = gpu_problem(y, m, patch, stride, K, seed, problem_id=problem_id, **hyper)
    prm, X, Mk = oracle_problem(y, m, patch, stride, K, seed, problem_id=problem_id, **hyper)
    st = ob.init_state(prm, X.shape[0], X.shape[1]) if state is None else state
    if state is not None:
        prob.set_state(D=st.D, W=st.W, Z=st.Z, logit_pi=st.ell, gamma_s=st.gamma_s,
                       gamma_eps=st.gamma_eps, t=st.t)
    ties = 0
    errs = []
    worst = {}
    for it in range(iters):
        prob.iterate(1, flags)
        gs = prob.get_state()
        st, rep = ob.iterate(prm, X, Mk, st, learn_dict=bool(flags & bpfa.LEARN_DICT),
                             follow_z=gs["Z"])
        assert rep.hard_mismatches == 0, "iteration %d: %d z mismatches away from ties, e.g. %s" % (
            it, rep.hard_mismatches, rep.hard_sites[:5])
        ties += rep.near_ties
        errs.append(compare_state(gs, st, tol, "iteration %d" % it))
        for k, v in state_errors(gs, st).items():
            worst[k] = max(worst.get(k, 0.0), v)
    run_follow.worst = worst
    return prob, st, ties, errs


def test_one_iteration_parity_lattice64():
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    prob, st, ties, errs = run_follow(y, m, wl.patch, wl.stride, wl.K, wl.method_seed, 1)
    print("near-ties", ties, "errors D/W", errs)
    prob.close()


def test_trajectory_parity_lattice64_full_run():
    """The 64x64 workload, all 10 iterations, oracle coupled in follow mode."""
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    prob, st, ties, errs = run_follow(y, m, wl.patch, wl.stride, wl.K, wl.method_seed, wl.iters)
    xh = prob.reconstruct()
    ref = ob.reconstruct(st, wl.shape, wl.patch, wl.stride)
    e = assert_close(xh, ref, FP32_TOL, "reconstruction")
    print("near-ties %d; final errors D %.2e W %.2e recon %.2e" % (ties, errs[-1][0], errs[-1][1], e))
    record("lattice64 whole run, 10 iterations in follow mode, fp32", recon=e, **run_follow.worst)
    prob.close()


def test_sparse_code_only_parity():
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    prob, st, ties, errs = run_follow(y, m, wl.patch, wl.stride, wl.K, wl.method_seed, 3,
                                      flags=bpfa.SPARSE_CODE_ONLY)
    prob.close()


@pytest.mark.parametrize("shape,patch,stride,K,rho", [
    ((40, 36), (6, 5), (1, 1), 21, 0.2),          # ragged grid, odd K
    ((30, 30), (10, 10), (1, 1), 200, 0.15),      # several LDS tiles, two statistics row groups
    ((28, 28), (10, 10), (1, 1), 160, 0.2),       # the smallest K with two statistics row groups
    ((26, 26), (8, 8), (1, 1), 257, 0.2),         # one diagonal / B copy (K > 256), three row groups
    ((20, 18, 8), (4, 4, 2), (1, 1, 2), 24, 0.25),  # 3-D video patches with a time stride
    ((10, 9, 6, 5), (3, 3, 2, 2), (1, 1, 2, 1), 12, 0.3),  # 4-D patches spanning two frames
    ((24, 22, 3), (6, 6, 3), (1, 1, 1), 16, 0.3),  # full-depth patches (B_2 = M_2, e.g. RGB)
    ((20, 20, 3), (5, 5, 1), (1, 1, 1), 16, 0.3),  # one single-channel dictionary across layers
    ((26, 26), (12, 12), (1, 1), 16, 0.35),       # |Obs| ~ 50: 2 (20 and 24 rows) and 4 lanes per patch
    ((30, 30), (12, 12), (1, 1), 18, 0.28),       # |Obs| ~ 40: 2 lanes per patch, 16-, 20- and 24-row bodies
    ((22, 22), (12, 12), (1, 1), 12, 0.65),       # |Obs| ~ 94: 8 lanes per patch
    ((28, 28), (12, 12), (1, 1), 20, 0.2),        # |Obs| spread over 1, 2 and 4 lanes per patch
    ((20, 20), (12, 12), (1, 1), 8, 0.95),        # |Obs| ~ 137: 16 lanes per patch
    ((96, 96), (6, 6), (1, 1), 16, 0.95),         # 8 statistics chunks, one XCD per chunk
    ((400, 400), (4, 4), (1, 1), 8, 0.9),         # statistics blocks loop over several chunks
])
def test_parity_geometry_cases(shape, patch, stride, K, rho):
    y, m, g = case(shape, patch, stride, K, rho, seed=K)
    prob, st, ties, errs = run_follow(y, m, patch, stride, K, 0xABC0 + K, 3, problem_id=5)
    xh = prob.reconstruct()
    ref = ob.reconstruct(st, shape, patch, stride)
    assert_close(xh, ref, FP32_TOL, "reconstruction")
    prob.close()


def test_new_frame_keeps_codes():
    """set_frame without resetting codes: every patch keeps its (z, s) across a new mask."""
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    y2, m2, _ = synth.make_frame(wl, data_seed=99, rho=0.3)
    prob = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    prob.iterate(2)
    before = prob.get_state()
    prob.set_frame(y2.astype(np.float32), m2, reset_codes=False)
    after = prob.get_state()
    for k in ("D", "W", "Z", "logit_pi"):
        assert np.array_equal(before[k], after[k]), k
    prm, X, Mk = oracle_problem(y2, m2, wl.patch, wl.stride, wl.K, wl.method_seed)
    st = ob.State(D=after["D"].astype(np.float64), W=after["W"].astype(np.float64),
                  Z=after["Z"].astype(bool), ell=after["logit_pi"], gamma_s=after["gamma_s"],
                  gamma_eps=after["gamma_eps"], t=after["t"])
    prob.iterate(1)
    gs = prob.get_state()
    st, rep = ob.iterate(prm, X, Mk, st, follow_z=gs["Z"])
    assert rep.hard_mismatches == 0
    compare_state(gs, st, FP32_TOL, "kept codes")
    prob.set_frame(y2.astype(np.float32), m2, reset_codes=True)
    assert not prob.get_state()["Z"].any()
    prob.close()


def test_reconstruct_from_injected_state():
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    prm, X, Mk = oracle_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    st = ob.init_state(prm, X.shape[0], X.shape[1])
    st, _ = ob.iterate(prm, X, Mk, st)
    prob = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    prob.set_state(D=st.D, W=st.W, Z=st.Z, logit_pi=st.ell, gamma_s=st.gamma_s,
                   gamma_eps=st.gamma_eps, t=st.t)
    xh = prob.reconstruct()
    st32 = ob.State(D=st.D.astype(np.float32).astype(np.float64),
                    W=st.W.astype(np.float32).astype(np.float64), Z=st.Z, ell=st.ell,
                    gamma_s=st.gamma_s, gamma_eps=st.gamma_eps, t=st.t)
    ref = ob.reconstruct(st32, wl.shape, wl.patch, wl.stride)
    assert_close(xh, ref, 1e-6, "reconstruction")
    gs = prob.get_state()
    assert np.array_equal(gs["W"], st.W.astype(np.float32))
    assert np.array_equal(gs["Z"].astype(bool), st.Z)
    assert np.array_equal(gs["D"], st.D.astype(np.float32))
    prob.close()


def test_reconstruct_identity_dyadic():
    """D = I and W = exact patches of a dyadic image: the overlap average is the image, bit for bit."""
    shape, patch, stride = (24, 20), (4, 4), (1, 1)
    rng = np.random.Generator(np.random.PCG64(9))
    img = (rng.integers(0, 64, size=shape) / 64.0).astype(np.float32)
    ones = np.ones(shape, np.uint8)
    X, _ = patches.extract(img, ones, patch, stride)
    P = X.shape[1]
    prob = gpu_problem(img, ones, patch, stride, K=P, seed=1)
    prob.set_state(D=np.eye(P), W=X, Z=X != 0)
    xh = prob.reconstruct()
    assert np.array_equal(xh, img)
    prob.close()


def test_iterations_are_deterministic():
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    outs = []
    for _ in range(2):
        prob = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
        prob.iterate(4)
        s = prob.get_state()
        outs.append((s["D"], s["W"], s["gamma_s"], s["gamma_eps"], prob.reconstruct()))
        prob.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_resume_from_state_is_bit_exact():
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    a = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    a.iterate(3)
    mid = a.get_state()
    a.iterate(2)
    end_a = a.get_state()
    b = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    b.set_state(**{k: mid[k] for k in ("D", "W", "Z", "logit_pi", "gamma_s", "gamma_eps", "t")})
    b.iterate(2)
    end_b = b.get_state()
    for k in ("D", "W", "Z", "logit_pi"):
        assert np.array_equal(end_a[k], end_b[k]), k
    assert end_a["gamma_eps"] == end_b["gamma_eps"] and end_a["t"] == end_b["t"]
    a.close()
    b.close()


def test_transfer_dictionary():
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    src = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    src.iterate(3)
    y2, m2, _ = synth.make_frame(wl, data_seed=77, rho=0.15)
    dst = gpu_problem(y2, m2, wl.patch, wl.stride, wl.K, wl.method_seed + 1, problem_id=2)
    dst.transfer_dictionary(src)
    s, d = src.get_state(), dst.get_state()
    assert np.array_equal(s["D"], d["D"]) and np.array_equal(s["logit_pi"], d["logit_pi"])
    assert s["gamma_s"] == d["gamma_s"] and s["gamma_eps"] == d["gamma_eps"]
    # sparse coding against the transferred dictionary matches the oracle
    prm, X, Mk = oracle_problem(y2, m2, wl.patch, wl.stride, wl.K, wl.method_seed + 1, problem_id=2)
    st = ob.State(D=d["D"].astype(np.float64), W=np.zeros((X.shape[0], wl.K)),
                  Z=np.zeros((X.shape[0], wl.K), bool), ell=d["logit_pi"], gamma_s=d["gamma_s"],
                  gamma_eps=d["gamma_eps"], t=d["t"])
    dst.iterate(1, bpfa.SPARSE_CODE_ONLY)
    gs = dst.get_state()
    st, rep = ob.iterate(prm, X, Mk, st, learn_dict=False, follow_z=gs["Z"])
    assert rep.hard_mismatches == 0
    compare_state(gs, st, FP32_TOL, "transfer")
    with pytest.raises(bpfa.BpfaError):
        other = gpu_problem(y, m, (4, 4), (1, 1), wl.K, 1)
        other.transfer_dictionary(src)
    src.close()
    dst.close()


def test_numeric_failure_is_reported():
    """A non-finite pixel value drives the sums non-finite; the library reports ENUMERIC."""
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    y = y.astype(np.float32)
    m = m.copy()
    y[5, 5] = np.inf
    m[5, 5] = 1
    prob = gpu_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    prob.iterate(1)
    with pytest.raises(bpfa.BpfaError) as ei:
        prob.sync()
    assert ei.value.status == bpfa.ENUMERIC
    prob.close()
