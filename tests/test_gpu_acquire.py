"""Acquisition policies on the serving path (Feature summary: pre-determined
indexing methods and on-the-fly strategic selection).

* The device's masks equal the oracle's for the uniform and line-hop rules
  bit for bit, and for the targeted rule on given weights except at ties
  (none expected: both sides compute p in binary64 from the same weights,
  differing only in the order of the weights' sum).
* A stream with the targeted policy: each frame's mask is drawn from the
  posterior variance of the last two samples of the stream's previous frame.
  The served masks and reconstructions equal a problem handle driven through
  the same frames with bpfa_acquire_mask and bpfa_mean_accumulate /
  bpfa_variance_get, bit for bit; and the oracle, following the handle's z
  decisions, draws its own masks from its own variance: the same masks
  (except at certified near-ties, where it adopts the served one), the
  handle's state after every iteration within the binary32 bar, the
  reconstructions within 1e-5.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import acquire as oa  # noqa: E402
from oracle import bpfa as ob  # noqa: E402
from oracle import patches, philox  # noqa: E402
from parity_util import FP32_TOL, assert_close, record  # noqa: E402

from paper_2311_15061_amd import bpfa, serve  # noqa: E402
from test_gpu_parity import compare_state  # noqa: E402
import synth  # noqa: E402

SEED = 0xACC1
PATCH = (6, 6)
K = 24


@pytest.mark.parametrize("shape,rho,stream,frame", [
    ((64, 64), 0.1, 0, 0), ((37, 50), 0.25, 3, 7), ((12, 10, 9), 0.3, 1, 2), ((300,), 0.05, 2, 11)])
def test_uniform_and_line_hop_masks_match_oracle(shape, rho, stream, frame):
    for kind, ref in (("uniform", oa.uniform_mask), ("line_hop", oa.line_hop_mask)):
        got = serve.acquire_mask(kind, shape, SEED, stream, frame, fraction=rho)
        want = ref(shape, rho, SEED, stream, frame)
        assert np.array_equal(got, want), (kind, shape)


def _near_tie_mismatches(got, weights, rho, share, stream, frame, tol):
    """Sites where got differs from the oracle's targeted mask: (near-ties, hard)."""
    want = oa.targeted_mask(weights, rho, share, SEED, stream, frame)
    diff = np.nonzero(got.ravel() != want.ravel())[0]
    if diff.size == 0:
        return 0, 0
    p = oa.targeted_probabilities(weights, rho, share)[diff]
    u = philox.uniform(philox.block(SEED, stream, philox.TAG_ACQ, diff.astype(np.uint64),
                                    np.zeros(diff.size, np.uint64), frame)[0])
    tie = np.abs(u - p) <= tol * p
    return int(tie.sum()), int((~tie).sum())


@pytest.mark.parametrize("share", [0.0, 0.6, 1.0])
def test_targeted_masks_match_oracle_on_given_weights(share):
    rng = np.random.Generator(np.random.PCG64(7))
    shape = (80, 72)
    w = rng.gamma(0.5, size=shape).astype(np.float32)
    w[rng.random(shape) < 0.2] = 0.0
    got = serve.acquire_mask("targeted", shape, SEED, 4, 5, fraction=0.15, targeted_share=share,
                             weights=w)
    ties, hard = _near_tie_mismatches(got, w.astype(np.float64), 0.15, share, 4, 5, 1e-12)
    assert hard == 0 and ties == 0
    # no weights yet: the uniform rule
    got0 = serve.acquire_mask("targeted", shape, SEED, 4, 5, fraction=0.15, targeted_share=share)
    assert np.array_equal(got0, oa.uniform_mask(shape, 0.15, SEED, 4, 5))


def test_targeted_stream_matches_direct_path_and_oracle():
    stream, sc_iters, dict_every, V, rho, share = 1, 2, 2, 2, 0.2, 0.6
    wl = synth.workload("stem512")
    scenes = [synth.make_frame(wl, data_seed=900 + f, shape=(40, 40))[0].astype(np.float32)
              for f in range(4)]
    print("targeted stream: 4 frames of 40 x 40, rho %.2f, share %.2f" % (rho, share), flush=True)
    srv = serve.Server(patch=PATCH, K=K, n_streams=2, sc_iters=sc_iters, dict_every=dict_every,
                       max_slots=2, seed=SEED)
    srv.set_policy(stream, "targeted", fraction=rho, targeted_share=share, var_samples=V)
    tickets = [srv.submit_scene(stream, y)[0] for y in scenes]
    srv.drain()
    res = {r["ticket"]: r for r in srv.poll()}
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == 4 and stats["failed"] == 0

    prm = ob.Params(K=K, seed=SEED, problem_id=stream)
    st = ob.init_state(prm, 1, int(np.prod(PATCH)))
    var_gpu, var_orc, gs = None, None, None
    ties_total = 0
    worst = {}
    for f, y in enumerate(scenes):
        r = res[tickets[f]]
        assert r["status"] == bpfa.OK and r["frame_index"] == f
        # the direct path: the same mask from the previous frame's variance
        m = serve.acquire_mask("targeted", y.shape, SEED, stream, f, fraction=rho,
                               targeted_share=share, weights=var_gpu)
        assert np.array_equal(r["mask"], m), "frame %d mask" % f
        # the oracle's own mask from its own variance, adopting the served
        # decision only at certified near-ties
        if var_orc is None:
            assert np.array_equal(m, oa.uniform_mask(y.shape, rho, SEED, stream, f))
        else:
            ties, hard = _near_tie_mismatches(m, var_orc, rho, share, stream, f, 1e-4)
            assert hard == 0, "frame %d: %d mask decisions differ away from ties" % (f, hard)
            ties_total += ties
        learn_frame = (f + 1) % dict_every == 0
        its = [False] * sc_iters + ([True] if learn_frame else [])
        X, Mk = patches.extract(y.astype(np.float64), m, PATCH, (1, 1))
        N = X.shape[0]
        st = ob.State(D=st.D, W=np.zeros((N, K)), Z=np.zeros((N, K), bool), ell=st.ell,
                      gamma_s=st.gamma_s, gamma_eps=st.gamma_eps, t=st.t)
        prob = bpfa.Problem(y, m, PATCH, K=K, seed=SEED, problem_id=stream)
        if gs is not None:
            prob.set_state(D=gs["D"], logit_pi=gs["logit_pi"], gamma_s=gs["gamma_s"],
                           gamma_eps=gs["gamma_eps"], t=gs["t"])
        kept = []
        for i, learn in enumerate(its):
            prob.iterate(1, bpfa.LEARN_DICT if learn else bpfa.SPARSE_CODE_ONLY)
            gs = prob.get_state()
            st, rep = ob.iterate(prm, X, Mk, st, learn_dict=learn, follow_z=gs["Z"])
            assert rep.hard_mismatches == 0, "frame %d: %s" % (f, rep.hard_sites[:5])
            compare_state(gs, st, FP32_TOL, "frame %d" % f)
            if i >= len(its) - V:
                prob.mean_accumulate()
                kept.append(st)
        xh = prob.reconstruct()
        var_gpu, _ = prob.posterior_variance()
        prob.close()
        assert np.array_equal(r["out"], xh), "served frame %d differs from the handle's" % f
        worst["recon"] = max(worst.get("recon", 0.0), assert_close(
            xh, ob.reconstruct(st, y.shape, PATCH, (1, 1)), FP32_TOL, "frame %d reconstruction" % f))
        var_orc = ob.posterior_variance(kept, y.shape, PATCH, (1, 1))
        worst["variance"] = max(worst.get("variance", 0.0),
                                assert_close(var_gpu, var_orc, 1e-4, "frame %d variance" % f))
    print("mask near-ties adopted: %d" % ties_total, flush=True)
    record("targeted acquisition stream, 4 frames 40 px, K=24, fp32", mask_near_ties=ties_total,
           **worst)
