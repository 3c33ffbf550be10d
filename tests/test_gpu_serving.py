"""GPU tests of the serving form (include/bpfa_serve.h).

* A stream's reconstructions equal those of a problem handle driven directly
  through the same sequence (set_frame, sparse-coding iterations, a
  dictionary iteration every dict_every-th frame, reconstruct); the handle's
  path is itself checked against the oracle in test_gpu_parity.py.
* A stream's results are bit-identical alone and in a mix of streams with
  frames of several sizes in flight at once.
* Admission respects the HBM budget: frames larger than the whole budget
  fail with ENOMEM, the slot bytes never exceed the budget, and idle slots of
  other shapes are evicted to make room.
* Frames replayed from a slot's captured graph equal frames launched
  directly, bit for bit, in both precision forms and for both kinds of frame
  (with and without the dictionary iteration).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2311_15061_amd import bpfa  # noqa: E402
from paper_2311_15061_amd import serve  # noqa: E402
import synth  # noqa: E402

PATCH = (6, 6)
K = 24
SEED = 0x5EED


def frames_for(stream, n, sizes=(40, 52)):
    rng = np.random.Generator(np.random.PCG64(100 + stream))
    out = []
    wl = synth.workload("stem512")
    for f in range(n):
        side = int(sizes[f % len(sizes)])
        y, m, _ = synth.make_frame(wl, data_seed=int(rng.integers(1 << 30)), shape=(side, side),
                                   rho=float(rng.uniform(0.1, 0.3)))
        out.append((y.astype(np.float32), m))
    return out


def run_server(frames_by_stream, n_streams, max_slots=4, sc_iters=2, dict_every=3, budget=8 << 30,
               order="interleave", precision="bf16", use_graphs=True):
    print("server: streams=%d slots=%d %s graphs=%d" % (n_streams, max_slots, precision, use_graphs),
          flush=True)
    srv = serve.Server(patch=PATCH, K=K, n_streams=n_streams, sc_iters=sc_iters,
                       dict_every=dict_every, max_slots=max_slots, hbm_budget=budget, seed=SEED,
                       precision=precision, use_graphs=use_graphs)
    tickets = {}
    if order == "interleave":
        n = max(len(v) for v in frames_by_stream.values())
        seq = [(s, i) for i in range(n) for s in sorted(frames_by_stream) if i < len(frames_by_stream[s])]
    else:
        seq = [(s, i) for s in sorted(frames_by_stream) for i in range(len(frames_by_stream[s]))]
    for s, i in seq:
        y, m = frames_by_stream[s][i]
        t, out = srv.submit(s, y, m)
        tickets[t] = (s, i)
    srv.drain()
    res = srv.poll(10000)
    stats = srv.stats()
    srv.close()
    outs = {}
    for r in res:
        s, i = tickets[r["ticket"]]
        outs[(s, i)] = (r["status"], r["out"], r)
    return outs, stats


def direct_sequence(frames, stream, sc_iters=2, dict_every=3, precision="bf16"):
    """The same work through one problem handle per frame shape... sharing the
    stream's state through set_frame on a single handle per size would change
    shapes, so the state is carried explicitly with get/set_state."""
    state = None
    outs = []
    for i, (y, m) in enumerate(frames):
        prob = bpfa.Problem(y, m, PATCH, K=K, seed=SEED, problem_id=stream)
        prob.set_precision(precision)
        if state is not None:
            prob.set_state(D=state["D"], logit_pi=state["logit_pi"], gamma_s=state["gamma_s"],
                           gamma_eps=state["gamma_eps"], t=state["t"])
        prob.iterate(sc_iters, bpfa.SPARSE_CODE_ONLY)
        if dict_every and (i + 1) % dict_every == 0:
            prob.iterate(1, bpfa.LEARN_DICT)
        outs.append(prob.reconstruct())
        state = prob.get_state(want_codes=False)
        prob.close()
    return outs


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_stream_matches_direct_problem_path(precision):
    frames = frames_for(1, 4)
    outs, stats = run_server({1: frames}, n_streams=2, precision=precision)
    ref = direct_sequence(frames, stream=1, precision=precision)
    for i in range(len(frames)):
        st, out, r = outs[(1, i)]
        assert st == bpfa.OK
        assert r["frame_index"] == i and r["learned"] == int((i + 1) % 3 == 0)
        assert np.array_equal(out, ref[i]), "frame %d differs" % i


def test_alone_and_in_mix_are_bit_identical():
    f0 = frames_for(0, 5)
    alone, _ = run_server({0: f0}, n_streams=4, max_slots=1)
    mix = {s: frames_for(s, 5, sizes=(40, 52, 34)) for s in range(1, 4)}
    mix[0] = f0
    mixed, stats = run_server(mix, n_streams=4, max_slots=4)
    assert stats["completed"] == 20 and stats["failed"] == 0
    for i in range(5):
        assert alone[(0, i)][0] == bpfa.OK and mixed[(0, i)][0] == bpfa.OK
        assert np.array_equal(alone[(0, i)][1], mixed[(0, i)][1]), "frame %d" % i
    assert stats["peak_slot_bytes"] <= 8 << 30


def test_transferred_dictionary():
    wl = synth.workload("stem512")
    y, m, _ = synth.make_frame(wl, data_seed=5, shape=(48, 48), rho=0.3)
    teacher = bpfa.Problem(y.astype(np.float32), m, PATCH, K=K, seed=77)
    teacher.iterate(4)
    frames = frames_for(2, 2)
    srv = serve.Server(patch=PATCH, K=K, n_streams=3, sc_iters=2, dict_every=0, seed=SEED,
                       precision="bf16")
    srv.set_dictionary(2, teacher)
    for y2, m2 in frames:
        srv.submit(2, y2, m2)
    srv.drain()
    res = sorted(srv.poll(), key=lambda r: r["ticket"])
    srv.close()
    ts = teacher.get_state(want_codes=False)
    state = dict(D=ts["D"], logit_pi=ts["logit_pi"], gamma_s=ts["gamma_s"],
                 gamma_eps=ts["gamma_eps"], t=1)
    for i, (y2, m2) in enumerate(frames):
        prob = bpfa.Problem(y2, m2, PATCH, K=K, seed=SEED, problem_id=2)
        prob.set_precision("bf16")
        prob.set_state(**state)
        prob.iterate(2, bpfa.SPARSE_CODE_ONLY)
        assert np.array_equal(res[i]["out"], prob.reconstruct())
        s = prob.get_state(want_codes=False)
        state = dict(D=s["D"], logit_pi=s["logit_pi"], gamma_s=s["gamma_s"],
                     gamma_eps=s["gamma_eps"], t=s["t"])
        prob.close()
    with pytest.raises(bpfa.BpfaError):
        small = bpfa.Problem(y.astype(np.float32), m, (4, 4), K=K, seed=1)
        srv2 = serve.Server(patch=PATCH, K=K, n_streams=1)
        try:
            srv2.set_dictionary(0, small)
        finally:
            srv2.close()
    teacher.close()


def test_admission_by_hbm_budget():
    a = frames_for(0, 2, sizes=(40,))
    b = frames_for(1, 2, sizes=(52,))
    need_a = bpfa.workspace_size(bpfa.make_params((40, 40), PATCH, K=K))
    need_b = bpfa.workspace_size(bpfa.make_params((52, 52), PATCH, K=K))
    # a budget below one workspace: every frame is refused, nothing is allocated
    outs, stats = run_server({0: a}, n_streams=2, budget=need_a // 2)
    assert all(v[0] == bpfa.ENOMEM for v in outs.values())
    assert stats["peak_slot_bytes"] == 0 and stats["failed"] == 2
    # room for one slot at a time: frames of two sizes alternate by eviction
    budget = max(need_a, need_b) + 1
    outs, stats = run_server({0: a, 1: b}, n_streams=2, budget=budget)
    assert stats["completed"] == 4 and stats["failed"] == 0
    assert stats["peak_slot_bytes"] <= budget
    assert stats["slot_evictions"] >= 1


def test_failed_frame_leaves_stream_state():
    """A frame whose noise-precision draw underflows (no observed pixel under the
    vague Ga(1e-6, 1e-6) prior: ENUMERIC) is reported failed and leaves its
    stream's dictionary state and Philox iteration counter untouched: the next
    frame equals a direct run that skips the failed frame."""
    good = frames_for(3, 2)
    side = good[0][0].shape[0]
    empty = (good[0][0], np.zeros((side, side), np.uint8))
    seq = [good[0], empty, good[1]]
    outs, stats = run_server({3: seq}, n_streams=4, dict_every=0, precision="fp32")
    assert outs[(3, 0)][0] == bpfa.OK
    assert outs[(3, 1)][0] == bpfa.ENUMERIC
    assert outs[(3, 2)][0] == bpfa.OK
    assert stats["failed"] == 1 and stats["completed"] == 2
    ref = direct_sequence(good, stream=3, dict_every=0, precision="fp32")
    assert np.array_equal(outs[(3, 0)][1], ref[0])
    assert np.array_equal(outs[(3, 2)][1], ref[1]), "frame after the failure"


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_graph_replay_matches_direct_launches(precision):
    """Two streams, frames of two sizes, a dictionary iteration every third
    frame: each slot runs its first frame of a kind directly, captures the
    second and replays the rest.  The same sequence with graphs off gives
    the same reconstructions bit for bit."""
    frames = {s: frames_for(10 + s, 8, sizes=(40, 52)) for s in range(2)}
    graphed, gst = run_server(frames, n_streams=2, max_slots=4, precision=precision, use_graphs=True)
    direct, dst = run_server(frames, n_streams=2, max_slots=4, precision=precision, use_graphs=False)
    print("graph captures %d, replayed frames %d" % (gst["graph_captures"], gst["graph_frames"]),
          flush=True)
    assert gst["completed"] == 16 and dst["completed"] == 16
    assert gst["graph_captures"] >= 2 and gst["graph_frames"] >= 6
    assert dst["graph_captures"] == 0 and dst["graph_frames"] == 0
    for key in direct:
        assert graphed[key][0] == bpfa.OK and direct[key][0] == bpfa.OK
        assert np.array_equal(graphed[key][1], direct[key][1]), "frame %s" % (key,)
