"""Free-running parity: no follow mode.

The GPU and the binary64 oracle each run a whole workload from the prior
start, every iteration a sparse-coding and a dictionary-learning step, with
nothing passed between them but the seed.  Their chains draw the same
Philox numbers, so they stay equal until a decision near a tie rounds
differently and then go their own ways; what must agree is the quality of
the result: the PSNR of the final sample's overlap-averaged reconstruction
against the ground truth within 0.1 dB of the oracle's, in both precision
forms.

* 64 x 64 lattice (K = 32, 10 iterations): the oracle runs beside the GPU.
* 512 x 512 frame (K = 128, 20 iterations) and 1024 x 1024 frame (K = 256,
  20 iterations): the oracle's PSNR is the stored value that
  tests/golden/make_free_running.py writes by running the oracle alone.
"""
import json
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import bpfa as ob  # noqa: E402
from oracle import patches  # noqa: E402
from parity_util import record  # noqa: E402

from paper_2311_15061_amd import bpfa  # noqa: E402
import synth  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PSNR_TOL_DB = 0.1


def psnr_db(x, ref):
    err = np.asarray(x, np.float64) - np.asarray(ref, np.float64)
    return 10.0 * math.log10(1.0 / float(np.mean(err * err)))


def _gpu_run(wl, y, m, precision):
    print("case: %s free-running %d iterations, %s" % (wl.name, wl.iters, precision), flush=True)
    prob = bpfa.Problem(np.asarray(y, np.float32), m, wl.patch, wl.stride, K=wl.K, seed=wl.method_seed)
    prob.set_precision(precision)
    return prob


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_free_running_lattice64(precision):
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    X, Mk = patches.extract(y, m, wl.patch, wl.stride)
    prm = ob.Params(K=wl.K, seed=wl.method_seed)
    st = ob.init_state(prm, X.shape[0], X.shape[1])
    prob = _gpu_run(wl, y, m, precision)
    same_until = 0
    for it in range(wl.iters):
        st, _ = ob.iterate(prm, X, Mk, st)
        prob.iterate(1, bpfa.LEARN_DICT)
        if same_until == it and np.array_equal(prob.get_state()["Z"].astype(bool), st.Z):
            same_until = it + 1
    xh = prob.reconstruct()
    prob.close()
    p_gpu = psnr_db(xh, g)
    p_ref = psnr_db(ob.reconstruct(st, wl.shape, wl.patch, wl.stride), g)
    print("lattice64 %s: PSNR %.4f dB, oracle %.4f dB; z equal for the first %d of %d iterations"
          % (precision, p_gpu, p_ref, same_until, wl.iters), flush=True)
    record("lattice64 free-running, %s" % precision, psnr_db=p_gpu, oracle_psnr_db=p_ref,
           psnr_diff_db=p_gpu - p_ref, z_equal_iterations=same_until)
    assert abs(p_gpu - p_ref) <= PSNR_TOL_DB


@pytest.mark.parametrize("name,precision", [("stem512", "fp32"), ("stem512", "bf16"),
                                            ("stem1024", "fp32"), ("stem1024", "bf16")])
def test_free_running_against_stored_oracle_psnr(name, precision):
    path = os.path.join(GOLDEN, "free_running_%s.json" % name)
    with open(path) as fh:
        gold = json.load(fh)
    wl = synth.workload(name)
    assert gold["iters"] == wl.iters and gold["K"] == wl.K and gold["seed"] == wl.method_seed
    y, m, g = synth.make_frame(wl)
    prob = _gpu_run(wl, y, m, precision)
    prob.iterate(wl.iters, bpfa.LEARN_DICT)
    xh = prob.reconstruct()
    prob.close()
    p_gpu = psnr_db(xh, g)
    print("%s %s: PSNR %.4f dB, stored oracle %.4f dB" % (name, precision, p_gpu, gold["psnr_db"]),
          flush=True)
    record("%s free-running, %s" % (name, precision), psnr_db=p_gpu, oracle_psnr_db=gold["psnr_db"],
           psnr_diff_db=p_gpu - gold["psnr_db"])
    assert abs(p_gpu - gold["psnr_db"]) <= PSNR_TOL_DB
