"""Writes the free-running golden values of the named workloads.

For each workload the binary64 oracle runs the workload's full iteration
count (every iteration a sparse-coding and a dictionary-learning step, the
BPFA section's sampler) from the prior start, with no coupling to any other
implementation.  Stored with the run's settings in
free_running_<workload>.json next to this script: the PSNR against the
ground truth of the last sample's overlap-averaged reconstruction, of every
iteration's sample, and of the posterior mean of the second half of the
samples (the sample mean of their reconstructions).  Only the oracle and the
seeded input generator are imported.

    python tests/golden/make_free_running.py stem512 stem1024
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import bpfa as ob  # noqa: E402
from oracle import patches  # noqa: E402


def psnr_db(x, ref):
    """10 log10(1 / mean squared error), data range 1 (the data are scaled to [0, 1])."""
    err = np.asarray(x, np.float64) - np.asarray(ref, np.float64)
    return 10.0 * math.log10(1.0 / float(np.mean(err * err)))


def run(name):
    wl = synth.workload(name)
    y, m, g = synth.make_frame(wl)
    X, Mk = patches.extract(y, m, wl.patch, wl.stride)
    prm = ob.Params(K=wl.K, seed=wl.method_seed)
    st = ob.init_state(prm, X.shape[0], X.shape[1])
    t0 = time.time()
    per_iter = []
    burn = wl.iters - wl.iters // 2
    acc = np.zeros(wl.shape)
    for it in range(wl.iters):
        st, _ = ob.iterate(prm, X, Mk, st)
        xh = ob.reconstruct(st, wl.shape, wl.patch, wl.stride)
        per_iter.append(psnr_db(xh, g))
        if it >= burn:
            acc += xh          # the posterior mean's sum, as ob.posterior_mean forms it
        print("%s iteration %d: PSNR %.4f dB, mean active %.3f, %.0f s" % (
            name, it + 1, per_iter[-1], st.Z.sum() / st.Z.shape[0], time.time() - t0), flush=True)
    out = {
        "workload": name, "iters": wl.iters, "K": wl.K, "seed": wl.method_seed,
        "psnr_db": per_iter[-1], "psnr_db_per_iteration": per_iter,
        "mean_burn_in": burn, "mean_samples": wl.iters - burn,
        "psnr_db_posterior_mean": psnr_db(acc / (wl.iters - burn), g),
        "mean_active": float(st.Z.sum() / st.Z.shape[0]), "gamma_eps": st.gamma_eps,
        "gamma_s": st.gamma_s, "oracle_seconds": time.time() - t0,
        "written_by": "tests/golden/make_free_running.py",
    }
    with open(os.path.join(HERE, "free_running_%s.json" % name), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    for name in sys.argv[1:]:
        run(name)
