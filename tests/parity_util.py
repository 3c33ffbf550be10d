"""Helpers shared by the GPU parity tests (oracle on the CPU, HIP library on the GPU)."""
import json
import os

import numpy as np

import synth
from oracle import bpfa as ob
from oracle import patches

FP32_TOL = 1e-5


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def assert_close(a, b, tol=FP32_TOL, what=""):
    """Normwise relative error <= tol and elementwise |a-b| <= tol (|b| + rms(b))."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    e = rel_err(a, b)
    assert e <= tol, "%s: normwise relative error %.3e > %.1e" % (what, e, tol)
    rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
    bad = np.abs(a - b) > tol * (np.abs(b) + rms) + 1e-30
    assert not bad.any(), "%s: %d elements off, worst %.3e at %s" % (
        what, int(bad.sum()), float(np.abs(a - b).max()), np.unravel_index(np.argmax(np.abs(a - b)), a.shape))
    return e


def case(shape, patch, stride, K, rho, seed, fp64=False, data_seed=None):
    """A small synthetic lattice problem of arbitrary dimension."""
    rng = np.random.Generator(np.random.PCG64(seed if data_seed is None else data_seed))
    if len(shape) == 2:
        wl = synth.Workload("case", tuple(shape), tuple(patch), tuple(stride), K=K, iters=1, rho=rho,
                            lattice="hex", period=6.0, sigma=1.5, dose=100.0, vacancy=0.05,
                            data_seed=int(rng.integers(1 << 30)), fp64_input=fp64)
        y, m, g = synth.make_frame(wl)
    else:
        y = rng.random(shape).astype(np.float64 if fp64 else np.float32)
        m = synth.make_mask(shape, rho, rng)
        g = y.astype(np.float64)
    return y, m, g


def oracle_problem(y, m, patch, stride, K, seed, problem_id=0, **hyper):
    X, Mk = patches.extract(y, m, patch, stride)
    prm = ob.Params(K=K, seed=seed, problem_id=problem_id, **hyper)
    return prm, X, Mk


def state_errors(gs, st):
    """Relative errors against the binary64 oracle of every sampler output:
    normwise for D, W and logit pi, relative for the two precisions."""
    return {"D": rel_err(gs["D"], st.D), "W": rel_err(gs["W"], st.W),
            "logit_pi": rel_err(gs["logit_pi"], st.ell),
            "gamma_s": abs(gs["gamma_s"] / st.gamma_s - 1.0),
            "gamma_eps": abs(gs["gamma_eps"] / st.gamma_eps - 1.0)}


def record(config, **errors):
    """Append one line of measured errors against binary64 to the file named by
    the BPFA_PARITY_RECORD environment variable (nothing when it is unset)."""
    path = os.environ.get("BPFA_PARITY_RECORD")
    line = {"config": config}
    line.update({k: (float(v) if isinstance(v, (float, np.floating)) else v) for k, v in errors.items()})
    print("errors vs binary64:", json.dumps(line), flush=True)
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(line) + "\n")
