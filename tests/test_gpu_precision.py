"""GPU parity of the reconstruction's contraction in both precision forms.

The patch models y_i = D^T w_i run either in binary32 on the vector ALUs
over each patch's active atoms (BPFA_FP32), or densely on the BF16 matrix
cores as head products plus one binary32 correction pass (BPFA_BF16).  States are injected (binary32-representable D and W), so the
oracle's binary64 overlap average of the same state is the reference:

* FP32 form: within 1e-6 (binary32 rounding of short sums).
* BF16 form: within the BF16 bar 2e-2, and within 1e-4, which only holds
  if the correction pass runs (a head-only BF16 product errs by ~2^-9).
* A sampled trajectory (lattice 64 x 64, 10 iterations) reconstructed in the
  BF16 form stays within 2e-2 of the oracle, and its PSNR against the clean
  image within 0.1 dB of the oracle's.
Shapes cover one and several 32-row tiles of P with a ragged last tile,
several 64-atom stages with a ragged tail, patch counts that leave a ragged
last 128-patch block, and 3-D patches.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import bpfa as ob  # noqa: E402
from oracle import patches  # noqa: E402
from parity_util import FP32_TOL, assert_close, oracle_problem, rel_err  # noqa: E402

from paper_2311_15061_amd import bpfa, metrics  # noqa: E402
import synth  # noqa: E402


def injected_case(shape, patch, stride, K, density, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    img = rng.random(shape).astype(np.float32)
    mask = (rng.random(shape) < 0.3).astype(np.uint8)
    X, _ = patches.extract(img, mask, patch, stride)
    N, P = X.shape
    D = (rng.standard_normal((K, P)) / np.sqrt(P)).astype(np.float32)
    Z = rng.random((N, K)) < density
    W = np.where(Z, rng.standard_normal((N, K)), 0.0).astype(np.float32)
    return img, mask, D, W, Z


@pytest.mark.parametrize("shape,patch,stride,K,density", [
    ((64, 64), (8, 8), (1, 1), 32, 0.3),          # P = 64: two full row tiles, one atom stage
    ((47, 45), (10, 10), (1, 1), 128, 0.1),       # P = 100: ragged row tile, 2 stages, ragged blocks
    ((30, 30), (12, 12), (1, 1), 200, 0.15),      # P = 144 (5 tiles), ragged 4th stage
    ((20, 18, 8), (4, 4, 2), (1, 1, 2), 24, 0.4),  # 3-D, P = 32, K < one stage
    ((9, 9), (3, 3), (1, 1), 5, 1.0),             # P = 9, K = 5, dense codes, N = 49 < one block
    ((40, 40), (16, 16), (2, 2), 70, 0.2),        # P = 256 (8 tiles), strided grid
])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_reconstruction_contraction(shape, patch, stride, K, density, precision):
    img, mask, D, W, Z = injected_case(shape, patch, stride, K, density, seed=K + len(shape))
    print("case: %s shape=%s patch=%s K=%d" % (precision, shape, patch, K), flush=True)
    prob = bpfa.Problem(img, mask, patch, stride, K=K, seed=3)
    prob.set_state(D=D, W=W, Z=Z)
    prob.set_precision(precision)
    xh = prob.reconstruct()
    st = ob.State(D=D.astype(np.float64), W=W.astype(np.float64), Z=Z, ell=np.zeros(K),
                  gamma_s=1.0, gamma_eps=1.0, t=1)
    ref = ob.reconstruct(st, shape, patch, stride)
    e = rel_err(xh, ref)
    print("  error vs binary64: %.3e" % e, flush=True)
    if precision == "fp32":
        assert_close(xh, ref, 1e-6, "fp32 reconstruction")
    else:
        assert_close(xh, ref, 2e-2, "bf16 reconstruction")
        assert_close(xh, ref, 1e-4, "bf16 reconstruction with its correction pass")
    prob.close()


def test_precision_is_per_handle_and_switchable():
    img, mask, D, W, Z = injected_case((40, 40), (8, 8), (1, 1), 48, 0.2, seed=11)
    prob = bpfa.Problem(img, mask, (8, 8), (1, 1), K=48, seed=3)
    prob.set_state(D=D, W=W, Z=Z)
    a = prob.reconstruct()
    prob.set_precision("bf16")
    b = prob.reconstruct()
    prob.set_precision("fp32")
    c = prob.reconstruct()
    assert np.array_equal(a, c)
    assert not np.array_equal(a, b)
    assert bpfa.lib.bpfa_set_precision(prob.handle, 7) == bpfa.EINVAL
    with pytest.raises(ValueError):
        prob.set_precision("fp16")
    prob.close()


def test_bf16_trajectory_and_psnr_lattice64():
    wl = synth.workload("lattice64")
    y, m, g = synth.make_frame(wl)
    prm, X, Mk = oracle_problem(y, m, wl.patch, wl.stride, wl.K, wl.method_seed)
    prob = bpfa.Problem(y.astype(np.float32), m, wl.patch, wl.stride, K=wl.K, seed=wl.method_seed)
    prob.set_precision("bf16")
    st = ob.init_state(prm, X.shape[0], X.shape[1])
    for it in range(wl.iters):
        prob.iterate(1)
        gs = prob.get_state()
        st, rep = ob.iterate(prm, X, Mk, st, follow_z=gs["Z"])
        assert rep.hard_mismatches == 0, "iteration %d" % it
    xh = prob.reconstruct()
    ref = ob.reconstruct(st, wl.shape, wl.patch, wl.stride)
    e = assert_close(xh, ref, 2e-2, "bf16 reconstruction after %d iterations" % wl.iters)
    p_gpu = metrics.psnr(xh.astype(np.float64), g)
    p_ref = metrics.psnr(ref, g)
    print("bf16 reconstruction: error vs binary64 %.3e, PSNR %.4f dB vs oracle %.4f dB"
          % (e, p_gpu, p_ref), flush=True)
    assert abs(p_gpu - p_ref) <= 0.1
    prob.close()


def test_bf16_rejected_for_patches_over_256_pixels():
    """The matrix-core tiles hold at most 256 patch pixels: asking a handle with
    17 x 17 patches for the BF16 form fails at once (ESHAPE), and the handle
    keeps reconstructing in binary32."""
    rng = np.random.Generator(np.random.PCG64(5))
    img = rng.random((24, 24)).astype(np.float32)
    mask = (rng.random((24, 24)) < 0.3).astype(np.uint8)
    prob = bpfa.Problem(img, mask, (17, 17), K=8, seed=3)
    with pytest.raises(bpfa.BpfaError) as ei:
        prob.set_precision("bf16")
    assert ei.value.status == bpfa.ESHAPE
    prob.iterate(1)
    assert np.all(np.isfinite(prob.reconstruct()))
    prob.close()
