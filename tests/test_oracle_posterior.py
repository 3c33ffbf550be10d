"""Pins of the oracle's posterior-mean reconstruction (average of the kept
Gibbs samples' overlap-averaged reconstructions)."""
import itertools

import numpy as np
import pytest

from oracle import bpfa, patches


def _states(shape, patch, stride, K, S, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    N = int(np.prod(patches.grid_shape(shape, patch, stride)))
    P = int(np.prod(patch))
    out = []
    for _ in range(S):
        Z = rng.random((N, K)) < 0.3
        W = Z * rng.standard_normal((N, K))
        out.append(bpfa.State(D=rng.standard_normal((K, P)), W=W, Z=Z, ell=np.zeros(K),
                              gamma_s=1.0, gamma_eps=1.0, t=1))
    return out


def _brute_force_mean(states, shape, patch, stride):
    """Pixel by pixel from the definitions: for every pixel q, over the samples,
    the mean of the patch models of the patches that cover q at the offset
    that lands on q."""
    grid = patches.grid_shape(shape, patch, stride)
    origins = [tuple(g * s for g, s in zip(gi, stride)) for gi in itertools.product(*map(range, grid))]
    offsets = list(itertools.product(*map(range, patch)))
    out = np.zeros(shape)
    for q in itertools.product(*map(range, shape)):
        total = 0.0
        for st in states:
            Y = st.W @ st.D
            vals = [Y[i, j] for i, o in enumerate(origins) for j, b in enumerate(offsets)
                    if all(oo + bb == qq for oo, bb, qq in zip(o, b, q))]
            total += sum(vals) / len(vals)
        out[q] = total / len(states)
    return out


@pytest.mark.parametrize("shape,patch,stride", [((7, 6), (3, 2), (1, 2)), ((5, 4, 4), (2, 2, 2), (1, 1, 2))])
def test_posterior_mean_brute_force(shape, patch, stride):
    states = _states(shape, patch, stride, K=5, S=3, seed=11)
    got = bpfa.posterior_mean(states, shape, patch, stride)
    ref = _brute_force_mean(states, shape, patch, stride)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_posterior_mean_of_one_sample_is_its_reconstruction():
    shape, patch, stride = (9, 8), (3, 3), (1, 1)
    st = _states(shape, patch, stride, K=4, S=1, seed=3)[0]
    assert np.array_equal(bpfa.posterior_mean([st], shape, patch, stride),
                          bpfa.reconstruct(st, shape, patch, stride))


def test_posterior_mean_is_linear_in_the_patch_models():
    """Mean of overlap averages = overlap average of the mean patch models."""
    shape, patch, stride = (10, 9), (4, 3), (2, 1)
    states = _states(shape, patch, stride, K=6, S=4, seed=5)
    Ybar = sum(st.W @ st.D for st in states) / len(states)
    assert np.allclose(bpfa.posterior_mean(states, shape, patch, stride),
                       patches.overlap_average(Ybar, shape, patch, stride), rtol=1e-12, atol=1e-12)


def test_posterior_mean_needs_a_sample():
    with pytest.raises(ValueError):
        bpfa.posterior_mean([], (4, 4), (2, 2), (1, 1))


def test_posterior_variance_two_samples_closed_form():
    """n = 2: the unbiased variance is (a - b)^2 / 2 pixel by pixel."""
    shape, patch, stride = (8, 7), (3, 2), (1, 1)
    s1, s2 = _states(shape, patch, stride, K=4, S=2, seed=9)
    a = bpfa.reconstruct(s1, shape, patch, stride)
    b = bpfa.reconstruct(s2, shape, patch, stride)
    assert np.allclose(bpfa.posterior_variance([s1, s2], shape, patch, stride), (a - b) ** 2 / 2,
                       rtol=1e-12, atol=1e-15)


def test_posterior_variance_matches_numpy_and_vanishes_on_repeats():
    shape, patch, stride = (9, 6, 3), (3, 2, 3), (1, 1, 1)
    states = _states(shape, patch, stride, K=5, S=5, seed=13)
    stack = np.stack([_brute_force_mean([st], shape, patch, stride) for st in states])
    assert np.allclose(bpfa.posterior_variance(states, shape, patch, stride),
                       np.var(stack, axis=0, ddof=1), rtol=1e-10, atol=1e-14)
    # repeated samples: zero up to the rounding of the mean
    x = bpfa.reconstruct(states[0], shape, patch, stride)
    v0 = bpfa.posterior_variance([states[0]] * 3, shape, patch, stride)
    assert np.all(v0 <= 1e-30 * (1.0 + x * x))
    with pytest.raises(ValueError):
        bpfa.posterior_variance(states[:1], shape, patch, stride)
