"""Gamma draws in binary64 from Philox attempts (Marsaglia & Tsang 2000).

Test infrastructure, not product code (see ``oracle/__init__.py``).

Method: G. Marsaglia and W. W. Tsang, "A simple method for generating gamma
variables", ACM TOMS 26(3), 2000.  For shape alpha >= 1 set d = alpha - 1/3 and
c = 1/sqrt(9 d); draw x ~ N(0,1), v = (1 + c x)^3, reject v <= 0, accept when
ln u < x^2/2 + d - d v + d ln v, and return d v.  For alpha < 1 the same paper's
boost is used: Ga(alpha) = Ga(alpha + 1) * U^(1/alpha), here in log space so
that tiny results (shape 1/K) do not underflow.

Attempt j of a draw reads the Philox block (c0, j, t, tag): words 0 and 1 give
x by the cosine branch of Box-Muller, word 2 gives the acceptance uniform, and
word 3 of attempt 0 gives the boost uniform.  At most 64 attempts are made.
"""
import math

import numpy as np

from . import philox

MAX_ATTEMPTS = 64


class GammaAttemptsExhausted(RuntimeError):
    pass


def log_gamma_draw(shape, seed, problem_id, tag, c0, t):
    """ln of a Ga(shape, 1) variate, with its Philox attempt stream."""
    if not (shape > 0.0) or not math.isfinite(shape):
        raise ValueError("gamma shape must be positive and finite, got %r" % (shape,))
    alpha = shape + 1.0 if shape < 1.0 else shape
    d = alpha - 1.0 / 3.0
    c = 1.0 / math.sqrt(9.0 * d)
    log_boost = 0.0
    for j in range(MAX_ATTEMPTS):
        w = philox.block_int(seed, problem_id, tag, c0, j, t)
        if j == 0 and shape < 1.0:
            log_boost = math.log(philox.uniform_int(w[3])) / shape
        u1 = philox.uniform_int(w[0])
        u2 = philox.uniform_int(w[1])
        x = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
        cx = c * x
        if cx <= -1.0:
            continue
        log_v = 3.0 * math.log1p(cx)
        v = math.exp(log_v)
        ua = philox.uniform_int(w[2])
        if math.log(ua) < 0.5 * x * x + d - d * v + d * log_v:
            return math.log(d) + log_v + log_boost
    raise GammaAttemptsExhausted("no acceptance in %d attempts" % MAX_ATTEMPTS)
