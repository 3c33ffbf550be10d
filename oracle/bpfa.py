"""Plain binary64 Gibbs sampler for Beta-Process Factor Analysis (BPFA).

Test infrastructure, not product code (see ``oracle/__init__.py``).

The paper (section "Beta-Process Factor Analysis") names BPFA, its
per-iteration dictionary-learning and sparse-coding steps and blind
inpainting from the observed pixels only, and defers the model to the works
it cites (Paisley & Carin, ICML 2009; Zhou et al., NIPS 2009).  The model
written out here is the finite-K beta-process approximation of those works,
with the likelihood restricted to observed pixels Obs(i) of each patch:

    x_ip ~ N( sum_k d_kp z_ik s_ik , 1/gamma_eps )   for p in Obs(i)
    d_k  ~ N(0, I_P / P)         s_ik ~ N(0, 1/gamma_s)
    z_ik ~ Bernoulli(pi_k)       pi_k ~ Beta(a/K, b(K-1)/K)
    gamma_s ~ Ga(c, d)           gamma_eps ~ Ga(e, f)        (shape, rate)

State: D (K x P), W = Z * S (N x K, inactive weights are not instantiated),
ell_k = logit pi_k, gamma_s, gamma_eps and the iteration number t.

One iteration, in this order:
  1. z/s sweep: every patch independently, atoms k = 0 .. K-1 in order, draws
     z_ik from its conditional with s_ik integrated out, then s_ik given z_ik;
  2. dictionary: atoms k = 0 .. K-1 in order, d_k from its Gaussian
     conditional (skipped in sparse-coding-only iterations);
  3. pi_k from its Beta conditional, as ell_k = ln G_A - ln G_B;
  4. gamma_s; 5. gamma_eps (residual after step 2); 6. t <- t + 1.

Mini-batch epochs (the Time-to-solution section trains for "complete
epochs"; the paper gives no schedule, so this is a reading): the patches are
dealt into B batches, patch i to batch i mod B; an epoch takes the batches in
ascending order, and each batch step is one iteration of steps 1-6 in which
the sweep visits only that batch's patches and the global draws (2-5) use
the batch's statistics scaled by s = N / n_b, i.e. the conditionals given a
data set made of s copies of the batch.  Every batch step is an iteration
number of its own (t advances per step), so each step draws fresh numbers.
With B = 1 a batch step is exactly the full iteration.

Random numbers come from oracle.philox under the stream contract described
there; a GPU implementation that follows the same contract draws the same
uniforms, so the two can be compared draw by draw.
"""
import dataclasses
import math

import numpy as np

from . import gamma as _gamma
from . import philox


@dataclasses.dataclass
class Params:
    K: int
    a: float = 1.0
    b: float = 1.0
    c: float = 1e-6
    d: float = 1e-6
    e: float = 1e-6
    f: float = 1e-6
    gamma_s0: float = 1.0
    gamma_eps0: float = 100.0
    seed: int = 0
    problem_id: int = 0


@dataclasses.dataclass
class State:
    D: np.ndarray          # K x P
    W: np.ndarray          # N x K, z * s
    Z: np.ndarray          # N x K, bool
    ell: np.ndarray        # K, logit pi
    gamma_s: float
    gamma_eps: float
    t: int

    def copy(self):
        return State(self.D.copy(), self.W.copy(), self.Z.copy(), self.ell.copy(),
                     float(self.gamma_s), float(self.gamma_eps), int(self.t))


@dataclasses.dataclass
class SweepReport:
    near_ties: int = 0          # follow mode: mismatches adopted as certified near-ties
    hard_mismatches: int = 0    # follow mode: mismatches away from the threshold
    tie_sites: list = dataclasses.field(default_factory=list)   # (i, k) of adopted ties
    hard_sites: list = dataclasses.field(default_factory=list)


# ---------------------------------------------------------------- draws ----

def zs_uniforms(params, i, k, t):
    """Sweep draws for patches i at atom k: (u_z, n).

    Block (i, k // 2, t, ZS): word (k mod 2) is the z uniform of atom k; words
    2 and 3 make one Box-Muller pair, cosine branch for the even atom of the
    pair and sine branch for the odd one.
    """
    w = philox.block(params.seed, params.problem_id, philox.TAG_ZS, i, k // 2, t)
    u_z = philox.uniform(w[k % 2])
    n_cos, n_sin = philox.box_muller(philox.uniform(w[2]), philox.uniform(w[3]))
    return u_z, (n_cos if k % 2 == 0 else n_sin)


def dict_normal(params, p, k, t):
    """Dictionary draw for positions p of atom k: cosine branch of block (p, k, t, DICT)."""
    w = philox.block(params.seed, params.problem_id, philox.TAG_DICT, p, k, t)
    return philox.box_muller(philox.uniform(w[0]), philox.uniform(w[1]))[0]


def init_normal(params, p, k):
    w = philox.block(params.seed, params.problem_id, philox.TAG_INIT, p, k, 0)
    return philox.box_muller(philox.uniform(w[0]), philox.uniform(w[1]))[0]


# ------------------------------------------------------ conditionals ----

def z_log_odds(ell_k, gamma_s, gamma_eps, delta, rho):
    """ln p(z=1|.) - ln p(z=0|.) with s_ik integrated out.

    delta = sum_{Obs} d_kp^2, rho = sum_{Obs} d_kp e_p where e is the patch
    residual with atom k's own contribution added back.  Integrating
    N(s; 0, 1/gamma_s) against exp(-gamma_eps/2 |e - d s|^2) gives the factor
    sqrt(gamma_s / lam) exp((gamma_eps rho)^2 / (2 lam)), lam = gamma_s + gamma_eps delta.
    Returns (L, lam, q) with q the exponent term.
    """
    lam = gamma_s + gamma_eps * delta
    q = (gamma_eps * rho) ** 2 / (2.0 * lam)
    return ell_k + 0.5 * np.log(gamma_s / lam) + q, lam, q


def s_posterior(gamma_s, gamma_eps, delta, rho):
    """s_ik | z_ik = 1: Gaussian with precision lam and mean gamma_eps rho / lam."""
    lam = gamma_s + gamma_eps * delta
    return gamma_eps * rho / lam, lam


def dict_conditional(P, gamma_eps, A, b):
    """d_kp | rest: precision P + gamma_eps A, mean gamma_eps b / precision.

    A = sum_i m_ip w_ik^2 and b = sum_i m_ip w_ik (x_ip - sum_{j != k} d_jp w_ij).
    """
    lam = P + gamma_eps * A
    return gamma_eps * b / lam, lam


def logit_uniform(u):
    return np.log(u) - np.log1p(-u)


# ------------------------------------------------------------- steps ----

def init_state(params, N, P):
    """Prior draw of D (d_kp = n / sqrt(P)), no active atoms, pi_k at its prior mean."""
    K = params.K
    p = np.arange(P, dtype=np.uint64)
    D = np.stack([init_normal(params, p, k) for k in range(K)]) / math.sqrt(P)
    ell0 = math.log(params.a / K) - math.log(params.b * (K - 1) / K) if K > 1 else 0.0
    return State(D=D, W=np.zeros((N, K)), Z=np.zeros((N, K), dtype=bool),
                 ell=np.full(K, ell0), gamma_s=float(params.gamma_s0),
                 gamma_eps=float(params.gamma_eps0), t=1)


def residual(X, Mk, D, W):
    """r_ip = m_ip (x_ip - sum_k d_kp w_ik): zero at unobserved entries."""
    return Mk * (X - W @ D)


def sweep(params, X, Mk, st, follow_z=None, tie_tol=1e-4, patch_ids=None):
    """Step 1: z/s sweep.  Patches are independent; atoms go in ascending order.

    patch_ids: the grid index of every row of X (default 0..N-1); a subset of
    the patches can be swept on its own because patches are independent given
    (D, pi, gamma) and each draws from its own Philox counters.

    Follow mode (follow_z given): where the drawn z differs from follow_z at a
    point whose log-odds lie within tie_tol * (1 + |ell_k| + |ln(gs/lam)|/2 + q)
    of the uniform's logit, the follow value is adopted and the site recorded
    as a near-tie; any other difference is recorded as a hard mismatch (and the
    oracle keeps its own draw).
    Returns (W, Z, residual after the sweep, report).
    """
    N, K = st.W.shape
    W = st.W.copy()
    Z = st.Z.copy()
    R = residual(X, Mk, st.D, W)
    Mf = Mk.astype(np.float64)
    gs, ge = st.gamma_s, st.gamma_eps
    rep = SweepReport()
    ii = np.arange(N, dtype=np.uint64) if patch_ids is None else np.asarray(patch_ids, np.uint64)
    for k in range(K):
        dk = st.D[k]
        w_old = W[:, k]
        delta = Mf @ (dk * dk)
        rho = R @ dk + delta * w_old
        L, lam, q = z_log_odds(st.ell[k], gs, ge, delta, rho)
        u_z, n = zs_uniforms(params, ii, k, st.t)
        lu = logit_uniform(u_z)
        z = lu < L
        if follow_z is not None:
            fz = follow_z[:, k].astype(bool)
            diff = np.nonzero(z != fz)[0]
            if diff.size:
                scale = 1.0 + abs(st.ell[k]) + np.abs(0.5 * np.log(gs / lam[diff])) + q[diff]
                tie = np.abs(lu[diff] - L[diff]) <= tie_tol * scale
                for i in diff[tie]:
                    rep.tie_sites.append((int(i), k))
                for i in diff[~tie]:
                    rep.hard_sites.append((int(i), k))
                rep.near_ties += int(tie.sum())
                rep.hard_mismatches += int((~tie).sum())
                z[diff[tie]] = fz[diff[tie]]
        mean, lam_s = s_posterior(gs, ge, delta, rho)
        w_new = np.where(z, mean + n / np.sqrt(lam_s), 0.0)
        dw = w_new - w_old
        rows = np.nonzero(dw)[0]
        if rows.size:
            R[rows] -= Mf[rows] * (dw[rows, None] * dk[None, :])
        W[:, k] = w_new
        Z[:, k] = z
    return W, Z, R, rep


def dictionary_update(params, Mk, st, W, R, positions=None, prior_P=None, scale=1.0):
    """Step 2: atoms in order; every position p of d_k from its conditional.

    R is the residual of the current dictionary and W; both the returned D and
    the residual reflect the new atoms.  Positions are independent given W, so
    the columns of a subset of positions can be updated on their own: pass the
    column subsets of Mk, R and st.D, their position indices and the full
    patch dimension P (the prior precision).  scale multiplies the data
    statistics A and b (a mini-batch step's N / n_b); the prior is not scaled.
    """
    K, P = st.D.shape
    D = st.D.copy()
    R = R.copy()
    Mf = Mk.astype(np.float64)
    ge = st.gamma_eps
    pp = np.arange(P, dtype=np.uint64) if positions is None else np.asarray(positions, np.uint64)
    P = P if prior_P is None else prior_P
    for k in range(K):
        w = W[:, k]
        rows = np.nonzero(w)[0]
        mw = Mf[rows] * w[rows, None]                       # m_ip w_ik
        A = scale * (mw * w[rows, None]).sum(axis=0)
        b = scale * (mw * (R[rows] + D[k][None, :] * w[rows, None])).sum(axis=0)
        mean, lam = dict_conditional(P, ge, A, b)
        d_new = mean + dict_normal(params, pp, k, st.t) / np.sqrt(lam)
        R[rows] -= mw * (d_new - D[k])[None, :]
        D[k] = d_new
    return D, R


def pi_update(params, Z, t, scale=1.0):
    """Step 3: pi_k | Z ~ Beta(a/K + n_k, b(K-1)/K + N - n_k), kept as its logit.

    With scale s (a mini-batch step over the N rows of Z) the counts are
    s n_k and s N: the Beta conditional given s copies of the batch."""
    N, K = Z.shape
    nk = Z.sum(axis=0)
    ell = np.empty(K)
    for k in range(K):
        la = _gamma.log_gamma_draw(params.a / K + scale * nk[k], params.seed, params.problem_id,
                                   philox.TAG_PI_A, k, t)
        lb = _gamma.log_gamma_draw(params.b * (K - 1) / K + scale * N - scale * nk[k], params.seed,
                                   params.problem_id, philox.TAG_PI_B, k, t)
        ell[k] = la - lb
    return ell


def gamma_s_update(params, Z, W, t, scale=1.0):
    """Step 4: gamma_s ~ Ga(c + sum(z)/2, d + sum(w^2)/2) over active weights
    (both sums multiplied by scale in a mini-batch step)."""
    shape = params.c + 0.5 * (scale * float(Z.sum()))
    rate = params.d + 0.5 * (scale * float((W * W).sum()))
    lg = _gamma.log_gamma_draw(shape, params.seed, params.problem_id, philox.TAG_GS, 0, t)
    return math.exp(lg) / rate


def gamma_eps_update(params, Mk, R, t, scale=1.0):
    """Step 5: gamma_eps ~ Ga(e + |Obs|/2, f + sum_{Obs} r^2 / 2) (both sums
    multiplied by scale in a mini-batch step)."""
    shape = params.e + 0.5 * (scale * float(Mk.sum()))
    rate = params.f + 0.5 * (scale * float((R * R).sum()))
    lg = _gamma.log_gamma_draw(shape, params.seed, params.problem_id, philox.TAG_GE, 0, t)
    return math.exp(lg) / rate


def iterate(params, X, Mk, st, learn_dict=True, follow_z=None, tie_tol=1e-4):
    """One Gibbs iteration (steps 1-6).  Returns (new state, sweep report)."""
    W, Z, R, rep = sweep(params, X, Mk, st, follow_z=follow_z, tie_tol=tie_tol)
    D = st.D
    if learn_dict:
        D, R = dictionary_update(params, Mk, st, W, R)
    ell = pi_update(params, Z, st.t)
    gs = gamma_s_update(params, Z, W, st.t)
    ge = gamma_eps_update(params, Mk, R, st.t)
    return State(D=D, W=W, Z=Z, ell=ell, gamma_s=gs, gamma_eps=ge, t=st.t + 1), rep


def batch_rows(N, n_batches, batch):
    """Patches of mini-batch `batch`: every patch i with i mod n_batches == batch."""
    return np.arange(batch, N, n_batches)


def minibatch_step(params, X, Mk, st, n_batches, batch, learn_dict=True, follow_z=None,
                   tie_tol=1e-4):
    """One mini-batch step, iteration number st.t: the sweep visits the n_b
    patches of `batch` only (the others keep their codes), then the dictionary,
    pi, gamma_s and gamma_eps are drawn from the conditionals given the batch
    with its statistics scaled by s = N / n_b.  follow_z (N x K) is consulted
    on the batch's rows.  Returns (new state, sweep report of the batch)."""
    N = X.shape[0]
    rows = batch_rows(N, n_batches, batch)
    scale = N / rows.size
    sub = State(D=st.D, W=st.W[rows], Z=st.Z[rows], ell=st.ell, gamma_s=st.gamma_s,
                gamma_eps=st.gamma_eps, t=st.t)
    fz = None if follow_z is None else np.asarray(follow_z)[rows]
    Wb, Zb, Rb, rep = sweep(params, X[rows], Mk[rows], sub, follow_z=fz, tie_tol=tie_tol,
                            patch_ids=rows)
    D = st.D
    if learn_dict:
        D, Rb = dictionary_update(params, Mk[rows], sub, Wb, Rb, scale=scale)
    ell = pi_update(params, Zb, st.t, scale=scale)
    gs = gamma_s_update(params, Zb, Wb, st.t, scale=scale)
    ge = gamma_eps_update(params, Mk[rows], Rb, st.t, scale=scale)
    W = st.W.copy()
    Z = st.Z.copy()
    W[rows] = Wb
    Z[rows] = Zb
    return State(D=D, W=W, Z=Z, ell=ell, gamma_s=gs, gamma_eps=ge, t=st.t + 1), rep


def epochs(params, X, Mk, st, n_epochs, n_batches, learn_dict=True):
    """n_epochs passes over all patches, each the n_batches mini-batch steps in
    ascending batch order (n_epochs * n_batches iteration numbers)."""
    for _ in range(n_epochs):
        for b in range(n_batches):
            st, _ = minibatch_step(params, X, Mk, st, n_batches, b, learn_dict=learn_dict)
    return st


def reconstruct(st, shape, patch, stride):
    """Overlap average of the patch models D^T w_i (last Gibbs sample)."""
    from . import patches
    return patches.overlap_average(st.W @ st.D, shape, patch, stride)


def posterior_mean(states, shape, patch, stride):
    """Posterior-mean reconstruction: the average over the kept Gibbs samples
    (those after burn-in, in any order) of each sample's overlap-averaged
    reconstruction -- the Monte Carlo estimate of E[x | y] from the sampler
    of the BPFA section (reading: the paper names averaging samples for
    frame interpolation of N-D data but gives no estimator; this is the plain
    sample mean)."""
    states = list(states)
    if not states:
        raise ValueError("posterior mean of no samples")
    acc = np.zeros(shape, dtype=np.float64)
    for st in states:
        acc += reconstruct(st, shape, patch, stride)
    return acc / len(states)


def posterior_variance(states, shape, patch, stride):
    """Per-pixel unbiased sample variance of the kept samples' reconstructions,
    (1 / (n - 1)) sum_s (x_s - mean)^2 -- the spread that on-the-fly targeted
    signal selection (Feature summary) can steer acquisition by (reading:
    the paper names strategic selection without a criterion)."""
    states = list(states)
    if len(states) < 2:
        raise ValueError("posterior variance needs at least two samples")
    mean = posterior_mean(states, shape, patch, stride)
    acc = np.zeros(shape, dtype=np.float64)
    for st in states:
        acc += (reconstruct(st, shape, patch, stride) - mean) ** 2
    return acc / (len(states) - 1)
