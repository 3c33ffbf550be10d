"""Lattice images, masks and the named workloads.

Recipe (per frame):
  1. atom sites on a square or hexagonal lattice covering the image plus a
     3-sigma margin, offset by half a period; each site is dropped with the
     vacancy probability; amplitudes A ~ U[0.5, 1];
  2. clean image I = sum_sites A exp(-|q - r|^2 / (2 sigma^2)) (+ background),
     scaled so that max I = 1;
  3. counts ~ Poisson(dose * I); data y = counts / max(counts), and the ground
     truth g = dose * I / max(counts) on the same scale;
  4. mask: exactly round(rho * M) sampled pixels, uniform without replacement
     (per frame for videos), 1 = sampled.
All randomness comes from numpy's PCG64 with the seed given.
"""
import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    shape: tuple
    patch: tuple
    stride: tuple
    K: int
    iters: int
    rho: float
    lattice: str            # "square" or "hex"
    period: float
    sigma: float
    dose: float
    vacancy: float = 0.0
    ramp: float = 0.0       # linear background along the diagonal, fraction of peak
    drift: float = 0.0      # px per frame along x (videos: last axis is time)
    flicker: float = 0.0    # per-frame multiplicative N(0, flicker) intensity jitter
    fp64_input: bool = False
    data_seed: int = 1000
    method_seed: int = 0xB1FA0000


WORKLOADS = {
    "lattice64": Workload("lattice64", (64, 64), (8, 8), (1, 1), K=32, iters=10, rho=0.25,
                          lattice="square", period=6.0, sigma=1.5, dose=200.0,
                          fp64_input=True, data_seed=1001, method_seed=0xB1FA0001),
    "stem512": Workload("stem512", (512, 512), (10, 10), (1, 1), K=128, iters=20, rho=0.10,
                        lattice="hex", period=8.0, sigma=2.0, dose=100.0, vacancy=0.05,
                        data_seed=1002, method_seed=0xB1FA0002),
    "stem1024": Workload("stem1024", (1024, 1024), (10, 10), (1, 1), K=256, iters=20, rho=0.10,
                         lattice="hex", period=8.0, sigma=2.0, dose=50.0, vacancy=0.05,
                         ramp=0.3, data_seed=1003, method_seed=0xB1FA0003),
    "video256": Workload("video256", (256, 256, 64), (8, 8, 4), (1, 1, 2), K=192, iters=15,
                         rho=0.15, lattice="hex", period=8.0, sigma=2.0, dose=100.0,
                         vacancy=0.05, drift=0.3, flicker=0.05, data_seed=1004,
                         method_seed=0xB1FA0004),
}

SERVING_SIZES = (256, 512, 1024)


def workload(name):
    return WORKLOADS[name]


def _sites(h, w, lattice, period, sigma, rng, vacancy):
    margin = 3.0 * sigma + period
    if lattice == "square":
        ys = np.arange(-margin, h + margin, period) + period / 2
        xs = np.arange(-margin, w + margin, period) + period / 2
        yy, xx = np.meshgrid(ys, xs, indexing="ij")
    elif lattice == "hex":
        rows = np.arange(-margin, h + margin, period * math.sqrt(3) / 2)
        pts = []
        for j, y in enumerate(rows):
            x0 = -margin + (period / 2 if j % 2 else 0.0) + period / 2
            xs = np.arange(x0, w + margin, period)
            pts.append(np.stack([np.full_like(xs, y + period / 2), xs], 1))
        p = np.concatenate(pts)
        yy, xx = p[:, 0], p[:, 1]
    else:
        raise ValueError(lattice)
    yy, xx = np.ravel(yy), np.ravel(xx)
    keep = rng.random(yy.size) >= vacancy
    amp = rng.uniform(0.5, 1.0, size=yy.size)
    return yy[keep], xx[keep], amp[keep]


def _render(h, w, yy, xx, amp, sigma, dx=0.0):
    img = np.zeros((h, w))
    rad = int(math.ceil(4 * sigma))
    off = np.arange(-rad, rad + 1)
    xs = xx + dx
    cy = np.rint(yy).astype(np.int64)
    cx = np.rint(xs).astype(np.int64)
    py = cy[:, None] + off[None, :]                  # sites x window
    px = cx[:, None] + off[None, :]
    gy = np.exp(-(py - yy[:, None]) ** 2 / (2 * sigma ** 2)) * amp[:, None]
    gx = np.exp(-(px - xs[:, None]) ** 2 / (2 * sigma ** 2))
    vy = (py >= 0) & (py < h)
    vx = (px >= 0) & (px < w)
    for a in range(off.size):
        for b in range(off.size):
            m = vy[:, a] & vx[:, b]
            np.add.at(img, (py[m, a], px[m, b]), gy[m, a] * gx[m, b])
    return img


def make_mask(shape, rho, rng, per_frame_last_axis=False):
    """Exactly round(rho * M) sampled pixels (per frame along the last axis if asked)."""
    shape = tuple(shape)
    if per_frame_last_axis:
        frame = int(np.prod(shape[:-1]))
        m = np.zeros((shape[-1], frame), dtype=np.uint8)
        for f in range(shape[-1]):
            m[f, rng.choice(frame, size=int(round(rho * frame)), replace=False)] = 1
        return np.ascontiguousarray(np.moveaxis(m.reshape((shape[-1],) + shape[:-1]), 0, -1))
    total = int(np.prod(shape))
    m = np.zeros(total, dtype=np.uint8)
    m[rng.choice(total, size=int(round(rho * total)), replace=False)] = 1
    return m.reshape(shape)


def _poisson_normalise(clean, dose, rng):
    clean = clean / clean.max()
    counts = rng.poisson(dose * clean).astype(np.float64)
    top = counts.max()
    return counts / top, dose * clean / top


def make_frame(wl, data_seed=None, shape=None, rho=None):
    """(y, mask, ground_truth) for a workload; y is float64 or float32 per the workload."""
    if isinstance(wl, str):
        wl = WORKLOADS[wl]
    rng = np.random.Generator(np.random.PCG64(wl.data_seed if data_seed is None else data_seed))
    shape = tuple(wl.shape if shape is None else shape)
    rho = wl.rho if rho is None else rho
    if len(shape) == 2:
        h, w = shape
        yy, xx, amp = _sites(h, w, wl.lattice, wl.period, wl.sigma, rng, wl.vacancy)
        clean = _render(h, w, yy, xx, amp, wl.sigma)
        if wl.ramp:
            q = (np.arange(h)[:, None] + np.arange(w)[None, :]) / (h + w - 2)
            clean = clean + wl.ramp * clean.max() * q
        y, g = _poisson_normalise(clean, wl.dose, rng)
        mask = make_mask(shape, rho, rng)
    elif len(shape) == 3:
        h, w, nf = shape
        yy, xx, amp = _sites(h, w, wl.lattice, wl.period, wl.sigma, rng,
                             wl.vacancy)
        frames = []
        for f in range(nf):
            fr = _render(h, w, yy, xx, amp, wl.sigma, dx=wl.drift * f)
            frames.append(fr * (1.0 + wl.flicker * rng.standard_normal()))
        clean = np.stack(frames, axis=-1)
        y, g = _poisson_normalise(clean, wl.dose, rng)
        mask = make_mask(shape, rho, rng, per_frame_last_axis=True)
    else:
        raise ValueError("generators cover 2-D images and 2-D + time videos")
    dtype = np.float64 if wl.fp64_input else np.float32
    return y.astype(dtype), mask, g


def make_serving_frame(rng):
    """One live-feed frame: size uniform over 256^2 / 512^2 / 1024^2, rho ~ U[0.05, 0.25]."""
    base = WORKLOADS["stem512"]
    side = int(rng.choice(SERVING_SIZES))
    rho = float(rng.uniform(0.05, 0.25))
    seed = int(rng.integers(0, 2 ** 31))
    y, mask, g = make_frame(base, data_seed=seed, shape=(side, side), rho=rho)
    return y, mask, g, rho
