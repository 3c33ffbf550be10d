"""Benchmark: BPFA blind-inpainting frames on one MI355X.

One step = one full reconstruction of a 512 x 512 STEM-like frame (hexagonal
lattice, period 8 px, 5% vacancies, Poisson 100 e-/px, 10% sampled pixels,
10 x 10 patches at stride 1 = 253,009 patches, K = 128 atoms): restart the
sampler from its prior, build the patch index of the frame (inputs already in
HBM), 20 Gibbs iterations (z/s sweep, dictionary update, pi / gamma draws),
overlap-averaged reconstruction into HBM.

value = patch-atom Gibbs updates per second over the whole step,
N * K * 20 / (seconds per frame); frames/s is reported beside it.
The roofline object describes the kernel that takes the most time per frame
(the z/s sweep on the 512 x 512 frame, the dictionary-statistics kernel on
the 1024 x 1024 frame and the video); `kernels` holds the roofline of both.
Their durations come from HIP events the library records around each launch
on the handle's stream during the timed region.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz = one full-rate 32-bit lane op
# per lane per clock; quarter-rate ops (transcendentals, 32x32->64 products) cost 4.
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12
# The statistics kernel adds 64-bit fixed-point terms into LDS accumulators:
# one LDS atomic add of 8 bytes per term.  A CU's LDS moves 128 bytes per
# clock, so at most 16 such adds per CU per clock: 256 x 16 x 2.4 GHz.
PEAK_LDS_ADDS64 = 256 * 16 * 2.4e9


def sweep_ops_per_update(obs_per_patch):
    """Algorithmic lane-op cost of one patch-atom update.

    Philox4x32-10, one block per two updates: 10 rounds x (2 wide products at
    4 + 2 three-way xors) = 100 -> 50.  Uniform transforms: 4.  Box-Muller per
    two updates: log, sqrt, sin, cos (4 x 4) + 3 -> 10.  z and s: rsqrt, exp
    (2 x 4) + 12.  Dot products and residual update: 3 FMAs per observed pixel.
    """
    return 50.0 + 4.0 + 10.0 + 20.0 + 3.0 * obs_per_patch


def stats_terms(n_active, n_obs):
    """Algorithmic 64-bit accumulations of one dictionary-statistics launch:
    every observed pixel of patch i (a visit) adds the n_a (n_a + 1) / 2
    products w_j w_k (j <= k) of the patch's active atoms to C_p, its n_a
    products w_k x_ip to B_p and x_ip^2 to the residual sum."""
    import numpy as np
    na = np.asarray(n_active, np.float64)
    return float(np.sum(np.asarray(n_obs, np.float64) * (na * (na + 1) / 2 + na + 1)))


def kernel_source_hash(names=("kernels_sweep.hip", "internal.hpp", "philox.hpp")):
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2311_15061_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


STATS_SOURCES = ("kernels_dict.hip", "internal.hpp")


def measured_traffic(workload, kernel="sweep"):
    """HBM bytes per launch of the sweep (or the statistics kernel) from the
    committed rocprofv3 counter summary, or None when it is missing or was
    taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.json" % (kernel, workload))
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    names = STATS_SOURCES if kernel == "stats" else ("kernels_sweep.hip", "internal.hpp", "philox.hpp")
    if rec.get("kernel_source_hash") != kernel_source_hash(names):
        return None
    return rec.get("hbm_bytes_per_launch")


def frame_stats_terms(prob, y_d, m_d, iters):
    """Replays one frame (the timed steps are identical: same prior, frame and
    Philox streams) and returns the statistics kernel's algorithmic terms per
    launch, averaged over the frame's iterations."""
    import numpy as np
    from paper_2311_15061_amd import bpfa
    _, n_obs = prob.patch_index()
    prob.reset_state()
    prob.set_frame(y_d, m_d, reset_codes=True)
    total = 0.0
    for _ in range(iters):
        prob.iterate(1, bpfa.LEARN_DICT)
        Z = prob.get_state()["Z"]
        total += stats_terms(Z.sum(axis=1), n_obs)
    return total / iters


def cpu_baseline(wl, y, m, iters):
    """The binary64 oracle, as it is, on this host: `iters` iterations of the same frame."""
    import numpy as np
    from oracle import bpfa as ob
    from oracle import patches
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = 1
    X, Mk = patches.extract(y, m, wl.patch, wl.stride)
    prm = ob.Params(K=wl.K, seed=wl.method_seed)
    st = ob.init_state(prm, X.shape[0], X.shape[1])
    t0 = time.perf_counter()
    for _ in range(iters):
        st, _ = ob.iterate(prm, X, Mk, st)
    dt = time.perf_counter() - t0
    N = X.shape[0]
    return {"value": N * wl.K * iters / dt, "unit": "updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": "%d Gibbs iteration(s) of the %s frame (%d patches x %d atoms), binary64 "
                      "NumPy oracle, %.1f s; BLAS threads %d, elementwise NumPy on one core"
                      % (iters, wl.name, N, wl.K, dt, threads)}


def serving_run(duration_s=8.0, rate=30.0, n_streams=4, seed=7, saturate_frames=48,
                precision="fp32"):
    """Live-feed serving: Poisson arrivals at `rate` frames/s over `n_streams`
    streams, sizes uniform over 256^2 / 512^2 / 1024^2, sampled fraction
    U[5%, 25%] per frame, K = 128 10 x 10 dictionary learned on a separate
    512^2 frame (20 iterations) and transferred to every stream; 5
    sparse-coding iterations per frame plus a dictionary iteration every 10th
    frame of a stream.  Then a saturation run submits `saturate_frames` at
    once.  Frame contents are drawn from a few seeded lattice images per size
    with a fresh mask per frame.  `precision` is the reconstruction's form
    (binary32 sparse, or BF16 matrix cores with the correction pass)."""
    import numpy as np
    from paper_2311_15061_amd import bpfa, serve
    import synth
    base = synth.workload("stem512")
    rng = np.random.Generator(np.random.PCG64(seed))
    images = {}
    for side in synth.lattice.SERVING_SIZES:
        images[side] = [synth.make_frame(base, data_seed=5000 + side + j, shape=(side, side))[0]
                        for j in range(3)]
    y, m, _ = synth.make_frame(base, data_seed=4242)
    teacher = bpfa.Problem(y.astype(np.float32), m, base.patch, K=base.K, seed=0xD1C7)
    teacher.iterate(20)
    srv = serve.Server(patch=base.patch, K=base.K, n_streams=n_streams, sc_iters=5, dict_every=10,
                       max_slots=2 * n_streams, hbm_budget=64 << 30, seed=0x5E7E, precision=precision)
    for st in range(n_streams):
        srv.set_dictionary(st, teacher)
    teacher.close()

    def make_request():
        side = int(rng.choice(synth.lattice.SERVING_SIZES))
        img = images[side][int(rng.integers(len(images[side])))]
        rho = float(rng.uniform(0.05, 0.25))
        mask = synth.make_mask((side, side), rho, rng)
        return int(rng.integers(n_streams)), side, img, mask

    # warm start: every frame size once per slot pair, so that slot workspaces exist
    for j in range(2 * n_streams):
        side = synth.lattice.SERVING_SIZES[j % len(synth.lattice.SERVING_SIZES)]
        srv.submit(j % n_streams, images[side][0], synth.make_mask((side, side), 0.1, rng))
    srv.drain()
    srv.poll(100000)

    # Poisson arrivals, submitted from this thread at their scheduled times
    t_arr = np.cumsum(rng.exponential(1.0 / rate, size=int(duration_s * rate * 1.5) + 8))
    t_arr = t_arr[t_arr < duration_s]
    reqs = [make_request() for _ in range(len(t_arr))]
    sizes = {}
    t0 = time.perf_counter()
    for when, (st, side, img, mask) in zip(t_arr, reqs):
        delay = t0 + when - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ticket, _ = srv.submit(st, img, mask)
        sizes[ticket] = side
    srv.drain()
    wall = time.perf_counter() - t0
    res = srv.poll(100000)
    lat = {side: [] for side in synth.lattice.SERVING_SIZES}
    for r in res:
        if r["status"] == 0:
            lat[sizes[r["ticket"]]].append(r["latency_ms"])
    out = {"precision": precision, "arrival_rate": rate, "duration_s": duration_s,
           "frames": len(res),
           "failed": sum(1 for r in res if r["status"] != 0),
           "frames_per_s": len(res) / wall, "streams": n_streams}
    for side, v in lat.items():
        if v:
            out["p50_ms_%d" % side] = float(np.percentile(v, 50))
            out["p99_ms_%d" % side] = float(np.percentile(v, 99))
            out["n_%d" % side] = len(v)
    # saturation: everything at once
    reqs = [make_request() for _ in range(saturate_frames)]
    t0 = time.perf_counter()
    for st, side, img, mask in reqs:
        srv.submit(st, img, mask)
    srv.drain()
    out["saturated_frames_per_s"] = saturate_frames / (time.perf_counter() - t0)
    srv.poll(100000)
    out["slot_stats"] = srv.stats()
    srv.close()
    return out


def isolated_latency(frames=20, precision="fp32"):
    """Per-frame latency with nothing else in flight: one stream, one frame at a
    time (submit, wait for its result), for every serving frame size, with the
    slots' graph replay on and off.  The frame work is the serving leg's (5
    sparse-coding iterations, K = 128, 10 x 10 patches, 10% sampled), from
    submission to the reconstruction in host memory; two warm-up frames per
    size let each slot capture its graph first."""
    import numpy as np
    from paper_2311_15061_amd import bpfa, serve
    import synth
    base = synth.workload("stem512")
    out = {}
    for graphs in (True, False):
        srv = serve.Server(patch=base.patch, K=base.K, n_streams=1, sc_iters=5, dict_every=0,
                           max_slots=3, hbm_budget=64 << 30, seed=0x15, precision=precision,
                           use_graphs=graphs)
        for side in synth.lattice.SERVING_SIZES:
            y, _, _ = synth.make_frame(base, data_seed=6000 + side, shape=(side, side))
            rng = np.random.Generator(np.random.PCG64(side))
            lat = []
            for f in range(frames + 2):
                m = synth.make_mask((side, side), 0.10, rng)
                srv.submit(0, y, m)
                srv.drain()
                r = srv.poll(10)
                assert r and r[0]["status"] == 0, r
                if f >= 2:
                    lat.append(r[0]["latency_ms"])
            key = "%s_%d" % ("graph" if graphs else "direct", side)
            out[key + "_p50_ms"] = float(np.percentile(lat, 50))
            out[key + "_p99_ms"] = float(np.percentile(lat, 99))
        st = srv.stats()
        out[("graph" if graphs else "direct") + "_replayed_frames"] = st["graph_frames"]
        srv.close()
    return out


def time_to_solution(epochs=2, reps=3, batches=(16,)):
    """Context for the paper's one published timing (Time-to-solution section:
    a greyscale 1024 x 1024 image, a dictionary of 64 atoms of 10 x 10 patches
    trained for two complete epochs, about 4 s on an RTX 3060), in both
    readings of an epoch: one full-batch Gibbs iteration over every patch, and
    a pass of mini-batch steps over a partition into B batches (patch i in
    batch i mod B, each step's statistics scaled by N / n_b).  The frame is the
    1024 x 1024 synthetic lattice with K = 64.  Timed like a user's call, from
    host buffers to the reconstruction in host memory, workspace allocation and
    the patch index included; median of `reps` runs after one warm-up run."""
    import dataclasses
    import statistics
    import numpy as np
    from paper_2311_15061_amd import bpfa
    import synth
    wl = dataclasses.replace(synth.workload("stem1024"), name="stem1024_k64", K=64)
    y, m, _ = synth.make_frame(wl)
    y = np.ascontiguousarray(y, np.float32)
    m = np.ascontiguousarray(m, np.uint8)

    def timed(run):
        times = []
        for r in range(reps + 1):
            t0 = time.perf_counter()
            prob = bpfa.Problem(y, m, wl.patch, wl.stride, K=wl.K, seed=wl.method_seed)
            run(prob)
            xh = prob.reconstruct()
            prob.close()
            if r:
                times.append(time.perf_counter() - t0)
        assert np.all(np.isfinite(xh))
        return statistics.median(times)

    out = {"workload": "1024x1024 lattice, 10x10 patches stride 1, K=64, %d epochs" % epochs,
           "reading": "epoch = one Gibbs iteration over all patches (full batch)",
           "seconds": timed(lambda p: p.iterate(epochs, bpfa.LEARN_DICT)), "runs": reps,
           "paper_seconds": 4.0, "paper_hardware": "NVIDIA RTX 3060 (context only)"}
    for B in batches:
        out["minibatch_%d_seconds" % B] = timed(lambda p: p.epochs(epochs, B))
        out["minibatch_%d_reading" % B] = ("epoch = %d mini-batch steps over patch i in batch i mod %d"
                                           % (B, B))
    return out


def multichannel_run(iters=10):
    """Multi-channel patches on a 512 x 512 x 3 frame (the stem512 lattice in
    three layers of different gain, 10% of each layer sampled): one
    single-channel 10 x 10 x 1 dictionary across the layers, and full-depth
    10 x 10 x 3 patches (N-dimensional inpainting section); ms per Gibbs
    iteration and patch-atom updates per second."""
    import numpy as np
    from paper_2311_15061_amd import bpfa, sampling
    import synth
    wl = synth.workload("stem512")
    y2, _, _ = synth.make_frame(wl)
    y = np.stack([y2 * s for s in (1.0, 0.8, 0.6)], axis=-1).astype(np.float32)
    m = sampling.uniform_mask(y.shape, 0.10, seed=21)
    out = {}
    for name, patch in (("single_channel_10x10x1", (10, 10, 1)), ("full_depth_10x10x3", (10, 10, 3))):
        prob = bpfa.Problem(y, m, patch, (1, 1, 1), K=wl.K, seed=wl.method_seed)
        prob.iterate(2)
        prob.sync()
        t0 = time.perf_counter()
        prob.iterate(iters)
        prob.sync()
        dt = (time.perf_counter() - t0) / iters
        out[name] = {"patches": prob.N, "ms_per_iteration": 1e3 * dt,
                     "updates_per_s": prob.N * prob.K / dt}
        prob.close()
    return out


def targeted_run(burn_in=10, samples=5, more=10):
    """On-the-fly strategic selection on the stem512 frame: 5% of the pixels
    sampled uniformly, `burn_in` iterations, `samples` accumulated samples;
    the mask is then refined to 10% either by posterior-variance-weighted
    draws or uniformly, and the frame continues `more` iterations from the
    kept codes.  PSNR/SSIM of the last sample against the ground truth."""
    import numpy as np
    from paper_2311_15061_amd import bpfa, metrics, sampling
    import synth
    wl = synth.workload("stem512")
    y, _, g = synth.make_frame(wl)
    y = np.ascontiguousarray(y, np.float32)
    base = sampling.uniform_mask(wl.shape, 0.05, seed=31)
    out = {"base_fraction": 0.05, "refined_fraction": 0.10}
    for how in ("targeted", "uniform"):
        prob = bpfa.Problem(y, base, wl.patch, wl.stride, K=wl.K, seed=wl.method_seed)
        prob.iterate(burn_in)
        for _ in range(samples):
            prob.iterate(1)
            prob.mean_accumulate()
        var, _ = prob.posterior_variance()
        if how == "targeted":
            m2 = sampling.targeted_mask(var, 0.10, seed=32, base=base)
        else:
            m2 = sampling.targeted_mask(np.ones(wl.shape), 0.10, seed=32, base=base)
        prob.set_frame(y, m2, reset_codes=False)
        prob.iterate(more)
        x = prob.reconstruct()
        out["psnr_db_" + how] = metrics.psnr(x, g)
        out["ssim_" + how] = metrics.ssim(x, g)
        prob.close()
    return out


def recon_forms(prob, wl, torch, np):
    """The reconstruction's contraction in both precision forms on the handle's
    current state: ms per reconstruction (10 timed after one untimed) and the
    outputs."""
    rec_ms, outs = {}, {}
    for prec in ("fp32", "bf16"):
        prob.set_precision(prec)
        o = torch.empty(wl.shape, dtype=torch.float32, device="cuda")
        prob.reconstruct(o)
        prob.set_timing(True)
        for _ in range(10):
            prob.reconstruct(o)
        rec_ms[prec] = prob.stats()["ms_recon"] / 10
        prob.set_timing(False)
        outs[prec] = o.cpu().numpy().astype(np.float64)
    prob.set_precision("fp32")
    return rec_ms, outs


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="stem512")
    ap.add_argument("--iters", type=int, default=None, help="Gibbs iterations per frame")
    ap.add_argument("--cpu-iters", type=int, default=3, help="oracle iterations timed on the host")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-seconds", type=float, default=8.0)
    ap.add_argument("--no-tts", action="store_true", help="skip the paper's time-to-solution context run")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the multi-channel and targeted-selection runs")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving leg (binary32 form): print its JSON and exit")
    ap.add_argument("--saturate-frames", type=int, default=48,
                    help="frames of the serving leg's saturation burst")
    ap.add_argument("--timed-only", action="store_true",
                    help="only the timed frames and the reconstruction in both precision forms "
                         "(for profiler runs): no roofline work count, posterior-mean, quality or "
                         "extra legs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES three times (the "
                         "reference kernel that scales the HBM byte counters) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2311_15061_amd import bpfa
    from paper_2311_15061_amd import metrics
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "copies": 3}), flush=True)
        return
    if args.serving_only:
        print(json.dumps(serving_run(duration_s=args.serving_seconds,
                                     saturate_frames=args.saturate_frames)), flush=True)
        return
    wl = synth.workload(args.workload)
    iters = args.iters or wl.iters
    y, m, g = synth.make_frame(wl)
    y_d = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    m_d = torch.from_numpy(np.ascontiguousarray(m, np.uint8)).cuda()
    out_d = torch.empty(wl.shape, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    prob = bpfa.Problem(y_d, m_d, wl.patch, wl.stride, K=wl.K, seed=wl.method_seed,
                        stream=stream.cuda_stream)
    N, K = prob.N, prob.K

    def step():
        prob.reset_state()
        prob.set_frame(y_d, m_d, reset_codes=True)
        prob.iterate(iters, bpfa.LEARN_DICT)
        prob.reconstruct(out_d)

    # the first frame on fresh caches and allocations, timed on its own (warm-up)
    first_ms = None
    for w in range(args.warmup):
        t_w = time.perf_counter()
        step()
        if w == 0:
            prob.sync()
            first_ms = 1e3 * (time.perf_counter() - t_w)
    prob.sync()
    prob.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = prob.stats()
    prob.set_timing(False)
    # after the timed region: the spread of single frames, each run alone
    # (synchronised) and timed on the host
    frame_ms = []
    for _ in range(args.steps):
        t_f = time.perf_counter()
        step()
        prob.sync()
        frame_ms.append(1e3 * (time.perf_counter() - t_f))
    frame_ms.sort()

    ms_step = 1e3 * elapsed / args.steps
    updates = float(N) * K * iters
    value = updates * args.steps / elapsed
    sweep_ms = st["ms_sweep"] / max(st["n_sweeps"], 1)
    obs_per_patch = st["n_obs"] / N
    ops = N * K * sweep_ops_per_update(obs_per_patch)
    achieved = ops / (sweep_ms * 1e-3)
    traffic = measured_traffic(args.workload)

    res = {
        "metric": "patch-atom Gibbs updates/sec + frames/sec, p99 frame latency at 512^2",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": wl.name, "shape": list(wl.shape), "patch": list(wl.patch),
                   "stride": list(wl.stride), "K": K, "patches": N, "sampled_fraction": wl.rho,
                   "gibbs_iters_per_frame": iters, "parallelism": "single GPU"},
        "frames_per_s": args.steps / elapsed,
        "frame_ms_alone": {"median": frame_ms[len(frame_ms) // 2], "min": frame_ms[0],
                           "max": frame_ms[-1], "frames": len(frame_ms),
                           "first_frame_cold": first_ms},
        "phase_ms_per_frame": {
            "index": st["ms_index"] / args.steps, "sweep": st["ms_sweep"] / args.steps,
            "dictionary": st["ms_dict"] / args.steps, "scalars": st["ms_scalars"] / args.steps,
            "reconstruct": st["ms_recon"] / args.steps},
        "sweep_updates_per_s": N * K / (sweep_ms * 1e-3),
        "mean_active_atoms": st["mean_active"],
        "phase_ms_per_frame_dict_stats": st["ms_dict_stats"] / args.steps,
    }
    stats_ms = st["ms_dict_stats"] / max(st["n_sweeps"], 1)
    if args.timed_only:
        res["kernels"] = {"sweep_kernel": {"ms_per_launch": sweep_ms},
                          "dict_stats_kernel": {"ms_per_launch": stats_ms}}
        res["reconstruct_ms"], _ = recon_forms(prob, wl, torch, np)
        prob.close()
        print(json.dumps(res), flush=True)
        return
    terms = frame_stats_terms(prob, y_d, m_d, iters)
    lds_achieved = terms / (stats_ms * 1e-3)
    kernels = {
        "sweep_kernel": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                         "unit": "TOP/s", "frac": achieved / PEAK_LANE_OPS, "traffic": traffic,
                         "ms_per_launch": sweep_ms, "ms_per_frame": st["ms_sweep"] / args.steps,
                         "ops_per_update": sweep_ops_per_update(obs_per_patch),
                         "kernel_source_hash": kernel_source_hash()},
        "dict_stats_kernel": {"bound": "lds", "achieved": lds_achieved / 1e12,
                              "peak": PEAK_LDS_ADDS64 / 1e12, "unit": "T 64-bit LDS adds/s",
                              "frac": lds_achieved / PEAK_LDS_ADDS64,
                              "traffic": measured_traffic(args.workload, "stats"),
                              "ms_per_launch": stats_ms,
                              "ms_per_frame": st["ms_dict_stats"] / args.steps,
                              "terms_per_launch": terms,
                              "kernel_source_hash": kernel_source_hash(STATS_SOURCES)},
    }
    dominant = max(kernels, key=lambda k: kernels[k]["ms_per_frame"])
    res["roofline"] = dict(kernel=dominant, **kernels[dominant])
    res["kernels"] = kernels
    res["reconstruct_ms"], outs = recon_forms(prob, wl, torch, np)
    # posterior mean over the last half of a frame's iterations (after burn-in)
    prob.reset_state()
    prob.set_frame(y_d, m_d, reset_codes=True)
    prob.iterate(iters - iters // 2, bpfa.LEARN_DICT)
    for _ in range(iters // 2):
        prob.iterate(1, bpfa.LEARN_DICT)
        prob.mean_accumulate()
    pm, n_kept = prob.posterior_mean()          # host copy: synchronises the handle's stream
    # cost of one accumulation (a reconstruction plus the binary64 add), 20 in a row
    prob.sync()
    t_acc = time.perf_counter()
    for _ in range(20):
        prob.mean_accumulate()
    prob.sync()
    acc_ms = 1e3 * (time.perf_counter() - t_acc) / 20
    prob.mean_reset()
    res["posterior_mean"] = {"samples": n_kept, "burn_in": iters - iters // 2,
                             "accumulate_ms": acc_ms}
    if not args.no_quality:
        res["posterior_mean"]["psnr_db"] = metrics.psnr(pm, g)
        res["posterior_mean"]["ssim"] = metrics.ssim(pm, g)
    if not args.no_quality:
        x = out_d.cpu().numpy()
        res["psnr_db"] = metrics.psnr(x, g)
        res["ssim"] = metrics.ssim(x, g)
        res["psnr_db_bf16"] = metrics.psnr(outs["bf16"], g)
        res["bf16_vs_fp32_rel_err"] = float(np.linalg.norm(outs["bf16"] - outs["fp32"]) /
                                            np.linalg.norm(outs["fp32"]))
    if not args.no_serving:
        # both reconstruction forms under the same arrival sequence; the
        # faster binary32 form is the server's default and the headline p99
        sv = serving_run(duration_s=args.serving_seconds, precision="fp32",
                         saturate_frames=args.saturate_frames)
        res["serving"] = sv
        res["serving_bf16"] = serving_run(duration_s=args.serving_seconds, precision="bf16",
                                          saturate_frames=args.saturate_frames)
        res["p99_frame_latency_ms_512"] = sv.get("p99_ms_512")
        res["serving_isolated_latency"] = isolated_latency()
    if not args.no_tts:
        res["paper_time_to_solution"] = time_to_solution()
    if not args.no_extras:
        res["multichannel"] = multichannel_run()
        res["targeted_selection"] = targeted_run()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, y, m, args.cpu_iters)
    prob.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
