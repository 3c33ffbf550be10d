/*
 * bpfa_serve.h -- live-feed serving on top of libbpfa.
 *
 * The paper's abstract and introduction describe frame-by-frame
 * reconstruction of a time-variable feed, and its feature summary lists
 * multiple simultaneous problems and dictionary transfer between sources.
 * A server holds one dictionary state (D, logit pi, gamma_s, gamma_eps and the
 * Philox iteration counter) per feed stream, resident on the device, and
 * reconstructs submitted frames of any 1..4-D shape: each frame starts with
 * zero codes and the stream's state, runs `sc_iters` sparse-coding iterations
 * (plus one dictionary-learning iteration on every `dict_every`-th frame of the
 * stream), writes the overlap-averaged reconstruction and carries the updated
 * state back to its stream.  Frames of one stream run in submission order;
 * frames of different streams overlap on the device (continuous batching):
 * a frame is admitted as soon as a slot for its shape is free and the
 * workspaces fit the HBM budget, and slots of other shapes are freed when idle.
 * Results of a stream do not depend on what else is in flight: every kernel
 * is deterministic and a stream's random numbers depend only on its own
 * counter (problem id = stream index, t continuing across its frames).
 *
 * Each slot replays its frame body (patch index, iterations, state export,
 * reconstruction) from a HIP graph captured on its second frame of a kind
 * (with or without the dictionary iteration); the per-frame plan of the
 * index is built on the device, so one graph serves every frame of the
 * slot's shape, and a frame costs an upload, the state import, one graph
 * launch and the result copy.
 *
 * Threading: submit / poll / stats may be called from any thread; the server
 * runs one dispatcher thread and one worker thread per slot.
 */
#ifndef BPFA_SERVE_H
#define BPFA_SERVE_H

#include "bpfa.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bpfa_server* bpfa_server_t;

typedef struct {
  int32_t ndim;
  int64_t patch[4], stride[4];     /* patch shape B and stride S of every frame */
  int32_t K;
  double a, b, c, d, e, f;         /* priors, as in bpfa_params */
  double gamma_s0, gamma_eps0;
  uint64_t seed;
  int32_t n_streams;               /* feed streams, 1..4096 */
  int32_t sc_iters;                /* sparse-coding iterations per frame (>= 1) */
  int32_t dict_every;              /* dictionary iteration on every n-th frame of a stream; 0 = never */
  int32_t max_slots;               /* frames in flight at most (>= 1) */
  uint64_t hbm_budget;             /* bytes of slot workspaces the server may hold */
  int32_t device;
  int32_t precision;               /* BPFA_FP32 or BPFA_BF16: contraction precision of every slot */
  int32_t use_graphs;              /* 1: replay each slot's frame body from a captured HIP graph
                                      (after one uncaptured frame of each kind); 0: launch directly.
                                      Results are the same either way. */
} bpfa_server_params;

/* Defaults: 2-D 10 x 10 patches stride 1, K = 128, priors as bpfa_params_default,
 * 4 streams, 5 sparse-coding iterations, dictionary every 10 frames, 4 slots,
 * 16 GiB budget, device 0, binary32 reconstruction (BPFA_FP32; the BF16 form
 * is selectable and is slower on these sparse codes), graph replay on. */
void bpfa_server_params_default(bpfa_server_params* p);

/* Start a server.  EINVAL / ESHAPE for bad parameters (ESHAPE also for
 * BPFA_BF16 with patches of more than 256 pixels), EDEVICE on HIP errors. */
bpfa_status bpfa_server_create(const bpfa_server_params* p, bpfa_server_t* out);

/* Dictionary transfer (feature summary) into stream `stream`: copies D,
 * logit pi and the gammas from a problem (same P and K) and resets the
 * stream's frame count; ESHAPE on a size mismatch.  Waits for the stream to
 * be idle. */
bpfa_status bpfa_server_set_dictionary(bpfa_server_t s, int32_t stream, bpfa_t src);

/* Queue one frame of `stream`.  image / mask: host memory, prod(shape)
 * floats / bytes, copied before return.  out: host memory of prod(shape)
 * floats that the caller keeps valid until the ticket is reported by
 * bpfa_server_poll (the reconstruction is written there).  *ticket gets a
 * number increasing with submission.  ESHAPE if the shape is invalid for the
 * server's patch geometry. */
bpfa_status bpfa_server_submit(bpfa_server_t s, int32_t stream, const int64_t* shape,
                               const float* image, const uint8_t* mask, float* out,
                               uint64_t* ticket);

/* A frame that fails (status != BPFA_OK, e.g. ENUMERIC when one of its
 * draws failed) leaves its stream's dictionary state and iteration counter
 * as the last successful frame left them: the next frame of the stream
 * starts from there. */
typedef struct {
  uint64_t ticket;
  int32_t stream;
  int32_t status;        /* bpfa_status of the frame (ENOMEM: larger than the whole budget) */
  int64_t frame_index;   /* index of the frame within its stream */
  int64_t pixels;
  double latency_ms;     /* submission to reconstruction in host memory */
  double queue_ms;       /* submission to admission */
  int32_t learned;       /* 1 if the frame ran a dictionary iteration */
} bpfa_serve_result;

/* Acquisition policies of a stream (Feature summary: pre-determined indexing
 * methods, and on-the-fly strategic selections that improve the
 * reconstruction; the paper gives no rule, these are the library's).  Masks
 * are drawn on the device from Philox4x32-10 under the server's seed with
 * counter (pixel or line, hop, frame index of the stream, 8 | stream << 8);
 * word 0 gives the uniform u = (floor(w / 2^9) + 1/2) 2^-23 and a pixel is
 * acquired when u < p (binary64):
 *   BPFA_ACQ_UNIFORM   p = fraction for every pixel;
 *   BPFA_ACQ_LINE_HOP  each line along the last axis from a random start by
 *                      hops of 1 .. hmax pixels, hmax = max(1,
 *                      floor(2 / fraction + 1/2) - 1): start floor(u hmax)
 *                      (counter (line, 0)), hop j moves floor(u_j hmax) + 1
 *                      (counter (line, j));
 *   BPFA_ACQ_TARGETED  p_q = min(1, (1 - s) f + s f M v_q / sum v) with f the
 *                      fraction, s = targeted_share, M the pixel count and v
 *                      the per-pixel posterior variance of the last
 *                      var_samples samples of the stream's previous frame
 *                      (the uniform rule when the stream has no variance of
 *                      this shape yet, or sum v = 0).
 * BPFA_ACQ_CALLER (the default) takes the caller's masks only. */
enum { BPFA_ACQ_CALLER = 0, BPFA_ACQ_UNIFORM = 1, BPFA_ACQ_LINE_HOP = 2, BPFA_ACQ_TARGETED = 3 };

typedef struct {
  int32_t kind;            /* BPFA_ACQ_* */
  int32_t var_samples;     /* TARGETED: the last 2 .. (sc_iters + 1) samples of a frame whose
                              spread steers the next frame */
  double fraction;         /* expected acquired fraction, (0, 1] */
  double targeted_share;   /* TARGETED: share of the expected acquisitions placed by v, [0, 1] */
} bpfa_acq_policy;

/* Set stream `stream`'s policy (waits for the stream to be idle; a new
 * policy forgets the stream's variance).  EINVAL for a bad stream, kind,
 * fraction, share or sample count. */
bpfa_status bpfa_server_set_policy(bpfa_server_t s, int32_t stream, const bpfa_acq_policy* policy);

/* Queue one frame of a stream whose policy is not BPFA_ACQ_CALLER: `scene`
 * (host, prod(shape) floats, copied before return) is what the instrument
 * would see; the server acquires the pixels its policy draws for this frame
 * and reconstructs from those only.  out as for bpfa_server_submit; mask_out,
 * if not NULL, receives the frame's mask (prod(shape) bytes, 1 = acquired;
 * valid when the ticket is reported).  EINVAL for a stream without a policy. */
bpfa_status bpfa_server_submit_scene(bpfa_server_t s, int32_t stream, const int64_t* shape,
                                     const float* scene, float* out, uint8_t* mask_out,
                                     uint64_t* ticket);

/* The mask the policy gives frame `frame` of stream `stream` under `seed`
 * (the server's rule, computed on the device `device`): ndim / shape as for a
 * frame, weights the variance v for BPFA_ACQ_TARGETED (NULL: the uniform
 * rule), mask prod(shape) bytes; weights and mask of kind `mem`.
 * Synchronises.  EINVAL for a bad policy. */
bpfa_status bpfa_acquire_mask(const bpfa_acq_policy* policy, int32_t ndim, const int64_t* shape,
                              const float* weights, uint64_t seed, int32_t stream, int64_t frame,
                              uint8_t* mask, bpfa_mem mem, int32_t device);

/* Completed frames since the last poll, oldest first; at most `max`.  */
bpfa_status bpfa_server_poll(bpfa_server_t s, bpfa_serve_result* results, int32_t max,
                             int32_t* n);

/* Block until every submitted frame has completed. */
bpfa_status bpfa_server_drain(bpfa_server_t s);

typedef struct {
  int64_t submitted, completed, failed;
  int64_t in_flight, queued;
  int64_t slots, slot_bytes;       /* live slots and their workspace bytes */
  int64_t peak_slot_bytes;
  int64_t slot_creations, slot_evictions;
  int64_t graph_frames;            /* frames whose body was replayed from a captured graph */
  int64_t graph_captures;          /* graphs captured (one per slot and kind of frame) */
} bpfa_serve_stats;

bpfa_status bpfa_server_stats(bpfa_server_t s, bpfa_serve_stats* st);

/* Stop the threads (after draining) and free every device resource. */
void bpfa_server_destroy(bpfa_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* BPFA_SERVE_H */
