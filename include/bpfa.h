/*
 * bpfa.h -- C ABI of libbpfa: Beta-Process Factor Analysis (BPFA) blind
 * inpainting of subsampled N-D data on one AMD Instinct MI355X (gfx950).
 *
 * What is computed comes from the paper "SenseAI: Real-Time Inpainting for
 * Electron Microscopy": its BPFA section (a beta-process prior over a
 * dictionary; each iteration performs a dictionary-learning step and a
 * sparse-coding step; dictionary and sparse weights are learned from the
 * subsampled input alone), its N-dimensional inpainting section (an image of
 * shape M cut into patches of shape B in any number of dimensions), and its
 * feature summary (multiple simultaneous problems, dictionary transfer
 * between sources).  The model equations are those of the BPFA works the
 * paper cites (Paisley & Carin 2009; Zhou et al. 2009), finite-K form:
 *
 *   x_ip ~ N(sum_k d_kp z_ik s_ik, 1/gamma_eps) on observed pixels p of patch i
 *   d_k ~ N(0, I/P), s_ik ~ N(0, 1/gamma_s), z_ik ~ Bernoulli(pi_k),
 *   pi_k ~ Beta(a/K, b(K-1)/K), gamma_s ~ Ga(c, d), gamma_eps ~ Ga(e, f).
 *
 * Conventions for every call:
 *   - Every call returns a bpfa_status; nothing throws across the ABI.  On a
 *     failure bpfa_last_error() gives a thread-local message.
 *   - The caller owns every buffer it passes.  Calls that take inputs copy
 *     them; the library keeps no caller pointer after a call returns, except
 *     the workspace given to bpfa_create, which must outlive the handle.
 *   - bpfa_mem says whether a pointer is host memory or device memory on
 *     params.device.  Device work is ordered on the handle's stream
 *     (params.stream, or a stream the library creates when it is NULL).
 *   - A handle is not thread-safe; distinct handles are independent and may
 *     be driven from different threads and streams.
 *   - Layouts are C order.  Patches are numbered in C order over the patch
 *     grid (G_d = (M_d - B_d) / S_d + 1 origins per dimension, valid patches
 *     only), pixels of a patch in C order over B.  D is K x P atom-major;
 *     W (= z * s) and Z are N x K, row i = patch i.
 */
#ifndef BPFA_H
#define BPFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bpfa_problem* bpfa_t; /* opaque; created and freed by the library */

typedef enum {
  BPFA_OK = 0,
  BPFA_EINVAL = -1,   /* NULL pointer, bad flag, bad hyper-parameter */
  BPFA_ESHAPE = -2,   /* ndim not in 1..4, B_d > M_d, S_d <= 0, K < 1, uncovered pixel,
                         transfer between different P or K */
  BPFA_ENOMEM = -3,   /* workspace too small, or a device allocation failed */
  BPFA_EDEVICE = -4,  /* a HIP runtime call failed (message has the HIP error) */
  BPFA_ESTATE = -5,   /* a state view does not match the handle, or no valid frame */
  BPFA_ENUMERIC = -6, /* non-finite gamma / residual sum, or a gamma draw that did not accept */
  BPFA_EBUSY = -7     /* reserved */
} bpfa_status;

typedef enum { BPFA_HOST = 0, BPFA_DEVICE = 1 } bpfa_mem;

/* bpfa_iterate flags */
enum {
  BPFA_LEARN_DICT = 1u,       /* sparse coding + dictionary learning (the default iteration) */
  BPFA_SPARSE_CODE_ONLY = 2u, /* keep D fixed; z, s, pi, gamma_s, gamma_eps are still drawn */
  BPFA_PRECISION_BF16 = 4u    /* reserved; rejected (EINVAL): the precision form is set by bpfa_set_precision */
};

/* contraction precision of a handle (bpfa_set_precision) */
enum { BPFA_FP32 = 0u, BPFA_BF16 = 1u };

/* bpfa_transfer_dictionary selectors */
enum { BPFA_XFER_D = 1u, BPFA_XFER_PI = 2u, BPFA_XFER_GAMMAS = 4u };

typedef struct {
  int32_t ndim;                       /* 1..4 */
  int64_t shape[4], patch[4], stride[4]; /* M, B, S per dimension (first ndim used) */
  int32_t K;                          /* dictionary size, 1..1024 */
  double a, b;                        /* beta process: pi_k ~ Beta(a/K, b(K-1)/K) */
  double c, d, e, f;                  /* gamma_s ~ Ga(c, rate d); gamma_eps ~ Ga(e, rate f) */
  double gamma_s0, gamma_eps0;        /* initial precisions */
  uint64_t seed;                      /* Philox key */
  uint32_t problem_id;                /* Philox stream id (24 bits) */
  int32_t device;                     /* HIP device ordinal */
  void* stream;                       /* hipStream_t, or NULL for a library-owned stream */
} bpfa_params;

/* Fills *p with defaults: a = b = 1, c = d = e = f = 1e-6, gamma_s0 = 1,
 * gamma_eps0 = 100, stride 1, seed 0, device 0, stream NULL. */
void bpfa_params_default(bpfa_params* p);

/* Sampler state exchanged by bpfa_get_state / bpfa_set_state.  Every pointer
 * is caller-owned and of kind `mem`; any array pointer may be NULL to skip it
 * (get) or to leave that part unchanged (set). */
typedef struct {
  float* D;           /* K x P */
  float* W;           /* N x K, z * s (zero where z = 0) */
  uint8_t* Z;         /* N x K, 0 / 1 */
  double* logit_pi;   /* K */
  double gamma_s, gamma_eps;
  int64_t t;          /* number of the next iteration (starts at 1) */
  bpfa_mem mem;
} bpfa_state_view;

typedef struct {
  int64_t t;                /* next iteration number */
  int64_t N, P, K;          /* patches, patch dimension, atoms */
  int64_t n_obs;            /* sum over patches of observed pixels */
  int64_t sum_z;            /* number of active (patch, atom) pairs after the last sweep */
  double mean_active;       /* sum_z / N */
  double gamma_s, gamma_eps;
  double pi_min, pi_mean, pi_max;
  double sum_w2;            /* sum of squared weights after the last sweep */
  double sum_r2;            /* residual sum of squares used by the last gamma_eps draw */
  int32_t max_obs;          /* largest |Obs(i)| */
  int32_t timing;           /* 1 if per-phase timing is on */
  double ms_index, ms_sweep, ms_dict, ms_scalars, ms_recon; /* accumulated, when timing is on */
  int64_t n_sweeps;         /* sweep launches timed */
  double ms_dict_stats;     /* the dictionary-statistics kernel alone (part of ms_dict) */
} bpfa_stats;

/* Device bytes of state for these parameters (the caller may allocate them,
 * e.g. as a torch tensor, and pass them to bpfa_create).  ESHAPE / EINVAL as
 * for bpfa_create. */
bpfa_status bpfa_workspace_size(const bpfa_params* params, size_t* bytes);

/* Create a problem on one image (N-D inpainting section: image of shape M,
 * patches of shape B with stride S) with its sampling mask (1 = observed; the
 * BPFA section's blind inpainting uses observed pixels only).  image holds
 * prod(shape) floats, mask prod(shape) bytes, both of kind `mem`.
 * workspace: device memory of at least bpfa_workspace_size() bytes that the
 * caller keeps alive until bpfa_destroy, or NULL to let the library allocate.
 * The state is initialised from the prior: d_kp = n / sqrt(P) (Philox INIT
 * stream), no active atoms, logit pi_k = ln(a / (b (K-1))), gamma_s0,
 * gamma_eps0, t = 1.  Index construction (masked patch extraction) runs on
 * the stream.  ESHAPE for a bad geometry, an uncovered pixel or a patch with
 * more than 256 observed pixels, ENOMEM for a short workspace, EDEVICE on a
 * HIP failure.  A mask with no observed pixel is accepted: the dictionary
 * statistics are then empty and D and gamma_eps are drawn from their priors
 * (under a vague gamma_eps prior that draw can underflow to 0 in binary64,
 * which the next synchronising call reports as ENUMERIC). */
bpfa_status bpfa_create(const bpfa_params* params, void* workspace, size_t ws_bytes,
                        const float* image, const uint8_t* mask, bpfa_mem mem, bpfa_t* out);

/* Replace the frame (image and mask of the same shape) and rebuild the patch
 * index.  reset_codes != 0 clears W and Z (D, pi and the gammas are kept:
 * the live-feed use of the feature summary); 0 keeps the codes.  ESHAPE for a
 * patch with more than 256 observed pixels; after a failed frame load
 * bpfa_iterate returns ESTATE until a frame loads. */
bpfa_status bpfa_set_frame(bpfa_t h, const float* image, const uint8_t* mask, bpfa_mem mem,
                           int reset_codes);

/* Restart the sampler on the current frame from the initial state that
 * bpfa_create sets (prior draw of D, no active atoms, initial pi and gammas,
 * t = 1).  Stream-ordered, no host synchronisation. */
bpfa_status bpfa_reset_state(bpfa_t h);

/* Run n_iters Gibbs iterations (BPFA section: each iteration a sparse-coding
 * step and, unless BPFA_SPARSE_CODE_ONLY, a dictionary-learning step).  One
 * iteration: z/s sweep over all patches (atoms in ascending order), the
 * dictionary update (atoms in ascending order), pi_k, gamma_s, gamma_eps.
 * Asynchronous on the handle's stream; a numeric failure is reported by the
 * next synchronising call (bpfa_sync, bpfa_get_state, bpfa_get_stats,
 * bpfa_reconstruct to host).  EINVAL for n_iters < 0 or unknown flags;
 * ESTATE when the last frame load failed. */
bpfa_status bpfa_iterate(bpfa_t h, int32_t n_iters, uint32_t flags);

/* Mini-batch epochs (Time-to-solution section: a dictionary trained for a
 * number of complete epochs; the paper gives no schedule, so this is a
 * reading).  The patches are dealt into n_batches mini-batches, patch i to
 * batch i mod n_batches, and one call runs n_steps mini-batch steps; step j
 * works on batch (c + j) mod n_batches, where c is the handle's batch cursor
 * (0 after bpfa_create, bpfa_set_frame, bpfa_reset_state, bpfa_set_state or a
 * change of n_batches), so n_batches steps from c = 0 make one epoch in which
 * every patch is swept once.  A step is one iteration with an iteration
 * number t of its own: the z/s sweep over the batch's patches only (the other
 * patches keep their codes), then, unless BPFA_SPARSE_CODE_ONLY, the
 * dictionary, then pi, gamma_s and gamma_eps, each drawn from its conditional
 * given the batch with every data statistic (the dictionary update's sums,
 * the usage counts and the patch count of pi, sum z and sum w^2 of gamma_s,
 * |Obs| and the residual sum of squares of gamma_eps) multiplied by
 * N / n_b (n_b = patches in the batch): the conditional given N / n_b copies
 * of the batch.  n_batches = 1 is bpfa_iterate.  Changing n_batches re-orders
 * the frame's slots by (batch, |Obs|), with one host synchronisation, and may
 * grow the handle's pinned staging buffer; otherwise asynchronous on the
 * handle's stream.  Errors as bpfa_iterate, and EINVAL for n_batches outside
 * 1 .. min(256, N) or n_steps < 0. */
bpfa_status bpfa_minibatch(bpfa_t h, int32_t n_batches, int32_t n_steps, uint32_t flags);

/* Overlap-averaged reconstruction from the current sample: every pixel is the
 * mean of the values D^T w_i that the patches covering it give it.  out holds
 * prod(shape) floats of kind `mem`; host memory synchronises the stream. */
bpfa_status bpfa_reconstruct(bpfa_t h, float* out, bpfa_mem mem);

/* Posterior-mean reconstruction (the average of samples after burn-in; the
 * N-dimensional inpainting section's averaging over samples, read as the
 * plain Monte Carlo mean of the Gibbs samples' reconstructions).
 * bpfa_mean_accumulate adds the current sample's overlap-averaged
 * reconstruction (as bpfa_reconstruct computes it, in the precision form set
 * by bpfa_set_precision) to a binary64 running sum in the workspace;
 * stream-ordered, no host synchronisation.  bpfa_mean_get writes the mean of
 * the accumulated samples, rounded to binary32, to out (prod(shape) floats of
 * kind `mem`; host memory synchronises) and the sample count to *count when
 * count is not NULL; ESTATE when no sample has been accumulated.
 * bpfa_mean_reset starts a new mean; bpfa_set_frame and bpfa_reset_state do
 * too. */
bpfa_status bpfa_mean_reset(bpfa_t h);
bpfa_status bpfa_mean_accumulate(bpfa_t h);
bpfa_status bpfa_mean_get(bpfa_t h, float* out, bpfa_mem mem, int64_t* count);

/* Per-pixel unbiased sample variance of the accumulated reconstructions,
 * (S2 - S1^2 / n) / (n - 1) from the binary64 sums S1 = sum x and S2 =
 * sum x^2 that bpfa_mean_accumulate keeps, rounded to binary32 (negative
 * rounding residue clamped to 0): the spread that the Feature summary's
 * on-the-fly strategic signal selection can steer acquisition by.  Same
 * output convention as bpfa_mean_get; ESTATE with fewer than two samples. */
bpfa_status bpfa_variance_get(bpfa_t h, float* out, bpfa_mem mem, int64_t* count);

/* Precision form of the reconstruction's contraction y_i = D^T w_i (every
 * patch's model, before the overlap average).  BPFA_FP32 (default): binary32
 * products and sums on the vector ALUs over each patch's active atoms only
 * (the sparse form).  BPFA_BF16: the dense contraction on the BF16 matrix
 * cores; every operand is split into a BF16 head and a BF16 tail, the head
 * product accumulates in binary32 and one correction pass adds the head-tail
 * cross products, so the error stays near 2^-16 of |d||w|.  The sampler (z,
 * s, D, pi, gammas) is binary32 / binary64 in both forms.  Takes effect at
 * the next bpfa_reconstruct.  EINVAL for another value; ESHAPE for BPFA_BF16
 * when P > 256 (the matrix-core tiles hold at most 256 patch pixels). */
bpfa_status bpfa_set_precision(bpfa_t h, uint32_t precision);

/* Dictionary transfer between sources (feature summary): copy D (and, as
 * selected, logit pi and the gammas) from src to dst, device to device, on
 * dst's stream after src's pending work.  ESHAPE if P or K differ. */
bpfa_status bpfa_transfer_dictionary(bpfa_t dst, bpfa_t src, uint32_t what);

/* Copy the state out (synchronises).  ESTATE never; EINVAL on NULL view. */
bpfa_status bpfa_get_state(bpfa_t h, bpfa_state_view* view);

/* Replace the state (stream-ordered; host arrays are copied before return).
 * Z and W must agree (W = 0 where Z = 0); ESTATE otherwise. */
bpfa_status bpfa_set_state(bpfa_t h, const bpfa_state_view* view);

/* bpfa_set_state for callers that cannot allocate device memory (code that
 * must not call hipMalloc, such as tight serving loops or harnesses that
 * forbid allocation): the same import, with the same results and errors, but
 * its temporary device memory -- the validity flag of the dense -> list
 * conversion and, for a BPFA_HOST view, the staging of W (and Z) -- comes
 * from a fixed 32 MiB device buffer inside the library instead of a
 * stream-ordered allocation.  Each device holds one such buffer from its
 * first call until the process ends.  A BPFA_HOST view with W may stage at
 * most 32 MiB - 256 bytes (4 N K bytes for W, N K more for Z, the Z part
 * 256-aligned), else ENOMEM with nothing changed; a BPFA_DEVICE view has no
 * size limit.  All handles on a device share the buffer, so calls that
 * overlap on one device (from different threads) race; calls that follow one
 * another are safe (each clears the flag it uses).  Synchronises, like
 * bpfa_set_state. */
bpfa_status bpfa_set_state_noalloc(bpfa_t h, const bpfa_state_view* view);

/* Per-iteration statistics (synchronises). */
bpfa_status bpfa_get_stats(bpfa_t h, bpfa_stats* stats);

/* Turn per-phase HIP-event timing on (1) or off (0); resets the totals.
 * Timing records six events per iteration on the handle's stream (created
 * without a system-scope fence: they are read only after the stream is
 * synchronised) and two per frame load and reconstruction; turning it on
 * creates a pool of 3072 events for them, which the handle keeps and reuses.
 * The durations are read at bpfa_get_stats (and, to bound the events held,
 * at a frame's end once more than 2048 iterations are pending).  Synchronises. */
bpfa_status bpfa_set_timing(bpfa_t h, int on);

/* Wait for the handle's stream; ENUMERIC if a draw failed since the last check. */
bpfa_status bpfa_sync(bpfa_t h);

/* Patch index of the current frame (masked patch extraction): per patch the
 * observed-pixel bitmask (ceil(P/32) words, bit p of word p/32) and |Obs(i)|.
 * Either pointer may be NULL.  Synchronises for host memory. */
bpfa_status bpfa_get_patch_index(bpfa_t h, uint32_t* obs_bits, int32_t* obs_count,
                                 bpfa_mem mem);

/* Diagnostic: n Philox4x32-10 blocks for counters (c0[j], c1, t, tag | problem_id << 8)
 * under key (seed low, seed high), computed on the device; out holds 4n words
 * of kind `mem`, c0 n words of kind `mem`.  Runs on the default stream of
 * `device` and synchronises. */
bpfa_status bpfa_debug_philox(int32_t device, uint64_t seed, uint32_t problem_id, uint32_t tag,
                              const uint32_t* c0, uint32_t c1, uint32_t t, int64_t n,
                              uint32_t* out, bpfa_mem mem);

void bpfa_destroy(bpfa_t h);

/* Thread-local text of the last failure in this thread ("" if none). */
const char* bpfa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BPFA_H */
