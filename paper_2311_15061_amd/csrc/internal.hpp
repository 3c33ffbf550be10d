// Internal layout shared by the host runtime and the kernels of libbpfa.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bpfa {

constexpr int kWave = 64;
constexpr int kMaxDim = 4;
// 8 waves share one LDS copy of the dictionary tile; at <= 128 VGPRs (4 waves
// per SIMD) two blocks fill a CU, so the LDS tile is not what caps residency
constexpr int kSweepBlock = 512;
constexpr int kSweepWaves = kSweepBlock / 64;
constexpr int kSweepWavesPerSimd = 4;
constexpr int kSlotAlign = 256;
constexpr int kLdsTileBytes = 64 * 1024;
constexpr int kDictBlock = 1024;
constexpr int kDictVpt = 6;       // visits per thread of one statistics chunk, held in registers
constexpr int kChainLdsMaxK = 128;  // largest K whose binary64 C_p (K x K) the chain stages in LDS
constexpr int kLdsBytes = 160 * 1024 - 1024;   // per block, leaving room for static arrays
constexpr int kDictChunkTarget = 4608; // visits per statistics chunk the row-group size leaves room for
constexpr int kSortBlock = 256;        // patches per block of the slot sort
constexpr int kMaxBatches = 256;       // mini-batches of the epoch schedule, at most

// Patch geometry (all sizes fit 32 bits; checked at create).
struct Geom {
  int32_t ndim, P, PW, K;
  int32_t N, Mtot;
  int32_t M[kMaxDim], B[kMaxDim], S[kMaxDim], G[kMaxDim];
  int32_t mstride[kMaxDim];   // image element strides
};

// Device-resident scalars: read by kernels, written by kernels, so an
// iteration needs no host round trip.
struct DevScalars {
  double gamma_s, gamma_eps;
  double sum_w2;          // after the last sweep
  double sum_r2_sweep;    // residual sum of squares after the last sweep
  double sum_r2_dict;     // after the last dictionary update (statistics form)
  double sum_r2_used;     // the one the last gamma_eps draw used
  double scale_c, scale_b;// fixed-point scales of the dictionary statistics
  double pi_min, pi_mean, pi_max;
  long long t;            // next iteration number
  long long sum_z;
  long long n_obs;        // sum_i |Obs(i)|
  int max_obs;
  int status;             // bit 0: non-finite value, bit 1: gamma draw without acceptance
  float wmax;             // max |w| after the last sweep
  float ymax;             // max |y| over observed pixels
  int n_omega;            // number of observed pixels
  uint32_t problem_id;    // Philox stream id: the kernels form their stream words from it,
                          // so a captured launch sequence serves any problem id
};

// lane classes of the sweep: patches with |Obs| in [lo, hi] get `lanes` lanes
constexpr int kLaneClasses = 5;

// Per-frame plan, built on the device from the slot sort and the frame's
// scalars, so that no launch of an iteration depends on host knowledge of the
// frame (the sweep and statistics grids are fixed per handle and read their
// ranges from here).
struct FramePlan {
  int all_waves[2];                 // wavefront range of a full sweep: [0, n_waves)
  int jpad;                         // observed rows per slot the slot tables write (>= 4, mult. of 4)
  int bad;                          // 1: a patch has more than 256 observed pixels
  int dict_chunks;                  // statistics partials per (p, row group) for this frame
  int dict_cv;                      // observed pixels per statistics chunk
  int dict_xcd;                     // dict_chunks is a multiple of 8: XCD-aligned chunk mapping
  int n_batches;
  int batch_wave0[kMaxBatches + 1]; // first wavefront of each mini-batch (+ the total)
  int batch_slot0[kMaxBatches + 1]; // first slot of each mini-batch (+ N)
  long long batch_nobs[kMaxBatches];
  // per (batch, lane class): first slot, end slot, first wavefront (+ the total)
  int cls_s0[kMaxBatches * kLaneClasses];
  int cls_s1[kMaxBatches * kLaneClasses];
  int cls_w0[kMaxBatches * kLaneClasses + 1];
};

struct SweepPart {
  double sum_w2, sum_r2;
  long long sum_z;
  float wmax;
  int pad_;
};

// Arguments of the z/s sweep.
struct SweepArgs {
  int N, Npad, P, K, KT, KS;     // KT atoms per LDS tile, KS = KT + 1 (odd column stride)
  uint32_t key0, key1, stream;   // Philox key and stream word (tag | problem_id << 8; the
                                 // kernel takes problem_id from the device scalars)
  const uint32_t* perm;          // slot -> patch
  const FramePlan* plan;         // jpad: obs rows written per slot (padding rows hold P / 0)
  const uint16_t* obs_idx;       // [J][Npad] pixel offset p in the patch (P = padding)
  const float* obs_val;          // [J][Npad] observed value (0 = padding)
  const float* D;                // K x P
  const float* Ck;               // K: logit pi_k + ln(gamma_s) / 2
  const DevScalars* scal;
  const int2* list_in;           // [N][K] by patch: active (atom, weight bits), ascending atom
  const int32_t* nact_in;        // [N] by patch
  int2* list_out;
  int32_t* nact_out;
  int32_t* cnt;                  // [gridDim][K] z counts per block
  SweepPart* part;               // [gridDim]
};

struct Buffers {
  float* image = nullptr;
  uint8_t* mask = nullptr;
  int32_t* poff = nullptr;       // P: linear image offset of in-patch pixel p
  int32_t* pcoord = nullptr;     // P x 4: its coordinates
  uint32_t* obs_bits = nullptr;  // N x PW
  int32_t* obs_count = nullptr;  // N
  uint32_t* perm = nullptr;      // Npad slot -> patch
  int32_t* inv_perm = nullptr;   // N patch -> slot
  uint16_t* obs_idx = nullptr;   // [Jcap][Npad]
  float* obs_val = nullptr;      // [Jcap][Npad]
  int4* sweep_waves = nullptr;   // per-frame wavefront table (first slot, slots, lanes per slot, J)
  FramePlan* plan = nullptr;
  int32_t* sort_hist = nullptr;  // [batch][P + 1][sort blocks of the batch]
  int32_t* sort_bin = nullptr;   // [batch][P + 1]: key totals, then key offsets
  int32_t* omega = nullptr;      // observed pixel indices, ascending (Mtot capacity)
  int4* omega_c = nullptr;       // their coordinates (unused dimensions 0)
  int32_t* omega_blk = nullptr;  // per-block counts / offsets of the compaction
  float* D = nullptr;            // K x P
  int2* list[2] = {nullptr, nullptr};
  int32_t* nact[2] = {nullptr, nullptr};
  float* Ck = nullptr;           // K
  double* ell = nullptr;         // K
  DevScalars* scal = nullptr;
  long long* nk = nullptr;       // K
  int32_t* sw_cnt = nullptr;     // sweep blocks x K
  SweepPart* sw_part = nullptr;  // sweep blocks
  int32_t* vpatch = nullptr;     // [p][Mtot]: patch that shows observed pixel v at offset p, or -1
  float* omega_y = nullptr;      // Mtot: value of observed pixel v
  uint16_t* goff = nullptr;      // N x (row groups - 1): list entries of patch i below each later
                                 // statistics row group's first row
  long long* dpart = nullptr;    // dictionary statistics partials
  double* dx2 = nullptr;         // P x chunks: sum of y^2 over visits
  double* Cfull = nullptr;       // P x K x K
  double* Bvec = nullptr;        // P x K
  double* diag = nullptr;        // P x K: C_p[k][k]
  double* x2p = nullptr;         // P: sum of x^2 over the visits of position p
  double* sumr2_p = nullptr;     // P
  float* Y = nullptr;            // P x Npad patch models D^T w_i (reconstruction)
};

// Plan of the dictionary-statistics pass: row groups of the K x K triangle
// that fit the LDS accumulator, and patch-visit chunks per (p, row group).
struct DictPlan {
  int RG = 1;                  // row groups (at most 48: K <= 1024, and a group holds >= 11.5k entries)
  int row0[65];                // row group r covers atoms [row0[r], row0[r+1])
  long long ent0[65];          // triangle entry offset of row0[r]
  int chunks = 1;
  int chunk_visits = 0;        // observed pixels per chunk (LDS visit records)
  int copies = 1;              // copies of a group's diagonal and B accumulators (lane groups)
  int copy_rows = 0;           // rows of the largest row group (each copy holds 2 x copy_rows)
  int xcd = 0;                 // chunks is a multiple of 8: map each chunk's blocks to one XCD
  long long rec_len_total = 0; // sum over row groups of (entries + rows)
  long long tri_entries = 0;   // K (K + 1) / 2
};

// bytes of LDS of the statistics kernel
// statistics LDS: accumulators | sink region | diagonal / B copies | K + 1
// bins | chunk visit records.  The sink region holds one slot per lane and K
// spare slots: a term that belongs to no accumulator of the block adds into
// (lane slot + column).
__host__ __device__ inline int dict_sink_entries(int K) { return kWave + K; }
// lane groups with their own copy of the diagonal and B accumulators: a few
// atoms are active in a third to a half of all patches, so the lanes of one
// instruction meet on their diagonal and B entries (the LDS serialises
// atomics to one address); K > 256 keeps one copy (its groups have few rows)
__host__ __device__ inline int dict_copies(int K) { return K <= 256 ? 4 : 1; }
// a chunk visit record: patch (int32), observed value (float), the list's
// length from the block's row group on and its offset there (uint16 each)
constexpr int kDictVisitBytes = 12;
inline size_t dict_stats_lds(int K, long long rec_stride, int copy_entries, int chunk_visits) {
  return (size_t)(rec_stride + dict_sink_entries(K) + copy_entries) * 8 + (size_t)(K + 1) * 4 +
         (size_t)chunk_visits * kDictVisitBytes;
}

// Sweep LDS: tile (P + 1) x KS floats | [wave][K] z counts (bytes) | per-wave
// partials (per wave 2 doubles + 1 int64 + 1 float), 8-byte aligned.
__host__ __device__ inline size_t sweep_red_offset(int P, int KS, int K) {
  const size_t off = (size_t)(P + 1) * KS * 4 + (size_t)K * kSweepWaves;
  return (off + 7) & ~(size_t)7;
}
inline size_t sweep_lds_bytes(int P, int KS, int K) {
  return sweep_red_offset(P, KS, K) + (size_t)kSweepWaves * (8 + 8 + 8 + 4);
}


// ---- launchers (each checks its own launch and returns the HIP status) ----
hipError_t launch_index(const Geom& g, const Buffers& b, int Npad, hipStream_t st);
// slot tables: rows up to the plan's jpad
hipError_t launch_slots(const Geom& g, const Buffers& b, int Npad, hipStream_t st);
hipError_t launch_omega(const Geom& g, const Buffers& b, hipStream_t st);
// p[0 .. n) = v (a kernel, so that it can be captured into a graph)
hipError_t launch_fill_i32(int32_t* p, long long n, int32_t v, hipStream_t st);
// visit table over the frame's observed pixels (count read on the device)
hipError_t launch_visit_table(const Geom& g, const Buffers& b, hipStream_t st);
// Frame plan and wavefront table from the slot sort of n_batches batches.
// Statistics chunking: the launch is sized for `dict_chunks_max` chunks of
// `dict_cv_max` observed pixels for each of `dict_npr` (position, row group)
// pairs; `dict_slots` blocks of it run at once.
hipError_t launch_frame_plan(const Geom& g, const Buffers& b, int n_batches, long long wave_cap,
                             int dict_chunks_max, int dict_cv_max, int dict_slots, int dict_npr,
                             hipStream_t st);
hipError_t launch_init_dict(const Geom& g, const Buffers& b, uint32_t key0, uint32_t key1,
                            uint32_t stream, hipStream_t st);
// the sweep over the wavefronts [range[0], range[1]) of the table (a device
// pair): `blocks` blocks, one per 8-wave group, or (strided) a fixed grid of
// `blocks` blocks that stride over the groups
hipError_t launch_sweep(const int4* waves, const int* range, int blocks, bool strided, size_t lds,
                        const SweepArgs& a, hipStream_t st);
// lanes per patch of the sweep for a patch with c observed pixels
inline int sweep_lanes(int c) { return c <= 16 ? 1 : c <= 48 ? 2 : c <= 64 ? 4 : c <= 128 ? 8 : 16; }
// wavefronts the sweep table can need for N slots: at least 4 slots per wave
// except the last wave of each (batch, lanes per slot) run
inline long long sweep_wave_capacity(long long N) { return (N + 3) / 4 + 8LL * kMaxBatches + 16; }
hipError_t launch_sort(const Geom& g, const Buffers& b, int n_batches, hipStream_t st);
// histogram entries of the slot sort for n_batches mini-batches
size_t sort_hist_entries(const Geom& g, int n_batches);
// copy the new lists of slots slot0 .. slot0 + nslots - 1 from buffer `from` to the other
hipError_t launch_list_copy(const Geom& g, const Buffers& b, int from, int slot0, int nslots,
                            hipStream_t st);
// block partials of the sweep over the wavefront range (device pair)
hipError_t launch_sweep_reduce(const Geom& g, const Buffers& b, const int* range, hipStream_t st);
// statistics over the visits of patches i with i mod n_batches == batch
// (chunk count, chunk size and mapping from the frame plan; plan.chunks and
// plan.chunk_visits give the launch's maximum; the grid covers grid_chunks
// chunk slots, at least the frame's)
hipError_t launch_list_groups(const Geom& g, const Buffers& b, const DictPlan& plan, int cur,
                              int n_batches, int batch, hipStream_t st);
hipError_t launch_dict_stats(const Geom& g, const Buffers& b, const DictPlan& plan, int grid_chunks,
                             int cur, int n_batches, int batch, hipStream_t st);
hipError_t launch_dict_reduce(const Geom& g, const Buffers& b, const DictPlan& plan,
                              hipStream_t st);
// the chain draws with the data statistics multiplied by `scale` (a
// mini-batch step's N / n_b; 1 for a full iteration)
hipError_t launch_dict_reduce_chain_lds(const Geom& g, const Buffers& b, const DictPlan& plan,
                                        double scale, uint32_t key0, uint32_t key1,
                                        uint32_t stream, hipStream_t st);
hipError_t launch_dict_chain(const Geom& g, const Buffers& b, const DictPlan& plan, double scale,
                             uint32_t key0, uint32_t key1, uint32_t stream, hipStream_t st);
// Batch of a step: n_b patches with n_obs_b observed pixels and its statistics
// scaled by `scale`; a full iteration is {N, -1 (the frame's count), 1}.
struct StepBatch {
  long long n_b;
  long long n_obs_b;
  double scale;
};
// (the Philox stream id is the device scalars' problem_id)
hipError_t launch_scalars(const Geom& g, const Buffers& b, const double* hyper, int learn_dict,
                          const StepBatch& sb, uint32_t key0, uint32_t key1, hipStream_t st);
// posterior moments: (sum, sum2) = (x, x^2) (first) or += (x, x^2);
// mean = sum / count; variance = (sum2 - sum^2 / count) / (count - 1)
hipError_t launch_mean_add(long long n, const float* x, double* sum, double* sum2, bool first,
                           hipStream_t st);
hipError_t launch_mean_get(long long n, const double* sum, double count, float* out, hipStream_t st);
hipError_t launch_variance_get(long long n, const double* sum, const double* sum2, double count,
                               float* out, hipStream_t st);
// Acquisition masks (policies of bpfa_serve.h): kinds and the Philox
// counter words of one mask (seed, frame index, stream word).
enum { kAcqUniform = 1, kAcqLineHop = 2, kAcqTargeted = 3 };
struct AcqArgs {
  long long M;            // pixels
  double rho, share;      // expected acquired fraction; targeted share
  uint32_t key0, key1, frame, stream_word;
};
// mask[0 .. M) for the policy `kind` (targeted: weights may be NULL, then
// the uniform rule; wsum is one binary64 of device scratch)
hipError_t launch_acquire(const AcqArgs& a, int kind, int ndim, const int64_t* shape,
                          const float* weights, double* wsum, uint8_t* mask, hipStream_t st);
hipError_t launch_recon(const Geom& g, const Buffers& b, int cur, int Npad, float* out, bool bf16,
                        hipStream_t st);
hipError_t launch_recon_patches_mfma(const Geom& g, const Buffers& b, int cur, hipStream_t st);
size_t recon_mfma_lds(int P);
hipError_t launch_lists_to_dense(const Geom& g, const Buffers& b, int cur, float* W, uint8_t* Z,
                                 hipStream_t st);
hipError_t launch_dense_to_lists(const Geom& g, const Buffers& b, int cur, int Npad,
                                 const float* W, const uint8_t* Z, int* bad, hipStream_t st);
hipError_t launch_ck(const Geom& g, const Buffers& b, hipStream_t st);
// next iteration number (t > 0), Philox stream id and (clear_status) no
// recorded failure, stream-ordered
hipError_t launch_set_t(DevScalars* scal, long long t, uint32_t problem_id, hipStream_t st,
                        bool clear_status);
hipError_t launch_reset_scalars(const Geom& g, const Buffers& b, double ell0, double gamma_s0,
                                double gamma_eps0, hipStream_t st);
hipError_t launch_debug_philox(uint32_t key0, uint32_t key1, uint32_t c1, uint32_t t,
                               uint32_t stream, const uint32_t* c0, long long n, uint32_t* out,
                               hipStream_t st);

}  // namespace bpfa

// ---- runtime helpers shared with the serving engine (not part of the C ABI) ----
struct bpfa_problem;
namespace bpfa {
// bytes of a dictionary-state blob: D (K x P f32), logit pi (K f64), gamma_s, gamma_eps (f64)
size_t dict_blob_bytes(int K, int P);
// copy the problem's dictionary state into / out of a device blob, on the problem's stream
int problem_export_dict(bpfa_problem* h, void* blob);
// load a blob, set the Philox stream id and the next iteration number
int problem_import_dict(bpfa_problem* h, const void* blob, long long t, uint32_t problem_id);
int problem_dims(bpfa_problem* h, int* K, int* P);
// A served frame in three stream-ordered parts.  upload: the frame's image
// and mask from pinned host memory (no synchronisation; the buffers must
// stay valid until the stream has copied them).  body: patch index (codes
// cleared), sc_iters sparse-coding iterations, a dictionary iteration if
// `learn`, the reconstruction into the workspace, and with var_samples >= 2
// the per-pixel posterior variance of the last var_samples samples (their
// reconstructions' binary64 moments, as bpfa_mean_accumulate keeps them) --
// launches only, with no pointer that changes between frames, so the body
// can be captured into a graph and replayed for any frame of the handle's
// shape.  result:
// the reconstruction to host `out`, then a synchronisation that reports a
// refused frame (ESHAPE) or a failed draw (ENUMERIC).
int problem_upload_frame(bpfa_problem* h, const float* image, const uint8_t* mask);
int problem_frame_body(bpfa_problem* h, int sc_iters, int learn, int var_samples);
int problem_frame_result(bpfa_problem* h, float* out);
hipStream_t problem_stream(bpfa_problem* h);
// the frame's image only (its mask drawn on the device by problem_acquire)
int problem_upload_image(bpfa_problem* h, const float* image);
// the frame's mask from an acquisition policy (a.M is set from the handle)
int problem_acquire(bpfa_problem* h, const AcqArgs& a, int kind, const float* weights);
const float* problem_variance(bpfa_problem* h);   // device, the last served frame's variance
const uint8_t* problem_mask(bpfa_problem* h);     // device, the frame's mask
int problem_set_id(bpfa_problem* h, uint32_t problem_id);
}  // namespace bpfa
