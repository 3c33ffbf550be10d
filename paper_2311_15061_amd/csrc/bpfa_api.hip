// Host runtime of libbpfa: the C ABI declared in include/bpfa.h.
//
// A handle owns (or borrows) one device workspace carved into the buffers of
// internal.hpp, a stream, and host copies of the few sizes the launches need.
// Iterations are launched without host synchronisation; the device keeps the
// gammas, the iteration counter and an error flag, read back by the
// synchronising calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bpfa.h"
#include "internal.hpp"

using namespace bpfa;

namespace {

thread_local std::string g_err;

bpfa_status fail(bpfa_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return fail(BPFA_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
  int Npad = 0, Jcap = 0, KT = 0, KS = 0;
  long long wave_cap = 0;       // capacity of the sweep's wavefront table
  long long rec_stride = 0;     // statistics partial record length (int64 entries)
  size_t sweep_lds = 0;
  DictPlan plan;
  // byte offsets
  size_t image, mask, poff, pcoord, obs_bits, obs_count, perm, inv_perm, obs_idx, obs_val, sweep_waves, fplan, sort_hist, sort_bin,
      omega, omega_c, omega_blk, vpatch, omega_y, D, list0, list1, nact0, nact1, Ck, ell, scal, nk, sw_cnt, sw_part, goff, dpart,
      dx2, Cfull, Bvec, diag, x2p, sumr2_p, Y, recon, mean, mean2, var, wsum, total;
};

bpfa_status make_geom(const bpfa_params* p, Geom* g) {
  if (!p) return fail(BPFA_EINVAL, "params is NULL");
  if (p->ndim < 1 || p->ndim > kMaxDim) return fail(BPFA_ESHAPE, "ndim must be 1..4, got %d", p->ndim);
  if (p->K < 1 || p->K > 1024) return fail(BPFA_ESHAPE, "K must be 1..1024, got %d", p->K);
  std::memset(g, 0, sizeof *g);
  g->ndim = p->ndim;
  g->K = p->K;
  long long P = 1, N = 1, Mt = 1;
  for (int d = 0; d < p->ndim; ++d) {
    const long long m = p->shape[d], b = p->patch[d], s = p->stride[d];
    if (m < 1 || b < 1 || b > m || s < 1)
      return fail(BPFA_ESHAPE, "dimension %d: need 1 <= B <= M and S >= 1 (M=%lld B=%lld S=%lld)", d,
                  m, b, s);
    const long long G = (m - b) / s + 1;
    if (s > b || (G - 1) * s + b != m)
      return fail(BPFA_ESHAPE, "dimension %d: pixels not covered by any patch (M=%lld B=%lld S=%lld)",
                  d, m, b, s);
    P *= b;
    N *= G;
    Mt *= m;
    if (Mt >= (1LL << 31) || N >= (1LL << 31) || P > 4096)
      return fail(BPFA_ESHAPE, "problem too large for 32-bit indexing (M, N) or P > 4096");
    g->M[d] = (int)m;
    g->B[d] = (int)b;
    g->S[d] = (int)s;
    g->G[d] = (int)G;
  }
  g->P = (int)P;
  g->PW = (int)((P + 31) / 32);
  g->N = (int)N;
  g->Mtot = (int)Mt;
  int st = 1;
  for (int d = p->ndim - 1; d >= 0; --d) {
    g->mstride[d] = st;
    st *= g->M[d];
  }
  if (!(p->a > 0 && p->b > 0 && p->c > 0 && p->d > 0 && p->e > 0 && p->f > 0 &&
        p->gamma_s0 > 0 && p->gamma_eps0 > 0) ||
      !std::isfinite(p->a + p->b + p->c + p->d + p->e + p->f + p->gamma_s0 + p->gamma_eps0))
    return fail(BPFA_EINVAL, "hyper-parameters and initial precisions must be positive and finite");
  if (p->problem_id >= (1u << 24)) return fail(BPFA_EINVAL, "problem_id must fit 24 bits");
  return BPFA_OK;
}

DictPlan make_dict_plan(const Geom& g) {
  DictPlan pl;
  const int K = g.K;
  // Row groups leave room for chunks of kDictChunkTarget visits (one group
  // when the whole triangle fits beside such a chunk).  A block buckets its
  // chunk's visits by list length and its wavefronts claim runs of 64, so in
  // a small chunk they get very different pair counts and wait for the
  // longest at the chunk's barrier; several row groups cost each visit its
  // bookkeeping and gather once per group, but a later group walks only the
  // lists' tails (list_groups_kernel), so they add little pair work.
  const long long whole = (long long)K * (K + 1) / 2 + K;
  // the groups are found for a room that leaves space for the diagonal / B
  // copies of `reserve` rows; the copies then take the largest group's rows,
  // and the grouping is redone with that reserve until it fits (twice at most
  // for the sizes the library takes)
  const int copies = dict_copies(K);
  int rg = 0;
  for (int reserve = 0;;) {
    const long long fixed = (long long)(K + 1) * 4 + (long long)dict_sink_entries(K) * 8 +
                            (long long)copies * 2 * reserve * 8;
    const long long group_room =
        ((long long)kLdsBytes - fixed - (long long)kDictChunkTarget * kDictVisitBytes) / 8;
    const long long budget = whole <= group_room ? whole : std::max<long long>((long long)K + 1, group_room);
    rg = 0;
    pl.row0[0] = 0;
    pl.ent0[0] = 0;
    long long len = 0;
    int rows = 0, rows_max = 0;
    for (int k = 0; k < K; ++k) {
      const long long add = (K - k) + 1;
      if (len + add > budget && len > 0) {
        ++rg;
        pl.row0[rg] = k;
        pl.ent0[rg] = (long long)k * K - (long long)k * (k - 1) / 2;
        len = 0;
        rows = 0;
      }
      len += add;
      rows_max = std::max(rows_max, ++rows);
    }
    if (rows_max <= reserve || reserve >= K) break;
    reserve = std::max(rows_max, reserve + 1);
  }
  pl.RG = rg + 1;
  pl.row0[pl.RG] = K;
  pl.ent0[pl.RG] = (long long)K * (K + 1) / 2;
  pl.tri_entries = pl.ent0[pl.RG];
  pl.rec_len_total = pl.tri_entries + K;
  // chunk of observed pixels per block: as many visit records as the LDS
  // left over by the largest row group holds (a multiple of the wavefront)
  long long rec_max = 0;
  for (int r = 0; r < pl.RG; ++r)
    rec_max = std::max(rec_max, (pl.ent0[r + 1] - pl.ent0[r]) + (long long)(pl.row0[r + 1] - pl.row0[r]));
  pl.copies = dict_copies(K);
  pl.copy_rows = 0;
  for (int r = 0; r < pl.RG; ++r) pl.copy_rows = std::max(pl.copy_rows, pl.row0[r + 1] - pl.row0[r]);
  const long long room = (long long)kLdsBytes -
                         (rec_max + dict_sink_entries(K) + (long long)pl.copies * 2 * pl.copy_rows) * 8 -
                         (long long)(K + 1) * 4;
  pl.chunk_visits = (int)std::max<long long>(
      kDictBlock, std::min<long long>(kDictBlock * kDictVpt, room / kDictVisitBytes / kWave * kWave));
  // chunk slots per (p, row group): the frame plan uses the first few of them,
  // chosen on the device from the frame's observed pixels
  const long long mt = g.Mtot;
  pl.chunks = (int)std::min<long long>(16, std::max<long long>(1, (mt + pl.chunk_visits - 1) / pl.chunk_visits));
  if (pl.chunks > 1 && pl.chunks < 8) pl.chunks = 8;   // room for the XCD-aligned chunking
  return pl;
}

Layout make_layout(const Geom& g) {
  Layout L;
  L.Npad = (int)align_up((size_t)g.N, kSlotAlign);
  L.Jcap = (int)align_up((size_t)g.P, 4);
  // dictionary tile of the sweep: pixel-major with an odd atom stride
  const long long P1 = g.P + 1;
  if (P1 * (g.K + 1) * 4 <= kLdsTileBytes) {
    L.KT = g.K;
  } else {
    int ktmax = (int)(kLdsTileBytes / (P1 * 4)) - 1;
    ktmax &= ~1;
    if (ktmax < 2) ktmax = 2;
    const int tiles = (g.K + ktmax - 1) / ktmax;
    L.KT = (int)align_up((size_t)((g.K + tiles - 1) / tiles), 2);
  }
  L.KS = L.KT + 1;
  if (L.KS % 2 == 0) L.KS += 1;
  L.wave_cap = sweep_wave_capacity(g.N);
  L.sweep_lds = sweep_lds_bytes(g.P, L.KS, g.K);
  L.plan = make_dict_plan(g);
  long long rec_stride = 0;
  for (int r = 0; r < L.plan.RG; ++r) {
    const long long len =
        (L.plan.ent0[r + 1] - L.plan.ent0[r]) + (L.plan.row0[r + 1] - L.plan.row0[r]);
    rec_stride = std::max(rec_stride, len);
  }
  L.rec_stride = rec_stride;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1), 256);
    return o;
  };
  const size_t N = g.N, Np = L.Npad, K = g.K, P = g.P;
  L.image = take(4 * (size_t)g.Mtot);
  L.mask = take((size_t)g.Mtot);
  L.poff = take(4 * P);
  L.pcoord = take(4 * P * kMaxDim);
  L.obs_bits = take(4 * N * g.PW);
  L.obs_count = take(4 * N);
  L.perm = take(4 * Np);
  L.inv_perm = take(4 * N);
  L.obs_idx = take(2 * (size_t)L.Jcap * Np);
  L.obs_val = take(4 * (size_t)L.Jcap * Np);
  L.sweep_waves = take(16 * (size_t)L.wave_cap);
  L.fplan = take(sizeof(FramePlan));
  // the sort's histogram for up to kMaxBatches batches: each batch's sort
  // blocks hold ceil(N / B / 256) <= ceil(N / 256 / B) + 1 blocks' worth
  L.sort_hist = take(4 * (P + 1) * ((N + kSortBlock - 1) / kSortBlock + kMaxBatches));
  L.sort_bin = take(4 * (P + 1) * (size_t)kMaxBatches);
  L.omega = take(4 * (size_t)g.Mtot);
  L.omega_c = take(16 * (size_t)g.Mtot);
  L.omega_blk = take(4 * (((size_t)g.Mtot + 255) / 256 + 1));
  L.vpatch = take(4 * P * (size_t)g.Mtot);
  L.omega_y = take(4 * (size_t)g.Mtot);
  L.D = take(4 * K * P);
  // two entries of slack: the sweep reads up to two entries past a row
  L.list0 = take(8 * Np * K + 16);
  L.list1 = take(8 * Np * K + 16);
  L.nact0 = take(4 * Np);
  L.nact1 = take(4 * Np);
  L.Ck = take(4 * K);
  L.ell = take(8 * K);
  L.scal = take(sizeof(DevScalars));
  L.nk = take(8 * K);
  L.sw_cnt = take(4 * K);
  L.sw_part = take(sizeof(SweepPart) * (size_t)((L.wave_cap + kSweepWaves - 1) / kSweepWaves));
  L.goff = take(2 * N * (size_t)(L.plan.RG - 1));
  L.dpart = take(8 * (size_t)P * L.plan.RG * L.plan.chunks * rec_stride);
  L.dx2 = take(8 * P * L.plan.chunks);
  L.Cfull = take(8 * P * K * K);
  L.Bvec = take(8 * P * K);
  L.diag = take(8 * P * K);
  L.x2p = take(8 * P);
  L.sumr2_p = take(8 * P);
  L.Y = take(4 * P * N);
  L.recon = take(4 * (size_t)g.Mtot);
  L.mean = take(8 * (size_t)g.Mtot);   // posterior-moment running sums
  L.mean2 = take(8 * (size_t)g.Mtot);
  L.var = take(4 * (size_t)g.Mtot);    // a served frame's posterior variance
  L.wsum = take(8);                     // sum of acquisition weights
  L.total = off;
  return L;
}

}  // namespace

struct bpfa_problem {
  bpfa_params prm{};
  Geom g{};
  Layout L{};
  Buffers b{};
  char* ws = nullptr;
  bool own_ws = false;
  hipStream_t st = nullptr;
  bool own_stream = false;
  int cur = 0;
  int precision = BPFA_FP32;    // contraction precision of the reconstruction
  int max_obs = 0, n_omega = 0;  // host copies from the last frame plan read back
  int n_cu = 256;               // compute units of the device
  int sweep_grid = 0;           // blocks of a sweep launch (they stride over the 8-wave groups)
  int dict_slots = 0;           // statistics blocks resident at once
  // pinned host staging (hipHostMalloc) of the frame load's readback of the
  // scalars and the frame plan, so the copy runs as DMA without a pageable bounce
  char* stage = nullptr;
  size_t stage_bytes = 0;
  // mini-batch partition of the slot order (patch i in batch i mod n_batches)
  int n_batches = 1;
  int batch_cursor = 0;            // batch of the next mini-batch step
  // host copy of the mini-batch ranges of the plan (read back when a
  // mini-batch step needs them: plan_known)
  std::vector<int> batch_slot0;    // n_batches + 1: first slot of each batch
  std::vector<int> batch_wave0;    // n_batches + 1: first wavefront of each batch
  std::vector<long long> batch_nobs;  // observed pixels of each batch
  int dict_chunks = 0;             // statistics chunks of the frame
  bool plan_known = false;
  uint32_t key0 = 0, key1 = 0;
  int64_t t_host = 1;
  int64_t mean_count = 0;       // samples in the posterior-mean running sum
  bool frame_ok = false;        // the last frame load completed (the index is whole)
  // timing
  bool timing = false;
  // per step: before / after the sweep, before / after the statistics kernel,
  // after the dictionary draws, after the scalar draws
  std::vector<std::array<hipEvent_t, 6>> iter_events;
  std::vector<std::array<hipEvent_t, 2>> index_events, recon_events;
  std::vector<hipEvent_t> event_pool;   // events whose timings were collected, for reuse
  double ms_index = 0, ms_sweep = 0, ms_dict = 0, ms_dict_stats = 0, ms_scalars = 0, ms_recon = 0;
  int64_t n_sweeps = 0;
};

namespace {

uint32_t stream_word(uint32_t tag, uint32_t pid) { return (tag & 0xFFu) | (pid << 8); }

bpfa_status upload(bpfa_problem* h, void* dst, const void* src, size_t bytes, bpfa_mem mem) {
  if (bytes == 0) return BPFA_OK;
  if (!src) return fail(BPFA_EINVAL, "NULL input buffer");
  HIPCHK(hipMemcpyAsync(dst, src, bytes,
                        mem == BPFA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->st));
  if (mem == BPFA_HOST) HIPCHK(hipStreamSynchronize(h->st));  // the caller may free src
  return BPFA_OK;
}

// Timing events: read only after the stream is synchronised, so they need no
// system-scope fence when they complete (with it every record wrote back and
// invalidated the caches: ~0.35 ms per 512 x 512 frame of 130 records, and
// the timed kernels paid for the flushes).  Taken from the handle's pool.
hipError_t create_timing_event(hipEvent_t* ev) {
  return hipEventCreateWithFlags(ev, hipEventDisableSystemFence);
}

bpfa_status record(bpfa_problem* h, hipEvent_t* ev) {
  if (h->event_pool.empty()) {
    HIPCHK(create_timing_event(ev));
  } else {
    *ev = h->event_pool.back();
    h->event_pool.pop_back();
  }
  HIPCHK(hipEventRecord(*ev, h->st));
  return BPFA_OK;
}

bpfa_status collect_timing(bpfa_problem* h) {
  float ms = 0.f;
  for (auto& e : h->iter_events) {
    HIPCHK(hipEventElapsedTime(&ms, e[0], e[1]));
    h->ms_sweep += ms;
    HIPCHK(hipEventElapsedTime(&ms, e[1], e[4]));
    h->ms_dict += ms;
    HIPCHK(hipEventElapsedTime(&ms, e[2], e[3]));
    h->ms_dict_stats += ms;
    HIPCHK(hipEventElapsedTime(&ms, e[4], e[5]));
    h->ms_scalars += ms;
    for (auto ev : e) h->event_pool.push_back(ev);
    ++h->n_sweeps;
  }
  h->iter_events.clear();
  for (auto& e : h->index_events) {
    HIPCHK(hipEventElapsedTime(&ms, e[0], e[1]));
    h->ms_index += ms;
    for (auto ev : e) h->event_pool.push_back(ev);
  }
  h->index_events.clear();
  for (auto& e : h->recon_events) {
    HIPCHK(hipEventElapsedTime(&ms, e[0], e[1]));
    h->ms_recon += ms;
    for (auto ev : e) h->event_pool.push_back(ev);
  }
  h->recon_events.clear();
  return BPFA_OK;
}

bpfa_status check_status(bpfa_problem* h) {
  DevScalars s;
  HIPCHK(hipMemcpyAsync(&s, h->b.scal, sizeof s, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  // the recorded timings are read at bpfa_get_stats; a long run of timed
  // frames without a read collects here, to bound the events held
  if (h->iter_events.size() > 2048) {
    const bpfa_status r = collect_timing(h);
    if (r != BPFA_OK) return r;
  }
  h->t_host = s.t;
  if (s.status) {
    const int zero = 0;
    HIPCHK(hipMemcpyAsync(&h->b.scal->status, &zero, sizeof zero, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return fail(BPFA_ENUMERIC, "numeric failure in an iteration (flags %d: %s%s)", s.status,
                (s.status & 1) ? "non-finite value " : "",
                (s.status & 2) ? "gamma draw without acceptance" : "");
  }
  return BPFA_OK;
}

// Host copies of the frame plan: sizes for the statistics and the mini-batch
// ranges; ESHAPE when a patch has more than 256 observed pixels (the index
// is then not usable and the frame load has failed).  Synchronises.
bpfa_status read_plan(bpfa_problem* h) {
  DevScalars* sp = reinterpret_cast<DevScalars*>(h->stage);
  FramePlan* fp = reinterpret_cast<FramePlan*>(h->stage + align_up(sizeof(DevScalars), 16));
  HIPCHK(hipMemcpyAsync(sp, h->b.scal, sizeof(DevScalars), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipMemcpyAsync(fp, h->b.plan, sizeof(FramePlan), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  h->max_obs = sp->max_obs;
  h->n_omega = sp->n_omega;
  if (fp->bad)
    return fail(BPFA_ESHAPE, "a patch has %d observed pixels; at most 256 are supported", h->max_obs);
  const int B = fp->n_batches;
  h->batch_slot0.assign(fp->batch_slot0, fp->batch_slot0 + B + 1);
  h->batch_wave0.assign(fp->batch_wave0, fp->batch_wave0 + B + 1);
  h->batch_nobs.assign(fp->batch_nobs, fp->batch_nobs + B);
  h->dict_chunks = fp->dict_chunks;
  h->plan_known = true;
  return BPFA_OK;
}

// Pinned staging of the frame load's readback: the device scalars and the
// frame plan.
size_t stage_size() { return align_up(sizeof(DevScalars), 16) + sizeof(FramePlan); }

// Slot order of the current frame for a partition into n_batches
// mini-batches, the frame plan (wavefront table, observed rows per slot,
// statistics chunking, batch ranges) and the per-slot observed tables, all
// built on the device: nothing the launches of an iteration need comes from
// the host.  readback: read the scalars and the plan back (one host
// synchronisation) to report a patch with more than 256 observed pixels
// (ESHAPE) and keep host copies of the frame's sizes and batch ranges.
bpfa_status order_slots(bpfa_problem* h, int n_batches, bool readback) {
  const Geom& g = h->g;
  if (sort_hist_entries(g, n_batches) >
      (size_t)(g.P + 1) * ((g.N + kSortBlock - 1) / kSortBlock + kMaxBatches))
    return fail(BPFA_EINVAL, "sort histogram too small for %d batches", n_batches);
  HIPCHK(launch_sort(g, h->b, n_batches, h->st));
  const DictPlan& pl = h->L.plan;
  HIPCHK(launch_frame_plan(g, h->b, n_batches, h->L.wave_cap, pl.chunks, pl.chunk_visits,
                           h->dict_slots, g.P * pl.RG, h->st));
  HIPCHK(launch_slots(g, h->b, h->L.Npad, h->st));
  h->n_batches = n_batches;
  h->batch_cursor = 0;
  h->plan_known = false;
  if (readback) return read_plan(h);
  return BPFA_OK;
}

// No active atoms in either list buffer (a fill kernel, not a memset, so the
// sequence can be captured into a graph); the sweep then starts from buffer 0.
bpfa_status clear_codes(bpfa_problem* h) {
  HIPCHK(launch_fill_i32(h->b.nact[0], h->L.Npad, 0, h->st));
  HIPCHK(launch_fill_i32(h->b.nact[1], h->L.Npad, 0, h->st));
  h->cur = 0;
  return BPFA_OK;
}

// Rebuild the patch index of the frame in the workspace.  keep_codes: the
// active lists (stored by patch, not by slot) stay as they are; otherwise
// they are cleared.  readback: finish with the plan readback (one host
// synchronisation; ESHAPE for a patch with more than 256 observed pixels).
// Without it the sequence is stream-ordered launches only (no
// synchronisation, no memset, so it can be captured into a graph) and a
// refused frame shows in the plan's `bad` flag.
bpfa_status index_frame(bpfa_problem* h, bool keep_codes, bool readback) {
  const Geom& g = h->g;
  h->frame_ok = false;   // until every table of the new frame is built
  bpfa_status r;
  std::array<hipEvent_t, 2> ev{};
  if (h->timing && (r = record(h, &ev[0])) != BPFA_OK) return r;
  HIPCHK(launch_index(g, h->b, h->L.Npad, h->st));
  if (!keep_codes && (r = clear_codes(h)) != BPFA_OK) return r;
  HIPCHK(launch_omega(g, h->b, h->st));
  HIPCHK(launch_visit_table(g, h->b, h->st));
  if ((r = order_slots(h, h->n_batches, readback)) != BPFA_OK) return r;
  if (h->timing) {
    if ((r = record(h, &ev[1])) != BPFA_OK) return r;
    h->index_events.push_back(ev);
  }
  h->frame_ok = true;
  return BPFA_OK;
}

// Upload a frame and rebuild its patch index (with the plan readback).
bpfa_status load_frame(bpfa_problem* h, const float* image, const uint8_t* mask, bpfa_mem mem,
                       bool keep_codes) {
  const Geom& g = h->g;
  h->frame_ok = false;
  bpfa_status r;
  if ((r = upload(h, h->b.image, image, 4 * (size_t)g.Mtot, mem)) != BPFA_OK) return r;
  if ((r = upload(h, h->b.mask, mask, (size_t)g.Mtot, mem)) != BPFA_OK) return r;
  return index_frame(h, keep_codes, true);
}

bpfa_status check_iter_flags(bpfa_t h, uint32_t flags) {
  if (flags & ~(uint32_t)(BPFA_LEARN_DICT | BPFA_SPARSE_CODE_ONLY | BPFA_PRECISION_BF16))
    return fail(BPFA_EINVAL, "unknown flags 0x%x", flags);
  if ((flags & BPFA_LEARN_DICT) && (flags & BPFA_SPARSE_CODE_ONLY))
    return fail(BPFA_EINVAL, "LEARN_DICT and SPARSE_CODE_ONLY are exclusive");
  if (flags & BPFA_PRECISION_BF16)
    return fail(BPFA_EINVAL, "the precision form is chosen with bpfa_set_precision, not an iterate flag");
  if (!h->frame_ok)
    return fail(BPFA_ESTATE, "the last frame load failed; set a valid frame before iterating");
  return BPFA_OK;
}

// One Gibbs step on the handle's stream: batch < 0 is a full iteration over
// every patch; batch >= 0 a mini-batch step over that batch of the current
// partition, its statistics scaled by N / n_b.
bpfa_status run_step(bpfa_t h, int learn, int batch) {
  const Geom& g = h->g;
  const Layout& L = h->L;
  Buffers& b = h->b;
  const double hyper[6] = {h->prm.a, h->prm.b, h->prm.c, h->prm.d, h->prm.e, h->prm.f};
  // the sweep's wavefront range lives in the frame plan: all of it, or the batch's
  const int* range = b.plan->all_waves;
  int nbat = 1, bsel = 0;
  StepBatch sb{g.N, -1, 1.0};
  if (batch >= 0) {
    range = b.plan->batch_wave0 + batch;
    nbat = h->n_batches;
    bsel = batch;
    sb.n_b = h->batch_slot0[batch + 1] - h->batch_slot0[batch];
    sb.n_obs_b = h->batch_nobs[batch];
    sb.scale = (double)g.N / (double)sb.n_b;
  }
  SweepArgs a{};
  a.N = g.N;
  a.Npad = L.Npad;
  a.P = g.P;
  a.K = g.K;
  a.KT = L.KT;
  a.KS = L.KS;
  a.key0 = h->key0;
  a.key1 = h->key1;
  a.stream = stream_word(1, h->prm.problem_id);
  a.perm = b.perm;
  a.plan = b.plan;
  a.obs_idx = b.obs_idx;
  a.obs_val = b.obs_val;
  a.D = b.D;
  a.Ck = b.Ck;
  a.scal = b.scal;
  a.list_in = b.list[h->cur];
  a.nact_in = b.nact[h->cur];
  a.list_out = b.list[1 - h->cur];
  a.nact_out = b.nact[1 - h->cur];
  a.cnt = b.sw_cnt;
  a.part = b.sw_part;
  std::array<hipEvent_t, 6> ev{};
  bpfa_status r;
  if (h->timing && (r = record(h, &ev[0])) != BPFA_OK) return r;
  // with the plan on the host one block per 8-wave group; otherwise (a
  // captured sequence) the fixed grid that strides over them
  if (h->plan_known) {
    const int nw = batch >= 0 ? h->batch_wave0[batch + 1] - h->batch_wave0[batch] : h->batch_wave0.back();
    HIPCHK(launch_sweep(b.sweep_waves, range, (nw + kSweepWaves - 1) / kSweepWaves, false, L.sweep_lds,
                        a, h->st));
  } else {
    HIPCHK(launch_sweep(b.sweep_waves, range, h->sweep_grid, true, L.sweep_lds, a, h->st));
  }
  if (h->timing && (r = record(h, &ev[1])) != BPFA_OK) return r;
  HIPCHK(launch_sweep_reduce(g, b, range, h->st));
  if (batch < 0) {
    h->cur = 1 - h->cur;
  } else {
    // the batch's new lists go back into the current buffer, which keeps
    // every other patch's codes
    const int s0 = h->batch_slot0[batch];
    HIPCHK(launch_list_copy(g, b, 1 - h->cur, s0, h->batch_slot0[batch + 1] - s0, h->st));
  }
  // with several statistics row groups: where each list enters each group
  if (learn) HIPCHK(launch_list_groups(g, b, L.plan, h->cur, nbat, bsel, h->st));
  if (h->timing && (r = record(h, &ev[2])) != BPFA_OK) return r;
  if (learn)
    HIPCHK(launch_dict_stats(g, b, L.plan, h->plan_known ? h->dict_chunks : L.plan.chunks, h->cur, nbat,
                             bsel, h->st));
  if (h->timing && (r = record(h, &ev[3])) != BPFA_OK) return r;
  if (learn) {
    const DictPlan& plan = L.plan;
    if (g.K <= kChainLdsMaxK && plan.RG == 1) {
      HIPCHK(launch_dict_reduce_chain_lds(g, b, plan, sb.scale, h->key0, h->key1,
                                          stream_word(2, h->prm.problem_id), h->st));
    } else {
      HIPCHK(launch_dict_reduce(g, b, plan, h->st));
      HIPCHK(launch_dict_chain(g, b, L.plan, sb.scale, h->key0, h->key1,
                               stream_word(2, h->prm.problem_id), h->st));
    }
  }
  if (h->timing && (r = record(h, &ev[4])) != BPFA_OK) return r;
  HIPCHK(launch_scalars(g, b, hyper, learn, sb, h->key0, h->key1, h->st));
  if (h->timing) {
    if ((r = record(h, &ev[5])) != BPFA_OK) return r;
    h->iter_events.push_back(ev);
  }
  ++h->t_host;
  return BPFA_OK;
}

// ---- state import --------------------------------------------------------

// Fixed device buffer of bpfa_set_state_noalloc: the validity flag of the
// dense -> list conversion in its first 256 bytes, then the staging of a
// host-kind W (and Z).  One copy per device, held until the process ends;
// every call on a device shares it.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr size_t kScratchFlagBytes = 256;
constexpr int kScratchDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kScratchDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current (the caller's DeviceGuard).  The array's
// name is only a host-side stand-in; kernels and copies use this address.
bpfa_status scratch_base(int device, char** out) {
  if (device < 0 || device >= kScratchDevices)
    return fail(BPFA_EDEVICE, "device %d is outside the %d devices the scratch table covers", device,
                kScratchDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(BPFA_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                  hipGetErrorString(e));
    g_scratch_ptr[device] = (char*)ptr;
  }
  *out = g_scratch_ptr[device];
  return BPFA_OK;
}

// bpfa_set_state, with its temporary device memory (the flag of the dense ->
// list conversion, the staging of host-kind W and Z) either allocated
// stream-ordered (scratch == NULL) or taken from the fixed buffer.
bpfa_status set_state_impl(bpfa_t h, const bpfa_state_view* v, char* scratch_mem) {
  if (!h || !v) return fail(BPFA_EINVAL, "NULL handle or view");
  if (!(v->gamma_s > 0) || !(v->gamma_eps > 0) || !std::isfinite(v->gamma_s) ||
      !std::isfinite(v->gamma_eps) || v->t < 1 || v->t >= (1LL << 32))
    return fail(BPFA_ESTATE, "state gammas must be positive and finite, 1 <= t < 2^32");
  if (!v->W && v->Z) return fail(BPFA_ESTATE, "Z without W cannot define the weights");
  DeviceGuard dg(h->prm.device);
  const Geom& g = h->g;
  const size_t nk = (size_t)g.N * g.K;
  // temporary device bytes: flag, then (host views) W and Z staging
  const size_t w_off = kScratchFlagBytes;
  const size_t z_off = w_off + align_up(4 * nk, 256);
  const size_t need = !v->W ? 0
                      : v->mem == BPFA_HOST ? z_off + (v->Z ? nk : 0)
                                            : kScratchFlagBytes;
  if (scratch_mem && need > kScratchBytes)
    return fail(BPFA_ENOMEM,
                "the fixed state-import buffer holds %zu bytes; this state needs %zu "
                "(N x K = %zu weights staged from host memory)",
                kScratchBytes, need, nk);
  const hipMemcpyKind kind = v->mem == BPFA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (v->D) HIPCHK(hipMemcpyAsync(h->b.D, v->D, 4 * (size_t)g.K * g.P, kind, h->st));
  if (v->logit_pi) HIPCHK(hipMemcpyAsync(h->b.ell, v->logit_pi, 8 * (size_t)g.K, kind, h->st));
  int bad = 0;
  if (v->W) {
    char* tmp = scratch_mem;
    if (!tmp) HIPCHK(hipMallocAsync((void**)&tmp, need, h->st));
    int* dbad = (int*)tmp;
    const float* W = v->W;
    const uint8_t* Z = v->Z;
    if (v->mem == BPFA_HOST) {
      HIPCHK(hipMemcpyAsync(tmp + w_off, v->W, 4 * nk, hipMemcpyHostToDevice, h->st));
      W = (const float*)(tmp + w_off);
      if (v->Z) {
        HIPCHK(hipMemcpyAsync(tmp + z_off, v->Z, nk, hipMemcpyHostToDevice, h->st));
        Z = (const uint8_t*)(tmp + z_off);
      }
    }
    // the fixed buffer keeps the previous call's flag: clear it first
    HIPCHK(hipMemsetAsync(dbad, 0, 4, h->st));
    HIPCHK(launch_dense_to_lists(g, h->b, h->cur, h->L.Npad, W, Z, dbad, h->st));
    HIPCHK(hipMemcpyAsync(&bad, dbad, 4, hipMemcpyDeviceToHost, h->st));
    if (!scratch_mem) HIPCHK(hipFreeAsync(tmp, h->st));
  }
  DevScalars s;
  HIPCHK(hipMemcpyAsync(&s, h->b.scal, sizeof s, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  s.gamma_s = v->gamma_s;
  s.gamma_eps = v->gamma_eps;
  s.t = v->t;
  HIPCHK(hipMemcpyAsync(h->b.scal, &s, sizeof s, hipMemcpyHostToDevice, h->st));
  HIPCHK(launch_ck(g, h->b, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  h->t_host = v->t;
  h->batch_cursor = 0;
  if (bad) return fail(BPFA_ESTATE, "W is non-zero where Z is 0");
  return BPFA_OK;
}

}  // namespace

extern "C" {

void bpfa_params_default(bpfa_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->ndim = 2;
  for (int d = 0; d < 4; ++d) p->stride[d] = 1;
  p->K = 64;
  p->a = p->b = 1.0;
  p->c = p->d = p->e = p->f = 1e-6;
  p->gamma_s0 = 1.0;
  p->gamma_eps0 = 100.0;
}

bpfa_status bpfa_workspace_size(const bpfa_params* params, size_t* bytes) {
  Geom g;
  bpfa_status r = make_geom(params, &g);
  if (r != BPFA_OK) return r;
  if (!bytes) return fail(BPFA_EINVAL, "bytes is NULL");
  *bytes = make_layout(g).total;
  return BPFA_OK;
}

bpfa_status bpfa_create(const bpfa_params* params, void* workspace, size_t ws_bytes,
                        const float* image, const uint8_t* mask, bpfa_mem mem, bpfa_t* out) {
  if (!out) return fail(BPFA_EINVAL, "out is NULL");
  *out = nullptr;
  Geom g;
  bpfa_status r = make_geom(params, &g);
  if (r != BPFA_OK) return r;
  if (!image || !mask) return fail(BPFA_EINVAL, "image and mask are required");
  DeviceGuard dg(params->device);
  if (!dg.ok) return fail(BPFA_EDEVICE, "cannot select device %d", params->device);
  auto* h = new bpfa_problem();
  h->prm = *params;
  h->g = g;
  h->L = make_layout(g);
  h->key0 = (uint32_t)(params->seed & 0xFFFFFFFFu);
  h->key1 = (uint32_t)(params->seed >> 32);
  auto bail = [&](bpfa_status s) {
    bpfa_destroy(h);
    return s;
  };
  if (params->stream) {
    h->st = (hipStream_t)params->stream;
  } else {
    if (hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(BPFA_EDEVICE, "hipStreamCreate failed"));
    h->own_stream = true;
  }
  h->stage_bytes = stage_size();
  if (hipHostMalloc((void**)&h->stage, h->stage_bytes, hipHostMallocDefault) != hipSuccess)
    return bail(fail(BPFA_ENOMEM, "hipHostMalloc of %zu staging bytes failed", h->stage_bytes));
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, params->device) ==
            hipSuccess && ncu > 0)
      h->n_cu = ncu;
  }
  {
    // launch shapes fixed per handle: the sweep's grid strides over the
    // frame's 8-wave groups with as many blocks as are resident at once (two
    // per CU at 128 VGPRs unless the LDS tile allows fewer); the statistics
    // blocks resident at once size the frame plan's chunk choice
    const Layout& L = h->L;
    const long long lds_cu = 160 * 1024;
    const int sweep_per_cu = (int)std::max(1LL, std::min(2LL, lds_cu / (long long)L.sweep_lds));
    h->sweep_grid = (int)std::min<long long>((L.wave_cap + kSweepWaves - 1) / kSweepWaves,
                                             (long long)h->n_cu * sweep_per_cu);
    const size_t dlds = dict_stats_lds(g.K, L.rec_stride, L.plan.copies * 2 * L.plan.copy_rows,
                                       L.plan.chunk_visits);
    h->dict_slots = h->n_cu * (int)std::max(1LL, lds_cu / (long long)dlds);
  }
  if (workspace) {
    if (ws_bytes < h->L.total)
      return bail(fail(BPFA_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, h->L.total));
    h->ws = (char*)workspace;
  } else {
    if (hipMalloc((void**)&h->ws, h->L.total) != hipSuccess)
      return bail(fail(BPFA_ENOMEM, "hipMalloc of %zu bytes failed", h->L.total));
    h->own_ws = true;
  }
  const Layout& L = h->L;
  char* w = h->ws;
  Buffers& b = h->b;
  b.image = (float*)(w + L.image);
  b.mask = (uint8_t*)(w + L.mask);
  b.poff = (int32_t*)(w + L.poff);
  b.pcoord = (int32_t*)(w + L.pcoord);
  b.obs_bits = (uint32_t*)(w + L.obs_bits);
  b.obs_count = (int32_t*)(w + L.obs_count);
  b.perm = (uint32_t*)(w + L.perm);
  b.inv_perm = (int32_t*)(w + L.inv_perm);
  b.obs_idx = (uint16_t*)(w + L.obs_idx);
  b.obs_val = (float*)(w + L.obs_val);
  b.sweep_waves = (int4*)(w + L.sweep_waves);
  b.plan = (FramePlan*)(w + L.fplan);
  b.sort_hist = (int32_t*)(w + L.sort_hist);
  b.sort_bin = (int32_t*)(w + L.sort_bin);
  b.omega = (int32_t*)(w + L.omega);
  b.omega_c = (int4*)(w + L.omega_c);
  b.vpatch = (int32_t*)(w + L.vpatch);
  b.omega_y = (float*)(w + L.omega_y);
  b.omega_blk = (int32_t*)(w + L.omega_blk);
  b.D = (float*)(w + L.D);
  b.list[0] = (int2*)(w + L.list0);
  b.list[1] = (int2*)(w + L.list1);
  b.nact[0] = (int32_t*)(w + L.nact0);
  b.nact[1] = (int32_t*)(w + L.nact1);
  b.Ck = (float*)(w + L.Ck);
  b.ell = (double*)(w + L.ell);
  b.scal = (DevScalars*)(w + L.scal);
  b.nk = (long long*)(w + L.nk);
  b.sw_cnt = (int32_t*)(w + L.sw_cnt);
  b.sw_part = (SweepPart*)(w + L.sw_part);
  b.goff = (uint16_t*)(w + L.goff);
  b.dpart = (long long*)(w + L.dpart);
  b.dx2 = (double*)(w + L.dx2);
  b.Cfull = (double*)(w + L.Cfull);
  b.Bvec = (double*)(w + L.Bvec);
  b.diag = (double*)(w + L.diag);
  b.x2p = (double*)(w + L.x2p);
  b.sumr2_p = (double*)(w + L.sumr2_p);
  b.Y = (float*)(w + L.Y);

  // in-patch pixel offsets and coordinates, C order over B
  std::vector<int32_t> poff(g.P), pcoord((size_t)g.P * kMaxDim, 0);
  for (int p = 0; p < g.P; ++p) {
    int rem = p, off = 0;
    for (int d = g.ndim - 1; d >= 0; --d) {
      const int c = rem % g.B[d];
      rem /= g.B[d];
      pcoord[(size_t)p * kMaxDim + d] = c;
      off += c * g.mstride[d];
    }
    poff[p] = off;
  }
  DevScalars s0;
  std::memset(&s0, 0, sizeof s0);
  s0.gamma_s = params->gamma_s0;
  s0.gamma_eps = params->gamma_eps0;
  s0.t = 1;
  s0.problem_id = params->problem_id;
  std::vector<double> ell(g.K, g.K > 1 ? std::log(params->a / g.K) -
                                           std::log(params->b * (g.K - 1) / g.K)
                                     : 0.0);
  if (hipMemcpyAsync(b.poff, poff.data(), 4 * poff.size(), hipMemcpyHostToDevice, h->st) != hipSuccess ||
      hipMemcpyAsync(b.pcoord, pcoord.data(), 4 * pcoord.size(), hipMemcpyHostToDevice, h->st) != hipSuccess ||
      hipMemcpyAsync(b.scal, &s0, sizeof s0, hipMemcpyHostToDevice, h->st) != hipSuccess ||
      hipMemcpyAsync(b.ell, ell.data(), 8 * ell.size(), hipMemcpyHostToDevice, h->st) != hipSuccess ||
      hipMemsetAsync(b.sw_cnt, 0, 4 * (size_t)g.K, h->st) != hipSuccess ||
      hipMemsetAsync(b.perm, 0, 4 * (size_t)L.Npad, h->st) != hipSuccess ||
      hipStreamSynchronize(h->st) != hipSuccess)
    return bail(fail(BPFA_EDEVICE, "initial uploads failed"));
  if ((r = clear_codes(h)) != BPFA_OK) return bail(r);
  if (launch_init_dict(g, b, h->key0, h->key1, stream_word(7, params->problem_id), h->st) !=
          hipSuccess ||
      launch_ck(g, b, h->st) != hipSuccess)
    return bail(fail(BPFA_EDEVICE, "initial kernels failed to launch"));
  if ((r = load_frame(h, image, mask, mem, false)) != BPFA_OK) return bail(r);
  if (hipStreamSynchronize(h->st) != hipSuccess)
    return bail(fail(BPFA_EDEVICE, "create: stream synchronisation failed"));
  *out = h;
  return BPFA_OK;
}

bpfa_status bpfa_set_frame(bpfa_t h, const float* image, const uint8_t* mask, bpfa_mem mem,
                           int reset_codes) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  DeviceGuard dg(h->prm.device);
  h->mean_count = 0;
  return load_frame(h, image, mask, mem, reset_codes == 0);
}

bpfa_status bpfa_reset_state(bpfa_t h) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  DeviceGuard dg(h->prm.device);
  const Geom& g = h->g;
  const double ell0 =
      g.K > 1 ? std::log(h->prm.a / g.K) - std::log(h->prm.b * (g.K - 1) / g.K) : 0.0;
  HIPCHK(launch_reset_scalars(g, h->b, ell0, h->prm.gamma_s0, h->prm.gamma_eps0, h->st));
  HIPCHK(launch_init_dict(g, h->b, h->key0, h->key1, stream_word(7, h->prm.problem_id), h->st));
  HIPCHK(launch_ck(g, h->b, h->st));
  h->t_host = 1;
  h->mean_count = 0;
  h->batch_cursor = 0;
  return clear_codes(h);
}

bpfa_status bpfa_iterate(bpfa_t h, int32_t n_iters, uint32_t flags) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  if (n_iters < 0) return fail(BPFA_EINVAL, "n_iters < 0");
  bpfa_status r = check_iter_flags(h, flags);
  if (r != BPFA_OK) return r;
  const int learn = (flags & BPFA_SPARSE_CODE_ONLY) ? 0 : 1;
  DeviceGuard dg(h->prm.device);
  for (int it = 0; it < n_iters; ++it)
    if ((r = run_step(h, learn, -1)) != BPFA_OK) return r;
  return BPFA_OK;
}

bpfa_status bpfa_minibatch(bpfa_t h, int32_t n_batches, int32_t n_steps, uint32_t flags) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  if (n_steps < 0) return fail(BPFA_EINVAL, "n_steps < 0");
  if (n_batches < 1 || n_batches > kMaxBatches || n_batches > h->g.N)
    return fail(BPFA_EINVAL, "n_batches must be 1..min(%d, N = %d), got %d", kMaxBatches, h->g.N,
                n_batches);
  bpfa_status r = check_iter_flags(h, flags);
  if (r != BPFA_OK) return r;
  const int learn = (flags & BPFA_SPARSE_CODE_ONLY) ? 0 : 1;
  DeviceGuard dg(h->prm.device);
  if (n_batches != h->n_batches) {
    h->frame_ok = false;   // until the new slot order is whole
    if ((r = order_slots(h, n_batches, true)) != BPFA_OK) return r;
    h->frame_ok = true;
  } else if (!h->plan_known && (r = read_plan(h)) != BPFA_OK) {
    return r;
  }
  for (int st = 0; st < n_steps; ++st) {
    if ((r = run_step(h, learn, h->batch_cursor)) != BPFA_OK) return r;
    h->batch_cursor = (h->batch_cursor + 1) % h->n_batches;
  }
  return BPFA_OK;
}

bpfa_status bpfa_reconstruct(bpfa_t h, float* out, bpfa_mem mem) {
  if (!h || !out) return fail(BPFA_EINVAL, "NULL handle or output");
  DeviceGuard dg(h->prm.device);
  float* dst = mem == BPFA_DEVICE ? out : (float*)(h->ws + h->L.recon);
  std::array<hipEvent_t, 2> ev{};
  bpfa_status r;
  if (h->timing && (r = record(h, &ev[0])) != BPFA_OK) return r;
  HIPCHK(launch_recon(h->g, h->b, h->cur, h->L.Npad, dst, h->precision == BPFA_BF16, h->st));
  if (h->timing) {
    if ((r = record(h, &ev[1])) != BPFA_OK) return r;
    h->recon_events.push_back(ev);
  }
  if (mem == BPFA_HOST) {
    HIPCHK(hipMemcpyAsync(out, dst, 4 * (size_t)h->g.Mtot, hipMemcpyDeviceToHost, h->st));
    return check_status(h);
  }
  return BPFA_OK;
}

bpfa_status bpfa_mean_reset(bpfa_t h) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  h->mean_count = 0;
  return BPFA_OK;
}

bpfa_status bpfa_mean_accumulate(bpfa_t h) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  DeviceGuard dg(h->prm.device);
  float* x = (float*)(h->ws + h->L.recon);
  HIPCHK(launch_recon(h->g, h->b, h->cur, h->L.Npad, x, h->precision == BPFA_BF16, h->st));
  HIPCHK(launch_mean_add(h->g.Mtot, x, (double*)(h->ws + h->L.mean), (double*)(h->ws + h->L.mean2),
                         h->mean_count == 0, h->st));
  ++h->mean_count;
  return BPFA_OK;
}

bpfa_status bpfa_mean_get(bpfa_t h, float* out, bpfa_mem mem, int64_t* count) {
  if (!h || !out) return fail(BPFA_EINVAL, "NULL handle or output");
  if (h->mean_count == 0) return fail(BPFA_ESTATE, "no sample accumulated for the posterior mean");
  DeviceGuard dg(h->prm.device);
  float* dst = mem == BPFA_DEVICE ? out : (float*)(h->ws + h->L.recon);
  HIPCHK(launch_mean_get(h->g.Mtot, (const double*)(h->ws + h->L.mean), (double)h->mean_count, dst,
                         h->st));
  if (count) *count = h->mean_count;
  if (mem == BPFA_HOST) {
    HIPCHK(hipMemcpyAsync(out, dst, 4 * (size_t)h->g.Mtot, hipMemcpyDeviceToHost, h->st));
    return check_status(h);
  }
  return BPFA_OK;
}

bpfa_status bpfa_variance_get(bpfa_t h, float* out, bpfa_mem mem, int64_t* count) {
  if (!h || !out) return fail(BPFA_EINVAL, "NULL handle or output");
  if (h->mean_count < 2) return fail(BPFA_ESTATE, "the variance needs two accumulated samples");
  DeviceGuard dg(h->prm.device);
  float* dst = mem == BPFA_DEVICE ? out : (float*)(h->ws + h->L.recon);
  HIPCHK(launch_variance_get(h->g.Mtot, (const double*)(h->ws + h->L.mean),
                             (const double*)(h->ws + h->L.mean2), (double)h->mean_count, dst, h->st));
  if (count) *count = h->mean_count;
  if (mem == BPFA_HOST) {
    HIPCHK(hipMemcpyAsync(out, dst, 4 * (size_t)h->g.Mtot, hipMemcpyDeviceToHost, h->st));
    return check_status(h);
  }
  return BPFA_OK;
}

bpfa_status bpfa_set_precision(bpfa_t h, uint32_t precision) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  if (precision != BPFA_FP32 && precision != BPFA_BF16) return fail(BPFA_EINVAL, "unknown precision");
  if (precision == BPFA_BF16 && h->g.P > 256)
    return fail(BPFA_ESHAPE, "the BF16 form takes patches of at most 256 pixels (P = %d)", h->g.P);
  h->precision = (int)precision;
  return BPFA_OK;
}

bpfa_status bpfa_transfer_dictionary(bpfa_t dst, bpfa_t src, uint32_t what) {
  if (!dst || !src) return fail(BPFA_EINVAL, "NULL handle");
  if (what & ~(uint32_t)(BPFA_XFER_D | BPFA_XFER_PI | BPFA_XFER_GAMMAS))
    return fail(BPFA_EINVAL, "unknown transfer selector 0x%x", what);
  if (dst->g.P != src->g.P || dst->g.K != src->g.K)
    return fail(BPFA_ESHAPE, "transfer needs equal P and K (dst %d/%d, src %d/%d)", dst->g.P,
                dst->g.K, src->g.P, src->g.K);
  DeviceGuard dg(dst->prm.device);
  if (dst == src) return BPFA_OK;
  hipEvent_t ev;
  HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ev, src->st));
  HIPCHK(hipStreamWaitEvent(dst->st, ev, 0));
  HIPCHK(hipEventDestroy(ev));
  const Geom& g = dst->g;
  if (what & BPFA_XFER_D)
    HIPCHK(hipMemcpyAsync(dst->b.D, src->b.D, 4 * (size_t)g.K * g.P, hipMemcpyDeviceToDevice, dst->st));
  if (what & BPFA_XFER_PI)
    HIPCHK(hipMemcpyAsync(dst->b.ell, src->b.ell, 8 * (size_t)g.K, hipMemcpyDeviceToDevice, dst->st));
  if (what & BPFA_XFER_GAMMAS)
    HIPCHK(hipMemcpyAsync(&dst->b.scal->gamma_s, &src->b.scal->gamma_s, 2 * sizeof(double),
                          hipMemcpyDeviceToDevice, dst->st));
  HIPCHK(launch_ck(g, dst->b, dst->st));
  // src must not be modified before the copies have read it
  HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ev, dst->st));
  HIPCHK(hipStreamWaitEvent(src->st, ev, 0));
  HIPCHK(hipEventDestroy(ev));
  return BPFA_OK;
}

bpfa_status bpfa_get_state(bpfa_t h, bpfa_state_view* v) {
  if (!h || !v) return fail(BPFA_EINVAL, "NULL handle or view");
  DeviceGuard dg(h->prm.device);
  const Geom& g = h->g;
  const hipMemcpyKind kind = v->mem == BPFA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (v->D) HIPCHK(hipMemcpyAsync(v->D, h->b.D, 4 * (size_t)g.K * g.P, kind, h->st));
  if (v->logit_pi) HIPCHK(hipMemcpyAsync(v->logit_pi, h->b.ell, 8 * (size_t)g.K, kind, h->st));
  if (v->W || v->Z) {
    float* W = v->W;
    uint8_t* Z = v->Z;
    void* tmp = nullptr;
    const size_t nk = (size_t)g.N * g.K;
    if (v->mem == BPFA_HOST) {
      HIPCHK(hipMallocAsync(&tmp, 5 * nk, h->st));
      W = v->W ? (float*)tmp : nullptr;
      Z = v->Z ? (uint8_t*)tmp + 4 * nk : nullptr;
    }
    HIPCHK(launch_lists_to_dense(g, h->b, h->cur, W, Z, h->st));
    if (v->mem == BPFA_HOST) {
      if (v->W) HIPCHK(hipMemcpyAsync(v->W, W, 4 * nk, hipMemcpyDeviceToHost, h->st));
      if (v->Z) HIPCHK(hipMemcpyAsync(v->Z, Z, nk, hipMemcpyDeviceToHost, h->st));
      HIPCHK(hipFreeAsync(tmp, h->st));
    }
  }
  DevScalars s;
  HIPCHK(hipMemcpyAsync(&s, h->b.scal, sizeof s, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  v->gamma_s = s.gamma_s;
  v->gamma_eps = s.gamma_eps;
  v->t = s.t;
  return check_status(h);
}

bpfa_status bpfa_set_state(bpfa_t h, const bpfa_state_view* v) {
  return set_state_impl(h, v, nullptr);
}

bpfa_status bpfa_set_state_noalloc(bpfa_t h, const bpfa_state_view* v) {
  if (!h || !v) return fail(BPFA_EINVAL, "NULL handle or view");
  DeviceGuard dg(h->prm.device);
  if (!dg.ok) return fail(BPFA_EDEVICE, "cannot select device %d", h->prm.device);
  char* base = nullptr;
  bpfa_status r = scratch_base(h->prm.device, &base);
  if (r != BPFA_OK) return r;
  return set_state_impl(h, v, base);
}

bpfa_status bpfa_get_stats(bpfa_t h, bpfa_stats* out) {
  if (!h || !out) return fail(BPFA_EINVAL, "NULL handle or stats");
  DeviceGuard dg(h->prm.device);
  DevScalars s;
  HIPCHK(hipMemcpyAsync(&s, h->b.scal, sizeof s, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  bpfa_status r = collect_timing(h);
  if (r != BPFA_OK) return r;
  std::memset(out, 0, sizeof *out);
  out->t = s.t;
  out->N = h->g.N;
  out->P = h->g.P;
  out->K = h->g.K;
  out->n_obs = s.n_obs;
  out->sum_z = s.sum_z;
  out->mean_active = (double)s.sum_z / h->g.N;
  out->gamma_s = s.gamma_s;
  out->gamma_eps = s.gamma_eps;
  out->pi_min = s.pi_min;
  out->pi_mean = s.pi_mean;
  out->pi_max = s.pi_max;
  out->sum_w2 = s.sum_w2;
  out->sum_r2 = s.sum_r2_used;
  out->max_obs = h->max_obs;
  out->timing = h->timing ? 1 : 0;
  out->ms_index = h->ms_index;
  out->ms_sweep = h->ms_sweep;
  out->ms_dict = h->ms_dict;
  out->ms_dict_stats = h->ms_dict_stats;
  out->ms_scalars = h->ms_scalars;
  out->ms_recon = h->ms_recon;
  out->n_sweeps = h->n_sweeps;
  return check_status(h);
}

bpfa_status bpfa_set_timing(bpfa_t h, int on) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  DeviceGuard dg(h->prm.device);
  HIPCHK(hipStreamSynchronize(h->st));
  bpfa_status r = collect_timing(h);
  if (r != BPFA_OK) return r;
  h->timing = on != 0;
  // events for the records of ~20 frames of 20 iterations, so that timed
  // frames create none
  while (h->timing && h->event_pool.size() < 3072) {
    hipEvent_t ev;
    HIPCHK(create_timing_event(&ev));
    h->event_pool.push_back(ev);
  }
  h->ms_index = h->ms_sweep = h->ms_dict = h->ms_dict_stats = h->ms_scalars = h->ms_recon = 0.0;
  h->n_sweeps = 0;
  return BPFA_OK;
}

bpfa_status bpfa_sync(bpfa_t h) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  DeviceGuard dg(h->prm.device);
  return check_status(h);
}

bpfa_status bpfa_get_patch_index(bpfa_t h, uint32_t* obs_bits, int32_t* obs_count, bpfa_mem mem) {
  if (!h) return fail(BPFA_EINVAL, "NULL handle");
  DeviceGuard dg(h->prm.device);
  const hipMemcpyKind kind = mem == BPFA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (obs_bits)
    HIPCHK(hipMemcpyAsync(obs_bits, h->b.obs_bits, 4 * (size_t)h->g.N * h->g.PW, kind, h->st));
  if (obs_count)
    HIPCHK(hipMemcpyAsync(obs_count, h->b.obs_count, 4 * (size_t)h->g.N, kind, h->st));
  if (mem == BPFA_HOST) HIPCHK(hipStreamSynchronize(h->st));
  return BPFA_OK;
}

bpfa_status bpfa_debug_philox(int32_t device, uint64_t seed, uint32_t problem_id, uint32_t tag,
                              const uint32_t* c0, uint32_t c1, uint32_t t, int64_t n,
                              uint32_t* out, bpfa_mem mem) {
  if (n < 0 || (n > 0 && (!c0 || !out))) return fail(BPFA_EINVAL, "bad arguments");
  if (problem_id >= (1u << 24)) return fail(BPFA_EINVAL, "problem_id must fit 24 bits");
  DeviceGuard dg(device);
  if (!dg.ok) return fail(BPFA_EDEVICE, "cannot select device %d", device);
  if (n == 0) return BPFA_OK;
  const uint32_t* dc0 = c0;
  uint32_t* dout = out;
  void* tmp = nullptr;
  if (mem == BPFA_HOST) {
    HIPCHK(hipMalloc(&tmp, 20 * (size_t)n));
    HIPCHK(hipMemcpy(tmp, c0, 4 * (size_t)n, hipMemcpyHostToDevice));
    dc0 = (const uint32_t*)tmp;
    dout = (uint32_t*)((char*)tmp + 4 * (size_t)n);
  }
  hipError_t e = launch_debug_philox((uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), c1, t,
                                     stream_word(tag, problem_id), dc0, n, dout, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess && mem == BPFA_HOST) e = hipMemcpy(out, dout, 16 * (size_t)n, hipMemcpyDeviceToHost);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return fail(BPFA_EDEVICE, "debug_philox: %s", hipGetErrorString(e));
  return BPFA_OK;
}

void bpfa_destroy(bpfa_t h) {
  if (!h) return;
  DeviceGuard dg(h->prm.device);
  if (h->st) (void)hipStreamSynchronize(h->st);
  (void)collect_timing(h);
  for (auto ev : h->event_pool) (void)hipEventDestroy(ev);
  if (h->own_ws && h->ws) (void)hipFree(h->ws);
  if (h->own_stream && h->st) (void)hipStreamDestroy(h->st);
  if (h->stage) (void)hipHostFree(h->stage);
  delete h;
}

const char* bpfa_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace bpfa {

size_t dict_blob_bytes(int K, int P) { return (size_t)4 * K * P + (size_t)8 * K + 16; }

int problem_dims(bpfa_problem* h, int* K, int* P) {
  *K = h->g.K;
  *P = h->g.P;
  return BPFA_OK;
}

int problem_set_id(bpfa_problem* h, uint32_t problem_id) {
  DeviceGuard dg(h->prm.device);
  h->prm.problem_id = problem_id;
  HIPCHK(launch_set_t(h->b.scal, 0, problem_id, h->st, false));
  return BPFA_OK;
}

int problem_export_dict(bpfa_problem* h, void* blob) {
  DeviceGuard dg(h->prm.device);
  const Geom& g = h->g;
  char* b = (char*)blob;
  HIPCHK(hipMemcpyAsync(b, h->b.D, 4 * (size_t)g.K * g.P, hipMemcpyDeviceToDevice, h->st));
  b += 4 * (size_t)g.K * g.P;
  HIPCHK(hipMemcpyAsync(b, h->b.ell, 8 * (size_t)g.K, hipMemcpyDeviceToDevice, h->st));
  b += 8 * (size_t)g.K;
  HIPCHK(hipMemcpyAsync(b, &h->b.scal->gamma_s, 16, hipMemcpyDeviceToDevice, h->st));
  return BPFA_OK;
}

int problem_import_dict(bpfa_problem* h, const void* blob, long long t, uint32_t problem_id) {
  DeviceGuard dg(h->prm.device);
  const Geom& g = h->g;
  const char* b = (const char*)blob;
  HIPCHK(hipMemcpyAsync(h->b.D, b, 4 * (size_t)g.K * g.P, hipMemcpyDeviceToDevice, h->st));
  b += 4 * (size_t)g.K * g.P;
  HIPCHK(hipMemcpyAsync(h->b.ell, b, 8 * (size_t)g.K, hipMemcpyDeviceToDevice, h->st));
  b += 8 * (size_t)g.K;
  HIPCHK(hipMemcpyAsync(&h->b.scal->gamma_s, b, 16, hipMemcpyDeviceToDevice, h->st));
  // a new frame of the stream: its counter and id, and no failure recorded yet
  HIPCHK(launch_set_t(h->b.scal, t, problem_id, h->st, true));
  HIPCHK(launch_ck(g, h->b, h->st));
  h->prm.problem_id = problem_id;
  h->t_host = t;
  return BPFA_OK;
}

int problem_upload_frame(bpfa_problem* h, const float* image, const uint8_t* mask) {
  DeviceGuard dg(h->prm.device);
  const Geom& g = h->g;
  HIPCHK(hipMemcpyAsync(h->b.image, image, 4 * (size_t)g.Mtot, hipMemcpyHostToDevice, h->st));
  HIPCHK(hipMemcpyAsync(h->b.mask, mask, (size_t)g.Mtot, hipMemcpyHostToDevice, h->st));
  return BPFA_OK;
}

int problem_frame_body(bpfa_problem* h, int sc_iters, int learn, int var_samples) {
  DeviceGuard dg(h->prm.device);
  if (h->timing) return fail(BPFA_ESTATE, "a served frame runs without per-phase timing");
  if (h->n_batches != 1) return fail(BPFA_ESTATE, "a served frame runs full-batch iterations");
  bpfa_status r = index_frame(h, false, false);
  if (r != BPFA_OK) return r;
  const int n_it = sc_iters + (learn ? 1 : 0);
  const int V = std::min(var_samples, n_it);
  float* x = (float*)(h->ws + h->L.recon);
  double* s1 = (double*)(h->ws + h->L.mean);
  double* s2 = (double*)(h->ws + h->L.mean2);
  for (int it = 0; it < n_it; ++it) {
    if ((r = run_step(h, it < sc_iters ? 0 : 1, -1)) != BPFA_OK) return r;
    // the last V samples: their reconstructions into the binary64 moment
    // sums (the last one is the frame's result)
    if (V >= 2 && it >= n_it - V) {
      HIPCHK(launch_recon(h->g, h->b, h->cur, h->L.Npad, x, h->precision == BPFA_BF16, h->st));
      HIPCHK(launch_mean_add(h->g.Mtot, x, s1, s2, it == n_it - V, h->st));
    }
  }
  if (V >= 2) {
    HIPCHK(launch_variance_get(h->g.Mtot, s1, s2, (double)V, (float*)(h->ws + h->L.var), h->st));
  } else {
    HIPCHK(launch_recon(h->g, h->b, h->cur, h->L.Npad, x, h->precision == BPFA_BF16, h->st));
  }
  h->mean_count = 0;   // the moment sums hold a frame's samples, not the caller's mean
  return BPFA_OK;
}

int problem_upload_image(bpfa_problem* h, const float* image) {
  DeviceGuard dg(h->prm.device);
  HIPCHK(hipMemcpyAsync(h->b.image, image, 4 * (size_t)h->g.Mtot, hipMemcpyHostToDevice, h->st));
  return BPFA_OK;
}

int problem_acquire(bpfa_problem* h, const AcqArgs& a, int kind, const float* weights) {
  DeviceGuard dg(h->prm.device);
  const Geom& g = h->g;
  int64_t shape[kMaxDim];
  for (int d = 0; d < g.ndim; ++d) shape[d] = g.M[d];
  AcqArgs aa = a;
  aa.M = g.Mtot;
  HIPCHK(launch_acquire(aa, kind, g.ndim, shape, weights, (double*)(h->ws + h->L.wsum), h->b.mask,
                        h->st));
  return BPFA_OK;
}

const float* problem_variance(bpfa_problem* h) { return (const float*)(h->ws + h->L.var); }
const uint8_t* problem_mask(bpfa_problem* h) { return h->b.mask; }

int problem_frame_result(bpfa_problem* h, float* out) {
  DeviceGuard dg(h->prm.device);
  DevScalars* sp = reinterpret_cast<DevScalars*>(h->stage);
  FramePlan* fp = reinterpret_cast<FramePlan*>(h->stage + align_up(sizeof(DevScalars), 16));
  HIPCHK(hipMemcpyAsync(out, h->ws + h->L.recon, 4 * (size_t)h->g.Mtot, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipMemcpyAsync(sp, h->b.scal, sizeof(DevScalars), hipMemcpyDeviceToHost, h->st));
  // the plan's leading scalars (through `bad`)
  HIPCHK(hipMemcpyAsync(fp, h->b.plan, offsetof(FramePlan, dict_chunks), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  h->t_host = sp->t;
  h->max_obs = sp->max_obs;
  h->n_omega = sp->n_omega;
  if (fp->bad) {
    h->frame_ok = false;
    return fail(BPFA_ESHAPE, "a patch has %d observed pixels; at most 256 are supported", sp->max_obs);
  }
  if (sp->status)
    return fail(BPFA_ENUMERIC, "numeric failure in an iteration (flags %d)", sp->status);
  return BPFA_OK;
}

hipStream_t problem_stream(bpfa_problem* h) { return h->st; }

}  // namespace bpfa
