// Serving engine of libbpfa: the C ABI declared in include/bpfa_serve.h.
//
// Frames wait in per-stream FIFOs.  A dispatcher thread admits the oldest
// frame whose stream is idle as soon as a slot of its shape is free; slots
// (a problem handle with its own HIP stream and workspace) are created while
// the HBM budget allows and idle slots of other shapes are evicted to make
// room.  One worker thread per slot runs a frame: upload the frame, load the
// stream's dictionary state, then the frame body -- patch index,
// sparse-coding iterations (plus one dictionary iteration every
// dict_every-th frame), the reconstruction -- then save the state into the
// stream's second blob and copy the reconstruction into the caller's buffer.
// Nothing in the body depends on host knowledge of the frame (the per-frame
// plan lives on the device), so after the first frame of each kind a slot
// captures the body into a HIP graph and replays it for every later frame
// of that kind: one launch instead of ~40, and no host round trip between
// upload and result.  Slots work on separate streams, so frames of different
// feed streams overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bpfa_serve.h"
#include "internal.hpp"
#include "philox.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Frame {
  uint64_t ticket = 0;
  int stream = 0;
  std::vector<int64_t> shape;
  int64_t pixels = 0;
  float* img = nullptr;       // pinned copies of the caller's inputs
  uint8_t* mask = nullptr;
  float* out = nullptr;       // caller's host buffer
  Clock::time_point submit_t, admit_t;
  int64_t frame_index = 0;
  long long t0 = 1;           // first Philox iteration number of this frame
  bool learn = false;
  bool scene = false;         // the stream's policy draws the mask (img is the scene)
  uint8_t* mask_out = nullptr;  // caller's host buffer for the drawn mask, or NULL
};

struct Slot {
  std::vector<int64_t> shape;
  bpfa_t h = nullptr;
  size_t bytes = 0;
  // the frame body as a replayable graph per kind of frame (0: sparse coding
  // only, 1: with the dictionary iteration); the first frame of a kind runs
  // uncaptured, the second is captured
  // [learn][variance kept]
  hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int runs[2][2] = {{0, 0}, {0, 0}};
  bool graphs_ok = true;      // a capture failed: this slot runs uncaptured from then on
  int64_t graph_frames = 0, captures = 0;
  bool busy = false;
  bool stop = false;
  Frame* job = nullptr;
  std::thread worker;
  std::condition_variable cv;
};

struct StreamState {
  void* blob = nullptr;       // device: D, logit pi, gammas
  void* pending = nullptr;    // device: where a frame saves its state until it is known good
  bpfa_acq_policy pol{};      // acquisition policy (kind BPFA_ACQ_CALLER: the caller's masks)
  // targeted policy: the posterior variance of the last good frame (weights)
  // and of the frame in flight (pending), device, both of shape wshape
  float* weights = nullptr;
  float* wpending = nullptr;
  size_t wcap = 0;            // floats each weight buffer holds
  std::vector<int64_t> wshape;
  bool wvalid = false;
  long long t = 1;
  int64_t frames = 0;
  bool busy = false;
  std::deque<Frame*> fifo;
};

}  // namespace

struct bpfa_server {
  bpfa_server_params prm{};
  int K = 0, P = 0;
  std::mutex mu;
  std::condition_variable cv_disp, cv_done;
  std::vector<StreamState> streams;
  std::vector<Slot*> slots;
  std::vector<bpfa_serve_result> results;
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, failed = 0, in_flight = 0, queued = 0;
  int64_t slot_bytes = 0, peak_slot_bytes = 0, creations = 0, evictions = 0;
  int64_t graph_frames = 0, captures = 0;   // of destroyed slots (live slots keep their own)
  bool stopping = false;
  std::thread dispatcher;
};

namespace {

bpfa_params frame_params(const bpfa_server_params& s, const std::vector<int64_t>& shape) {
  bpfa_params p;
  bpfa_params_default(&p);
  p.ndim = s.ndim;
  for (int d = 0; d < 4; ++d) {
    p.shape[d] = d < s.ndim ? shape[d] : 0;
    p.patch[d] = s.patch[d];
    p.stride[d] = s.stride[d];
  }
  p.K = s.K;
  p.a = s.a;
  p.b = s.b;
  p.c = s.c;
  p.d = s.d;
  p.e = s.e;
  p.f = s.f;
  p.gamma_s0 = s.gamma_s0;
  p.gamma_eps0 = s.gamma_eps0;
  p.seed = s.seed;
  p.device = s.device;
  p.stream = nullptr;   // each slot owns a stream
  return p;
}

void finish(bpfa_server* s, Frame* f, int status, bool learned) {
  bpfa_serve_result r{};
  r.ticket = f->ticket;
  r.stream = f->stream;
  r.status = status;
  r.frame_index = f->frame_index;
  r.pixels = f->pixels;
  const Clock::time_point now = Clock::now();
  r.latency_ms = ms_between(f->submit_t, now);
  r.queue_ms = ms_between(f->submit_t, status == BPFA_OK ? f->admit_t : now);
  r.learned = learned ? 1 : 0;
  s->results.push_back(r);
  if (status == BPFA_OK) ++s->completed;
  else ++s->failed;
  (void)hipHostFree(f->img);
  if (f->mask) (void)hipHostFree(f->mask);
  delete f;
}

// The frame body on the slot's stream: replayed from the slot's graph for this
// kind of frame when one is captured; otherwise run directly, and captured
// on the way when this kind has run once before (the direct run also sets
// the kernels' launch attributes) and graphs are on.  A capture that fails
// leaves the slot on direct runs.
int run_body(bpfa_server* s, Slot* sl, int learn, int var_samples) {
  bpfa_t h = sl->h;
  const int sc = s->prm.sc_iters;
  const int kv = var_samples >= 2 ? 1 : 0;
  hipStream_t hs = bpfa::problem_stream(h);
  hipGraphExec_t& exec = sl->exec[learn][kv];
  if (exec) {
    ++sl->graph_frames;
    return hipGraphLaunch(exec, hs) == hipSuccess ? BPFA_OK : BPFA_EDEVICE;
  }
  const bool capture = s->prm.use_graphs && sl->graphs_ok && sl->runs[learn][kv] >= 1;
  ++sl->runs[learn][kv];
  if (!capture) return bpfa::problem_frame_body(h, sc, learn, var_samples);
  if (hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    sl->graphs_ok = false;
    (void)hipGetLastError();
    return bpfa::problem_frame_body(h, sc, learn, var_samples);
  }
  const int st = bpfa::problem_frame_body(h, sc, learn, var_samples);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(hs, &graph);
  hipGraphExec_t ex = nullptr;
  const bool ok = st == BPFA_OK && e == hipSuccess && graph != nullptr &&
                  hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) == hipSuccess;
  if (graph) (void)hipGraphDestroy(graph);
  if (!ok) {
    (void)hipGetLastError();
    sl->graphs_ok = false;
    return bpfa::problem_frame_body(h, sc, learn, var_samples);
  }
  exec = ex;
  ++sl->captures;
  ++sl->graph_frames;
  return hipGraphLaunch(ex, hs) == hipSuccess ? BPFA_OK : BPFA_EDEVICE;
}

// one frame on a slot (called by the slot's worker without the server lock).
// The updated state goes to the stream's pending blob (outside the graph:
// the blobs belong to streams, a slot serves any stream); the caller swaps
// it in as the stream's state only when the frame succeeded, so a frame that
// was refused (ESHAPE) or whose draws failed (ENUMERIC) leaves the stream at
// its last good state and iteration.
int run_frame(bpfa_server* s, Slot* sl, Frame* f, StreamState* ss) {
  bpfa_t h = sl->h;
  hipStream_t hs = bpfa::problem_stream(h);
  const bpfa_acq_policy& pol = ss->pol;
  const bool targeted = pol.kind == BPFA_ACQ_TARGETED;
  int st;
  if (f->scene) {
    // the policy's mask for this frame of the stream, drawn on the device
    st = bpfa::problem_upload_image(h, f->img);
    if (st != BPFA_OK) return st;
    bpfa::AcqArgs a{};
    a.rho = pol.fraction;
    a.share = pol.targeted_share;
    a.key0 = (uint32_t)(s->prm.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(s->prm.seed >> 32);
    a.frame = (uint32_t)f->frame_index;
    a.stream_word = bpfa::kTagAcq | ((uint32_t)f->stream << 8);
    const float* w = targeted && ss->wvalid && ss->wshape == f->shape ? ss->weights : nullptr;
    st = bpfa::problem_acquire(h, a, pol.kind, w);
  } else {
    st = bpfa::problem_upload_frame(h, f->img, f->mask);
  }
  if (st != BPFA_OK) return st;
  st = bpfa::problem_import_dict(h, ss->blob, f->t0, (uint32_t)f->stream);
  if (st != BPFA_OK) return st;
  st = run_body(s, sl, f->learn ? 1 : 0, targeted ? pol.var_samples : 0);
  if (st == BPFA_OK) st = bpfa::problem_export_dict(h, ss->pending);
  if (st == BPFA_OK && targeted) {
    // the frame's variance steers the stream's next frame once the frame is good
    const size_t px = (size_t)f->pixels;
    if (ss->wcap < px) {
      (void)hipStreamSynchronize(hs);
      (void)hipFree(ss->weights);
      (void)hipFree(ss->wpending);
      ss->weights = ss->wpending = nullptr;
      ss->wcap = 0;
      ss->wvalid = false;
      if (hipMalloc((void**)&ss->weights, 4 * px) != hipSuccess ||
          hipMalloc((void**)&ss->wpending, 4 * px) != hipSuccess)
        st = BPFA_ENOMEM;
      else
        ss->wcap = px;
    }
    if (st == BPFA_OK &&
        hipMemcpyAsync(ss->wpending, bpfa::problem_variance(h), 4 * px, hipMemcpyDeviceToDevice, hs) !=
            hipSuccess)
      st = BPFA_EDEVICE;
  }
  if (st == BPFA_OK && f->mask_out &&
      hipMemcpyAsync(f->mask_out, bpfa::problem_mask(h), (size_t)f->pixels, hipMemcpyDeviceToHost, hs) !=
          hipSuccess)
    st = BPFA_EDEVICE;
  if (st != BPFA_OK) {
    (void)hipStreamSynchronize(hs);   // the frame's buffers stay valid until then
    return st;
  }
  // synchronises the slot's stream; reports a refused frame or a numeric
  // failure of any iteration of this frame
  return bpfa::problem_frame_result(h, f->out);
}

void worker_loop(bpfa_server* s, Slot* sl) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    sl->cv.wait(lk, [&] { return sl->stop || sl->job != nullptr; });
    if (sl->job == nullptr && sl->stop) return;
    Frame* f = sl->job;
    StreamState* ss = &s->streams[f->stream];
    lk.unlock();
    const int st = run_frame(s, sl, f, ss);
    lk.lock();
    const bool learned = f->learn;
    if (st == BPFA_OK) {
      std::swap(ss->blob, ss->pending);   // the frame's state becomes the stream's
      if (ss->pol.kind == BPFA_ACQ_TARGETED) {
        std::swap(ss->weights, ss->wpending);
        ss->wshape = f->shape;
        ss->wvalid = true;
      }
      ss->t = f->t0 + s->prm.sc_iters + (learned ? 1 : 0);
    }
    ss->busy = false;
    sl->busy = false;
    sl->job = nullptr;
    --s->in_flight;
    finish(s, f, st, learned);
    s->cv_disp.notify_all();
    s->cv_done.notify_all();
  }
}

void destroy_slot(Slot* sl) {
  if (sl->worker.joinable()) sl->worker.join();
  for (auto& row : sl->exec)
    for (auto& ex : row)
      if (ex) (void)hipGraphExecDestroy(ex);
  if (sl->h) bpfa_destroy(sl->h);
  delete sl;
}

// called with the lock held; may release it while creating a slot
// *fail_status != OK: the frame cannot run (larger than the whole budget, or
// the slot could not be built); nullptr with OK: wait for a slot to free up
Slot* acquire_slot(bpfa_server* s, const std::vector<int64_t>& shape, size_t need,
                   std::unique_lock<std::mutex>& lk, int* fail_status) {
  *fail_status = need > s->prm.hbm_budget ? BPFA_ENOMEM : BPFA_OK;
  if (*fail_status != BPFA_OK) return nullptr;
  for (Slot* sl : s->slots)
    if (!sl->busy && sl->shape == shape) return sl;
  // evict only when that makes room: the idle slots of other shapes together
  // must free enough bytes and slot count, or nothing is evicted and the frame
  // waits (the dispatcher then tries other streams' frames)
  {
    int64_t idle_bytes = 0;
    int idle_n = 0;
    for (Slot* x : s->slots)
      if (!x->busy && x->shape != shape) {
        idle_bytes += (int64_t)x->bytes;
        ++idle_n;
      }
    if ((uint64_t)(s->slot_bytes - idle_bytes) + need > s->prm.hbm_budget ||
        (int)s->slots.size() - idle_n >= s->prm.max_slots)
      return nullptr;
  }
  // make room: evict idle slots of other shapes until the new one fits
  while ((uint64_t)s->slot_bytes + need > s->prm.hbm_budget ||
         (int)s->slots.size() >= s->prm.max_slots) {
    auto it = std::find_if(s->slots.begin(), s->slots.end(),
                           [&](Slot* x) { return !x->busy && x->shape != shape; });
    if (it == s->slots.end()) return nullptr;   // wait for a slot to free up
    Slot* ev = *it;
    s->slots.erase(it);
    s->slot_bytes -= (int64_t)ev->bytes;
    ++s->evictions;
    s->graph_frames += ev->graph_frames;
    s->captures += ev->captures;
    ev->stop = true;
    ev->cv.notify_all();
    lk.unlock();
    destroy_slot(ev);
    lk.lock();
  }
  Slot* sl = new Slot();
  sl->shape = shape;
  sl->bytes = need;
  sl->busy = true;   // reserved while it is being built
  s->slots.push_back(sl);
  s->slot_bytes += (int64_t)need;
  s->peak_slot_bytes = std::max(s->peak_slot_bytes, s->slot_bytes);
  ++s->creations;
  lk.unlock();
  // a slot starts on an all-zero frame; every job uploads its own
  bpfa_params fp = frame_params(s->prm, shape);
  int64_t px = 1;
  for (int d = 0; d < s->prm.ndim; ++d) px *= shape[d];
  std::vector<float> zimg((size_t)px, 0.f);
  std::vector<uint8_t> zmask((size_t)px, 0);
  bpfa_t h = nullptr;
  int st = bpfa_create(&fp, nullptr, 0, zimg.data(), zmask.data(), BPFA_HOST, &h);
  if (st == BPFA_OK) st = bpfa_set_precision(h, (uint32_t)s->prm.precision);
  if (st != BPFA_OK && h) {
    bpfa_destroy(h);
    h = nullptr;
  }
  lk.lock();
  if (st != BPFA_OK) {
    s->slots.erase(std::find(s->slots.begin(), s->slots.end(), sl));
    s->slot_bytes -= (int64_t)need;
    delete sl;
    *fail_status = st;
    return nullptr;
  }
  sl->h = h;
  sl->busy = false;
  sl->worker = std::thread(worker_loop, s, sl);
  return sl;
}

void dispatcher_loop(bpfa_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progress = true;
    while (progress) {
      progress = false;
      // head-of-stream frames of idle streams, oldest first; a frame that
      // must wait for a slot does not hold back the younger ones behind it
      std::vector<Frame*> heads;
      for (auto& ss : s->streams)
        if (!ss.busy && !ss.fifo.empty()) heads.push_back(ss.fifo.front());
      std::sort(heads.begin(), heads.end(),
                [](const Frame* a, const Frame* b) { return a->ticket < b->ticket; });
      Frame* best = nullptr;
      Slot* sl = nullptr;
      for (Frame* cand : heads) {
        bpfa_params fp = frame_params(s->prm, cand->shape);
        size_t need = 0;
        if (bpfa_workspace_size(&fp, &need) != BPFA_OK) need = (size_t)-1;
        int fail_status = BPFA_OK;
        Slot* got = acquire_slot(s, cand->shape, need, lk, &fail_status);
        if (fail_status != BPFA_OK) {
          StreamState& fs = s->streams[cand->stream];
          fs.fifo.pop_front();
          --s->queued;
          finish(s, cand, fail_status, false);
          s->cv_done.notify_all();
          progress = true;
          break;   // the lock may have been released: rescan
        }
        if (got) {
          best = cand;
          sl = got;
          break;
        }
      }
      if (progress) continue;
      if (!best) break;   // every candidate waits for a slot
      StreamState& ss = s->streams[best->stream];
      ss.fifo.pop_front();
      --s->queued;
      ss.busy = true;
      best->frame_index = ss.frames++;
      best->t0 = ss.t;
      best->learn = s->prm.dict_every > 0 && (best->frame_index + 1) % s->prm.dict_every == 0;
      best->admit_t = Clock::now();
      sl->busy = true;
      sl->job = best;
      ++s->in_flight;
      sl->cv.notify_all();
      progress = true;
    }
    if (s->stopping && s->in_flight == 0 && s->queued == 0) return;
    s->cv_disp.wait(lk);
  }
}

int64_t frame_pixels(int ndim, const int64_t* shape) {
  int64_t px = 1;
  for (int d = 0; d < ndim; ++d) px *= shape[d];
  return px;
}

}  // namespace

extern "C" {

void bpfa_server_params_default(bpfa_server_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->ndim = 2;
  for (int d = 0; d < 4; ++d) {
    p->patch[d] = d < 2 ? 10 : 1;
    p->stride[d] = 1;
  }
  p->K = 128;
  p->a = p->b = 1.0;
  p->c = p->d = p->e = p->f = 1e-6;
  p->gamma_s0 = 1.0;
  p->gamma_eps0 = 100.0;
  p->n_streams = 4;
  p->sc_iters = 5;
  p->dict_every = 10;
  p->max_slots = 4;
  p->hbm_budget = 16ull << 30;
  p->precision = BPFA_FP32;
  p->use_graphs = 1;
}

bpfa_status bpfa_server_create(const bpfa_server_params* p, bpfa_server_t* out) {
  if (!p || !out) return BPFA_EINVAL;
  *out = nullptr;
  if (p->n_streams < 1 || p->n_streams > 4096 || p->sc_iters < 1 || p->dict_every < 0 ||
      p->max_slots < 1 || p->hbm_budget == 0 ||
      (p->precision != BPFA_FP32 && p->precision != BPFA_BF16))
    return BPFA_EINVAL;
  {
    int64_t P = 1;
    for (int d = 0; d < p->ndim && d < 4; ++d) P *= p->patch[d];
    if (p->precision == BPFA_BF16 && P > 256) return BPFA_ESHAPE;   // matrix-core tiles hold 256 pixels
  }
  // validate the patch geometry and priors on the smallest frame that holds one patch
  std::vector<int64_t> probe(4, 1);
  for (int d = 0; d < p->ndim && d < 4; ++d) probe[d] = p->patch[d];
  bpfa_params fp = frame_params(*p, probe);
  size_t bytes = 0;
  bpfa_status st = bpfa_workspace_size(&fp, &bytes);
  if (st != BPFA_OK) return st;
  auto* s = new bpfa_server();
  s->prm = *p;
  s->K = p->K;
  s->P = 1;
  for (int d = 0; d < p->ndim; ++d) s->P *= (int)p->patch[d];
  s->streams.resize(p->n_streams);
  // every stream starts from the prior: build it once on a probe problem
  std::vector<float> zimg(frame_pixels(p->ndim, probe.data()), 0.f);
  std::vector<uint8_t> zmask(zimg.size(), 0);
  bpfa_t h0 = nullptr;
  st = bpfa_create(&fp, nullptr, 0, zimg.data(), zmask.data(), BPFA_HOST, &h0);
  if (st != BPFA_OK) {
    delete s;
    return st;
  }
  // stream n starts from its own prior draw (Philox stream id n), as a problem created with id n
  const size_t blob = bpfa::dict_blob_bytes(s->K, s->P);
  for (int n = 0; n < p->n_streams; ++n) {
    StreamState& ss = s->streams[n];
    bpfa::problem_set_id(h0, (uint32_t)n);
    if (hipMalloc(&ss.blob, blob) != hipSuccess || hipMalloc(&ss.pending, blob) != hipSuccess ||
        bpfa_reset_state(h0) != BPFA_OK ||
        bpfa::problem_export_dict(h0, ss.blob) != BPFA_OK) {
      bpfa_destroy(h0);
      bpfa_server_destroy(s);
      return BPFA_ENOMEM;
    }
  }
  st = bpfa_sync(h0);
  bpfa_destroy(h0);
  if (st != BPFA_OK) {
    bpfa_server_destroy(s);
    return st;
  }
  s->dispatcher = std::thread(dispatcher_loop, s);
  *out = s;
  return BPFA_OK;
}

bpfa_status bpfa_server_set_dictionary(bpfa_server_t s, int32_t stream, bpfa_t src) {
  if (!s || !src || stream < 0 || stream >= s->prm.n_streams) return BPFA_EINVAL;
  int K = 0, P = 0;
  bpfa::problem_dims(src, &K, &P);
  if (K != s->K || P != s->P) return BPFA_ESHAPE;
  std::unique_lock<std::mutex> lk(s->mu);
  StreamState& ss = s->streams[stream];
  s->cv_done.wait(lk, [&] { return !ss.busy && ss.fifo.empty(); });
  ss.busy = true;   // keep the dispatcher away while the blob changes
  lk.unlock();
  int st = bpfa::problem_export_dict(src, ss.blob);
  if (st == BPFA_OK) st = bpfa_sync(src);
  lk.lock();
  ss.frames = 0;
  ss.busy = false;
  s->cv_disp.notify_all();
  return (bpfa_status)st;
}

namespace {

// Queue a frame: mask NULL for a scene (the stream's policy draws it).
bpfa_status queue_frame(bpfa_server_t s, int32_t stream, const int64_t* shape, const float* image,
                        const uint8_t* mask, float* out, uint8_t* mask_out, uint64_t* ticket) {
  const Clock::time_point arrival = Clock::now();
  std::vector<int64_t> shp(shape, shape + s->prm.ndim);
  bpfa_params fp = frame_params(s->prm, shp);
  size_t need = 0;
  bpfa_status st = bpfa_workspace_size(&fp, &need);
  if (st != BPFA_OK) return st;
  auto* f = new Frame();
  f->stream = stream;
  f->shape = shp;
  f->pixels = frame_pixels(s->prm.ndim, shape);
  f->out = out;
  f->scene = mask == nullptr;
  f->mask_out = mask_out;
  if (hipHostMalloc((void**)&f->img, 4 * (size_t)f->pixels, hipHostMallocDefault) != hipSuccess ||
      (mask && hipHostMalloc((void**)&f->mask, (size_t)f->pixels, hipHostMallocDefault) != hipSuccess)) {
    (void)hipHostFree(f->img);
    delete f;
    return BPFA_ENOMEM;
  }
  std::memcpy(f->img, image, 4 * (size_t)f->pixels);
  if (mask) std::memcpy(f->mask, mask, (size_t)f->pixels);
  std::lock_guard<std::mutex> lk(s->mu);
  if (f->scene && s->streams[stream].pol.kind == BPFA_ACQ_CALLER) {
    (void)hipHostFree(f->img);
    delete f;
    return BPFA_EINVAL;
  }
  f->submit_t = arrival;
  f->ticket = s->next_ticket++;
  if (ticket) *ticket = f->ticket;
  s->streams[stream].fifo.push_back(f);
  ++s->submitted;
  ++s->queued;
  s->cv_disp.notify_all();
  return BPFA_OK;
}

bool policy_ok(const bpfa_acq_policy* p, int sc_iters) {
  if (!p) return false;
  if (p->kind < BPFA_ACQ_CALLER || p->kind > BPFA_ACQ_TARGETED) return false;
  if (p->kind == BPFA_ACQ_CALLER) return true;
  if (!(p->fraction > 0.0 && p->fraction <= 1.0)) return false;
  if (p->kind == BPFA_ACQ_TARGETED &&
      (!(p->targeted_share >= 0.0 && p->targeted_share <= 1.0) || p->var_samples < 2 ||
       p->var_samples > sc_iters + 1))
    return false;
  return true;
}

}  // namespace

bpfa_status bpfa_server_submit(bpfa_server_t s, int32_t stream, const int64_t* shape,
                               const float* image, const uint8_t* mask, float* out,
                               uint64_t* ticket) {
  if (!s || !shape || !image || !mask || !out || stream < 0 || stream >= s->prm.n_streams)
    return BPFA_EINVAL;
  return queue_frame(s, stream, shape, image, mask, out, nullptr, ticket);
}

bpfa_status bpfa_server_submit_scene(bpfa_server_t s, int32_t stream, const int64_t* shape,
                                     const float* scene, float* out, uint8_t* mask_out,
                                     uint64_t* ticket) {
  if (!s || !shape || !scene || !out || stream < 0 || stream >= s->prm.n_streams)
    return BPFA_EINVAL;
  return queue_frame(s, stream, shape, scene, nullptr, out, mask_out, ticket);
}

bpfa_status bpfa_server_set_policy(bpfa_server_t s, int32_t stream, const bpfa_acq_policy* policy) {
  if (!s || stream < 0 || stream >= s->prm.n_streams || !policy_ok(policy, s->prm.sc_iters))
    return BPFA_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  StreamState& ss = s->streams[stream];
  s->cv_done.wait(lk, [&] { return !ss.busy && ss.fifo.empty(); });
  ss.pol = *policy;
  ss.wvalid = false;
  return BPFA_OK;
}

bpfa_status bpfa_acquire_mask(const bpfa_acq_policy* policy, int32_t ndim, const int64_t* shape,
                              const float* weights, uint64_t seed, int32_t stream, int64_t frame,
                              uint8_t* mask, bpfa_mem mem, int32_t device) {
  if (!policy || policy->kind == BPFA_ACQ_CALLER || !policy_ok(policy, 1 << 20) || !shape || !mask ||
      ndim < 1 || ndim > 4 || stream < 0 || stream >= (1 << 24) || frame < 0)
    return BPFA_EINVAL;
  int64_t M = 1;
  for (int d = 0; d < ndim; ++d) {
    if (shape[d] < 1) return BPFA_EINVAL;
    M *= shape[d];
  }
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return BPFA_EDEVICE;
  bpfa::AcqArgs a{};
  a.M = M;
  a.rho = policy->fraction;
  a.share = policy->targeted_share;
  a.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
  a.key1 = (uint32_t)(seed >> 32);
  a.frame = (uint32_t)frame;
  a.stream_word = bpfa::kTagAcq | ((uint32_t)stream << 8);
  char* tmp = nullptr;
  const size_t wbytes = weights && policy->kind == BPFA_ACQ_TARGETED ? 4 * (size_t)M : 0;
  const size_t need = 16 + wbytes + (mem == BPFA_HOST ? (size_t)M : 0);
  hipError_t e = hipMalloc((void**)&tmp, need);
  const float* w = wbytes ? weights : nullptr;
  uint8_t* m = mask;
  if (e == hipSuccess && wbytes && mem == BPFA_HOST) {
    e = hipMemcpy(tmp + 16, weights, wbytes, hipMemcpyHostToDevice);
    w = (const float*)(tmp + 16);
  }
  if (mem == BPFA_HOST) m = (uint8_t*)(tmp + 16 + wbytes);
  if (e == hipSuccess) e = bpfa::launch_acquire(a, policy->kind, ndim, shape, w, (double*)tmp, m, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess && mem == BPFA_HOST) e = hipMemcpy(mask, m, (size_t)M, hipMemcpyDeviceToHost);
  if (tmp) (void)hipFree(tmp);
  if (prev >= 0) (void)hipSetDevice(prev);
  return e == hipSuccess ? BPFA_OK : BPFA_EDEVICE;
}

bpfa_status bpfa_server_poll(bpfa_server_t s, bpfa_serve_result* results, int32_t max, int32_t* n) {
  if (!s || !n || (max > 0 && !results)) return BPFA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  const int32_t k = std::min<int32_t>(max, (int32_t)s->results.size());
  for (int32_t i = 0; i < k; ++i) results[i] = s->results[i];
  s->results.erase(s->results.begin(), s->results.begin() + k);
  *n = k;
  return BPFA_OK;
}

bpfa_status bpfa_server_drain(bpfa_server_t s) {
  if (!s) return BPFA_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->in_flight == 0 && s->queued == 0; });
  return BPFA_OK;
}

bpfa_status bpfa_server_stats(bpfa_server_t s, bpfa_serve_stats* st) {
  if (!s || !st) return BPFA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->failed = s->failed;
  st->in_flight = s->in_flight;
  st->queued = s->queued;
  st->slots = (int64_t)s->slots.size();
  st->slot_bytes = s->slot_bytes;
  st->peak_slot_bytes = s->peak_slot_bytes;
  st->slot_creations = s->creations;
  st->slot_evictions = s->evictions;
  st->graph_frames = s->graph_frames;
  st->graph_captures = s->captures;
  for (Slot* sl : s->slots) {
    st->graph_frames += sl->graph_frames;
    st->graph_captures += sl->captures;
  }
  return BPFA_OK;
}

void bpfa_server_destroy(bpfa_server_t s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv_disp.notify_all();
  }
  if (s->dispatcher.joinable()) s->dispatcher.join();
  std::vector<Slot*> slots;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    slots.swap(s->slots);
    for (Slot* sl : slots) {
      sl->stop = true;
      sl->cv.notify_all();
    }
  }
  for (Slot* sl : slots) destroy_slot(sl);
  for (auto& ss : s->streams) {
    for (Frame* f : ss.fifo) {
      (void)hipHostFree(f->img);
      (void)hipHostFree(f->mask);
      delete f;
    }
    if (ss.blob) (void)hipFree(ss.blob);
    if (ss.pending) (void)hipFree(ss.pending);
    if (ss.weights) (void)hipFree(ss.weights);
    if (ss.wpending) (void)hipFree(ss.wpending);
  }
  delete s;
}

}  // extern "C"
