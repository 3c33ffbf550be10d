// Masked patch extraction (N-dimensional inpainting section: an image of
// shape M cut into overlapping patches of shape B with stride S; blind
// inpainting uses only the observed pixels of each patch).
//
// index_kernel   one thread per patch: observed-pixel bitmask and |Obs(i)|.
// sort_*         stable counting sort of the patches by (mini-batch, |Obs(i)|)
//                into slots (per-block histograms, per-key scans over blocks,
//                ranks inside a block): deterministic, so results do not
//                depend on scheduling; the sweep's blocks then hold patches
//                of one batch and nearly equal |Obs|.
// slots_kernel   one thread per slot: the observed offsets p (ascending) and
//                values of the slot's patch, stored [j][slot] so that a wave
//                reads them coalesced; padding entries point at offset P,
//                which the sweep keeps at zero.
// omega_*        ordered compaction of the observed pixels (the dictionary
//                statistics visit patches through them).
#include <algorithm>

#include "internal.hpp"
#include "philox.hpp"

namespace bpfa {

__device__ __forceinline__ int patch_origin(const Geom& g, int i) {
  int rem = i, org = 0;
  for (int d = g.ndim - 1; d >= 0; --d) {
    const int gd = rem % g.G[d];
    rem /= g.G[d];
    org += gd * g.S[d] * g.mstride[d];
  }
  return org;
}

__global__ void frame_reset_kernel(DevScalars* scal) {
  scal->max_obs = 0;
  scal->n_obs = 0;
  scal->ymax = 0.f;
  scal->n_omega = 0;
}

__global__ __launch_bounds__(256) void index_kernel(Geom g, const uint8_t* __restrict__ mask,
                                                    const int32_t* __restrict__ poff,
                                                    uint32_t* __restrict__ bits,
                                                    int32_t* __restrict__ count,
                                                    uint32_t* __restrict__ perm, int Npad,
                                                    DevScalars* scal) {
  __shared__ int s_max[4];
  __shared__ long long s_sum[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0;
  if (i < g.N) {
    const int org = patch_origin(g, i);
    for (int w = 0; w < g.PW; ++w) {
      // the word's 32 mask bytes are loaded together (a load-test loop waits
      // out one memory latency per pixel); positions past P read pixel 0
      const int pe = min(32, g.P - 32 * w);
      uint8_t v[32];
#pragma unroll
      for (int b = 0; b < 32; ++b) v[b] = mask[org + poff[min(32 * w + b, g.P - 1)]];
      uint32_t word = 0;
#pragma unroll
      for (int b = 0; b < 32; ++b)
        if (b < pe && v[b]) word |= 1u << b;
      cnt += __popc(word);
      bits[(size_t)i * g.PW + w] = word;
    }
    count[i] = cnt;
  }
  if (i >= g.N && i < Npad) perm[i] = 0u;   // padding slots
  // block max / sum of |Obs| (integers: order-free)
  int m = cnt;
  long long s = cnt;
  for (int o = 32; o > 0; o >>= 1) {
    m = max(m, __shfl_xor(m, o));
    s += __shfl_xor(s, o);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    s_max[wid] = m;
    s_sum[wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int bm = 0;
    long long bs = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      bm = max(bm, s_max[w]);
      bs += s_sum[w];
    }
    atomicMax(&scal->max_obs, bm);
    atomicAdd((unsigned long long*)&scal->n_obs, (unsigned long long)bs);
  }
}

__global__ __launch_bounds__(256) void slots_kernel(Geom g, const float* __restrict__ image,
                                                    const int32_t* __restrict__ poff,
                                                    const uint32_t* __restrict__ bits,
                                                    const int32_t* __restrict__ count,
                                                    const uint32_t* __restrict__ perm,
                                                    uint16_t* __restrict__ obs_idx,
                                                    float* __restrict__ obs_val,
                                                    int Npad,
                                                    const FramePlan* __restrict__ plan) {
  const int Jcap4 = plan->jpad;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;   // grid covers Npad exactly
  const bool valid = s < g.N;
  int cnt = 0;
  if (valid) {
    const int i = (int)perm[s];
    cnt = count[i];
    const int org = patch_origin(g, i);
    int j = 0;
    for (int w = 0; w < g.PW; ++w) {
      uint32_t word = bits[(size_t)i * g.PW + w];
      // observed pixels in batches of 8 whose image loads issue together
      // (an empty batch entry reads pixel 0 of the patch and is not stored)
      while (word) {
        int pb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          pb[u] = -1;
          if (word) {
            pb[u] = 32 * w + __builtin_ctz(word);
            word &= word - 1;
          }
        }
        float vb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) vb[u] = image[org + poff[max(pb[u], 0)]];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (pb[u] >= 0) {
            obs_idx[(size_t)j * Npad + s] = (uint16_t)pb[u];
            obs_val[(size_t)j * Npad + s] = vb[u];
            ++j;
          }
      }
    }
  }
  for (int j = cnt; j < Jcap4; ++j) {
    obs_idx[(size_t)j * Npad + s] = (uint16_t)g.P;
    obs_val[(size_t)j * Npad + s] = 0.f;
  }
}

// exclusive scan in place of data[0 .. n) by one block of 1024 threads; returns the total
__device__ int block_scan_1024(int* __restrict__ data, int n, int* s_tot) {
  const int tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += data[b];
  s_tot[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = tid >= o ? s_tot[tid - o] : 0;
    __syncthreads();
    s_tot[tid] += v;
    __syncthreads();
  }
  int run = s_tot[tid] - sum;
  for (int b = b0; b < b1; ++b) {
    const int c = data[b];
    data[b] = run;
    run += c;
  }
  const int total = s_tot[1023];
  __syncthreads();
  return total;
}

// ---- stable counting sort of patches by (batch, |Obs(i)|) ------------------
//
// With B mini-batches patch i belongs to batch i mod B, and the slots hold
// batch 0's patches first, then batch 1's, ..., each batch in ascending
// |Obs| (ties in ascending patch index).  Batch b's patches are the rows
// r = 0 .. nr_b - 1 of i = r B + b; each batch is counted by its own
// sort blocks of 256 rows, so the histogram holds (P + 1) entries per block as
// in the single-batch sort.  Histogram layout [b][c][block of b], bins [b][c].
// With B = 1 this is the plain counting sort by |Obs|.

struct SortShape {
  int B;     // batches
  int nrow;  // rows per batch: ceil(N / B)
  int nbb;   // sort blocks per batch: ceil(nrow / kSortBlock)
};

__device__ __forceinline__ int sort_patch(const Geom& g, const SortShape& ss, int b, int blk, int tid) {
  const int r = blk * kSortBlock + tid;
  const long long i = (long long)r * ss.B + b;
  return (r < ss.nrow && i < g.N) ? (int)i : -1;
}

__global__ __launch_bounds__(kSortBlock) void sort_hist_kernel(Geom g, SortShape ss,
                                                               const int32_t* __restrict__ count,
                                                               int32_t* __restrict__ hist) {
  extern __shared__ int s_h[];
  const int b = blockIdx.x / ss.nbb, blk = blockIdx.x % ss.nbb;
  for (int v = threadIdx.x; v <= g.P; v += kSortBlock) s_h[v] = 0;
  __syncthreads();
  const int i = sort_patch(g, ss, b, blk, threadIdx.x);
  if (i >= 0) atomicAdd(&s_h[count[i]], 1);
  __syncthreads();
  for (int v = threadIdx.x; v <= g.P; v += kSortBlock)
    hist[((size_t)b * (g.P + 1) + v) * ss.nbb + blk] = s_h[v];
}

// one block per key (b, c): exclusive scan over b's blocks, total into bins[key]
__global__ __launch_bounds__(1024) void sort_scan_kernel(int32_t* __restrict__ hist, int nbb,
                                                         int32_t* __restrict__ bins) {
  __shared__ int s_tot[1024];
  const int t = block_scan_1024(hist + (size_t)blockIdx.x * nbb, nbb, s_tot);
  if (threadIdx.x == 0) bins[blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void sort_bins_kernel(int nbins, int32_t* __restrict__ bins) {
  __shared__ int s_tot[1024];
  block_scan_1024(bins, nbins, s_tot);
}

__global__ __launch_bounds__(kSortBlock) void sort_scatter_kernel(Geom g, SortShape ss,
                                                                  const int32_t* __restrict__ count,
                                                                  const int32_t* __restrict__ hist,
                                                                  const int32_t* __restrict__ bins,
                                                                  uint32_t* __restrict__ perm,
                                                                  int32_t* __restrict__ inv_perm) {
  __shared__ int s_c[kSortBlock];
  const int b = blockIdx.x / ss.nbb, blk = blockIdx.x % ss.nbb;
  const int i = sort_patch(g, ss, b, blk, threadIdx.x);
  const int c = i >= 0 ? count[i] : -1;
  s_c[threadIdx.x] = c;
  __syncthreads();
  if (i < 0) return;
  int rank = 0;
  for (int t = 0; t < (int)threadIdx.x; ++t) rank += s_c[t] == c;
  const size_t key = (size_t)b * (g.P + 1) + c;
  const int slot = bins[key] + hist[key * ss.nbb + blk] + rank;
  perm[slot] = (uint32_t)i;
  inv_perm[i] = slot;
}

hipError_t launch_sort(const Geom& g, const Buffers& b, int n_batches, hipStream_t st) {
  SortShape ss;
  ss.B = n_batches;
  ss.nrow = (g.N + n_batches - 1) / n_batches;
  ss.nbb = (ss.nrow + kSortBlock - 1) / kSortBlock;
  const int blocks = n_batches * ss.nbb;
  const int keys = n_batches * (g.P + 1);
  sort_hist_kernel<<<blocks, kSortBlock, (g.P + 1) * sizeof(int), st>>>(g, ss, b.obs_count, b.sort_hist);
  sort_scan_kernel<<<keys, 1024, 0, st>>>(b.sort_hist, ss.nbb, b.sort_bin);
  sort_bins_kernel<<<1, 1024, 0, st>>>(keys, b.sort_bin);
  sort_scatter_kernel<<<blocks, kSortBlock, 0, st>>>(g, ss, b.obs_count, b.sort_hist, b.sort_bin,
                                                     b.perm, b.inv_perm);
  return hipGetLastError();
}

// histogram entries the sort needs for n_batches batches
size_t sort_hist_entries(const Geom& g, int n_batches) {
  const long long nrow = (g.N + n_batches - 1) / n_batches;
  const long long nbb = (nrow + kSortBlock - 1) / kSortBlock;
  return (size_t)n_batches * (size_t)(g.P + 1) * (size_t)nbb;
}

// ---- mini-batch steps: the batch's new lists back into the current buffer ----

// one thread per slot of the batch: the patch's list row (n_a entries and the
// end marker) and its count, from the sweep's output buffer to its input
__global__ __launch_bounds__(256) void list_copy_kernel(int K, int slot0, int nslots,
                                                        const uint32_t* __restrict__ perm,
                                                        const int2* __restrict__ src,
                                                        const int32_t* __restrict__ nsrc,
                                                        int2* __restrict__ dst,
                                                        int32_t* __restrict__ ndst) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  const size_t i = perm[slot0 + s];
  const int na = nsrc[i];
  const int n = na < K ? na + 1 : K;
  const int2* a = src + i * K;
  int2* d = dst + i * K;
  for (int e = 0; e < n; ++e) d[e] = a[e];
  ndst[i] = na;
}

hipError_t launch_list_copy(const Geom& g, const Buffers& b, int from, int slot0, int nslots,
                            hipStream_t st) {
  if (nslots <= 0) return hipSuccess;
  list_copy_kernel<<<(nslots + 255) / 256, 256, 0, st>>>(g.K, slot0, nslots, b.perm, b.list[from],
                                                         b.nact[from], b.list[1 - from],
                                                         b.nact[1 - from]);
  return hipGetLastError();
}

// ---- ordered compaction of observed pixels ---------------------------------

__global__ __launch_bounds__(256) void omega_count_kernel(int Mtot, const uint8_t* __restrict__ mask,
                                                          const float* __restrict__ image,
                                                          int32_t* __restrict__ blk,
                                                          DevScalars* scal) {
  __shared__ int s_c[4];
  __shared__ float s_y[4];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = q < Mtot && mask[q] != 0;
  float y = on ? fabsf(image[q]) : 0.f;
  const unsigned long long bal = __ballot(on);
  for (int o = 32; o > 0; o >>= 1) y = fmaxf(y, __shfl_xor(y, o));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    s_c[wid] = __popcll(bal);
    s_y[wid] = y;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    float ym = 0.f;
    for (int w = 0; w < 4; ++w) {
      c += s_c[w];
      ym = fmaxf(ym, s_y[w]);
    }
    blk[blockIdx.x] = c;
    // non-negative floats order like their bit patterns
    atomicMax((int*)&scal->ymax, __float_as_int(ym));
  }
}

// exclusive scan of the per-block counts, one block of 1024 threads
__global__ __launch_bounds__(1024) void omega_scan_kernel(int nb, int32_t* __restrict__ blk,
                                                          DevScalars* scal) {
  __shared__ int s_tot[1024];
  const int total = block_scan_1024(blk, nb, s_tot);
  if (threadIdx.x == 0) scal->n_omega = total;
}

__global__ __launch_bounds__(256) void omega_write_kernel(Geom g, const uint8_t* __restrict__ mask,
                                                          const int32_t* __restrict__ blk,
                                                          int32_t* __restrict__ omega,
                                                          int4* __restrict__ omega_c) {
  const int Mtot = g.Mtot;
  __shared__ int s_c[4];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = q < Mtot && mask[q] != 0;
  const unsigned long long bal = __ballot(on);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) s_c[wid] = __popcll(bal);
  __syncthreads();
  int base = blk[blockIdx.x];
  for (int w = 0; w < wid; ++w) base += s_c[w];
  const unsigned long long below = (lane == 0) ? 0ull : (bal & ((~0ull) >> (64 - lane)));
  if (on) {
    const int v = base + __popcll(below);
    omega[v] = q;
    int c[kMaxDim] = {0, 0, 0, 0};
    int rem = q;
    for (int d = g.ndim - 1; d >= 0; --d) {
      c[d] = rem % g.M[d];
      rem /= g.M[d];
    }
    omega_c[v] = make_int4(c[0], c[1], c[2], c[3]);
  }
}

// ---- prior draw of the dictionary: d_kp = n / sqrt(P), binary64 ----------

__global__ void init_dict_kernel(Geom g, float* __restrict__ D, uint32_t key0, uint32_t key1,
                                 uint32_t stream) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.K * g.P) return;
  const int k = idx / g.P, p = idx % g.P;
  const Block4 r = philox10((uint32_t)p, (uint32_t)k, 0u, stream, key0, key1);
  const double n = sqrt(-2.0 * log(u01d(r.w0))) * cos(2.0 * M_PI * u01d(r.w1));
  D[idx] = (float)(n / sqrt((double)g.P));
}

// ---- frame plan: wavefront table, slot rows, statistics chunking ----------
//
// Built on the device from the slot sort's key offsets, so a frame load needs
// no host round trip.  Within a batch the slots ascend in |Obs|; the sweep
// gives a patch with |Obs| in class c = [lo_c, hi_c] lanes_c lanes, and cuts
// each (batch, class) run of slots into wavefronts of 64 / lanes_c slots
// (the last one shorter).  A wavefront's register count J covers its last,
// largest slot: J = max(4, |Obs| rounded up to even) for one lane per patch;
// for a group of L lanes 12 or 16 (L J >= |Obs|), and 20 or 24 too for two
// lanes (patches with 33-48 observed pixels: fewer lanes per patch repeat the
// pair's draws and decisions fewer times).

__device__ __constant__ int kClassLo[kLaneClasses] = {0, 17, 49, 65, 129};
__device__ __constant__ int kClassHi[kLaneClasses] = {16, 48, 64, 128, 256};
__device__ __constant__ int kClassLanes[kLaneClasses] = {1, 2, 4, 8, 16};

struct PlanArgs {
  int n_batches;
  int dict_chunks_max, dict_cv_max, dict_slots, dict_npr;   // npr: (p, row group) pairs
};

// one block of 1024 threads
__global__ __launch_bounds__(1024) void frame_plan_kernel(Geom g, PlanArgs pa,
                                                          const int32_t* __restrict__ bins,
                                                          const DevScalars* __restrict__ scal,
                                                          FramePlan* __restrict__ plan) {
  __shared__ int s_tot[1024];
  __shared__ long long s_red[1024];
  const int B = pa.n_batches, P = g.P, tid = threadIdx.x;
  const int E = B * kLaneClasses;
  // first slot of batch b with |Obs| >= c (c > P: the batch's end)
  auto start = [&](int b, int c) -> int {
    if (c <= P) return bins[(size_t)b * (P + 1) + c];
    return b + 1 < B ? bins[(size_t)(b + 1) * (P + 1)] : g.N;
  };
  for (int e = tid; e < E; e += 1024) {
    const int b = e / kLaneClasses, c = e - b * kLaneClasses;
    const int s0 = start(b, min(kClassLo[c], P + 1));
    const int s1 = start(b, min(kClassHi[c] + 1, P + 1));
    const int per = kWave / kClassLanes[c];
    plan->cls_s0[e] = s0;
    plan->cls_s1[e] = s1;
    plan->cls_w0[e] = (s1 - s0 + per - 1) / per;   // wavefront count, scanned below
  }
  __syncthreads();
  const int total = block_scan_1024(plan->cls_w0, E, s_tot);
  if (tid == 0) {
    plan->cls_w0[E] = total;
    plan->all_waves[0] = 0;
    plan->all_waves[1] = total;
    plan->n_batches = B;
    plan->batch_wave0[B] = total;
    plan->batch_slot0[B] = g.N;
    const int mo = scal->max_obs;
    plan->bad = mo > 256 ? 1 : 0;
    const int jcap = (P + 3) & ~3;
    plan->jpad = min(jcap, max(4, (mo + 3) & ~3));
    // statistics chunking: the chunk count c >= need that minimises the
    // block rounds per chunk, rounds(c) / c (ties: the smaller c)
    const int nom = scal->n_omega;
    const int need = min(pa.dict_chunks_max, max(1, (nom + pa.dict_cv_max - 1) / pa.dict_cv_max));
    int best = need;
    double best_cost = 1e300;
    for (int cc = need; cc <= pa.dict_chunks_max; ++cc) {
      const long long blocks = (long long)pa.dict_npr * cc;
      const double cost = (double)((blocks + pa.dict_slots - 1) / pa.dict_slots) / cc;
      if (cost < best_cost * (1.0 - 1e-9)) {
        best_cost = cost;
        best = cc;
      }
    }
    const int per = (nom + best - 1) / best;
    plan->dict_chunks = best;
    plan->dict_cv = min(pa.dict_cv_max, max(kWave, (per + kWave - 1) / kWave * kWave));
    plan->dict_xcd = best % 8 == 0 ? 1 : 0;
  }
  __syncthreads();
  for (int b = tid; b < B; b += 1024) {
    plan->batch_wave0[b] = plan->cls_w0[b * kLaneClasses];
    plan->batch_slot0[b] = start(b, 0);
  }
  // observed pixels of each batch: sum over |Obs| = c of c times the bin size
  for (int b = 0; b < B; ++b) {
    long long part = 0;
    for (int c = 1 + tid; c <= P; c += 1024) part += (long long)c * (start(b, c + 1) - start(b, c));
    s_red[tid] = part;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
      if (tid < o) s_red[tid] += s_red[tid + o];
      __syncthreads();
    }
    if (tid == 0) plan->batch_nobs[b] = s_red[0];
    __syncthreads();
  }
}

// one thread per wavefront of the table
__global__ __launch_bounds__(256) void plan_waves_kernel(int E, const FramePlan* __restrict__ plan,
                                                         const int32_t* __restrict__ count,
                                                         const uint32_t* __restrict__ perm,
                                                         int4* __restrict__ waves) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= plan->all_waves[1]) return;
  // the last (batch, class) whose first wavefront is <= w (empty runs share
  // their offset with the next one, so this is the run that holds w)
  int lo = 0, hi = E - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (plan->cls_w0[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  const int c = lo % kLaneClasses;
  const int lanes = kClassLanes[c], per = kWave / lanes;
  const int slot = plan->cls_s0[lo] + (w - plan->cls_w0[lo]) * per;
  const int ns = min(per, plan->cls_s1[lo] - slot);
  const int clast = count[perm[slot + ns - 1]];
  // rows per lane: the smallest compiled body that holds the wave's largest patch
  int J = 16;
  if (lanes == 1) J = max(4, (clast + 1) & ~1);
  else if (lanes == 2 && clast > 32) J = clast <= 40 ? 20 : 24;
  else if (clast <= 12 * lanes) J = 12;
  waves[w] = make_int4(slot, ns, lanes, J);
}

hipError_t launch_frame_plan(const Geom& g, const Buffers& b, int n_batches, long long wave_cap,
                             int dict_chunks_max, int dict_cv_max, int dict_slots, int dict_npr,
                             hipStream_t st) {
  PlanArgs pa{n_batches, dict_chunks_max, dict_cv_max, dict_slots, dict_npr};
  frame_plan_kernel<<<1, 1024, 0, st>>>(g, pa, b.sort_bin, b.scal, b.plan);
  const int E = n_batches * kLaneClasses;
  plan_waves_kernel<<<(unsigned)((wave_cap + 255) / 256), 256, 0, st>>>(E, b.plan, b.obs_count,
                                                                       b.perm, b.sweep_waves);
  return hipGetLastError();
}

// ---- launchers ----------------------------------------------------------

hipError_t launch_index(const Geom& g, const Buffers& b, int Npad, hipStream_t st) {
  frame_reset_kernel<<<1, 1, 0, st>>>(b.scal);
  const int n = max(g.N, Npad);
  index_kernel<<<(n + 255) / 256, 256, 0, st>>>(g, b.mask, b.poff, b.obs_bits, b.obs_count,
                                                b.perm, Npad, b.scal);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* __restrict__ p, long long n, int32_t v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, long long n, int32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>(1024, (n + 255) / 256);
  fill_i32_kernel<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_omega(const Geom& g, const Buffers& b, hipStream_t st) {
  const int nb = (g.Mtot + 255) / 256;
  omega_count_kernel<<<nb, 256, 0, st>>>(g.Mtot, b.mask, b.image, b.omega_blk, b.scal);
  omega_scan_kernel<<<1, 1024, 0, st>>>(nb, b.omega_blk, b.scal);
  omega_write_kernel<<<nb, 256, 0, st>>>(g, b.mask, b.omega_blk, b.omega, b.omega_c);
  return hipGetLastError();
}

hipError_t launch_slots(const Geom& g, const Buffers& b, int Npad, hipStream_t st) {
  slots_kernel<<<Npad / 256, 256, 0, st>>>(g, b.image, b.poff, b.obs_bits, b.obs_count, b.perm,
                                           b.obs_idx, b.obs_val, Npad, b.plan);
  return hipGetLastError();
}

hipError_t launch_init_dict(const Geom& g, const Buffers& b, uint32_t key0, uint32_t key1,
                            uint32_t stream, hipStream_t st) {
  const int n = g.K * g.P;
  init_dict_kernel<<<(n + 255) / 256, 256, 0, st>>>(g, b.D, key0, key1, stream);
  return hipGetLastError();
}

}  // namespace bpfa
