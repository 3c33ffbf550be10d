// Dictionary update (BPFA section: the dictionary-learning step).
//
// With the prior d_k ~ N(0, I/P), the conditional of d_kp given everything
// else is Gaussian with precision lam = P + gamma_eps A and mean
// gamma_eps b / lam, where A = sum_i m_ip w_ik^2 and
// b = sum_i m_ip w_ik (x_ip - sum_{j != k} d_jp w_ij); atoms go in ascending
// order.  Writing C_p = sum_i m_ip w_i w_i^T and B_p = sum_i m_ip x_ip w_i,
//     A = C_p[k][k],   b = B_p[k] - sum_{j != k} C_p[k][j] d_jp
// (new d_j for j < k, old for j > k) -- the same draws as the residual form,
// different only in rounding.  Every pixel position p is then an independent
// chain over k, and the residual sum of squares after the update is
// sum_p (X2_p - 2 d_p.B_p + d_p^T C_p d_p) with X2_p = sum_i m_ip x_ip^2.
//
// dict_stats_kernel: one block per (p, row group of the K x K triangle,
//   chunk of observed pixels).  The visits of the chunk (observed pixel q,
//   the patch whose origin is q - b(p)) are first grouped by the length of
//   the patch's active list from the block's row group on (a later group
//   starts at the offset list_groups_kernel found) in LDS, so a wavefront's
//   lanes share a pair loop bound; then a lane stages those entries in
//   registers and adds their outer product into LDS.  Sums are 64-bit fixed point: the
//   binary64 product of two binary32 weights is exact, it is scaled by a power
//   of two and rounded to an integer by adding 1.5 * 2^52 (exact for
//   |x| < 2^51); integer adds are associative, so the statistics do not
//   depend on scheduling.
// dict_reduce_kernel: sums the chunk partials, one block per (p, 32 x 32
//   tile of the upper triangle), into the symmetric binary64 C_p, B_p and
//   the diagonal.
// dict_chain_kernel: one wavefront per p runs the chain with rows of C_p
//   prefetched ahead of use, keeping u = C_p d current instead of reducing a
//   dot product per step, draws d_kp with the Philox DICT stream, and forms
//   the residual sum of squares.
#include <algorithm>

#include "internal.hpp"
#include "philox.hpp"

namespace bpfa {

constexpr int kStatsCap = 16;   // active entries of a patch held in registers

// a visit of the statistics pass: patch, its list's length from the block's
// row group on and the offset where that part starts, the observed value, the
// wave's bound on the length, and the first kStatsCap entries of that part
struct VisitRow {
  int pid, na, off, wmax;
  double y;
  int2 raw[kStatsCap];
};


// chunks: chunk slots of the launch (the partials' stride); chunk_visits: the
// largest chunk (the LDS layout).  A frame uses the first dict_chunks slots of
// dict_cv visits each (frame plan).
struct DictPlanDev {
  int RG, chunks, K, chunk_visits, xcd, copies, copy_rows;
  int row0[65];
  long long ent0[65];
  long long rec_stride;
};

__device__ __forceinline__ long long tri_off(int k, int K) {
  return (long long)k * K - (long long)k * (k - 1) / 2;
}

// round-to-nearest of x (|x| < 2^51) as a 64-bit integer
__device__ __forceinline__ unsigned long long to_fixed(double x) {
  return (unsigned long long)(__double_as_longlong(x + 6755399441055744.0) -
                              0x4338000000000000LL);
}

// origin = q - b(p): every coordinate non-negative, on the stride grid, inside the grid
__device__ __forceinline__ int visit_patch(const Geom& g, const int4 qc, const int* bc) {
  const int qv[kMaxDim] = {qc.x, qc.y, qc.z, qc.w};
  int pidx = 0;
  bool ok = true;
  for (int d = 0; d < g.ndim; ++d) {
    const int od = qv[d] - bc[d];
    const int gd = g.S[d] == 1 ? od : od / g.S[d];
    ok = ok && od >= 0 && gd * g.S[d] == od && gd < g.G[d];
    pidx = pidx * g.G[d] + gd;
  }
  return ok ? pidx : -1;
}

// Pair accumulation of one visit, in straight-line code.  Byte offsets into
// the block's LDS: the group's triangle rows, its B entries, then the sink
// region (one slot per lane followed by K spare slots).  A term whose row lies
// outside the group (or past the patch's n_a) goes to sink + 8 column, inside
// the sink region; a column past n_a is replaced by a column the row holds
// (the lane's last staged atom, or the row's own diagonal) with a zero
// weight.  Row offsets pass through an empty asm so that the compiler keeps
// one select per row instead of turning the choice into exec-mask branches
// around every term (branches put the CU's one scalar unit back in the loop).
struct StatsRow {
  char* lds;
  unsigned sink;          // this lane's sink slot
  unsigned copy;          // this lane's copy of the group's diagonal, then B, accumulators
  int r0, r1, e0, tw, E;  // group rows, its first triangle entry, 2K - 1, its entry count
  int R;                  // rows per copy
  double sc, ysb;
  __device__ __forceinline__ bool in(int k) const { return k >= r0 && k < r1; }
  // entry (k, j) of row k, j >= k, sits at row_byte(k) + 8 j:
  // tri_off(k, K) - k = k (2K - 1 - k) / 2 (an integer)
  __device__ __forceinline__ unsigned row_byte(int k) const {
    return 8u * (unsigned)((int)(__umul24((unsigned)k, (unsigned)(tw - k)) >> 1) - e0);
  }
  __device__ __forceinline__ unsigned b_byte(int k) const { return 8u * (unsigned)(E + k - r0); }
  __device__ __forceinline__ unsigned row_or_sink(bool in_group, int k) const {
    unsigned o = in_group ? row_byte(k) : sink;
    asm volatile("" : "+v"(o));
    return o;
  }
  __device__ __forceinline__ unsigned b_or_sink(bool in_group, int k) const {
    unsigned o = in_group ? b_byte(k) : sink;
    asm volatile("" : "+v"(o));
    return o;
  }
  // the lane group's copies of entry (k, k) and of B_p[k]
  __device__ __forceinline__ unsigned diag_copy_or_sink(bool in_group, int k) const {
    unsigned o = in_group ? copy + 8u * (unsigned)(k - r0) : sink;
    asm volatile("" : "+v"(o));
    return o;
  }
  __device__ __forceinline__ unsigned b_copy_or_sink(bool in_group, int k) const {
    unsigned o = in_group ? copy + 8u * (unsigned)(R + k - r0) : sink;
    asm volatile("" : "+v"(o));
    return o;
  }
  __device__ __forceinline__ void add(unsigned off, double x) const {
    atomicAdd(reinterpret_cast<unsigned long long*>(lds + off), to_fixed(x));
  }
};

// A register stage of up to kStatsCap list entries: weights (0 past the
// patch's n_a) and column offsets (8 x atom; past n_a the last valid atom's, a
// column every staged row holds since lists ascend).  A row is live when its
// weight is non-zero: a listed entry whose weight is exactly zero adds only
// zeros, so sending its terms to the sink leaves every sum unchanged.
struct Stage {
  unsigned col[kStatsCap];
  double ww[kStatsCap];
  __device__ __forceinline__ int atom(int a) const { return (int)(col[a] >> 3); }
  __device__ __forceinline__ bool live(int a) const { return ww[a] != 0.0; }
};

__device__ __forceinline__ void stage_from(Stage& s, const int2 (&raw)[kStatsCap], int nv) {
  unsigned last = 0;
#pragma unroll
  for (int a = 0; a < kStatsCap; ++a) {
    const bool in = a < nv;
    s.ww[a] = in ? (double)__int_as_float(raw[a].y) : 0.0;
    last = in ? 8u * (unsigned)raw[a].x : last;
    s.col[a] = last;
  }
}

// Holds the stage's values where this is called: an empty asm that reads and
// writes them, with a memory clobber so that no later load moves above it.
__device__ __forceinline__ void pin_stage(Stage& s) {
#pragma unroll
  for (int a = 0; a < kStatsCap; ++a) asm volatile("" : "+v"(s.col[a]), "+v"(s.ww[a]) : : "memory");
}

// SKIP: with several row groups a row no lane of the wave holds in this
// block's group (it adds only to the sinks) is skipped whole by a uniform
// branch; a lane's rows in the group are a prefix of its staged entries, so
// this bounds the rows by the wave's longest prefix.  With one group every
// staged row is in it and the test is left out.
template <int NB, bool SKIP>
__device__ __forceinline__ void stats_pairs(const StatsRow& sr, const Stage& s) {
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    const int k = s.atom(a);
    const bool ina = s.live(a) && sr.in(k);
    if (SKIP && __builtin_amdgcn_ballot_w64(ina) == 0) continue;
    // B_p[k] and the diagonal (k, k) go to the lane group's copies; the
    // pairs (k, j), j > k, to the shared rows
    sr.add(sr.b_copy_or_sink(ina, k), s.ww[a] * sr.ysb);
    const double was = s.ww[a] * sr.sc;
    sr.add(sr.diag_copy_or_sink(ina, k), was * s.ww[a]);
    const unsigned rb = sr.row_or_sink(ina, k);
#pragma unroll
    for (int b = a + 1; b < NB; ++b) sr.add(rb + s.col[b], was * s.ww[b]);
  }
}

template <bool SKIP>
__device__ __forceinline__ void stats_stage(const StatsRow& sr, const Stage& s, int bound) {
  switch (min(bound, kStatsCap)) {
    case 1: stats_pairs<1, SKIP>(sr, s); break;
    case 2: stats_pairs<2, SKIP>(sr, s); break;
    case 3: stats_pairs<3, SKIP>(sr, s); break;
    case 4: stats_pairs<4, SKIP>(sr, s); break;
    case 5: stats_pairs<5, SKIP>(sr, s); break;
    case 6: stats_pairs<6, SKIP>(sr, s); break;
    case 7: stats_pairs<7, SKIP>(sr, s); break;
    case 8: stats_pairs<8, SKIP>(sr, s); break;
    case 9: stats_pairs<9, SKIP>(sr, s); break;
    case 10: stats_pairs<10, SKIP>(sr, s); break;
    case 11: stats_pairs<11, SKIP>(sr, s); break;
    case 12: stats_pairs<12, SKIP>(sr, s); break;
    case 13: stats_pairs<13, SKIP>(sr, s); break;
    case 14: stats_pairs<14, SKIP>(sr, s); break;
    case 15: stats_pairs<15, SKIP>(sr, s); break;
    case 16: stats_pairs<16, SKIP>(sr, s); break;
    default: break;
  }
}

// pairs of the staged rows with list entry b read from memory (b past the
// stage; a lane whose list ends before b adds zeros at its last staged column)
__device__ __forceinline__ void stats_stage_with(const StatsRow& sr, const Stage& s,
                                                 const unsigned (&rb)[kStatsCap],
                                                 const double (&wsc)[kStatsCap], bool inb, int2 eb) {
  const double wb = inb ? (double)__int_as_float(eb.y) : 0.0;
  const unsigned cb = inb ? 8u * (unsigned)eb.x : s.col[kStatsCap - 1];
#pragma unroll
  for (int a = 0; a < kStatsCap; ++a) sr.add(rb[a] + cb, wsc[a] * wb);
}

__device__ __forceinline__ void stage_rows(const StatsRow& sr, const Stage& s,
                                           unsigned (&rb)[kStatsCap], double (&wsc)[kStatsCap]) {
#pragma unroll
  for (int a = 0; a < kStatsCap; ++a) {
    const int k = s.atom(a);
    rb[a] = sr.row_or_sink(s.live(a) && sr.in(k), k);
    wsc[a] = s.ww[a] * sr.sc;
  }
}

// entries b = from .. wmax - 1 read from memory: each one's B entry and its
// pairs (a, b) with the entries a = from .. b, also read from memory (the
// rare tails past the register stages); L is the patch's list row
__device__ __forceinline__ void stats_tail(const StatsRow& sr, const int2* L, int na,
                                           int from, int b, bool inb, int2 eb) {
  const double wb = inb ? (double)__int_as_float(eb.y) : 0.0;
  sr.add(sr.b_or_sink(inb && sr.in(eb.x), eb.x), wb * sr.ysb);
  for (int a = from; a <= b; ++a) {
    int2 ea = make_int2(-1, 0);
    if (a < na) ea = L[a];
    const bool ina = a < na && sr.in(ea.x);
    const unsigned rb = sr.row_or_sink(ina, ea.x);
    // a column past n_a: the row's own diagonal, with a zero weight
    const unsigned cb = inb ? 8u * (unsigned)eb.x : 8u * (unsigned)max(ea.x, 0);
    sr.add(rb + cb, (double)__int_as_float(ea.y) * sr.sc * wb);
  }
}

// Per frame: for every position p and observed pixel v (in omega order), the
// patch whose origin is q_v - b(p), or -1 when that origin is off the grid;
// and the observed values in omega order.
__global__ __launch_bounds__(256) void visit_table_kernel(Geom g, const DevScalars* __restrict__ scal,
                                                          const int4* __restrict__ omega_c,
                                                          const int32_t* __restrict__ omega,
                                                          const float* __restrict__ image,
                                                          const int32_t* __restrict__ pcoord,
                                                          int32_t* __restrict__ vpatch,
                                                          float* __restrict__ omega_y) {
  const int nom = scal->n_omega;
  const int p = blockIdx.y;
  int bc[kMaxDim] = {0, 0, 0, 0};
  for (int d = 0; d < g.ndim; ++d) bc[d] = pcoord[p * kMaxDim + d];
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nom; v += gridDim.x * blockDim.x) {
    vpatch[(size_t)p * g.Mtot + v] = visit_patch(g, omega_c[v], bc);
    if (p == 0) omega_y[v] = image[omega[v]];
  }
}

// the grid strides over the frame's observed pixels (their count is read on
// the device): up to 64 blocks of 256 per position
hipError_t launch_visit_table(const Geom& g, const Buffers& b, hipStream_t st) {
  const dim3 grid((unsigned)std::min<long long>(64, ((long long)g.Mtot + 255) / 256), (unsigned)g.P);
  visit_table_kernel<<<grid, 256, 0, st>>>(g, b.scal, b.omega_c, b.omega, b.image, b.pcoord,
                                           b.vpatch, b.omega_y);
  return hipGetLastError();
}

// LDS: rec int64 accumulators | 64 per-lane sinks | K + 1 int bin starts | chunk visits (patch
// int32, y float, n_a uint16).  Visits are bucketed by n_a inside the block so
// each wavefront's pair loop runs to a bound its lanes share.
template <bool SKIP>
__global__ __launch_bounds__(kDictBlock) void dict_stats_kernel(
    Geom g, DictPlanDev pl, const FramePlan* __restrict__ fplan, const int32_t* __restrict__ vpatch,
    const float* __restrict__ omega_y, const int2* __restrict__ list,
    const int32_t* __restrict__ nact, const uint16_t* __restrict__ goff,
    const DevScalars* __restrict__ scal,
    long long* __restrict__ dpart, double* __restrict__ dx2, int n_batches, int batch) {
  extern __shared__ long long acc[];
  __shared__ double s_x2[kDictBlock / kWave];
  __shared__ int s_total, s_next;
  // this frame's chunking: cc chunks of cvf observed pixels (the launch has
  // room for pl.chunks chunks of pl.chunk_visits)
  const int nom = scal->n_omega;
  const int cc = fplan->dict_chunks, cvf = fplan->dict_cv;
  const int npr = g.P * pl.RG;
  if ((int)blockIdx.x >= npr * cc) return;   // chunk slots this frame leaves empty
  // block -> (chunk c, position p, row group rg).  Workgroups are dispatched
  // round-robin over the 8 XCDs; with cc a multiple of 8 every block of
  // chunk c has blockIdx = c mod 8, and an XCD takes all (p, rg) blocks of
  // one chunk before its next chunk, so the blocks that read the same
  // patches' lists (a band of image rows) run together on one L2.
  int c, prg;
  if (fplan->dict_xcd) {
    const int j = blockIdx.x >> 3;
    c = (blockIdx.x & 7) + 8 * (j / npr);
    prg = j % npr;
  } else {
    c = blockIdx.x % cc;
    prg = blockIdx.x / cc;
  }
  const int p = prg / pl.RG, rg = prg % pl.RG;
  const int r0 = pl.row0[rg], r1 = pl.row0[rg + 1];
  const long long e0 = pl.ent0[rg];
  const int E = (int)(pl.ent0[rg + 1] - e0);
  const int rec = E + (r1 - r0);
  const int K = g.K;
  // copies of the group's diagonal and B accumulators, one per lane group
  long long* cpy = acc + pl.rec_stride + dict_sink_entries(K);
  const int ncopy = pl.copies * 2 * pl.copy_rows;
  int* bins = reinterpret_cast<int*>(cpy + ncopy);   // K + 1 counts, then starts
  int* v_pat = bins + (K + 1);
  float* v_y = reinterpret_cast<float*>(v_pat + pl.chunk_visits);
  uint16_t* v_na = reinterpret_cast<uint16_t*>(v_y + pl.chunk_visits);
  uint16_t* v_off = v_na + pl.chunk_visits;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  for (int e = tid; e < rec; e += kDictBlock) acc[e] = 0;
  for (int e = tid; e < ncopy; e += kDictBlock) cpy[e] = 0;

  const double sc = scal->scale_c, sb = scal->scale_b;
  const unsigned sink = (unsigned)((pl.rec_stride + lane) * 8);   // this lane's sink slot
  const unsigned copy = (unsigned)((pl.rec_stride + dict_sink_entries(K) +
                                    (long long)(lane / (kWave / pl.copies)) * 2 * pl.copy_rows) * 8);
  const int32_t* vs = vpatch + (size_t)p * g.Mtot;
  double x2 = 0.0;

  // block c of its (p, row group) takes chunks c, c + cc, ... of the observed pixels
  for (int ch = c; ch * cvf < nom; ch += cc) {
  const int v0 = ch * cvf, v1 = min(nom, v0 + cvf);
  for (int e = tid; e <= K; e += kDictBlock) bins[e] = 0;
  __syncthreads();

  // pass 1: this thread's visits (at most kDictVpt) in registers; rank within its n_a bin.
  // Every load is issued (indices clamped into the chunk and the patch range)
  // and the result selected afterwards, so the loads of all visits are in
  // flight together instead of each behind a branch and its own wait.
  int r_pat[kDictVpt], r_na[kDictVpt], r_off[kDictVpt], r_rank[kDictVpt];
  float r_y[kDictVpt];
#pragma unroll
  for (int u = 0; u < kDictVpt; ++u) {
    const int v = v0 + tid + u * kDictBlock;
    const int vc = min(v, v1 - 1);   // v0 < v1: an observed pixel of the chunk
    const int pat = vs[vc];
    r_y[u] = omega_y[vc];
    r_pat[u] = v < v1 ? pat : -1;
  }
  // a mini-batch step counts only the visits of its batch's patches
  if (n_batches > 1) {
#pragma unroll
    for (int u = 0; u < kDictVpt; ++u)
      if (r_pat[u] >= 0 && r_pat[u] % n_batches != batch) r_pat[u] = -1;
  }
#pragma unroll
  for (int u = 0; u < kDictVpt; ++u) {
    // a later row group skips the list's entries below its first row (lists
    // ascend, and a pair (j, k), j <= k, belongs to row j's group)
    const int pc = max(r_pat[u], 0);
    const int off = rg > 0 ? (int)goff[(size_t)pc * (pl.RG - 1) + (rg - 1)] : 0;
    const int n = nact[pc];
    r_off[u] = r_pat[u] >= 0 ? off : 0;
    r_na[u] = r_pat[u] >= 0 ? n - off : 0;
  }
#pragma unroll
  for (int u = 0; u < kDictVpt; ++u) {
    r_rank[u] = 0;
    if (r_pat[u] >= 0) {
      r_rank[u] = atomicAdd(&bins[r_na[u]], 1);
      if (rg == 0) x2 += (double)r_y[u] * (double)r_y[u];
    }
  }
  __syncthreads();
  if (tid < kWave) {   // exclusive scan of the bins by one wavefront
    int run = 0;
    for (int b0 = 0; b0 <= K; b0 += kWave) {
      const int b = b0 + lane;
      const int x = b <= K ? bins[b] : 0;
      int incl = x;
      for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
      }
      if (b <= K) bins[b] = run + incl - x;
      run += __shfl(incl, kWave - 1);
    }
    if (lane == 0) {
      s_total = run;
      s_next = kDictBlock / kWave;   // pass 3's first unclaimed run
    }
  }
  __syncthreads();
  // pass 2: place the visits, grouped by n_a
#pragma unroll
  for (int u = 0; u < kDictVpt; ++u)
    if (r_pat[u] >= 0) {
      const int pos = bins[r_na[u]] + r_rank[u];
      v_pat[pos] = r_pat[u];
      v_y[pos] = r_y[u];
      v_na[pos] = (uint16_t)r_na[u];
      v_off[pos] = (uint16_t)r_off[u];
    }
  __syncthreads();
  const int nvis = s_total;
  // pass 3: outer products into the accumulators.  The visits, sorted by
  // list length, form runs of 64 (one per wavefront step) claimed from the
  // longest down: wavefront w takes run w, then the next unclaimed one, so
  // the wavefronts finish the chunk nearly together (longest runs first).
  // A run's list rows are fetched while the run before it accumulates.
  const int nruns = (nvis + kWave - 1) / kWave;
  // A run's visit records (a lane past the visits reads record 0 and keeps
  // zeros) and the first entries of each lane's list row, up to the run's
  // bound (a clamped index stays inside the patch's list row).
  auto fetch = [&](int run, VisitRow& f) {
    const int vi = nvis - kWave * (run + 1) + lane;
    const bool on = vi >= 0;
    const int vc = max(vi, 0);
    const int pid = v_pat[vc], na = (int)v_na[vc], off = (int)v_off[vc];
    const float y = v_y[vc];
    f.pid = on ? pid : 0;
    f.na = on ? na : 0;
    f.off = on ? off : 0;
    f.y = on ? (double)y : 0.0;
    // visits ascend by length, so the run's longest list is its last lane's
    // (a run's last lane always holds a visit)
    f.wmax = __builtin_amdgcn_readlane(f.na, kWave - 1);
    const int2* L = list + (size_t)f.pid * K + f.off;
    const int lim = K - 1 - f.off;
#pragma unroll
    for (int a = 0; a < kStatsCap; ++a) {
      f.raw[a] = make_int2(-1, 0);
      if (a < f.wmax) f.raw[a] = L[min(a, lim)];
    }
  };
  auto clear = [&](VisitRow& f) {
    f.pid = f.na = f.off = f.wmax = 0;
    f.y = 0.0;
#pragma unroll
    for (int a = 0; a < kStatsCap; ++a) f.raw[a] = make_int2(-1, 0);
  };
  VisitRow q[2];
  int run = tid / kWave;
  clear(q[0]);
  if (run < nruns) fetch(run, q[0]);
  while (run < nruns) {
    int nxt = 0;
    if (lane == 0) nxt = atomicAdd(&s_next, 1);
    nxt = __builtin_amdgcn_readfirstlane(nxt);
    // Stage this run's entries first (its rows were loaded one run ago), then
    // issue the next run's loads: their number depends on that run's bound,
    // so a use of this run's rows after them would wait for all of them.
    Stage s;
    stage_from(s, q[0].raw, min(q[0].na, kStatsCap));
    pin_stage(s);
    clear(q[1]);
    if (nxt < nruns) fetch(nxt, q[1]);
    const int pid = q[0].pid, na = q[0].na, wmax = q[0].wmax;
    const int2* L = list + (size_t)pid * K + q[0].off;
    const int lim = K - 1 - q[0].off;   // last index inside the patch's list row
    const StatsRow sr{reinterpret_cast<char*>(acc), sink, copy, r0, r1, (int)e0, 2 * K - 1, E,
                      pl.copy_rows, sc, q[0].y * sb};
    stats_stage<SKIP>(sr, s, wmax);
    if (wmax > kStatsCap) {
      // lists longer than the register stage (the wave's bound past
      // kStatsCap).  (1) every later entry, one at a time with the next in
      // flight, paired with the staged entries; (2) entries kStatsCap ..
      // 2 kStatsCap - 1, loaded together, replace the stage in registers:
      // their B entries and the pairs among them, by the same bodies (holding
      // them in registers through (1) as well would spill); (3) entries past
      // both stages (rare): pairs with the second stage, then B entries and
      // pairs among themselves from memory
      unsigned rb[kStatsCap];
      double wsc[kStatsCap];
      stage_rows(sr, s, rb, wsc);
      const int n2 = min(wmax, 2 * kStatsCap) - kStatsCap;
      int2 eb = L[min(kStatsCap, lim)];
      for (int b = kStatsCap; b < wmax; ++b) {
        const int2 cur = eb;
        if (b + 1 < wmax) eb = L[min(b + 1, lim)];
        stats_stage_with(sr, s, rb, wsc, b < na, cur);
      }
      int2 raw2[kStatsCap];
#pragma unroll
      for (int u = 0; u < kStatsCap; ++u) {
        raw2[u] = make_int2(-1, 0);
        if (u < n2) raw2[u] = L[min(kStatsCap + u, lim)];
      }
      stage_from(s, raw2, min(max(na - kStatsCap, 0), kStatsCap));
      stats_stage<SKIP>(sr, s, n2);
      if (wmax > 2 * kStatsCap) {
        stage_rows(sr, s, rb, wsc);
        for (int b = 2 * kStatsCap; b < wmax; ++b) {
          int2 eb = make_int2(-1, 0);
          if (b < na) eb = L[b];
          stats_stage_with(sr, s, rb, wsc, b < na, eb);
          stats_tail(sr, L, na, 2 * kStatsCap, b, b < na, eb);
        }
      }
    }
    q[0] = q[1];
    run = nxt;
  }
  __syncthreads();   // the visit records are rewritten by the next chunk
  }
  __syncthreads();
  // the copies into the group's diagonal and B entries (each thread its rows)
  for (int i = tid; i < r1 - r0; i += kDictBlock) {
    long long dsum = 0, bsum = 0;
    for (int cpi = 0; cpi < pl.copies; ++cpi) {
      dsum += cpy[(size_t)cpi * 2 * pl.copy_rows + i];
      bsum += cpy[(size_t)cpi * 2 * pl.copy_rows + pl.copy_rows + i];
    }
    const int k = r0 + i;
    acc[(int)(tri_off(k, K) - e0)] += dsum;   // entry (k, k)
    acc[E + i] += bsum;
  }
  __syncthreads();
  long long* out = dpart + (size_t)(prg * pl.chunks + c) * pl.rec_stride;
  for (int e = tid; e < rec; e += kDictBlock) out[e] = acc[e];
  if (rg == 0) {
    for (int o = kWave / 2; o > 0; o >>= 1) x2 += __shfl_xor(x2, o);
    if (lane == 0) s_x2[tid / kWave] = x2;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < kDictBlock / kWave; ++w) t += s_x2[w];
      dx2[p * pl.chunks + c] = t;
    }
  }
}

// One block per (p, 32 x 32 tile of the upper triangle of C_p): entry (k, j),
// j >= k, is the sum of the chunk partials of row k's group; the block writes
// the tile's rows and, through LDS, its transpose below the diagonal, both in
// whole rows (a write of C_p[j][k] per entry strides by K); the diagonal
// tiles also write diag and B_p, the first one X2_p.
constexpr int kRedTile = 32;
// the sum of n int64 values spaced `stride` apart, eight loads in flight (a
// loop that adds each load before issuing the next waits out one memory
// latency per value); integer adds are exact in any order
__device__ __forceinline__ long long sum_strided(const long long* __restrict__ x, size_t stride,
                                                 int n) {
  long long s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int c = 0;
  for (; c + 8 <= n; c += 8) {
    long long t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = x[(size_t)(c + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += t[u];
  }
  for (; c < n; ++c) s[0] += x[(size_t)c * stride];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

__global__ __launch_bounds__(256) void dict_reduce_kernel(
    Geom g, DictPlanDev pl, const FramePlan* __restrict__ fplan, const long long* __restrict__ dpart,
    const double* __restrict__ dx2, const DevScalars* __restrict__ scal, double* __restrict__ Cfull,
    double* __restrict__ Bvec, double* __restrict__ diag, double* __restrict__ x2p) {
  __shared__ double tile[kRedTile][kRedTile + 1];
  const int K = g.K;
  const int nt = (K + kRedTile - 1) / kRedTile, ntri = nt * (nt + 1) / 2;
  const int p = blockIdx.x / ntri;
  int t = blockIdx.x - p * ntri, ti = 0;
  while (t >= nt - ti) {   // tile (ti, tj), ti <= tj, rows of the upper triangle in order
    t -= nt - ti;
    ++ti;
  }
  const int tj = ti + t;
  const int cc = fplan->dict_chunks;
  const double inv_c = 1.0 / scal->scale_c;
  double* C = Cfull + (size_t)p * K * K;
  const int tx = threadIdx.x % kRedTile, ty = threadIdx.x / kRedTile;
  const int j = tj * kRedTile + tx;
  for (int r = ty; r < kRedTile; r += 256 / kRedTile) {
    const int k = ti * kRedTile + r;
    double v = 0.0;
    if (k < K && j < K && j >= k) {
      int rg = 0;
      while (rg + 1 < pl.RG && pl.row0[rg + 1] <= k) ++rg;
      const long long* rec = dpart + (size_t)(p * pl.RG + rg) * pl.chunks * pl.rec_stride;
      const long long ek = tri_off(k, K) - pl.ent0[rg] - k;
      const long long sum = sum_strided(rec + ek + j, (size_t)pl.rec_stride, cc);
      v = (double)sum * inv_c;
      C[(size_t)k * K + j] = v;
      if (j == k) diag[(size_t)p * K + k] = v;
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < kRedTile; r += 256 / kRedTile) {
    const int jr = tj * kRedTile + r, kc = ti * kRedTile + tx;
    if (jr < K && kc < jr) C[(size_t)jr * K + kc] = tile[tx][r];
  }
  if (ti == tj && threadIdx.x < kRedTile) {
    const int k = ti * kRedTile + threadIdx.x;
    if (k < K) {
      int rg = 0;
      while (rg + 1 < pl.RG && pl.row0[rg + 1] <= k) ++rg;
      const long long* rec = dpart + (size_t)(p * pl.RG + rg) * pl.chunks * pl.rec_stride;
      const int E = (int)(pl.ent0[rg + 1] - pl.ent0[rg]);
      const long long sum = sum_strided(rec + E + (k - pl.row0[rg]), (size_t)pl.rec_stride, cc);
      Bvec[(size_t)p * K + k] = (double)sum / scal->scale_b;
    }
    if (ti == 0 && threadIdx.x == 0) {
      double x2 = 0.0;
      for (int c = 0; c < cc; ++c) x2 += dx2[p * pl.chunks + c];
      x2p[p] = x2;
    }
  }
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The standard normal of the draw of d_jp: Box-Muller on the DICT Philox
// block (p, j, t); `stream` carries the tag and the problem id.
__device__ __forceinline__ double chain_normal(int p, int j, uint32_t t, uint32_t stream,
                                               uint32_t key0, uint32_t key1) {
  const Block4 rb = philox10((uint32_t)p, (uint32_t)j, t, stream, key0, key1);
  return sqrt(-2.0 * log(u01d(rb.w0))) * cos(2.0 * M_PI * u01d(rb.w1));
}

// One wavefront per position p.  Lane l owns components j = l + 64 m of d
// and of u = C_p d.  With g_k = gamma_eps / lam_k and the constant
// t_k = g_k (B_k + C_kk d_k) + n_k / sqrt(lam_k) (d_k not yet redrawn),
// step k is d_k' = t_k - g_k u_k, and every lane adds C_p[k][j] (d_k' - d_k)
// to its u_j: no reduction per step, and at the end d.u = d^T C_p d.
// C: C_p (K x K, symmetric) in global memory or LDS; Bp, diagp: B_p and the
// diagonal of C_p; x2: X2_p.
// scale: the data statistics enter the conditional multiplied by it (a
// mini-batch step's N / n_b), i.e. gamma_eps scale in place of gamma_eps in
// lam and g; the residual sum of squares stays the batch's own.
// u0, nrm: u = C_p d and the normals n_j when the caller has them at hand.
template <int KPL, int PF>
__device__ __forceinline__ void chain_run(const Geom& g, int p, int lane, const double* C,
                                          const double* Bp, const double* diagp, double x2,
                                          DevScalars* scal, float* __restrict__ D,
                                          double* __restrict__ sumr2_p, double scale,
                                          uint32_t key0, uint32_t key1, uint32_t stream,
                                          const double* u0 = nullptr, const double* nrm = nullptr) {
  static_assert(kWave % PF == 0, "a ring slot keeps its row across register groups");
  const int K = g.K, P = g.P;
  const uint32_t t = (uint32_t)scal->t;
  // the tag comes with `stream`, the problem id from the device scalars
  stream = (stream & 0xFFu) | (scal->problem_id << 8);
  const double ge = scal->gamma_eps * scale;
  double dreg[KPL], ureg[KPL], greg[KPL], treg[KPL], breg[KPL];
#pragma unroll
  for (int m = 0; m < KPL; ++m) {
    const int j = lane + kWave * m;
    dreg[m] = ureg[m] = greg[m] = treg[m] = breg[m] = 0.0;
    if (j < K) {
      const double n = nrm ? nrm[j] : chain_normal(p, j, t, stream, key0, key1);
      const double cjj = diagp[j];
      const double lam = (double)P + ge * cjj;
      breg[m] = Bp[j];
      dreg[m] = (double)D[(size_t)j * P + p];
      greg[m] = ge / lam;
      treg[m] = fma(greg[m], fma(cjj, dreg[m], breg[m]), n / sqrt(lam));
    }
  }
  // u = C d with the old dictionary: given (u0), or rows streamed PF at a time
  if (u0) {
#pragma unroll
    for (int m = 0; m < KPL; ++m) {
      const int j = lane + kWave * m;
      if (j < K) ureg[m] = u0[j];
    }
  }
  for (int kb = 0; u0 == nullptr && kb < K; kb += PF) {
    double v[PF][KPL];
#pragma unroll
    for (int u = 0; u < PF; ++u)
#pragma unroll
      for (int m = 0; m < KPL; ++m) {
        const int j = lane + kWave * m, k = kb + u;
        v[u][m] = (k < K && j < K) ? C[(size_t)k * K + j] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int k = kb + u;
      if (k < K) {
        double dk = 0.0;
#pragma unroll
        for (int m = 0; m < KPL; ++m)
          if ((k >> 6) == m) dk = readlane_d(dreg[m], k & 63);
#pragma unroll
        for (int m = 0; m < KPL; ++m) ureg[m] = fma(v[u][m], dk, ureg[m]);
      }
    }
  }
  // the chain, rows of C_p (= columns, by symmetry) prefetched PF ahead.
  // Loads are unconditional (row and column clamped into the matrix; rows
  // past K are never consumed and lanes past K only feed u entries that are
  // never read), so a refill lands in its ring slot with no select and is
  // waited for only PF steps later.  The loop is split by register group m
  // (steps 64 m .. 64 m + 63), so the readlanes and the d update name one
  // register each.
  double ring[PF][KPL];
#pragma unroll
  for (int u = 0; u < PF; ++u)
#pragma unroll
    for (int m = 0; m < KPL; ++m)
      ring[u][m] = C[(size_t)min(u, K - 1) * K + min(lane + kWave * m, K - 1)];
#pragma unroll
  for (int m = 0; m < KPL; ++m) {
    const int kend = min(K, kWave * (m + 1));
    for (int kb = kWave * m; kb < kend; kb += PF) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int k = kb + u;
        if (k < kend) {
          const int kl = k - kWave * m;
          // every lane forms t - g u from its own registers; lane kl's value is
          // the draw of d_k, and only its change is broadcast (one readlane
          // on the step-to-step path instead of four and their moves)
          const double dn = fma(-greg[m], ureg[m], treg[m]);
          const double delta = readlane_d(dn - dreg[m], kl);
#pragma unroll
          for (int mm = 0; mm < KPL; ++mm) ureg[mm] = fma(ring[u][mm], delta, ureg[mm]);
          if (lane == kl) dreg[m] = dn;
        }
        // the refill is issued on every step, taken or not, so each trip
        // issues the same loads and a slot's wait counts only the loads
        // issued after it, not every load in flight
        const int kn = min(k + PF, K - 1);
#pragma unroll
        for (int mm = 0; mm < KPL; ++mm)
          ring[u][mm] = C[(size_t)kn * K + min(lane + kWave * mm, K - 1)];
      }
    }
  }
  // new atoms' column p; residual sum of squares X2 - 2 d.B + d.(C d).
  // Every draw stays in dreg, so a non-finite draw is found here.
  double quad = 0.0, lin = 0.0;
  bool bad = false;
#pragma unroll
  for (int m = 0; m < KPL; ++m) {
    const int j = lane + kWave * m;
    if (j < K) {
      bad = bad || !isfinite(dreg[m]);
      D[(size_t)j * P + p] = (float)dreg[m];
      quad = fma(ureg[m], dreg[m], quad);
      lin = fma(breg[m], dreg[m], lin);
    }
  }
  quad = wave_sum_d(quad);
  lin = wave_sum_d(lin);
  const bool any_bad = __builtin_amdgcn_ballot_w64(bad) != 0;
  if (lane == 0) {
    sumr2_p[p] = x2 - 2.0 * lin + quad;
    if (any_bad) atomicOr(&scal->status, 1);
  }
}

template <int KPL, int PF>
__global__ __launch_bounds__(kWave) void dict_chain_kernel(
    Geom g, const double* __restrict__ Cfull, const double* __restrict__ Bvec,
    const double* __restrict__ diag, const double* __restrict__ x2p, DevScalars* scal,
    float* __restrict__ D, double* __restrict__ sumr2_p, double scale, uint32_t key0,
    uint32_t key1, uint32_t stream) {
  const int p = blockIdx.x, K = g.K;
  chain_run<KPL, PF>(g, p, threadIdx.x, Cfull + (size_t)p * K * K, Bvec + (size_t)p * K,
                     diag + (size_t)p * K, x2p[p], scal, D, sumr2_p, scale, key0, key1, stream);
}

// The chain with C_p staged in LDS.  One block per p sums the chunk partials
// of the packed triangle into the symmetric K x K matrix in LDS, forms u = C_p d (old d) with
// all its threads (partial sums over 1024 / K slices of k, added in a fixed
// order), then wavefront 0 runs the chain reading rows from LDS.
template <int KPL>
__global__ __launch_bounds__(1024) void dict_chain_lds_kernel(
    Geom g, DictPlanDev pl, const FramePlan* __restrict__ fplan, const long long* __restrict__ dpart,
    const double* __restrict__ dx2, DevScalars* scal, float* __restrict__ D,
    double* __restrict__ sumr2_p, double scale, uint32_t key0, uint32_t key1, uint32_t stream) {
  extern __shared__ double Cs[];                 // K x K, then the u partials
  __shared__ double s_B[kChainLdsMaxK], s_diag[kChainLdsMaxK], s_d[kChainLdsMaxK],
      s_u[kChainLdsMaxK], s_n[kChainLdsMaxK];
  __shared__ double s_x2;
  const int p = blockIdx.x, K = g.K, P = g.P, tid = threadIdx.x;
  const int E = K * (K + 1) / 2;
  // The statistics of position p: its chunk partials (one row group: the
  // packed upper triangle of C_p, then B_p) summed over the frame's chunks,
  // each entry loaded once (coalesced, two chunks in flight), scaled as the
  // fixed point was, and the triangle written into both halves of the
  // symmetric matrix in LDS.
  constexpr int kRedPT = 9;   // ceil((K (K + 1) / 2 + K) / 1024) for K <= 128
  {
    const int cc = fplan->dict_chunks;
    const long long* rec = dpart + (size_t)p * pl.chunks * pl.rec_stride;
    long long v[kRedPT];
#pragma unroll
    for (int i = 0; i < kRedPT; ++i) v[i] = 0;
    int c = 0;
    for (; c + 1 < cc; c += 2) {
      long long t0[kRedPT], t1[kRedPT];
#pragma unroll
      for (int i = 0; i < kRedPT; ++i) {
        const int e = min(tid + 1024 * i, E + K - 1);
        t0[i] = rec[(size_t)c * pl.rec_stride + e];
        t1[i] = rec[(size_t)(c + 1) * pl.rec_stride + e];
      }
#pragma unroll
      for (int i = 0; i < kRedPT; ++i) v[i] += t0[i] + t1[i];
    }
    if (c < cc) {
#pragma unroll
      for (int i = 0; i < kRedPT; ++i)
        v[i] += rec[(size_t)c * pl.rec_stride + min(tid + 1024 * i, E + K - 1)];
    }
    const double inv_c = 1.0 / scal->scale_c, sbs = scal->scale_b;
#pragma unroll
    for (int i = 0; i < kRedPT; ++i) {
      const int e = tid + 1024 * i;
      if (e < E) {
        // row a of entry e: rows a = K - 1, K - 2, ... hold 1, 2, ... entries
        // from the end, so q = K - 1 - a is the triangular root of E - 1 - e
        const int r = E - 1 - e;
        int q = (int)((sqrtf(8.f * (float)r + 1.f) - 1.f) * 0.5f);
        if (q * (q + 1) / 2 > r) --q;
        if ((q + 1) * (q + 2) / 2 <= r) ++q;
        const int a = K - 1 - q;
        const int bcol = a + (e - (a * K - a * (a - 1) / 2));
        const double x = (double)v[i] * inv_c;
        Cs[a * K + bcol] = x;
        Cs[bcol * K + a] = x;
      } else if (e < E + K) {
        s_B[e - E] = (double)v[i] / sbs;
      }
    }
    if (tid == 0) {
      double x2 = 0.0;
      for (int cq = 0; cq < cc; ++cq) x2 += dx2[p * pl.chunks + cq];
      s_x2 = x2;
    }
  }
  for (int k = tid; k < K; k += 1024) s_d[k] = (double)D[(size_t)k * P + p];
  __syncthreads();
  for (int k = tid; k < K; k += 1024) s_diag[k] = Cs[k * K + k];
  // the chain's normals, drawn by the wavefronts after the first while the
  // block forms u (the chain itself runs on the first)
  if (tid >= kWave && tid - kWave < K)
    s_n[tid - kWave] = chain_normal(p, tid - kWave, (uint32_t)scal->t,
                                    (stream & 0xFFu) | (scal->problem_id << 8), key0, key1);
  // u_j = sum_k C[k][j] d_k: slice s of the k range per thread group
  double* up = Cs + (size_t)K * K;               // [slices][K]
  const int slices = 1024 / K, per = (K + slices - 1) / slices;
  if (tid < slices * K) {
    const int j = tid % K, sl = tid / K;
    double acc = 0.0;
    for (int k = sl * per; k < min(K, (sl + 1) * per); ++k) acc = fma(Cs[k * K + j], s_d[k], acc);
    up[sl * K + j] = acc;
  }
  __syncthreads();
  for (int j = tid; j < K; j += 1024) {
    double u = 0.0;
    for (int sl = 0; sl < slices; ++sl) u += up[sl * K + j];
    s_u[j] = u;
  }
  __syncthreads();
  if (tid < kWave)
    // 8 row loads in flight: the LDS counter holds at most 15 outstanding,
    // so a deeper ring makes every step wait for all of them
    chain_run<KPL, 8 / KPL>(g, p, tid, Cs, s_B, s_diag, s_x2, scal, D, sumr2_p, scale, key0, key1,
                            stream, s_u, s_n);
}

static DictPlanDev to_dev(const Geom& g, const DictPlan& plan) {
  DictPlanDev d{};
  d.RG = plan.RG;
  d.chunks = plan.chunks;
  d.chunk_visits = plan.chunk_visits;
  d.xcd = plan.xcd;
  d.K = g.K;
  d.copies = plan.copies;
  d.copy_rows = plan.copy_rows;
  long long stride = 0;
  for (int r = 0; r <= plan.RG; ++r) {
    d.row0[r] = plan.row0[r];
    d.ent0[r] = plan.ent0[r];
  }
  for (int r = 0; r < plan.RG; ++r) {
    const long long len = (plan.ent0[r + 1] - plan.ent0[r]) + (plan.row0[r + 1] - plan.row0[r]);
    stride = len > stride ? len : stride;
  }
  d.rec_stride = stride;
  return d;
}

// With several row groups: per patch, the number of its list entries below
// each later group's first row (lists ascend), so a block of that group
// starts the patch's pairs there.  One thread per patch (of the step's
// batch); the first entries are loaded together, a longer list continues
// from memory only while its entries stay below the boundary.
__global__ __launch_bounds__(256) void list_groups_kernel(int N, int K, DictPlanDev pl,
                                                          const int2* __restrict__ list,
                                                          const int32_t* __restrict__ nact,
                                                          uint16_t* __restrict__ goff, int n_batches,
                                                          int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N || (n_batches > 1 && i % n_batches != batch)) return;
  const int na = nact[i];
  const int2* L = list + (size_t)i * K;
  int x[kStatsCap];
#pragma unroll
  for (int a = 0; a < kStatsCap; ++a) x[a] = a < na ? L[a].x : K;
  for (int r = 1; r < pl.RG; ++r) {
    const int lo = pl.row0[r];
    int e = 0;
#pragma unroll
    for (int a = 0; a < kStatsCap; ++a) e += x[a] < lo ? 1 : 0;
    if (e == kStatsCap)
      while (e < na && L[e].x < lo) ++e;
    goff[(size_t)i * (pl.RG - 1) + (r - 1)] = (uint16_t)e;
  }
}

hipError_t launch_list_groups(const Geom& g, const Buffers& b, const DictPlan& plan, int cur,
                              int n_batches, int batch, hipStream_t st) {
  if (plan.RG <= 1) return hipSuccess;
  list_groups_kernel<<<(g.N + 255) / 256, 256, 0, st>>>(g.N, g.K, to_dev(g, plan), b.list[cur],
                                                        b.nact[cur], b.goff, n_batches, batch);
  return hipGetLastError();
}

hipError_t launch_dict_stats(const Geom& g, const Buffers& b, const DictPlan& plan, int grid_chunks,
                             int cur, int n_batches, int batch, hipStream_t st) {
  const DictPlanDev d = to_dev(g, plan);
  // blocks for grid_chunks chunk slots per (p, row group): the frame's count
  // when the host knows it, else all of them (blocks of slots the frame
  // leaves empty return at once)
  const int blocks = g.P * plan.RG * std::max(1, std::min(grid_chunks, plan.chunks));
  // the LDS holds visit records for the largest chunk the plan allows
  const size_t lds = dict_stats_lds(g.K, d.rec_stride, plan.copies * 2 * plan.copy_rows, plan.chunk_visits);
  const bool skip = plan.RG >= 2;
  hipError_t e = hipFuncSetAttribute(
      skip ? (const void*)dict_stats_kernel<true> : (const void*)dict_stats_kernel<false>,
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (skip)
    dict_stats_kernel<true><<<blocks, kDictBlock, lds, st>>>(
        g, d, b.plan, b.vpatch, b.omega_y, b.list[cur], b.nact[cur], b.goff, b.scal, b.dpart, b.dx2,
        n_batches, batch);
  else
    dict_stats_kernel<false><<<blocks, kDictBlock, lds, st>>>(
        g, d, b.plan, b.vpatch, b.omega_y, b.list[cur], b.nact[cur], b.goff, b.scal, b.dpart, b.dx2,
        n_batches, batch);
  return hipGetLastError();
}

hipError_t launch_dict_reduce(const Geom& g, const Buffers& b, const DictPlan& plan,
                              hipStream_t st) {
  const DictPlanDev d = to_dev(g, plan);
  const int nt = (g.K + kRedTile - 1) / kRedTile;
  dict_reduce_kernel<<<g.P * (nt * (nt + 1) / 2), 256, 0, st>>>(g, d, b.plan, b.dpart, b.dx2, b.scal, b.Cfull,
                                                b.Bvec, b.diag, b.x2p);
  return hipGetLastError();
}

hipError_t launch_dict_chain(const Geom& g, const Buffers& b, const DictPlan& plan, double scale,
                             uint32_t key0, uint32_t key1, uint32_t stream, hipStream_t st) {
  (void)plan;
  const int kpl = (g.K + kWave - 1) / kWave;
#define BPFA_CHAIN(KP, PFV)                                                              \
  dict_chain_kernel<KP, PFV><<<g.P, kWave, 0, st>>>(g, b.Cfull, b.Bvec, b.diag, b.x2p,  \
                                                    b.scal, b.D, b.sumr2_p, scale, key0, \
                                                    key1, stream)
  if (kpl <= 1) BPFA_CHAIN(1, 16);
  else if (kpl <= 2) BPFA_CHAIN(2, 16);
  else if (kpl <= 4) BPFA_CHAIN(4, 8);
  else if (kpl <= 8) BPFA_CHAIN(8, 4);
  else if (kpl <= 16) BPFA_CHAIN(16, 2);
  else return hipErrorInvalidValue;
#undef BPFA_CHAIN
  return hipGetLastError();
}

size_t dict_chain_lds_bytes(int K) { return (size_t)K * K * 8 + (size_t)(1024 / K) * K * 8; }

hipError_t launch_dict_reduce_chain_lds(const Geom& g, const Buffers& b, const DictPlan& plan,
                                        double scale, uint32_t key0, uint32_t key1,
                                        uint32_t stream, hipStream_t st) {
  if (g.K > kChainLdsMaxK || plan.RG != 1) return hipErrorInvalidValue;
  const DictPlanDev d = to_dev(g, plan);
  hipError_t e = hipSuccess;
  const size_t lds = dict_chain_lds_bytes(g.K);
  if (g.K <= kWave) {
    e = hipFuncSetAttribute((const void*)dict_chain_lds_kernel<1>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dict_chain_lds_kernel<1><<<g.P, 1024, lds, st>>>(g, d, b.plan, b.dpart, b.dx2, b.scal, b.D,
                                                     b.sumr2_p, scale, key0, key1, stream);
  } else {
    e = hipFuncSetAttribute((const void*)dict_chain_lds_kernel<2>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dict_chain_lds_kernel<2><<<g.P, 1024, lds, st>>>(g, d, b.plan, b.dpart, b.dx2, b.scal, b.D,
                                                     b.sumr2_p, scale, key0, key1, stream);
  }
  return hipGetLastError();
}

}  // namespace bpfa
