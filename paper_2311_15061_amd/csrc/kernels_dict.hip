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
//   the patch whose origin is q - b(p)) are first grouped by the patch's
//   number of active atoms n_a in LDS, so a wavefront's lanes share a pair
//   loop bound; then a lane stages a patch's active entries in registers and
//   adds its outer product into LDS.  Sums are 64-bit fixed point: the
//   binary64 product of two binary32 weights is exact, it is scaled by a power
//   of two and rounded to an integer by adding 1.5 * 2^52 (exact for
//   |x| < 2^51); integer adds are associative, so the statistics do not
//   depend on scheduling.
// dict_reduce_kernel: sums the chunk partials, one block per (p, row k),
//   into the symmetric binary64 C_p, B_p and the diagonal.
// dict_chain_kernel: one wavefront per p runs the chain with rows of C_p
//   prefetched ahead of use, keeping u = C_p d current instead of reducing a
//   dot product per step, draws d_kp with the Philox DICT stream, and forms
//   the residual sum of squares.
#include "internal.hpp"
#include "philox.hpp"

namespace bpfa {

constexpr int kStatsCap = 16;   // active entries of a patch held in registers

struct DictPlanDev {
  int RG, chunks, K, chunk_visits, xcd;
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

__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Per frame: for every position p and observed pixel v (in omega order), the
// slot of the patch whose origin is q_v - b(p), or -1 when that origin is
// off the grid; and the observed values in omega order.
__global__ __launch_bounds__(256) void visit_table_kernel(Geom g, int nom, const int4* __restrict__ omega_c,
                                                          const int32_t* __restrict__ omega,
                                                          const float* __restrict__ image,
                                                          const int32_t* __restrict__ pcoord,
                                                          const int32_t* __restrict__ inv_perm,
                                                          int32_t* __restrict__ vslot,
                                                          float* __restrict__ omega_y) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (v >= nom) return;
  int bc[kMaxDim] = {0, 0, 0, 0};
  for (int d = 0; d < g.ndim; ++d) bc[d] = pcoord[p * kMaxDim + d];
  const int pidx = visit_patch(g, omega_c[v], bc);
  vslot[(size_t)p * g.Mtot + v] = pidx >= 0 ? inv_perm[pidx] : -1;
  if (p == 0) omega_y[v] = image[omega[v]];
}

hipError_t launch_visit_table(const Geom& g, const Buffers& b, int n_omega, hipStream_t st) {
  if (n_omega <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n_omega + 255) / 256), (unsigned)g.P);
  visit_table_kernel<<<grid, 256, 0, st>>>(g, n_omega, b.omega_c, b.omega, b.image, b.pcoord,
                                           b.inv_perm, b.vslot, b.omega_y);
  return hipGetLastError();
}

// LDS: rec int64 accumulators | K + 1 int bin starts | chunk visits (slot
// int32, y float, n_a uint16).  Visits are bucketed by n_a inside the block so
// each wavefront's pair loop runs to a bound its lanes share.
__global__ __launch_bounds__(kDictBlock) void dict_stats_kernel(
    Geom g, DictPlanDev pl, int nom, const int32_t* __restrict__ vslot,
    const float* __restrict__ omega_y, const int2* __restrict__ list,
    const int32_t* __restrict__ nact, const DevScalars* __restrict__ scal,
    long long* __restrict__ dpart, double* __restrict__ dx2) {
  extern __shared__ long long acc[];
  __shared__ double s_x2[kDictBlock / kWave];
  __shared__ int s_total;
  // block -> (chunk c, position p, row group rg).  Workgroups are dispatched
  // round-robin over the 8 XCDs; with chunks a multiple of 8 every block of
  // chunk c has blockIdx = c mod 8, so the P blocks that read the same
  // patches' lists share one L2.
  int c, prg;
  if (pl.xcd) {
    const int cg = pl.chunks >> 3, j = blockIdx.x >> 3;
    c = (blockIdx.x & 7) + 8 * (j % cg);
    prg = j / cg;
  } else {
    c = blockIdx.x % pl.chunks;
    prg = blockIdx.x / pl.chunks;
  }
  const int p = prg / pl.RG, rg = prg % pl.RG;
  const int r0 = pl.row0[rg], r1 = pl.row0[rg + 1];
  const long long e0 = pl.ent0[rg];
  const int E = (int)(pl.ent0[rg + 1] - e0);
  const int rec = E + (r1 - r0);
  const int K = g.K;
  int* bins = reinterpret_cast<int*>(acc + pl.rec_stride);          // K + 1 counts, then starts
  int* v_slot = bins + (K + 1);
  float* v_y = reinterpret_cast<float*>(v_slot + pl.chunk_visits);
  uint16_t* v_na = reinterpret_cast<uint16_t*>(v_y + pl.chunk_visits);
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  for (int e = tid; e < rec; e += kDictBlock) acc[e] = 0;

  const double sc = scal->scale_c, sb = scal->scale_b;
  const int32_t* vs = vslot + (size_t)p * g.Mtot;
  double x2 = 0.0;

  // block c of its (p, row group) takes chunks c, c + chunks, ... of the observed pixels
  for (int ch = c; ch * pl.chunk_visits < nom; ch += pl.chunks) {
  const int v0 = ch * pl.chunk_visits, v1 = min(nom, v0 + pl.chunk_visits);
  for (int e = tid; e <= K; e += kDictBlock) bins[e] = 0;
  __syncthreads();

  // pass 1: this thread's visits (at most kDictVpt) in registers; rank within its n_a bin
  int r_slot[kDictVpt], r_na[kDictVpt], r_rank[kDictVpt];
  float r_y[kDictVpt];
#pragma unroll
  for (int u = 0; u < kDictVpt; ++u) {
    const int v = v0 + tid + u * kDictBlock;
    r_slot[u] = -1;
    r_y[u] = 0.f;
    if (v < v1) {
      r_slot[u] = vs[v];
      r_y[u] = omega_y[v];
    }
  }
#pragma unroll
  for (int u = 0; u < kDictVpt; ++u) r_na[u] = r_slot[u] >= 0 ? nact[r_slot[u]] : 0;
#pragma unroll
  for (int u = 0; u < kDictVpt; ++u) {
    r_rank[u] = 0;
    if (r_slot[u] >= 0) {
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
    if (lane == 0) s_total = run;
  }
  __syncthreads();
  // pass 2: place the visits, grouped by n_a
#pragma unroll
  for (int u = 0; u < kDictVpt; ++u)
    if (r_slot[u] >= 0) {
      const int pos = bins[r_na[u]] + r_rank[u];
      v_slot[pos] = r_slot[u];
      v_y[pos] = r_y[u];
      v_na[pos] = (uint16_t)r_na[u];
    }
  __syncthreads();
  const int nvis = s_total;
  // pass 3: outer products into the accumulators
  for (int vb = 0; vb < nvis; vb += kDictBlock) {
    const int vi = vb + tid;
    const bool on = vi < nvis;
    const int slot = on ? v_slot[vi] : 0;
    const int na = on ? (int)v_na[vi] : 0;
    const double y = on ? (double)v_y[vi] : 0.0;
    const int wmax = __builtin_amdgcn_readfirstlane(wave_max_i(na));
    const int2* L = list + (size_t)slot * K;
    int kk[kStatsCap];
    double ww[kStatsCap];
#pragma unroll
    for (int a = 0; a < kStatsCap; ++a) {
      kk[a] = -1;
      ww[a] = 0.0;
      if (a < wmax && a < na) {
        const int2 e = L[a];
        kk[a] = e.x;
        ww[a] = (double)__int_as_float(e.y);
      }
    }
    const double ysb = y * sb;
#pragma unroll
    for (int a = 0; a < kStatsCap; ++a) {
      if (a < wmax) {
        if (kk[a] >= r0 && kk[a] < r1) {
          atomicAdd((unsigned long long*)&acc[E + (kk[a] - r0)], to_fixed(ww[a] * ysb));
          const double wa = ww[a] * sc;
          const int base = (int)(tri_off(kk[a], K) - e0) - kk[a];
#pragma unroll
          for (int b = a; b < kStatsCap; ++b)
            if (b < wmax && kk[b] >= 0)
              atomicAdd((unsigned long long*)&acc[base + kk[b]], to_fixed(wa * ww[b]));
        }
      }
    }
    // entries beyond the register stage: every pair (a, b), a <= b, with b >= kStatsCap
    if (wmax > kStatsCap) {
      for (int b = kStatsCap; b < na; ++b) {
        const int2 eb = L[b];
        const double wb = (double)__int_as_float(eb.y);
        if (eb.x >= r0 && eb.x < r1)
          atomicAdd((unsigned long long*)&acc[E + (eb.x - r0)], to_fixed(wb * ysb));
        for (int a = 0; a <= b; ++a) {
          const int2 ea = L[a];
          if (ea.x >= r0 && ea.x < r1) {
            const int base = (int)(tri_off(ea.x, K) - e0) - ea.x;
            atomicAdd((unsigned long long*)&acc[base + eb.x],
                      to_fixed((double)__int_as_float(ea.y) * sc * wb));
          }
        }
      }
    }
  }
  __syncthreads();   // the visit records are rewritten by the next chunk
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

// one block per (p, row k): C_p[k][j] = C_p[j][k] for j >= k, B_p[k], diag, X2_p
__global__ __launch_bounds__(256) void dict_reduce_kernel(
    Geom g, DictPlanDev pl, const long long* __restrict__ dpart, const double* __restrict__ dx2,
    const DevScalars* __restrict__ scal, double* __restrict__ Cfull, double* __restrict__ Bvec,
    double* __restrict__ diag, double* __restrict__ x2p) {
  const int K = g.K;
  const int p = blockIdx.x / K, k = blockIdx.x % K;
  int rg = 0;
  while (rg + 1 < pl.RG && pl.row0[rg + 1] <= k) ++rg;
  const long long e0 = pl.ent0[rg];
  const int E = (int)(pl.ent0[rg + 1] - e0);
  const long long* rec = dpart + (size_t)(p * pl.RG + rg) * pl.chunks * pl.rec_stride;
  const long long ek = tri_off(k, K) - e0 - k;
  const double inv_c = 1.0 / scal->scale_c;
  double* C = Cfull + (size_t)p * K * K;
  for (int j = k + threadIdx.x; j < K; j += blockDim.x) {
    long long sum = 0;
    for (int c = 0; c < pl.chunks; ++c) sum += rec[(size_t)c * pl.rec_stride + ek + j];
    const double v = (double)sum * inv_c;
    C[(size_t)k * K + j] = v;
    C[(size_t)j * K + k] = v;
    if (j == k) diag[(size_t)p * K + k] = v;
  }
  if (threadIdx.x == 0) {
    long long sum = 0;
    for (int c = 0; c < pl.chunks; ++c) sum += rec[(size_t)c * pl.rec_stride + E + (k - pl.row0[rg])];
    Bvec[(size_t)p * K + k] = (double)sum / scal->scale_b;
    if (k == 0) {
      double x2 = 0.0;
      for (int c = 0; c < pl.chunks; ++c) x2 += dx2[p * pl.chunks + c];
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

// One wavefront per position p.  Lane l owns components j = l + 64 m of d
// and of u = C_p d.  With g_k = gamma_eps / lam_k and the constant
// t_k = g_k (B_k + C_kk d_k) + n_k / sqrt(lam_k) (d_k not yet redrawn),
// step k is d_k' = t_k - g_k u_k, and every lane adds C_p[k][j] (d_k' - d_k)
// to its u_j: no reduction per step, and at the end d.u = d^T C_p d.
template <int KPL, int PF>
__global__ __launch_bounds__(kWave) void dict_chain_kernel(
    Geom g, const double* __restrict__ Cfull, const double* __restrict__ Bvec,
    const double* __restrict__ diag, const double* __restrict__ x2p, DevScalars* scal,
    float* __restrict__ D, double* __restrict__ sumr2_p, uint32_t key0, uint32_t key1,
    uint32_t stream) {
  const int p = blockIdx.x, lane = threadIdx.x, K = g.K, P = g.P;
  const double* C = Cfull + (size_t)p * K * K;
  const uint32_t t = (uint32_t)scal->t;
  const double ge = scal->gamma_eps;
  double dreg[KPL], ureg[KPL], greg[KPL], treg[KPL], breg[KPL];
#pragma unroll
  for (int m = 0; m < KPL; ++m) {
    const int j = lane + kWave * m;
    dreg[m] = ureg[m] = greg[m] = treg[m] = breg[m] = 0.0;
    if (j < K) {
      const Block4 rb = philox10((uint32_t)p, (uint32_t)j, t, stream, key0, key1);
      const double n = sqrt(-2.0 * log(u01d(rb.w0))) * cos(2.0 * M_PI * u01d(rb.w1));
      const double cjj = diag[(size_t)p * K + j];
      const double lam = (double)P + ge * cjj;
      breg[m] = Bvec[(size_t)p * K + j];
      dreg[m] = (double)D[(size_t)j * P + p];
      greg[m] = ge / lam;
      treg[m] = fma(greg[m], fma(cjj, dreg[m], breg[m]), n / sqrt(lam));
    }
  }
  // u = C d with the old dictionary, rows streamed PF at a time
  for (int kb = 0; kb < K; kb += PF) {
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
  // the chain, rows of C_p (= columns, by symmetry) prefetched PF ahead
  double ring[PF][KPL];
#pragma unroll
  for (int u = 0; u < PF; ++u)
#pragma unroll
    for (int m = 0; m < KPL; ++m) {
      const int j = lane + kWave * m;
      ring[u][m] = (u < K && j < K) ? C[(size_t)u * K + j] : 0.0;
    }
  bool bad = false;
  for (int kb = 0; kb < K; kb += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int k = kb + u;
      if (k < K) {
        double uk = 0.0, dk = 0.0, gk = 0.0, tk = 0.0;
#pragma unroll
        for (int m = 0; m < KPL; ++m)
          if ((k >> 6) == m) {
            const int kl = k & 63;
            uk = readlane_d(ureg[m], kl);
            dk = readlane_d(dreg[m], kl);
            gk = readlane_d(greg[m], kl);
            tk = readlane_d(treg[m], kl);
          }
        const double dn = fma(-gk, uk, tk);
        bad = bad || !isfinite(dn);
        const double delta = dn - dk;
#pragma unroll
        for (int m = 0; m < KPL; ++m) {
          ureg[m] = fma(ring[u][m], delta, ureg[m]);
          if (k == lane + kWave * m) dreg[m] = dn;
        }
        const int kn = k + PF;
#pragma unroll
        for (int m = 0; m < KPL; ++m) {
          const int j = lane + kWave * m;
          ring[u][m] = (kn < K && j < K) ? C[(size_t)kn * K + j] : 0.0;
        }
      }
    }
  }
  // new atoms' column p; residual sum of squares X2 - 2 d.B + d.(C d)
  double quad = 0.0, lin = 0.0;
#pragma unroll
  for (int m = 0; m < KPL; ++m) {
    const int j = lane + kWave * m;
    if (j < K) {
      D[(size_t)j * P + p] = (float)dreg[m];
      quad = fma(ureg[m], dreg[m], quad);
      lin = fma(breg[m], dreg[m], lin);
    }
  }
  quad = wave_sum_d(quad);
  lin = wave_sum_d(lin);
  if (lane == 0) {
    sumr2_p[p] = x2p[p] - 2.0 * lin + quad;
    if (bad) atomicOr(&scal->status, 1);
  }
}

static DictPlanDev to_dev(const Geom& g, const DictPlan& plan) {
  DictPlanDev d{};
  d.RG = plan.RG;
  d.chunks = plan.chunks;
  d.chunk_visits = plan.chunk_visits;
  d.xcd = plan.xcd;
  d.K = g.K;
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

hipError_t launch_dict_stats(const Geom& g, const Buffers& b, const DictPlan& plan, int cur,
                             int n_omega, hipStream_t st) {
  const DictPlanDev d = to_dev(g, plan);
  const int blocks = g.P * plan.RG * plan.chunks;
  // the LDS holds visit records for the largest chunk the plan allows
  const size_t lds = dict_stats_lds(g.K, d.rec_stride, plan.chunk_visits);
  hipError_t e = hipFuncSetAttribute((const void*)dict_stats_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  dict_stats_kernel<<<blocks, kDictBlock, lds, st>>>(g, d, n_omega, b.vslot, b.omega_y,
                                                     b.list[cur], b.nact[cur], b.scal, b.dpart,
                                                     b.dx2);
  return hipGetLastError();
}

hipError_t launch_dict_reduce(const Geom& g, const Buffers& b, const DictPlan& plan,
                              hipStream_t st) {
  const DictPlanDev d = to_dev(g, plan);
  dict_reduce_kernel<<<g.P * g.K, 256, 0, st>>>(g, d, b.dpart, b.dx2, b.scal, b.Cfull, b.Bvec,
                                                b.diag, b.x2p);
  return hipGetLastError();
}

hipError_t launch_dict_chain(const Geom& g, const Buffers& b, const DictPlan& plan,
                             uint32_t key0, uint32_t key1, uint32_t stream, hipStream_t st) {
  (void)plan;
  const int kpl = (g.K + kWave - 1) / kWave;
#define BPFA_CHAIN(KP, PFV)                                                              \
  dict_chain_kernel<KP, PFV><<<g.P, kWave, 0, st>>>(g, b.Cfull, b.Bvec, b.diag, b.x2p,  \
                                                    b.scal, b.D, b.sumr2_p, key0, key1, \
                                                    stream)
  if (kpl <= 1) BPFA_CHAIN(1, 16);
  else if (kpl <= 2) BPFA_CHAIN(2, 16);
  else if (kpl <= 4) BPFA_CHAIN(4, 8);
  else if (kpl <= 8) BPFA_CHAIN(8, 4);
  else if (kpl <= 16) BPFA_CHAIN(16, 2);
  else return hipErrorInvalidValue;
#undef BPFA_CHAIN
  return hipGetLastError();
}

}  // namespace bpfa
