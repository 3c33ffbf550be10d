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
//   chunk of observed pixels).  A lane takes observed pixel q and the patch
//   whose origin is q - b(p); its active entries are staged in registers and
//   its outer product is added into LDS.  Sums are 64-bit fixed point: the
//   binary64 product of two binary32 weights is exact, it is scaled by a power
//   of two and rounded to an integer by adding 1.5 * 2^52 (exact for
//   |x| < 2^51); integer adds are associative, so the statistics do not
//   depend on scheduling.
// dict_reduce_kernel: sums the chunk partials, one block per (p, row k),
//   into the symmetric binary64 C_p, B_p and the diagonal.
// dict_chain_kernel: one wavefront per p runs the chain with rows of C_p
//   prefetched ahead of use, draws d_kp with the Philox DICT stream, and forms
//   the residual sum of squares.
#include "internal.hpp"
#include "philox.hpp"

namespace bpfa {

constexpr int kStatsCap = 16;   // active entries of a patch held in registers

struct DictPlanDev {
  int RG, chunks, K, pad_;
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

__global__ __launch_bounds__(kDictBlock) void dict_stats_kernel(
    Geom g, DictPlanDev pl, const int4* __restrict__ omega_c, const int32_t* __restrict__ omega,
    const float* __restrict__ image, const int32_t* __restrict__ pcoord,
    const int32_t* __restrict__ inv_perm, const int2* __restrict__ list,
    const int32_t* __restrict__ nact, const DevScalars* __restrict__ scal,
    long long* __restrict__ dpart, double* __restrict__ dx2) {
  extern __shared__ long long acc[];
  __shared__ double s_x2[kDictBlock / kWave];
  const int per_p = pl.RG * pl.chunks;
  const int p = blockIdx.x / per_p;
  const int rg = (blockIdx.x % per_p) / pl.chunks;
  const int c = blockIdx.x % pl.chunks;
  const int r0 = pl.row0[rg], r1 = pl.row0[rg + 1];
  const long long e0 = pl.ent0[rg];
  const int E = (int)(pl.ent0[rg + 1] - e0);
  const int rec = E + (r1 - r0);
  const int K = g.K;
  for (int e = threadIdx.x; e < rec; e += kDictBlock) acc[e] = 0;
  __syncthreads();

  const double sc = scal->scale_c, sb = scal->scale_b;
  const int nom = scal->n_omega;
  const int per = (nom + pl.chunks - 1) / pl.chunks;
  const int v0 = min(nom, c * per), v1 = min(nom, v0 + per);
  int bc[kMaxDim] = {0, 0, 0, 0};
  for (int d = 0; d < g.ndim; ++d) bc[d] = pcoord[p * kMaxDim + d];

  double x2 = 0.0;
  for (int v = v0 + (int)threadIdx.x; v < v1; v += kDictBlock) {
    const int4 qc = omega_c[v];
    const int qv[kMaxDim] = {qc.x, qc.y, qc.z, qc.w};
    // origin = q - b(p): every coordinate non-negative, on the stride grid, inside the grid
    int pidx = 0;
    bool ok = true;
    for (int d = 0; d < g.ndim; ++d) {
      const int od = qv[d] - bc[d];
      const int gd = g.S[d] == 1 ? od : od / g.S[d];
      ok = ok && od >= 0 && gd * g.S[d] == od && gd < g.G[d];
      pidx = pidx * g.G[d] + gd;
    }
    if (!ok) continue;
    const int slot = inv_perm[pidx];
    const int na = nact[slot];
    const double y = (double)image[omega[v]];
    if (rg == 0) x2 += y * y;
    const int2* L = list + (size_t)slot * K;
    int kk[kStatsCap];
    double ww[kStatsCap];
#pragma unroll
    for (int a = 0; a < kStatsCap; ++a) {
      kk[a] = -1;
      ww[a] = 0.0;
      if (a < na) {
        const int2 e = L[a];
        kk[a] = e.x;
        ww[a] = (double)__int_as_float(e.y);
      }
    }
    const double ysb = y * sb;
#pragma unroll
    for (int a = 0; a < kStatsCap; ++a) {
      if (kk[a] >= r0 && kk[a] < r1) {
        atomicAdd((unsigned long long*)&acc[E + (kk[a] - r0)], to_fixed(ww[a] * ysb));
        const double wa = ww[a] * sc;
        const int base = (int)(tri_off(kk[a], K) - e0) - kk[a];
#pragma unroll
        for (int b = a; b < kStatsCap; ++b)
          if (kk[b] >= 0) atomicAdd((unsigned long long*)&acc[base + kk[b]], to_fixed(wa * ww[b]));
      }
    }
    // entries beyond the register stage: every pair (a, b), a <= b, with b >= kStatsCap
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
  __syncthreads();
  long long* out = dpart + (size_t)blockIdx.x * pl.rec_stride;
  for (int e = threadIdx.x; e < rec; e += kDictBlock) out[e] = acc[e];
  if (rg == 0) {
    for (int o = kWave / 2; o > 0; o >>= 1) x2 += __shfl_xor(x2, o);
    if ((threadIdx.x & (kWave - 1)) == 0) s_x2[threadIdx.x / kWave] = x2;
    __syncthreads();
    if (threadIdx.x == 0) {
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

template <int KPL, int PF>
__global__ __launch_bounds__(kWave) void dict_chain_kernel(
    Geom g, const double* __restrict__ Cfull, const double* __restrict__ Bvec,
    const double* __restrict__ diag, const double* __restrict__ x2p, DevScalars* scal,
    float* __restrict__ D, double* __restrict__ sumr2_p, uint32_t key0, uint32_t key1,
    uint32_t stream) {
  __shared__ double s_B[64 * KPL], s_n[64 * KPL], s_diag[64 * KPL], s_d[64 * KPL];
  const int p = blockIdx.x, lane = threadIdx.x, K = g.K, P = g.P;
  const double* C = Cfull + (size_t)p * K * K;
  const uint32_t t = (uint32_t)scal->t;
  double dreg[KPL];
#pragma unroll
  for (int m = 0; m < KPL; ++m) {
    const int j = lane + kWave * m;
    dreg[m] = 0.0;
    if (j < K) {
      const Block4 rb = philox10((uint32_t)p, (uint32_t)j, t, stream, key0, key1);
      s_n[j] = sqrt(-2.0 * log(u01d(rb.w0))) * cos(2.0 * M_PI * u01d(rb.w1));
      s_B[j] = Bvec[(size_t)p * K + j];
      s_diag[j] = diag[(size_t)p * K + j];
      dreg[m] = (double)D[(size_t)j * P + p];
    }
  }
  __syncthreads();

  // the chain over atoms, rows of C_p prefetched PF ahead
  const double ge = scal->gamma_eps;
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
        double part = 0.0;
#pragma unroll
        for (int m = 0; m < KPL; ++m) {
          const int j = lane + kWave * m;
          if (j != k) part = fma(ring[u][m], dreg[m], part);
        }
        const double tot = wave_sum_d(part);
        const double lam = (double)P + ge * s_diag[k];
        const double dn = ge * (s_B[k] - tot) / lam + s_n[k] / sqrt(lam);
        bad = bad || !isfinite(dn);
#pragma unroll
        for (int m = 0; m < KPL; ++m)
          if (k == lane + kWave * m) dreg[m] = dn;
        const int kn = k + PF;
#pragma unroll
        for (int m = 0; m < KPL; ++m) {
          const int j = lane + kWave * m;
          ring[u][m] = (kn < K && j < K) ? C[(size_t)kn * K + j] : 0.0;
        }
      }
    }
  }

  // new atoms' column p; residual sum of squares at position p
#pragma unroll
  for (int m = 0; m < KPL; ++m) {
    const int j = lane + kWave * m;
    if (j < K) {
      s_d[j] = dreg[m];
      D[(size_t)j * P + p] = (float)dreg[m];
    }
  }
  __syncthreads();
  double cd[KPL];
#pragma unroll
  for (int m = 0; m < KPL; ++m) cd[m] = 0.0;
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
      const double dk = k < K ? s_d[k] : 0.0;
#pragma unroll
      for (int m = 0; m < KPL; ++m) cd[m] = fma(v[u][m], dk, cd[m]);
    }
  }
  double quad = 0.0, lin = 0.0;
#pragma unroll
  for (int m = 0; m < KPL; ++m) {
    const int j = lane + kWave * m;
    if (j < K) {
      quad = fma(cd[m], dreg[m], quad);
      lin = fma(s_B[j], dreg[m], lin);
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
                             int Npad, hipStream_t st) {
  (void)Npad;
  const DictPlanDev d = to_dev(g, plan);
  const int blocks = g.P * plan.RG * plan.chunks;
  const size_t lds = (size_t)d.rec_stride * sizeof(long long);
  hipError_t e = hipFuncSetAttribute((const void*)dict_stats_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  dict_stats_kernel<<<blocks, kDictBlock, lds, st>>>(g, d, b.omega_c, b.omega, b.image, b.pcoord,
                                                     b.inv_perm, b.list[cur], b.nact[cur], b.scal,
                                                     b.dpart, b.dx2);
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
