// Conjugate scalar draws of an iteration (BPFA section; the model's
// beta-process and gamma priors):
//   logit pi_k = ln G_A - ln G_B,  G_A ~ Ga(a/K + n_k), G_B ~ Ga(b(K-1)/K + N - n_k)
//   gamma_s   ~ Ga(c + sum(z)/2, rate d + sum(w^2)/2)
//   gamma_eps ~ Ga(e + sum|Obs|/2, rate f + sum(r^2)/2)
// A mini-batch step (the epoch schedule's reading of the Time-to-solution
// section) draws them given its batch of n_b patches with every count and
// sum multiplied by s = N / n_b: n_k -> s n_k, N -> s n_b, and so on.
// Gamma variates follow Marsaglia & Tsang (ACM TOMS 2000) in binary64: for
// shape alpha >= 1, d = alpha - 1/3, c = 1/sqrt(9 d), x ~ N(0,1),
// v = (1 + c x)^3, accept when ln u < x^2/2 + d - d v + d ln v; for alpha < 1
// the same paper's boost Ga(alpha + 1) U^(1/alpha), kept in log space.
// Attempt j of draw c0 reads Philox block (c0, j, t, tag): words 0, 1 give x
// (Box-Muller cosine branch), word 2 the acceptance uniform, word 3 of
// attempt 0 the boost uniform; at most 64 attempts.
#include "internal.hpp"
#include "philox.hpp"

namespace bpfa {

// returns false when no attempt accepted
__device__ bool log_gamma_draw(double shape, uint32_t key0, uint32_t key1, uint32_t stream,
                               uint32_t c0, uint32_t t, double* out) {
  if (!(shape > 0.0) || !isfinite(shape)) return false;
  const double alpha = shape < 1.0 ? shape + 1.0 : shape;
  const double d = alpha - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
  double log_boost = 0.0;
  for (uint32_t j = 0; j < 64; ++j) {
    const Block4 w = philox10(c0, j, t, stream, key0, key1);
    if (j == 0 && shape < 1.0) log_boost = log(u01d(w.w3)) / shape;
    const double x = sqrt(-2.0 * log(u01d(w.w0))) * cos(2.0 * M_PI * u01d(w.w1));
    const double cx = c * x;
    if (cx <= -1.0) continue;
    const double log_v = 3.0 * log1p(cx);
    const double v = exp(log_v);
    if (log(u01d(w.w2)) < 0.5 * x * x + d - d * v + d * log_v) {
      *out = log(d) + log_v + log_boost;
      return true;
    }
  }
  return false;
}

__global__ __launch_bounds__(256) void scalars_kernel(Geom g, double a, double b, double c,
                                                      double dd, double e, double f,
                                                      int learn_dict, StepBatch sb, uint32_t key0,
                                                      uint32_t key1,
                                                      int32_t* __restrict__ nk,
                                                      const double* __restrict__ sumr2_p,
                                                      double* __restrict__ ell,
                                                      float* __restrict__ Ck, DevScalars* scal) {
  __shared__ double s_gs, s_ge, s_sr2;
  __shared__ long long s_z;
  __shared__ int s_bad;
  __shared__ double s_min[256], s_max[256], s_sum[256];
  __shared__ long long s_zp[256];
  const int K = g.K, tid = threadIdx.x;
  const uint32_t pid = scal->problem_id;
  const uint32_t t = (uint32_t)scal->t;
  // sum(z) and the residual sum of squares: strided partials, fixed-order tree
  long long zp = 0;
  double rp = 0.0;
  for (int k = tid; k < K; k += 256) zp += nk[k];
  if (learn_dict)
    for (int p = tid; p < g.P; p += 256) rp += sumr2_p[p];
  s_zp[tid] = zp;
  s_sum[tid] = rp;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      s_zp[tid] += s_zp[tid + o];
      s_sum[tid] += s_sum[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    s_z = s_zp[0];
    double sr2 = scal->sum_r2_sweep;
    if (learn_dict) {
      sr2 = s_sum[0];
      scal->sum_r2_dict = sr2;
    }
    s_sr2 = sr2;
    s_bad = 0;
  }
  __syncthreads();
  int bad = 0;
  for (int i = tid; i < K + 2; i += 256) {
    double lg = 0.0;
    if (i < K) {
      const double nki = (double)nk[i];
      double la = 0.0, lb = 0.0;
      const double s = sb.scale;
      const bool oka = log_gamma_draw(a / K + s * nki, key0, key1, stream_word(kTagPiA, pid),
                                      (uint32_t)i, t, &la);
      const bool okb = log_gamma_draw(b * (K - 1) / K + s * (double)sb.n_b - s * nki, key0, key1,
                                      stream_word(kTagPiB, pid), (uint32_t)i, t, &lb);
      if (!oka || !okb || !isfinite(la - lb)) bad |= 2;
      ell[i] = la - lb;
    } else if (i == K) {
      const double shape = c + 0.5 * (sb.scale * (double)s_z);
      const double rate = dd + 0.5 * (sb.scale * scal->sum_w2);
      if (!log_gamma_draw(shape, key0, key1, stream_word(kTagGS, pid), 0u, t, &lg)) bad |= 2;
      s_gs = exp(lg) / rate;
    } else {
      const double nobs = sb.n_obs_b >= 0 ? (double)sb.n_obs_b : (double)scal->n_obs;
      const double shape = e + 0.5 * (sb.scale * nobs);
      const double rate = f + 0.5 * (sb.scale * s_sr2);
      if (!log_gamma_draw(shape, key0, key1, stream_word(kTagGE, pid), 0u, t, &lg)) bad |= 2;
      s_ge = exp(lg) / rate;
    }
  }
  if (bad) atomicOr(&s_bad, bad);
  __syncthreads();
  const double gs = s_gs, ge = s_ge;
  const double half_log_gs = 0.5 * log(gs);
  double mn = 1.0, mx = 0.0, sm = 0.0;
  for (int k = tid; k < K; k += 256) {
    Ck[k] = (float)(ell[k] + half_log_gs);
    const double pk = 1.0 / (1.0 + exp(-ell[k]));
    mn = fmin(mn, pk);
    mx = fmax(mx, pk);
    sm += pk;
    nk[k] = 0;                      // counts restart for the next sweep
  }
  s_min[tid] = mn;
  s_max[tid] = mx;
  s_sum[tid] = sm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      s_min[tid] = fmin(s_min[tid], s_min[tid + o]);
      s_max[tid] = fmax(s_max[tid], s_max[tid + o]);
      s_sum[tid] += s_sum[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    mn = s_min[0];
    mx = s_max[0];
    sm = s_sum[0];
    int st = s_bad;
    if (!isfinite(gs) || !(gs > 0.0) || !isfinite(ge) || !(ge > 0.0) || !isfinite(s_sr2)) st |= 1;
    scal->status |= st;
    scal->gamma_s = gs;
    scal->gamma_eps = ge;
    scal->sum_r2_used = s_sr2;
    scal->sum_z = s_z;
    scal->pi_min = mn;
    scal->pi_max = mx;
    scal->pi_mean = sm / K;
    scal->t = scal->t + 1;
  }
}

hipError_t launch_scalars(const Geom& g, const Buffers& b, const double* h, int learn_dict,
                          const StepBatch& sb, uint32_t key0, uint32_t key1, hipStream_t st) {
  scalars_kernel<<<1, 256, 0, st>>>(g, h[0], h[1], h[2], h[3], h[4], h[5], learn_dict, sb, key0,
                                    key1, b.sw_cnt, b.sumr2_p, b.ell, b.Ck, b.scal);
  return hipGetLastError();
}

__global__ void ck_kernel(int K, const double* __restrict__ ell, const DevScalars* scal,
                          float* __restrict__ Ck) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) Ck[k] = (float)(ell[k] + 0.5 * log(scal->gamma_s));
}

hipError_t launch_ck(const Geom& g, const Buffers& b, hipStream_t st) {
  ck_kernel<<<(g.K + 255) / 256, 256, 0, st>>>(g.K, b.ell, b.scal, b.Ck);
  return hipGetLastError();
}

__global__ void reset_scalars_kernel(int K, double ell0, double gs0, double ge0,
                                     double* __restrict__ ell, int32_t* __restrict__ nk,
                                     DevScalars* scal) {
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    ell[k] = ell0;
    nk[k] = 0;
  }
  if (threadIdx.x == 0) {
    scal->gamma_s = gs0;
    scal->gamma_eps = ge0;
    scal->t = 1;
  }
}

hipError_t launch_reset_scalars(const Geom& g, const Buffers& b, double ell0, double gamma_s0,
                                double gamma_eps0, hipStream_t st) {
  reset_scalars_kernel<<<1, 256, 0, st>>>(g.K, ell0, gamma_s0, gamma_eps0, b.ell, b.sw_cnt,
                                          b.scal);
  return hipGetLastError();
}

__global__ void set_t_kernel(DevScalars* scal, long long t, uint32_t problem_id, int clear_status) {
  if (t > 0) scal->t = t;
  scal->problem_id = problem_id;
  if (clear_status) scal->status = 0;
}

hipError_t launch_set_t(DevScalars* scal, long long t, uint32_t problem_id, hipStream_t st,
                        bool clear_status) {
  set_t_kernel<<<1, 1, 0, st>>>(scal, t, problem_id, clear_status ? 1 : 0);
  return hipGetLastError();
}

__global__ void debug_philox_kernel(uint32_t key0, uint32_t key1, uint32_t c1, uint32_t t,
                                    uint32_t stream, const uint32_t* __restrict__ c0,
                                    long long n, uint32_t* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Block4 r = philox10(c0[i], c1, t, stream, key0, key1);
  out[4 * i + 0] = r.w0;
  out[4 * i + 1] = r.w1;
  out[4 * i + 2] = r.w2;
  out[4 * i + 3] = r.w3;
}

hipError_t launch_debug_philox(uint32_t key0, uint32_t key1, uint32_t c1, uint32_t t,
                               uint32_t stream, const uint32_t* c0, long long n, uint32_t* out,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  debug_philox_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(key0, key1, c1, t, stream, c0,
                                                                   n, out);
  return hipGetLastError();
}

}  // namespace bpfa
