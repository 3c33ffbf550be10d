// z/s Gibbs sweep (BPFA section: the sparse-coding step of an iteration).
//
// For every patch i independently and atoms k = 0 .. K-1 in order:
//   delta = sum_{Obs} d_kp^2,  rho = sum_{Obs} d_kp (r_p + d_kp w_ik)
//   lam   = gamma_s + gamma_eps delta
//   z_ik  = [logit u < ell_k + ln(gamma_s / lam) / 2 + (gamma_eps rho)^2 / (2 lam)]
//   s_ik  = gamma_eps rho / lam + n / sqrt(lam)   if z_ik, else w_ik = 0
//   r    -= d_k (w_new - w_old)
// with the log-odds of z taken with s integrated out.  The comparison is
// evaluated in the equivalent form u sqrt(lam) < (1 - u) exp(C_k + q) with
// C_k = ell_k + ln(gamma_s) / 2 and q = (gamma_eps rho)^2 / (2 lam).
//
// Mapping onto gfx950: one lane per patch, 64 patches per wavefront, 8
// wavefronts per block.  A lane keeps its patch's residual on the observed
// pixels in VGPRs for the whole atom loop; the dictionary tile sits in LDS
// pixel-major with an odd atom stride (column p of atom k at p * KS + k), so
// the per-lane gathers d_{k, p_j} hit different banks.  Padding slots of the
// observed list point at a zero row.  Inner loops run to the wavefront's
// largest |Obs| (uniform), in steps of four.  One Philox block serves two
// atoms: two z uniforms and one Box-Muller pair.  Active atoms are carried
// between iterations as per-patch lists (atom, weight) in ascending atom
// order, so the sweep streams only what is non-zero.
#include "internal.hpp"
#include "philox.hpp"

namespace bpfa {

__device__ __forceinline__ void load_tile(const SweepArgs& a, float* lds, int k0, int k1) {
  const int kt = k1 - k0;
  const int n = kt * a.P;
  for (int idx = threadIdx.x; idx < n; idx += kSweepBlock) {
    const int kk = idx / a.P, p = idx - kk * a.P;
    lds[p * a.KS + kk] = a.D[(size_t)(k0 + kk) * a.P + p];
  }
  for (int kk = threadIdx.x; kk < a.KS; kk += kSweepBlock) lds[a.P * a.KS + kk] = 0.f;
}

template <int JMAX>
struct LaneState {
  int addr[JMAX];   // LDS float index of column p_j (p_j * KS)
  float r[JMAX];    // residual on observed pixel j
};

template <int JMAX>
__device__ __forceinline__ void dot_delta_rho(const LaneState<JMAX>& ls, const float* __restrict__ col,
                                              int Jw, float& delta, float& rho) {
  float d0 = 0.f, d1 = 0.f, r0 = 0.f, r1 = 0.f;
#pragma unroll
  for (int j0 = 0; j0 < JMAX; j0 += 4) {
    if (j0 < Jw) {
      const float a0 = col[ls.addr[j0 + 0]], a1 = col[ls.addr[j0 + 1]];
      const float a2 = col[ls.addr[j0 + 2]], a3 = col[ls.addr[j0 + 3]];
      d0 = fmaf(a0, a0, d0);
      r0 = fmaf(a0, ls.r[j0 + 0], r0);
      d1 = fmaf(a1, a1, d1);
      r1 = fmaf(a1, ls.r[j0 + 1], r1);
      d0 = fmaf(a2, a2, d0);
      r0 = fmaf(a2, ls.r[j0 + 2], r0);
      d1 = fmaf(a3, a3, d1);
      r1 = fmaf(a3, ls.r[j0 + 3], r1);
    }
  }
  delta = d0 + d1;
  rho = r0 + r1;
}

template <int JMAX>
__device__ __forceinline__ void residual_axpy(LaneState<JMAX>& ls, const float* __restrict__ col,
                                              int Jw, float c) {
#pragma unroll
  for (int j0 = 0; j0 < JMAX; j0 += 4) {
    if (j0 < Jw) {
#pragma unroll
      for (int u = 0; u < 4; ++u) ls.r[j0 + u] = fmaf(-col[ls.addr[j0 + u]], c, ls.r[j0 + u]);
    }
  }
}

template <int JMAX>
__global__ __launch_bounds__(kSweepBlock) void sweep_kernel(SweepArgs a) {
  extern __shared__ float lds[];
  int* cnt_lds = reinterpret_cast<int*>(lds + (a.P + 1) * a.KS);
  __shared__ double s_w2[kSweepBlock / kWave], s_r2[kSweepBlock / kWave];
  __shared__ long long s_z[kSweepBlock / kWave];
  __shared__ float s_wm[kSweepBlock / kWave];

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int s = blockIdx.x * kSweepBlock + tid;
  const bool valid = s < a.N;
  const float gs = (float)a.scal->gamma_s;
  const float ge = (float)a.scal->gamma_eps;
  const uint32_t t = (uint32_t)a.scal->t;
  const int Jw = __builtin_amdgcn_readfirstlane(a.wave_J[s / kWave]);
  const uint32_t ip = a.perm[s];

  LaneState<JMAX> ls;
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    if (j < Jw) {
      ls.addr[j] = (int)a.obs_idx[(size_t)j * a.Npad + s] * a.KS;
      ls.r[j] = a.obs_val[(size_t)j * a.Npad + s];
    } else {
      ls.addr[j] = a.P * a.KS;
      ls.r[j] = 0.f;
    }
  }
  for (int k = tid; k < a.K; k += kSweepBlock) cnt_lds[k] = 0;

  const int ntiles = (a.K + a.KT - 1) / a.KT;
  const int na = valid ? a.nact_in[s] : 0;
  const int2* __restrict__ lin = a.list_in + (size_t)s * a.K;

  // pass 1: residual of the previous sample, r = x - sum_k d_k w_k on Obs(i)
  int ia = 0;
  for (int tile = 0; tile < ntiles; ++tile) {
    const int k0 = tile * a.KT, k1 = min(a.K, k0 + a.KT);
    __syncthreads();
    load_tile(a, lds, k0, k1);
    __syncthreads();
    for (;;) {
      bool more = ia < na;
      int2 e = make_int2(0, 0);
      if (more) e = lin[ia];
      more = more && e.x < k1;
      if (!__any(more)) break;
      if (more) {
        residual_axpy<JMAX>(ls, lds + (e.x - k0), Jw, __int_as_float(e.y));
        ++ia;
      }
    }
  }

  // pass 2: the sweep
  const int2 sent = make_int2(a.K, 0);
  int cur = 0;
  int2 e0 = na > 0 ? lin[0] : sent;
  int2 e1 = na > 1 ? lin[1] : sent;
  int nout = 0;
  int2* __restrict__ lout = a.list_out + (size_t)s * a.K;
  float sw2 = 0.f, wmx = 0.f;

  auto atom = [&](int k, int k0, float uz, float n) {
    const float* col = lds + (k - k0);
    float delta, rho;
    dot_delta_rho<JMAX>(ls, col, Jw, delta, rho);
    const bool hit = e0.x == k;
    const float wold = hit ? __int_as_float(e0.y) : 0.f;
    if (hit) {
      e0 = e1;
      ++cur;
      e1 = (cur + 1 < na) ? lin[cur + 1] : sent;
    }
    rho = fmaf(delta, wold, rho);
    const float lam = fmaf(ge, delta, gs);
    const float rs = __frsqrt_rn(lam);
    const float ger = ge * rho;
    const float mean = ger * rs * rs;
    const float q = 0.5f * ger * mean;
    const float lhs = uz * lam * rs;
    const float rhs = (1.f - uz) * __expf(a.Ck[k] + q);
    const bool z = valid && (lhs < rhs);
    const float snew = z ? fmaf(n, rs, mean) : 0.f;
    const float dw = snew - wold;
    if (dw != 0.f) residual_axpy<JMAX>(ls, col, Jw, dw);
    if (z) {
      lout[nout++] = make_int2(k, __float_as_int(snew));
      sw2 = fmaf(snew, snew, sw2);
      wmx = fmaxf(wmx, fabsf(snew));
    }
    const unsigned long long bal = __ballot(z);
    if (lane == 0 && bal) atomicAdd(&cnt_lds[k], (int)__popcll(bal));
  };

  for (int tile = 0; tile < ntiles; ++tile) {
    const int k0 = tile * a.KT, k1 = min(a.K, k0 + a.KT);
    if (ntiles > 1) {
      __syncthreads();
      load_tile(a, lds, k0, k1);
      __syncthreads();
    }
    for (int k = k0; k < k1; k += 2) {
      const Block4 rb = philox10(ip, (uint32_t)(k >> 1), t, a.stream, a.key0, a.key1);
      const float rad = sqrtf(-2.f * __logf(u01f(rb.w2)));
      const float ang = u01f(rb.w3);                 // revolutions
      const float n0 = rad * __builtin_amdgcn_cosf(ang);
      const float n1 = rad * __builtin_amdgcn_sinf(ang);
      atom(k, k0, u01f(rb.w0), n0);
      if (k + 1 < k1) atom(k + 1, k0, u01f(rb.w1), n1);
    }
  }

  if (valid) a.nact_out[s] = nout;
  float r2 = 0.f;
#pragma unroll
  for (int j = 0; j < JMAX; ++j) r2 = fmaf(ls.r[j], ls.r[j], r2);

  // deterministic block partials: fixed butterfly, then waves in order
  double dw2 = (double)sw2, dr2 = (double)r2;
  long long dz = nout;
  float dm = wmx;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    dw2 += __shfl_xor(dw2, o);
    dr2 += __shfl_xor(dr2, o);
    dz += __shfl_xor(dz, o);
    dm = fmaxf(dm, __shfl_xor(dm, o));
  }
  if (lane == 0) {
    s_w2[wid] = dw2;
    s_r2[wid] = dr2;
    s_z[wid] = dz;
    s_wm[wid] = dm;
  }
  __syncthreads();
  if (tid == 0) {
    SweepPart p{0.0, 0.0, 0, 0.f, 0};
    for (int w = 0; w < kSweepBlock / kWave; ++w) {
      p.sum_w2 += s_w2[w];
      p.sum_r2 += s_r2[w];
      p.sum_z += s_z[w];
      p.wmax = fmaxf(p.wmax, s_wm[w]);
    }
    a.part[blockIdx.x] = p;
  }
  for (int k = tid; k < a.K; k += kSweepBlock) {
    const int c = cnt_lds[k];
    if (c) atomicAdd(&a.cnt[k], c);
  }
}

hipError_t launch_sweep(int JMAX, int blocks, size_t lds, const SweepArgs& a, hipStream_t st) {
  switch (JMAX) {
#define BPFA_SWEEP_CASE(J) \
  case J: {                                                                            \
    hipError_t e_ = hipFuncSetAttribute((const void*)sweep_kernel<J>,                   \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    if (e_ != hipSuccess) return e_;                                                    \
    sweep_kernel<J><<<blocks, kSweepBlock, lds, st>>>(a);                               \
    break;                                                                              \
  }
    BPFA_SWEEP_CASE(8)
    BPFA_SWEEP_CASE(16)
    BPFA_SWEEP_CASE(24)
    BPFA_SWEEP_CASE(32)
    BPFA_SWEEP_CASE(48)
    BPFA_SWEEP_CASE(64)
    BPFA_SWEEP_CASE(96)
    BPFA_SWEEP_CASE(128)
    BPFA_SWEEP_CASE(256)
#undef BPFA_SWEEP_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- reduction of the sweep's block partials (fixed order) ---------------

__global__ __launch_bounds__(256) void sweep_reduce_kernel(int blocks, const SweepPart* __restrict__ part,
                                                           DevScalars* scal) {
  __shared__ double s_w2[256], s_r2[256];
  __shared__ long long s_z[256];
  __shared__ float s_m[256];
  double w2 = 0.0, r2 = 0.0;
  long long z = 0;
  float m = 0.f;
  for (int b = threadIdx.x; b < blocks; b += 256) {
    const SweepPart p = part[b];
    w2 += p.sum_w2;
    r2 += p.sum_r2;
    z += p.sum_z;
    m = fmaxf(m, p.wmax);
  }
  s_w2[threadIdx.x] = w2;
  s_r2[threadIdx.x] = r2;
  s_z[threadIdx.x] = z;
  s_m[threadIdx.x] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 256; ++i) {
      w2 += s_w2[i];
      r2 += s_r2[i];
      z += s_z[i];
      m = fmaxf(m, s_m[i]);
    }
    scal->sum_w2 = w2;
    scal->sum_r2_sweep = r2;
    scal->sum_z = z;
    scal->wmax = m;
    // fixed-point scales of the dictionary statistics: every accumulated sum
    // stays below 2^61 in magnitude
    const double nv = (double)max(scal->n_omega, 1);
    const double wm = (double)m, ym = (double)scal->ymax;
    int ex;
    const double bc = nv * wm * wm;
    frexp(bc, &ex);
    scal->scale_c = bc > 0.0 ? ldexp(1.0, 61 - ex) : 1.0;
    const double bb = nv * wm * ym;
    frexp(bb, &ex);
    scal->scale_b = bb > 0.0 ? ldexp(1.0, 61 - ex) : 1.0;
  }
}

hipError_t launch_sweep_reduce(const Geom& g, const Buffers& b, int blocks, hipStream_t st) {
  (void)g;
  sweep_reduce_kernel<<<1, 256, 0, st>>>(blocks, b.sw_part, b.scal);
  return hipGetLastError();
}

}  // namespace bpfa
