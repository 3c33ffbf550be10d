// Masked patch extraction (N-dimensional inpainting section: an image of
// shape M cut into overlapping patches of shape B with stride S; blind
// inpainting uses only the observed pixels of each patch).
//
// index_kernel   one thread per patch: observed-pixel bitmask and |Obs(i)|.
// slots_kernel   one thread per slot: the observed offsets p (ascending) and
//                values of the slot's patch, stored [j][slot] so that a wave
//                reads them coalesced; padding entries point at offset P,
//                which the sweep keeps at zero.  Per 64-slot wave the largest
//                |Obs| (rounded up to 4) bounds the sweep's inner loops.
// omega_*        ordered compaction of the observed pixels (the dictionary
//                statistics visit patches through them).
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
                                                    uint32_t* __restrict__ perm,
                                                    int32_t* __restrict__ inv_perm, int Npad,
                                                    DevScalars* scal) {
  __shared__ int s_max[4];
  __shared__ long long s_sum[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0;
  if (i < g.N) {
    const int org = patch_origin(g, i);
    for (int w = 0; w < g.PW; ++w) {
      uint32_t word = 0;
      const int pe = min(32, g.P - 32 * w);
      for (int b = 0; b < pe; ++b) {
        if (mask[org + poff[32 * w + b]]) {
          word |= 1u << b;
          ++cnt;
        }
      }
      bits[(size_t)i * g.PW + w] = word;
    }
    count[i] = cnt;
    inv_perm[i] = i;
  }
  if (i < Npad) perm[i] = (i < g.N) ? (uint32_t)i : 0u;
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
                                                    int32_t* __restrict__ wave_J, int Npad,
                                                    int Jcap4) {
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
      while (word) {
        const int b = __builtin_ctz(word);
        word &= word - 1;
        const int p = 32 * w + b;
        obs_idx[(size_t)j * Npad + s] = (uint16_t)p;
        obs_val[(size_t)j * Npad + s] = image[org + poff[p]];
        ++j;
      }
    }
  }
  for (int j = cnt; j < Jcap4; ++j) {
    obs_idx[(size_t)j * Npad + s] = (uint16_t)g.P;
    obs_val[(size_t)j * Npad + s] = 0.f;
  }
  int m = cnt;
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) wave_J[s >> 6] = (m + 3) & ~3;
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
  const int tid = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += blk[b];
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
    const int c = blk[b];
    blk[b] = run;
    run += c;
  }
  if (tid == 1023) scal->n_omega = s_tot[1023];
}

__global__ __launch_bounds__(256) void omega_write_kernel(int Mtot, const uint8_t* __restrict__ mask,
                                                          const int32_t* __restrict__ blk,
                                                          int32_t* __restrict__ omega) {
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
  if (on) omega[base + __popcll(below)] = q;
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

// ---- launchers ----------------------------------------------------------

hipError_t launch_index(const Geom& g, const Buffers& b, int Npad, hipStream_t st) {
  frame_reset_kernel<<<1, 1, 0, st>>>(b.scal);
  const int n = max(g.N, Npad);
  index_kernel<<<(n + 255) / 256, 256, 0, st>>>(g, b.mask, b.poff, b.obs_bits, b.obs_count,
                                                b.perm, b.inv_perm, Npad, b.scal);
  return hipGetLastError();
}

hipError_t launch_omega(const Geom& g, const Buffers& b, hipStream_t st) {
  const int nb = (g.Mtot + 255) / 256;
  omega_count_kernel<<<nb, 256, 0, st>>>(g.Mtot, b.mask, b.image, b.omega_blk, b.scal);
  omega_scan_kernel<<<1, 1024, 0, st>>>(nb, b.omega_blk, b.scal);
  omega_write_kernel<<<nb, 256, 0, st>>>(g.Mtot, b.mask, b.omega_blk, b.omega);
  return hipGetLastError();
}

hipError_t launch_slots(const Geom& g, const Buffers& b, int Npad, int Jcap4, hipStream_t st) {
  slots_kernel<<<Npad / 256, 256, 0, st>>>(g, b.image, b.poff, b.obs_bits, b.obs_count, b.perm,
                                           b.obs_idx, b.obs_val, b.wave_J, Npad, Jcap4);
  return hipGetLastError();
}

hipError_t launch_init_dict(const Geom& g, const Buffers& b, uint32_t key0, uint32_t key1,
                            uint32_t stream, hipStream_t st) {
  const int n = g.K * g.P;
  init_dict_kernel<<<(n + 255) / 256, 256, 0, st>>>(g, b.D, key0, key1, stream);
  return hipGetLastError();
}

}  // namespace bpfa
