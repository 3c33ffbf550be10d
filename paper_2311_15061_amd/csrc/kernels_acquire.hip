// Acquisition masks of a served stream (Feature summary: pre-determined
// indexing methods, and on-the-fly strategic selections that improve the
// reconstruction).  The paper gives no rule; these are the library's:
//
//   uniform   every pixel q independently with probability rho;
//   line hop  each line along the last axis visited from a random start by
//             random hops of 1 .. hmax pixels, hmax = max(1, floor(2/rho + 1/2) - 1)
//             (mean hop about 1 / rho);
//   targeted  p_q = min(1, (1 - lam) rho + lam rho M v_q / sum v), v the
//             stream's last per-pixel posterior variance (p_q = rho when
//             sum v = 0): a share lam of the expected rho M acquisitions
//             follows the model's uncertainty.
//
// Random numbers: Philox4x32-10 under the server's seed, counter (pixel or
// line, hop, frame index, kTagAcq | stream << 8), word 0 as the 23-bit
// uniform u; a pixel is acquired when u < p (binary64).
#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "philox.hpp"

namespace bpfa {

__device__ __forceinline__ double acq_uniform(uint32_t c0, uint32_t c1, const AcqArgs& a) {
  return u01d(philox10(c0, c1, a.frame, a.stream_word, a.key0, a.key1).w0);
}

__global__ __launch_bounds__(256) void acquire_uniform_kernel(AcqArgs a, uint8_t* __restrict__ mask) {
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < a.M;
       q += (long long)gridDim.x * blockDim.x)
    mask[q] = acq_uniform((uint32_t)q, 0u, a) < a.rho ? 1 : 0;
}

// one thread per line along the last axis
__global__ __launch_bounds__(256) void acquire_line_hop_kernel(AcqArgs a, long long lines, int L,
                                                               int hmax, uint8_t* __restrict__ mask) {
  const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (r >= lines) return;
  uint8_t* row = mask + r * L;
  for (int c = 0; c < L; ++c) row[c] = 0;
  long long pos = (long long)floor(acq_uniform((uint32_t)r, 0u, a) * hmax);
  for (uint32_t j = 1; pos < L; ++j) {
    row[pos] = 1;
    pos += (long long)floor(acq_uniform((uint32_t)r, j, a) * hmax) + 1;
  }
}

// sum of the weights in binary64, fixed order (strided partials, then a tree)
__global__ __launch_bounds__(1024) void weight_sum_kernel(long long M, const float* __restrict__ w,
                                                          double* __restrict__ out) {
  __shared__ double s[1024];
  double acc = 0.0;
  for (long long q = threadIdx.x; q < M; q += 1024) acc += (double)w[q];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

__global__ __launch_bounds__(256) void acquire_targeted_kernel(AcqArgs a, const float* __restrict__ w,
                                                               const double* __restrict__ wsum,
                                                               uint8_t* __restrict__ mask) {
  const double total = *wsum;
  // (1 - lam) rho + lam rho M v / total, each operation rounded once (no
  // contraction into fused multiply-adds)
  const double base = __dmul_rn(1.0 - a.share, a.rho);
  const double scale = __dmul_rn(__dmul_rn(a.share, a.rho), (double)a.M);
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < a.M;
       q += (long long)gridDim.x * blockDim.x) {
    double p = a.rho;
    if (total > 0.0) p = fmin(1.0, __dadd_rn(base, __ddiv_rn(__dmul_rn(scale, (double)w[q]), total)));
    mask[q] = acq_uniform((uint32_t)q, 0u, a) < p ? 1 : 0;
  }
}

hipError_t launch_acquire(const AcqArgs& a, int kind, int ndim, const int64_t* shape,
                          const float* weights, double* wsum, uint8_t* mask, hipStream_t st) {
  if (a.M <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<long long>(4096, (a.M + 255) / 256);
  if (kind == kAcqLineHop) {
    const int L = (int)shape[ndim - 1];
    const long long lines = a.M / L;
    const int hmax = std::max(1, (int)std::floor(2.0 / a.rho + 0.5) - 1);
    acquire_line_hop_kernel<<<(unsigned)((lines + 255) / 256), 256, 0, st>>>(a, lines, L, hmax, mask);
  } else if (kind == kAcqTargeted && weights) {
    weight_sum_kernel<<<1, 1024, 0, st>>>(a.M, weights, wsum);
    acquire_targeted_kernel<<<blocks, 256, 0, st>>>(a, weights, wsum, mask);
  } else {
    // uniform, or targeted with no weights yet (p = rho everywhere)
    acquire_uniform_kernel<<<blocks, 256, 0, st>>>(a, mask);
  }
  return hipGetLastError();
}

}  // namespace bpfa
