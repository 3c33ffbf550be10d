// Overlap-averaged reconstruction and conversions of the sampler state.
//
// recon_sparse_kernel (binary32 form): the patch models y_i = D^T w_i from
//   the active lists, one thread per (patch, run of 32 in-patch offsets), the
//   dictionary's columns of that run staged in LDS; stored pixel-major,
//   Y[p][i], so that neighbouring output pixels read neighbouring patches.
//   (The BF16 form is the matrix-core kernel in kernels_recon_mfma.hip.)
// recon_pixel_kernel: one thread per image pixel q sums Y[p][i] over every
//   patch i and in-patch offset p with o_i + b(p) = q, in ascending p, and
//   divides by the number of such pairs (the coverage of q).
#include "internal.hpp"

namespace bpfa {

constexpr int kRsChunk = 32;       // in-patch offsets per thread
constexpr int kRsStride = 36;      // LDS row stride (floats) of a dictionary atom's run
constexpr int kRsCap = 16;         // active entries of a patch held in registers

// grid (patch blocks, offset runs); LDS K x kRsStride floats
__global__ __launch_bounds__(256) void recon_sparse_kernel(Geom g, const float* __restrict__ D,
                                                           const int2* __restrict__ list,
                                                           const int32_t* __restrict__ nact,
                                                           float* __restrict__ Y) {
  extern __shared__ __attribute__((aligned(16))) float dl[];
  const int tid = threadIdx.x, P = g.P, K = g.K;
  const int p0 = blockIdx.y * kRsChunk;
  const int pc = min(kRsChunk, P - p0);
  for (int idx = tid; idx < K * kRsChunk; idx += 256) {
    const int k = idx / kRsChunk, u = idx - k * kRsChunk;
    dl[k * kRsStride + u] = u < pc ? D[(size_t)k * P + p0 + u] : 0.f;
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + tid;
  if (i >= g.N) return;
  const int na = nact[i];
  const int2* L = list + (size_t)i * K;
  // the first kRsCap entries, loaded without conditions so the loads issue back
  // to back (a clamped index stays inside the list row)
  int2 raw[kRsCap];
#pragma unroll
  for (int a = 0; a < kRsCap; ++a) raw[a] = L[min(a, K - 1)];
  float acc[kRsChunk];
#pragma unroll
  for (int u = 0; u < kRsChunk; ++u) acc[u] = 0.f;
  auto add = [&](int k, float w) {
    const float4* row = reinterpret_cast<const float4*>(dl + k * kRsStride);
#pragma unroll
    for (int q = 0; q < kRsChunk / 4; ++q) {
      const float4 d = row[q];
      acc[4 * q + 0] = fmaf(d.x, w, acc[4 * q + 0]);
      acc[4 * q + 1] = fmaf(d.y, w, acc[4 * q + 1]);
      acc[4 * q + 2] = fmaf(d.z, w, acc[4 * q + 2]);
      acc[4 * q + 3] = fmaf(d.w, w, acc[4 * q + 3]);
    }
  };
#pragma unroll
  for (int a = 0; a < kRsCap; ++a)
    if (a < na) add(raw[a].x, __int_as_float(raw[a].y));
  for (int a = kRsCap; a < na; ++a) {
    const int2 e = L[a];
    add(e.x, __int_as_float(e.y));
  }
#pragma unroll
  for (int u = 0; u < kRsChunk; ++u)
    if (u < pc) Y[(size_t)(p0 + u) * g.N + i] = acc[u];
}

size_t recon_sparse_lds(int K) { return (size_t)K * kRsStride * 4; }

// The pairs (i, p) that cover q form a box: per dimension the in-patch
// offsets b_d <= q_d congruent to q_d mod S_d with q_d - b_d <= (G_d - 1) S_d.
// The box is walked in C order of b, i.e. in ascending p.
__global__ __launch_bounds__(256) void recon_pixel_kernel(Geom g, const float* __restrict__ Y,
                                                          float* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.Mtot) return;
  // per padded dimension (leading dimensions of size 1): first offset, count,
  // and the strides of p and i
  int lo[kMaxDim], cnt[kMaxDim], gs[kMaxDim], pst[kMaxDim], ist[kMaxDim], st[kMaxDim];
  int rem = q, ps = 1, is = 1;
  for (int e = kMaxDim - 1; e >= 0; --e) {
    const int d = e - (kMaxDim - g.ndim);
    if (d < 0) {
      lo[e] = 0; cnt[e] = 1; gs[e] = 0; pst[e] = 0; ist[e] = 0; st[e] = 1;
      continue;
    }
    const int qd = rem % g.M[d];
    rem /= g.M[d];
    const int S = g.S[d];
    int b0 = qd - (g.G[d] - 1) * S;          // congruent to qd mod S
    if (b0 < 0) b0 += ((-b0 + S - 1) / S) * S;
    const int b1 = min(g.B[d] - 1, qd);
    lo[e] = b0;
    cnt[e] = b1 >= b0 ? (b1 - b0) / S + 1 : 0;
    gs[e] = (qd - b0) / S;
    st[e] = S;
    pst[e] = ps;
    ist[e] = is;
    ps *= g.B[d];
    is *= g.G[d];
  }
  const size_t N = (size_t)g.N;
  float acc = 0.f;
  for (int a0 = 0; a0 < cnt[0]; ++a0)
    for (int a1 = 0; a1 < cnt[1]; ++a1)
      for (int a2 = 0; a2 < cnt[2]; ++a2) {
        const int p2 = (lo[0] + a0 * st[0]) * pst[0] + (lo[1] + a1 * st[1]) * pst[1] +
                       (lo[2] + a2 * st[2]) * pst[2];
        const int i2 = (gs[0] - a0) * ist[0] + (gs[1] - a1) * ist[1] + (gs[2] - a2) * ist[2];
        const float* y = Y + (size_t)(p2 + lo[3] * pst[3]) * N + (i2 + gs[3] * ist[3]);
        const size_t dy = (size_t)st[3] * pst[3] * N - (size_t)ist[3];
        for (int a3 = 0; a3 < cnt[3]; ++a3, y += dy) acc += *y;
      }
  out[q] = acc / (float)(cnt[0] * cnt[1] * cnt[2] * cnt[3]);
}

// Posterior moments over Gibbs samples: each sample's reconstruction and its
// square are added to binary64 running sums (the first sample overwrites
// them); the mean is the sum divided by the sample count, rounded to
// binary32.  x^2 of a binary32 x is exact in binary64.
__global__ __launch_bounds__(256) void mean_add_kernel(long long n, const float* __restrict__ x,
                                                       double* __restrict__ sum,
                                                       double* __restrict__ sum2, int first) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double v = (double)x[i];
    sum[i] = first ? v : sum[i] + v;
    sum2[i] = first ? v * v : sum2[i] + v * v;
  }
}

__global__ __launch_bounds__(256) void variance_get_kernel(long long n, const double* __restrict__ sum,
                                                           const double* __restrict__ sum2,
                                                           double count, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double s = sum[i];
    out[i] = (float)fmax(0.0, (sum2[i] - s * s / count) / (count - 1.0));
  }
}

hipError_t launch_variance_get(long long n, const double* sum, const double* sum2, double count,
                               float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  variance_get_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, sum, sum2, count, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void mean_get_kernel(long long n, const double* __restrict__ sum,
                                                       double count, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)(sum[i] / count);
}

hipError_t launch_mean_add(long long n, const float* x, double* sum, double* sum2, bool first,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  mean_add_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, x, sum, sum2, first ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_mean_get(long long n, const double* sum, double count, float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  mean_get_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, sum, count, out);
  return hipGetLastError();
}

hipError_t launch_recon(const Geom& g, const Buffers& b, int cur, int Npad, float* out, bool bf16,
                        hipStream_t st) {
  (void)Npad;
  if (bf16) {
    const hipError_t e = launch_recon_patches_mfma(g, b, cur, st);
    if (e != hipSuccess) return e;
  } else {
    const size_t lds = recon_sparse_lds(g.K);
    const hipError_t e = hipFuncSetAttribute((const void*)recon_sparse_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((g.N + 255) / 256), (unsigned)((g.P + kRsChunk - 1) / kRsChunk));
    recon_sparse_kernel<<<grid, 256, lds, st>>>(g, b.D, b.list[cur], b.nact[cur], b.Y);
  }
  recon_pixel_kernel<<<(g.Mtot + 255) / 256, 256, 0, st>>>(g, b.Y, out);
  return hipGetLastError();
}

// ---- state conversions ----------------------------------------------------

// per-patch active lists -> dense W, Z (patch order)
__global__ __launch_bounds__(256) void lists_to_dense_kernel(Geom g, const int2* __restrict__ list,
                                                             const int32_t* __restrict__ nact,
                                                             float* __restrict__ W,
                                                             uint8_t* __restrict__ Z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const size_t row = (size_t)i * g.K;
  if (W)
    for (int k = 0; k < g.K; ++k) W[row + k] = 0.f;
  if (Z)
    for (int k = 0; k < g.K; ++k) Z[row + k] = 0;
  const int na = nact[i];
  const int2* L = list + row;
  for (int a = 0; a < na; ++a) {
    const int2 e = L[a];
    if (W) W[row + e.x] = __int_as_float(e.y);
    if (Z) Z[row + e.x] = 1;
  }
}

hipError_t launch_lists_to_dense(const Geom& g, const Buffers& b, int cur, float* W, uint8_t* Z,
                                 hipStream_t st) {
  lists_to_dense_kernel<<<(g.N + 255) / 256, 256, 0, st>>>(g, b.list[cur], b.nact[cur], W, Z);
  return hipGetLastError();
}

// W, Z dense in patch order -> per-patch active lists.  A row whose Z and W
// disagree (W != 0 where Z = 0) sets *bad.
__global__ __launch_bounds__(256) void dense_to_lists_kernel(Geom g, const float* __restrict__ W,
                                                             const uint8_t* __restrict__ Z,
                                                             int2* __restrict__ list,
                                                             int32_t* __restrict__ nact,
                                                             int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const size_t row = (size_t)i * g.K;
  int2* L = list + row;
  int na = 0;
  for (int k = 0; k < g.K; ++k) {
    const float w = W[row + k];
    const bool z = Z ? Z[row + k] != 0 : w != 0.f;
    if (z) L[na++] = make_int2(k, __float_as_int(w));
    else if (w != 0.f) atomicOr(bad, 1);
  }
  if (na < g.K) L[na] = make_int2(-1, 0);   // end marker the sweep relies on
  nact[i] = na;
}

hipError_t launch_dense_to_lists(const Geom& g, const Buffers& b, int cur, int Npad,
                                 const float* W, const uint8_t* Z, int* bad, hipStream_t st) {
  (void)Npad;
  dense_to_lists_kernel<<<(g.N + 255) / 256, 256, 0, st>>>(g, W, Z, b.list[cur], b.nact[cur], bad);
  return hipGetLastError();
}

}  // namespace bpfa
