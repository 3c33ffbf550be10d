// Overlap-averaged reconstruction and conversions of the sampler state.
//
// recon_patch_kernel: the patch models y_i = D^T w_i, one thread per (patch,
//   run of 16 in-patch offsets) reading the patch's active list once; stored
//   pixel-major, Y[p][i], so that neighbouring output pixels read
//   neighbouring patches.
// recon_pixel_kernel: one thread per image pixel q sums Y[p][i] over every
//   patch i and in-patch offset p with o_i + b(p) = q, in ascending p, and
//   divides by the number of such pairs (the coverage of q).
#include "internal.hpp"

namespace bpfa {

constexpr int kReconChunk = 16;   // in-patch offsets per thread

// thread (chunk c, slot s): y_i[p] for p in [16 c, 16 c + 16), one pass over the entries
__global__ __launch_bounds__(256) void recon_patch_kernel(Geom g, const float* __restrict__ D,
                                                          const int32_t* __restrict__ inv_perm,
                                                          const int2* __restrict__ list,
                                                          const int32_t* __restrict__ nact,
                                                          float* __restrict__ Y) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t % g.N);
  const int c = (int)(t / g.N);
  const int p0 = c * kReconChunk;
  if (p0 >= g.P) return;
  const int s = inv_perm[i];
  const int na = nact[s];
  const int2* L = list + (size_t)s * g.K;
  float acc[kReconChunk];
#pragma unroll
  for (int u = 0; u < kReconChunk; ++u) acc[u] = 0.f;
  const bool full = p0 + kReconChunk <= g.P;
  for (int a = 0; a < na; ++a) {
    const int2 e = L[a];
    const float w = __int_as_float(e.y);
    const float* row = D + (size_t)e.x * g.P + p0;
#pragma unroll
    for (int u = 0; u < kReconChunk; ++u)
      if (full || p0 + u < g.P) acc[u] = fmaf(row[u], w, acc[u]);
  }
#pragma unroll
  for (int u = 0; u < kReconChunk; ++u)
    if (full || p0 + u < g.P) Y[(size_t)(p0 + u) * g.N + i] = acc[u];
}

__global__ __launch_bounds__(256) void recon_pixel_kernel(Geom g, const int32_t* __restrict__ pcoord,
                                                          const float* __restrict__ Y,
                                                          float* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.Mtot) return;
  int qc[kMaxDim];
  int rem = q;
  for (int d = g.ndim - 1; d >= 0; --d) {
    qc[d] = rem % g.M[d];
    rem /= g.M[d];
  }
  float acc = 0.f;
  int cnt = 0;
  for (int p = 0; p < g.P; ++p) {
    int pidx = 0;
    bool ok = true;
    for (int d = 0; d < g.ndim; ++d) {
      const int od = qc[d] - pcoord[p * kMaxDim + d];
      const int gd = od / g.S[d];
      ok = ok && od >= 0 && gd * g.S[d] == od && gd < g.G[d];
      pidx = pidx * g.G[d] + gd;
    }
    if (ok) {
      acc += Y[(size_t)p * g.N + pidx];
      ++cnt;
    }
  }
  out[q] = acc / (float)cnt;
}

hipError_t launch_recon(const Geom& g, const Buffers& b, int cur, int Npad, float* out,
                        hipStream_t st) {
  (void)Npad;
  const long long n = (long long)g.N * ((g.P + kReconChunk - 1) / kReconChunk);
  recon_patch_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(g, b.D, b.inv_perm, b.list[cur],
                                                                  b.nact[cur], b.Y);
  recon_pixel_kernel<<<(g.Mtot + 255) / 256, 256, 0, st>>>(g, b.pcoord, b.Y, out);
  return hipGetLastError();
}

// ---- state conversions ----------------------------------------------------

__global__ __launch_bounds__(256) void lists_to_dense_kernel(Geom g, const uint32_t* __restrict__ perm,
                                                             const int2* __restrict__ list,
                                                             const int32_t* __restrict__ nact,
                                                             float* __restrict__ W,
                                                             uint8_t* __restrict__ Z) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const size_t row = (size_t)perm[s] * g.K;
  if (W)
    for (int k = 0; k < g.K; ++k) W[row + k] = 0.f;
  if (Z)
    for (int k = 0; k < g.K; ++k) Z[row + k] = 0;
  const int na = nact[s];
  const int2* L = list + (size_t)s * g.K;
  for (int a = 0; a < na; ++a) {
    const int2 e = L[a];
    if (W) W[row + e.x] = __int_as_float(e.y);
    if (Z) Z[row + e.x] = 1;
  }
}

hipError_t launch_lists_to_dense(const Geom& g, const Buffers& b, int cur, float* W, uint8_t* Z,
                                 hipStream_t st) {
  lists_to_dense_kernel<<<(g.N + 255) / 256, 256, 0, st>>>(g, b.perm, b.list[cur], b.nact[cur], W,
                                                           Z);
  return hipGetLastError();
}

// W, Z dense in patch order -> per-slot active lists.  A row whose Z and W
// disagree (W != 0 where Z = 0) sets *bad.
__global__ __launch_bounds__(256) void dense_to_lists_kernel(Geom g, const int32_t* __restrict__ inv_perm,
                                                             const float* __restrict__ W,
                                                             const uint8_t* __restrict__ Z,
                                                             int2* __restrict__ list,
                                                             int32_t* __restrict__ nact,
                                                             int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const int s = inv_perm[i];
  const size_t row = (size_t)i * g.K;
  int2* L = list + (size_t)s * g.K;
  int na = 0;
  for (int k = 0; k < g.K; ++k) {
    const float w = W[row + k];
    const bool z = Z ? Z[row + k] != 0 : w != 0.f;
    if (z) L[na++] = make_int2(k, __float_as_int(w));
    else if (w != 0.f) atomicOr(bad, 1);
  }
  nact[s] = na;
}

hipError_t launch_dense_to_lists(const Geom& g, const Buffers& b, int cur, int Npad,
                                 const float* W, const uint8_t* Z, int* bad, hipStream_t st) {
  (void)Npad;
  dense_to_lists_kernel<<<(g.N + 255) / 256, 256, 0, st>>>(g, b.inv_perm, W, Z, b.list[cur],
                                                           b.nact[cur], bad);
  return hipGetLastError();
}

// codes kept across a new frame: slot rows move from the previous slot order to the new one
__global__ __launch_bounds__(256) void remap_lists_kernel(Geom g, const int32_t* __restrict__ prev_inv,
                                                          const int32_t* __restrict__ inv_perm,
                                                          const int2* __restrict__ list_in,
                                                          const int32_t* __restrict__ nact_in,
                                                          int2* __restrict__ list_out,
                                                          int32_t* __restrict__ nact_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const int so = prev_inv[i], sn = inv_perm[i];
  const int na = nact_in[so];
  const int2* src = list_in + (size_t)so * g.K;
  int2* dst = list_out + (size_t)sn * g.K;
  for (int a = 0; a < na; ++a) dst[a] = src[a];
  nact_out[sn] = na;
}

hipError_t launch_remap_lists(const Geom& g, const Buffers& b, int cur, hipStream_t st) {
  remap_lists_kernel<<<(g.N + 255) / 256, 256, 0, st>>>(g, b.inv_prev, b.inv_perm, b.list[cur],
                                                        b.nact[cur], b.list[1 - cur],
                                                        b.nact[1 - cur]);
  return hipGetLastError();
}

}  // namespace bpfa
