// Overlap-averaged reconstruction and conversions of the sampler state.
//
// recon_patch_kernel: one lane per slot computes the patch model
//   y_i = D^T w_i (P values) from its active list and stores it pixel-major,
//   Y[p][i], so that neighbouring output pixels read neighbouring patches.
// recon_pixel_kernel: one thread per image pixel q sums Y[p][i] over every
//   patch i and in-patch offset p with o_i + b(p) = q, in ascending p, and
//   divides by the number of such pairs (the coverage of q).
#include "internal.hpp"

namespace bpfa {

__global__ __launch_bounds__(256) void recon_patch_kernel(Geom g, const float* __restrict__ D,
                                                          const uint32_t* __restrict__ perm,
                                                          const int2* __restrict__ list,
                                                          const int32_t* __restrict__ nact,
                                                          float* __restrict__ Y) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int i = (int)perm[s];
  const int na = nact[s];
  const int2* L = list + (size_t)s * g.K;
  for (int p = 0; p < g.P; ++p) {
    float acc = 0.f;
    for (int a = 0; a < na; ++a) {
      const int2 e = L[a];
      acc = fmaf(D[(size_t)e.x * g.P + p], __int_as_float(e.y), acc);
    }
    Y[(size_t)p * g.N + i] = acc;
  }
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
  recon_patch_kernel<<<(g.N + 255) / 256, 256, 0, st>>>(g, b.D, b.perm, b.list[cur], b.nact[cur],
                                                        b.Y);
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

}  // namespace bpfa
