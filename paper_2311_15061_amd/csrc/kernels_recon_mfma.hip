// Patch models of the overlap-averaged reconstruction on the matrix cores.
//
// y_i = D^T w_i for every patch is the dense contraction Y = D^T W
// (P x K times K x N), with W the patches' codes densified tile by tile from
// their active lists.  A block takes 128 patches and all P rows: four
// wavefronts each own 32 patches (one 32-column tile of C) and every
// 32-row tile of P; atoms are staged through LDS 64 at a time.
//
// This is the BF16 precision form: each operand is split x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi); C += hi.hi (v_mfma_f32_32x32x16_bf16) plus
// one correction pass hi.lo + lo.hi, accumulated in binary32; the dropped
// lo.lo term is below 2^-16 of |x||w|.  (The binary32 form works from the
// sparse lists on the vector ALUs: recon_sparse_kernel.)
//
// Output Y[p][i] (pixel-major), read by recon_pixel_kernel for the average.
#include "internal.hpp"

namespace bpfa {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRmTile = 128;         // patches per block
constexpr int kRmKc = 64;            // atoms per LDS stage
constexpr int kRmStride = kRmKc + 8; // row stride (16-bit units) of the bf16 tiles
constexpr int kRmCap = 16;           // active entries of a patch held in registers

__device__ __forceinline__ uint16_t bf16_bits(float x) {   // round to nearest even
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// MT: 32-row tiles of P (P <= 32 MT)
template <int MT>
__global__ __launch_bounds__(256) void recon_mfma_kernel(Geom g, const float* __restrict__ D,
                                                         const int2* __restrict__ list,
                                                         const int32_t* __restrict__ nact,
                                                         float* __restrict__ Y) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i0 = blockIdx.x * kRmTile;
  const int P = g.P, K = g.K, N = g.N;
  // this thread densifies patch i0 + tid of the tile (first 128 threads)
  const int my_i = i0 + tid;
  const bool owner = tid < kRmTile && my_i < N;
  int na = 0;
  const int2* L = list;
  if (owner) {
    na = nact[my_i];
    L = list + (size_t)my_i * K;
  }
  // the patch's first kRmCap entries, loaded without conditions so the loads
  // issue back to back (a clamped index stays inside the list row)
  int2 raw[kRmCap];
#pragma unroll
  for (int a = 0; a < kRmCap; ++a) raw[a] = L[min(a, K - 1)];
  int ek[kRmCap];
  float ew[kRmCap];
#pragma unroll
  for (int a = 0; a < kRmCap; ++a) {
    ek[a] = a < na ? raw[a].x : -1;
    ew[a] = __int_as_float(raw[a].y);
  }
  f32x16 acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[m][r] = 0.f;

  for (int kc = 0; kc < K; kc += kRmKc) {
    __syncthreads();
    {
      uint16_t* a_hi = reinterpret_cast<uint16_t*>(smem);
      uint16_t* a_lo = a_hi + MT * 32 * kRmStride;
      uint16_t* b_hi = a_lo + MT * 32 * kRmStride;
      uint16_t* b_lo = b_hi + kRmTile * kRmStride;
      // A = D^T chunk: a[m][kk] = D[kc + kk][m]
      for (int idx = tid; idx < MT * 32 * kRmKc; idx += 256) {
        const int kk = idx / (MT * 32), m = idx - kk * (MT * 32);
        const int k = kc + kk;
        const float v = (m < P && k < K) ? D[(size_t)k * P + m] : 0.f;
        const uint16_t h = bf16_bits(v);
        a_hi[m * kRmStride + kk] = h;
        a_lo[m * kRmStride + kk] = bf16_bits(v - bf16_value(h));
      }
      for (int idx = tid; idx < kRmTile * kRmKc; idx += 256) {
        const int n = idx / kRmKc, kk = idx - n * kRmKc;
        b_hi[n * kRmStride + kk] = 0;
        b_lo[n * kRmStride + kk] = 0;
      }
      __syncthreads();
      if (owner) {
#pragma unroll
        for (int a = 0; a < kRmCap; ++a)
          if (ek[a] >= kc && ek[a] < kc + kRmKc) {
            const uint16_t h = bf16_bits(ew[a]);
            b_hi[tid * kRmStride + (ek[a] - kc)] = h;
            b_lo[tid * kRmStride + (ek[a] - kc)] = bf16_bits(ew[a] - bf16_value(h));
          }
        for (int a = kRmCap; a < na; ++a) {   // entries beyond the register stage
          const int2 e = L[a];
          if (e.x >= kc && e.x < kc + kRmKc) {
            const float w = __int_as_float(e.y);
            const uint16_t h = bf16_bits(w);
            b_hi[tid * kRmStride + (e.x - kc)] = h;
            b_lo[tid * kRmStride + (e.x - kc)] = bf16_bits(w - bf16_value(h));
          }
        }
      }
      __syncthreads();
      const int col = lane & 31, kq = (lane >> 5) * 8;
#pragma unroll
      for (int ks = 0; ks < kRmKc; ks += 16) {
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&b_hi[(wv * 32 + col) * kRmStride + ks + kq]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&b_lo[(wv * 32 + col) * kRmStride + ks + kq]);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&a_hi[(m * 32 + col) * kRmStride + ks + kq]);
          const bf16x8 al = *reinterpret_cast<const bf16x8*>(&a_lo[(m * 32 + col) * kRmStride + ks + kq]);
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[m], 0, 0, 0);
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[m], 0, 0, 0);
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[m], 0, 0, 0);
        }
      }
    }
  }
  // lane holds column (patch) lane % 32 and rows 8 (r / 4) + 4 (lane / 32) + r % 4
  const int n = i0 + wv * 32 + (lane & 31);
  if (n < N) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (row < P) Y[(size_t)row * N + n] = acc[m][r];
      }
  }
}

size_t recon_mfma_lds(int P) {
  const int MT = (P + 31) / 32;
  return (size_t)2 * 2 * (MT * 32 + kRmTile) * kRmStride;
}

template <int MT>
static hipError_t launch_mt(const Geom& g, const Buffers& b, int cur, hipStream_t st) {
  const size_t lds = recon_mfma_lds(g.P);
  const int blocks = (g.N + kRmTile - 1) / kRmTile;
  const hipError_t e = hipFuncSetAttribute((const void*)recon_mfma_kernel<MT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  recon_mfma_kernel<MT><<<blocks, 256, lds, st>>>(g, b.D, b.list[cur], b.nact[cur], b.Y);
  return hipGetLastError();
}

// patch models on the matrix cores; P up to 256
hipError_t launch_recon_patches_mfma(const Geom& g, const Buffers& b, int cur, hipStream_t st) {
  switch ((g.P + 31) / 32) {
    case 1: return launch_mt<1>(g, b, cur, st);
    case 2: return launch_mt<2>(g, b, cur, st);
    case 3: return launch_mt<3>(g, b, cur, st);
    case 4: return launch_mt<4>(g, b, cur, st);
    case 5: return launch_mt<5>(g, b, cur, st);
    case 6: return launch_mt<6>(g, b, cur, st);
    case 7: return launch_mt<7>(g, b, cur, st);
    case 8: return launch_mt<8>(g, b, cur, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bpfa
