// Counter-based random numbers for the Gibbs sweep on gfx950.
//
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, section 3.2): ten rounds,
// each taking the two 32x32->64-bit products of counter words 0 and 2 with
// two fixed odd multipliers, swapping and xoring the halves with the other two
// words and the round key; the key advances by a Weyl increment per round.
//
// Stream contract (shared in specification with the CPU oracle, not in code):
//   key     = (seed low 32 bits, seed high 32 bits)
//   counter = (c0, c1, iteration t, tag | problem_id << 8)
//   uniform = (floor(w / 2^9) + 1/2) * 2^-23, exact in binary32 and binary64
//   normal  = Box-Muller (cos / sin branches of one radius / angle pair).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpfa {

enum : uint32_t {
  kTagZS = 1, kTagDict = 2, kTagPiA = 3, kTagPiB = 4, kTagGS = 5, kTagGE = 6, kTagInit = 7,
  kTagAcq = 8   // acquisition masks of a served stream
};

struct Block4 { uint32_t w0, w1, w2, w3; };

__device__ __forceinline__ Block4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Block4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t stream_word(uint32_t tag, uint32_t problem_id) {
  return (tag & 0xFFu) | (problem_id << 8);
}

__device__ __forceinline__ float u01f(uint32_t w) {
  return ((float)(w >> 9) + 0.5f) * 1.1920928955078125e-07f;  // 2^-23
}

__device__ __forceinline__ double u01d(uint32_t w) {
  return ((double)(w >> 9) + 0.5) * 1.1920928955078125e-07;
}

}  // namespace bpfa
