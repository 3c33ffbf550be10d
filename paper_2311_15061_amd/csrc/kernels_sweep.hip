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
// Mapping onto gfx950:
//  * slots (patches) are sorted by |Obs(i)| once per frame and cut into
//    wavefronts by a per-frame table: a patch with |Obs| <= 16 gets one lane,
//    larger ones 2, 4, 8 or 16 lanes (<= 32, 64, 128, 256 observed pixels),
//    each lane holding at most 16 of the patch's observed pixels; every
//    wavefront has one lane count and one register count J, and runs a body
//    compiled for exactly that J: the residual on the observed pixels lives
//    in J VGPRs for the whole atom loop, with no per-element guards.  One
//    kernel covers every |Obs|, so the long patches run beside the bulk in
//    the same launch instead of trailing it;
//  * the lanes of one patch form an aligned group; their partial dot
//    products are summed by a butterfly of DPP lane permutations (VALU
//    operand modifiers, not LDS-crossbar shuffles), so every lane of the
//    group holds the same sums (addition is commutative at every level), draws the same
//    numbers from the patch's Philox counters and takes the same decisions;
//    only the group's first lane writes the patch's outputs;
//  * 8 wavefronts per block share one LDS copy of the dictionary tile; the
//    kernel is held to 128 VGPRs so two blocks (4 waves per SIMD) fit a CU,
//    and a 512 x 512 frame's waves are all resident at once;
//  * the tile is pixel-major with an odd atom stride (d_kp at p * KS + k):
//    a lane's gathers for its observed pixels hit different banks, and the
//    values of atoms k and k+1 at one pixel are adjacent, so one ds_read2
//    serves a pair of atoms;
//  * atoms go in pairs: one pass gives delta and rho of both atoms and the
//    cross term g = sum d_k d_{k+1}; after atom k's draw the pair's second rho
//    is corrected by -(w_new - w_old) g, exactly the effect of the residual
//    update on it; the residual takes both updates in one second pass;
//  * one Philox block per pair: two z uniforms and one Box-Muller pair;
//  * active atoms travel between iterations as per-patch lists
//    (atom, weight) in ascending atom order, stored in patch order (not slot
//    order) so that the dictionary statistics, which visit patches by
//    position, read neighbouring rows.
#include "internal.hpp"
#include "philox.hpp"

namespace bpfa {

typedef __attribute__((address_space(3))) float lds_f;
typedef __attribute__((address_space(1))) uint64_t g_entry;   // one (atom, weight) list entry

constexpr float kLn2 = 0.69314718055994531f;
constexpr float kLog2e = 1.44269504088896341f;
constexpr int kPass1Batch = 8;   // list entries loaded together when rebuilding the residual

__device__ __forceinline__ void load_tile(const SweepArgs& a, float* lds, int k0, int k1) {
  const int kt = k1 - k0;
  const int n = kt * a.P;
  for (int idx = threadIdx.x; idx < n; idx += kSweepBlock) {
    const int kk = idx / a.P, p = idx - kk * a.P;
    lds[p * a.KS + kk] = a.D[(size_t)(k0 + kk) * a.P + p];
  }
  // zero columns kt .. KS-1 of every row and the whole padding row p = P
  const int padc = a.KS - kt;
  for (int idx = threadIdx.x; idx < a.P * padc; idx += kSweepBlock) {
    const int p = idx / padc, kk = kt + (idx - p * padc);
    lds[p * a.KS + kk] = 0.f;
  }
  for (int kk = threadIdx.x; kk < a.KS; kk += kSweepBlock) lds[a.P * a.KS + kk] = 0.f;
}

// value of the partner lane under a data-parallel-primitive permutation (a
// VALU operand modifier: no trip through the LDS crossbar)
template <int CTRL>
__device__ __forceinline__ float dpp_partner(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <-> 15 - i within 16 lanes

// sum over the LPP lanes of an aligned group, the same value in every lane: a
// butterfly in which each stage pairs every lane with one of the other half
// of its group (after the previous stages all lanes of a half hold the same
// sum), and a + b = b + a, so the group's lanes agree bit for bit
template <int LPP>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (LPP >= 2) v += dpp_partner<kDppQuadXor1>(v);
  if constexpr (LPP >= 4) v += dpp_partner<kDppQuadXor2>(v);
  if constexpr (LPP >= 8) v += dpp_partner<kDppHalfMirror>(v);
  if constexpr (LPP >= 16) v += dpp_partner<kDppMirror>(v);
  return v;
}

// One wavefront: slots wt.x .. wt.x + wt.y - 1, LPP lanes per slot, J
// observed pixels per lane (lane `sub` of a group holds rows sub*J .. sub*J+J-1)
template <int J, int LPP>
__device__ __forceinline__ void sweep_wave(const SweepArgs& a, int blk, int nslots, int slot0,
                                           int jpad, uint32_t zs_stream, int tid, uint32_t key0,
                                           uint32_t key1, int npad) {
  extern __shared__ float lds[];
  uint8_t* cnt_lds = reinterpret_cast<uint8_t*>(lds + (a.P + 1) * a.KS);  // [wave][K] z counts
  // per-wave partials in the dynamic LDS, not in static __shared__ arrays:
  // wavefronts of one block run different instantiations of this body
  char* red = reinterpret_cast<char*>(lds) + sweep_red_offset(a.P, a.KS, a.K);
  double* s_w2 = reinterpret_cast<double*>(red);
  double* s_r2 = s_w2 + kSweepWaves;
  long long* s_z = reinterpret_cast<long long*>(s_r2 + kSweepWaves);
  float* s_wm = reinterpret_cast<float*>(s_z + kSweepWaves);

  const int lane = tid & (kWave - 1), wid = tid / kWave;
  const int grp = lane / LPP, sub = lane - grp * LPP;
  const int s = slot0 + grp;
  const bool valid = grp < nslots;
  const bool lead = valid && sub == 0;
  const float gs = (float)a.scal->gamma_s;
  const float ge = (float)a.scal->gamma_eps;
  const uint32_t t = (uint32_t)a.scal->t;
  const uint32_t ip = valid ? a.perm[s] : 0u;
  const int K = a.K;

  lds_f* const L = (lds_f*)lds;
  // column p_j of the tile (p_j = P: the zero row) for each of the lane's
  // rows: a pointer per row, or for the longest bodies two 16-bit float offsets
  // per register (the tile is below 64 K floats), unpacked at each use
  constexpr bool kPacked = J > 20;
  lds_f* colp[kPacked ? 1 : J];
  uint32_t colk[kPacked ? (J + 1) / 2 : 1];
  float r[J];        // residual on this lane's observed pixels
#pragma unroll
  for (int jj = 0; jj < J; ++jj) {
    const int j = sub * J + jj;
    int p = a.P;
    float x = 0.f;
    if (valid && j < jpad) {
      p = a.obs_idx[(size_t)j * npad + s];
      x = a.obs_val[(size_t)j * npad + s];
    }
    if constexpr (kPacked) {
      const uint32_t o = (uint32_t)(p * a.KS);
      if (jj & 1) colk[jj >> 1] |= o << 16;
      else colk[jj >> 1] = o;
    } else {
      colp[jj] = L + p * a.KS;
    }
    r[jj] = x;
  }
  auto col = [&](int jj) -> lds_f* {
    if constexpr (kPacked) return L + ((jj & 1) ? (colk[jj >> 1] >> 16) : (colk[jj >> 1] & 0xFFFFu));
    else return colp[jj];
  };
  uint8_t* const cnt_w = cnt_lds + wid * K;
  const float* __restrict__ Ck = a.Ck;

  const int ntiles = (K + a.KT - 1) / a.KT;
  const int na = valid ? a.nact_in[ip] : 0;
  const int2* __restrict__ lin = a.list_in + (size_t)ip * K;

  // pass 1: residual of the previous sample, r = x - sum_k d_k w_k on Obs(i)
  int ia = 0;
  for (int tile = 0; tile < ntiles; ++tile) {
    const int k0 = tile * a.KT, k1 = min(K, k0 + a.KT);
    __syncthreads();
    load_tile(a, lds, k0, k1);
    __syncthreads();
    // entries in batches whose loads issue together (a clamped index stays in
    // the row); the entries of the tile form a prefix of each batch
    for (;;) {
      int2 eb[kPass1Batch];
#pragma unroll
      for (int u = 0; u < kPass1Batch; ++u) eb[u] = lin[min(ia + u, K - 1)];
      int used = 0;
#pragma unroll
      for (int u = 0; u < kPass1Batch; ++u) {
        if (ia + u < na && eb[u].x < k1) {
          const float w = __int_as_float(eb[u].y);
          const int ko = eb[u].x - k0;
#pragma unroll
          for (int j = 0; j < J; ++j) r[j] = fmaf(-col(j)[ko], w, r[j]);
          used = u + 1;
        }
      }
      ia += used;
      if (!__any(used == kPass1Batch)) break;
    }
  }

  // pass 2: the sweep.  e0, e1 are the next two unconsumed entries of the
  // previous sample's list.  A row with na < K holds the marker atom -1 at
  // position na, so an entry read past it is never taken: the marker is
  // never matched, and what follows it is only promoted once the marker is
  // taken.  Reads reach at most two entries past the row (the buffer has
  // that slack); with na = K they happen after the last atom.
  const int2 mark = make_int2(-1, 0);
  int cur = 0;
  int2 e0 = na > 0 ? lin[0] : mark;
  int2 e1 = na > 1 ? lin[1] : mark;
  // (atom, weight bits) as one 64-bit word: atom in the low half, like int2
  auto entry = [](int k, float w) -> uint64_t {
    return (uint64_t)(uint32_t)k | ((uint64_t)__float_as_uint(w) << 32);
  };
  g_entry* const lout = (g_entry*)(a.list_out + (size_t)ip * K);
  g_entry* lp = lout;
  float sw2 = 0.f;
  uint32_t wmb = 0u;
  const uint64_t leads = __builtin_amdgcn_ballot_w64(lead);

  // one atom: decision and weight given its delta and rho (own term not yet added)
  auto decide = [&](int k, float delta, float rho, float wold, float uz, float n) -> float {
    rho = fmaf(delta, wold, rho);
    const float lam = fmaf(ge, delta, gs);
    const float rs = __builtin_amdgcn_rsqf(lam);
    const float ger = ge * rho;
    const float mean = ger * rs * rs;
    const float q = 0.5f * ger * mean;
    const float lhs = uz * lam * rs;
    const float rhs = (1.f - uz) * __builtin_amdgcn_exp2f((Ck[k] + q) * kLog2e);
    const bool cmp = lhs < rhs;
    const bool z = valid && cmp;
    const float snew = z ? fmaf(n, rs, mean) : 0.f;
    // ballot of the compare itself (leads holds only valid lanes)
    const int nz = (int)__popcll(__builtin_amdgcn_ballot_w64(cmp) & leads);
    if (lane == 0) cnt_w[k] = (uint8_t)nz;   // every (wave, atom) is visited exactly once
    // snew = 0 unless z: the sums take exact zeros (only lead lanes count);
    // |snew| as bits orders like its value
    sw2 = fmaf(snew, snew, sw2);
    wmb = max(wmb, __float_as_uint(snew) & 0x7FFFFFFFu);
    if (z && lead) *lp++ = entry(k, snew);
    return snew - wold;
  };

  for (int tile = 0; tile < ntiles; ++tile) {
    const int k0 = tile * a.KT, k1 = min(K, k0 + a.KT);
    if (ntiles > 1) {
      __syncthreads();
      load_tile(a, lds, k0, k1);
      __syncthreads();
    }
    for (int k = k0; k < k1; k += 2) {
      // the offset is hidden from loop strength reduction: each read address
      // is then one add of this scalar to the column base, not a per-column
      // induction register plus a copy
      int ko = k - k0;
      asm volatile("" : "+s"(ko));
      // packed column offsets are unpacked at each use, not once for the
      // whole loop (that would hold J registers again)
      if constexpr (kPacked) {
#pragma unroll
        for (int i = 0; i < (J + 1) / 2; ++i) asm volatile("" : "+v"(colk[i]));
      }
      // old weights of the pair; the next two entries are fetched now and
      // first needed by the next pair
      const bool c0 = e0.x == k;
      const float wo0 = c0 ? __int_as_float(e0.y) : 0.f;
      const int2 f = c0 ? e1 : e0;
      const bool c1 = f.x == k + 1;
      const float wo1 = c1 ? __int_as_float(f.y) : 0.f;
      const int adv = (int)c0 + (int)c1;
      if (adv != 0) {
        cur += adv;
        e0 = lin[cur];
        e1 = lin[cur + 1];
      }
      const Block4 rb = philox10(ip, (uint32_t)(k >> 1), t, zs_stream, key0, key1);
      float dl0 = 0.f, dl1 = 0.f, rh0 = 0.f, rh1 = 0.f, g01 = 0.f;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const float x0 = col(j)[ko], x1 = col(j)[ko + 1];
        dl0 = fmaf(x0, x0, dl0);
        dl1 = fmaf(x1, x1, dl1);
        rh0 = fmaf(x0, r[j], rh0);
        rh1 = fmaf(x1, r[j], rh1);
        g01 = fmaf(x0, x1, g01);
      }
      dl0 = group_sum<LPP>(dl0);
      dl1 = group_sum<LPP>(dl1);
      rh0 = group_sum<LPP>(rh0);
      rh1 = group_sum<LPP>(rh1);
      g01 = group_sum<LPP>(g01);
      const float u2 = u01f(rb.w2);
      const float rad = __builtin_amdgcn_sqrtf(-2.f * kLn2 * __builtin_amdgcn_logf(u2));
      const float ang = u01f(rb.w3);                 // revolutions
      const float n0 = rad * __builtin_amdgcn_cosf(ang);
      const float n1 = rad * __builtin_amdgcn_sinf(ang);
      const float dw0 = decide(k, dl0, rh0, wo0, u01f(rb.w0), n0);
      float dw1 = 0.f;
      if (k + 1 < k1) dw1 = decide(k + 1, dl1, fmaf(-dw0, g01, rh1), wo1, u01f(rb.w1), n1);
      // re-read the pair's columns rather than keep 2 J values live across the draws
      asm volatile("" ::: "memory");
      if (dw0 != 0.f || dw1 != 0.f) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const float x0 = col(j)[ko], x1 = col(j)[ko + 1];
          r[j] = fmaf(-x1, dw1, fmaf(-x0, dw0, r[j]));
        }
      }
    }
  }

  const int nout = (int)(lp - lout);
  if (lead) {
    a.nact_out[ip] = nout;
    if (nout < K) *lp = entry(-1, 0.f);
  }
  float r2 = 0.f;
#pragma unroll
  for (int j = 0; j < J; ++j) r2 = fmaf(r[j], r[j], r2);

  // deterministic block partials: fixed butterfly, then waves in order (sw2
  // and the z count from the lead lanes only, r2 from every lane; the lanes
  // of a group hold the same max)
  double dw2 = lead ? (double)sw2 : 0.0, dr2 = (double)r2;
  long long dz = lead ? nout : 0;
  float dm = __uint_as_float(wmb);
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
    SweepPart pt{0.0, 0.0, 0, 0.f, 0};
    for (int w = 0; w < kSweepWaves; ++w) {
      pt.sum_w2 += s_w2[w];
      pt.sum_r2 += s_r2[w];
      pt.sum_z += s_z[w];
      pt.wmax = fmaxf(pt.wmax, s_wm[w]);
    }
    a.part[blk] = pt;
  }
  for (int k = tid; k < K; k += kSweepBlock) {
    int c = 0;
    for (int w = 0; w < kSweepWaves; ++w) c += cnt_lds[w * K + k];
    if (c) atomicAdd(&a.cnt[k], c);
  }
}

// One 8-wave group of the launch's wavefront range: wavefront w of group grp
// reads its (first slot, slots, lanes per slot, J) from the table and runs the
// body compiled for that pair; the group's partials go to entry grp.
// Wavefronts past the range run with no valid lane (every body passes the
// same barriers).  tid, keys and npad are passed in so that the strided
// kernel can hide them from loop-invariant hoisting.
__device__ __forceinline__ void sweep_group(const SweepArgs& a, const int4* __restrict__ waves, int w0,
                                            int nwaves, int grp, int jpad, uint32_t zs, int tid,
                                            uint32_t key0, uint32_t key1, int npad) {
  const int w = grp * kSweepWaves + tid / kWave;
  int4 wt = make_int4(0, 0, 1, 4);
  if (w < nwaves) wt = waves[w0 + w];
  const int slot0 = __builtin_amdgcn_readfirstlane(wt.x);
  const int ns = __builtin_amdgcn_readfirstlane(wt.y);
  const int lpp = __builtin_amdgcn_readfirstlane(wt.z);
  const int J = __builtin_amdgcn_readfirstlane(wt.w);
#define BPFA_BODY(JJ, LL) sweep_wave<JJ, LL>(a, grp, ns, slot0, jpad, zs, tid, key0, key1, npad)
  switch (lpp) {
    case 1:
      switch (J) {
        case 4: BPFA_BODY(4, 1); break;
        case 6: BPFA_BODY(6, 1); break;
        case 8: BPFA_BODY(8, 1); break;
        case 10: BPFA_BODY(10, 1); break;
        case 12: BPFA_BODY(12, 1); break;
        case 14: BPFA_BODY(14, 1); break;
        default: BPFA_BODY(16, 1); break;
      }
      break;
    case 2:
      if (J <= 12) BPFA_BODY(12, 2);
      else if (J <= 16) BPFA_BODY(16, 2);
      else if (J <= 20) BPFA_BODY(20, 2);
      else BPFA_BODY(24, 2);
      break;
    case 4:
      if (J <= 12) BPFA_BODY(12, 4);
      else BPFA_BODY(16, 4);
      break;
    case 8:
      if (J <= 12) BPFA_BODY(12, 8);
      else BPFA_BODY(16, 8);
      break;
    default:
      if (J <= 12) BPFA_BODY(12, 16);
      else BPFA_BODY(16, 16);
      break;
  }
#undef BPFA_BODY
}

// The sweep over the table's wavefronts [range[0], range[1]) (a pair in
// device memory).  STRIDED = false: one block per 8-wave group (the grid is
// the group count, known on the host).  STRIDED = true: a grid fixed per
// handle strides over the groups, so a launch needs no host knowledge of the
// frame (captured launch sequences); the values the bodies derive lane and
// key constants from are made opaque per group, which keeps the loop from
// hoisting them into spilled registers.
template <bool STRIDED>
__global__ __launch_bounds__(kSweepBlock, kSweepWavesPerSimd) void sweep_kernel(const SweepArgs a, const int4* __restrict__ waves,
                                                            const int* __restrict__ range) {
  const int w0 = __builtin_amdgcn_readfirstlane(range[0]);
  const int nwaves = __builtin_amdgcn_readfirstlane(range[1]) - w0;
  // observed rows per slot and the stream word, from the frame plan and the
  // device scalars (kept out of `a`, which stays in kernel-argument memory)
  const int jpad = __builtin_amdgcn_readfirstlane(a.plan->jpad);
  const uint32_t zs = (a.stream & 0xFFu) |
                      ((uint32_t)__builtin_amdgcn_readfirstlane(a.scal->problem_id) << 8);
  const int ngroups = (nwaves + kSweepWaves - 1) / kSweepWaves;
  if constexpr (STRIDED) {
    for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
      int tid = threadIdx.x, npad = a.Npad;
      uint32_t key0 = a.key0, key1 = a.key1;
      asm volatile("" : "+v"(tid), "+s"(npad), "+s"(key0), "+s"(key1));
      sweep_group(a, waves, w0, nwaves, grp, jpad, zs, tid, key0, key1, npad);
    }
  } else {
    if ((int)blockIdx.x < ngroups)
      sweep_group(a, waves, w0, nwaves, blockIdx.x, jpad, zs, threadIdx.x, a.key0, a.key1, a.Npad);
  }
}

hipError_t launch_sweep(const int4* waves, const int* range, int blocks, bool strided, size_t lds,
                        const SweepArgs& a, hipStream_t st) {
  if (blocks <= 0) return hipSuccess;
  const void* fn = strided ? (const void*)sweep_kernel<true> : (const void*)sweep_kernel<false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (strided) sweep_kernel<true><<<blocks, kSweepBlock, lds, st>>>(a, waves, range);
  else sweep_kernel<false><<<blocks, kSweepBlock, lds, st>>>(a, waves, range);
  return hipGetLastError();
}

// ---- reduction of the sweep's block partials (fixed order) ---------------

// largest power of two s with bound * s <= 2^50 and n * bound * s < 2^62
__device__ double fixed_scale(double bound, double n) {
  if (!(bound > 0.0) || !isfinite(bound)) return 1.0;
  int e1, e2;
  frexp(bound, &e1);        // bound < 2^e1
  frexp(bound * n, &e2);    // n * bound < 2^e2
  return ldexp(1.0, min(50 - e1, 62 - e2));
}

__global__ __launch_bounds__(256) void sweep_reduce_kernel(const int* __restrict__ range,
                                                           const SweepPart* __restrict__ part,
                                                           DevScalars* scal) {
  const int blocks = (range[1] - range[0] + kSweepWaves - 1) / kSweepWaves;   // 8-wave groups
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
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_w2[threadIdx.x] += s_w2[threadIdx.x + o];
      s_r2[threadIdx.x] += s_r2[threadIdx.x + o];
      s_z[threadIdx.x] += s_z[threadIdx.x + o];
      s_m[threadIdx.x] = fmaxf(s_m[threadIdx.x], s_m[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scal->sum_w2 = s_w2[0];
    scal->sum_r2_sweep = s_r2[0];
    scal->sum_z = s_z[0];
    scal->wmax = s_m[0];
    // fixed-point scales of the dictionary statistics: each rounded term
    // stays below 2^50 in magnitude (exact rounding by the 1.5 * 2^52 add)
    // and every sum of at most n_omega terms below 2^62
    const double nv = (double)max(scal->n_omega, 1);
    const double wm = (double)s_m[0], ym = (double)scal->ymax;
    scal->scale_c = fixed_scale(wm * wm, nv);
    scal->scale_b = fixed_scale(wm * ym, nv);
  }
}

hipError_t launch_sweep_reduce(const Geom& g, const Buffers& b, const int* range, hipStream_t st) {
  (void)g;
  sweep_reduce_kernel<<<1, 256, 0, st>>>(range, b.sw_part, b.scal);
  return hipGetLastError();
}

}  // namespace bpfa
