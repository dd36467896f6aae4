// Device primitives of the IS shape-overlap engine (gfx950, wave64).
//
// Everything here runs in FP32 on the vector ALU except Philox (32-bit
// integer multiplies) and the per-molecule preparation (FP64).  Notation
// follows the paper: o_i = exp(-alpha_i |r - c_i|^2), m = sum o_i,
// u = 1 - prod (1 - o_i), w = u / m, Z = sum (pi/alpha_i)^(3/2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shape_normal_poly.hpp"

namespace shape {

constexpr int kWave = 64;

// Prepared atom record used by every hot loop: centre and the exponent scale
// for exp2, a2 = alpha * log2(e), so that o = exp2(-a2 |r - c|^2).
struct __align__(16) Atom {
  float x, y, z, a2;
};

// Sampling record of an atom: standard deviation 1/sqrt(2 alpha) of its
// mixture component and the component-selection threshold (word 0 of the
// Philox block selects component j = #{i < N-1 : word0 >= thr_i}).
struct __align__(8) AtomSampling {
  float sd;
  uint32_t thr;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds; each round multiplies
// words 0 and 2 by the two round constants and mixes high halves with the
// other words and the key; the key advances by the Weyl constants.  The
// products are written as 32x32->64-bit multiplies so that each is one
// v_mad_u64_u32 rather than a v_mul_hi_u32/v_mul_lo_u32 pair.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k.x, (uint32_t)p1,
                   (uint32_t)(p0 >> 32) ^ c.w ^ k.y, (uint32_t)p0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// Standard normal from the top 24 bits b of a Philox word: u = (b + 1/2) 2^-24,
// z = Phi^-1(u) = sqrt(2) erfinv(x), x = 2u - 1 = b 2^-23 + (2^-24 - 1), which
// one FP32 fma forms exactly, so the tails are resolved to the last bit.
// erfinv after Giles (2011): z = x P(L), L = -log2(1 - x^2), with one
// polynomial in L for L < kSplit and one in sqrt(L) above it (coefficients
// from gen_normal_poly.py; relative error below 3e-7 over every 24-bit u).
// The tail branch runs only when some lane of the wave needs it.
__device__ __forceinline__ float normal_from_bits(uint32_t word) {
  using namespace normal_poly;
  const float x = fmaf((float)(word >> 8), 0x1p-23f, 0x1p-24f - 1.0f);
  const float ax = fabsf(x);
  const float y = (1.0f - ax) * (1.0f + ax);  // 1 - x^2 >= 2^-24 (1 + 2^-24)
  const float L = -__builtin_amdgcn_logf(y);
  float p;
  if (L < kSplit) {
    const float t = fmaf(L, kCenScale, kCenOff);
    p = kCen[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) p = fmaf(p, t, kCen[i]);
  } else {
    const float t = fmaf(__builtin_amdgcn_sqrtf(L), kTailScale, kTailOff);
    p = kTail[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) p = fmaf(p, t, kTail[i]);
  }
  return x * p;
}

// Component of a molecule's mixture selected by a Philox word:
// j = #{i < n-1 : word >= thr_i}.  The thresholds are non-decreasing, so the
// count is found by binary lifting in ceil(log2(n)) steps (the step count is
// the same for every lane); every index read is below n-1.
__device__ __forceinline__ int select_component(const AtomSampling* samp, int n, uint32_t word) {
  const int last = n - 1;
  int j = 0;
  if (last > 0) {
    for (int step = 1 << (31 - __builtin_clz((unsigned)last)); step > 0; step >>= 1) {
      const int c = j + step;
      const int idx = (c < last ? c : last) - 1;
      if (c <= last && word >= samp[idx].thr) j = c;
    }
  }
  return j;
}

// Guide table of a molecule's component choice, built once per molecule in
// LDS: guide[g] = #{i < n-1 : thr_i <= g 2^24} for the top eight bits g of
// a word.  Every threshold counted there lies at or below any word whose top
// bits are g, so that word's count starts at guide[g] and steps only over
// the thresholds inside its 2^24-wide bucket (on average (n-1)/256 of them):
// the same count as select_component's, from one table read and a short
// scan instead of ceil(log2(n)) dependent reads.
constexpr int kGuideBits = 8;
constexpr int kGuideSize = 1 << kGuideBits;

__device__ __forceinline__ void build_guide(const AtomSampling* samp, int n, int* guide,
                                            int tid, int nthreads) {
  const int last = n - 1;
  for (int g = tid; g < kGuideSize; g += nthreads) {
    const uint32_t x = (uint32_t)g << (32 - kGuideBits);
    int c = 0;  // largest c <= last with thr_{c-1} <= x (thresholds non-decreasing)
    if (last > 0) {
      for (int step = 1 << (31 - __builtin_clz((unsigned)last)); step > 0; step >>= 1) {
        const int t = c + step;
        if (t <= last && samp[t - 1].thr <= x) c = t;
      }
    }
    guide[g] = c;
  }
}

__device__ __forceinline__ int select_component_guided(const AtomSampling* samp,
                                                       const int* guide, int n,
                                                       uint32_t word) {
  const int last = n - 1;
  int j = guide[word >> (32 - kGuideBits)];
  while (j < last && word >= samp[j].thr) ++j;
  return j;
}

// Sample point k of a molecule (exact draw from its normalised mixture):
// component by integer thresholds, then r = c_j + z * sd_j per axis.
// atoms/samp point at the molecule's own records (LDS or global); guide, if
// given, is the molecule's guide table (the component is the same).
__device__ __forceinline__ void sample_point(const Atom* atoms, const AtomSampling* samp,
                                             int n, uint32_t mol_id, uint64_t k, uint2 key,
                                             float& rx, float& ry, float& rz,
                                             const int* guide = nullptr) {
  const uint4 x = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)(k >> 32), mol_id, 0u), key);
  const int j = guide ? select_component_guided(samp, guide, n, x.x)
                      : select_component(samp, n, x.x);
  const Atom c = atoms[j];
  const float sd = samp[j].sd;
  rx = fmaf(normal_from_bits(x.y), sd, c.x);
  ry = fmaf(normal_from_bits(x.z), sd, c.y);
  rz = fmaf(normal_from_bits(x.w), sd, c.z);
}

// Antithetic sample k (each draw paired with its reflection about its
// component's centre): samples 2p and 2p+1 use Philox block p; the odd one
// takes the normals with the opposite sign.
__device__ __forceinline__ void sample_point_anti(const Atom* atoms, const AtomSampling* samp,
                                                  int n, uint32_t mol_id, uint64_t k, uint2 key,
                                                  float& rx, float& ry, float& rz,
                                                  const int* guide = nullptr) {
  const uint64_t p = k >> 1;
  const float sg = (k & 1) ? -1.0f : 1.0f;
  const uint4 x = philox4x32_10(make_uint4((uint32_t)p, (uint32_t)(p >> 32), mol_id, 0u), key);
  const int j = guide ? select_component_guided(samp, guide, n, x.x)
                      : select_component(samp, n, x.x);
  const Atom c = atoms[j];
  const float sd = samp[j].sd;
  rx = fmaf(sg * normal_from_bits(x.y), sd, c.x);
  ry = fmaf(sg * normal_from_bits(x.z), sd, c.y);
  rz = fmaf(sg * normal_from_bits(x.w), sd, c.z);
}

// Both members of antithetic pair p from one Philox block.
__device__ __forceinline__ void sample_pair(const Atom* atoms, const AtomSampling* samp, int n,
                                            uint32_t mol_id, uint64_t p, uint2 key, float& ax,
                                            float& ay, float& az, float& bx, float& by,
                                            float& bz, const int* guide = nullptr) {
  const uint4 x = philox4x32_10(make_uint4((uint32_t)p, (uint32_t)(p >> 32), mol_id, 0u), key);
  const int j = guide ? select_component_guided(samp, guide, n, x.x)
                      : select_component(samp, n, x.x);
  const Atom c = atoms[j];
  const float sd = samp[j].sd;
  const float zx = normal_from_bits(x.y), zy = normal_from_bits(x.z), zz = normal_from_bits(x.w);
  ax = fmaf(zx, sd, c.x);
  ay = fmaf(zy, sd, c.y);
  az = fmaf(zz, sd, c.z);
  bx = fmaf(-zx, sd, c.x);
  by = fmaf(-zy, sd, c.y);
  bz = fmaf(-zz, sd, c.z);
}

__device__ __forceinline__ float occupancy(const Atom& a, float rx, float ry, float rz) {
  const float dx = rx - a.x, dy = ry - a.y, dz = rz - a.z;
  const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  return __builtin_amdgcn_exp2f(-a.a2 * d2);
}

// Union complement q = prod (1 - o_i) of a molecule at S points (the caller
// initialises q to 1); u = 1 - q.  One fused multiply-add per atom and point.
template <int S>
__device__ __forceinline__ void eval_union(const Atom* __restrict__ atoms, int n,
                                           const float (&rx)[S], const float (&ry)[S],
                                           const float (&rz)[S], float (&q)[S]) {
#pragma unroll 2
  for (int i = 0; i < n; ++i) {
    const Atom a = atoms[i];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float o = occupancy(a, rx[s], ry[s], rz[s]);
      q[s] = fmaf(-q[s], o, q[s]);
    }
  }
}

// First-order density m = sum o_i and union complement q at S points.
template <int S>
__device__ __forceinline__ void eval_density(const Atom* __restrict__ atoms, int n,
                                             const float (&rx)[S], const float (&ry)[S],
                                             const float (&rz)[S], float (&m)[S],
                                             float (&q)[S]) {
#pragma unroll 2
  for (int i = 0; i < n; ++i) {
    const Atom a = atoms[i];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float o = occupancy(a, rx[s], ry[s], rz[s]);
      m[s] += o;
      q[s] = fmaf(-q[s], o, q[s]);
    }
  }
}

// ---------------------------------------------------------------------------
// Expanded-quadratic atom records.  In a frame centred at `ref`, with
// c' = c - ref and r' = r - ref, the exponent of o = exp2(-e) is
//   e = a2 |r' - c'|^2 = a2 |r'|^2 + (-2 a2 c') . r' + a2 |c'|^2,
// four fused multiply-adds per atom once |r'|^2 is known for the point.
// Records are formed in FP64 and rounded once; frames keep |r'| at the size
// of a molecule so the cancellation in e stays at FP32 rounding level.
// ---------------------------------------------------------------------------
struct __align__(16) AtomRec {
  float bx, by, bz, c;  // -2 a2 c', a2 |c'|^2
};

__device__ __forceinline__ void make_rec(const Atom& a, float rx, float ry, float rz,
                                         AtomRec& rec, float& a2) {
  const double x = (double)a.x - (double)rx, y = (double)a.y - (double)ry,
               z = (double)a.z - (double)rz;
  const double k = (double)a.a2;
  rec.bx = (float)(-2.0 * k * x);
  rec.by = (float)(-2.0 * k * y);
  rec.bz = (float)(-2.0 * k * z);
  rec.c = (float)(k * (x * x + y * y + z * z));
  a2 = a.a2;
}

__device__ __forceinline__ float occupancy_x(const AtomRec& b, float a2, float rx, float ry,
                                             float rz, float r2) {
  float e = fmaf(a2, r2, b.c);
  e = fmaf(b.bx, rx, e);
  e = fmaf(b.by, ry, e);
  e = fmaf(b.bz, rz, e);
  return __builtin_amdgcn_exp2f(-e);
}

// Union complement q = prod(1 - o_i) at S points (expanded form).
template <int S>
__device__ __forceinline__ void eval_union_x(const AtomRec* __restrict__ rec,
                                             const float* __restrict__ a2, int n,
                                             const float (&rx)[S], const float (&ry)[S],
                                             const float (&rz)[S], const float (&r2)[S],
                                             float (&q)[S]) {
#pragma unroll 2
  for (int i = 0; i < n; ++i) {
    const AtomRec b = rec[i];
    const float a = a2[i];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float o = occupancy_x(b, a, rx[s], ry[s], rz[s], r2[s]);
      q[s] = fmaf(-q[s], o, q[s]);
    }
  }
}

// First-order density m and union complement q at S points (expanded form).
template <int S>
__device__ __forceinline__ void eval_density_x(const AtomRec* __restrict__ rec,
                                               const float* __restrict__ a2, int n,
                                               const float (&rx)[S], const float (&ry)[S],
                                               const float (&rz)[S], const float (&r2)[S],
                                               float (&m)[S], float (&q)[S]) {
#pragma unroll 2
  for (int i = 0; i < n; ++i) {
    const AtomRec b = rec[i];
    const float a = a2[i];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float o = occupancy_x(b, a, rx[s], ry[s], rz[s], r2[s]);
      m[s] += o;
      q[s] = fmaf(-q[s], o, q[s]);
    }
  }
}

// First-order density m and union u itself at S points (expanded form), u
// by the cancellation-free recurrence u <- u + o - u o.  Slightly dearer than
// tracking q = 1 - u, but u keeps its relative precision where every o_i is
// small, so w = u/m stays accurate in a molecule's tails (where a moved
// partner can sit during alignment).
template <int S>
__device__ __forceinline__ void eval_density_u_x(const AtomRec* __restrict__ rec,
                                                 const float* __restrict__ a2, int n,
                                                 const float (&rx)[S], const float (&ry)[S],
                                                 const float (&rz)[S], const float (&r2)[S],
                                                 float (&m)[S], float (&u)[S]) {
#pragma unroll 2
  for (int i = 0; i < n; ++i) {
    const AtomRec b = rec[i];
    const float a = a2[i];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float o = occupancy_x(b, a, rx[s], ry[s], rz[s], r2[s]);
      m[s] += o;
      u[s] = fmaf(-u[s], o, u[s] + o);
    }
  }
}

// |r|^2 of a point.
__device__ __forceinline__ float norm2(float x, float y, float z) {
  return fmaf(x, x, fmaf(y, y, z * z));
}

// Bounded weight w = u/m in [0, 1] (m > 0 for every sampled point; guard 0).
// u times the hardware reciprocal of m: within 2 ulp of the quotient.
__device__ __forceinline__ float bounded_weight(float u, float m) {
  return m > 0.0f ? fminf(u * __builtin_amdgcn_rcpf(m), 1.0f) : 0.0f;
}

// ---------------------------------------------------------------------------
// Wave-level reductions (fixed butterfly order: deterministic).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Wave sum by DPP: an inclusive scan inside each row of 16 lanes (shifts 1,
// 2, 4, 8), then lane 15 of rows 0 and 2 is added into rows 1 and 3 and lane
// 31 into rows 2 and 3, leaving the total in lane 63, which is returned to
// every lane.  Fixed order: deterministic.
template <int Ctrl, int RowMask>
__device__ __forceinline__ float dpp_step(float v) {
  const int s = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), Ctrl, RowMask, 0xf, true);
  return v + __builtin_bit_cast(float, s);
}
// Sum over each row of 16 lanes, returned to all 16 lanes of the row: XOR
// partners 1 and 2 inside each quad (quad_perm), then the mirror lane of the
// other quad (row_half_mirror) and of the other half row (row_mirror).  Each
// step adds two partials that the partner lane adds in the other order, and
// the sum of two floats does not depend on their order, so every lane of a
// row ends with the same bits.
__device__ __forceinline__ float row_sum16(float v) {
  v = dpp_step<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_step<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_step<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_step<0x140, 0xf>(v);  // row_mirror
  return v;
}
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v = dpp_step<0x111, 0xf>(v);  // row_shr:1
  v = dpp_step<0x112, 0xf>(v);  // row_shr:2
  v = dpp_step<0x114, 0xf>(v);  // row_shr:4
  v = dpp_step<0x118, 0xf>(v);  // row_shr:8
  v = dpp_step<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
  v = dpp_step<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Workgroups go to the chip's eight XCDs, each with its own L2, in
// round-robin order of blockIdx.  xcd_chunk(b, G) renumbers them so that
// tiles of kXcdTile consecutive items are each handled by one XCD (tile t on
// XCD t mod 8): neighbouring molecules, whose records share cache lines, then
// meet in one L2 instead of being fetched by two, and a tile's outputs fill
// whole lines.  Tiles, not one contiguous range per XCD, keep the XCDs evenly
// loaded when the work per item drifts along the index (a sorted library).
// A bijection on [0, G): below F = G - G mod (8 kXcdTile) block b = 8 k + x
// (XCD x, its k-th block) takes item (8 (k / T) + x) T + k mod T, which runs
// over [0, F) once; blocks from F on keep their index.
constexpr int kXcds = 8;
constexpr int kXcdTile = 64;
__device__ __forceinline__ int xcd_chunk(int b, int G) {
  const int F = G - G % (kXcds * kXcdTile);
  if (b >= F) return b;
  const int x = b % kXcds, k = b / kXcds;
  return ((k / kXcdTile) * kXcds + x) * kXcdTile + k % kXcdTile;
}

// Lane l's FP64 value, read by every lane (l wave-uniform).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const long long hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((hi << 32) | lo);
}

// Orders LDS writes of this wave before its later LDS reads (wave-private
// staging needs no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace shape
