// Learned triage for confidence-bounded screening: per-molecule features, the
// dense layers of a small MLP on the matrix cores (BF16 or FP32 operands,
// FP32 accumulation), its loss, Adam, and top-k selection.
#include "shape_kernels.hpp"

#include <algorithm>
#include <utility>
#include <vector>

#include <math.h>

namespace shape {

// ---------------------------------------------------------------------------
// Features, one wave per molecule (24 floats):
//   [0..15]  counts of |c_i - mu| in 0.5 A bins over [0, 8), last bin open
//   [16..18] sqrt of the descending eigenvalues of the mixture covariance
//            sum pi_i (c_i c_i^T + I/(2 alpha_i)) - mu mu^T, pi_i = v_i / Z
//   [19..22] atoms in the width classes alpha < 0.767, [0.767, 0.893),
//            [0.893, 0.995), >= 0.995
//   [23]     first-order self-overlap sum_ij (pi/(a_i+a_j))^(3/2)
//            exp(-a_i a_j/(a_i+a_j) |c_i-c_j|^2)
// Moments in two passes (mean, then centred second moments); the overlap sum
// over the i < j triangle is spread over all 64 lanes.
// ---------------------------------------------------------------------------

// Eigenvalues of a symmetric 3 x 3 matrix, descending, by the trigonometric
// closed form (Smith, CACM 1961).
__device__ void sym3_eigen_desc(double a00, double a11, double a22, double a01, double a02,
                                double a12, double ev[3]) {
  const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const double q = (a00 + a11 + a22) / 3.0;
  if (p1 <= 1e-300 * (q * q + 1e-300)) {
    ev[0] = a00; ev[1] = a11; ev[2] = a22;
  } else {
    const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
    const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1;
    const double p = sqrt(p2 / 6.0);
    const double ip = 1.0 / p;
    const double c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip;
    const double c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
    double r = 0.5 * (c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) +
                      c02 * (c01 * c12 - c11 * c02));
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double phi = acos(r) / 3.0;
    ev[0] = q + 2.0 * p * cos(phi);
    ev[2] = q + 2.0 * p * cos(phi + 2.0943951023931954923);
    ev[1] = 3.0 * q - ev[0] - ev[2];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (ev[j] > ev[i]) {
        const double t = ev[i];
        ev[i] = ev[j];
        ev[j] = t;
      }
}

// First-order Gaussian pair terms (pi/(a+b))^(3/2) exp(-a b/(a+b) d2) below,
// from hardware rsqrt, reciprocal and exp2 (features, not estimates: ~1e-6
// relative): a diagonal term (2a)^(-3/2) is rs^3 with rs = 1/sqrt(2a).

// Pair terms of the self-overlap triangle in the width form of the
// cross-overlaps: with b = 1/(log2(e) a) and B = b^(3/2) per atom and
// k = 1/(b_i + b_j), the term (a_i + a_j)^(-3/2) exp(-a_i a_j/(a_i+a_j) d2)
// is log2(e)^(3/2) B_i B_j k^(3/2) exp2(-k d2).  Padding atoms have B = 0
// and b = 1 (finite, no contribution).  FP32 for widths from 1e-6 to 1e6.
struct TriAtom {
  float x, y, z, b, B;
};

__device__ __forceinline__ TriAtom tri_atom(const float4* sC, int i, int n) {
  TriAtom t{0.f, 0.f, 0.f, 1.f, 0.f};
  if (i < n) {
    const float4 c = sC[i];
    t.x = c.x; t.y = c.y; t.z = c.z;
    t.b = __builtin_amdgcn_rcpf(1.44269504088896f * c.w);
    t.B = t.b * __builtin_amdgcn_sqrtf(t.b);
  }
  return t;
}

// v from the lane C places before this one in its row of 16 (row rotation)
template <int C>
__device__ __forceinline__ float row_ror(float v) {
  if constexpr (C == 0) {
    return v;
  } else {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x120 + C, 0xf, 0xf, true));
  }
}

// acc + B_p k^(3/2) exp2(-k d2) for this lane's atom s and the atom p of the
// lane C places back in the row
template <int C>
__device__ __forceinline__ float tri_term(const TriAtom& s, const TriAtom& p, float acc) {
  const float dx = row_ror<C>(p.x) - s.x, dy = row_ror<C>(p.y) - s.y,
              dz = row_ror<C>(p.z) - s.z;
  const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  const float r = __builtin_amdgcn_rsqf(row_ror<C>(p.b) + s.b);
  const float kk = r * r;
  const float e = __builtin_amdgcn_exp2f(-kk * d2);
  return fmaf(row_ror<C>(p.B) * (kk * r), e, acc);
}

template <int... C>
__device__ __forceinline__ float tri_terms(const TriAtom& s, const TriAtom& p, float acc,
                                           std::integer_sequence<int, C...>) {
  ((acc = tri_term<C>(s, p, acc)), ...);
  return acc;
}

// The caller's arrays are read directly (no preparation pass): validity as
// in the preparation (offsets in range, 1..max_atoms atoms, alpha > 0, all
// values finite; otherwise NaN features and the data-error flag), and
// Z = sum (pi/alpha_i)^(3/2) as an FP32 sum (a descriptor's scale, not an
// estimate).
// One molecule per 16-lane row, four per wave: a drug-sized molecule fills
// its row's lanes, and each sum is a 16-lane row sum (row_sum16, the same
// bits in every lane of the row).  Histogram and width-class counts are
// integer LDS atomics (exact, independent of their order).  The overlap
// triangle i < j runs over 16-atom blocks, so a wave runs as long as its
// largest molecule's triangle: given a launch order (molecules
// by descending size, order[slot] = molecule), the wave's four rows take
// slots 4 b .. 4 b + 3 and hold molecules of about one size.  A molecule's
// features depend on it alone, so the order changes no output.
constexpr int kFeatRows = 4;

__global__ __launch_bounds__(64) void k_features(MolsDev in, const int* __restrict__ order,
                                                 int* __restrict__ flag,
                                                 float* __restrict__ out,
                                                 float* __restrict__ mom) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sCount[kFeatRows][20];  // 16 radial bins, 4 width classes
  const int lane = threadIdx.x, l16 = lane & 15, row = lane >> 4;
  int mol;
  if (order) {
    const int slot = blockIdx.x * kFeatRows + row;
    mol = slot < in.n_mols ? order[slot] : in.n_mols;
  } else {
    mol = xcd_chunk(blockIdx.x, gridDim.x) * kFeatRows + row;
  }
  float4* sC = reinterpret_cast<float4*>(smem) + (size_t)row * in.max_atoms;  // x, y, z, alpha
  const bool live = mol < in.n_mols;
  int a0 = 0, n = 0;
  bool bad = false;
  if (live) {
    a0 = in.off[mol];
    const int a1 = in.off[mol + 1];
    n = a1 - a0;
    bad = !(a0 >= 0 && (int64_t)a1 <= in.n_atoms && n >= 1 && n <= in.max_atoms);
    if (bad) n = 0;
  }
  for (int k = l16; k < 20; k += 16) sCount[row][k] = 0;
  // staging: the row's first 64 atoms (four per lane) are requested before
  // any is used, so that their loads overlap; larger molecules go on in a
  // loop
  float zl = 0.f;
  const auto stage = [&](float4 c, int i) {
    if (!(c.w > 0.0f) || !isfinite(c.w) || !isfinite(c.x) || !isfinite(c.y) || !isfinite(c.z))
      bad = true;
    sC[i] = c;
    const float t = 3.14159265358979f * __builtin_amdgcn_rcpf(c.w);
    zl += t * __builtin_amdgcn_sqrtf(t);
  };
  const auto fetch = [&](int i) {
    const float* p = in.xyz + 3 * (int64_t)(a0 + i);
    return make_float4(p[0], p[1], p[2], in.alpha[a0 + i]);
  };
  {
    float4 st[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (l16 + 16 * k < n) st[k] = fetch(l16 + 16 * k);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (l16 + 16 * k < n) stage(st[k], l16 + 16 * k);
  }
  for (int i = l16 + 64; i < n; i += 16) stage(fetch(i), i);
  // a row is bad if any of its lanes saw bad data: OR over the row's bits
  const uint64_t bb = __ballot(bad);
  bad = ((bb >> (16 * row)) & 0xFFFFull) != 0;
  if (bad) n = 0;  // the row skips every pass and writes NaN below
  wave_lds_sync();
  const float iZ = 1.0f / row_sum16(zl);
  // pass 1: mixture mean
  float mx = 0.f, my = 0.f, mz = 0.f;
  for (int i = l16; i < n; i += 16) {
    const float4 c = sC[i];
    // descriptors, not estimates: hardware reciprocal and square root (1 ulp)
    const float t = 3.14159265358979f * __builtin_amdgcn_rcpf(c.w);
    const float pi = t * __builtin_amdgcn_sqrtf(t) * iZ;
    mx = fmaf(pi, c.x, mx); my = fmaf(pi, c.y, my); mz = fmaf(pi, c.z, mz);
  }
  mx = row_sum16(mx); my = row_sum16(my); mz = row_sum16(mz);
  // pass 2: centred second moments, radial histogram, width classes
  float sxx = 0.f, syy = 0.f, szz = 0.f, sxy = 0.f, sxz = 0.f, syz = 0.f;
  for (int i = l16; i < n; i += 16) {
    const float4 c = sC[i];
    const float ia = __builtin_amdgcn_rcpf(c.w);
    const float t = 3.14159265358979f * ia;
    const float pi = t * __builtin_amdgcn_sqrtf(t) * iZ;
    const float x = c.x - mx, y = c.y - my, z = c.z - mz, h = 0.5f * ia;
    sxx = fmaf(pi, fmaf(x, x, h), sxx); syy = fmaf(pi, fmaf(y, y, h), syy);
    szz = fmaf(pi, fmaf(z, z, h), szz);
    sxy = fmaf(pi * x, y, sxy); sxz = fmaf(pi * x, z, sxz); syz = fmaf(pi * y, z, syz);
    const float r = __builtin_amdgcn_sqrtf(fmaf(x, x, fmaf(y, y, z * z)));
    int bin = (int)floorf(r * 2.0f);
    bin = bin > 15 ? 15 : bin;
    const int cls = c.w < 0.767f ? 0 : (c.w < 0.893f ? 1 : (c.w < 0.995f ? 2 : 3));
    atomicAdd(&sCount[row][bin], 1);
    atomicAdd(&sCount[row][16 + cls], 1);
  }
  sxx = row_sum16(sxx); syy = row_sum16(syy); szz = row_sum16(szz);
  sxy = row_sum16(sxy); sxz = row_sum16(sxz); syz = row_sum16(syz);
  // first-order self-overlap: diagonal + 2 x the i < j triangle.  Diagonal
  // terms are summed as (2a)^(-3/2); pi^(3/2), the triangle's factor 2 and
  // the width form's log2(e)^(3/2) are applied to the row sums.
  float fo = 0.f, tri = 0.f;
  for (int i = l16; i < n; i += 16) {
    const float a = sC[i].w, rs = __builtin_amdgcn_rsqf(a + a);
    fo = fmaf(rs * rs, rs, fo);
  }
  // The triangle by 16-atom blocks a <= b of the row's atoms (padded with
  // atoms of weight 0): each lane holds one atom of block a and one of block
  // b, and row rotations bring it every atom of block b in turn (tri_terms),
  // so the terms read no LDS.
  const int nb = (n + 15) >> 4;
  for (int ba = 0; ba < nb; ++ba) {
    const TriAtom own = tri_atom(sC, 16 * ba + l16, n);
    // the diagonal block: rotations 1..7, and 8 on half of the lanes (the
    // pairs at rotation 8 are met twice in the row)
    float acc = tri_terms(own, own, 0.f, std::integer_sequence<int, 1, 2, 3, 4, 5, 6, 7>{});
    const float a8 = tri_term<8>(own, own, 0.f);
    acc += l16 < 8 ? a8 : 0.f;
    for (int bb = ba + 1; bb < nb; ++bb) {
      const TriAtom other = tri_atom(sC, 16 * bb + l16, n);
      acc = tri_terms(own, other, acc, std::make_integer_sequence<int, 16>{});
    }
    tri = fmaf(own.B, acc, tri);
  }
  const float fo_sum =
      5.56832799683170785f * (row_sum16(fo) + 2.0f * 1.73285334265681730f * row_sum16(tri));
  wave_lds_sync();  // the counts are complete
  if (!live) return;
  float* f = out + (size_t)mol * 24;
  float* mm = mom + (size_t)mol * 6;
  if (bad) {
    for (int k = l16; k < 24; k += 16) f[k] = __builtin_nanf("");
    if (l16 < 6) mm[l16] = __builtin_nanf("");
    if (l16 == 0) atomicOr(flag, 1);
    return;
  }
  f[l16] = (float)sCount[row][l16];
  if (l16 < 4) f[19 + l16] = (float)sCount[row][16 + l16];
  // the covariance goes to k_features_eigen, which diagonalises one matrix
  // per lane rather than one per row
  if (l16 == 0) {
    mm[0] = sxx; mm[1] = syy; mm[2] = szz;
    mm[3] = sxy; mm[4] = sxz; mm[5] = syz;
    f[23] = fo_sum;
  }
}

// Features [16..18]: square roots of the descending eigenvalues of each
// molecule's mixture covariance (FP64 closed form), one molecule per thread.
__global__ void k_features_eigen(int n_mols, const float* __restrict__ mom,
                                 float* __restrict__ out) {
  const int mol = blockIdx.x * blockDim.x + threadIdx.x;
  if (mol >= n_mols) return;
  const float* mm = mom + (size_t)mol * 6;
  if (isnan(mm[0])) return;  // invalid molecule: its features are NaN already
  double ev[3];
  sym3_eigen_desc(mm[0], mm[1], mm[2], mm[3], mm[4], mm[5], ev);
  float* f = out + (size_t)mol * 24;
  for (int k = 0; k < 3; ++k) f[16 + k] = (float)sqrt(ev[k] > 0.0 ? ev[k] : 0.0);
}

// First-order cross-overlap of (query, library molecule) pairs at their
// current poses, Eq. fo: sum_ij (pi/(a_i+a_j))^(3/2)
// exp(-a_i a_j/(a_i+a_j) |c_i - c_j|^2).  Four waves per workgroup share the
// query's atoms in LDS; each wave walks a contiguous run of pairs, one pair
// at a time with all 64 lanes.  The query is the same for every pair, so the
// lanes are laid out as NI query slots x 64/NI phases: lane l holds query
// atom i = ib + l % NI in registers and walks the library molecule's atoms
// j = l / NI, l / NI + 64/NI, ... as LDS broadcasts.  Slots past the query's
// last atom hold a phantom atom 10^18 A away whose terms are exactly zero.
// A pair is only ~15 terms per lane, so the wave hides the memory latency
// itself: the headers (molecule index, atom range) of 64 pairs are read at
// once, one per lane, and the next pair's atoms are loaded while the current
// pair's terms are summed.  FP32 sums, DPP wave sum.
//
// Per term the widths enter as b = 1/a' (a' = log2(e) a): with
// k = 1/(b_i + b_j) = a'_i a'_j/(a'_i + a'_j), the term is
// (pi log2(e))^(3/2) (b_i b_j)^(3/2) k^(3/2) exp2(-k d^2), and
// b_j^(3/2) exp2(-k d^2) = exp2(-k d^2 + 1.5 log2 b_j), so a term is one
// rsq (k^(1/2)), one exp2 and five VALU; b_i^(3/2) scales the lane's sum
// once.  The squared distance is the expanded form
// |c_i|^2 + |c_j|^2 - 2 c_i . c_j (four VALU) in a frame centred on the
// query's centroid, where the atoms that overlap have small coordinates: an
// FP32 emulation over molecules of 1-256 atoms (with correctly rounded rsq,
// exp2 and log2; the hardware's are within a few ulp) stays within 7e-7 of
// the FP64 closed form.  Library widths use the hardware reciprocal and
// log2 (once per atom and pair).
constexpr int kFoWaves = 4;

__device__ __forceinline__ bool atom_ok(float al, float x, float y, float z) {
  return al > 0.0f && isfinite(al) && isfinite(x) && isfinite(y) && isfinite(z);
}

// The caller's arrays are read directly (no preparation pass); a molecule
// with invalid data (offsets out of range, alpha <= 0, non-finite values)
// gives NaN and raises the data-error flag; a pair index outside the
// library gives NaN.
constexpr int kFoChunks = SHAPE_MAX_ATOMS / kWave;  // library atoms per lane, at most

// Phantom atoms 10^18 A from every real atom, the query's at +10^18 and the
// library's at -10^18 on each axis (so two phantoms are 2 10^18 apart too),
// both with b = 1: every term with a phantom is exactly zero (exp2 of minus
// a huge number), so padded slots need no branch.  Query records hold
// (-2 c, |c|^2), library records (c, |c|^2).
__device__ __forceinline__ float4 fo_phantom_query() {
  return make_float4(-2e18f, -2e18f, -2e18f, 3e36f);
}
__device__ __forceinline__ float4 fo_phantom_lib() {
  return make_float4(-1e18f, -1e18f, -1e18f, 3e36f);
}

// NI query slots x 64/NI phases; CH chunks of 64 library atoms per lane at
// most (1 when no library molecule passes 64 atoms).
template <int NI, int CH>
__global__ __launch_bounds__(kWave * kFoWaves) void k_fo_cross(
    MolsDev Q, MolsDev L, const int* __restrict__ pairs, int n_pairs, int per_wave,
    int* __restrict__ flag, float* __restrict__ out) {
  constexpr int kPhases = kWave / NI;
  constexpr int kUnroll = 2;
  constexpr int kPad = kPhases * kUnroll;  // library atoms padded to a multiple of this
  // query records [max_q]; each wave's library atoms [max_b padded], two
  // 16-byte words per atom (c, |c|^2) and (b, 1.5 log2 b, -, -) read from one
  // address; the query's widths (b, b^1.5) [max_q]
  extern __shared__ float4 fo_lds[];
  __shared__ float4 s_cen;  // the query's centroid
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int max_b_pad = (L.max_atoms + kPad - 1) / kPad * kPad;
  float4* sA = fo_lds;
  float4* sB = fo_lds + Q.max_atoms + 2 * w * max_b_pad;
  float2* sAw = reinterpret_cast<float2*>(fo_lds + Q.max_atoms + 2 * kFoWaves * max_b_pad);
  // this wave's pairs [p_begin, p_end)
  const int64_t g = (int64_t)blockIdx.x * kFoWaves + w;
  const int p_begin = (int)min((int64_t)n_pairs, g * per_wave);
  const int p_end = (int)min((int64_t)n_pairs, (int64_t)p_begin + per_wave);
  const int q0 = Q.off[0], q1 = Q.off[1], nq = q1 - q0;
  const bool q_range = q0 >= 0 && (int64_t)q1 <= Q.n_atoms && nq >= 1 && nq <= Q.max_atoms;
  if (w == 0) {  // centroid: lane-strided sums in atom order, one DPP wave sum
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    if (q_range) {
      for (int i = lane; i < nq; i += kWave) {
        sx += Q.xyz[3 * (q0 + i)];
        sy += Q.xyz[3 * (q0 + i) + 1];
        sz += Q.xyz[3 * (q0 + i) + 2];
      }
    }
    sx = wave_sum_dpp(sx);
    sy = wave_sum_dpp(sy);
    sz = wave_sum_dpp(sz);
    const float inv = 1.0f / (float)(q_range ? nq : 1);
    if (lane == 0) s_cen = make_float4(sx * inv, sy * inv, sz * inv, 0.0f);
  }
  __syncthreads();
  const float4 cen = s_cen;
  int q_bad = q_range ? 0 : 1;
  if (q_range) {
    for (int i = threadIdx.x; i < nq; i += kWave * kFoWaves) {
      const float al = Q.alpha[q0 + i];
      const float x = Q.xyz[3 * (q0 + i)], y = Q.xyz[3 * (q0 + i) + 1],
                  z = Q.xyz[3 * (q0 + i) + 2];
      if (!atom_ok(al, x, y, z)) q_bad = 1;
      const float dx = x - cen.x, dy = y - cen.y, dz = z - cen.z;
      const float b = 1.0f / (1.44269504088896f * al);
      sA[i] = make_float4(-2.0f * dx, -2.0f * dy, -2.0f * dz, fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
      sAw[i] = make_float2(b, b * sqrtf(b));
    }
  }
  // reached by every wave (no return before it); the outcome is grid-uniform
  if (__syncthreads_or(q_bad)) {
    for (int p = p_begin + lane; p < p_end; p += kWave) out[p] = __builtin_nanf("");
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flag, 1);
    return;
  }
  const int li = lane % NI, ph = lane / NI;
  for (int sub = p_begin; sub < p_end; sub += kWave) {
    const int cnt = min(kWave, p_end - sub);
    // headers of up to 64 pairs, one per lane: bit 0 the atom range is
    // valid, bit 1 the molecule index lies in the library
    int hb0 = 0, hnb = 0, hfl = 0;
    if (lane < cnt) {
      const int m = pairs ? pairs[sub + lane] : sub + lane;
      if (m >= 0 && m < L.n_mols) {
        hb0 = L.off[m];
        const int b1 = L.off[m + 1];
        hnb = b1 - hb0;
        hfl = 2 | ((hb0 >= 0 && (int64_t)b1 <= L.n_atoms && hnb >= 1 && hnb <= L.max_atoms)
                       ? 1 : 0);
      }
    }
    // atoms (x, y, z, alpha) of one pair into registers, lane j owns atoms
    // j, j + 64, ...; the loads stay in flight until the values are used
    float4 nxt[CH];
    auto load = [&](int k) {
      const int b0 = __builtin_amdgcn_readlane(hb0, k), nb = __builtin_amdgcn_readlane(hnb, k);
      const bool ok = __builtin_amdgcn_readlane(hfl, k) & 1;
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int j = c * kWave + lane;
        if (ok && j < nb) {
          const size_t a = (size_t)b0 + j;
          nxt[c] = make_float4(L.xyz[3 * a], L.xyz[3 * a + 1], L.xyz[3 * a + 2], L.alpha[a]);
        }
      }
    };
    load(0);
    for (int k = 0; k < cnt; ++k) {
      const int p = sub + k;
      const int nb = __builtin_amdgcn_readlane(hnb, k), fl = __builtin_amdgcn_readlane(hfl, k);
      const int nb_pad = (nb + kPad - 1) / kPad * kPad;
      bool a_bad = false;
      if (fl & 1) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int j = c * kWave + lane;
          if (j < nb) {
            const float4 a = nxt[c];
            if (!atom_ok(a.w, a.x, a.y, a.z)) a_bad = true;
            const float dx = a.x - cen.x, dy = a.y - cen.y, dz = a.z - cen.z;
            const float b = __builtin_amdgcn_rcpf(1.44269504088896f * a.w);
            sB[2 * j] = make_float4(dx, dy, dz, fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
            sB[2 * j + 1] = make_float4(b, 1.5f * __builtin_amdgcn_logf(b), 0.0f, 0.0f);
          } else if (j < nb_pad) {
            sB[2 * j] = fo_phantom_lib();
            sB[2 * j + 1] = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
          }
        }
      }
      const bool data_bad = __ballot(a_bad) != 0;
      if (k + 1 < cnt) load(k + 1);  // the next pair's atoms arrive during this pair's terms
      if (!(fl & 1) || data_bad) {
        if (lane == 0) {
          out[p] = __builtin_nanf("");
          // invalid data is flagged; an index outside the library only gives NaN
          if (data_bad || (fl & 2)) atomicOr(flag, 1);
        }
        continue;
      }
      wave_lds_sync();
      float acc = 0.0f;
      for (int ib = 0; ib < nq; ib += NI) {  // one block unless the query passes NI atoms
        const int i = ib + li;
        const bool real = i < nq;
        const float4 ci = real ? sA[i] : fo_phantom_query();
        const float2 wi = real ? sAw[i] : make_float2(1.0f, 1.0f);
        const int n_iter = nb_pad / kPad;  // wave-uniform trip count
        float accb = 0.0f;
        for (int t = 0; t < n_iter; ++t) {
          const int j = ph + t * kPad;
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const float4 cj = sB[2 * (j + u * kPhases)];
            const float4 wj = sB[2 * (j + u * kPhases) + 1];
            const float d2 = fmaf(ci.x, cj.x, fmaf(ci.y, cj.y, fmaf(ci.z, cj.z, ci.w + cj.w)));
            const float r = __builtin_amdgcn_rsqf(wi.x + wj.x);  // k^(1/2)
            const float kk = r * r;
            accb = fmaf(kk * r, __builtin_amdgcn_exp2f(fmaf(-kk, d2, wj.y)), accb);
          }
        }
        acc = fmaf(accb, wi.y, acc);
      }
      const float sum = 9.64909578231936f * wave_sum_dpp(acc);  // (pi log2(e))^(3/2)
      if (lane == 0) out[p] = sum;
      wave_lds_sync();  // every read of this pair's atoms before the next pair's writes
    }
  }
}

__device__ __forceinline__ float pair_feature(const float* __restrict__ fq,
                                              const float* __restrict__ flib, int q, int m,
                                              int j, const float* __restrict__ fo_cross, int p,
                                              const float* __restrict__ mean,
                                              const float* __restrict__ inv_std) {
  const int k = j % 24;
  const float a = fq[(size_t)q * 24 + k], b = flib[(size_t)m * 24 + k];
  float raw;
  switch (j / 24) {
    case 0: raw = a; break;
    case 1: raw = b; break;
    case 2: raw = fabsf(a - b); break;
    default: raw = a * b; break;
  }
  if (fo_cross && k == 23 && j >= 48) {
    const float o = fo_cross[p];
    raw = (j < 72) ? o / (a + b - o) : o;
  }
  return (raw - mean[j]) * inv_std[j];
}

__global__ void k_pair_features(const float* __restrict__ fq, const float* __restrict__ flib,
                                const int* __restrict__ qidx, const int* __restrict__ idx, int n,
                                const float* __restrict__ fo_cross,
                                const float* __restrict__ mean,
                                const float* __restrict__ inv_std, float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * 96) return;
  const int p = (int)(t / 96), j = (int)(t % 96);
  const int m = idx ? idx[p] : p;
  const int q = qidx ? qidx[p] : 0;
  out[t] = pair_feature(fq, flib, q, m, j, fo_cross, p, mean, inv_std);
}

// ---------------------------------------------------------------------------
// Dense layer on the matrix cores:
//   C[m][n] = epilogue( sum_k A[m][k] B[k][n] )
// A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn] (any transposition),
// epilogue: + bias[n], then ReLU, or multiplication by 1[gate[m][n] > 0]
// (ReLU backward).  BF16: v_mfma_f32_16x16x32_bf16, operands rounded to
// nearest even (LDS-tiled kernel below); FP32: v_mfma_f32_16x16x4f32
// (workgroup tile 64 x 64, 4 waves x 32 x 32, each 2 x 2 MFMA 16 x 16 tiles).
// Lane l supplies row (or column) l mod 16 and k-group l / 16; result element
// (4 (l/16) + r, l mod 16) sits in accumulator r of lane l.
// ---------------------------------------------------------------------------
typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

// D += A B for a 16 x 32 by 32 x 16 BF16 tile on v_mfma_f32_16x16x32_bf16:
// lane l supplies row (or column) l mod 16 and k = 8 (l / 16) .. 8 (l / 16) + 7
// (layout checked on the GPU); the result layout is that of the 16x16x16 form.
__device__ __forceinline__ v4f mfma_bf16_k32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                 __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// Float to bfloat16 by gfx950's v_cvt_pk_bf16_f32 (round to nearest even;
// NaN stays NaN): the one conversion of every BF16 operand in the library,
// so the staged products, the fused network kernels and the packed weights
// round alike.  to_bf16x2 converts two values (x in the low half) in one
// instruction.
__device__ __forceinline__ uint32_t to_bf16x2(float x, float y) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f{x, y}), v2bf));
}

__device__ __forceinline__ short to_bf16(float x) { return (short)(to_bf16x2(x, 0.f) & 0xFFFFu); }

// FP32 products (tight-parity mode): operands read straight from global
// memory, one v_mfma_f32_16x16x4f32 step per 4 values of k.
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs g) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int kb = g.part ? blockIdx.z * g.k_chunk : 0;
  const int ke = g.part ? min(g.K, kb + g.k_chunk) : g.K;
  for (int k0 = kb; k0 < ke; k0 += 4) {
    float a[2], b[2];
    const int k = k0 + lk;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = m0 + 16 * i + li;
      a[i] = (m < g.M && k < ke) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + 16 * j + li;
      b[j] = (n < g.N && k < ke) ? g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + 16 * i + 4 * lk + r;
        const int n = n0 + 16 * j + li;
        if (m < g.M && n < g.N && g.part) {
          g.part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = acc[i][j][r];
        } else if (m < g.M && n < g.N) {
          float v = acc[i][j][r];
          if (g.bias) v += g.bias[n];
          if (g.flags & SHAPE_GEMM_RELU) v = v > 0.f ? v : 0.f;
          if (g.gate && !(g.gate[(int64_t)m * g.sgm + n] > 0.f)) v = 0.f;
          g.C[(int64_t)m * g.scm + n] = v;
        }
      }
}

// BF16 dense layer with LDS tiling: workgroup tile TM x TN (128 x 128, or
// 64 x 64 for products whose large tiles would leave CUs idle), k-slab 32.
// Both operands are staged as bfloat16 with k contiguous (A_s[m][k],
// B_s[n][k]), loaded from global memory along whichever dimension is
// contiguous there, so every wave reads whole cache lines.  Each of the four
// waves computes a (TM/2) x (TN/2) sub-tile of 16 x 16 MFMA tiles, one
// v_mfma_f32_16x16x32_bf16 per tile and slab.  Every output element
// accumulates k in the same order (slabs of 32, increasing) whatever the tile
// size, so both sizes give the same bits.
constexpr int kTK = 32, kLdk = kTK + 8;

// One output tile (bx, by) of split bz: the body of k_gemm_bf16_tiled, also
// run by k_gemm_set for each product of a batch.
template <int TM, int TN>
__device__ __forceinline__ void gemm_bf16_tile(const GemmArgs& g, int bx, int by, int bz) {
  constexpr int FM = TM / 32, FN = TN / 32;           // MFMA tiles per wave
  constexpr int RA = TM * kTK / 256, RB = TN * kTK / 256;  // staged values per thread
  __shared__ __align__(16) short As[TM * kLdk];
  __shared__ __align__(16) short Bs[TN * kLdk];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int bm = by * TM, bn = bx * TN;
  const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * (TN / 2);
  const int li = lane & 15, lk = lane >> 4;
  v4f acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const bool a_kfast = g.sak == 1;
  const bool b_nfast = g.sbn == 1;
  const int kb = g.part ? bz * g.k_chunk : 0;
  const int ke = g.part ? min(g.K, kb + g.k_chunk) : g.K;
  // Slabs of kTK values of k: slab s+1 is read from global memory into
  // registers while the matrix cores work on slab s from LDS.
  float pa[RA], pb[RB];
  auto load_slab = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r) {  // A: TM x 32 elements
      int m, k;
      if (a_kfast) {
        k = tid & 31;
        m = (tid >> 5) + 8 * r;
      } else {
        m = tid % TM;
        k = tid / TM + (256 / TM) * r;
      }
      const int gm = bm + m, gk = k0 + k;
      pa[r] = (gm < g.M && gk < ke) ? g.A[(int64_t)gm * g.sam + (int64_t)gk * g.sak] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {  // B: 32 x TN elements
      int n, k;
      if (b_nfast) {
        n = tid % TN;
        k = tid / TN + (256 / TN) * r;
      } else {
        k = tid & 31;
        n = (tid >> 5) + 8 * r;
      }
      const int gn = bn + n, gk = k0 + k;
      pb[r] = (gn < g.N && gk < ke) ? g.B[(int64_t)gk * g.sbk + (int64_t)gn * g.sbn] : 0.f;
    }
  };
  auto store_slab = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int m = a_kfast ? (tid >> 5) + 8 * r : tid % TM;
      const int k = a_kfast ? tid & 31 : tid / TM + (256 / TM) * r;
      As[m * kLdk + k] = to_bf16(pa[r]);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {  // stored transposed as Bs[n][k]
      const int n = b_nfast ? tid % TN : (tid >> 5) + 8 * r;
      const int k = b_nfast ? tid / TN + (256 / TN) * r : tid & 31;
      Bs[n * kLdk + k] = to_bf16(pb[r]);
    }
  };
  if (kb < ke) load_slab(kb);
  for (int k0 = kb; k0 < ke; k0 += kTK) {
    store_slab();
    __syncthreads();
    if (k0 + kTK < ke) load_slab(k0 + kTK);
    {
      v8s a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = *reinterpret_cast<const v8s*>(&As[(wm + 16 * i + li) * kLdk + 8 * lk]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        b[j] = *reinterpret_cast<const v8s*>(&Bs[(wn + 16 * j + li) * kLdk + 8 * lk]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = mfma_bf16_k32(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = bm + wm + 16 * i + 4 * lk + r;
        const int n = bn + wn + 16 * j + li;
        if (m < g.M && n < g.N && g.part) {
          g.part[((int64_t)bz * g.M + m) * g.N + n] = acc[i][j][r];
        } else if (m < g.M && n < g.N) {
          float v = acc[i][j][r];
          if (g.bias) v += g.bias[n];
          if (g.flags & SHAPE_GEMM_RELU) v = v > 0.f ? v : 0.f;
          if (g.gate && !(g.gate[(int64_t)m * g.sgm + n] > 0.f)) v = 0.f;
          g.C[(int64_t)m * g.scm + n] = v;
        }
      }
}

// Split-K reduction: C[m][n] = epilogue(sum_z part[z][m][n]), z in order.
template <int TM, int TN>
__global__ __launch_bounds__(256, 2) void k_gemm_bf16_tiled(GemmArgs g) {
  gemm_bf16_tile<TM, TN>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Up to kGemmSetMax BF16 products with 64 x 64 tiles in one launch (the
// weight gradients of all layers): workgroup b runs tile b - blk0[t] of
// product t, numbered split-major like the single launch's grid, so every
// product gets exactly its single-launch arithmetic.
struct GemmSet {
  int n;
  GemmArgs g[kGemmSetMax];
  int tx[kGemmSetMax], ty[kGemmSetMax], splits[kGemmSetMax];
  int blk0[kGemmSetMax + 1];   // first workgroup of each product
  int64_t el0[kGemmSetMax + 1];  // first reduced element of each product (split ones)
};

__global__ __launch_bounds__(256, 2) void k_gemm_set(GemmSet s) {
  int t = 0;
  while (t + 1 < s.n && (int)blockIdx.x >= s.blk0[t + 1]) ++t;  // uniform
  const int local = (int)blockIdx.x - s.blk0[t];
  const int per = s.tx[t] * s.ty[t];
  const int r = local % per;
  gemm_bf16_tile<64, 64>(s.g[t], r % s.tx[t], r / s.tx[t], local / per);
}

__global__ void k_splitk_reduce(GemmArgs g, int splits) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)g.M * g.N) return;
  const int m = (int)(t / g.N), n = (int)(t % g.N);
  float v = 0.0f;
  for (int z = 0; z < splits; ++z) v += g.part[(int64_t)z * g.M * g.N + t];
  if (g.bias) v += g.bias[n];
  if (g.flags & SHAPE_GEMM_RELU) v = v > 0.f ? v : 0.f;
  if (g.gate && !(g.gate[(int64_t)m * g.sgm + n] > 0.f)) v = 0.f;
  g.C[(int64_t)m * g.scm + n] = v;
}

// The split-K reductions of a GemmSet in one launch (k_splitk_reduce's
// arithmetic per element).
__global__ void k_splitk_reduce_set(GemmSet s) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s.el0[s.n]) return;
  int t = 0;
  while (t + 1 < s.n && e >= s.el0[t + 1]) ++t;
  const GemmArgs& g = s.g[t];
  const int64_t q = e - s.el0[t];
  const int m = (int)(q / g.N), n = (int)(q % g.N);
  float v = 0.0f;
  for (int z = 0; z < s.splits[t]; ++z) v += g.part[(int64_t)z * g.M * g.N + q];
  if (g.bias) v += g.bias[n];
  if (g.flags & SHAPE_GEMM_RELU) v = v > 0.f ? v : 0.f;
  if (g.gate && !(g.gate[(int64_t)m * g.sgm + n] > 0.f)) v = 0.f;
  g.C[(int64_t)m * g.scm + n] = v;
}

// ---------------------------------------------------------------------------
// Fused surrogate inference for the 96-256-256-256-2 network: pair features,
// standardisation and all four layers in one kernel, activations resident in
// LDS.  The arithmetic is that of shape_pair_features followed by one
// shape_gemm per layer (BF16 operands rounded to nearest even, FP32
// accumulation over k in steps of 32 in increasing order on the same matrix
// instruction, bias then ReLU in FP32), so the outputs agree bit for bit; only
// the HBM round trips of the features and activations are gone.
//
// Weights are first packed to BF16 in MFMA fragment order: for layer l,
// block (kb, nb) of 32 x 16 holds 64 lanes x 8 values, lane = 16 (k%32 / 8) +
// n%16, value k%8, so one wave reads a B fragment as 1 KB of contiguous
// bytes.  The last layer's 2 outputs are padded to 16 columns with zeros.
// ---------------------------------------------------------------------------
constexpr int kMlpIn = 96, kMlpHid = 256, kMlpOut = 2;
constexpr int kMlpLd = kMlpHid + 8;     // LDS row stride (bf16 elements)

__host__ __device__ constexpr int mlp_pack_offset(int layer) {
  // fragment blocks of 32 x 16 (512 bf16) per layer: 3x16, 8x16, 8x16, 8x1
  return layer == 0 ? 0
       : layer == 1 ? 3 * 16 * 512
       : layer == 2 ? (3 * 16 + 8 * 16) * 512
                    : (3 * 16 + 2 * 8 * 16) * 512;
}
constexpr int kMlpPackElems = (3 * 16 + 2 * 8 * 16 + 8) * 512;

__global__ void k_mlp_pack(const float* __restrict__ params, short* __restrict__ packed) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kMlpPackElems) return;
  int layer = 3;
  while (layer > 0 && t < mlp_pack_offset(layer)) --layer;
  const int local = t - mlp_pack_offset(layer);
  const int n_in = layer == 0 ? kMlpIn : kMlpHid;
  const int n_out = layer == 3 ? kMlpOut : kMlpHid;
  const int nbs = layer == 3 ? 1 : kMlpHid / 16;   // column blocks
  const int blk = local / 512, within = local % 512;
  const int kb = blk / nbs, nb = blk % nbs;
  const int lane = within / 8, e = within % 8;
  const int k = kb * 32 + 8 * (lane >> 4) + e;
  const int n = nb * 16 + (lane & 15);
  // offset of W_layer in the flat W0, b0, W1, b1, ... vector
  int off = 0;
  for (int l = 0; l < layer; ++l) {
    const int i_ = l == 0 ? kMlpIn : kMlpHid;
    const int o_ = l == 3 ? kMlpOut : kMlpHid;
    off += i_ * o_ + o_;
  }
  const float v = (n < n_out && k < n_in) ? params[off + k * n_out + n] : 0.0f;
  packed[t] = to_bf16(v);
}

struct MlpArgs {
  const float* fq;
  const float* flib;
  const int* qidx;
  const int* idx;
  int n;
  const float* fo_cross;
  const float* mean;
  const float* inv_std;
  const v8s* W;        // packed weights (kMlpPackElems bf16)
  const float* b[4];   // biases of the four layers
  float* out;          // [n][2]
  float* x_out;        // training forward: standardised features [n][96]
  float* h_out[3];     // and the hidden activations [n][256] (FP32, after ReLU)
};

// Staging of the fused network kernels: the standardised pair features of
// rows [row0, row0 + ROWS) rounded to bf16 into H (rows beyond n zero);
// kAct also writes them to a.x_out (FP32), kF into the FP32 staging F (row
// stride kTrLdf).  Thread (part h, row r) writes feature blocks h BPT .. h
// BPT + BPT - 1 of row r — the blocks are f_q, f_m, |f_q - f_m|, f_q * f_m,
// 24 values each; h is uniform per wave, so the statistics are scalar loads.
// Same expressions as pair_feature.
constexpr int kTrLdf = kMlpHid + 4;   // FP32 staging row stride (floats)

template <int ROWS, bool kAct, bool kF>
__device__ __forceinline__ void mlp_stage_features(const MlpArgs& a, int row0, short* H,
                                                   float* F) {
  // threads per row (the first NH x ROWS threads of the workgroup take part)
  constexpr int NH = ROWS >= 64 ? 256 / ROWS : 4;
  constexpr int BPT = 4 / NH;      // feature blocks of 24 per thread
  constexpr int FPT = 24 * BPT;    // features per thread
  const int tid = threadIdx.x;
  const int r = tid & (ROWS - 1);
  // the part is uniform per wave when ROWS >= 64 (then scalar statistics)
  const int h = ROWS >= 64 ? __builtin_amdgcn_readfirstlane(tid / ROWS) : tid / ROWS;
  const int p = row0 + r;
  float raw[FPT];
  if (p < a.n) {
    const int m = a.idx ? a.idx[p] : p;
    const int q = a.qidx ? a.qidx[p] : 0;
    const float* fa = a.fq + (size_t)q * 24;
    const float* fb = a.flib + (size_t)m * 24;
    float va[24], vb[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) {
      va[k] = fa[k];
      vb[k] = fb[k];
    }
#pragma unroll
    for (int bb = 0; bb < BPT; ++bb) {
      const int b = h * BPT + bb;  // uniform
      float* out = raw + 24 * bb;
      if (b == 0) {
#pragma unroll
        for (int k = 0; k < 24; ++k) out[k] = va[k];
      } else if (b == 1) {
#pragma unroll
        for (int k = 0; k < 24; ++k) out[k] = vb[k];
      } else if (b == 2) {
#pragma unroll
        for (int k = 0; k < 24; ++k) out[k] = fabsf(va[k] - vb[k]);
      } else {
#pragma unroll
        for (int k = 0; k < 24; ++k) out[k] = va[k] * vb[k];
      }
      if (a.fo_cross && b >= 2) {
        const float o = a.fo_cross[p];
        out[23] = b == 2 ? o / (va[23] + vb[23] - o) : o;
      }
    }
    const float* mu = a.mean + FPT * h;
    const float* is = a.inv_std + FPT * h;
#pragma unroll
    for (int t = 0; t < FPT; ++t) raw[t] = (raw[t] - mu[t]) * is[t];
    if (kAct) {
      float4* xo = reinterpret_cast<float4*>(a.x_out + (size_t)p * kMlpIn + FPT * h);
#pragma unroll
      for (int c = 0; c < FPT / 4; ++c)
        xo[c] = make_float4(raw[4 * c], raw[4 * c + 1], raw[4 * c + 2], raw[4 * c + 3]);
    }
  } else {
#pragma unroll
    for (int t = 0; t < FPT; ++t) raw[t] = 0.0f;
  }
  if (kF) {
    float4* fo = reinterpret_cast<float4*>(F + r * kTrLdf + FPT * h);
#pragma unroll
    for (int c = 0; c < FPT / 4; ++c)
      fo[c] = make_float4(raw[4 * c], raw[4 * c + 1], raw[4 * c + 2], raw[4 * c + 3]);
  }
  uint2* dst = reinterpret_cast<uint2*>(&H[r * kMlpLd + FPT * h]);
#pragma unroll
  for (int c = 0; c < FPT / 4; ++c)
    dst[c] = make_uint2(to_bf16x2(raw[4 * c], raw[4 * c + 1]),
                        to_bf16x2(raw[4 * c + 2], raw[4 * c + 3]));
}

// One layer of the fused network kernels as the transposed product: wave w
// computes outputs [64 w, 64 w + 64) (weights as the A operand, fragments
// packed as by k_mlp_pack) for all RB x 16 rows of H (activations, k along
// the row, as the B operand), kbs k-blocks of 32 in increasing order.  Lane
// (li, lk) ends with row 16 i + li, outputs 64 w + 16 j + 4 lk .. + 3 in
// acc[i][j].
template <int RB>
__device__ __forceinline__ void mlp_layer_mfma(const v8s* __restrict__ W, const short* H, int kbs,
                                               int wave, int lane, v4f (&acc)[RB][4]) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  // weight fragments one k-block ahead of the products
  v8s bn[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) bn[j] = W[(wave * 4 + j) * kWave + lane];
  for (int kb = 0; kb < kbs; ++kb) {
    v8s b[4], x[RB];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = bn[j];
    if (kb + 1 < kbs) {
#pragma unroll
      for (int j = 0; j < 4; ++j) bn[j] = W[((kb + 1) * 16 + wave * 4 + j) * kWave + lane];
    }
#pragma unroll
    for (int i = 0; i < RB; ++i)
      x[i] = *reinterpret_cast<const v8s*>(&H[(16 * i + li) * kMlpLd + kb * 32 + 8 * lk]);
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = mfma_bf16_k32(b[j], x[i], acc[i][j]);
  }
}

// The training kernel's form of these products: eight waves, wave w
// computing outputs [32 w, 32 w + 32) (two 16-column fragments), with every
// weight fragment of the layer loaded up front (KBS k-blocks x 2 per lane),
// so that a layer's loads are in flight together and during the previous
// layer's epilogue.  Lane (li, lk) ends with row 16 i + li, outputs 32 w +
// 16 j + 4 lk .. + 3 in acc[i][j].
template <int KBS>
__device__ __forceinline__ void mlp_frags_load(const v8s* __restrict__ W, int wave, int lane,
                                               v8s (&w)[8][2]) {
#pragma unroll
  for (int kb = 0; kb < KBS; ++kb)
#pragma unroll
    for (int j = 0; j < 2; ++j) w[kb][j] = W[(kb * 16 + wave * 2 + j) * kWave + lane];
}

template <int RB, int KBS>
__device__ __forceinline__ void mlp_frags_mfma(const v8s (&w)[8][2], const short* H, int lane,
                                               v4f (&acc)[RB][2]) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < KBS; ++kb) {
    v8s x[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
      x[i] = *reinterpret_cast<const v8s*>(&H[(16 * i + li) * kMlpLd + kb * 32 + 8 * lk]);
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16_k32(w[kb][j], x[i], acc[i][j]);
  }
}

// Output layer (2 columns, padded to 16) of the fused network kernels: rows
// [rbase, rbase + 16 OB) of H against the packed W_3; lane (li, lk) ends with
// column li, rows rbase + 16 i + 4 lk .. + 3 in acc[i].
template <int OB>
__device__ __forceinline__ void mlp_out_mfma(const v8s* __restrict__ W, const short* H, int rbase,
                                             int lane, v4f (&acc)[OB]) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < OB; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int kb = 0; kb < kMlpHid / 32; ++kb) {
    const v8s b = W[kb * kWave + lane];
#pragma unroll
    for (int i = 0; i < OB; ++i) {
      const v8s x = *reinterpret_cast<const v8s*>(
          &H[(rbase + 16 * i + li) * kMlpLd + kb * 32 + 8 * lk]);
      acc[i] = mfma_bf16_k32(x, b, acc[i]);
    }
  }
}

// kAct (training forward): the FP32 standardised features and hidden
// activations are also written out (the backward's inputs), the same values
// that shape_pair_features and the per-layer products would have written.
// ROWS pairs per workgroup (128, or 64 for more workgroups and residency).
template <int ROWS, bool kAct>
__global__ __launch_bounds__(256, ROWS == 64 ? 4 : 2) void k_mlp_infer(MlpArgs a) {
  constexpr int RB = ROWS / 16;    // row blocks of 16 per wave in the hidden layers
  __shared__ __align__(16) short H[ROWS * kMlpLd];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = blockIdx.x * ROWS;
  mlp_stage_features<ROWS, kAct, false>(a, row0, H, nullptr);
  __syncthreads();
  // three hidden layers: wave w computes all ROWS rows x columns [64 w, 64 w + 64)
  // as the transposed product (weights as the A operand, activations as B),
  // so a lane's four results are four consecutive columns of one row: one
  // 8-byte LDS store each after bias, ReLU and a packed bf16 conversion
#pragma unroll 1
  for (int l = 0; l < 3; ++l) {
    const int kbs = (l == 0 ? kMlpIn : kMlpHid) / 32;
    v4f acc[RB][4];
    mlp_layer_mfma<RB>(a.W + mlp_pack_offset(l) / 8, H, kbs, wave, lane, acc);
    __syncthreads();  // every wave has read this layer's input
    const float* bias = a.b[l];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // lane (li, lk) holds row 16 i + li, columns col0 .. col0 + 3
      const int col0 = wave * 64 + 16 * j + 4 * lk;
      const float4 bc = make_float4(bias[col0], bias[col0 + 1], bias[col0 + 2], bias[col0 + 3]);
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        float v0 = acc[i][j][0] + bc.x, v1 = acc[i][j][1] + bc.y;
        float v2 = acc[i][j][2] + bc.z, v3 = acc[i][j][3] + bc.w;
        v0 = v0 > 0.f ? v0 : 0.f;
        v1 = v1 > 0.f ? v1 : 0.f;
        v2 = v2 > 0.f ? v2 : 0.f;
        v3 = v3 > 0.f ? v3 : 0.f;
        *reinterpret_cast<uint2*>(&H[(16 * i + li) * kMlpLd + col0]) =
            make_uint2(to_bf16x2(v0, v1), to_bf16x2(v2, v3));
        if (kAct && row0 + 16 * i + li < a.n)
          *reinterpret_cast<float4*>(a.h_out[l] + (size_t)(row0 + 16 * i + li) * kMlpHid +
                                     col0) = make_float4(v0, v1, v2, v3);
      }
    }
    __syncthreads();
  }
  // output layer: wave w computes rows [RPW w, RPW w + RPW), RPW = ROWS / 4
  {
    constexpr int RPW = ROWS / 4, OB = RPW / 16;
    v4f acc[OB];
    mlp_out_mfma<OB>(a.W + mlp_pack_offset(3) / 8, H, RPW * wave, lane, acc);
    if (li < kMlpOut) {
      const float bc = a.b[3][li];
#pragma unroll
      for (int i = 0; i < OB; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int p = row0 + RPW * wave + 16 * i + 4 * lk + r;
          if (p < a.n) a.out[(size_t)p * kMlpOut + li] = acc[i][r] + bc;
        }
    }
  }
}

// Seeded sample budgets of the refined pairs: the network's standardised
// log-scale output s (column 1 of raw row idx[i]) becomes
// sigma = exp(s y_std + y_mean), the per-sample SE scale of T, and the budget
// n = (sigma / tau)^2 is rounded up to whole rounds and kept within
// [round, cap] (NaN: cap).  FP64.
__global__ void k_seed_budget(const float* __restrict__ raw, int64_t ld,
                              const int* __restrict__ idx, int k, double y_mean, double y_std,
                              double tau, int round, int cap, int* __restrict__ n_start) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int r = idx ? idx[i] : i;
  const double s = (double)raw[(int64_t)r * ld + 1] * y_std + y_mean;
  const double n = exp(2.0 * s) / (tau * tau);
  double b = ceil(n / (double)round) * (double)round;
  if (!(b <= (double)cap)) b = (double)cap;  // also NaN
  if (b < (double)round) b = (double)round;
  n_start[i] = (int)b;
}

// Column sums of A[M][N] (row stride lda), deterministic: stage 1 sums
// chunks of kColRows rows per column (threads along columns, coalesced; many
// chunks so that a 4096-row batch fills the chip), stage 2 adds the chunk
// partials in order.
constexpr int kColRows = 32;

__global__ void k_colsum_partial(const float* __restrict__ A, int M, int N, int64_t lda,
                                 float* __restrict__ part) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  if (n >= N) return;
  const int m0 = chunk * kColRows, m1 = min(M, m0 + kColRows);
  float s = 0.f;
  for (int m = m0; m < m1; ++m) s += A[(int64_t)m * lda + n];
  part[(size_t)chunk * N + n] = s;
}

__global__ void k_colsum_final(const float* __restrict__ part, int chunks, int N,
                               float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  // chunk order; the loads of eight chunks are issued before their adds
  double s = 0.0;
  int c = 0;
  for (; c + 8 <= chunks; c += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(c + u) * N + n];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; c < chunks; ++c) s += part[(size_t)c * N + n];
  out[n] = (float)s;
}

// Column sums of up to kColSetMax matrices in one launch, each column with
// exactly the operations of k_colsum_partial + k_colsum_final: FP32 sums over
// chunks of kColRows rows, then the chunk sums added in order in FP64.  A
// workgroup takes 16 columns of one matrix; its 64 groups of 16 threads form
// 64 chunk sums at a time (a chunk's 32 loads issued together, the adds in
// row order), which the first group then adds in chunk order.
struct ColsumSet {
  int n;
  int M[kColSetMax], N[kColSetMax];
  int64_t lda[kColSetMax];
  const float* A[kColSetMax];
  float* out[kColSetMax];
  int blk0[kColSetMax + 1];  // first workgroup of each matrix
};

__global__ __launch_bounds__(1024) void k_colsum_set(ColsumSet s) {
  __shared__ float part[64][16];
  int t = 0;
  while (t + 1 < s.n && (int)blockIdx.x >= s.blk0[t + 1]) ++t;  // uniform
  const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int n = ((int)blockIdx.x - s.blk0[t]) * 16 + c;
  const int M = s.M[t], N = s.N[t];
  const int64_t lda = s.lda[t];
  const float* __restrict__ A = s.A[t];
  const int chunks = (M + kColRows - 1) / kColRows;
  double S = 0.0;
  for (int c0 = 0; c0 < chunks; c0 += 64) {
    const int ch = c0 + g;
    float v = 0.f;
    if (n < N && ch < chunks) {
      const int m0 = ch * kColRows;
      float x[kColRows];
#pragma unroll
      for (int r = 0; r < kColRows; ++r)
        x[r] = m0 + r < M ? A[(int64_t)(m0 + r) * lda + n] : 0.f;
#pragma unroll
      for (int r = 0; r < kColRows; ++r)
        if (m0 + r < M) v += x[r];
    }
    part[g][c] = v;
    __syncthreads();
    if (g == 0 && n < N) {
      const int u1 = min(64, chunks - c0);
      for (int u = 0; u < u1; ++u) S += part[u][c];
    }
    __syncthreads();
  }
  if (g == 0 && n < N) s.out[t][n] = (float)S;
}

// Weighted mean squared error over a batch: loss = sum_j w_j mean_b (y - t)^2,
// grad = 2 w_j (y - t) / B.  Loss partials per block, then one block sums them
// in order.  The two terms of one element, shared with the fused training
// step: e = y - t.
__device__ __forceinline__ float mse_grad(float w, float e, int B) { return 2.f * w * e / (float)B; }
__device__ __forceinline__ double mse_loss(float w, float e, int B) {
  return (double)w * (double)e * (double)e / (double)B;
}

__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y,
                                             const float* __restrict__ t,
                                             const float* __restrict__ w, int B, int N,
                                             float* __restrict__ grad,
                                             double* __restrict__ partial) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (i < (int64_t)B * N) {
    const int j = (int)(i % N);
    const float e = y[i] - t[i];
    grad[i] = mse_grad(w[j], e, B);
    l = mse_loss(w[j], e, B);
  }
  l = wave_sum(l);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = l;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum_partials(const double* __restrict__ partial, int n, float* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += partial[i];
  *out = (float)s;
}

// One Adam update at step t (bias-corrected moments); returns the new
// parameter and updates the moments.  Shared by k_adam and the fused
// training step.
__device__ __forceinline__ float adam_apply(float p, float g, float& m, float& v, int t, float lr,
                                            float b1, float b2, float eps) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  const float mi = fmaf(b1, m, (1.f - b1) * g);
  const float vi = fmaf(b2, v, (1.f - b2) * g * g);
  m = mi;
  v = vi;
  return p - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Adam on a flat FP32 vector; the step counter is read from device memory
// and advanced by k_step_bump after the update.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, const int* __restrict__ step, float lr,
                       float b1, float b2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = *step + 1;
  float mi = m[i], vi = v[i];
  p[i] = adam_apply(p[i], g[i], mi, vi, t, lr, b1, b2, eps);
  m[i] = mi;
  v[i] = vi;
}

__global__ void k_step_bump(int* step) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
}

// ---------------------------------------------------------------------------
// Fused training step of the 96-256-256-256-2 BF16 network: one minibatch's
// forward, weighted MSE, backward and Adam update in two launches, with the
// arithmetic of shape_mlp_forward, shape_mse, shape_mlp_backward (BF16) and
// shape_adam, so the same bits:
//
//   k_mlp_train, one workgroup per 32 rows: the forward of k_mlp_infer; the
//   MSE gradient and k_mse's per-wave loss sums; the input-gradient chain
//   g_2 = (g_3 W_3^T) . [h3 > 0], g_1, g_0 as transposed products on the
//   matrix cores (weights as the A operand, the previous gradient in LDS as
//   B, the ReLU gates kept as bits from the forward); the FP32 sums of every
//   gradient column over 32-row chunks (the first stage of the bias
//   gradients); and every layer's input and gradient as bf16 columns
//   (actT[l][feature][row], gT[l][unit][row]), the operands of the weight
//   gradients.
//
//   k_mlp_update, one workgroup per 32 x 32 tile of a weight matrix: the
//   weight gradient in shape_gemm_set's split-K chunks (each chunk one MFMA
//   accumulation over its k-blocks of 32 rows, the eight waves taking eight
//   chunks at a time), the chunks added in order in FP32; bias gradients as
//   the FP64 sums of the chunk sums in order; the loss; Adam; and the
//   updated weights packed to bf16 for the next step's forward and chain.
//
// Chain-packed weights: W_l (l = 1, 2, 3) as the A operand of the transposed
// product dz W_l^T: block (kb, mb) of 32 outputs x 16 inputs holds 64 lanes x
// 8 values, lane = 16 (o%32 / 8) + i%16, value o%8; W_3's two outputs are
// padded to 32 with zeros.  Stored after the forward packing.
// ---------------------------------------------------------------------------
constexpr int kTrRows = 32;   // minibatch rows per workgroup of k_mlp_train (32 or 64)

// Layout of the bf16 columns of a layer's inputs or gradients (width w, n
// rows): blocks of kColRows rows, each holding every feature's 32 rows
// contiguously, so 16 features of one k-block of 32 rows are 1 KB of
// consecutive bytes (one fragment load of the weight gradient).
__host__ __device__ constexpr size_t mlp_blk_index(int w, int f, int r) {
  return ((size_t)(r / kColRows) * w + f) * kColRows + r % kColRows;
}

__host__ __device__ constexpr int mlp_packT_offset(int layer) {
  // blocks of 32 x 16 per layer: W_3 1 x 16, W_2 8 x 16, W_1 8 x 16
  return kMlpPackElems + (layer == 3 ? 0 : layer == 2 ? 16 * 512 : (16 + 8 * 16) * 512);
}
constexpr int kMlpPackAllElems = kMlpPackElems + (16 + 2 * 8 * 16) * 512;
static_assert(kMlpPackAllElems * 2 == SHAPE_MLP_PACK_BYTES, "packed size");

__host__ __device__ constexpr int mlp_param_offset(int layer) {
  return layer == 0 ? 0
       : layer == 1 ? kMlpIn * kMlpHid + kMlpHid
       : layer == 2 ? kMlpIn * kMlpHid + kMlpHid + kMlpHid * kMlpHid + kMlpHid
                    : kMlpIn * kMlpHid + kMlpHid + 2 * (kMlpHid * kMlpHid + kMlpHid);
}

// Position of W_l[i][o] in the forward packing and in the chain packing.
__device__ __forceinline__ int mlp_pack_index(int l, int i, int o) {
  const int nbs = l == 3 ? 1 : kMlpHid / 16;
  return mlp_pack_offset(l) + ((i >> 5) * nbs + (o >> 4)) * 512 +
         (16 * ((i & 31) >> 3) + (o & 15)) * 8 + (i & 7);
}
__device__ __forceinline__ int mlp_packT_index(int l, int i, int o) {
  return mlp_packT_offset(l) + ((o >> 5) * 16 + (i >> 4)) * 512 +
         (16 * ((o & 31) >> 3) + (i & 15)) * 8 + (o & 7);
}

__global__ void k_mlp_pack_chain(const float* __restrict__ params, short* __restrict__ packed) {
  const int t = kMlpPackElems + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kMlpPackAllElems) return;
  const int layer = t < mlp_packT_offset(2) ? 3 : t < mlp_packT_offset(1) ? 2 : 1;
  const int local = t - mlp_packT_offset(layer);
  const int n_out = layer == 3 ? kMlpOut : kMlpHid;
  const int blk = local / 512, within = local % 512;
  const int kb = blk / 16, mb = blk % 16;
  const int lane = within / 8, e = within % 8;
  const int o = kb * 32 + 8 * (lane >> 4) + e;
  const int i = mb * 16 + (lane & 15);
  const float v = o < n_out ? params[mlp_param_offset(layer) + i * n_out + o] : 0.0f;
  packed[t] = to_bf16(v);
}

struct MlpTrainArgs {
  MlpArgs f;             // features, packed weights (both packings), biases, n = batch rows
  const float* target;   // [n][2]
  const float* lw;       // [2] loss weights
  int* step;
  short* actT[4];        // x, h1, h2, h3 by column, blocked (mlp_blk_index), bf16
  short* gT[4];          // g_0 .. g_3 by column, blocked, bf16
  float* bsum[4];        // [n / 32][width_{l+1}]: FP32 sums of g_l over 32-row chunks
  double* loss_part;     // [n / 32]: loss sums of k_mse's waves
};

__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) { return to_bf16x2(lo, hi); }

// Column c, rows [32 h, 32 h + 32) (one chunk of kColRows rows) of the FP32
// staging to bf16 at dst (column-major, rows contiguous, 16-byte stores) and,
// if bs, the FP32 sum of the chunk in row order from 0.f (k_colsum_set's
// first stage).
__device__ __forceinline__ void mlp_column_out(const float* F, int c, int h, short* dst,
                                               float* bs) {
  const float* f = F + kColRows * h * kTrLdf + c;
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < kColRows / 8; ++q) {
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = f[(8 * q + e) * kTrLdf];
    if (bs) {
#pragma unroll
      for (int e = 0; e < 8; ++e) s += v[e];
    }
    *reinterpret_cast<uint4*>(dst + 8 * q) = make_uint4(
        to_bf16x2(v[0], v[1]), to_bf16x2(v[2], v[3]), to_bf16x2(v[4], v[5]), to_bf16x2(v[6], v[7]));
  }
  if (bs) *bs = s;
}

constexpr int kTrThreads = 512;   // eight waves: 32 output columns each

// Hidden-layer epilogue of the training forward (k_mlp_infer's arithmetic):
// bias (bc, per fragment), ReLU, bf16 into H for the next layer, FP32 into F
// for the column pass; returns the ReLU gates as bits 16 j + 4 i + r.
template <int RB>
__device__ __forceinline__ uint32_t train_hidden_out(const v4f (&acc)[RB][2], const float4 (&bc)[2],
                                                     short* H, float* F, int wave, int lane) {
  const int li = lane & 15, lk = lane >> 4;
  uint32_t gb = 0;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col0 = wave * 32 + 16 * j + 4 * lk;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      float v0 = acc[i][j][0] + bc[j].x, v1 = acc[i][j][1] + bc[j].y;
      float v2 = acc[i][j][2] + bc[j].z, v3 = acc[i][j][3] + bc[j].w;
      const int bit = 16 * j + 4 * i;
      gb |= (uint32_t)(v0 > 0.f) << bit | (uint32_t)(v1 > 0.f) << (bit + 1) |
            (uint32_t)(v2 > 0.f) << (bit + 2) | (uint32_t)(v3 > 0.f) << (bit + 3);
      v0 = v0 > 0.f ? v0 : 0.f;
      v1 = v1 > 0.f ? v1 : 0.f;
      v2 = v2 > 0.f ? v2 : 0.f;
      v3 = v3 > 0.f ? v3 : 0.f;
      *reinterpret_cast<uint2*>(&H[(16 * i + li) * kMlpLd + col0]) =
          make_uint2(to_bf16x2(v0, v1), to_bf16x2(v2, v3));
      *reinterpret_cast<float4*>(&F[(16 * i + li) * kTrLdf + col0]) = make_float4(v0, v1, v2, v3);
    }
  }
  return gb;
}

// x where gate bit `bit` is set, else +0 (shape_gemm's gate): the bit as an
// all-ones or all-zeros mask on the float's bits.
__device__ __forceinline__ float gate_bit(float x, uint32_t gb, int bit) {
  const uint32_t mk = (uint32_t)((int32_t)(gb << (31 - bit)) >> 31);
  return __uint_as_float(__float_as_uint(x) & mk);
}

// Chain epilogue: the product zeroed where the gate is off, FP32 into F and,
// when another product follows, bf16 into H.
template <int RB>
__device__ __forceinline__ void train_chain_out(const v4f (&acc)[RB][2], uint32_t gb, bool to_h,
                                                short* H, float* F, int wave, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col0 = wave * 32 + 16 * j + 4 * lk;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int bit = 16 * j + 4 * i;
      const float v0 = gate_bit(acc[i][j][0], gb, bit), v1 = gate_bit(acc[i][j][1], gb, bit + 1);
      const float v2 = gate_bit(acc[i][j][2], gb, bit + 2), v3 = gate_bit(acc[i][j][3], gb, bit + 3);
      if (to_h)
        *reinterpret_cast<uint2*>(&H[(16 * i + li) * kMlpLd + col0]) =
            make_uint2(to_bf16x2(v0, v1), to_bf16x2(v2, v3));
      *reinterpret_cast<float4*>(&F[(16 * i + li) * kTrLdf + col0]) = make_float4(v0, v1, v2, v3);
    }
  }
}

__device__ __forceinline__ void load_bias(const float* __restrict__ b, int wave, int lane,
                                          float4 (&bc)[2]) {
  const int lk = lane >> 4;
#pragma unroll
  for (int j = 0; j < 2; ++j)
    bc[j] = *reinterpret_cast<const float4*>(b + wave * 32 + 16 * j + 4 * lk);
}

template <int ROWS>
__global__ __launch_bounds__(kTrThreads, 1) void k_mlp_train(MlpTrainArgs a) {
  constexpr int RB = ROWS / 16;                // row blocks of 16
  constexpr int kHalves = ROWS / kColRows;     // 32-row chunks
  constexpr int kStage = (ROWS >= 64 ? 256 / ROWS : 4) * ROWS;  // feature-staging threads
  __shared__ __align__(16) short H[ROWS * kMlpLd];
  __shared__ __align__(16) float F[ROWS * kTrLdf];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int li = lane & 15, lk = lane >> 4;
  const int row0 = blockIdx.x * ROWS;
  const int n = a.f.n;
  // column pass: thread (col, half) takes rows [32 half, 32 half + 32) of one column
  const int col = tid & (kMlpHid - 1), half = tid / kMlpHid;
  const bool col_pass = half < kHalves;
  const v8s* __restrict__ W = a.f.W;
  // the step number the update kernel's Adam uses (nothing else reads it here)
  if (blockIdx.x == 0 && tid == 0) *a.step += 1;
  // each layer's weight fragments (and biases) are requested before the
  // previous layer's epilogue, the first layer's before the feature gather
  v8s w[8][2];
  float4 bc[2];
  mlp_frags_load<kMlpIn / 32>(W + mlp_pack_offset(0) / 8, wave, lane, w);
  load_bias(a.f.b[0], wave, lane, bc);
  if (tid < kStage) mlp_stage_features<ROWS, false, true>(a.f, row0, H, F);
  __syncthreads();
  if (col_pass && col < kMlpIn)
    mlp_column_out(F, col, half, a.actT[0] + mlp_blk_index(kMlpIn, col, row0 + kColRows * half),
                   nullptr);
  // forward: hidden layers as in k_mlp_infer; the ReLU gates as bits of
  // gate[l], the activations by column for the update
  uint32_t gate[3];
  v4f acc[RB][2];
  mlp_frags_mfma<RB, kMlpIn / 32>(w, H, lane, acc);
  mlp_frags_load<8>(W + mlp_pack_offset(1) / 8, wave, lane, w);
  __syncthreads();  // H read by every wave, F by every column pass
  gate[0] = train_hidden_out<RB>(acc, bc, H, F, wave, lane);
  load_bias(a.f.b[1], wave, lane, bc);
  __syncthreads();
  if (col_pass)
    mlp_column_out(F, col, half, a.actT[1] + mlp_blk_index(kMlpHid, col, row0 + kColRows * half),
                 nullptr);
  mlp_frags_mfma<RB, 8>(w, H, lane, acc);
  mlp_frags_load<8>(W + mlp_pack_offset(2) / 8, wave, lane, w);
  __syncthreads();
  gate[1] = train_hidden_out<RB>(acc, bc, H, F, wave, lane);
  load_bias(a.f.b[2], wave, lane, bc);
  __syncthreads();
  if (col_pass)
    mlp_column_out(F, col, half, a.actT[2] + mlp_blk_index(kMlpHid, col, row0 + kColRows * half),
                 nullptr);
  mlp_frags_mfma<RB, 8>(w, H, lane, acc);
  // output layer fragments (one wave per block of 16 rows)
  v8s wo[8];
  if (wave < RB) {
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) wo[kb] = W[mlp_pack_offset(3) / 8 + kb * kWave + lane];
  }
  __syncthreads();
  gate[2] = train_hidden_out<RB>(acc, bc, H, F, wave, lane);
  __syncthreads();
  if (col_pass)
    mlp_column_out(F, col, half, a.actT[3] + mlp_blk_index(kMlpHid, col, row0 + kColRows * half),
                 nullptr);
  // output layer (mlp_out_mfma's products), then dloss/dy = g_3 and the loss
  // terms (e = y - t)
  {
    v4f ao = v4f{0.f, 0.f, 0.f, 0.f};
    float tg[4] = {0.f, 0.f, 0.f, 0.f};
    if (wave < RB) {
      if (li < kMlpOut) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          tg[r] = a.target[(size_t)(row0 + 16 * wave + 4 * lk + r) * kMlpOut + li];
      }
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        const v8s x = *reinterpret_cast<const v8s*>(
            &H[(16 * wave + li) * kMlpLd + kb * 32 + 8 * lk]);
        ao = mfma_bf16_k32(x, wo[kb], ao);
      }
    }
    mlp_frags_load<1>(W + mlp_packT_offset(3) / 8, wave, lane, w);
    __syncthreads();  // H and F free
    if (wave < RB && li < kMlpOut) {
      const float b3 = a.f.b[3][li];
      const float wl = a.lw[li];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * wave + 4 * lk + r;
        const float e = (ao[r] + b3) - tg[r];
        F[row * kTrLdf + li] = mse_grad(wl, e, n);
        F[row * kTrLdf + kMlpOut + li] = e;
      }
    }
    __syncthreads();
    if (tid < 4 * ROWS) {  // g_3 as the chain's B operand: one k-block, zero past 2 outputs
      const int row = tid >> 2, q = tid & 3;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (q == 0) v.x = to_bf16x2(F[row * kTrLdf], F[row * kTrLdf + 1]);
      *reinterpret_cast<uint4*>(&H[row * kMlpLd + 8 * q]) = v;
    }
    if (tid < 2 * ROWS) {
      // k_mse's loss sums: its wave covers 32 rows, lane 2 (row % 32) + j
      const int row = tid >> 1, j = tid & 1;
      double l = mse_loss(a.lw[j], F[row * kTrLdf + kMlpOut + j], n);
      l = wave_sum(l);
      if (lane == 0) a.loss_part[row0 / kColRows + wave] = l;
    } else if (tid >= 256 && tid < 256 + 2 * kHalves) {
      const int j = tid & 1, h = (tid - 256) >> 1;
      mlp_column_out(F, j, h, a.gT[3] + mlp_blk_index(kMlpOut, j, row0 + kColRows * h),
                     a.bsum[3] + (row0 / kColRows + h) * kMlpOut + j);
    }
    __syncthreads();
  }
  // chain: g_{l-1} = (g_l W_l^T) zeroed where h_l <= 0, l = 3, 2, 1
  mlp_frags_mfma<RB, 1>(w, H, lane, acc);
  mlp_frags_load<8>(W + mlp_packT_offset(2) / 8, wave, lane, w);
  __syncthreads();
  train_chain_out<RB>(acc, gate[2], true, H, F, wave, lane);
  __syncthreads();
  if (col_pass)
    mlp_column_out(F, col, half, a.gT[2] + mlp_blk_index(kMlpHid, col, row0 + kColRows * half),
                 a.bsum[2] + (size_t)(row0 / kColRows + half) * kMlpHid + col);
  mlp_frags_mfma<RB, 8>(w, H, lane, acc);
  mlp_frags_load<8>(W + mlp_packT_offset(1) / 8, wave, lane, w);
  __syncthreads();
  train_chain_out<RB>(acc, gate[1], true, H, F, wave, lane);
  __syncthreads();
  if (col_pass)
    mlp_column_out(F, col, half, a.gT[1] + mlp_blk_index(kMlpHid, col, row0 + kColRows * half),
                 a.bsum[1] + (size_t)(row0 / kColRows + half) * kMlpHid + col);
  mlp_frags_mfma<RB, 8>(w, H, lane, acc);
  __syncthreads();
  train_chain_out<RB>(acc, gate[0], false, H, F, wave, lane);
  __syncthreads();
  if (col_pass)
    mlp_column_out(F, col, half, a.gT[0] + mlp_blk_index(kMlpHid, col, row0 + kColRows * half),
                 a.bsum[0] + (size_t)(row0 / kColRows + half) * kMlpHid + col);
}

constexpr int kUpdTile = 32, kUpdLd = kUpdTile + 1;
constexpr int kUpdThreads = kUpdTile * kUpdTile;  // one output element per thread
constexpr int kUpdWaves = kUpdThreads / kWave;    // 16
constexpr int kUpdZ = 32;                          // chunk partials held in LDS at once
constexpr int kUpdKb = 4;                          // k-blocks loaded together
constexpr int kUpdChunks = 256;                    // bias chunk sums staged per pass
constexpr int kUpdBlocks = 192;                    // workgroups of k_mlp_update
// work codes of the workgroups: kind << 24 | layer << 16 | output tile << 8 |
// input tile; kind 0 = weight tile, 1 = bias tile, 2 = loss, -1 = none
constexpr int kUpdWeight = 0, kUpdBias = 1, kUpdLoss = 2;

struct MlpUpdateArgs {
  const short* actT[4];
  const short* gT[4];
  const float* bsum[4];
  const double* loss_part;
  int n;                  // batch rows
  int kc[4], splits[4];   // weight gradients: rows per split-K chunk, chunks
  int work[kUpdBlocks];   // work code of each workgroup
  float* params;
  float* m;
  float* v;
  const int* step;
  float lr, b1, b2, eps;
  float* grad;            // or NULL
  short* packed;          // forward and chain packings, rewritten
  float* loss;
};

// One 32 x 32 tile (outputs o0.., inputs i0..) of W_l: its gradient in
// shape_gemm_set's split-K chunks (each chunk from zero over its k-blocks in
// order, wave w taking chunks w, w + 16, ...; the partials of up to kUpdZ
// chunks in LDS, then added in chunk order from 0.f by the thread that owns
// the element; one chunk: the accumulation itself), then Adam and the two
// bf16 packings of the new weight.
__device__ __forceinline__ void upd_weights(const MlpUpdateArgs& a, int l, int o0, int i0,
                                            float (*P)[kUpdTile * kUpdLd]) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int li = lane & 15, lk = lane >> 4;
  const int n_in = l == 0 ? kMlpIn : kMlpHid, n_out = l == 3 ? kMlpOut : kMlpHid;
  const int n = a.n, kc = a.kc[l], splits = a.splits[l];
  const int el_i = tid / kUpdTile, el_o = tid % kUpdTile;
  // this thread's parameter and Adam moments, requested before the products
  const bool own = i0 + el_i < n_in && o0 + el_o < n_out;
  const int pw = mlp_param_offset(l) + (i0 + el_i) * n_out + o0 + el_o;
  float p_w = 0.f, m_w = 0.f, v_w = 0.f;
  if (own) {
    p_w = a.params[pw];
    m_w = a.m[pw];
    v_w = a.v[pw];
  }
  // fragment rows of this lane: A = g^T (m = output o), B = act^T (n = input
  // i); rows past the matrix read as zeros.  One k-block of every feature is
  // one block of the blocked layout: the next k-block lies w * 32 further.
  const short* ga[2];
  const short* gb[2];
  bool va[2], vb[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int o = o0 + 16 * t + li, i = i0 + 16 * t + li;
    va[t] = o < n_out;
    vb[t] = i < n_in;
    ga[t] = a.gT[l] + mlp_blk_index(n_out, va[t] ? o : 0, 8 * lk);
    gb[t] = a.actT[l] + mlp_blk_index(n_in, vb[t] ? i : 0, 8 * lk);
  }
  const size_t sa = (size_t)n_out * kColRows, sb = (size_t)n_in * kColRows;
  const v8s zero = v8s{0, 0, 0, 0, 0, 0, 0, 0};
  float g = 0.f;
  for (int z0 = 0; z0 < splits; z0 += kUpdZ) {
    for (int z = z0 + wave; z < min(splits, z0 + kUpdZ); z += kUpdWaves) {
      v4f acc[2][2];
#pragma unroll
      for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) acc[ob][ib] = v4f{0.f, 0.f, 0.f, 0.f};
      const int k1 = min(n, (z + 1) * kc);
      for (int k = z * kc; k < k1; k += 32 * kUpdKb) {
        const int nkb = min(kUpdKb, (k1 - k) / 32);
        v8s fa[kUpdKb][2], fb[kUpdKb][2];
#pragma unroll
        for (int q = 0; q < kUpdKb; ++q)
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const bool in = q < nkb;
            const size_t kb = (size_t)(k / kColRows + q);
            fa[q][t] = va[t] && in ? *reinterpret_cast<const v8s*>(ga[t] + kb * sa) : zero;
            fb[q][t] = vb[t] && in ? *reinterpret_cast<const v8s*>(gb[t] + kb * sb) : zero;
          }
#pragma unroll
        for (int q = 0; q < kUpdKb; ++q)
          if (q < nkb)
#pragma unroll
            for (int ob = 0; ob < 2; ++ob)
#pragma unroll
              for (int ib = 0; ib < 2; ++ib)
                acc[ob][ib] = mfma_bf16_k32(fa[q][ob], fb[q][ib], acc[ob][ib]);
      }
      // lane (li, lk): o = 16 ob + 4 lk + r, i = 16 ib + li of the tile
#pragma unroll
      for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            P[z - z0][(16 * ib + li) * kUpdLd + 16 * ob + 4 * lk + r] = acc[ob][ib][r];
    }
    __syncthreads();
    const int nz = min(kUpdZ, splits - z0), pi = el_i * kUpdLd + el_o;
    if (splits == 1) {
      g = P[0][pi];
    } else {
      // in order; the reads of eight partials issued before their adds
      int q0 = 0;
      for (; q0 + 8 <= nz; q0 += 8) {
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = P[q0 + q][pi];
#pragma unroll
        for (int q = 0; q < 8; ++q) g += v[q];
      }
      for (; q0 < nz; ++q0) g += P[q0][pi];
    }
    __syncthreads();
  }
  if (own) {
    if (a.grad) a.grad[pw] = g;
    const float p = adam_apply(p_w, g, m_w, v_w, *a.step, a.lr, a.b1, a.b2, a.eps);
    a.params[pw] = p;
    a.m[pw] = m_w;
    a.v[pw] = v_w;
    const short pb = to_bf16(p);
    const int i = i0 + el_i, o = o0 + el_o;
    a.packed[mlp_pack_index(l, i, o)] = pb;
    if (l > 0) a.packed[mlp_packT_index(l, i, o)] = pb;
  }
}

// Bias gradients of outputs o0 .. o0 + 31 of layer l: the FP64 sums of the
// 32-row chunk sums in chunk order (k_colsum_set's second stage), then Adam.
// The chunk sums are staged in LDS by all threads; a wave of 32 lanes adds.
__device__ __forceinline__ void upd_bias(const MlpUpdateArgs& a, int l, int o0, float* BS) {
  const int tid = threadIdx.x;
  const int n_in = l == 0 ? kMlpIn : kMlpHid, n_out = l == 3 ? kMlpOut : kMlpHid;
  const int chunks = a.n / kColRows;
  const int o = o0 + tid;
  const bool own = tid < kUpdTile && o < n_out;
  const int pb = mlp_param_offset(l) + n_in * n_out + o;
  float p_b = 0.f, m_b = 0.f, v_b = 0.f;
  if (own) {
    p_b = a.params[pb];
    m_b = a.m[pb];
    v_b = a.v[pb];
  }
  double S = 0.0;
  for (int c0 = 0; c0 < chunks; c0 += kUpdChunks) {
    const int nc = min(kUpdChunks, chunks - c0);
    for (int x = tid; x < nc * kUpdTile; x += kUpdThreads) {
      const int c = x / kUpdTile, oc = o0 + x % kUpdTile;
      BS[x] = oc < n_out ? a.bsum[l][(size_t)(c0 + c) * n_out + oc] : 0.f;
    }
    __syncthreads();
    if (tid < kUpdTile) {
      int c = 0;
      for (; c + 8 <= nc; c += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = BS[(c + u) * kUpdTile + tid];
#pragma unroll
        for (int u = 0; u < 8; ++u) S += v[u];
      }
      for (; c < nc; ++c) S += BS[c * kUpdTile + tid];
    }
    __syncthreads();
  }
  if (own) {
    const float gbias = (float)S;
    if (a.grad) a.grad[pb] = gbias;
    a.params[pb] = adam_apply(p_b, gbias, m_b, v_b, *a.step, a.lr, a.b1, a.b2, a.eps);
    a.m[pb] = m_b;
    a.v[pb] = v_b;
  }
}

// The minibatch loss: k_mse's block sums (its four waves of 32 rows, a
// missing wave 0) added in block order, as k_sum_partials.
__device__ __forceinline__ void upd_loss(const MlpUpdateArgs& a, double* LP) {
  const int tid = threadIdx.x;
  const int waves = a.n / kColRows, blocks = (waves + 3) / 4;
  double s = 0.0;
  for (int b0 = 0; b0 < blocks; b0 += kUpdThreads) {
    const int nb = min(kUpdThreads, blocks - b0);
    if (tid < nb) {
      double r[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int w = 4 * (b0 + tid) + q;
        r[q] = w < waves ? a.loss_part[w] : 0.0;
      }
      LP[tid] = r[0] + r[1] + r[2] + r[3];
    }
    __syncthreads();
    if (tid == 0) {
      int b = 0;
      for (; b + 8 <= nb; b += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = LP[b + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
      for (; b < nb; ++b) s += LP[b];
    }
    __syncthreads();
  }
  if (tid == 0) *a.loss = (float)s;
}

__global__ __launch_bounds__(kUpdThreads) void k_mlp_update(MlpUpdateArgs a) {
  __shared__ float P[kUpdZ][kUpdTile * kUpdLd];
  const int code = a.work[blockIdx.x];
  if (code < 0) return;
  const int kind = code >> 24, l = (code >> 16) & 0xFF;
  const int o0 = ((code >> 8) & 0xFF) * kUpdTile, i0 = (code & 0xFF) * kUpdTile;
  if (kind == kUpdWeight)
    upd_weights(a, l, o0, i0, P);
  else if (kind == kUpdBias)
    upd_bias(a, l, o0, &P[0][0]);
  else
    upd_loss(a, reinterpret_cast<double*>(&P[0][0]));
}

// ---------------------------------------------------------------------------
// Top-k (largest scores, ties to the lower index) by radix selection on the
// order-preserving 32-bit image of the scores (NaN ranks lowest), then an
// index-ordered compaction.  State in device memory:
//   sel[0] = key prefix found so far, sel[1] = still needed from the prefix,
//   sel[2] = number strictly above the final key.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t order_key(float x) {
  if (x != x) return 0u;
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(256) void k_radix_hist(const float* __restrict__ s, int n,
                                                    const uint32_t* __restrict__ sel, int shift,
                                                    uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t prefix = sel[0];
  const uint32_t pmask = shift >= 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = order_key(s[i]);
    if ((k & pmask) == (prefix & pmask)) atomicAdd(&h[(k >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// sel = {prefix 0, need k, above 0}; the histogram cleared (256 threads).
__global__ __launch_bounds__(256) void k_topk_init(uint32_t* __restrict__ hist,
                                                   uint32_t* __restrict__ sel, int k) {
  hist[threadIdx.x] = 0u;
  if (threadIdx.x < 3) sel[threadIdx.x] = threadIdx.x == 1 ? (uint32_t)k : 0u;
}

// One thread per bin (256): this digit of the k-th largest key is the
// largest bin b >= 1 whose count with all bins above it reaches the number
// still needed (bin 0 if there is none); the histogram is cleared for the
// next pass.
__global__ __launch_bounds__(256) void k_radix_pick(uint32_t* __restrict__ hist,
                                                    uint32_t* __restrict__ sel, int shift) {
  __shared__ uint32_t suf[257];
  const int t = threadIdx.x;
  const uint32_t need = sel[1];
  const uint32_t h = hist[t];
  suf[t] = h;
  if (t == 0) suf[256] = 0u;
  __syncthreads();
  // suf[b] = sum of the bins >= b (Hillis-Steele, towards lower bins)
  for (int d = 1; d < 256; d <<= 1) {
    const uint32_t add = t + d < 256 ? suf[t + d] : 0u;
    __syncthreads();
    suf[t] += add;
    __syncthreads();
  }
  if ((t == 0 || suf[t] >= need) && suf[t + 1] < need) {
    const uint32_t above = suf[t + 1];
    sel[0] |= (uint32_t)t << shift;
    sel[1] = need - above;
    sel[2] += above;
  }
  hist[t] = 0u;
}

// Per-block counts of selected elements (key > K, or key == K).
__global__ __launch_bounds__(256) void k_select_count(const float* __restrict__ s, int n,
                                                      const uint32_t* __restrict__ sel,
                                                      int* __restrict__ cnt_gt,
                                                      int* __restrict__ cnt_eq) {
  __shared__ int red[2][4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t K = sel[0];
  int gt = 0, eq = 0;
  if (i < n) {
    const uint32_t k = order_key(s[i]);
    gt = k > K;
    eq = k == K;
  }
  const int g = __popcll(__ballot(gt)), e = __popcll(__ballot(eq));
  if ((threadIdx.x & (kWave - 1)) == 0) {
    red[0][threadIdx.x / kWave] = g;
    red[1][threadIdx.x / kWave] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    cnt_gt[blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    cnt_eq[blockIdx.x] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// Exclusive scans of the block counts in one workgroup of 1024 threads (each
// thread owns a contiguous run of blocks; Hillis-Steele scan of the run
// totals in LDS).  Equal keys are admitted in index order up to the number
// still needed: with G, E the counts above and equal before block b,
// block b writes from G + min(E, need) and admits min(e_b, need - E) equal
// keys (at least 0).
constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void k_select_scan(int* __restrict__ cnt_gt,
                                                              int* __restrict__ cnt_eq,
                                                              int nblk,
                                                              const uint32_t* __restrict__ sel) {
  __shared__ int sg[kScanThreads], se[kScanThreads];
  const int t = threadIdx.x;
  const int per = (nblk + kScanThreads - 1) / kScanThreads;
  const int b0 = t * per, b1 = min(nblk, b0 + per);
  int g = 0, e = 0;
  for (int b = b0; b < b1; ++b) {
    g += cnt_gt[b];
    e += cnt_eq[b];
  }
  sg[t] = g;
  se[t] = e;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const int vg = t >= d ? sg[t - d] : 0, ve = t >= d ? se[t - d] : 0;
    __syncthreads();
    sg[t] += vg;
    se[t] += ve;
    __syncthreads();
  }
  const int need = (int)sel[1];
  int G = sg[t] - g, E = se[t] - e;  // exclusive prefixes of this thread's run
  for (int b = b0; b < b1; ++b) {
    const int gb = cnt_gt[b], eb = cnt_eq[b];
    const int left = need - E;
    const int take = left <= 0 ? 0 : (eb < left ? eb : left);
    cnt_gt[b] = G + (E < need ? E : need);  // output offset of the block
    cnt_eq[b] = take;                       // equal keys the block may emit
    G += gb;
    E += eb;
  }
}

__global__ __launch_bounds__(256) void k_select_write(const float* __restrict__ s, int n,
                                                      const uint32_t* __restrict__ sel,
                                                      const int* __restrict__ offs,
                                                      const int* __restrict__ take_eq,
                                                      int* __restrict__ out) {
  __shared__ int wgt[4], weq[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t K = sel[0];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  int gt = 0, eq = 0;
  if (i < n) {
    const uint32_t k = order_key(s[i]);
    gt = k > K;
    eq = k == K;
  }
  const uint64_t bg = __ballot(gt), be = __ballot(eq);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  if (lane == 0) {
    wgt[wave] = __popcll(bg);
    weq[wave] = __popcll(be);
  }
  __syncthreads();
  int og = 0, oe = 0;
  for (int w = 0; w < wave; ++w) {
    og += wgt[w];
    oe += weq[w];
  }
  const int eq_rank = oe + __popcll(be & below);
  const int gt_rank = og + __popcll(bg & below);
  // the block's output: gt and admitted eq elements interleaved in index order
  const int admitted_before = eq_rank < take_eq[blockIdx.x] ? eq_rank : take_eq[blockIdx.x];
  if (gt || (eq && eq_rank < take_eq[blockIdx.x])) out[offs[blockIdx.x] + gt_rank + admitted_before] = (int)i;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_features(const MolsDev& M, int* flag, float* out, float* mom,
                           hipStream_t st, const int* order) {
  if (M.n_mols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((M.n_mols + kFeatRows - 1) / kFeatRows)),
                     dim3(kWave), (size_t)kFeatRows * M.max_atoms * sizeof(float4), st, M,
                     order, flag, out, mom);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_features_eigen, dim3((unsigned)((M.n_mols + 255) / 256)), dim3(256), 0,
                     st, M.n_mols, mom, out);
  return hipGetLastError();
}

hipError_t launch_pair_features(const float* fq, const float* flib, const int* qidx,
                                const int* idx, int n, const float* fo_cross, const float* mean,
                                const float* inv_std, float* out, hipStream_t st) {
  const int64_t tot = (int64_t)n * 96;
  hipLaunchKernelGGL(k_pair_features, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, fq,
                     flib, qidx, idx, n, fo_cross, mean, inv_std, out);
  return hipGetLastError();
}

template <int NI, int CH>
static hipError_t launch_fo_cross_t(const MolsDev& Q, const MolsDev& L, const int* pairs,
                                    int n_pairs, int n_cu, int* flag, float* out,
                                    hipStream_t st) {
  constexpr int kPad = (kWave / NI) * 2;
  const int max_b_pad = (L.max_atoms + kPad - 1) / kPad * kPad;
  const dim3 block(kWave * kFoWaves);
  const size_t lds = (size_t)Q.max_atoms * (sizeof(float4) + sizeof(float2)) +
                     (size_t)kFoWaves * max_b_pad * 2 * sizeof(float4);
  // eight waves per SIMD over the chip, each with a contiguous run of pairs
  const int64_t waves_wanted = (int64_t)(n_cu > 0 ? n_cu : 256) * 32;
  const int per_wave = (int)((n_pairs + waves_wanted - 1) / waves_wanted);
  const int64_t waves = (n_pairs + per_wave - 1) / per_wave;
  const dim3 grid((unsigned)((waves + kFoWaves - 1) / kFoWaves));
  hipLaunchKernelGGL((k_fo_cross<NI, CH>), grid, block, lds, st, Q, L, pairs, n_pairs, per_wave,
                     flag, out);
  return hipGetLastError();
}

hipError_t launch_fo_cross(const MolsDev& Q, const MolsDev& L, const int* pairs, int n_pairs,
                           int n_cu, int* flag, float* out, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  // query slots: 16 (4 phases) up to 16 query atoms, 32 (2 phases) up to 32,
  // 64 beyond (blocks of 64); one chunk of library atoms per lane up to 64
  const bool one = L.max_atoms <= kWave;
  if (Q.max_atoms <= 16)
    return one ? launch_fo_cross_t<16, 1>(Q, L, pairs, n_pairs, n_cu, flag, out, st)
               : launch_fo_cross_t<16, kFoChunks>(Q, L, pairs, n_pairs, n_cu, flag, out, st);
  if (Q.max_atoms <= 32)
    return one ? launch_fo_cross_t<32, 1>(Q, L, pairs, n_pairs, n_cu, flag, out, st)
               : launch_fo_cross_t<32, kFoChunks>(Q, L, pairs, n_pairs, n_cu, flag, out, st);
  return one ? launch_fo_cross_t<64, 1>(Q, L, pairs, n_pairs, n_cu, flag, out, st)
             : launch_fo_cross_t<64, kFoChunks>(Q, L, pairs, n_pairs, n_cu, flag, out, st);
}

// Workgroup tile of launch_gemm: BF16 products use the LDS-tiled kernel,
// with 128 x 128 tiles when those give at least one workgroup per CU (256)
// and 64 x 64 tiles otherwise; FP32 products use the 64 x 64 kernel without
// LDS.
static bool gemm_tiled(const GemmArgs& g) { return (g.flags & SHAPE_GEMM_BF16) != 0; }

static int gemm_tile(const GemmArgs& g) {
  if (!gemm_tiled(g)) return 64;
  const int64_t big = (int64_t)((g.N + 127) / 128) * ((g.M + 127) / 128);
  return big >= 256 ? 128 : 64;
}

static dim3 gemm_grid(const GemmArgs& g) {
  const int t = gemm_tile(g);
  return dim3((unsigned)((g.N + t - 1) / t), (unsigned)((g.M + t - 1) / t));
}

// Products whose output tiles cannot fill the chip (the weight gradients:
// M x N = layer size, K = batch) split K so that >= 512 workgroups run,
// each over at least 128 values of k.
int gemm_splits(const GemmArgs& g) {
  const dim3 grid = gemm_grid(g);
  const int tiles = (int)(grid.x * grid.y);
  if (tiles >= 128 || g.K < 512) return 1;
  int s = (512 + tiles - 1) / tiles;
  const int by_k = g.K / 128;
  return s < by_k ? s : by_k;
}

hipError_t launch_gemm(const GemmArgs& g0, hipStream_t st) {
  GemmArgs g = g0;
  const bool tiled = gemm_tiled(g);
  const int tile = gemm_tile(g);
  dim3 grid = gemm_grid(g);
  int splits = g.part ? gemm_splits(g) : 1;
  if (splits > 1) {
    g.k_chunk = ((g.K + splits - 1) / splits + kTK - 1) / kTK * kTK;
    splits = (g.K + g.k_chunk - 1) / g.k_chunk;
    grid.z = (unsigned)splits;
  } else {
    g.part = nullptr;
    g.k_chunk = 0;
  }
  if (tiled && tile == 128) {
    hipLaunchKernelGGL((k_gemm_bf16_tiled<128, 128>), grid, dim3(256), 0, st, g);
  } else if (tiled) {
    hipLaunchKernelGGL((k_gemm_bf16_tiled<64, 64>), grid, dim3(256), 0, st, g);
  } else {
    hipLaunchKernelGGL(k_gemm_f32, grid, dim3(256), 0, st, g);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits <= 1) return e;
  const int64_t tot = (int64_t)g.M * g.N;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, g,
                     splits);
  return hipGetLastError();
}

bool gemm_set_fits(const GemmArgs& g) { return gemm_tiled(g) && gemm_tile(g) == 64; }

int64_t gemm_set_blocks(const GemmArgs& g) {
  const dim3 grid = gemm_grid(g);
  return (int64_t)grid.x * grid.y * gemm_splits(g);
}

size_t gemm_set_part_elems(const GemmArgs& g) {
  const int splits = gemm_splits(g);
  return splits > 1 ? (size_t)splits * g.M * g.N : 0;
}

hipError_t launch_gemm_set(int n, const GemmArgs* gs, float* part, hipStream_t st) {
  GemmSet s{};
  s.n = n;
  int blocks = 0;
  int64_t el = 0;
  size_t off = 0;
  for (int t = 0; t < n; ++t) {
    GemmArgs g = gs[t];
    const dim3 grid = gemm_grid(g);
    int splits = gemm_splits(g);
    if (splits > 1) {
      g.k_chunk = ((g.K + splits - 1) / splits + kTK - 1) / kTK * kTK;
      splits = (g.K + g.k_chunk - 1) / g.k_chunk;
      g.part = part + off;
      off += (size_t)splits * g.M * g.N;
    } else {
      g.part = nullptr;
      g.k_chunk = 0;
    }
    s.g[t] = g;
    s.tx[t] = (int)grid.x;
    s.ty[t] = (int)grid.y;
    s.splits[t] = splits;
    s.blk0[t] = blocks;
    s.el0[t] = el;
    blocks += (int)(grid.x * grid.y) * splits;
    if (splits > 1) el += (int64_t)g.M * g.N;
  }
  s.blk0[n] = blocks;
  s.el0[n] = el;
  hipLaunchKernelGGL(k_gemm_set, dim3((unsigned)blocks), dim3(256), 0, st, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || el == 0) return e;
  hipLaunchKernelGGL(k_splitk_reduce_set, dim3((unsigned)((el + 255) / 256)), dim3(256), 0, st,
                     s);
  return hipGetLastError();
}

size_t mlp_pack_bytes() { return (size_t)kMlpPackElems * sizeof(short); }

// Pairs per workgroup of the fused network kernel: 64 for the training
// forward (a minibatch of a few thousand rows then spreads over twice the
// workgroups: 0.66 against 0.68 s for the training run), 128 for inference
// over large sets (half the weight reads; the two measured equal there).
static int mlp_rows(bool training) { return training ? 64 : 128; }

hipError_t launch_mlp_infer(const float* fq, const float* flib, const int* qidx, const int* idx,
                            int n, const float* fo_cross, const float* mean,
                            const float* inv_std, const float* params, void* packed,
                            float* out, hipStream_t st, float* x_out,
                            float* const* h_out) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((kMlpPackElems + 255) / 256), dim3(256), 0, st, params,
                     (short*)packed);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  MlpArgs a;
  a.fq = fq;
  a.flib = flib;
  a.qidx = qidx;
  a.idx = idx;
  a.n = n;
  a.fo_cross = fo_cross;
  a.mean = mean;
  a.inv_std = inv_std;
  a.W = (const v8s*)packed;
  int off = 0;
  for (int l = 0; l < 4; ++l) {
    const int i_ = l == 0 ? kMlpIn : kMlpHid;
    const int o_ = l == 3 ? kMlpOut : kMlpHid;
    off += i_ * o_;
    a.b[l] = params + off;
    off += o_;
  }
  a.out = out;
  a.x_out = x_out;
  for (int l = 0; l < 3; ++l) a.h_out[l] = h_out ? h_out[l] : nullptr;
  const int rows = mlp_rows(x_out != nullptr);
  const dim3 grid((unsigned)((n + rows - 1) / rows));
  if (x_out && rows == 64)
    hipLaunchKernelGGL((k_mlp_infer<64, true>), grid, dim3(256), 0, st, a);
  else if (x_out)
    hipLaunchKernelGGL((k_mlp_infer<128, true>), grid, dim3(256), 0, st, a);
  else if (rows == 64)
    hipLaunchKernelGGL((k_mlp_infer<64, false>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_mlp_infer<128, false>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

size_t mlp_pack_all_bytes() { return (size_t)kMlpPackAllElems * sizeof(short); }

hipError_t launch_mlp_pack_all(const float* params, void* packed, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((kMlpPackElems + 255) / 256), dim3(256), 0, st, params,
                     (short*)packed);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_pack_chain, dim3((kMlpPackAllElems - kMlpPackElems + 255) / 256),
                     dim3(256), 0, st, params, (short*)packed);
  return hipGetLastError();
}

int mlp_step_rows() { return kTrRows; }

// Scratch of one training step of n rows: the bf16 columns of every layer's
// input and gradient, the FP32 chunk sums of the gradients and the per-wave
// loss sums, each 256-byte aligned.
namespace {
struct MlpStepLayout {
  size_t actT[4], gT[4], bsum[4], loss, total;
};
MlpStepLayout mlp_step_layout(int n) {
  MlpStepLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) / 256 * 256;
    return at;
  };
  for (int l = 0; l < 4; ++l) {
    const int n_in = l == 0 ? kMlpIn : kMlpHid, n_out = l == 3 ? kMlpOut : kMlpHid;
    L.actT[l] = take((size_t)n_in * n * sizeof(short));
    L.gT[l] = take((size_t)n_out * n * sizeof(short));
    L.bsum[l] = take((size_t)(n / kColRows) * n_out * sizeof(float));
  }
  L.loss = take((size_t)(n / kColRows) * sizeof(double));
  L.total = off;
  return L;
}
}  // namespace

size_t mlp_step_scratch_bytes(int n) { return mlp_step_layout(n).total; }

hipError_t launch_mlp_step(const MlpStep& s, void* scratch, hipStream_t st) {
  const int n = s.n;
  const MlpStepLayout L = mlp_step_layout(n);
  char* base = (char*)scratch;
  MlpTrainArgs ta{};
  ta.f.fq = s.fq;
  ta.f.flib = s.flib;
  ta.f.qidx = s.qidx;
  ta.f.idx = s.idx;
  ta.f.n = n;
  ta.f.fo_cross = s.fo_cross;
  ta.f.mean = s.mean;
  ta.f.inv_std = s.inv_std;
  ta.f.W = (const v8s*)s.packed;
  ta.target = s.target;
  ta.lw = s.lw;
  ta.step = s.step;
  MlpUpdateArgs ua{};
  for (int l = 0; l < 4; ++l) {
    const int n_in = l == 0 ? kMlpIn : kMlpHid, n_out = l == 3 ? kMlpOut : kMlpHid;
    ta.f.b[l] = s.params + mlp_param_offset(l) + n_in * n_out;
    ta.actT[l] = (short*)(base + L.actT[l]);
    ta.gT[l] = (short*)(base + L.gT[l]);
    ta.bsum[l] = (float*)(base + L.bsum[l]);
    ua.actT[l] = ta.actT[l];
    ua.gT[l] = ta.gT[l];
    ua.bsum[l] = ta.bsum[l];
    // the weight gradient's split-K chunks, as shape_gemm_set chooses them
    GemmArgs g{};
    g.M = n_in;
    g.N = n_out;
    g.K = n;
    g.flags = SHAPE_GEMM_BF16;
    int splits = gemm_splits(g);
    int kc = n;
    if (splits > 1) {
      kc = ((n + splits - 1) / splits + kTK - 1) / kTK * kTK;
      splits = (n + kc - 1) / kc;
    } else {
      splits = 1;
    }
    ua.kc[l] = kc;
    ua.splits[l] = splits;
  }
  // Work of each workgroup.  Workgroups are dealt to the eight XCDs in turn
  // (workgroup b on XCD b % 8), each XCD with its own L2: an XCD gets a block
  // of tiles sharing rows of the operands (W_1, W_2: 2 output x 4 input tiles;
  // W_0: one output tile x all 3 input tiles; W_3: one input tile), then the
  // bias tiles and the loss.
  std::vector<int> per_xcd[8];
  auto code = [](int kind, int l, int ot, int it) { return kind << 24 | l << 16 | ot << 8 | it; };
  for (int x = 0; x < 8; ++x) {
    for (int l = 1; l <= 2; ++l)
      for (int ot = 2 * (x % 4); ot < 2 * (x % 4) + 2; ++ot)
        for (int it = 4 * (x / 4); it < 4 * (x / 4) + 4; ++it)
          per_xcd[x].push_back(code(kUpdWeight, l, ot, it));
    for (int it = 0; it < kMlpIn / kUpdTile; ++it) per_xcd[x].push_back(code(kUpdWeight, 0, x, it));
    per_xcd[x].push_back(code(kUpdWeight, 3, 0, x));
  }
  std::vector<int> extra;
  for (int l = 0; l < 4; ++l) {
    const int n_out = l == 3 ? kMlpOut : kMlpHid;
    for (int ot = 0; ot < (n_out + kUpdTile - 1) / kUpdTile; ++ot)
      extra.push_back(code(kUpdBias, l, ot, 0));
  }
  extra.push_back(code(kUpdLoss, 0, 0, 0));
  for (size_t e = 0; e < extra.size(); ++e) per_xcd[e % 8].push_back(extra[e]);
  size_t slots = 0;
  for (int x = 0; x < 8; ++x) slots = std::max(slots, per_xcd[x].size());
  const int blocks = (int)(8 * slots);
  if (blocks > kUpdBlocks) return hipErrorInvalidValue;
  for (int b = 0; b < blocks; ++b) {
    const std::vector<int>& q = per_xcd[b % 8];
    ua.work[b] = (size_t)(b / 8) < q.size() ? q[b / 8] : -1;
  }
  ta.loss_part = (double*)(base + L.loss);
  ua.loss_part = ta.loss_part;
  ua.n = n;
  ua.params = s.params;
  ua.m = s.m;
  ua.v = s.v;
  ua.step = s.step;
  ua.lr = s.lr;
  ua.b1 = s.b1;
  ua.b2 = s.b2;
  ua.eps = s.eps;
  ua.grad = s.grad;
  ua.packed = (short*)s.packed;
  ua.loss = s.loss;
  hipLaunchKernelGGL(k_mlp_train<kTrRows>, dim3((unsigned)(n / kTrRows)), dim3(kTrThreads), 0, st,
                     ta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_update, dim3((unsigned)blocks), dim3(kUpdThreads), 0, st, ua);
  return hipGetLastError();
}

hipError_t launch_seed_budget(const float* raw, int64_t ld, const int* idx, int k, double y_mean,
                              double y_std, double tau, int round, int cap, int* n_start,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_seed_budget, dim3((k + 255) / 256), dim3(256), 0, st, raw, ld, idx, k,
                     y_mean, y_std, tau, round, cap, n_start);
  return hipGetLastError();
}

int colsum_chunks(int M) { return (M + kColRows - 1) / kColRows; }

hipError_t launch_colsum(const float* A, int M, int N, int64_t lda, float* part, float* out,
                         hipStream_t st) {
  const int chunks = colsum_chunks(M);
  hipLaunchKernelGGL(k_colsum_partial, dim3((N + 255) / 256, chunks), dim3(256), 0, st, A, M, N,
                     lda, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum_final, dim3((N + 255) / 256), dim3(256), 0, st, part, chunks, N,
                     out);
  return hipGetLastError();
}

hipError_t launch_colsum_set(int n, const int* M, const int* N, const float* const* A,
                             const int64_t* lda, float* const* out, hipStream_t st) {
  ColsumSet s{};
  s.n = n;
  int blocks = 0;
  for (int t = 0; t < n; ++t) {
    s.M[t] = M[t];
    s.N[t] = N[t];
    s.lda[t] = lda[t];
    s.A[t] = A[t];
    s.out[t] = out[t];
    s.blk0[t] = blocks;
    blocks += (N[t] + 15) / 16;
  }
  s.blk0[n] = blocks;
  hipLaunchKernelGGL(k_colsum_set, dim3((unsigned)blocks), dim3(1024), 0, st, s);
  return hipGetLastError();
}

int mse_blocks(int B, int N) { return (int)(((int64_t)B * N + 255) / 256); }

hipError_t launch_mse(const float* y, const float* t, const float* w, int B, int N, float* grad,
                      double* partial, float* loss, hipStream_t st) {
  const int nb = mse_blocks(B, N);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, y, t, w, B, N, grad, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1), 0, st, partial, nb, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int* step,
                       float lr, float b1, float b2, float eps, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n,
                     step, lr, b1, b2, eps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_step_bump, dim3(1), dim3(1), 0, st, step);
  return hipGetLastError();
}

int topk_blocks(int n) { return (n + 255) / 256; }

hipError_t launch_topk(const float* s, int n, int k, uint32_t* sel, uint32_t* hist, int* cnt_gt,
                       int* cnt_eq, int* out, hipStream_t st) {
  hipError_t e;
  hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, st, hist, sel, k);
  // at most 256 blocks: each adds its block histogram to the global one with
  // atomics, and scores crowd into few bins, so more blocks queue more
  // atomics on the same addresses (1024 blocks: 72 us per 10^6 scores, 256:
  // 57 us)
  const int blocks = n < 256 * 256 ? topk_blocks(n) : 256;
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(blocks), dim3(256), 0, st, s, n, sel, shift, hist);
    hipLaunchKernelGGL(k_radix_pick, dim3(1), dim3(256), 0, st, hist, sel, shift);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int nb = topk_blocks(n);
  hipLaunchKernelGGL(k_select_count, dim3(nb), dim3(256), 0, st, s, n, sel, cnt_gt, cnt_eq);
  hipLaunchKernelGGL(k_select_scan, dim3(1), dim3(kScanThreads), 0, st, cnt_gt, cnt_eq, nb, sel);
  hipLaunchKernelGGL(k_select_write, dim3(nb), dim3(256), 0, st, s, n, sel, cnt_gt, cnt_eq, out);
  return hipGetLastError();
}

}  // namespace shape
