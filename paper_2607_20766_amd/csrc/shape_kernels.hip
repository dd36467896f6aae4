// HIP kernels of the IS shape-overlap engine: molecule preparation, the
// single-pair estimator and fixed / adaptive screening.
//
// Data layout in HBM (prepared by k_prepare, one record per atom, CSR order):
//   Atom          16 B  (x, y, z, alpha*log2 e)       hot-loop operand
//   AtomSampling   8 B  (1/sqrt(2 alpha), threshold)  only for sampling
//   Z             FP64 per molecule, stream id per molecule, invalid flag.
#include "shape_kernels.hpp"

#include <math.h>

namespace shape {

// ---------------------------------------------------------------------------
// Eq. occ widths: alpha = kappa / (lambda R^2).
// ---------------------------------------------------------------------------
__global__ void k_alpha_from_radius(const float* __restrict__ R, int64_t n, double kappa,
                                    double lambda, float* __restrict__ alpha) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = (double)R[i];
  alpha[i] = (float)(kappa / (lambda * r * r));
}

// ---------------------------------------------------------------------------
// Molecule preparation, one wave per molecule (four per workgroup), FP64:
// mixture weights v_i = (pi/alpha_i)^(3/2) (= t sqrt t, t = pi/alpha_i), one
// atom per lane and chunk of 64; Z = sum v_i and the running sums behind the
// thresholds floor(2^32 cumsum(v)/Z) are the plain sequential sums in atom
// order, bit for bit: the wave adds the weights one lane at a time (read
// across lanes, no LDS round trips) and each lane keeps the running sum that
// ends at its own atom.  Inputs stay in registers between the two phases.
// ---------------------------------------------------------------------------
constexpr int kPrepWaves = 4;
constexpr int kPrepChunks = SHAPE_MAX_ATOMS / kWave;

__global__ __launch_bounds__(256) void k_prepare(MolsDev in, Prepared out, int* __restrict__ flag,
                                                 int* __restrict__ set_flag,
                                                 const int* __restrict__ which, int n_which) {
  // FP64 without contraction: Z and the thresholds are the values the plain
  // expressions define, bit for bit.
#pragma clang fp contract(off)
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int idx = blockIdx.x * kPrepWaves + w;
  if (idx >= n_which) return;
  const int m = which ? which[idx] : idx;  // a listed index may repeat
  if (m < 0 || m >= in.n_mols) return;     // or lie outside: the screen flags it
  const int a0 = in.off[m], a1 = in.off[m + 1];
  const int n = a1 - a0;
  const bool range_bad = !(a0 >= 0 && (int64_t)a1 <= in.n_atoms && n >= 1 && n <= in.max_atoms);
  const int n_ok = range_bad ? 0 : n;  // n_ok <= SHAPE_MAX_ATOMS
  bool bad = range_bad;
  float px[kPrepChunks], py[kPrepChunks], pz[kPrepChunks], pa[kPrepChunks];
  double run[kPrepChunks];  // running sum through this lane's atom of each chunk
  float cx = 0.0f, cy = 0.0f, cz = 0.0f;
  double cum = 0.0;
#pragma unroll
  for (int c = 0; c < kPrepChunks; ++c) {
    px[c] = py[c] = pz[c] = 0.0f;
    pa[c] = 1.0f;
    run[c] = 0.0;
    if (c * kWave >= n_ok) continue;  // uniform
    const int i = c * kWave + lane;
    double v = 0.0;
    if (i < n_ok) {
      const float al = in.alpha[a0 + i];
      const float x = in.xyz[3 * (a0 + i)], y = in.xyz[3 * (a0 + i) + 1],
                  z = in.xyz[3 * (a0 + i) + 2];
      if (!(al > 0.0f) || !isfinite(al) || !isfinite(x) || !isfinite(y) || !isfinite(z))
        bad = true;
      const double t = M_PI / (double)al;
      v = t * sqrt(t);
      px[c] = x;
      py[c] = y;
      pz[c] = z;
      pa[c] = al;
      cx += x;
      cy += y;
      cz += z;
    }
    const int cnt = min(kWave, n_ok - c * kWave);
    for (int j = 0; j < cnt; ++j) {
      cum += readlane_f64(v, j);
      if (lane == j) run[c] = cum;
    }
  }
  bad = __ballot(bad) != 0;
  if (lane == 0) {
    out.id[m] = in.id ? in.id[m] : (uint32_t)m;
    out.bad[m] = bad ? 1 : 0;
  }
  if (bad) {
    if (lane == 0) {
      out.Z[m] = __builtin_nan("");
      out.centre[m] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      atomicOr(flag, 1);
      if (set_flag) atomicOr(set_flag, 1);
    }
    return;
  }
  // the centre is only the origin of the molecule's frame: FP32 sums
  const float scx = wave_sum_dpp(cx), scy = wave_sum_dpp(cy), scz = wave_sum_dpp(cz);
  const double Z = cum;
  if (lane == 0) {
    out.Z[m] = Z;
    const float inv_n = 1.0f / (float)n;
    out.centre[m] = make_float4(scx * inv_n, scy * inv_n, scz * inv_n, 0.0f);
  }
  const double log2e = 1.4426950408889634074;
#pragma unroll
  for (int c = 0; c < kPrepChunks; ++c) {
    const int i = c * kWave + lane;
    if (i >= n) continue;
    const double al = (double)pa[c];
    Atom a;
    a.x = px[c];
    a.y = py[c];
    a.z = pz[c];
    a.a2 = (float)(al * log2e);
    out.atom[a0 + i] = a;
    AtomSampling smp;
    smp.sd = (float)(1.0 / sqrt(2.0 * al));
    if (i + 1 < n) {
      double f = floor(4294967296.0 * (run[c] / Z));
      if (f > 4294967295.0) f = 4294967295.0;
      smp.thr = (uint32_t)f;
    } else {
      smp.thr = 0xFFFFFFFFu;
    }
    out.samp[a0 + i] = smp;
  }
}

// Re-raises the invalid-data flag for a molecule set reused from an earlier
// preparation that found invalid molecules.
__global__ void k_flag_or(int* __restrict__ flag, const int* __restrict__ set_flag) {
  if (threadIdx.x == 0 && *set_flag) atomicOr(flag, 1);
}

__global__ void k_fill_int(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Block reduction of K doubles (wave butterflies, then waves in order).
// ---------------------------------------------------------------------------
template <int K>
__device__ void block_sum(double (&v)[K], double* lds /* [4][K] */) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = wave_sum(v[j]);
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < K; ++j) lds[wave * K + j] = v[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += lds[w * K + j];
      v[j] = s;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Single pair: per-block partial sums of the eleven per-sample quantities of
// one side (samples from P, partner Q):
//   f1 = w_P u_Q, f2 = w_P u_P, f3 = w_P, f4 = m_Q, f5 = m_P
// sums: f1, f1^2, f2, f2^2, f3, f3^2, f4, f4^2, f5, f5^2, f1 f2.
// blockIdx.y = side (0: P = A, 1: P = B).
// ---------------------------------------------------------------------------
constexpr int kEstSPT = 8;

__global__ __launch_bounds__(256) void k_est_partials(Prepared A, Prepared B, int64_t n_a,
                                                      int64_t n_b, uint2 key, int anti,
                                                      double* __restrict__ partials,
                                                      int nblk, const int* __restrict__ offA,
                                                      const int* __restrict__ offB) {
  __shared__ Atom sP[SHAPE_MAX_ATOMS];
  __shared__ Atom sQ[SHAPE_MAX_ATOMS];
  __shared__ AtomSampling sS[SHAPE_MAX_ATOMS];
  __shared__ double red[4 * kEstSums];
  const int side = blockIdx.y;
  const Prepared& P = side ? B : A;
  const Prepared& Q = side ? A : B;
  const int* offP = side ? offB : offA;
  const int* offQ = side ? offA : offB;
  const int64_t n = side ? n_b : n_a;
  const int64_t units = anti ? n / 2 : n;  // independent terms: samples or pairs
  const int p0 = offP[0], np = offP[1] - offP[0];
  const int q0 = offQ[0], nq = offQ[1] - offQ[0];
  const uint32_t idp = P.id[0];
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    sP[i] = P.atom[p0 + i];
    sS[i] = P.samp[p0 + i];
  }
  for (int i = threadIdx.x; i < nq; i += blockDim.x) sQ[i] = Q.atom[q0 + i];
  __syncthreads();
  float acc[kEstSums];
#pragma unroll
  for (int j = 0; j < kEstSums; ++j) acc[j] = 0.0f;
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * kEstSPT;
  for (int s = 0; s < kEstSPT; ++s) {
    const int64_t u = base + (int64_t)s * blockDim.x + threadIdx.x;
    if (u >= units) break;
    // the unit's term: the sample itself, or the mean over an antithetic pair
    float f[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    const int members = anti ? 2 : 1;
    for (int mbr = 0; mbr < members; ++mbr) {
      float rx[1], ry[1], rz[1];
      if (anti)
        sample_point_anti(sP, sS, np, idp, (uint64_t)(2 * u + mbr), key, rx[0], ry[0], rz[0]);
      else
        sample_point(sP, sS, np, idp, (uint64_t)u, key, rx[0], ry[0], rz[0]);
      float mp[1] = {0.0f}, qp[1] = {1.0f}, mq[1] = {0.0f}, qq[1] = {1.0f};
      eval_density<1>(sP, np, rx, ry, rz, mp, qp);
      eval_density<1>(sQ, nq, rx, ry, rz, mq, qq);
      const float uP = 1.0f - qp[0], uQ = 1.0f - qq[0];
      const float w = bounded_weight(uP, mp[0]);
      f[0] += w * uQ; f[1] += w * uP; f[2] += w; f[3] += mq[0]; f[4] += mp[0];
    }
    if (anti)
#pragma unroll
      for (int j = 0; j < 5; ++j) f[j] *= 0.5f;
    acc[0] += f[0]; acc[1] += f[0] * f[0];
    acc[2] += f[1]; acc[3] += f[1] * f[1];
    acc[4] += f[2]; acc[5] += f[2] * f[2];
    acc[6] += f[3]; acc[7] += f[3] * f[3];
    acc[8] += f[4]; acc[9] += f[4] * f[4];
    acc[10] += f[0] * f[1];
  }
  double v[kEstSums];
#pragma unroll
  for (int j = 0; j < kEstSums; ++j) v[j] = (double)acc[j];
  block_sum<kEstSums>(v, red);
  if (threadIdx.x == 0) {
    double* dst = partials + ((size_t)side * nblk + blockIdx.x) * kEstSums;
#pragma unroll
    for (int j = 0; j < kEstSums; ++j) dst[j] = v[j];
  }
}

// Mean, sample variance (n-1) and covariance from running sums.
struct Moments {
  double n, s, ss;
  __device__ double mean() const { return s / n; }
  __device__ double var() const {
    const double v = (ss - s * s / n) / (n - 1.0);
    return v > 0.0 ? v : 0.0;
  }
};

__global__ __launch_bounds__(256) void k_est_finalize(const double* __restrict__ partials,
                                                      int nblk, Prepared A, Prepared B,
                                                      int64_t n_a, int64_t n_b, int anti,
                                                      shape_result* __restrict__ out) {
  __shared__ double red[4 * 2 * kEstSums];
  double v[2 * kEstSums];
#pragma unroll
  for (int j = 0; j < 2 * kEstSums; ++j) v[j] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
      for (int j = 0; j < kEstSums; ++j)
        v[side * kEstSums + j] += partials[((size_t)side * nblk + b) * kEstSums + j];
  }
  block_sum<2 * kEstSums>(v, red);
  if (threadIdx.x != 0) return;
  const double Za = A.Z[0], Zb = B.Z[0];
  // independent terms per side: samples, or antithetic pair means
  const double na = (double)(anti ? n_a / 2 : n_a), nb = (double)(anti ? n_b / 2 : n_b);
  const double* a = v;
  const double* b = v + kEstSums;
  auto mom = [](double n, const double* s, int j) { return Moments{n, s[2 * j], s[2 * j + 1]}; };
  const Moments a1 = mom(na, a, 0), a2 = mom(na, a, 1), a3 = mom(na, a, 2), a4 = mom(na, a, 3),
                a5 = mom(na, a, 4);
  const Moments b1 = mom(nb, b, 0), b2 = mom(nb, b, 1), b3 = mom(nb, b, 2), b4 = mom(nb, b, 3),
                b5 = mom(nb, b, 4);
  const double cov_a = (a[10] - a[0] * a[2] / na) / (na - 1.0);
  const double cov_b = (b[10] - b[0] * b[2] / nb) / (nb - 1.0);
  shape_result r;
  r.O_ab_from_a = Za * a1.mean();
  r.O_ab_from_b = Zb * b1.mean();
  const double se_xa = Za * sqrt(a1.var() / na), se_xb = Zb * sqrt(b1.var() / nb);
  r.O_ab = 0.5 * (r.O_ab_from_a + r.O_ab_from_b);
  r.se_O_ab = 0.5 * sqrt(se_xa * se_xa + se_xb * se_xb);
  r.O_aa = Za * a2.mean();
  r.O_bb = Zb * b2.mean();
  r.se_O_aa = Za * sqrt(a2.var() / na);
  r.se_O_bb = Zb * sqrt(b2.var() / nb);
  r.V_a = Za * a3.mean();
  r.V_b = Zb * b3.mean();
  r.se_V_a = Za * sqrt(a3.var() / na);
  r.se_V_b = Zb * sqrt(b3.var() / nb);
  r.Ofo_ab_is = 0.5 * (Za * a4.mean() + Zb * b4.mean());
  r.Ofo_aa_is = Za * a5.mean();
  r.Ofo_bb_is = Zb * b5.mean();
  const double S = r.O_aa + r.O_bb, D = S - r.O_ab;
  r.T = r.O_ab / D;
  r.se_T = fabs(S / (D * D)) * r.se_O_ab;
  const double g_ab = S / (D * D), g_s = -r.O_ab / (D * D);
  const double var_s = r.se_O_aa * r.se_O_aa + r.se_O_bb * r.se_O_bb;
  const double cov = 0.5 * Za * Za * cov_a / na + 0.5 * Zb * Zb * cov_b / nb;
  const double vt = g_ab * g_ab * r.se_O_ab * r.se_O_ab + g_s * g_s * var_s + 2.0 * g_ab * g_s * cov;
  r.se_T_full = sqrt(vt > 0.0 ? vt : 0.0);
  r.n_a = n_a;
  r.n_b = n_b;
  *out = r;
}

// ---------------------------------------------------------------------------
// Query-side sample cache for screening: the query's own samples, weights and
// self integrand are the same for every library partner (random numbers are
// keyed by molecule), so they are computed once per call.  Points are kept in
// the query's frame (origin at its centre):
//   qs[k] = (r'_k, w_A(r_k)),  qf2[k] = w_A u_A at r_k.
// The densities use the expanded form with the same records the screening
// kernel builds, so a library copy of the query reproduces them bit for bit.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_query_cache(Prepared Qp, const int* __restrict__ offQ,
                                                     int64_t n, uint2 key, int anti,
                                                     float4* __restrict__ qs,
                                                     float* __restrict__ qf2) {
  __shared__ Atom sF[SHAPE_MAX_ATOMS];          // frame coordinates for sampling
  __shared__ AtomSampling sS[SHAPE_MAX_ATOMS];
  __shared__ AtomRec sR[SHAPE_MAX_ATOMS];
  __shared__ float sA[SHAPE_MAX_ATOMS];
  // an invalid query is never staged (its atom count is not trusted); the
  // screening kernel then reports every pair as NaN without reading the cache
  if (Qp.bad[0] != 0) return;
  const int q0 = offQ[0], nq = offQ[1] - offQ[0];
  const float4 cq = Qp.centre[0];
  for (int i = threadIdx.x; i < nq; i += blockDim.x) {
    const Atom a = Qp.atom[q0 + i];
    Atom f = a;
    f.x = a.x - cq.x;
    f.y = a.y - cq.y;
    f.z = a.z - cq.z;
    sF[i] = f;
    sS[i] = Qp.samp[q0 + i];
    make_rec(a, cq.x, cq.y, cq.z, sR[i], sA[i]);
  }
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float rx[1], ry[1], rz[1], r2[1];
  if (anti)
    sample_point_anti(sF, sS, nq, Qp.id[0], (uint64_t)k, key, rx[0], ry[0], rz[0]);
  else
    sample_point(sF, sS, nq, Qp.id[0], (uint64_t)k, key, rx[0], ry[0], rz[0]);
  r2[0] = norm2(rx[0], ry[0], rz[0]);
  float m[1] = {0.0f}, q[1] = {1.0f};
  eval_density_x<1>(sR, sA, nq, rx, ry, rz, r2, m, q);
  const float u = 1.0f - q[0];
  const float w = bounded_weight(u, m[0]);
  qs[k] = make_float4(rx[0], ry[0], rz[0], w);
  qf2[k] = w * u;
}

// ---------------------------------------------------------------------------
// Screening kernel: one single-wave workgroup per (query, library) pair, so
// the pair index comes from blockIdx and is uniform by construction (no
// cross-lane broadcast); the hardware dispatcher balances pairs of uneven
// size.  Pairs are renumbered so that each XCD screens tiles of consecutive
// library molecules (xcd_chunk).  Per round, `round_side` samples on each side:
//   side A (query samples, from the cache): f1 = w_A u_B, f2 = w_A u_A
//   side B (library samples, drawn here):   f1 = w_B u_A, f2 = w_B u_B
// FP32 in-lane sums per round, FP64 lane accumulators across rounds, wave
// butterflies for the pair totals (every lane ends with the same value).
// Adaptive mode takes the stopping decision on SE(T) in FP64 after every
// round; the decision is read from the first lane so the branch is scalar.
// ---------------------------------------------------------------------------
// Work granularity of the screening kernel: kSA (kSB) side-A (side-B) points
// per lane are evaluated together against each atom record read from LDS.
// Every variant assigns the same samples to the same lanes and accumulates
// them in the same order, so all variants give bit-identical results; the
// autotuner picks the fastest for a workload.
const int kScreenVariantShape[kScreenVariants][2] = {
    {4, 2}, {2, 2}, {4, 1}, {4, 4}, {8, 2}, {2, 1}, {8, 4}, {2, 4}};

__device__ __forceinline__ double se_tanimoto(double n, double Za, double Zb, double a1,
                                              double a11, double a2, double b1, double b11,
                                              double b2, double* T_out, double* Oab_out,
                                              double* Oaa_out, double* Obb_out) {
#pragma clang fp contract(off)
  const double xa = Za * a1 / n, xb = Zb * b1 / n;
  double va = (a11 - a1 * a1 / n) / (n - 1.0);
  double vb = (b11 - b1 * b1 / n) / (n - 1.0);
  va = va > 0.0 ? va : 0.0;
  vb = vb > 0.0 ? vb : 0.0;
  const double se_a = Za * sqrt(va / n), se_b = Zb * sqrt(vb / n);
  const double O_ab = 0.5 * (xa + xb);
  const double se_O = 0.5 * sqrt(se_a * se_a + se_b * se_b);
  const double O_aa = Za * a2 / n, O_bb = Zb * b2 / n;
  const double S = O_aa + O_bb, D = S - O_ab;
  if (T_out) *T_out = O_ab / D;
  if (Oab_out) *Oab_out = O_ab;
  if (Oaa_out) *Oaa_out = O_aa;
  if (Obb_out) *Obb_out = O_bb;
  return fabs(S / (D * D)) * se_O;
}

template <int kSA, int kSB>
__global__ __launch_bounds__(64) void k_screen(ScreenArgs a) {
  // No implicit multiply-add contraction: the fused operations are written
  // out, so every tile variant rounds identically.
#pragma clang fp contract(off)
  // LDS (per pair, n = atoms):
  //   sBF   [max_b] Atom          library atoms in the library frame (sampling)
  //   sBS   [max_b] AtomSampling  their sampling records
  //   sBB   [max_b] AtomRec + a2  library atoms, library frame (own density)
  //   sBA   [max_b] AtomRec + a2  library atoms, query frame (side A partner)
  //   sAB   [max_q] AtomRec + a2  query atoms, library frame (side B partner)
  //   guide [kGuideSize] int      the library molecule's component guide
  // 16-byte records first, then the 8-byte, then the 4-byte arrays, so every
  // array is aligned to its element size whatever the atom counts.
  extern __shared__ __align__(16) unsigned char smem[];
  Atom* sBF = reinterpret_cast<Atom*>(smem);
  AtomRec* sBB = reinterpret_cast<AtomRec*>(sBF + a.max_b);
  AtomRec* sBA = sBB + a.max_b;
  AtomRec* sAB = sBA + a.max_b;
  AtomSampling* sBS = reinterpret_cast<AtomSampling*>(sAB + a.max_q);
  float* aBB = reinterpret_cast<float*>(sBS + a.max_b);
  float* aBA = aBB + a.max_b;
  float* aAB = aBA + a.max_b;
  int* guide = reinterpret_cast<int*>(aAB + a.max_q);  // [kGuideSize] of the library molecule
  const int lane = threadIdx.x;
  // grid = n_pairs; a launch order, when given, is a permutation of the pairs
  const int p = a.order ? a.order[blockIdx.x] : xcd_chunk(blockIdx.x, gridDim.x);
  if (p < 0 || p >= a.n_pairs) return;
  const int m = a.pairs ? a.pairs[p] : p;
  const bool bad = a.Q.bad[0] != 0 || m < 0 || m >= a.n_lib || a.L.bad[m] != 0;
  if (bad) {
    if (lane == 0) {
      const float nanv = __builtin_nanf("");
      a.T[p] = nanv;
      a.se_T[p] = nanv;
      if (a.O_ab) a.O_ab[p] = nanv;
      if (a.O_aa) a.O_aa[p] = nanv;
      if (a.O_bb) a.O_bb[p] = nanv;
      if (a.n_used) a.n_used[p] = 0;
    }
    return;
  }
  const int q0 = a.offQ[0], nq = a.offQ[1] - a.offQ[0];
  const int b0 = a.offL[m], nb = a.offL[m + 1] - b0;
  const float4 cA = a.Q.centre[0];
  const float4 cB = a.L.centre[m];
  for (int i = lane; i < nq; i += kWave) make_rec(a.Q.atom[q0 + i], cB.x, cB.y, cB.z, sAB[i], aAB[i]);
  for (int i = lane; i < nb; i += kWave) {
    const Atom at = a.L.atom[b0 + i];
    Atom f = at;
    f.x = at.x - cB.x;
    f.y = at.y - cB.y;
    f.z = at.z - cB.z;
    sBF[i] = f;
    sBS[i] = a.L.samp[b0 + i];
    make_rec(at, cB.x, cB.y, cB.z, sBB[i], aBB[i]);
    make_rec(at, cA.x, cA.y, cA.z, sBA[i], aBA[i]);
  }
  __syncthreads();
  build_guide(sBS, nb, guide, lane, kWave);
  __syncthreads();
  const double Za = a.Q.Z[0];
  const uint32_t idb = a.L.id[m];
  const double Zb = a.L.Z[m];
  const int rs = a.round_side;
  const int per_lane = rs / kWave;
  // Running sums over both sides, identical in every lane: per round each
  // lane's FP32 partials are summed across the wave (DPP) and added in FP64.
  // S[0..2] = sum f1, sum f1^2, sum f2 on side A; S[3..5] the same on side B.
  double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t n_side = 0;
  const int64_t first_check = a.n_start ? (int64_t)a.n_start[p] : 0;
  const double tau2x4 = 4.0 * a.tau * a.tau;
  // Slot i of a lane in a round holds sample n_side + lane + 64 i (i.i.d.),
  // or for antithetic sampling member i & 1 of pair n_side/2 + lane +
  // 64 (i >> 1), i.e. sample n_side + 2 lane + 128 (i >> 1) + (i & 1); the
  // pair's two members sit in consecutive slots of one lane and enter the
  // sums as one term, their mean (pend* holds the first member).
  const bool anti = a.anti != 0;
  float pa1 = 0.f, pa2 = 0.f, pb1 = 0.f, pb2 = 0.f;
  for (;;) {
    float fa[3] = {0.f, 0.f, 0.f};
    float fb[3] = {0.f, 0.f, 0.f};
    // side A: query samples from the cache (query frame), partner = library
    for (int t = 0; t < per_lane; t += kSA) {
      float rx[kSA], ry[kSA], rz[kSA], r2[kSA], w[kSA], f2[kSA], q[kSA], valid[kSA];
#pragma unroll
      for (int s = 0; s < kSA; ++s) {
        const bool ok = (t + s) < per_lane;
        const int i = ok ? t + s : t;
        const int k = anti ? (int)n_side + 2 * lane + 2 * kWave * (i >> 1) + (i & 1)
                           : (int)n_side + lane + kWave * i;
        const float4 c = a.qs[k];
        rx[s] = c.x; ry[s] = c.y; rz[s] = c.z; w[s] = c.w;
        r2[s] = norm2(c.x, c.y, c.z);
        f2[s] = a.qf2[k];
        q[s] = 1.0f;
        valid[s] = ok ? 1.0f : 0.0f;
      }
      eval_union_x<kSA>(sBA, aBA, nb, rx, ry, rz, r2, q);
#pragma unroll
      for (int s = 0; s < kSA; ++s) {
        const float f1 = w[s] * (1.0f - q[s]) * valid[s];
        if (!anti) {
          fa[0] += f1; fa[1] = fmaf(f1, f1, fa[1]);
          fa[2] = fmaf(f2[s], valid[s], fa[2]);
        } else if (((t + s) & 1) == 0) {
          pa1 = f1;
          pa2 = f2[s] * valid[s];
        } else {
          const float g1 = 0.5f * (pa1 + f1), g2 = 0.5f * (pa2 + f2[s] * valid[s]);
          fa[0] += g1; fa[1] = fmaf(g1, g1, fa[1]);
          fa[2] += g2;
        }
      }
    }
    // side B: library samples drawn here (library frame), partner = query
    for (int t = 0; t < per_lane; t += kSB) {
      float rx[kSB], ry[kSB], rz[kSB], r2[kSB], mb[kSB], qb[kSB], qa[kSB], valid[kSB];
#pragma unroll
      for (int s = 0; s < kSB; ++s) {
        const bool ok = (t + s) < per_lane;
        const int i = ok ? t + s : t;
        if (!anti) {
          const int64_t k = n_side + (int64_t)lane + (int64_t)kWave * i;
          sample_point(sBF, sBS, nb, idb, (uint64_t)k, a.key, rx[s], ry[s], rz[s], guide);
        } else if (kSB % 2 == 0) {
          // both members of the pair from one Philox block (t and s even)
          if ((s & 1) == 0) {
            const int64_t pr = n_side / 2 + (int64_t)lane + (int64_t)kWave * (i >> 1);
            sample_pair(sBF, sBS, nb, idb, (uint64_t)pr, a.key, rx[s], ry[s], rz[s],
                        rx[s + 1 < kSB ? s + 1 : s], ry[s + 1 < kSB ? s + 1 : s],
                        rz[s + 1 < kSB ? s + 1 : s], guide);
          }
        } else {
          const int64_t k = n_side + 2 * (int64_t)lane + 2 * (int64_t)kWave * (i >> 1) + (i & 1);
          sample_point_anti(sBF, sBS, nb, idb, (uint64_t)k, a.key, rx[s], ry[s], rz[s], guide);
        }
        valid[s] = ok ? 1.0f : 0.0f;
      }
#pragma unroll
      for (int s = 0; s < kSB; ++s) {
        r2[s] = norm2(rx[s], ry[s], rz[s]);
        mb[s] = 0.0f; qb[s] = 1.0f; qa[s] = 1.0f;
      }
      eval_density_x<kSB>(sBB, aBB, nb, rx, ry, rz, r2, mb, qb);
      eval_union_x<kSB>(sAB, aAB, nq, rx, ry, rz, r2, qa);
#pragma unroll
      for (int s = 0; s < kSB; ++s) {
        const float ub = 1.0f - qb[s];
        const float w = bounded_weight(ub, mb[s]) * valid[s];
        const float f1 = w * (1.0f - qa[s]);
        if (!anti) {
          fb[0] += f1; fb[1] = fmaf(f1, f1, fb[1]);
          fb[2] = fmaf(w, ub, fb[2]);
        } else if (((t + s) & 1) == 0) {
          pb1 = f1;
          pb2 = w * ub;
        } else {
          const float g1 = 0.5f * (pb1 + f1), g2 = 0.5f * (pb2 + w * ub);
          fb[0] += g1; fb[1] = fmaf(g1, g1, fb[1]);
          fb[2] += g2;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      S[j] += (double)wave_sum_dpp(fa[j]);
      S[3 + j] += (double)wave_sum_dpp(fb[j]);
    }
    n_side += rs;
    int stop;
    if (a.mode == SHAPE_SCREEN_ADAPTIVE) {
      if (2 * n_side >= a.cap_pair) {
        stop = 1;
      } else if (2 * n_side < first_check) {
        stop = 0;  // below the pair's seeded budget: no test yet
      } else {
        // SE(T) <= tau without divisions or roots: with n samples per side,
        // S' = Za a2 + Zb b2, D' = S' - (Za a1 + Zb b1)/2 and
        // V = n a11 - a1^2 (clamped at 0), the delta-method SE satisfies
        //   SE(T)^2 = S'^2 (Za^2 Va + Zb^2 Vb) / (4 (n-1) D'^4),
        // so the test is S'^2 (Za^2 Va + Zb^2 Vb) <= 4 tau^2 (n-1) D'^4 with
        // D' != 0 (NaN sums never stop).
        const double n = (double)(anti ? n_side / 2 : n_side);  // independent terms
        const double Sp = Za * S[2] + Zb * S[5];
        const double Dp = Sp - 0.5 * (Za * S[0] + Zb * S[3]);
        const double Va = fmax(n * S[1] - S[0] * S[0], 0.0);
        const double Vb = fmax(n * S[4] - S[3] * S[3], 0.0);
        const double lhs = Sp * Sp * (Za * Za * Va + Zb * Zb * Vb);
        const double D2 = Dp * Dp;
        stop = (Dp != 0.0 && lhs <= tau2x4 * (n - 1.0) * D2 * D2) ? 1 : 0;
      }
    } else {
      stop = n_side >= a.n_fixed ? 1 : 0;
    }
    if (__builtin_amdgcn_readfirstlane(stop)) break;
  }
  if (lane == 0) {
    double T, O_ab, O_aa, O_bb;
    const double se = se_tanimoto((double)(anti ? n_side / 2 : n_side), Za, Zb, S[0], S[1],
                                  S[2], S[3], S[4], S[5], &T, &O_ab, &O_aa, &O_bb);
    a.T[p] = (float)T;
    a.se_T[p] = (float)se;
    if (a.O_ab) a.O_ab[p] = (float)O_ab;
    if (a.O_aa) a.O_aa[p] = (float)O_aa;
    if (a.O_bb) a.O_bb[p] = (float)O_bb;
    if (a.n_used) a.n_used[p] = (int)(2 * n_side);
  }
}

// ---------------------------------------------------------------------------
// Export of the sampling steps of one prepared molecule (section
// "Importance-sampling estimator": exact draws from the normalised mixture),
// for exact comparison of the integer steps: the molecule's thresholds, and
// for samples k0 .. k0+n-1 the Philox block, the selected component (binary
// lifting, as in the single-pair, query-cache and alignment kernels) and the
// point (through the guide table, as in the screening kernel), computed by
// the same device functions as those kernels.  One thread per sample (and
// per atom for the thresholds); records from HBM.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sample_points(Prepared P, const int* __restrict__ off,
                                                       int mol, int64_t k0, int n, uint2 key,
                                                       int anti, uint32_t* __restrict__ thr,
                                                       uint32_t* __restrict__ words,
                                                       int* __restrict__ comp,
                                                       float* __restrict__ r) {
  __shared__ int guide[kGuideSize];  // the screening kernel's table, one entry per thread
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int a0 = off[mol], na = off[mol + 1] - a0;
  const Atom* atoms = P.atom + a0;
  const AtomSampling* samp = P.samp + a0;
  if (thr && i < na) thr[i] = samp[i].thr;
  build_guide(samp, na, guide, threadIdx.x, blockDim.x);
  __syncthreads();
  if (i >= n) return;
  const uint64_t k = (uint64_t)(k0 + i);
  const uint64_t blk = anti ? k >> 1 : k;
  const uint4 x =
      philox4x32_10(make_uint4((uint32_t)blk, (uint32_t)(blk >> 32), P.id[mol], 0u), key);
  if (words) reinterpret_cast<uint4*>(words)[i] = x;
  if (comp) comp[i] = select_component(samp, na, x.x);
  if (r) {
    // the point through the guide table: a component other than comp's
    // would move it far outside the bound of its floating-point steps
    float rx, ry, rz;
    if (anti)
      sample_point_anti(atoms, samp, na, P.id[mol], k, key, rx, ry, rz, guide);
    else
      sample_point(atoms, samp, na, P.id[mol], k, key, rx, ry, rz, guide);
    r[3 * (size_t)i] = rx;
    r[3 * (size_t)i + 1] = ry;
    r[3 * (size_t)i + 2] = rz;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
hipError_t launch_alpha_from_radius(const float* R, int64_t n, double kappa, double lambda,
                                    float* alpha, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_alpha_from_radius, dim3((unsigned)blocks), dim3(256), 0, st, R, n, kappa,
                     lambda, alpha);
  return hipGetLastError();
}

hipError_t launch_prepare(const MolsDev& in, const Prepared& out, int* flag, int* set_flag,
                          hipStream_t st, const int* which, int n_which) {
  const int n = which ? n_which : in.n_mols;
  if (n <= 0) return hipSuccess;
  const int blocks = (n + kPrepWaves - 1) / kPrepWaves;
  hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), 0, st, in, out, flag, set_flag, which,
                     n);
  return hipGetLastError();
}

hipError_t launch_flag_or(int* flag, const int* set_flag, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_or, dim3(1), dim3(64), 0, st, flag, set_flag);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

int est_blocks(int64_t n_units) {
  return (int)((n_units + 256 * kEstSPT - 1) / (256 * kEstSPT));
}

hipError_t launch_estimate(const Prepared& A, const Prepared& B, const int* offA,
                           const int* offB, int64_t n_a, int64_t n_b, uint2 key, int anti,
                           double* partials, int nblk, shape_result* out_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_est_partials, dim3(nblk, 2), dim3(256), 0, st, A, B, n_a, n_b, key, anti,
                     partials, nblk, offA, offB);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_est_finalize, dim3(1), dim3(256), 0, st, partials, nblk, A, B, n_a, n_b,
                     anti, out_dev);
  return hipGetLastError();
}

hipError_t launch_query_cache(const Prepared& Q, const int* offQ, int64_t n, uint2 key, int anti,
                              float4* qs, float* qf2, hipStream_t st) {
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_query_cache, dim3((unsigned)blocks), dim3(256), 0, st, Q, offQ, n, key,
                     anti, qs, qf2);
  return hipGetLastError();
}

hipError_t launch_sample_points(const Prepared& P, const int* off, int mol, int max_atoms,
                               int64_t k0, int n, uint2 key, int anti, uint32_t* thr,
                               uint32_t* words, int* comp, float* r, hipStream_t st) {
  const int threads = n > max_atoms ? n : max_atoms;
  const int blocks = (threads + 255) / 256;
  hipLaunchKernelGGL(k_sample_points, dim3(blocks), dim3(256), 0, st, P, off, mol, k0, n, key,
                     anti, thr, words, comp, r);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launch order of a grid with one workgroup per pair: largest estimated work
// first.  A pair's result depends on that pair alone, so the order in which
// workgroups take the pairs changes no output; it changes how long the last
// workgroups run on after the others have finished.  The caller states the
// work of a pair in atoms' worth from its atom counts (B's, or their square,
// in a quadratic pass) and seeded budget;
// pairs are bucketed by its logarithm, 8 buckets per octave.  With per_xcd,
// each XCD keeps the pairs xcd_chunk deals it (so its L2 still sees whole
// tiles of consecutive molecules and output lines) and takes them largest
// first: block b = 8 r + x, the r-th block the round-robin dispatch sends to
// XCD x, takes the r-th pair of XCD x's order; otherwise block b takes the
// b-th largest.  A counting sort over (group, bucket) in three launches:
// kOrderBlocks blocks histogram their contiguous share of the pairs in LDS;
// one thread per bucket sums its counts over the blocks (prefix and total);
// the same blocks again, each after an LDS scan of the totals, place their
// pairs with LDS atomics (the order inside a bucket is not fixed).  Every
// slot is written on every call, so no memory needs clearing.
// ---------------------------------------------------------------------------
constexpr int kOrderKeys = 256;                    // work buckets per group
constexpr int kOrderBuckets = kXcds * kOrderKeys;  // (group, bucket) pairs
constexpr int kOrderBlocks = 64;
constexpr int kOrderThreads = 1024;

// XCD of the block that xcd_chunk maps to item p of a grid of G blocks:
// below F = G - G mod (8 kXcdTile) tile p / kXcdTile sits on XCD tile mod 8;
// blocks from F on keep their index, so block p runs on XCD p mod 8.
__device__ __forceinline__ int xcd_of_item(int p, int G) {
  const int F = G - G % (kXcds * kXcdTile);
  return p >= F ? p % kXcds : (p / kXcdTile) % kXcds;
}

__device__ __forceinline__ int atoms_of(const int* off, int m, int max_atoms) {
  const int n = off[m + 1] - off[m];
  return n < 0 ? 0 : (n > max_atoms ? max_atoms : n);
}

__device__ __forceinline__ int order_key(const OrderArgs& o, int p) {
  const int g = o.per_xcd ? xcd_of_item(p, o.n) : 0;
  const int m = o.pairs ? o.pairs[p] : p;
  if (m < 0 || m >= o.nB_mols) return g * kOrderKeys;  // an invalid pair only writes NaN
  const uint64_t nb = (uint64_t)atoms_of(o.offB, m, o.max_b);
  uint64_t cost = (uint64_t)o.wB * (o.quad_b ? nb * nb : nb) + o.w0;
  if (o.offA) {
    const int ma = o.a_single ? 0 : p;
    if (ma < o.nA_mols) cost += (uint64_t)o.wA * (uint64_t)atoms_of(o.offA, ma, o.max_a);
  }
  if (o.n_start) {
    const int64_t s = o.n_start[p];
    const int64_t r = s <= o.round_pair ? 1
                    : (s >= o.cap ? o.cap / o.round_pair
                                  : (s + o.round_pair - 1) / o.round_pair);
    cost *= (uint64_t)r;
  }
  const uint32_t c = cost == 0 ? 1u : (cost > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)cost);
  const int e = 31 - __clz(c);
  const uint32_t mant = e >= 3 ? (c >> (e - 3)) & 7u : (c << (3 - e)) & 7u;
  return g * kOrderKeys + 8 * e + (int)mant;  // 8 e + 7 < kOrderKeys
}

__device__ __forceinline__ void order_share(int n, int& begin, int& end) {
  const int64_t per = ((int64_t)n + kOrderBlocks - 1) / kOrderBlocks;
  begin = (int)min((int64_t)n, (int64_t)blockIdx.x * per);
  end = (int)min((int64_t)n, (int64_t)begin + per);
}

// hist[k][b]: pairs of block b's share with key k (bucket-major, so that
// the scan reads each bucket's counts as 16 consecutive 16-byte words)
__global__ __launch_bounds__(kOrderThreads) void k_order_hist(OrderArgs o,
                                                              int* __restrict__ hist) {
  __shared__ int h[kOrderBuckets];
  for (int k = threadIdx.x; k < kOrderBuckets; k += kOrderThreads) h[k] = 0;
  __syncthreads();
  int begin, end;
  order_share(o.n, begin, end);
  for (int64_t p = begin + (int64_t)threadIdx.x; p < end; p += kOrderThreads)
    atomicAdd(&h[order_key(o, (int)p)], 1);
  __syncthreads();
  for (int k = threadIdx.x; k < kOrderBuckets; k += kOrderThreads)
    hist[k * kOrderBlocks + blockIdx.x] = h[k];
}

// One thread per key k: replaces hist[k][b] by the number of pairs with key k
// in blocks before b, and writes the key's total to tot[k].  hist is 16-byte
// aligned.
constexpr int kOrderScanThreads = 64;
__global__ __launch_bounds__(kOrderScanThreads) void k_order_scan(int* __restrict__ hist,
                                                                 int* __restrict__ tot) {
  constexpr int kVec = kOrderBlocks / 4;
  const int k = blockIdx.x * kOrderScanThreads + threadIdx.x;
  int4* row = reinterpret_cast<int4*>(hist + k * kOrderBlocks);
  int4 h[kVec];
#pragma unroll
  for (int i = 0; i < kVec; ++i) h[i] = row[i];
  int rank = 0;
#pragma unroll
  for (int i = 0; i < kVec; ++i) {
    int4 r;
    r.x = rank; rank += h[i].x;
    r.y = rank; rank += h[i].y;
    r.z = rank; rank += h[i].z;
    r.w = rank; rank += h[i].w;
    row[i] = r;
  }
  tot[k] = rank;
}

// Block b places its share: pair p with key k goes to rank
// (pairs of its group with larger keys) + (key-k pairs of earlier blocks) +
// (its arrival among block b's key-k pairs) of its group's order.
__global__ __launch_bounds__(kOrderThreads) void k_order_place(OrderArgs o,
                                                               const int* __restrict__ before,
                                                               const int* __restrict__ tot,
                                                               int* __restrict__ order) {
  constexpr int kPer = kOrderBuckets / kOrderThreads;
  __shared__ int cur[kOrderBuckets];
  int t[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int k = threadIdx.x + j * kOrderThreads;
    t[j] = tot[k];
    cur[k] = t[j];
  }
  __syncthreads();
  // suffix sums within each group's segment: cur[k] = its pairs with keys >= k
  for (int d = 1; d < kOrderKeys; d <<= 1) {
    int add[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int k = threadIdx.x + j * kOrderThreads;
      add[j] = (k % kOrderKeys) + d < kOrderKeys ? cur[k + d] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) cur[threadIdx.x + j * kOrderThreads] += add[j];
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int k = threadIdx.x + j * kOrderThreads;
    cur[k] += before[k * kOrderBlocks + blockIdx.x] - t[j];
  }
  __syncthreads();
  int begin, end;
  order_share(o.n, begin, end);
  const int groups = o.per_xcd ? kXcds : 1;
  for (int64_t p = begin + (int64_t)threadIdx.x; p < end; p += kOrderThreads) {
    const int key = order_key(o, (int)p);
    const int r = atomicAdd(&cur[key], 1);
    order[(int64_t)groups * r + key / kOrderKeys] = (int)p;
  }
}

int work_order_ints() { return kOrderBlocks * kOrderBuckets + kOrderBuckets; }

hipError_t launch_work_order(const OrderArgs& o, int* order, int* work, hipStream_t st) {
  int* tot = work + kOrderBlocks * kOrderBuckets;
  hipLaunchKernelGGL(k_order_hist, dim3(kOrderBlocks), dim3(kOrderThreads), 0, st, o, work);
  hipLaunchKernelGGL(k_order_scan, dim3(kOrderBuckets / kOrderScanThreads),
                     dim3(kOrderScanThreads), 0, st, work, tot);
  hipLaunchKernelGGL(k_order_place, dim3(kOrderBlocks), dim3(kOrderThreads), 0, st, o,
                     (const int*)work, (const int*)tot, order);
  return hipGetLastError();
}

size_t screen_lds_bytes(int max_q, int max_b) {
  return (size_t)max_b * (sizeof(Atom) + 2 * (sizeof(AtomRec) + sizeof(float)) +
                          sizeof(AtomSampling)) +
         (size_t)max_q * (sizeof(AtomRec) + sizeof(float)) + kGuideSize * sizeof(int);
}

template <int A, int B>
static void launch_screen_t(const ScreenArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_screen<A, B>), dim3((unsigned)a.n_pairs), dim3(kWave),
                     screen_lds_bytes(a.max_q, a.max_b), st, a);
}

hipError_t launch_screen(const ScreenArgs& a, int variant, hipStream_t st) {
  switch (variant) {
    case 0: launch_screen_t<4, 2>(a, st); break;
    case 1: launch_screen_t<2, 2>(a, st); break;
    case 2: launch_screen_t<4, 1>(a, st); break;
    case 3: launch_screen_t<4, 4>(a, st); break;
    case 4: launch_screen_t<8, 2>(a, st); break;
    case 5: launch_screen_t<2, 1>(a, st); break;
    case 6: launch_screen_t<8, 4>(a, st); break;
    case 7: launch_screen_t<2, 4>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace shape
