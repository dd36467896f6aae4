// Hybrid pipeline (section "Differentiable alignment and the hybrid
// pipeline"): rigid alignment on the analytic first-order overlap (Eq. fo,
// exact and cheap) from multiple starts — the given pose, the four proper
// principal-axis alignments and random rotations — then scoring of the
// superposed pair by the union estimator (the screening kernels).
//
// Pose convention as in the IS alignment: c''_j = R(q/|q|) c_j + t for B's
// atoms, q = (w, x, y, z) unnormalised, rotation about B's coordinate origin.
//
//   T_FO = O / (O_AA + O_BB - O),  O = sum_ij K_ij,
//   K_ij = (pi/(a_i+a_j))^(3/2) exp(-k_ij |c_i - c''_j|^2), k_ij = a_i a_j/(a_i+a_j)
//   dO/dc''_j = sum_i 2 k_ij K_ij (c_i - c''_j)
//   dO/dt = sum_j dO/dc''_j,  dO/dtheta = sum_j (c''_j - t) x dO/dc''_j
// and dT/dq follows from dtheta = 2 (w dv - dw v + v x dv) for q = (w, v).
#include "shape_kernels.hpp"

#include <math.h>

namespace shape {

// ---------------------------------------------------------------------------
// Starts: one thread per pair, FP64.
// ---------------------------------------------------------------------------

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations: eigenvalues
// descending, unit eigenvectors in the columns of V (row-major).
__device__ void jacobi3(double a[3][3], double V[9]) {
  double U[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 60; ++sweep) {
    const double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
    if (off < 1e-300) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double ukp = U[k][p], ukq = U[k][q];
          U[k][p] = c * ukp - s * ukq;
          U[k][q] = s * ukp + c * ukq;
        }
      }
  }
  int idx[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (a[idx[j]][idx[j]] > a[idx[i]][idx[i]]) {
        const int t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
      }
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) V[3 * r + c] = U[r][idx[c]];
}

// Mixture mean and principal axes of one molecule (weights v_i / Z,
// v_i = (pi/alpha_i)^(3/2)); axes as columns of U, descending variance, the
// largest-magnitude component of the first two positive, U right-handed.
__device__ void principal_frame(const float* xyz, const float* alpha, int n, double mu[3],
                                double U[9]) {
  double Z = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double t = M_PI / (double)alpha[i];
    const double v = t * sqrt(t);
    Z += v;
    m0 += v * (double)xyz[3 * i];
    m1 += v * (double)xyz[3 * i + 1];
    m2 += v * (double)xyz[3 * i + 2];
  }
  mu[0] = m0 / Z;
  mu[1] = m1 / Z;
  mu[2] = m2 / Z;
  double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i = 0; i < n; ++i) {
    const double t = M_PI / (double)alpha[i];
    const double w = t * sqrt(t) / Z;
    const double x[3] = {(double)xyz[3 * i] - mu[0], (double)xyz[3 * i + 1] - mu[1],
                         (double)xyz[3 * i + 2] - mu[2]};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) C[r][c] += w * x[r] * x[c];
  }
  jacobi3(C, U);
  for (int c = 0; c < 2; ++c) {
    int big = 0;
    for (int r = 1; r < 3; ++r)
      if (fabs(U[3 * r + c]) > fabs(U[3 * big + c])) big = r;
    if (U[3 * big + c] < 0)
      for (int r = 0; r < 3; ++r) U[3 * r + c] = -U[3 * r + c];
  }
  U[2] = U[3] * U[7] - U[6] * U[4];
  U[5] = U[6] * U[1] - U[0] * U[7];
  U[8] = U[0] * U[4] - U[3] * U[1];
}

__device__ void rot_of_quat(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

// Unit quaternion (w >= 0) of a rotation matrix, largest-diagonal branch.
__device__ void quat_of_rot(const double R[9], double q[4]) {
  const double tr = R[0] + R[4] + R[8];
  double w, x, y, z;
  if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
    const double s = sqrt(1.0 + tr) * 2.0;
    w = 0.25 * s; x = (R[7] - R[5]) / s; y = (R[2] - R[6]) / s; z = (R[3] - R[1]) / s;
  } else if (R[0] >= R[4] && R[0] >= R[8]) {
    const double s = sqrt(1.0 + R[0] - R[4] - R[8]) * 2.0;
    w = (R[7] - R[5]) / s; x = 0.25 * s; y = (R[1] + R[3]) / s; z = (R[2] + R[6]) / s;
  } else if (R[4] >= R[8]) {
    const double s = sqrt(1.0 + R[4] - R[0] - R[8]) * 2.0;
    w = (R[2] - R[6]) / s; x = (R[1] + R[3]) / s; y = 0.25 * s; z = (R[5] + R[7]) / s;
  } else {
    const double s = sqrt(1.0 + R[8] - R[0] - R[4]) * 2.0;
    w = (R[3] - R[1]) / s; x = (R[2] + R[6]) / s; y = (R[5] + R[7]) / s; z = 0.25 * s;
  }
  const double sg = w < 0 ? -1.0 : 1.0;
  q[0] = sg * w; q[1] = sg * x; q[2] = sg * y; q[3] = sg * z;
}

__global__ void k_fo_starts(MolsDev A, MolsDev B, const int* __restrict__ badA,
                            const int* __restrict__ badB, int n_random, uint2 key,
                            float* __restrict__ pose) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B.n_mols) return;
  const int n_starts = 5 + n_random;
  float* out = pose + (size_t)p * n_starts * 7;
  const int ma = A.n_mols == 1 ? 0 : p;
  if (badA[ma] != 0 || badB[p] != 0) {
    for (int c = 0; c < n_starts * 7; ++c) out[c] = __builtin_nanf("");
    return;
  }
  const int a0 = A.off[ma], na = A.off[ma + 1] - a0;
  const int b0 = B.off[p], nb = B.off[p + 1] - b0;
  out[0] = 1.f;
  for (int c = 1; c < 7; ++c) out[c] = 0.f;
  double muA[3], UA[9], muB[3], UB[9];
  principal_frame(A.xyz + 3 * (size_t)a0, A.alpha + a0, na, muA, UA);
  principal_frame(B.xyz + 3 * (size_t)b0, B.alpha + b0, nb, muB, UB);
  const double Ds[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
  for (int s = 0; s < 4 + n_random; ++s) {
    double R[9];
    if (s < 4) {
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double acc = 0.0;
          for (int k = 0; k < 3; ++k) acc += UA[3 * r + k] * Ds[s][k] * UB[3 * c + k];
          R[3 * r + c] = acc;
        }
    } else {
      // uniform rotation (Shoemake) from three 24-bit uniforms
      const uint4 x = philox4x32_10(make_uint4((uint32_t)(s - 4), (uint32_t)p, 0x5157A27u, 0u),
                                    key);
      const double u1 = ((double)(x.x >> 8) + 0.5) * 0x1p-24;
      const double u2 = ((double)(x.y >> 8) + 0.5) * 0x1p-24;
      const double u3 = ((double)(x.z >> 8) + 0.5) * 0x1p-24;
      const double q[4] = {sqrt(u1) * cos(2 * M_PI * u3), sqrt(1 - u1) * sin(2 * M_PI * u2),
                           sqrt(1 - u1) * cos(2 * M_PI * u2), sqrt(u1) * sin(2 * M_PI * u3)};
      rot_of_quat(q, R);
    }
    double q[4];
    quat_of_rot(R, q);
    float* o = out + 7 * (1 + s);
    for (int i = 0; i < 4; ++i) o[i] = (float)q[i];
    for (int a = 0; a < 3; ++a)
      o[4 + a] = (float)(muA[a] - (R[3 * a] * muB[0] + R[3 * a + 1] * muB[1] +
                                   R[3 * a + 2] * muB[2]));
  }
}

// ---------------------------------------------------------------------------
// First-order alignment: one wave per (pair, start); Adam runs inside the
// kernel, the pose and its moments stay in registers (wave-uniform).
// ---------------------------------------------------------------------------
// Row layout: at most kFoRowsStarts starts (rows of 16 lanes) per
// workgroup; moved-atom arrays of the rows at a stride of s float4 with
// s = 2 (mod 8), so the four rows of a wave read their broadcast atoms from
// four disjoint groups of LDS banks.
constexpr int kFoRowsStarts = 16;
constexpr size_t kFoRowsLdsMax = 48 * 1024;
__host__ __device__ inline int fo_rows_stride(int max_b) {
  return max_b + (((2 - max_b) % 8) + 8) % 8;
}

struct FoAlignArgs {
  MolsDev A, B;
  const int* badA;  // invalid-molecule flags of the prepared sets
  const int* badB;
  int n_starts, n_steps;
  float lr;
  float* pose;  // [pairs][starts][7], read and written
  float* T;     // [pairs][starts]
  float* grad;  // [pairs][starts][7] at the final pose, or nullptr
  const int* order;  // optional launch order of the row layout: block x takes pair order[x]
};

// One pass over the N_A x N_B atom pairs spread over the lanes (the row of
// flat index p stepped incrementally, as in the cross-overlap kernel):
// O, dO/dt and the torque about B's origin, summed over the wave.  Per term,
// the pose-independent factors come from the widths alone: with
// rs = 1/sqrt(a_i + a_j), (pi/(a_i+a_j))^(3/2) = pi^(3/2) rs^3 and
// k_ij = a_i a_j rs^2.  A lane's first kFoCache terms keep them in registers
// for the whole optimisation (fo_term_consts, filled once per wave); later
// terms derive them on the spot from one rsqrt.  The torque is accumulated
// as sum c''_j x f and shifted by -t x sum f once at the end.
constexpr int kFoCache = 16;

struct FoTermConsts {
  float kk[kFoCache];   // -log2(e) k_ij
  float pre[kFoCache];  // pi^(3/2) (a_i + a_j)^(-3/2)
  float f2[kFoCache];   // 2 k_ij
};

__device__ __forceinline__ void fo_consts(float ai, float aj, float& kk, float& pre, float& f2) {
  const float rs = __builtin_amdgcn_rsqf(ai + aj);
  const float ir = rs * rs;
  const float k = ai * aj * ir;
  kk = -1.44269504088896f * k;
  pre = 5.56832799683170785f * ir * rs;
  f2 = 2.f * k;
}

__device__ __forceinline__ void fo_term_consts(const float4* sA, int na, const float4* sB,
                                               int nb, FoTermConsts& c) {
  const int lane = threadIdx.x & (kWave - 1);
  const int di = kWave / nb, dj = kWave % nb;
  int i = lane / nb, j = lane % nb;
#pragma unroll
  for (int t = 0; t < kFoCache; ++t) {
    c.kk[t] = 0.f;
    c.pre[t] = 0.f;
    c.f2[t] = 0.f;
    if (i < na) {
      fo_consts(sA[i].w, sB[j].w, c.kk[t], c.pre[t], c.f2[t]);
      i += di;
      j += dj;
      if (j >= nb) {
        j -= nb;
        ++i;
      }
    }
  }
}

struct FoAcc {
  float O = 0.f, gx = 0.f, gy = 0.f, gz = 0.f, rx = 0.f, ry = 0.f, rz = 0.f;
  __device__ __forceinline__ void add(const float4& ci, const float4& cj, float kk, float pre,
                                      float f2) {
    const float dx = ci.x - cj.x, dy = ci.y - cj.y, dz = ci.z - cj.z;
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float K = pre * __builtin_amdgcn_exp2f(kk * d2);
    O += K;
    const float f = f2 * K;
    const float fx = f * dx, fy = f * dy, fz = f * dz;  // dO/dc''_j from this term
    gx += fx; gy += fy; gz += fz;
    rx = fmaf(cj.y, fz, fmaf(-cj.z, fy, rx));
    ry = fmaf(cj.z, fx, fmaf(-cj.x, fz, ry));
    rz = fmaf(cj.x, fy, fmaf(-cj.y, fx, rz));
  }
};

__device__ __forceinline__ void fo_pass(const float4* sA, int na, const float4* sM, int nb,
                                        float tx, float ty, float tz, const FoTermConsts& c,
                                        float (&r)[7]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int di = kWave / nb, dj = kWave % nb;
  int i = lane / nb, j = lane % nb;
  FoAcc acc;
#pragma unroll
  for (int t = 0; t < kFoCache; ++t) {
    if (i < na) {
      acc.add(sA[i], sM[j], c.kk[t], c.pre[t], c.f2[t]);
      i += di;
      j += dj;
      if (j >= nb) {
        j -= nb;
        ++i;
      }
    }
  }
  for (; i < na;) {
    const float4 ci = sA[i], cj = sM[j];
    float kk, pre, f2;
    fo_consts(ci.w, cj.w, kk, pre, f2);
    acc.add(ci, cj, kk, pre, f2);
    i += di;
    j += dj;
    if (j >= nb) {
      j -= nb;
      ++i;
    }
  }
  r[0] = wave_sum_dpp(acc.O);
  r[1] = wave_sum_dpp(acc.gx); r[2] = wave_sum_dpp(acc.gy); r[3] = wave_sum_dpp(acc.gz);
  // torque about B's origin: sum (c''_j - t) x f = sum c''_j x f - t x sum f
  r[4] = wave_sum_dpp(acc.rx) - (ty * r[3] - tz * r[2]);
  r[5] = wave_sum_dpp(acc.ry) - (tz * r[1] - tx * r[3]);
  r[6] = wave_sum_dpp(acc.rz) - (tx * r[2] - ty * r[1]);
}

// sum_ij K_ij of a molecule with itself (pose invariant), over all lanes.
__device__ __forceinline__ float fo_self(const float4* s, int n) {
  const int lane = threadIdx.x & (kWave - 1);
  const int di = kWave / n, dj = kWave % n;
  int i = lane / n, j = lane % n;
  float acc = 0.f;
  for (; i < n;) {
    const float4 ci = s[i], cj = s[j];
    const float sa = ci.w + cj.w;
    const float ir = __builtin_amdgcn_rcpf(sa);
    const float dx = ci.x - cj.x, dy = ci.y - cj.y, dz = ci.z - cj.z;
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float t = 3.14159265358979f * ir;
    acc += t * __builtin_amdgcn_sqrtf(t) *
           __builtin_amdgcn_exp2f(-1.44269504088896f * ci.w * cj.w * ir * d2);
    i += di;
    j += dj;
    if (j >= n) {
      j -= n;
      ++i;
    }
  }
  return wave_sum_dpp(acc);
}

__global__ __launch_bounds__(64) void k_fo_align(FoAlignArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int item = blockIdx.x;  // pair * n_starts + start
  const int pair = item / a.n_starts;
  const int ma = a.A.n_mols == 1 ? 0 : pair;
  if (a.badA[ma] != 0 || a.badB[pair] != 0) {
    if (lane == 0) {
      a.T[item] = __builtin_nanf("");
      if (a.grad)
        for (int c = 0; c < 7; ++c) a.grad[(size_t)item * 7 + c] = __builtin_nanf("");
    }
    return;
  }
  const int a0 = a.A.off[ma], na = a.A.off[ma + 1] - a0;
  const int b0 = a.B.off[pair], nb = a.B.off[pair + 1] - b0;
  float4* sA = reinterpret_cast<float4*>(smem);  // [max_a] x, y, z, alpha
  float4* sB = sA + a.A.max_atoms;               // [max_b] B as given
  float4* sM = sB + a.B.max_atoms;               // [max_b] B moved
  for (int i = lane; i < na; i += kWave)
    sA[i] = make_float4(a.A.xyz[3 * (a0 + i)], a.A.xyz[3 * (a0 + i) + 1],
                        a.A.xyz[3 * (a0 + i) + 2], a.A.alpha[a0 + i]);
  for (int j = lane; j < nb; j += kWave)
    sB[j] = make_float4(a.B.xyz[3 * (b0 + j)], a.B.xyz[3 * (b0 + j) + 1],
                        a.B.xyz[3 * (b0 + j) + 2], a.B.alpha[b0 + j]);
  wave_lds_sync();
  const float S = fo_self(sA, na) + fo_self(sB, nb);  // O_AA + O_BB
  FoTermConsts tc;
  fo_term_consts(sA, na, sB, nb, tc);
  // pose x (wave-uniform); lane c < 7 holds component c of the Adam state
  float x[7];
  float* ps = a.pose + (size_t)item * 7;
#pragma unroll
  for (int c = 0; c < 7; ++c) x[c] = ps[c];
  const int mine = lane < 7 ? lane : 6;
  float m_l = 0.f, v_l = 0.f;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float b1t = 1.f, b2t = 1.f;  // b1^t, b2^t as running products
  float T = 0.f, g[7];
  for (int it = 0; it <= a.n_steps; ++it) {
    // move B by the current pose
    const float n2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3];
    const float in = rsqrtf(n2);
    const float qw = x[0] * in, qx = x[1] * in, qy = x[2] * in, qz = x[3] * in;
    const float R0 = 1.f - 2.f * (qy * qy + qz * qz), R1 = 2.f * (qx * qy - qw * qz),
                R2 = 2.f * (qx * qz + qw * qy), R3 = 2.f * (qx * qy + qw * qz),
                R4 = 1.f - 2.f * (qx * qx + qz * qz), R5 = 2.f * (qy * qz - qw * qx),
                R6 = 2.f * (qx * qz - qw * qy), R7 = 2.f * (qy * qz + qw * qx),
                R8 = 1.f - 2.f * (qx * qx + qy * qy);
    for (int j = lane; j < nb; j += kWave) {
      const float4 c = sB[j];
      sM[j] = make_float4(fmaf(R0, c.x, fmaf(R1, c.y, fmaf(R2, c.z, x[4]))),
                          fmaf(R3, c.x, fmaf(R4, c.y, fmaf(R5, c.z, x[5]))),
                          fmaf(R6, c.x, fmaf(R7, c.y, fmaf(R8, c.z, x[6]))), c.w);
    }
    wave_lds_sync();
    float r[7];
    fo_pass(sA, na, sM, nb, x[4], x[5], x[6], tc, r);
    wave_lds_sync();  // sM is rewritten next step
    const float D = S - r[0];
    T = r[0] / D;
    const float iD = __builtin_amdgcn_rcpf(D);
    const float dTdO = S * iD * iD;
    const float gth[3] = {dTdO * r[4], dTdO * r[5], dTdO * r[6]};
    // dT/dq = (2/|q|) [ -v.g ; w g - v x g ]
    const float vdg = qx * gth[0] + qy * gth[1] + qz * gth[2];
    g[0] = 2.f * in * (-vdg);
    g[1] = 2.f * in * (qw * gth[0] - (qy * gth[2] - qz * gth[1]));
    g[2] = 2.f * in * (qw * gth[1] - (qz * gth[0] - qx * gth[2]));
    g[3] = 2.f * in * (qw * gth[2] - (qx * gth[1] - qy * gth[0]));
    g[4] = dTdO * r[1];
    g[5] = dTdO * r[2];
    g[6] = dTdO * r[3];
    if (it == a.n_steps) break;
    // Adam on -T (bias-corrected moments, betas 0.9 / 0.999), q renormalised;
    // reciprocals by the hardware (a step of length ~lr tolerates 1 ulp).
    // Lane c < 7 updates component c; the new pose is gathered by readlane.
    b1t *= b1;
    b2t *= b2;
    const float ic1 = __builtin_amdgcn_rcpf(1.f - b1t), ic2 = __builtin_amdgcn_rcpf(1.f - b2t);
    float g_l = g[0], x_l = x[0];
#pragma unroll
    for (int c = 1; c < 7; ++c) {
      g_l = mine == c ? g[c] : g_l;
      x_l = mine == c ? x[c] : x_l;
    }
    const float gc = -g_l;
    m_l = fmaf(b1, m_l, (1.f - b1) * gc);
    v_l = fmaf(b2, v_l, (1.f - b2) * gc * gc);
    const float den = __builtin_amdgcn_sqrtf(v_l * ic2) + eps;
    const float xn_l = x_l - a.lr * (m_l * ic1) * __builtin_amdgcn_rcpf(den);
    float xn[7];
#pragma unroll
    for (int c = 0; c < 7; ++c)
      xn[c] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, xn_l), c));
    const float inv = rsqrtf(xn[0] * xn[0] + xn[1] * xn[1] + xn[2] * xn[2] + xn[3] * xn[3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = xn[c] * inv;
#pragma unroll
    for (int c = 4; c < 7; ++c) x[c] = xn[c];
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 7; ++c) ps[c] = x[c];
    a.T[item] = T;
    if (a.grad)
#pragma unroll
      for (int c = 0; c < 7; ++c) a.grad[(size_t)item * 7 + c] = g[c];
  }
}

// ---------------------------------------------------------------------------
// First-order alignment, row layout: one workgroup per pair and up to 16
// starts, one start per 16-lane row of a wave, so the per-step work that
// does not scale with the atom pairs (rotation, reductions, Adam) is shared
// by four starts per wave instruction.  Lane l of a row owns A's atoms
// i = l + 16 r (r < RA; rows past N_A are padding whose terms add exactly
// 0) and walks all of B's moved atoms, read as LDS
// broadcasts.  The pose-independent constants of every atom pair,
// kk = -log2(e) k_ij and lq = log2((pi/(a_i+a_j))^(3/2)) + kk |c_i|^2 (A's
// atoms do not move), sit in an LDS table filled once per workgroup (padding
// rows: kk = 0, lq = -inf, so K = 0).  Per term, with d = c_i - c''_j and
// |d|^2 = |c_i|^2 + |c''_j|^2 + (-2 c_i) . c''_j:
//   K = exp2(kk (|c''_j|^2 + (-2 c_i) . c''_j) + lq)   (|c''_j|^2 stored
//       with the moved atom)
// (FP32 emulation on drug-sized molecules at random poses against FP64:
// relative error of O at most 7.7e-7, of its gradient 2.2e-6 (1.0e-6 and
// 3.3e-6 with |c_i|^2 added per term); 10 VALU + exp per term.)
// and the lane keeps O_i = sum_j K, W_i = sum_j kk K, P_i = sum_j kk K c''_j,
// so that F_i = sum_j kk K d = c_i W_i - P_i.  Since dO/dc''_j is parallel to d,
// c''_j x (s d) = c_i x (s d), so the torque about B's origin is
// sum_i c_i x F_i less t x sum F, formed once per lane instead of per term;
// dO/dc''_j = 2 k K d = -2 ln(2) kk K d scales F once at the end.
// Every lane of a row holds the same pose and gradient (row sums leave
// identical bits in all 16 lanes); Adam's seven components are updated one
// per lane (lanes 0-6 of the row, with their moments) and read back by the
// whole row, instead of all seven in every lane.
// ---------------------------------------------------------------------------
template <int RA>
__global__ __launch_bounds__(256) void k_fo_align_rows(FoAlignArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int RA16 = RA * 16;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int l16 = lane & 15, row = lane >> 4;
  const int pair = a.order ? a.order[blockIdx.x] : xcd_chunk(blockIdx.x, gridDim.x);
  const int s_raw = blockIdx.y * kFoRowsStarts + wave * 4 + row;
  const bool live = s_raw < a.n_starts;
  const int s = live ? s_raw : a.n_starts - 1;  // spare rows repeat the last start
  const size_t item = (size_t)pair * a.n_starts + s;
  const int ma = a.A.n_mols == 1 ? 0 : pair;
  if (a.badA[ma] != 0 || a.badB[pair] != 0) {
    if (live && l16 == 0) {
      a.T[item] = __builtin_nanf("");
      if (a.grad)
        for (int c = 0; c < 7; ++c) a.grad[item * 7 + c] = __builtin_nanf("");
    }
    return;
  }
  const int a0 = a.A.off[ma], na = a.A.off[ma + 1] - a0;
  const int b0 = a.B.off[pair], nb = a.B.off[pair + 1] - b0;
  const int stride = fo_rows_stride(a.B.max_atoms);
  const int n_rows = (int)(blockDim.x / 16);
  float4* sA = reinterpret_cast<float4*>(smem);  // [max_a] x, y, z, alpha
  float4* sB = sA + a.A.max_atoms;               // [max_b] B as given
  float4* sM = sB + a.B.max_atoms;               // [rows][stride] B moved, per start
  float2* tab = reinterpret_cast<float2*>(sM + (size_t)n_rows * stride);  // [max_b][RA16]
  for (int i = tid; i < na; i += blockDim.x)
    sA[i] = make_float4(a.A.xyz[3 * (a0 + i)], a.A.xyz[3 * (a0 + i) + 1],
                        a.A.xyz[3 * (a0 + i) + 2], a.A.alpha[a0 + i]);
  for (int j = tid; j < nb; j += blockDim.x)
    sB[j] = make_float4(a.B.xyz[3 * (b0 + j)], a.B.xyz[3 * (b0 + j) + 1],
                        a.B.xyz[3 * (b0 + j) + 2], a.B.alpha[b0 + j]);
  __syncthreads();
  for (int e = tid; e < nb * RA16; e += blockDim.x) {
    const int j = e / RA16, i = e % RA16;
    float kk = 0.f, pre = 0.f, f2, lq = -INFINITY;
    if (i < na) {
      const float4 c = sA[i];
      fo_consts(c.w, sB[j].w, kk, pre, f2);
      lq = fmaf(kk, norm2(c.x, c.y, c.z), log2f(pre));
    }
    tab[e] = make_float2(kk, lq);
  }
  __syncthreads();
  const float S = fo_self(sA, na) + fo_self(sB, nb);  // O_AA + O_BB
  float cx[RA], cy[RA], cz[RA];
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    const int i = l16 + 16 * r;
    const float4 c = i < na ? sA[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    cx[r] = c.x;
    cy[r] = c.y;
    cz[r] = c.z;
  }
  float4* mine = sM + (size_t)(wave * 4 + row) * stride;
  const float2* trow = tab + l16;
  // the pose in every lane of the row; Adam's moments of component
  // cA = min(l16, 6) in lane l16 (lanes past 6 repeat component 6)
  float x[7];
  float* ps = a.pose + item * 7;
#pragma unroll
  for (int c = 0; c < 7; ++c) x[c] = ps[c];
  const int cA = l16 < 7 ? l16 : 6;
  float mA = 0.f, vA = 0.f;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float b1t = 1.f, b2t = 1.f;
  float T = 0.f, g[7];
  for (int it = 0; it <= a.n_steps; ++it) {
    const float n2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3];
    const float in = rsqrtf(n2);
    const float qw = x[0] * in, qx = x[1] * in, qy = x[2] * in, qz = x[3] * in;
    const float R0 = 1.f - 2.f * (qy * qy + qz * qz), R1 = 2.f * (qx * qy - qw * qz),
                R2 = 2.f * (qx * qz + qw * qy), R3 = 2.f * (qx * qy + qw * qz),
                R4 = 1.f - 2.f * (qx * qx + qz * qz), R5 = 2.f * (qy * qz - qw * qx),
                R6 = 2.f * (qx * qz - qw * qy), R7 = 2.f * (qy * qz + qw * qx),
                R8 = 1.f - 2.f * (qx * qx + qy * qy);
    for (int j = l16; j < nb; j += 16) {
      const float4 c = sB[j];
      const float mx = fmaf(R0, c.x, fmaf(R1, c.y, fmaf(R2, c.z, x[4])));
      const float my = fmaf(R3, c.x, fmaf(R4, c.y, fmaf(R5, c.z, x[5])));
      const float mz = fmaf(R6, c.x, fmaf(R7, c.y, fmaf(R8, c.z, x[6])));
      mine[j] = make_float4(mx, my, mz, norm2(mx, my, mz));
    }
    wave_lds_sync();
    float O[RA], W[RA], Px[RA], Py[RA], Pz[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) O[r] = W[r] = Px[r] = Py[r] = Pz[r] = 0.f;
#pragma unroll 4
    for (int j = 0; j < nb; ++j) {
      const float4 cj = mine[j];
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        const float2 kp = trow[j * RA16 + 16 * r];
        const float e = fmaf(-2.f * cx[r], cj.x,
                             fmaf(-2.f * cy[r], cj.y, fmaf(-2.f * cz[r], cj.z, cj.w)));
        const float K = __builtin_amdgcn_exp2f(fmaf(kp.x, e, kp.y));
        O[r] += K;
        const float fs = kp.x * K;
        W[r] += fs;
        Px[r] = fmaf(fs, cj.x, Px[r]);
        Py[r] = fmaf(fs, cj.y, Py[r]);
        Pz[r] = fmaf(fs, cj.z, Pz[r]);
      }
    }
    wave_lds_sync();  // this start's moved atoms are rewritten next step
    float Fx[RA], Fy[RA], Fz[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      Fx[r] = fmaf(cx[r], W[r], -Px[r]);
      Fy[r] = fmaf(cy[r], W[r], -Py[r]);
      Fz[r] = fmaf(cz[r], W[r], -Pz[r]);
    }
    float o = O[0], fx = Fx[0], fy = Fy[0], fz = Fz[0];
    float tx = cy[0] * Fz[0] - cz[0] * Fy[0], ty = cz[0] * Fx[0] - cx[0] * Fz[0],
          tz = cx[0] * Fy[0] - cy[0] * Fx[0];
#pragma unroll
    for (int r = 1; r < RA; ++r) {
      o += O[r];
      fx += Fx[r];
      fy += Fy[r];
      fz += Fz[r];
      tx += cy[r] * Fz[r] - cz[r] * Fy[r];
      ty += cz[r] * Fx[r] - cx[r] * Fz[r];
      tz += cx[r] * Fy[r] - cy[r] * Fx[r];
    }
    const float sc = -1.38629436111989061f;  // -2 ln 2
    float r7[7];
    r7[0] = row_sum16(o);
    r7[1] = sc * row_sum16(fx);
    r7[2] = sc * row_sum16(fy);
    r7[3] = sc * row_sum16(fz);
    // torque about B's origin: sum c_i x F_i - t x sum F
    r7[4] = sc * row_sum16(tx) - (x[5] * r7[3] - x[6] * r7[2]);
    r7[5] = sc * row_sum16(ty) - (x[6] * r7[1] - x[4] * r7[3]);
    r7[6] = sc * row_sum16(tz) - (x[4] * r7[2] - x[5] * r7[1]);
    const float D = S - r7[0];
    const float iD = __builtin_amdgcn_rcpf(D);
    const float dTdO = S * iD * iD;
    const float gth[3] = {dTdO * r7[4], dTdO * r7[5], dTdO * r7[6]};
    const float vdg = qx * gth[0] + qy * gth[1] + qz * gth[2];
    g[0] = 2.f * in * (-vdg);
    g[1] = 2.f * in * (qw * gth[0] - (qy * gth[2] - qz * gth[1]));
    g[2] = 2.f * in * (qw * gth[1] - (qz * gth[0] - qx * gth[2]));
    g[3] = 2.f * in * (qw * gth[2] - (qx * gth[1] - qy * gth[0]));
    g[4] = dTdO * r7[1];
    g[5] = dTdO * r7[2];
    g[6] = dTdO * r7[3];
    if (it == a.n_steps) {
      T = r7[0] / D;  // only the final pose's T is returned
      break;
    }
    // Adam on -T, the one-start-per-wave kernel's arithmetic: lane l16 < 7
    // of the row updates component l16, then the row reads the seven new
    // components back from those lanes
    b1t *= b1;
    b2t *= b2;
    const float ic1 = __builtin_amdgcn_rcpf(1.f - b1t), ic2 = __builtin_amdgcn_rcpf(1.f - b2t);
    float gA = g[0], xA = x[0];
#pragma unroll
    for (int c = 1; c < 7; ++c) {
      if (cA == c) {
        gA = g[c];
        xA = x[c];
      }
    }
    {
      const float gc = -gA;
      mA = fmaf(b1, mA, (1.f - b1) * gc);
      vA = fmaf(b2, vA, (1.f - b2) * gc * gc);
      const float den = __builtin_amdgcn_sqrtf(vA * ic2) + eps;
      xA = xA - a.lr * (mA * ic1) * __builtin_amdgcn_rcpf(den);
    }
    float xn[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) xn[c] = __shfl(xA, (lane & ~15) + c, kWave);
    const float inv = rsqrtf(xn[0] * xn[0] + xn[1] * xn[1] + xn[2] * xn[2] + xn[3] * xn[3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = xn[c] * inv;
#pragma unroll
    for (int c = 4; c < 7; ++c) x[c] = xn[c];
  }
  if (live && l16 == 0) {
#pragma unroll
    for (int c = 0; c < 7; ++c) ps[c] = x[c];
    a.T[item] = T;
    if (a.grad)
#pragma unroll
      for (int c = 0; c < 7; ++c) a.grad[item * 7 + c] = g[c];
  }
}

// Best start per pair (largest T; lowest index on ties; NaN never wins):
// its pose and T.
__global__ void k_best_pose(const float* __restrict__ T, const float* __restrict__ pose,
                            int n_pairs, int n_starts, float* __restrict__ best_pose,
                            float* __restrict__ best_T) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  int b = 0;
  float bv = -INFINITY;
  for (int s = 0; s < n_starts; ++s) {
    const float t = T[(size_t)p * n_starts + s];
    if (t > bv) {
      bv = t;
      b = s;
    }
  }
  const float* src = pose + ((size_t)p * n_starts + b) * 7;
  for (int c = 0; c < 7; ++c) best_pose[(size_t)p * 7 + c] = src[c];
  if (best_T) best_T[p] = T[(size_t)p * n_starts + b];
}

// Conformer ensembles: the largest T of each group of consecutive entries
// (max over conformers); lowest index on ties, NaN never wins (a group of
// NaN gives NaN and index -1).
__global__ void k_group_max(const float* __restrict__ T, int64_t n_T, const int* __restrict__ goff,
                            int n_groups, float* __restrict__ best_T, int* __restrict__ best_idx,
                            int* __restrict__ flag) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  int b = -1;
  float bv = -INFINITY;
  const int e0 = goff[g], e1 = goff[g + 1];
  if (e0 < 0 || e1 > n_T || e1 < e0) {
    // a group outside T (or reversed) reads nothing: NaN, -1, data error
    best_T[g] = __builtin_nanf("");
    if (best_idx) best_idx[g] = -1;
    atomicOr(flag, 1);
    return;
  }
  for (int e = e0; e < e1; ++e) {
    const float t = T[e];
    if (t > bv || (b < 0 && t == bv)) {
      bv = t;
      b = e;
    }
  }
  best_T[g] = b < 0 ? __builtin_nanf("") : bv;
  if (best_idx) best_idx[g] = b;
}

// Moved coordinates xyz_out = R(q/|q|) xyz + t, one wave per molecule.
__global__ __launch_bounds__(64) void k_apply_pose(MolsDev M, const float* __restrict__ pose,
                                                   float* __restrict__ out) {
  const int mol = blockIdx.x;
  if (mol >= M.n_mols) return;
  const float* x = pose + (size_t)mol * 7;
  const float in = rsqrtf(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
  const float qw = x[0] * in, qx = x[1] * in, qy = x[2] * in, qz = x[3] * in;
  const float R0 = 1.f - 2.f * (qy * qy + qz * qz), R1 = 2.f * (qx * qy - qw * qz),
              R2 = 2.f * (qx * qz + qw * qy), R3 = 2.f * (qx * qy + qw * qz),
              R4 = 1.f - 2.f * (qx * qx + qz * qz), R5 = 2.f * (qy * qz - qw * qx),
              R6 = 2.f * (qx * qz - qw * qy), R7 = 2.f * (qy * qz + qw * qx),
              R8 = 1.f - 2.f * (qx * qx + qy * qy);
  const int a0 = M.off[mol], a1 = M.off[mol + 1];
  for (int i = a0 + (int)threadIdx.x; i < a1; i += kWave) {
    const float cx = M.xyz[3 * i], cy = M.xyz[3 * i + 1], cz = M.xyz[3 * i + 2];
    out[3 * i] = fmaf(R0, cx, fmaf(R1, cy, fmaf(R2, cz, x[4])));
    out[3 * i + 1] = fmaf(R3, cx, fmaf(R4, cy, fmaf(R5, cz, x[5])));
    out[3 * i + 2] = fmaf(R6, cx, fmaf(R7, cy, fmaf(R8, cz, x[6])));
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_fo_starts(const MolsDev& A, const MolsDev& B, const int* badA,
                            const int* badB, int n_random, uint2 key, float* pose,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_fo_starts, dim3((B.n_mols + 63) / 64), dim3(64), 0, st, A, B, badA, badB,
                     n_random, key, pose);
  return hipGetLastError();
}

size_t fo_align_lds_bytes(int max_a, int max_b) {
  return (size_t)(max_a + 2 * max_b) * sizeof(float4);
}

// Row-layout launch shape: rows (starts) per workgroup and its LDS bytes, or
// 0 when the row kernel does not apply (A over 64 atoms, LDS beyond
// kFoRowsLdsMax, or more start blocks than a grid's y extent) and the
// one-start-per-wave kernel runs instead.
static int fo_rows_per_block(int n_starts) {
  return n_starts >= kFoRowsStarts ? kFoRowsStarts : ((n_starts + 3) / 4) * 4;
}
static size_t fo_rows_lds_bytes(int max_a, int max_b, int n_starts) {
  const int ra = (max_a + 15) / 16;
  if (ra > 4 || (n_starts + kFoRowsStarts - 1) / kFoRowsStarts > 65535) return 0;
  const size_t bytes = (size_t)(max_a + max_b) * sizeof(float4) +
                       (size_t)fo_rows_per_block(n_starts) * fo_rows_stride(max_b) *
                           sizeof(float4) +
                       (size_t)ra * 16 * max_b * sizeof(float2);
  return bytes <= kFoRowsLdsMax ? bytes : 0;
}

bool fo_align_pair_major(int max_a, int max_b, int n_starts) {
  return fo_rows_lds_bytes(max_a, max_b, n_starts) > 0;
}

template <int RA>
static void launch_fo_rows_t(const FoAlignArgs& a, size_t lds, hipStream_t st) {
  const int rows = fo_rows_per_block(a.n_starts);
  const int blocks_y = (a.n_starts + kFoRowsStarts - 1) / kFoRowsStarts;
  hipLaunchKernelGGL((k_fo_align_rows<RA>), dim3((unsigned)a.B.n_mols, (unsigned)blocks_y),
                     dim3(rows / 4 * kWave), lds, st, a);
}

hipError_t launch_fo_align(const MolsDev& A, const MolsDev& B, const int* badA, const int* badB,
                           int n_starts, int n_steps, float lr, float* pose, float* T,
                           float* grad, hipStream_t st, const int* order) {
  FoAlignArgs a{A, B, badA, badB, n_starts, n_steps, lr, pose, T, grad, nullptr};
  const size_t lds = fo_rows_lds_bytes(A.max_atoms, B.max_atoms, n_starts);
  if (lds > 0) {
    a.order = order;
    switch ((A.max_atoms + 15) / 16) {
      case 1: launch_fo_rows_t<1>(a, lds, st); break;
      case 2: launch_fo_rows_t<2>(a, lds, st); break;
      case 3: launch_fo_rows_t<3>(a, lds, st); break;
      default: launch_fo_rows_t<4>(a, lds, st); break;
    }
    return hipGetLastError();
  }
  const int64_t items = (int64_t)B.n_mols * n_starts;
  hipLaunchKernelGGL(k_fo_align, dim3((unsigned)items), dim3(kWave),
                     fo_align_lds_bytes(A.max_atoms, B.max_atoms), st, a);
  return hipGetLastError();
}

hipError_t launch_best_pose(const float* T, const float* pose, int n_pairs, int n_starts,
                            float* best_pose, float* best_T, hipStream_t st) {
  hipLaunchKernelGGL(k_best_pose, dim3((n_pairs + 255) / 256), dim3(256), 0, st, T, pose,
                     n_pairs, n_starts, best_pose, best_T);
  return hipGetLastError();
}

hipError_t launch_group_max(const float* T, int64_t n_T, const int* goff, int n_groups,
                            float* best_T, int* best_idx, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_group_max, dim3((n_groups + 255) / 256), dim3(256), 0, st, T, n_T, goff,
                     n_groups, best_T, best_idx, flag);
  return hipGetLastError();
}

hipError_t launch_apply_pose(const MolsDev& M, const float* pose, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_apply_pose, dim3((unsigned)M.n_mols), dim3(kWave), 0, st, M, pose, out);
  return hipGetLastError();
}

}  // namespace shape
