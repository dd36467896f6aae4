// Differentiable rigid alignment (section "Differentiable alignment and the
// hybrid pipeline", Eqs. pose and grad): value and pose gradient of the
// aligned Tanimoto under common random numbers, and the Adam update.
//
// B is moved rigidly, c''_j = R(q/|q|) c_j + t; A's first n samples r_k and
// weights w_A(r_k) stay fixed, so
//   O(xi) = Z_A/n sum_k w_A(r_k) u_B(r_k; xi),  T = O / (O_aa + O_bb - O).
// Gradient of u_B at one point: du/dc''_j = beta_j (r - c''_j) with
// beta_j = 2 alpha_j o_j prod_{k != j} (1 - o_k).  With B0 = sum beta_j and
// C = sum beta_j c''_j (both carried through the atom loop by a forward
// recurrence, no division by 1 - o_j):
//   du/dt     = B0 r - C
//   du/dtheta = C x r - t' x (B0 r - C)     (infinitesimal rotation about B's
//                                             origin, t' = B's origin)
// and dT/dq follows from dtheta = 2 (w dv - dw v + v x dv) for q = (w, v).
#include "shape_kernels.hpp"

#include <math.h>

namespace shape {

constexpr int kAlignThreads = 256;
constexpr int kAlignWaves = kAlignThreads / kWave;
constexpr int kAS = 4;  // points per lane evaluated together

__device__ __forceinline__ void quat_rotation(float qw, float qx, float qy, float qz,
                                              float (&R)[9], float& inv_norm) {
  const float n2 = qw * qw + qx * qx + qy * qy + qz * qz;
  inv_norm = rsqrtf(n2);
  const float w = qw * inv_norm, x = qx * inv_norm, y = qy * inv_norm, z = qz * inv_norm;
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}

// Phase 1 (whole workgroup): A's samples in A's frame and their weights.
__device__ void align_samples(const AlignArgs& a, int pair, float4* sSamp, Atom* sAF,
                              AtomSampling* sAS, AtomRec* sAR, float* sAa) {
  const int a0 = a.offA[pair], na = a.offA[pair + 1] - a0;
  const float4 cA = a.A.centre[pair];
  for (int i = threadIdx.x; i < na; i += blockDim.x) {
    const Atom at = a.A.atom[a0 + i];
    Atom f = at;
    f.x = at.x - cA.x;
    f.y = at.y - cA.y;
    f.z = at.z - cA.z;
    sAF[i] = f;
    sAS[i] = a.A.samp[a0 + i];
    make_rec(at, cA.x, cA.y, cA.z, sAR[i], sAa[i]);
  }
  __syncthreads();
  const uint32_t ida = a.A.id[pair];
  for (int k = threadIdx.x; k < a.n_samples; k += blockDim.x) {
    float rx[1], ry[1], rz[1], r2[1], m[1] = {0.f}, u[1] = {0.f};
    sample_point(sAF, sAS, na, ida, (uint64_t)k, a.key, rx[0], ry[0], rz[0]);
    r2[0] = norm2(rx[0], ry[0], rz[0]);
    eval_density_u_x<1>(sAR, sAa, na, rx, ry, rz, r2, m, u);
    sSamp[k] = make_float4(rx[0], ry[0], rz[0], bounded_weight(u[0], m[0]));
  }
  __syncthreads();
}

// One Adam (Kingma and Ba) ascent step on T for a pose x[7] with moments
// m, v: step number t (from 1), gradient dT; the quaternion is renormalised.
// Shared by the fused optimisation in k_align and by k_adam_pose, so both
// take the same roundings.
__device__ __forceinline__ void adam_pose_step(float (&x)[7], float (&m)[7], float (&v)[7],
                                               const float (&dT)[7], int t, float lr, float b1,
                                               float b2, float eps) {
#pragma clang fp contract(off)
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  float xn[7];
#pragma unroll
  for (int c = 0; c < 7; ++c) {
    const float g = -dT[c];  // minimise -T
    m[c] = fmaf(b1, m[c], (1.f - b1) * g);
    v[c] = fmaf(b2, v[c], (1.f - b2) * g * g);
    xn[c] = x[c] - lr * (m[c] / c1) / (sqrtf(v[c] / c2) + eps);
  }
  const float inv = rsqrtf(xn[0] * xn[0] + xn[1] * xn[1] + xn[2] * xn[2] + xn[3] * xn[3]);
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] = xn[c] * inv;
#pragma unroll
  for (int c = 4; c < 7; ++c) x[c] = xn[c];
}

__global__ __launch_bounds__(kAlignThreads) void k_align(AlignArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  // 16-byte arrays first, then 8-byte, then 4-byte: each stays aligned.
  float4* sSamp = reinterpret_cast<float4*>(smem);                    // [n_samples]
  AtomRec* sAR = reinterpret_cast<AtomRec*>(sSamp + a.n_samples);     // [max_a]
  Atom* sAF = reinterpret_cast<Atom*>(sAR + a.max_a);                 // [max_a]
  float4* sBC = reinterpret_cast<float4*>(sAF + a.max_a);             // [waves][max_b]
  AtomRec* sBR = reinterpret_cast<AtomRec*>(sBC + kAlignWaves * a.max_b);  // [waves][max_b]
  AtomSampling* sAS = reinterpret_cast<AtomSampling*>(sBR + kAlignWaves * a.max_b);  // [max_a]
  float* sAa = reinterpret_cast<float*>(sAS + a.max_a);                    // [max_a]
  float* sBa = sAa + a.max_a;                                              // [waves][max_b]

  const int pair = a.order ? a.order[blockIdx.x] : blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const bool bad = a.A.bad[pair] != 0 || a.B.bad[pair] != 0;
  if (bad) {
    for (int i = threadIdx.x; i < a.n_starts; i += blockDim.x) {
      const size_t o = (size_t)pair * a.n_starts + i;
      a.T[o] = __builtin_nanf("");
      if (a.grad)
        for (int c = 0; c < 7; ++c) a.grad[o * 7 + c] = __builtin_nanf("");
    }
    return;
  }
  align_samples(a, pair, sSamp, sAF, sAS, sAR, sAa);

  const int b0 = a.offB[pair], nb = a.offB[pair + 1] - b0;
  const float4 cA = a.A.centre[pair];
  const double Za = a.A.Z[pair];
  const double S = (double)a.O_aa[pair] + (double)a.O_bb[pair];
  AtomRec* wR = sBR + wave * a.max_b;
  float* wa = sBa + wave * a.max_b;
  float4* wC = sBC + wave * a.max_b;
  const int per_lane = (a.n_samples + kWave - 1) / kWave;

  for (int st = wave; st < a.n_starts; st += kAlignWaves) {
    const size_t o = (size_t)pair * a.n_starts + st;
    float ps[7], am[7], av[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      ps[c] = a.pose[o * 7 + c];
      am[c] = 0.f;
      av[c] = 0.f;
    }
    for (int it = 0;; ++it) {  // it = Adam steps taken
      float R[9], inv_norm;
      quat_rotation(ps[0], ps[1], ps[2], ps[3], R, inv_norm);
      // B's origin in A's frame (the rotation centre)
      const float tx = ps[4] - cA.x, ty = ps[5] - cA.y, tz = ps[6] - cA.z;
      for (int i = lane; i < nb; i += kWave) {
        const Atom at = a.B.atom[b0 + i];
        Atom moved = at;
        moved.x = fmaf(R[0], at.x, fmaf(R[1], at.y, fmaf(R[2], at.z, tx)));
        moved.y = fmaf(R[3], at.x, fmaf(R[4], at.y, fmaf(R[5], at.z, ty)));
        moved.z = fmaf(R[6], at.x, fmaf(R[7], at.y, fmaf(R[8], at.z, tz)));
        make_rec(moved, 0.f, 0.f, 0.f, wR[i], wa[i]);
        // 2 alpha_j (c''_j, 1), with 2 alpha = 2 a2 ln 2
        const float two_al = 2.0f * 0.693147180559945309f * at.a2;
        wC[i] = make_float4(two_al * moved.x, two_al * moved.y, two_al * moved.z, two_al);
      }
      wave_lds_sync();
      float accO = 0.f, gtx = 0.f, gty = 0.f, gtz = 0.f, grx = 0.f, gry = 0.f, grz = 0.f;
      for (int t = 0; t < per_lane; t += kAS) {
        float rx[kAS], ry[kAS], rz[kAS], r2[kAS], w[kAS];
        float P[kAS], S0[kAS], Sx[kAS], Sy[kAS], Sz[kAS];
#pragma unroll
        for (int s = 0; s < kAS; ++s) {
          const int k = lane + kWave * (t + s);
          const bool ok = (t + s) < per_lane && k < a.n_samples;
          const float4 c = sSamp[ok ? k : 0];
          rx[s] = c.x; ry[s] = c.y; rz[s] = c.z;
          w[s] = ok ? c.w : 0.f;
          r2[s] = norm2(c.x, c.y, c.z);
          P[s] = 1.f; S0[s] = 0.f; Sx[s] = 0.f; Sy[s] = 0.f; Sz[s] = 0.f;
        }
        // unrolled by two: no loop-carried register copies between atoms
#pragma unroll 2
        for (int j = 0; j < nb; ++j) {
          const AtomRec b = wR[j];
          const float aj = wa[j];
          const float4 cj = wC[j];
#pragma unroll
          for (int s = 0; s < kAS; ++s) {
            // S <- S (1 - o) + o P c  written as  S + o (c P - S): two fused
            // operations per component, and P <- P - o P
            const float oj = occupancy_x(b, aj, rx[s], ry[s], rz[s], r2[s]);
            S0[s] = fmaf(oj, fmaf(cj.w, P[s], -S0[s]), S0[s]);
            Sx[s] = fmaf(oj, fmaf(cj.x, P[s], -Sx[s]), Sx[s]);
            Sy[s] = fmaf(oj, fmaf(cj.y, P[s], -Sy[s]), Sy[s]);
            Sz[s] = fmaf(oj, fmaf(cj.z, P[s], -Sz[s]), Sz[s]);
            P[s] = fmaf(-oj, P[s], P[s]);
          }
        }
#pragma unroll
        for (int s = 0; s < kAS; ++s) {
          // translation gradient of u at this point and the torque about B's origin
          const float gx = fmaf(S0[s], rx[s], -Sx[s]);
          const float gy = fmaf(S0[s], ry[s], -Sy[s]);
          const float gz = fmaf(S0[s], rz[s], -Sz[s]);
          const float cxr_x = Sy[s] * rz[s] - Sz[s] * ry[s];
          const float cxr_y = Sz[s] * rx[s] - Sx[s] * rz[s];
          const float cxr_z = Sx[s] * ry[s] - Sy[s] * rx[s];
          const float txg_x = ty * gz - tz * gy;
          const float txg_y = tz * gx - tx * gz;
          const float txg_z = tx * gy - ty * gx;
          accO = fmaf(w[s], 1.f - P[s], accO);
          gtx = fmaf(w[s], gx, gtx);
          gty = fmaf(w[s], gy, gty);
          gtz = fmaf(w[s], gz, gtz);
          grx = fmaf(w[s], cxr_x - txg_x, grx);
          gry = fmaf(w[s], cxr_y - txg_y, gry);
          grz = fmaf(w[s], cxr_z - txg_z, grz);
        }
      }
      // butterfly sums: every lane holds the totals, so T and its gradient
      // are wave-uniform and the Adam state can stay in registers
      const double sO = wave_sum((double)accO);
      const double s_tx = wave_sum((double)gtx), s_ty = wave_sum((double)gty),
                   s_tz = wave_sum((double)gtz);
      const double s_rx = wave_sum((double)grx), s_ry = wave_sum((double)gry),
                   s_rz = wave_sum((double)grz);
      const double scale = Za / (double)a.n_samples;
      const double O = scale * sO;
      const double D = S - O;
      const float T = (float)(O / D);
      const bool last = it >= a.n_steps;
      float g[7];
      if (a.grad || !last) {
        const double k = scale * S / (D * D);  // dT/dO * Z_A/n
        const double gth[3] = {k * s_rx, k * s_ry, k * s_rz};
        // dT/dq = (2/|q|) [ -v.g ; w g - v x g ] with (w, v) = q/|q|
        const double in = (double)inv_norm;
        const double w = ps[0] * in, vx = ps[1] * in, vy = ps[2] * in, vz = ps[3] * in;
        const double vdg = vx * gth[0] + vy * gth[1] + vz * gth[2];
        const double vxg_x = vy * gth[2] - vz * gth[1];
        const double vxg_y = vz * gth[0] - vx * gth[2];
        const double vxg_z = vx * gth[1] - vy * gth[0];
        g[0] = (float)(2.0 * in * (-vdg));
        g[1] = (float)(2.0 * in * (w * gth[0] - vxg_x));
        g[2] = (float)(2.0 * in * (w * gth[1] - vxg_y));
        g[3] = (float)(2.0 * in * (w * gth[2] - vxg_z));
        g[4] = (float)(k * s_tx);
        g[5] = (float)(k * s_ty);
        g[6] = (float)(k * s_tz);
      }
      wave_lds_sync();  // this pose's records are read before the next move
      if (last) {
        if (lane == 0) {
          a.T[o] = T;
          if (a.grad)
            for (int c = 0; c < 7; ++c) a.grad[o * 7 + c] = g[c];
          if (a.n_steps > 0)
            for (int c = 0; c < 7; ++c) a.pose_out[o * 7 + c] = ps[c];
        }
        break;
      }
      adam_pose_step(ps, am, av, g, it + 1, a.lr, 0.9f, 0.999f, 1e-8f);
    }
  }
}

// Self-overlap of each molecule from its own first n samples,
// O_MM = Z_M / n sum_k w_M u_M (pose invariant); one workgroup per molecule.
__global__ __launch_bounds__(256) void k_self_overlap(Prepared M, const int* __restrict__ off,
                                                      int n_mols, int n_samples, uint2 key,
                                                      float* __restrict__ out) {
  __shared__ Atom sF[SHAPE_MAX_ATOMS];
  __shared__ AtomSampling sS[SHAPE_MAX_ATOMS];
  __shared__ AtomRec sR[SHAPE_MAX_ATOMS];
  __shared__ float sA[SHAPE_MAX_ATOMS];
  __shared__ double red[4];
  const int mol = blockIdx.x;
  if (mol >= n_mols) return;
  if (M.bad[mol] != 0) {
    if (threadIdx.x == 0) out[mol] = __builtin_nanf("");
    return;
  }
  const int a0 = off[mol], na = off[mol + 1] - a0;
  const float4 c = M.centre[mol];
  for (int i = threadIdx.x; i < na; i += blockDim.x) {
    const Atom at = M.atom[a0 + i];
    Atom f = at;
    f.x = at.x - c.x;
    f.y = at.y - c.y;
    f.z = at.z - c.z;
    sF[i] = f;
    sS[i] = M.samp[a0 + i];
    make_rec(at, c.x, c.y, c.z, sR[i], sA[i]);
  }
  __syncthreads();
  float acc = 0.f;
  for (int k = threadIdx.x; k < n_samples; k += blockDim.x) {
    float rx[1], ry[1], rz[1], r2[1], m[1] = {0.f}, u[1] = {0.f};
    sample_point(sF, sS, na, M.id[mol], (uint64_t)k, key, rx[0], ry[0], rz[0]);
    r2[0] = norm2(rx[0], ry[0], rz[0]);
    eval_density_u_x<1>(sR, sA, na, rx, ry, rz, r2, m, u);
    acc += bounded_weight(u[0], m[0]) * u[0];
  }
  const double s = wave_sum((double)acc);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[w];
    out[mol] = (float)(M.Z[mol] * t / (double)n_samples);
  }
}

// Adam (Kingma and Ba) ascent on T over the seven pose parameters, one thread
// per pose; quaternions are renormalised after the update.  The step counter
// lives in device memory so the same launch can be replayed.
__global__ void k_adam_pose(float* __restrict__ pose, const float* __restrict__ dT,
                            float* __restrict__ m, float* __restrict__ v, int64_t n_poses,
                            int* __restrict__ step, float lr, float b1, float b2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = *step + 1;
  if (i < n_poses) {
    float x[7], mi[7], vi[7], g[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      x[c] = pose[i * 7 + c];
      mi[c] = m[i * 7 + c];
      vi[c] = v[i * 7 + c];
      g[c] = dT[i * 7 + c];
    }
    adam_pose_step(x, mi, vi, g, t, lr, b1, b2, eps);
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      pose[i * 7 + c] = x[c];
      m[i * 7 + c] = mi[c];
      v[i * 7 + c] = vi[c];
    }
  }
}

// Advances the device step counter after an Adam update (one thread).
__global__ void k_step_advance(int* step) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
}

// Best start per pair by final T (lowest index on ties; NaN never wins).
__global__ void k_best_start(const float* __restrict__ T, int n_pairs, int n_starts,
                             int* __restrict__ best) {
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
  best[p] = b;
}

size_t align_lds_bytes(int n_samples, int max_a, int max_b) {
  return (size_t)n_samples * sizeof(float4) +
         (size_t)max_a * (sizeof(AtomRec) + sizeof(Atom) + sizeof(float) + sizeof(AtomSampling)) +
         (size_t)kAlignWaves * max_b * (sizeof(float4) + sizeof(AtomRec) + sizeof(float));
}

hipError_t launch_align(const AlignArgs& a, int n_pairs, hipStream_t st) {
  hipLaunchKernelGGL(k_align, dim3((unsigned)n_pairs), dim3(kAlignThreads),
                     align_lds_bytes(a.n_samples, a.max_a, a.max_b), st, a);
  return hipGetLastError();
}

hipError_t launch_self_overlap(const Prepared& M, const int* off, int n_mols, int n_samples,
                               uint2 key, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_self_overlap, dim3((unsigned)n_mols), dim3(256), 0, st, M, off, n_mols,
                     n_samples, key, out);
  return hipGetLastError();
}

hipError_t launch_adam_pose(float* pose, const float* dT, float* m, float* v, int64_t n_poses,
                            int* step, float lr, float b1, float b2, float eps,
                            hipStream_t st) {
  const int64_t blocks = (n_poses + 255) / 256;
  hipLaunchKernelGGL(k_adam_pose, dim3((unsigned)blocks), dim3(256), 0, st, pose, dT, m, v,
                     n_poses, step, lr, b1, b2, eps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, st, step);
  return hipGetLastError();
}

hipError_t launch_best_start(const float* T, int n_pairs, int n_starts, int* best,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_best_start, dim3((n_pairs + 255) / 256), dim3(256), 0, st, T, n_pairs,
                     n_starts, best);
  return hipGetLastError();
}

}  // namespace shape
