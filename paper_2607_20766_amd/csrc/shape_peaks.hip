// Issue-rate microbenchmarks of the instructions the density loop, the
// sampler and the staging are built from (measurement support): FP32 fused
// multiply-add, the hardware exponential (v_exp_f32), the 32x32->64-bit
// integer multiply-add behind Philox (v_mad_u64_u32), and 16-byte LDS reads.
// Each kernel keeps eight independent chains per lane so that the issue rate,
// not the dependency latency, is what is timed; every lane writes its result
// so nothing is removed by the compiler.  The grid is 16 workgroups of 256
// lanes per compute unit (16 waves per SIMD).  gfx950 retires a wave64 FP32
// multiply-add in two cycles only when every operand is a VGPR (an SGPR or
// literal operand halves the rate), so the FMA probe keeps its multiplier and
// addend in VGPRs: its rate is the one the published 157.3 TFLOP/s FP32
// vector peak stands for (256 CUs x 4 SIMDs x 32 lanes x 2 flops x 2.4 GHz).
#include "shape_kernels.hpp"

namespace shape {

constexpr int kPeakChains = 8;

__global__ __launch_bounds__(256) void k_peak_fma(int iters, float b0, float c0,
                                                  float* __restrict__ out) {
  // per-lane operands: VGPRs, so each step is one full-rate v_fmac_f32
  const float b = b0 + 1e-9f * (float)threadIdx.x, c = c0 + 1e-9f * (float)threadIdx.x;
  float a[kPeakChains];
#pragma unroll
  for (int j = 0; j < kPeakChains; ++j) a[j] = (float)(threadIdx.x + j);
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kPeakChains; ++j) a[j] = fmaf(b, c, a[j]);
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kPeakChains; ++j) s += a[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// The same chains with the multiplier and addend as kernel arguments
// (SGPRs): the operand form that halves the FP32 issue rate.
__global__ __launch_bounds__(256) void k_peak_fma_sgpr(int iters, float b, float c,
                                                       float* __restrict__ out) {
  float a[kPeakChains];
#pragma unroll
  for (int j = 0; j < kPeakChains; ++j) a[j] = (float)(threadIdx.x + j);
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kPeakChains; ++j) a[j] = fmaf(b, a[j], c);
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kPeakChains; ++j) s += a[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_exp(int iters, float* __restrict__ out) {
  float a[kPeakChains];
#pragma unroll
  for (int j = 0; j < kPeakChains; ++j) a[j] = 0.25f + 0.01f * (float)j;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kPeakChains; ++j) a[j] = __builtin_amdgcn_exp2f(-a[j]);  // in (0, 1)
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kPeakChains; ++j) s += a[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_mad64(int iters, uint32_t k,
                                                    float* __restrict__ out) {
  uint64_t p[kPeakChains];
#pragma unroll
  for (int j = 0; j < kPeakChains; ++j) p[j] = threadIdx.x * 2654435761u + j;
  // p <- lo(p) k + p: one v_mad_u64_u32 whose result overwrites its addend
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kPeakChains; ++j) p[j] = (uint64_t)(uint32_t)p[j] * k + p[j];
  }
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kPeakChains; ++j) s ^= (uint32_t)p[j] ^ (uint32_t)(p[j] >> 32);
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

constexpr int kPeakLdsVec = 4096;  // float4 entries: 64 KiB

__global__ __launch_bounds__(256) void k_peak_lds(int iters, float* __restrict__ out) {
  __shared__ float4 buf[kPeakLdsVec];
  for (int i = threadIdx.x; i < kPeakLdsVec; i += blockDim.x)
    buf[i] = make_float4((float)i, 1.0f, 2.0f, 3.0f);
  __syncthreads();
  float4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = make_float4(0.f, 0.f, 0.f, 0.f);
  // consecutive lanes read consecutive 16-byte entries (no bank conflicts)
  int at = threadIdx.x;
#pragma unroll 2
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float4 v = buf[(at + j * 256) & (kPeakLdsVec - 1)];
      acc[j].x += v.x;
      acc[j].y += v.y;
      acc[j].z += v.z;
      acc[j].w += v.w;
    }
    at += 1024;
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j) s += acc[j].x + acc[j].y + acc[j].z + acc[j].w;
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int peak_blocks(int n_cu) { return 16 * n_cu; }

hipError_t launch_peak(int which, int n_cu, int iters, float* out, hipStream_t st) {
  const dim3 grid(peak_blocks(n_cu)), block(256);
  switch (which) {
    case 0: hipLaunchKernelGGL(k_peak_fma, grid, block, 0, st, iters, 0.999f, 1e-3f, out); break;
    case 1: hipLaunchKernelGGL(k_peak_exp, grid, block, 0, st, iters, out); break;
    case 2: hipLaunchKernelGGL(k_peak_mad64, grid, block, 0, st, iters, 0xD2511F53u, out); break;
    case 3: hipLaunchKernelGGL(k_peak_lds, grid, block, 0, st, iters, out); break;
    case 4:
      hipLaunchKernelGGL(k_peak_fma_sgpr, grid, block, 0, st, iters, 0.999f, 1e-3f, out);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Work per lane and loop iteration of each kernel: 8 FMAs, 8 exponentials,
// 8 integer multiply-adds, 4 x 16 bytes read from LDS, 8 FMAs.
double peak_work_per_iter(int which) {
  switch (which) {
    case 0: case 1: case 2: case 4: return (double)kPeakChains;
    case 3: return 4.0 * 16.0;
    default: return 0.0;
  }
}

}  // namespace shape
