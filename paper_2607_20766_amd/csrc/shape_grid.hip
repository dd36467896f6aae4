// Dense-grid quadrature reference (section "Importance-sampling estimator",
// the grid ground truth of the accuracy comparison): the union and
// first-order integrals of a pair by the trapezoid rule on a cubic grid,
// FP64 throughout.
//
// Grid: the box of all atom centres of A and B grown by `pad` on every side,
// spacing h, ceil(extent / h) + 1 points per axis, weights 1/2 on the two
// end planes of each axis (their integrands are negligible there).  The
// Gaussians separate over the axes, exp(-a |r - c|^2) =
// E_x(i, ix) E_y(i, iy) E_z(i, iz), so per point and atom one product of
// tabulated factors replaces the exponential.
//
// Outputs (in this order): int uA uB, int uA^2, int uB^2, int uA, int uB,
// int mA mB, int mA^2, int mB^2.
#include "shape_kernels.hpp"

#include <math.h>

namespace shape {

// Bounding box of the atom centres of A and B: box = (min x, y, z, max x, y, z).
__global__ void k_grid_box(const float* __restrict__ xa, int na, const float* __restrict__ xb,
                           int nb, double* __restrict__ box) {
  __shared__ double lo[3][kWave], hi[3][kWave];
  const int t = threadIdx.x;
  double l[3] = {1e300, 1e300, 1e300}, h[3] = {-1e300, -1e300, -1e300};
  for (int i = t; i < na + nb; i += kWave) {
    const float* c = i < na ? xa + 3 * i : xb + 3 * (i - na);
    for (int d = 0; d < 3; ++d) {
      l[d] = fmin(l[d], (double)c[d]);
      h[d] = fmax(h[d], (double)c[d]);
    }
  }
  for (int d = 0; d < 3; ++d) {
    lo[d][t] = l[d];
    hi[d][t] = h[d];
  }
  __syncthreads();
  if (t < 3) {
    double a = 1e300, b = -1e300;
    for (int k = 0; k < kWave; ++k) {
      a = fmin(a, lo[t][k]);
      b = fmax(b, hi[t][k]);
    }
    box[t] = a;
    box[3 + t] = b;
  }
}

// E[axis][atom][k] = exp(-alpha (lo_axis + k h - c_axis)^2), atoms of A then B.
__global__ void k_grid_tables(const float* __restrict__ xa, const float* __restrict__ aa, int na,
                              const float* __restrict__ xb, const float* __restrict__ ab, int nb,
                              GridDims g, double* __restrict__ E) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n_atoms = na + nb;
  const int64_t per_axis = (int64_t)n_atoms * g.nmax;
  if (t >= 3 * per_axis) return;
  const int axis = (int)(t / per_axis);
  const int64_t rem = t % per_axis;
  const int i = (int)(rem / g.nmax), k = (int)(rem % g.nmax);
  double v = 0.0;
  if (k < g.n[axis]) {
    const float c = i < na ? xa[3 * i + axis] : xb[3 * (i - na) + axis];
    const float al = i < na ? aa[i] : ab[i - na];
    const double d = g.lo[axis] + k * g.h - (double)c;
    v = exp(-(double)al * d * d);
  }
  E[t] = v;
}

constexpr int kGridThreads = 256;
constexpr int kGridSums = 8;

// One workgroup per (ix, iy) column: the per-atom factors E_x E_y in LDS,
// threads along z; FP64 block sums in fixed order.
__global__ __launch_bounds__(kGridThreads) void k_grid_columns(const double* __restrict__ E,
                                                               int na, int nb, GridDims g,
                                                               double* __restrict__ part) {
  extern __shared__ double sxy[];  // [na + nb]
  __shared__ double red[kGridThreads / kWave][kGridSums];
  const int col = blockIdx.x;
  const int ix = col / g.n[1], iy = col % g.n[1];
  const int n = na + nb;
  const int64_t per_axis = (int64_t)n * g.nmax;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    sxy[i] = E[(int64_t)i * g.nmax + ix] * E[per_axis + (int64_t)i * g.nmax + iy];
  __syncthreads();
  const double wxy = ((ix == 0 || ix == g.n[0] - 1) ? 0.5 : 1.0) *
                     ((iy == 0 || iy == g.n[1] - 1) ? 0.5 : 1.0);
  double s[kGridSums];
#pragma unroll
  for (int q = 0; q < kGridSums; ++q) s[q] = 0.0;
  const double* Ez = E + 2 * per_axis;
  for (int iz = threadIdx.x; iz < g.n[2]; iz += blockDim.x) {
    double mA = 0.0, pA = 1.0, mB = 0.0, pB = 1.0;
    for (int i = 0; i < na; ++i) {
      const double o = sxy[i] * Ez[(int64_t)i * g.nmax + iz];
      mA += o;
      pA *= 1.0 - o;
    }
    for (int i = na; i < n; ++i) {
      const double o = sxy[i] * Ez[(int64_t)i * g.nmax + iz];
      mB += o;
      pB *= 1.0 - o;
    }
    const double uA = 1.0 - pA, uB = 1.0 - pB;
    const double w = wxy * ((iz == 0 || iz == g.n[2] - 1) ? 0.5 : 1.0);
    s[0] += w * uA * uB;
    s[1] += w * uA * uA;
    s[2] += w * uB * uB;
    s[3] += w * uA;
    s[4] += w * uB;
    s[5] += w * mA * mB;
    s[6] += w * mA * mA;
    s[7] += w * mB * mB;
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < kGridSums; ++q) s[q] = wave_sum(s[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < kGridSums; ++q) red[wave][q] = s[q];
  __syncthreads();
  if (threadIdx.x < kGridSums) {
    double v = 0.0;
    for (int w = 0; w < kGridThreads / kWave; ++w) v += red[w][threadIdx.x];
    part[(int64_t)col * kGridSums + threadIdx.x] = v;
  }
}

// Column partials summed in a fixed order, times h^3: workgroup q sums
// integral q; thread t takes columns [t c/256, (t+1) c/256), then the 256
// thread sums are added in thread order.
__global__ __launch_bounds__(256) void k_grid_final(const double* __restrict__ part, int n_cols,
                                                    double h3, double* __restrict__ out) {
  __shared__ double red[256];
  const int q = blockIdx.x, t = threadIdx.x;
  const int per = (n_cols + 255) / 256;
  const int c0 = t * per, c1 = min(n_cols, c0 + per);
  double v = 0.0;
  for (int c = c0; c < c1; ++c) v += part[(int64_t)c * kGridSums + q];
  red[t] = v;
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += red[i];
    out[q] = s * h3;
  }
}

hipError_t launch_grid_box(const float* xa, int na, const float* xb, int nb, double* box,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_grid_box, dim3(1), dim3(kWave), 0, st, xa, na, xb, nb, box);
  return hipGetLastError();
}

hipError_t launch_grid(const float* xa, const float* aa, int na, const float* xb,
                       const float* ab, int nb, const GridDims& g, double* tables, double* part,
                       double* out, hipStream_t st) {
  const int n = na + nb;
  const int64_t tab = 3 * (int64_t)n * g.nmax;
  hipLaunchKernelGGL(k_grid_tables, dim3((unsigned)((tab + 255) / 256)), dim3(256), 0, st, xa,
                     aa, na, xb, ab, nb, g, tables);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int cols = g.n[0] * g.n[1];
  hipLaunchKernelGGL(k_grid_columns, dim3((unsigned)cols), dim3(kGridThreads),
                     (size_t)n * sizeof(double), st, tables, na, nb, g, part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grid_final, dim3(kGridSums), dim3(256), 0, st, part, cols, g.h * g.h * g.h,
                     out);
  return hipGetLastError();
}

}  // namespace shape
