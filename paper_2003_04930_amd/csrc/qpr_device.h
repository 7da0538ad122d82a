// Device helpers shared by the libqpr kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/qpr.h"

namespace qpr {

__device__ __forceinline__ int wave_sum_i(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ double wave_min_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum over a 1024-thread block in a fixed order; every thread gets the result.
__device__ __forceinline__ double block_sum_1024(double v, double* red) {
  const int t = threadIdx.x;
  v = wave_sum_d(v);
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < 16; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Sum over a block of `nw` waves in a fixed order; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* red, int nw) {
  const int t = threadIdx.x;
  v = wave_sum_d(v);
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Max over a block of `nw` waves; every thread gets the result.
__device__ __forceinline__ double block_max(double v, double* red, int nw) {
  const int t = threadIdx.x;
  v = wave_max_d(v);
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < nw; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

// What the gain (G p)_a needs: G itself is never stored.
struct GainView {
  int n, teleport;
  double alpha;
  const double* inv_outdeg;
  const int* dangling;
  const int* in_ptr;
  const int* in_idx;
};

// The teleport and dangling part of (G p)_a, given s = sum over in-links j of
// p_j / outDeg(j).
__device__ __forceinline__ double gain_finish(const GainView& g, int a, const double* p,
                                              double P, double D, double s) {
  double tel, dang;
  if (g.teleport == QPR_TELEPORT_PAPER_F) {
    const double inv = 1.0 / (double)(g.n - 1);
    const double pa = p[a];
    tel = (P - pa) * inv;
    dang = (D - (g.dangling[a] ? pa : 0.0)) * inv;
  } else {
    const double inv = 1.0 / (double)g.n;
    tel = P * inv;
    dang = D * inv;
  }
  return g.alpha * (s + dang) + (1.0 - g.alpha) * tel;
}

// (G p)_a for G = alpha S + (1 - alpha) T with dangling columns set to T,
// summing the in-links of a in one thread.
//   P = sum_j p_j,  D = sum over dangling j of p_j.
__device__ __forceinline__ double gain_row(const GainView& g, int a, const double* p,
                                           double P, double D) {
  double s = 0.0;
  const int e1 = g.in_ptr[a + 1];
  for (int e = g.in_ptr[a]; e < e1; ++e) {
    const int j = g.in_idx[e];
    s += p[j] * g.inv_outdeg[j];
  }
  return gain_finish(g, a, p, P, D, s);
}

}  // namespace qpr
