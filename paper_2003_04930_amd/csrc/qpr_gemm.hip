// Commutator product X = H_off * Y on the CDNA4 matrix cores.
//
// The coherent part of Eq. (1) needs [H, rho].  With H real symmetric and rho
// Hermitian, rho H = (H rho)^dag, so one complex product X = H_off rho (two
// real products, one per plane of rho) gives [H_off, rho] = X - X^dag; the
// epilogue applies that and the diagonal of H.  H_off is symmetric, so the
// MFMA A-fragment A[i][k] = H[m0+i][k0+k] equals H[k0+k][m0+i] and is read
// along rows of H, the same way as the B-fragment is read from Y.
//
// FP64: v_mfma_f64_16x16x4f64.  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r of lane l holds D[4r + l/16][l%16].
// Tiles are staged through LDS with double buffering (global loads of tile
// k+1 are in flight while tile k is multiplied).
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "qpr_common.h"
#include "qpr_device.h"

namespace qpr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
// Staging registers of the k-slab prefetch are native vectors: arrays of
// HIP's struct vector types (uint4, double2, float4) are not split into
// registers by the compiler and go through scratch memory, which makes every
// prefetch wait for its loads at once.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

// Bijective map from the hardware workgroup id (dispatched round-robin over
// the 8 XCDs) to a logical tile id such that each XCD receives a contiguous
// range of logical tiles, which then share operand blocks in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + (x < r ? x : r) + k;
}

// ------------------------------------------------------------ FP64 / FP32
// One template for both: 16x16x4 MFMA, one operand value per lane.
//   f64: accumulator register r of lane l holds D[4r + l/16][l%16]
//   f32: accumulator register r of lane l holds D[4(l/16) + r][l%16]
template <typename T>
struct MfmaK4;
template <>
struct MfmaK4<double> {
  typedef d4 acc_t;
  typedef d2v vec_t;
  static constexpr int EV = 2;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int r, int lr) { return 4 * r + lr; }
};
template <>
struct MfmaK4<float> {
  typedef f4 acc_t;
  typedef f4 vec_t;
  static constexpr int EV = 4;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int r, int lr) { return 4 * lr + r; }
};

// One BM x BN output tile (both planes) at (m0, n0).
// With `slabs` set, only the nslabs k-slabs it lists (slab j = k rows
// [j BK, j BK + BK), ascending) are multiplied: the block-sparse product skips
// the slabs in which this tile's BM rows of H_off are all zero.  Every output
// element still accumulates its slabs in ascending k with the same MFMA
// sequence, and a skipped slab would only have added exact zeros, so the
// result equals the dense product's.
template <typename T, int BM, int BN, int WM, int WN, int BK>
__device__ __forceinline__ void gemm_k4_tile(const T* __restrict__ H, const T* __restrict__ Yr,
                                             const T* __restrict__ Yi, T* __restrict__ Xr,
                                             T* __restrict__ Xi, int ld, int m0, int n0,
                                             const int* __restrict__ slabs = nullptr,
                                             int nslabs = 0) {
  typedef MfmaK4<T> M;
  typedef typename M::acc_t acc_t;
  typedef typename M::vec_t vec_t;
  constexpr int EV = M::EV;
  constexpr int NWM = BM / WM, NWN = BN / WN, NT = NWM * NWN * 64;
  constexpr int FM = WM / 16, FN = WN / 16;
  // rows padded by 16 elements: lane groups reading consecutive k-rows of a
  // fragment land 32 banks apart (64-bank LDS), so a half-wave read is
  // conflict-free for both FP64 and FP32
  constexpr int AP = BM + 16, BP = BN + 16;
  constexpr int NA = BK * BM / EV / NT, NB = BK * BN / EV / NT;
  static_assert(NA * NT * EV == BK * BM && NB * NT * EV == BK * BN, "tile/thread mismatch");
  __shared__ T As[2][BK * AP];
  __shared__ T Bs[2][2][BK * BP];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % NWM) * WM, wn0 = (wave / NWM) * WN;

  acc_t acc[2][FM][FN];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[p][i][j][r] = (T)0;

  vec_t ra[NA], rb[2][NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int v = tid + u * NT, row = v / (BM / EV), c = v % (BM / EV);
      ra[u] = *reinterpret_cast<const vec_t*>(H + (size_t)(k0 + row) * ld + m0 + EV * c);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int v = tid + u * NT, row = v / (BN / EV), c = v % (BN / EV);
      const size_t o = (size_t)(k0 + row) * ld + n0 + EV * c;
      rb[0][u] = *reinterpret_cast<const vec_t*>(Yr + o);
      rb[1][u] = *reinterpret_cast<const vec_t*>(Yi + o);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int v = tid + u * NT, row = v / (BM / EV), c = v % (BM / EV);
      *reinterpret_cast<vec_t*>(&As[buf][row * AP + EV * c]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int v = tid + u * NT, row = v / (BN / EV), c = v % (BN / EV);
      *reinterpret_cast<vec_t*>(&Bs[buf][0][row * BP + EV * c]) = rb[0][u];
      *reinterpret_cast<vec_t*>(&Bs[buf][1][row * BP + EV * c]) = rb[1][u];
    }
  };

  const int KT = slabs ? nslabs : ld / BK;
  auto kofs = [&](int kt) { return (slabs ? slabs[kt] : kt) * BK; };
  if (KT > 0) {
    gload(kofs(0));
    lstore(0);
  }
  __syncthreads();
  const int lr = lane >> 4, lc = lane & 15;
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) gload(kofs(kt + 1));
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[FM], b[2][FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[buf][(kk + lr) * AP + wm0 + i * 16 + lc];
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        b[0][j] = Bs[buf][0][(kk + lr) * BP + wn0 + j * 16 + lc];
        b[1][j] = Bs[buf][1][(kk + lr) * BP + wn0 + j * 16 + lc];
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[p][i][j] = M::mma(a[i], b[p][j], acc[p][i][j]);
    }
    if (kt + 1 < KT) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int p = 0; p < 2; ++p) {
    T* X = p ? Xi : Xr;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm0 + i * 16 + M::out_row(r, lr);
          const int col = n0 + wn0 + j * 16 + lc;
          X[(size_t)row * ld + col] = acc[p][i][j][r];
        }
  }
}

template <typename T, int BM, int BN, int WM, int WN, int BK = 16>
__global__ void __launch_bounds__((BM / WM) * (BN / WN) * 64)
    k_gemm_k4(const T* __restrict__ H, const T* __restrict__ Yr, const T* __restrict__ Yi,
              T* __restrict__ Xr, T* __restrict__ Xi, int ld, const DevState* __restrict__ st,
              int gate) {
  if (st->stop || (gate && st->hold)) return;
  const int tiles_m = ld / BM;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  gemm_k4_tile<T, BM, BN, WM, WN, BK>(H, Yr, Yi, Xr, Xi, ld, (logical % tiles_m) * BM,
                                      (logical / tiles_m) * BN);
}

// Block-sparse tile-skipping product (BM = 32 rows of H_off per tile, the
// granularity of the slab lists): tile (m0, n0) multiplies only the k-slabs
// of width BK listed for its block row, cnt[m0 / 32] of them at
// idx[(m0 / 32) * (ld / BK) ..] (built by k_block_pattern).
template <typename T, int BN, int WM, int WN, int BK>
__global__ void __launch_bounds__((32 / WM) * (BN / WN) * 64)
    k_gemm_k4_bs(const T* __restrict__ H, const T* __restrict__ Yr, const T* __restrict__ Yi,
                 T* __restrict__ Xr, T* __restrict__ Xi, int ld, const int* __restrict__ cnt,
                 const int* __restrict__ idx, const DevState* __restrict__ st, int gate) {
  if (st->stop || (gate && st->hold)) return;
  constexpr int BM = 32;
  const int tiles_m = ld / BM;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int mb = logical % tiles_m;
  gemm_k4_tile<T, BM, BN, WM, WN, BK>(H, Yr, Yi, Xr, Xi, ld, mb * BM, (logical / tiles_m) * BN,
                                      idx + (size_t)mb * (ld / BK), cnt[mb]);
}

// The slab lists of the block-sparse product: workgroup mb marks the k-slabs
// (width kBsK) holding a nonzero of rows [32 mb, 32 mb + 32) of H_off (from
// its CSR pattern) in LDS, then lists them in ascending order.
__global__ void __launch_bounds__(256) k_block_pattern(const int* __restrict__ h_ptr,
                                                        const int* __restrict__ h_idx, int n,
                                                        int ld, int* __restrict__ cnt,
                                                        int* __restrict__ idx) {
  extern __shared__ int flag[];
  const int mb = blockIdx.x, ks = ld / kBsK;
  for (int j = threadIdx.x; j < ks; j += blockDim.x) flag[j] = 0;
  __syncthreads();
  const int r0 = mb * kBsM, r1 = min(r0 + kBsM, n);
  if (r0 < n)
    for (int e = h_ptr[r0] + threadIdx.x; e < h_ptr[r1]; e += blockDim.x) flag[h_idx[e] / kBsK] = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    int* out = idx + (size_t)mb * ks;
    for (int j = 0; j < ks; ++j)
      if (flag[j]) out[c++] = j;
    cnt[mb] = c;
  }
}

// Persistent form for many systems: the grid strides over a device-side list
// of (system, tile) items; a system whose control block says stop (or hold,
// when gated) is skipped.  The item count is read from device memory so the
// host can shrink the list between replays of a captured graph.
template <typename T, int BM, int BN, int WM, int WN, int BK = 16>
__global__ void __launch_bounds__((BM / WM) * (BN / WN) * 64)
    k_gemm_k4_batch(const BatchGemm* __restrict__ args, const int2* __restrict__ items,
                    const int* __restrict__ nitems) {
  const int ni = *nitems;
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    const int2 item = items[it];
    const BatchGemm& g = args[item.x];
    if (g.st->stop || (g.gate && g.st->hold)) continue;
    const int tiles_m = g.ld / BM;
    gemm_k4_tile<T, BM, BN, WM, WN, BK>((const T*)g.H, (const T*)g.yr, (const T*)g.yi,
                                        (T*)g.xr, (T*)g.xi, g.ld, (item.y % tiles_m) * BM,
                                        (item.y / tiles_m) * BN);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- BF16x3
// X_p = H * (s1 + s2 + s3) with FP32 accumulation on v_mfma_f32_16x16x32_bf16.
// Lane l supplies A[l%16][8(l/16) .. 8(l/16)+7] and B[8(l/16) .. +7][l%16], so
// both operands are needed contiguous along k.  H is symmetric, so row m of H
// is its column m; the slices of R are stored row-major (R is symmetric) and
// the slices of the imaginary plane hold -I (I is antisymmetric), so row j of
// every stored slice is column j of the matrix it represents.
// Slice layout: sl[(p*3 + s) * ld*ld + row*ld + k], p = 0 real, 1 imaginary.
template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__((BM / WM) * (BN / WN) * 64)
    k_gemm_bf16x3(const uint16_t* __restrict__ H, const uint16_t* __restrict__ sl,
                  float* __restrict__ Xr, float* __restrict__ Xi, int ld,
                  const DevState* __restrict__ st, int gate) {
  constexpr int NWM = BM / WM, NWN = BN / WN, NT = NWM * NWN * 64;
  constexpr int BK = 32;          // one MFMA depth
  constexpr int RS = BK + 8;      // padded LDS row (bf16 elements): 80 bytes
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int NA = BM * (BK / 8) / NT;      // 16-byte loads per thread, A
  constexpr int NB = BN * (BK / 8) / NT;      // per plane-slice, B
  static_assert(NA * NT == BM * BK / 8 && NB * NT == BN * BK / 8, "tile/thread mismatch");
  __shared__ uint16_t As[2][BM * RS];
  __shared__ uint16_t Bs[2][6][BN * RS];
  if (st->stop || (gate && st->hold)) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_m = ld / BM;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int m0 = (logical % tiles_m) * BM, n0 = (logical / tiles_m) * BN;
  const int wm0 = (wave % NWM) * WM, wn0 = (wave / NWM) * WN;
  const size_t plane = (size_t)ld * ld;

  f4 acc[2][FM][FN];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[p][i][j] = f4{0.f, 0.f, 0.f, 0.f};

  u4v ra[NA], rb[6][NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int v = tid + u * NT, row = v / (BK / 8), c = v % (BK / 8);
      ra[u] = *reinterpret_cast<const u4v*>(H + (size_t)(m0 + row) * ld + k0 + 8 * c);
    }
#pragma unroll
    for (int ps = 0; ps < 6; ++ps)
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int v = tid + u * NT, row = v / (BK / 8), c = v % (BK / 8);
        rb[ps][u] = *reinterpret_cast<const u4v*>(sl + ps * plane + (size_t)(n0 + row) * ld + k0 + 8 * c);
      }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int v = tid + u * NT, row = v / (BK / 8), c = v % (BK / 8);
      *reinterpret_cast<u4v*>(&As[buf][row * RS + 8 * c]) = ra[u];
    }
#pragma unroll
    for (int ps = 0; ps < 6; ++ps)
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int v = tid + u * NT, row = v / (BK / 8), c = v % (BK / 8);
        *reinterpret_cast<u4v*>(&Bs[buf][ps][row * RS + 8 * c]) = rb[ps][u];
      }
  };

  const int KT = ld / BK;
  gload(0);
  lstore(0);
  __syncthreads();
  const int lr = lane >> 4, lc = lane & 15;
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) gload((kt + 1) * BK);
    bf8 a[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i)
      a[i] = *reinterpret_cast<const bf8*>(&As[buf][(wm0 + i * 16 + lc) * RS + 8 * lr]);
#pragma unroll
    for (int ps = 0; ps < 6; ++ps) {
      const int p = ps / 3;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const bf8 b = *reinterpret_cast<const bf8*>(&Bs[buf][ps][(wn0 + j * 16 + lc) * RS + 8 * lr]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
          acc[p][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[p][i][j], 0, 0, 0);
      }
    }
    if (kt + 1 < KT) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int p = 0; p < 2; ++p) {
    float* X = p ? Xi : Xr;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm0 + i * 16 + 4 * lr + r;
          const int col = n0 + wn0 + j * 16 + lc;
          X[(size_t)row * ld + col] = acc[p][i][j][r];
        }
  }
}

// Single-LDS-buffer form of the BF16x3 product: the next k-slab is staged in
// registers while the current one is multiplied out of LDS, so a workgroup
// holds one slab (A: BM x 32, B: 6 x BN x 32 bf16) instead of two, and two or
// three workgroups share a CU (the double-buffered 128x64 tile fits only one,
// a single wave per SIMD).  A larger BM amortises the six B slices over more
// rows of H.  Same fragment layout and slice order as k_gemm_bf16x3, so the
// product is bitwise the same.
template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__((BM / WM) * (BN / WN) * 64)
    k_gemm_bf16x3_sb(const uint16_t* __restrict__ H, const uint16_t* __restrict__ sl,
                     float* __restrict__ Xr, float* __restrict__ Xi, int ld,
                     const DevState* __restrict__ st, int gate) {
  constexpr int NWM = BM / WM, NWN = BN / WN, NT = NWM * NWN * 64;
  constexpr int BK = 32, RS = BK + 8;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int UA = BM * (BK / 8), UB = 6 * BN * (BK / 8);  // u4v units per slab
  constexpr int NA = (UA + NT - 1) / NT, NB = (UB + NT - 1) / NT;
  __shared__ uint16_t As[BM * RS];
  __shared__ uint16_t Bs[6 * BN * RS];
  if (st->stop || (gate && st->hold)) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_m = ld / BM;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int m0 = (logical % tiles_m) * BM, n0 = (logical / tiles_m) * BN;
  const int wm0 = (wave % NWM) * WM, wn0 = (wave / NWM) * WN;
  const size_t plane = (size_t)ld * ld;

  f4 acc[2][FM][FN];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[p][i][j] = f4{0.f, 0.f, 0.f, 0.f};

  u4v ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int v = tid + u * NT;
      if (UA % NT == 0 || v < UA)
        ra[u] = *reinterpret_cast<const u4v*>(H + (size_t)(m0 + v / 4) * ld + k0 + 8 * (v % 4));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int v = tid + u * NT;
      if (UB % NT == 0 || v < UB) {
        const int ps = v / (BN * 4), rem = v % (BN * 4);
        rb[u] = *reinterpret_cast<const u4v*>(sl + ps * plane + (size_t)(n0 + rem / 4) * ld +
                                                k0 + 8 * (rem % 4));
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int v = tid + u * NT;
      if (UA % NT == 0 || v < UA)
        *reinterpret_cast<u4v*>(&As[(v / 4) * RS + 8 * (v % 4)]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int v = tid + u * NT;
      if (UB % NT == 0 || v < UB) {
        const int ps = v / (BN * 4), rem = v % (BN * 4);
        *reinterpret_cast<u4v*>(&Bs[(ps * BN + rem / 4) * RS + 8 * (rem % 4)]) = rb[u];
      }
    }
  };

  const int KT = ld / BK;
  gload(0);
  lstore();
  __syncthreads();
  const int lr = lane >> 4, lc = lane & 15;
  for (int kt = 0; kt < KT; ++kt) {
    if (kt + 1 < KT) gload((kt + 1) * BK);
    bf8 a[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i)
      a[i] = *reinterpret_cast<const bf8*>(&As[(wm0 + i * 16 + lc) * RS + 8 * lr]);
#pragma unroll
    for (int ps = 0; ps < 6; ++ps) {
      const int p = ps / 3;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const bf8 b =
            *reinterpret_cast<const bf8*>(&Bs[(ps * BN + wn0 + j * 16 + lc) * RS + 8 * lr]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
          acc[p][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[p][i][j], 0, 0, 0);
      }
    }
    __syncthreads();
    if (kt + 1 < KT) {
      lstore();
      __syncthreads();
    }
  }

#pragma unroll
  for (int p = 0; p < 2; ++p) {
    float* X = p ? Xi : Xr;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm0 + i * 16 + 4 * lr + r;
          const int col = n0 + wn0 + j * 16 + lc;
          X[(size_t)row * ld + col] = acc[p][i][j][r];
        }
  }
}

// 32 x 32 x 16 form of the BF16x3 product (v_mfma_f32_32x32x16_bf16).  One
// instruction makes a 32 x 32 block from a 32 x 16 fragment of each operand:
// half the operand bytes per flop of the 16 x 16 x 32 form above, whose LDS
// reads (one A and one B fragment per 16 x 16 block) kept the matrix cores
// about a fifth busy.  Lane l supplies A[l%32][8(l/32) .. +7] and
// B[8(l/32) .. +7][l%32]; accumulator register r of lane l holds
// D[8(r/4) + 4(l/32) + r%4][l%32].  Each 32-deep k-slab is two instructions
// deep; slabs are double buffered in LDS (the next slab's global loads are in
// flight, in registers, while the current one is multiplied; then they go to
// the other buffer and one barrier ends the slab).  Within an instruction the
// products are summed sixteen at a time instead of thirty-two, so this family
// agrees with the 16 x 16 x 32 one within FP32 rounding, not bitwise; its own
// tile shapes agree bitwise with each other (same slice order, same k order).
typedef float f16v __attribute__((ext_vector_type(16)));
template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__((BM / WM) * (BN / WN) * 64)
    k_gemm_bf16x3_m32(const uint16_t* __restrict__ H, const uint16_t* __restrict__ sl,
                      float* __restrict__ Xr, float* __restrict__ Xi, int ld,
                      const DevState* __restrict__ st, int gate) {
  constexpr int NWM = BM / WM, NWN = BN / WN, NT = NWM * NWN * 64;
  constexpr int BK = 32, RS = BK + 8;  // padded LDS row: 80 bytes
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int UA = BM * (BK / 8), UB = 6 * BN * (BK / 8);  // 16-byte units per slab
  constexpr int NA = UA / NT, NB = UB / NT;
  static_assert(NA * NT == UA && NB * NT == UB, "slab units must divide over the threads");
  static_assert(FM * 32 == WM && FN * 32 == WN, "wave tiles are multiples of 32");
  __shared__ uint16_t As[2][BM * RS];
  __shared__ uint16_t Bs[2][6 * BN * RS];
  if (st->stop || (gate && st->hold)) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_m = ld / BM;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int m0 = (logical % tiles_m) * BM, n0 = (logical / tiles_m) * BN;
  const int wm0 = (wave % NWM) * WM, wn0 = (wave / NWM) * WN;
  const size_t plane = (size_t)ld * ld;

  f16v acc[2][FM][FN];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[p][i][j][r] = 0.f;

  // unit v of a slab: A row v / 4 (rows of H), else B slice ps = v' / (4 BN),
  // row v' % (4 BN) / 4; 16-byte chunk v % 4 of the row's 32 k values
  u4v ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int v = tid + u * NT;
      ra[u] = *reinterpret_cast<const u4v*>(H + (size_t)(m0 + v / 4) * ld + k0 + 8 * (v % 4));
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int v = tid + u * NT;
      const int ps = v / (BN * 4), rem = v % (BN * 4);
      rb[u] = *reinterpret_cast<const u4v*>(sl + ps * plane + (size_t)(n0 + rem / 4) * ld + k0 +
                                              8 * (rem % 4));
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int v = tid + u * NT;
      *reinterpret_cast<u4v*>(&As[buf][(v / 4) * RS + 8 * (v % 4)]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int v = tid + u * NT;
      const int ps = v / (BN * 4), rem = v % (BN * 4);
      *reinterpret_cast<u4v*>(&Bs[buf][(ps * BN + rem / 4) * RS + 8 * (rem % 4)]) = rb[u];
    }
  };

  const int KT = ld / BK;
  gload(0);
  lstore(0);
  __syncthreads();
  const int lr = lane >> 5, lc = lane & 31;
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf8 a[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = *reinterpret_cast<const bf8*>(&As[buf][(wm0 + i * 32 + lc) * RS + kk + 8 * lr]);
#pragma unroll
      for (int ps = 0; ps < 6; ++ps) {
        const int p = ps / 3;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const bf8 b = *reinterpret_cast<const bf8*>(
              &Bs[buf][(ps * BN + wn0 + j * 32 + lc) * RS + kk + 8 * lr]);
#pragma unroll
          for (int i = 0; i < FM; ++i)
            acc[p][i][j] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b, acc[p][i][j], 0, 0, 0);
        }
      }
    }
    if (kt + 1 < KT) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int p = 0; p < 2; ++p) {
    float* X = p ? Xi : Xr;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = m0 + wm0 + i * 32 + 8 * (r / 4) + 4 * lr + (r % 4);
          const int col = n0 + wn0 + j * 32 + lc;
          X[(size_t)row * ld + col] = acc[p][i][j][r];
        }
  }
}

template <typename Fn>
struct GemmCfg {
  int bm, bn;
  const char* name;
  Fn fn;
  int threads;
};

typedef void (*F64Fn)(const double*, const double*, const double*, double*, double*, int,
                      const DevState*, int);
typedef void (*F32Fn)(const float*, const float*, const float*, float*, float*, int,
                      const DevState*, int);
typedef void (*BFFn)(const uint16_t*, const uint16_t*, float*, float*, int, const DevState*, int);

const GemmCfg<F64Fn> kF64[] = {
    {64, 64, "f64_64x64_w32x32_k16", k_gemm_k4<double, 64, 64, 32, 32>, 256},
    {32, 32, "f64_32x32_w16x16_k16", k_gemm_k4<double, 32, 32, 16, 16>, 256},
    {128, 64, "f64_128x64_w64x32_k16", k_gemm_k4<double, 128, 64, 64, 32>, 256},
    {64, 128, "f64_64x128_w32x64_k16", k_gemm_k4<double, 64, 128, 32, 64>, 256},
    {64, 64, "f64_64x64_w64x32_k16", k_gemm_k4<double, 64, 64, 64, 32>, 128},
    {64, 64, "f64_64x64_w32x32_k32", k_gemm_k4<double, 64, 64, 32, 32, 32>, 256},
    {32, 32, "f64_32x32_w16x16_k32", k_gemm_k4<double, 32, 32, 16, 16, 32>, 256},
    {64, 32, "f64_64x32_w32x16_k32", k_gemm_k4<double, 64, 32, 32, 16, 32>, 256},
    {32, 64, "f64_32x64_w16x32_k32", k_gemm_k4<double, 32, 64, 16, 32, 32>, 256},
    {128, 128, "f64_128x128_w64x64_k16", k_gemm_k4<double, 128, 128, 64, 64>, 256},
    {128, 64, "f64_128x64_w32x32_k16", k_gemm_k4<double, 128, 64, 32, 32>, 512},
};
const GemmCfg<F32Fn> kF32[] = {
    {64, 64, "f32_64x64_w32x32_k16", k_gemm_k4<float, 64, 64, 32, 32>, 256},
    {32, 32, "f32_32x32_w32x32_k16", k_gemm_k4<float, 32, 32, 32, 32>, 64},
    {128, 64, "f32_128x64_w64x32_k16", k_gemm_k4<float, 128, 64, 64, 32>, 256},
    {64, 64, "f32_64x64_w64x32_k16", k_gemm_k4<float, 64, 64, 64, 32>, 128},
    {64, 64, "f32_64x64_w32x32_k32", k_gemm_k4<float, 64, 64, 32, 32, 32>, 256},
    {32, 32, "f32_32x32_w16x16_k32", k_gemm_k4<float, 32, 32, 16, 16, 32>, 256},
};
const GemmCfg<BFFn> kBF[] = {
    {64, 64, "bf16x3_64x64_w32x32", k_gemm_bf16x3<64, 64, 32, 32>, 256},
    {32, 32, "bf16x3_32x32_w32x32", k_gemm_bf16x3<32, 32, 32, 32>, 64},
    {64, 64, "bf16x3_64x64_w64x32", k_gemm_bf16x3<64, 64, 64, 32>, 128},
    {128, 64, "bf16x3_128x64_w64x32", k_gemm_bf16x3<128, 64, 64, 32>, 256},
    {128, 64, "bf16x3_128x64_w64x32_sb", k_gemm_bf16x3_sb<128, 64, 64, 32>, 256},
    {256, 64, "bf16x3_256x64_w64x32_sb", k_gemm_bf16x3_sb<256, 64, 64, 32>, 512},
    {128, 128, "bf16x3_128x128_w64x64_sb", k_gemm_bf16x3_sb<128, 128, 64, 64>, 256},
    {256, 128, "bf16x3_256x128_w64x64_sb", k_gemm_bf16x3_sb<256, 128, 64, 64>, 512},
    // 32 x 32 x 16 family (configurations 8..)
    {64, 64, "bf16x3_m32_64x64_w32x32", k_gemm_bf16x3_m32<64, 64, 32, 32>, 256},
    {128, 64, "bf16x3_m32_128x64_w64x32", k_gemm_bf16x3_m32<128, 64, 64, 32>, 256},
    {128, 64, "bf16x3_m32_128x64_w32x32", k_gemm_bf16x3_m32<128, 64, 32, 32>, 512},
    {256, 64, "bf16x3_m32_256x64_w64x32", k_gemm_bf16x3_m32<256, 64, 64, 32>, 512},
    {256, 64, "bf16x3_m32_256x64_w128x32", k_gemm_bf16x3_m32<256, 64, 128, 32>, 256},
    {128, 128, "bf16x3_m32_128x128_w64x32", k_gemm_bf16x3_m32<128, 128, 64, 32>, 512},
    {128, 128, "bf16x3_m32_128x128_w64x64", k_gemm_bf16x3_m32<128, 128, 64, 64>, 256},
};
// block-sparse tiles: 32 rows (the slab-list granularity) x BN columns
typedef void (*F64BsFn)(const double*, const double*, const double*, double*, double*, int,
                        const int*, const int*, const DevState*, int);
typedef void (*F32BsFn)(const float*, const float*, const float*, float*, float*, int,
                        const int*, const int*, const DevState*, int);
// (32 x 64 keeps three waves per SIMD; a 32 x 128 tile needs 86 KB of LDS
// for its double-buffered operands, one workgroup per CU)
const GemmCfg<F64BsFn> kF64Bs = {32, 64, "f64_bs_32x64_w16x32_k16",
                                 k_gemm_k4_bs<double, 64, 16, 32, kBsK>, 256};
const GemmCfg<F32BsFn> kF32Bs = {32, 64, "f32_bs_32x64_w32x32_k16",
                                 k_gemm_k4_bs<float, 64, 32, 32, kBsK>, 128};
constexpr int kNumF64 = sizeof(kF64) / sizeof(kF64[0]);
constexpr int kNumF32 = sizeof(kF32) / sizeof(kF32[0]);
constexpr int kNumBF = sizeof(kBF) / sizeof(kBF[0]);

}  // namespace

int gemm_num_cfgs(int kind) {
  return kind == OP_F64 ? kNumF64 : kind == OP_F32 ? kNumF32 : kind == OP_BF16X3 ? kNumBF : 0;
}

bool gemm_cfg_fits(int kind, int cfg, int ld) {
  if (cfg < 0 || cfg >= gemm_num_cfgs(kind)) return false;
  int bm, bn;
  if (kind == OP_F64) {
    bm = kF64[cfg].bm;
    bn = kF64[cfg].bn;
  } else if (kind == OP_F32) {
    bm = kF32[cfg].bm;
    bn = kF32[cfg].bn;
  } else {
    bm = kBF[cfg].bm;
    bn = kBF[cfg].bn;
  }
  return ld % bm == 0 && ld % bn == 0;
}

const char* gemm_cfg_name(int kind, int cfg) {
  if (cfg < 0 || cfg >= gemm_num_cfgs(kind)) return "?";
  return kind == OP_F64 ? kF64[cfg].name : kind == OP_F32 ? kF32[cfg].name : kBF[cfg].name;
}

// Tile choice per (kind, padded size): filled by the autotuner (qpr_autotune)
// or a tuning cache; configuration 0 otherwise.
namespace {
struct TuneEntry {
  int kind, ld, cfg;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
}  // namespace

void gemm_set_tuned(int kind, int ld, int cfg) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& e : g_tune)
    if (e.kind == kind && e.ld == ld) {
      e.cfg = cfg;
      return;
    }
  g_tune.push_back({kind, ld, cfg});
}

bool tuned_exact(int kind, int ld, int* cfg) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& e : g_tune)
    if (e.kind == kind && e.ld == ld) {
      *cfg = e.cfg;
      return true;
    }
  return false;
}

int gemm_default_cfg(int kind, int n) {
  const int ld = pad_n(n);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int best = -1, best_ld = 0;
  for (const auto& e : g_tune)  // exact size, else the nearest tuned size of the same kind
    if (e.kind == kind && (best < 0 || std::abs(e.ld - ld) < std::abs(best_ld - ld))) {
      best = e.cfg;
      best_ld = e.ld;
    }
  if (best >= 0) return best;
  // untuned defaults, from HIP-event sweeps on MI355X at N = 922, 1024, 1536,
  // 2048, 4096: small problems want more, smaller tiles; large ones 128-row
  // tiles (FP64 128x64: 4.03 ms at 4096, 0.87 of the FP64 peak; FP32 128x64:
  // 2.03 ms, 0.86)
  const bool big = ld >= 2048 && ld % 128 == 0;
  if (kind == OP_F64) return big ? 10 : 1;
  if (kind == OP_F32) return big ? 2 : 5;
  // BF16x3: 256 rows of H where ld allows -- the single-LDS-buffer 256x128
  // tile at 4096 (0.68 ms, 0.48 of the bf16 peak), the 32x32x16 256x64 tile
  // from 1536 (65 us; 92 us at 2048) -- else the 32x32x16 64x64 tile, which
  // divides every ld (25 us at 922 and 1024)
  if (ld % 256 == 0 && ld >= 4096) return 7;
  if (ld % 256 == 0 && ld >= 1536) return 11;
  return 8;
}

template <typename C>
static int pick(const C* table, int count, int cfg, int kind, int n, int ld) {
  if (cfg < 0 || cfg >= count) cfg = gemm_default_cfg(kind, n);
  if (cfg < 0 || cfg >= count || ld % table[cfg].bm || ld % table[cfg].bn) cfg = 0;
  return cfg;  // configuration 0 tiles 64 x 64, which divides every ld
}

hipError_t launch_block_pattern(const qpr_problem* P, const Ws& w, hipStream_t s) {
  const int ld = P->ld;
  k_block_pattern<<<ld / kBsM, 256, (size_t)(ld / kBsK) * sizeof(int), s>>>(
      P->h_ptr, P->h_idx, P->n, ld, w.bs_cnt, w.bs_idx);
  return hipGetLastError();
}

// The block-sparse product: 32 x 64 tiles (ld is a multiple of 64).
static hipError_t launch_gemm_bs(int kind, const qpr_problem* P, const Ws& w, const double* yr,
                                 const double* yi, int gate, hipStream_t s) {
  const int ld = P->ld;
  if (kind == OP_F64) {
    hipLaunchKernelGGL(kF64Bs.fn, dim3((ld / 32) * (ld / kF64Bs.bn)), dim3(kF64Bs.threads), 0, s,
                       P->h_off, yr, yi, w.x_r, w.x_i, ld, w.bs_cnt, w.bs_idx, w.st, gate);
    return hipGetLastError();
  }
  if (kind == OP_F32) {
    hipLaunchKernelGGL(kF32Bs.fn, dim3((ld / 32) * (ld / kF32Bs.bn)), dim3(kF32Bs.threads), 0, s,
                       P->h_off_f32, (const float*)w.lo_r, (const float*)w.lo_i, w.xf_r, w.xf_i,
                       ld, w.bs_cnt, w.bs_idx, w.st, gate);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;  // no block-sparse form of the three-slice bf16 product
}

hipError_t launch_gemm(int kind, int cfg, const qpr_problem* P, const Ws& w, const double* yr,
                       const double* yi, int gate, hipStream_t s) {
  if (cfg == kCfgBlockSparse) return launch_gemm_bs(kind, P, w, yr, yi, gate, s);
  const int ld = P->ld;
  if (kind == OP_F64) {
    const auto& c = kF64[pick(kF64, kNumF64, cfg, kind, P->n, ld)];
    hipLaunchKernelGGL(c.fn, dim3((ld / c.bm) * (ld / c.bn)), dim3(c.threads), 0, s, P->h_off, yr,
                       yi, w.x_r, w.x_i, ld, w.st, gate);
    return hipGetLastError();
  }
  if (kind == OP_F32) {
    const auto& c = kF32[pick(kF32, kNumF32, cfg, kind, P->n, ld)];
    hipLaunchKernelGGL(c.fn, dim3((ld / c.bm) * (ld / c.bn)), dim3(c.threads), 0, s,
                       P->h_off_f32, (const float*)w.lo_r, (const float*)w.lo_i, w.xf_r, w.xf_i,
                       ld, w.st, gate);
    return hipGetLastError();
  }
  if (kind == OP_BF16X3) {
    const auto& c = kBF[pick(kBF, kNumBF, cfg, kind, P->n, ld)];
    hipLaunchKernelGGL(c.fn, dim3((ld / c.bm) * (ld / c.bn)), dim3(c.threads), 0, s,
                       P->h_off_bf16, (const uint16_t*)w.sl, w.xf_r, w.xf_i, ld, w.st, gate);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

typedef void (*F64BatchFn)(const BatchGemm*, const int2*, const int*);
struct BatchCfg {
  int kind, bm, bn, threads;
  const char* name;
  F64BatchFn fn;
};
const BatchCfg kBatch[] = {
    {OP_F64, 64, 64, 256, "f64_64x64_w32x32_k16", k_gemm_k4_batch<double, 64, 64, 32, 32>},
    {OP_F64, 64, 64, 256, "f64_64x64_w32x32_k32", k_gemm_k4_batch<double, 64, 64, 32, 32, 32>},
    {OP_F64, 32, 32, 256, "f64_32x32_w16x16_k32", k_gemm_k4_batch<double, 32, 32, 16, 16, 32>},
    {OP_F32, 64, 64, 256, "f32_64x64_w32x32_k16", (F64BatchFn)k_gemm_k4_batch<float, 64, 64, 32, 32>},
    {OP_F32, 64, 64, 256, "f32_64x64_w32x32_k32", (F64BatchFn)k_gemm_k4_batch<float, 64, 64, 32, 32, 32>},
    {OP_F32, 32, 32, 256, "f32_32x32_w16x16_k32", (F64BatchFn)k_gemm_k4_batch<float, 32, 32, 16, 16, 32>},
};
constexpr int kNumBatch = sizeof(kBatch) / sizeof(kBatch[0]);

int batch_gemm_cfgs(int kind, int* out, int max) {
  int c = 0;
  for (int i = 0; i < kNumBatch; ++i)
    if (kBatch[i].kind == kind && c < max) out[c++] = i;
  return c;
}
int batch_gemm_tile(int cfg) { return cfg >= 0 && cfg < kNumBatch ? kBatch[cfg].bm : 64; }

hipError_t launch_gemm_batch(int cfg, const BatchGemm* args, const int2* items,
                             const int* nitems, int grid, hipStream_t s) {
  if (cfg < 0 || cfg >= kNumBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kBatch[cfg].fn, dim3(grid), dim3(kBatch[cfg].threads), 0, s, args, items,
                     nitems);
  return hipGetLastError();
}

}  // namespace qpr
