// Fused right-hand-side epilogue and the small per-step kernels.
//
// Right-hand side of Eq. (1) (GKSL anticommutator, jump operators
// sqrt(G_ij)|i><j| for all ordered pairs) in the real planes R = Re Y,
// I = Im Y, with X = H_off Y = A + iB from the product kernel and h = diag H:
//
//   Re L_ab = (1-w) [ B_ab + B_ba + (h_a - h_b) I_ab ] + w [ delta_ab g_a - (d_a + d_b)/2 R_ab ]
//   Im L_ab = (1-w) [ A_ba - A_ab - (h_a - h_b) R_ab ] - w (d_a + d_b)/2 I_ab
//
// where g = G diag(Y) is the gain of the jump terms (sum_k L_k Y L_k^dag =
// diag(G p)) and d_j = sum_i G_ij (sum_k L_k^dag L_k = diag(d)).  Every term
// is odd or even under (a,b) -> (b,a) exactly as written, so a Hermitian Y
// gives a bitwise Hermitian L.
//
// The same pass applies the classical RK4 stage update of Supplementary
// Note 2 (k_s = L(Y_s); Y_{s+1} = y_n + c_s dt k_s; acc accumulates k with
// weights 1,2,2,1; y_{n+1} = y_n + dt/6 (acc + k_4)) and, on reducing stages,
// leaves per-tile partials of ||k||_F^2 and a non-finite flag; a finishing
// step folds them in a fixed order and decides convergence (or the adaptive
// step) on the device.
#include <cmath>
#include <cstdio>
#include <type_traits>

#include "qpr_common.h"
#include "qpr_device.h"

namespace qpr {

namespace {

constexpr int TE = 32;       // epilogue tile edge
constexpr int ETHREADS = 512;
constexpr int ERS = ETHREADS / TE;  // tile rows covered per pass of the workgroup
constexpr int EM = TE / ERS;        // tile elements per thread
static_assert(ETHREADS % TE == 0 && TE % ERS == 0, "epilogue thread layout");

__device__ __forceinline__ uint16_t bf16_rn(float f) {
  // round-to-nearest-even float -> bf16 (inputs are finite here)
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double bf16_to_d(uint16_t h) {
  return (double)__uint_as_float(((unsigned int)h) << 16);
}

// Three bf16 slices s1 + s2 + s3 of v (each the bf16 rounding of what the
// previous slices leave), the residuals taken exactly in FP64.
__device__ __forceinline__ void split3(double v, uint16_t& s1, uint16_t& s2, uint16_t& s3) {
  s1 = bf16_rn((float)v);
  const double r1 = v - bf16_to_d(s1);
  s2 = bf16_rn((float)r1);
  const double r2 = r1 - bf16_to_d(s2);
  s3 = bf16_rn((float)r2);
}

// Two-level reduction over the `nb` tiles of one system: every tile writes its
// partials (sum, non-finite flag, max) with plain stores, and a one-workgroup
// finishing kernel launched after the tile kernel combines them in index
// order (deterministic).  The kernel boundary makes the partials visible; a
// last-tile ticket inside the tile kernel would need a device-scope release
// fence per workgroup, which on this multi-XCD part writes back the XCD's L2
// and serialises the workgroups.
__device__ __forceinline__ void tile_partials(double my_sum, int my_bad, double my_max,
                                              double* partials, double* red, int tile) {
  const int tid = threadIdx.x;
  double s = block_sum(my_sum, red, ETHREADS / 64);
  double m = block_max(my_max, red, ETHREADS / 64);
  int b = __syncthreads_or(my_bad);
  if (tid == 0) {
    partials[3 * tile] = s;
    partials[3 * tile + 1] = (double)b;
    partials[3 * tile + 2] = m;
  }
}

// The fold of one stage's partials by a 256-thread workgroup in a fixed order:
// thread t takes partials t + 256 j, accumulating j mod 4 separately (four
// loads in flight), the four combined as (0+1)+(2+3), then a fixed shuffle
// tree per wave and the four waves in order.  Every finisher -- the finishing
// kernels and the sparse-product launches that carry a finishing workgroup --
// runs it with 256 threads, so they agree bit for bit; in a larger workgroup
// the threads past the first 256 load nothing and only join the barriers.
constexpr int FOLD_THREADS = 256;
__device__ __forceinline__ void fold_partials(const double* partials, int nb, double& tot,
                                              int& bad, double& mx) {
  __shared__ double rs[FOLD_THREADS / 64], rb[FOLD_THREADS / 64], rm[FOLD_THREADS / 64];
  const int t = threadIdx.x;
  const bool act = t < FOLD_THREADS;
  double a[4] = {0.0, 0.0, 0.0, 0.0}, bb = 0.0, mm = 0.0;
  int i = act ? t : nb;
  for (; i + 3 * FOLD_THREADS < nb; i += 4 * FOLD_THREADS) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double* q = partials + 3 * (i + k * FOLD_THREADS);
      a[k] += q[0];
      bb = fmax(bb, q[1]);
      mm = fmax(mm, q[2]);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)  // at most three left after the loop above
    if (i + k * FOLD_THREADS < nb) {
      const double* q = partials + 3 * (i + k * FOLD_THREADS);
      a[k] += q[0];
      bb = fmax(bb, q[1]);
      mm = fmax(mm, q[2]);
    }
  const double acc = (a[0] + a[1]) + (a[2] + a[3]);
  const double ws = wave_sum_d(acc), wb = wave_max_d(bb), wm = wave_max_d(mm);
  if (act && (t & 63) == 0) {
    rs[t >> 6] = ws;
    rb[t >> 6] = wb;
    rm[t >> 6] = wm;
  }
  __syncthreads();
  tot = (rs[0] + rs[1]) + (rs[2] + rs[3]);
  bad = fmax(fmax(rb[0], rb[1]), fmax(rb[2], rb[3])) != 0.0;
  mx = fmax(fmax(rm[0], rm[1]), fmax(rm[2], rm[3]));
  __syncthreads();
}

// Tile pairs of the upper triangle: k -> (I, J), I <= J, column by column.
__device__ __forceinline__ void tri_decode(int k, int& I, int& J) {
  int j = (int)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
  while ((j + 1) * (j + 2) / 2 <= k) ++j;
  while (j * (j + 1) / 2 > k) --j;
  J = j;
  I = k - j * (j + 1) / 2;
}
__host__ __device__ constexpr int tri_tiles(int t) { return t * (t + 1) / 2; }

// Workgroups are dispatched round-robin over the 8 XCDs (bid % 8).  This
// renumbering gives XCD x one contiguous run of the nb logical indices (a
// bijection of [0, nb)), so neighbouring work items share its L2.
__device__ __forceinline__ int xcd_contiguous(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + (x < r ? x : r) + k;
}

// The fused sparse product: the two 32 x 32 blocks of X = H_off Y that tile
// pair (I, J) needs, gathered through the CSR of H_off straight into LDS.
// Task t < 32 is row b0 + t of X over columns a0.. (the transposed block, into
// Tr/Ti); task 32 + t (off-diagonal pairs) row a0 + t over columns b0.. (into
// Xr/Xi).  Wave w owns tasks w, w + 8, ..., with the 64 lanes on (plane,
// column).  The first eight neighbour indices of all its tasks come in one
// vector load (lane 8 j + k: entry k of task j) and are broadcast from there,
// so only the row loads are on the critical path; rows with more than eight
// neighbours finish with groups of eight read through the index array.  Each
// row is summed in the order of the separate sparse product (eight partials,
// fixed tree), so the two give bitwise the same X.
// T = float: the rows come from the FP32 copy of Y_s, summed in FP64 in the
// same order and rounded once to FP32, as the separate FP32 product does.
constexpr int FUSE_TASKS_IN_FLIGHT = 2;
template <typename T>
__device__ __forceinline__ void fused_gather(const ProbView& pv, const T* __restrict__ ysr,
                                             const T* __restrict__ ysi, int a0, int b0,
                                             bool diag, double (*Tr)[TE + 1], double (*Ti)[TE + 1],
                                             double (*Xr)[TE + 1], double (*Xi)[TE + 1]) {
  constexpr int NW = ETHREADS / 64, TPW = 2 * TE / NW, TQ = FUSE_TASKS_IN_FLIGHT;
  static_assert(TPW * 8 == 64 && TPW % TQ == 0, "eight index slots per task fill a wave");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ntask = diag ? TE : 2 * TE;
  // this lane's index slot: entry k of task j
  int e0 = 0, e1 = 0, idx = 0;
  {
    const int j = lane >> 3, k = lane & 7;
    const int t = wave + NW * j;
    const int row = t < TE ? b0 + t : a0 + t - TE;
    if (t < ntask && row < pv.n) {
      e0 = pv.h_ptr[row];
      e1 = pv.h_ptr[row + 1];
    }
    if (e1 > e0) idx = pv.h_idx[min(e0 + k, e1 - 1)];
  }
  const int ld = pv.ld, cl = lane & 31;
  const T* __restrict__ Yp = (lane >> 5) ? ysi : ysr;
  const double sg = (double)pv.hsign;
  const int jend = diag ? TPW / 2 : TPW;  // diagonal pairs: tasks w + 8 j < 32
#pragma unroll
  for (int j0 = 0; j0 < TPW; j0 += TQ) {
    if (j0 >= jend) break;
    double v[TQ][8];
    const T* base[TQ];
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const int t = wave + NW * (j0 + q);
      base[q] = Yp + (t < TE ? a0 : b0) + cl;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int r = __builtin_amdgcn_readlane(idx, 8 * (j0 + q) + k);
        v[q][k] = (double)base[q][(size_t)r * ld];
      }
    }
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const int jq = j0 + q, t = wave + NW * jq;
      const int f0 = __builtin_amdgcn_readlane(e0, 8 * jq);
      const int f1 = __builtin_amdgcn_readlane(e1, 8 * jq);
      // entry e into partial (e - e0) % 8, partials added in the fixed tree:
      // bitwise the sum the separate sparse product forms
      double* acc = v[q];
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] = 0.0 + (f0 + k < f1 ? acc[k] : 0.0);
      // rows with more than eight neighbours: groups of eight, the next
      // group's indices (wave-uniform, scalar loads) fetched while the
      // current group's rows are in flight, so a long row costs one memory
      // round trip per group rather than two
      int nx[8];
      if (f0 + 8 < f1) {
#pragma unroll
        for (int k = 0; k < 8; ++k) nx[k] = pv.h_idx[min(f0 + 8 + k, f1 - 1)];
      }
      for (int e = f0 + 8; e < f1; e += 8) {
        double u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = (double)base[q][(size_t)nx[k] * ld];
        if (e + 8 < f1) {
#pragma unroll
          for (int k = 0; k < 8; ++k) nx[k] = pv.h_idx[min(e + 8 + k, f1 - 1)];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += e + k < f1 ? u[k] : 0.0;
      }
      const double sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                         ((acc[4] + acc[5]) + (acc[6] + acc[7]));
      double val = sg * sum;
      if constexpr (sizeof(T) == 4) val = (double)(float)val;
      if (t < TE)
        ((lane >> 5) ? Ti : Tr)[t][cl] = val;
      else
        ((lane >> 5) ? Xi : Xr)[t - TE][cl] = val;
    }
  }
}

// One tile pair {(I, J), (J, I)}, I <= J, of the right-hand side and its RK4
// stage.  The state is Hermitian and L maps Hermitian to (bitwise) Hermitian,
// so only (I, J) is evaluated: y_n, the accumulator and the anchor residual
// are read there only (the accumulator is only ever stored there), while the
// next stage state -- which the product reads in full -- is written to (I, J)
// and, conjugated, to (J, I).
// XS_FUSED32S: every state plane (Y_s, y_n, the accumulator, the anchor
// residual and the output) is FP32 (the defect of the mixed solve held in
// single precision); the arithmetic stays FP64, each stored value is the
// FP32 rounding of the FP64 result, and the mirrored tile stores the
// conjugate of exactly that value (so the stored state stays bitwise
// Hermitian).
template <int XS, bool NT = false>
__device__ __forceinline__ void epilogue_tile(const ProbView& pv, const EpiArgs& a,
                                              DevState* __restrict__ st,
                                              double* __restrict__ partials, int tile) {
  __shared__ double Tr[TE][TE + 1], Ti[TE][TE + 1];
  __shared__ double Or[TE][TE + 1], Oi[TE][TE + 1];
  constexpr bool FUSED = XS == XS_FUSED64 || XS == XS_FUSED32 || XS == XS_FUSED32S;
  using ST = typename std::conditional<XS == XS_FUSED32S, float, double>::type;
  const ST* __restrict__ s_ysr = reinterpret_cast<const ST*>(a.ysr);
  const ST* __restrict__ s_ysi = reinterpret_cast<const ST*>(a.ysi);
  const ST* __restrict__ s_ynr = reinterpret_cast<const ST*>(a.ynr);
  const ST* __restrict__ s_yni = reinterpret_cast<const ST*>(a.yni);
  const ST* __restrict__ s_rar = reinterpret_cast<const ST*>(a.rar);
  const ST* __restrict__ s_rai = reinterpret_cast<const ST*>(a.rai);
  ST* s_accr = reinterpret_cast<ST*>(a.accr);
  ST* s_acci = reinterpret_cast<ST*>(a.acci);
  ST* s_outr = reinterpret_cast<ST*>(a.outr);
  ST* s_outi = reinterpret_cast<ST*>(a.outi);
  // fused: X(I, J) is gathered into Or/Oi; each thread reads its elements
  // there before it writes its outputs to the same places
  __shared__ double gs[TE];
  __shared__ double red[ETHREADS / 64];
  const int tid = threadIdx.x, tx = tid & (TE - 1), ty = tid / TE;
  const int n = pv.n, ld = pv.ld;
  int I, J;
  tri_decode(tile, I, J);
  const int a0 = I * TE, b0 = J * TE;
  const bool diag = I == J;
  const int b = b0 + tx;
  const bool bin = b < n;

  // All loads of this thread's four elements are issued before any store:
  // outputs may alias inputs (y_n is updated in place at the last RK4 stage),
  // so the compiler could not reorder them across the stores itself.
  const bool need_yn = a.mode != EPI_RHS;
  const bool need_acc = a.mode == EPI_S2 || a.mode == EPI_S3 || a.mode == EPI_S4;
  double xa[EM], xb[EM], yr_[EM], yi_[EM], nr_[EM], ni_[EM], cr_[EM], ci_[EM], rr_[EM], ri_[EM];
  // The accumulator and the Fehlberg stage derivatives are only ever touched
  // on the evaluated tile (I, J): they are stored Hermitian-packed by tile
  // pair -- pair t holds its 32 x 32 real block at [t][0] and imaginary block
  // at [t][1] (accr / kr[j] point at [0][0], acci / ki[j] = that + 32 * 32),
  // half the storage of two full planes, every access coalesced.
  // this thread's element m of the packed block sits at qoff + m * ERS * TE
  const unsigned qoff = (unsigned)tile * (2 * TE * TE) + (unsigned)(ty * TE + tx);
  // y_n, the anchor residual and the accumulator are read once per stage and
  // touched again only at the next stage: on large problems (NT) they are
  // loaded and the accumulator stored non-temporally, so they do not push the
  // gathered rows of Y_s out of the caches (at N = 4096: 249 -> 235 us per
  // FP32-state stage, 406 -> 397 us FP64; at N = 922, where the whole working
  // set stays cached, it costs ~7 % and is not used)
  auto ldt = [](const ST* p) -> double {
    if constexpr (NT) return (double)__builtin_nontemporal_load(p);
    else return (double)*p;
  };
  auto stt = [](ST* p, double v) {
    if constexpr (NT) __builtin_nontemporal_store((ST)v, p);
    else *p = (ST)v;
  };
  // The FP64 fused stage's output state (268 MB at N = 4096) cannot stay
  // cached until the next stage gathers it either, so there it is stored
  // non-temporally too (385 -> 375 us); an FP32 state (134 MB) can, and the
  // hint costs it 4 %
  auto sto = [](ST* p, double v) {
    if constexpr (NT && XS == XS_FUSED64) __builtin_nontemporal_store((ST)v, p);
    else *p = (ST)v;
  };
  auto load_state = [&](int m) {  // Y_s, anchor residual, y_n, accumulator at element m
    const int ar = a0 + ty + ERS * m;
    const size_t o = (size_t)ar * ld + b;
    const unsigned q = qoff + (unsigned)(m * ERS * TE);
    yr_[m] = yi_[m] = nr_[m] = ni_[m] = cr_[m] = ci_[m] = rr_[m] = ri_[m] = 0.0;
    if (bin && ar < n) {
      yr_[m] = (double)s_ysr[o];
      yi_[m] = (double)s_ysi[o];
      if (a.rar) {
        rr_[m] = ldt(&s_rar[o]);
        ri_[m] = ldt(&s_rai[o]);
      }
    }
    if (need_yn) {
      nr_[m] = ldt(&s_ynr[o]);
      ni_[m] = ldt(&s_yni[o]);
    }
    if (need_acc) {
      cr_[m] = ldt(&s_accr[q]);
      ci_[m] = ldt(&s_acci[q]);
    }
  };

  // transposed product tile: Tr[r][c] = X[b0 + r][a0 + c]
  if constexpr (XS == XS_FUSED32 || XS == XS_FUSED32S) {
    fused_gather<float>(pv, a.xfr, a.xfi, a0, b0, diag, Tr, Ti, Or, Oi);
  } else if constexpr (FUSED) {
    fused_gather<double>(pv, a.ysr, a.ysi, a0, b0, diag, Tr, Ti, Or, Oi);
  } else {
#pragma unroll
    for (int m = 0; m < EM; ++m) {
      const int r = ty + ERS * m;
      const size_t o = (size_t)(b0 + r) * ld + a0 + tx;
      if (XS != XS_DENSE32) {
        Tr[r][tx] = a.xr[o];
        Ti[r][tx] = a.xi[o];
      } else {
        Tr[r][tx] = (double)a.xfr[o];
        Ti[r][tx] = (double)a.xfi[o];
      }
    }
  }
  if (I == J) {  // gain of the jump terms on this tile's diagonal
    double sp = 0.0, sd = 0.0;
    for (int j = tid; j < n; j += ETHREADS) {
      const double v = a.ps[j];
      sp += v;
      sd += pv.dangling[j] ? v : 0.0;
    }
    const double P = block_sum(sp, red, ETHREADS / 64);
    const double D = block_sum(sd, red, ETHREADS / 64);
    // GL lanes per row, all 32 rows at once: lane k of a row takes in-links
    // k, k + GL, ... (four in flight), then a reduction over the GL lanes in
    // a fixed order.  The row sums are the critical path of a diagonal tile.
    GainView gv{n, pv.teleport, pv.alpha, pv.inv_outdeg, pv.dangling, pv.in_ptr, pv.in_idx};
    constexpr int GL = ETHREADS / TE;
    static_assert(GL <= 64 && (GL & (GL - 1)) == 0, "lanes of a row share a wave");
    const int q = tid / GL, k = tid % GL;
    const int ar = a0 + q;
    double sacc = 0.0;
    if (ar < n) {
      const int e1 = pv.in_ptr[ar + 1];
      int e = pv.in_ptr[ar] + k;
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
      for (; e + 3 * GL < e1; e += 4 * GL) {
        const int j0 = pv.in_idx[e], j1 = pv.in_idx[e + GL], j2 = pv.in_idx[e + 2 * GL],
                  j3 = pv.in_idx[e + 3 * GL];
        t0 += a.ps[j0] * pv.inv_outdeg[j0];
        t1 += a.ps[j1] * pv.inv_outdeg[j1];
        t2 += a.ps[j2] * pv.inv_outdeg[j2];
        t3 += a.ps[j3] * pv.inv_outdeg[j3];
      }
      for (; e < e1; e += GL) {
        const int j = pv.in_idx[e];
        t0 += a.ps[j] * pv.inv_outdeg[j];
      }
      sacc = (t0 + t1) + (t2 + t3);
    }
#pragma unroll
    for (int off = 1; off < GL; off <<= 1) sacc += __shfl_xor(sacc, off, 64);
    if (k == 0 && ar < n) gs[q] = gain_finish(gv, ar, a.ps, P, D, sacc);
  }
  __syncthreads();

  const double w = a.omega, cw = 1.0 - a.omega;
  const double hb = bin ? pv.h[b] : 0.0, db = bin ? pv.d[b] : 0.0;
  double ssum = 0.0, emax = 0.0;
  int sbad = 0;
  const int fstage = a.mode >= EPI_F1 ? a.mode - EPI_F1 + 1 : 0;  // Fehlberg stage 1..6
  const double hstep = fstage ? st->h : 0.0;
#pragma unroll
  for (int m = 0; m < EM; ++m) {
    const int ar = a0 + ty + ERS * m;
    const size_t o = (size_t)ar * ld + b;
    xa[m] = xb[m] = 0.0;
    if (bin && ar < n) {
      if (FUSED) {  // X(I, J) from LDS (the diagonal block is Tr/Ti itself)
        const int r = ty + ERS * m;
        xa[m] = diag ? Tr[r][tx] : Or[r][tx];
        xb[m] = diag ? Ti[r][tx] : Oi[r][tx];
      } else if (XS != XS_DENSE32) {
        xa[m] = a.xr[o];
        xb[m] = a.xi[o];
      } else {
        xa[m] = (double)a.xfr[o];
        xb[m] = (double)a.xfi[o];
      }
    }
    load_state(m);
  }
#pragma unroll
  for (int m = 0; m < EM; ++m) {
    const int r = ty + ERS * m;
    const int ar = a0 + r;
    const size_t o = (size_t)ar * ld + b;
    const unsigned q = qoff + (unsigned)(m * ERS * TE);  // packed accumulator / derivatives
    double kr = 0.0, ki = 0.0;
    const bool inside = bin && ar < n;
    if (inside) {
      const double A_ab = xa[m], B_ab = xb[m];
      const double A_ba = Tr[tx][r], B_ba = Ti[tx][r];
      const double R = yr_[m], Im = yi_[m];
      const double hab = pv.h[ar] - hb;
      const double dab = 0.5 * (pv.d[ar] + db);
      const double gd = (ar == b) ? gs[r] : 0.0;
      kr = cw * ((B_ab + B_ba) + hab * Im) + w * (gd - dab * R);
      ki = cw * ((A_ba - A_ab) - hab * R) - w * (dab * Im);
      if (a.rar) {
        kr += rr_[m];
        ki += ri_[m];
      }
      ssum += (diag ? 1.0 : 2.0) * (kr * kr + ki * ki);
      sbad |= !(isfinite(kr) && isfinite(ki));
    }
    double outr, outi;
    switch (a.mode) {
      case EPI_RHS:
        outr = kr;
        outi = ki;
        break;
      case EPI_S1:
        stt(&s_accr[q], kr);
        stt(&s_acci[q], ki);
        outr = nr_[m] + a.cdt * kr;
        outi = ni_[m] + a.cdt * ki;
        break;
      case EPI_S2:
      case EPI_S3:
        stt(&s_accr[q], cr_[m] + 2.0 * kr);
        stt(&s_acci[q], ci_[m] + 2.0 * ki);
        outr = nr_[m] + a.cdt * kr;
        outi = ni_[m] + a.cdt * ki;
        break;
      case EPI_S4:  // y_{n+1} = y_n + dt/6 (acc + k4)
        outr = nr_[m] + a.cdt * (cr_[m] + kr);
        outi = ni_[m] + a.cdt * (ci_[m] + ki);
        break;
      default: {  // Fehlberg stage fstage: K_s = k; next stage input, or at
                  // stage 6 the fourth-order candidate and the error estimate
        double sr = 0.0, si = 0.0, er = 0.0, ei = 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j)
          if (j < fstage - 1) {
            const double kjr = a.kr[j][q], kji = a.ki[j][q];
            sr += a.cf[j] * kjr;
            si += a.cf[j] * kji;
            er += a.ce[j] * kjr;
            ei += a.ce[j] * kji;
          }
        sr += a.cf[fstage - 1] * kr;
        si += a.cf[fstage - 1] * ki;
        er += a.ce[fstage - 1] * kr;
        ei += a.ce[fstage - 1] * ki;
        if (fstage < 6) {
          a.kwr[q] = kr;
          a.kwi[q] = ki;
        } else if (inside) {
          emax = fmax(emax, hstep * sqrt(er * er + ei * ei));
        }
        outr = nr_[m] + hstep * sr;
        outi = ni_[m] + hstep * si;
        break;
      }
    }
    if (!inside) {
      outr = 0.0;
      outi = 0.0;
    }
    if constexpr (sizeof(ST) == 4) {  // the stored (FP32) value, mirrored below as is
      outr = (double)(float)outr;
      outi = (double)(float)outi;
    }
    sto(&s_outr[o], outr);
    sto(&s_outi[o], outi);
    if (!diag) {
      Or[r][tx] = outr;
      Oi[r][tx] = outi;
    }
    if (a.pout && inside && ar == b) a.pout[ar] = outr;
    if (a.lor) {
      a.lor[o] = (float)outr;
      a.loi[o] = (float)outi;
    }
    if (a.slices) {
      const size_t plane = (size_t)ld * ld;
      uint16_t s1, s2, s3;
      split3(outr, s1, s2, s3);
      a.slices[o] = s1;
      a.slices[plane + o] = s2;
      a.slices[2 * plane + o] = s3;
      // imaginary plane stored negated: row b of -I is column b of I
      split3(-outi, s1, s2, s3);
      a.slices[3 * plane + o] = s1;
      a.slices[4 * plane + o] = s2;
      a.slices[5 * plane + o] = s3;
    }
  }

  if (!diag) {
    // mirror tile (J, I) = conj of tile (I, J), written row-major through LDS
    __syncthreads();
#pragma unroll
    for (int m = 0; m < EM; ++m) {
      const int r = ty + ERS * m;
      const size_t o = (size_t)(b0 + r) * ld + a0 + tx;
      const double outr = Or[tx][r], outi = -Oi[tx][r];
      sto(&s_outr[o], outr);
      sto(&s_outi[o], outi);
      if (a.lor) {
        a.lor[o] = (float)outr;
        a.loi[o] = (float)outi;
      }
      if (a.slices) {
        const size_t plane = (size_t)ld * ld;
        uint16_t s1, s2, s3;
        split3(outr, s1, s2, s3);
        a.slices[o] = s1;
        a.slices[plane + o] = s2;
        a.slices[2 * plane + o] = s3;
        split3(-outi, s1, s2, s3);
        a.slices[3 * plane + o] = s1;
        a.slices[4 * plane + o] = s2;
        a.slices[5 * plane + o] = s3;
      }
    }
  }

  if (a.mode == EPI_S1 || a.mode == EPI_RHS || fstage == 1 || fstage == 6)
    tile_partials(ssum, sbad, emax, partials, red, tile);
}

// Fehlberg stage number (1..6) of an epilogue mode, 0 for the others.
__host__ __device__ __forceinline__ int fehlberg_stage(int mode) {
  return mode >= EPI_F1 ? mode - EPI_F1 + 1 : 0;
}

// Whether an epilogue mode leaves partials for the finishing kernel.
__host__ __device__ __forceinline__ bool reduces(int mode) {
  const int f = fehlberg_stage(mode);
  return mode == EPI_S1 || mode == EPI_RHS || f == 1 || f == 6;
}

// The control block's update from the combined reductions of one stage:
// residual, convergence and step counting per check mode, or at the sixth
// Fehlberg stage the step control.
__device__ void finish_control(DevState* st, int check, int fstage, double tot, int bad,
                               double mx) {
  if (fstage == 6) {
    // Fehlberg step control (Supplementary Note 2, Eq. (S13)): accept when
    // |z - y| <= Tol h, next step h * (Tol h / (2 |z - y|))^(1/4), the factor
    // clamped to [0.1, 4] and the step to h_max.
    const double h = st->h, tolh = st->tol_step * h;
    const int ok = !bad && mx <= tolh;
    st->err = mx;
    st->accept = ok;
    if (ok) {
      st->t += h;
      st->accepted += 1;
    } else {
      st->rejected += 1;
    }
    if (bad) {
      st->nonfinite = 1;
      st->stop = 1;
    }
    double fac = mx > 0.0 ? pow(tolh / (2.0 * mx), 0.25) : 4.0;
    fac = fmin(4.0, fmax(0.1, fac));
    st->h = fmin(h * fac, st->h_max);
    return;
  }
  st->resid2 = tot;
  st->rhs_evals += 1;
  if (bad) {
    st->nonfinite = 1;
    st->stop = 1;
  } else if (check == CHK_PLAIN) {
    if (tot < st->tol2) {
      st->converged = 1;
      st->conv_step = st->step;
      st->stop = 1;
    } else if (st->step >= st->max_steps) {
      st->stop = 1;
    } else {
      st->step += 1;
    }
  } else if (check == CHK_DELTA) {
    // ||r_a + L_lowp(delta)|| estimates the residual of rho_a + delta: once it
    // meets 0.9 tol (or the step budget is spent) hold further steps so the
    // FP64 fold and judge run.
    if (tot < 0.81 * st->tol2 || st->step >= st->max_steps) st->hold = 1;
    else st->step += 1;
  } else if (check == CHK_RKF) {
    if (tot < st->tol2) {
      st->converged = 1;
      st->conv_step = st->accepted;
      st->stop = 1;
    } else if (st->step >= st->max_steps) {
      st->stop = 1;
    } else {
      st->step += 1;  // attempts
    }
  } else if (check == CHK_JUDGE) {
    st->judge2 = tot;
    st->folds += 1;
    if (tot < st->tol2) {
      st->converged = 1;
      st->conv_step = st->step;
      st->stop = 1;
    } else if (st->step >= st->max_steps) {
      st->stop = 1;
    } else {
      st->hold = 0;
    }
  }
}

// The finishing step of a reducing stage: fold its partials and update the
// control block.  Called by all FOLD_THREADS threads of the workgroup.
// Inlined: an out-of-line call gives the calling kernel a stack, whose set-up
// every wave pays (the row-major product went from 12 to 22 us at N = 922).
__device__ __forceinline__ void run_finish(const FinishJob& f) {
  DevState* st = f.st;
  if (st->stop || (f.gate && st->hold)) return;  // uniform: only this step writes them
  double tot, mx;
  int bad;
  fold_partials(f.partials, f.nb, tot, bad, mx);
  if (threadIdx.x == 0) finish_control(st, f.check, f.fstage, tot, bad, mx);
}

__global__ void __launch_bounds__(FOLD_THREADS) k_finish(FinishJob f) { run_finish(f); }

// One workgroup per running system (grid-stride over the system list).
__global__ void __launch_bounds__(FOLD_THREADS)
    k_finish_batch(const BatchEpi* __restrict__ args, const int* __restrict__ sys_list,
                   const int* __restrict__ nsys) {
  const int ns = *nsys;
  for (int it = blockIdx.x; it < ns; it += gridDim.x) {
    const BatchEpi& e = args[sys_list[it]];
    run_finish(FinishJob{e.partials, tri_tiles(e.pv.ld / TE), e.st, e.a.check,
                         fehlberg_stage(e.a.mode), e.a.gate});
  }
}

// six waves per SIMD (<= 80 VGPRs, no spills): three 512-thread workgroups
// per CU instead of two at the unconstrained 88 VGPRs
template <int XS, bool NT = false>
__global__ void __launch_bounds__(ETHREADS) __attribute__((amdgpu_waves_per_eu(6, 6)))
    k_epilogue(ProbView pv, EpiArgs a, DevState* __restrict__ st, double* __restrict__ partials) {
  if (st->stop || (a.gate && st->hold)) return;
  epilogue_tile<XS, NT>(pv, a, st, partials, blockIdx.x);
}

// The fused form (the sparse product gathered inside the tile), also at six
// waves per SIMD: with X sharing the output tiles it needs 34 KB of LDS, so
// three workgroups fit per CU.  Two gathers of eight rows in flight per wave
// keep it within 80 VGPRs; one more wave per SIMD would spill.
//
// It may carry the previous stage's finishing step as workgroup 0 (f.nb > 0),
// all 512 threads taking part.  The tiles then run beside it: a stop it sets
// is seen by some tiles of this launch and not others, which is harmless
// because the stages that follow stage 1 write only the next stage's inputs
// (y_n is written last, by stage 4 or the RKF45 commit, both gated), and the
// only control value they read, the RKF45 step size, changes at stage 6 only.
// With `xcd` set the tile pairs are renumbered so that each XCD takes one
// contiguous run of them: tile pairs are ordered by column block J, and the
// X(I, J) half of the gathers reads Y's block J only, so that slice stays in
// one L2 (fewer fetched bytes; at N = 4096 and above it costs more than it
// saves).
template <int XS, bool NT = false>
__global__ void __launch_bounds__(ETHREADS) __attribute__((amdgpu_waves_per_eu(6, 6)))
    k_epilogue_fused(ProbView pv, EpiArgs a, DevState* __restrict__ st,
                     double* __restrict__ partials, FinishJob f, int xcd) {
  const int extra = f.nb > 0;
  if (extra && blockIdx.x == 0) {
    run_finish(f);
    return;
  }
  if (st->stop || (a.gate && st->hold)) return;
  const int nb = gridDim.x - extra, bid = blockIdx.x - extra;
  epilogue_tile<XS, NT>(pv, a, st, partials, xcd ? xcd_contiguous(bid, nb) : bid);
}

// Batched form for many systems: workgroup i takes item i of the device-side
// (system, tile pair) list and the workgroups past its current length exit
// at once (the grid covers the list as built, before any system stopped).
// Without a grid-stride loop the tile code fits six waves per SIMD like the
// single-system kernel (the loop kept 106-115 VGPRs live: four waves, and
// 160 family systems took 9-21 % longer).  Each tile writes its partials into
// its own system's buffer; k_finish_batch folds them.
template <int XS>
__global__ void __launch_bounds__(ETHREADS) __attribute__((amdgpu_waves_per_eu(6, 6)))
    k_epilogue_batch(const BatchEpi* __restrict__ args, const int2* __restrict__ items,
                     const int* __restrict__ nitems) {
  if ((int)blockIdx.x >= *nitems) return;
  const int2 item = items[blockIdx.x];
  const BatchEpi& e = args[item.x];
  DevState* st = e.st;
  if (st->stop || (e.a.gate && st->hold)) return;
  epilogue_tile<XS>(e.pv, e.a, st, e.partials, item.y);
}

// Sparse commutator product X = H_off Y (FP64) through the CSR of H_off.
// Row a of X is the sum of the rows j of Y with (H_off)_aj != 0 (all entries
// are +-1), so the product is a gather: per output element, deg_H(a) loads.
//
// The neighbour list of a row is taken in groups of eight whose loads are all
// issued before any is used (see gather_rows for the short last group).
// Element e of the list goes to partial sum (e - e0) % 8 and the partials are
// added as ((0+1)+(2+3))+((4+5)+(6+7)): every variant gives bitwise the same X.
//
// Variants (one wave per (row, W columns of both planes) unless noted):
//  * column-chunk major (SpmmCM<W, RPW>): W = 32: lanes 0-31 take the real
//    plane, 32-63 the imaginary one; W = 64: lane l column l of both planes;
//    W = 128: lane l columns 2l, 2l+1 of both planes.  RPW rows per wave, four
//    waves per workgroup.  Workgroups are numbered chunk-major and remapped so
//    that each XCD (dispatch is round-robin over the 8 XCDs) owns a contiguous
//    run of column chunks: the Y rows one XCD gathers at a time are a
//    2 W x ld x 8-byte slice rather than the whole matrix.
//  * row major: workgroup (row, 128-column chunk), 256 threads, thread t
//    plane t / 128 and column t % 128; guarded (not predicated) short group.
// Measured on BA graphs: the row-major kernel is fastest at N ~ 1000 (the
// predicated loads cost more than the latency they hide there), 128-column
// chunks at N >= 2048.
// Rows a >= n are left untouched (the epilogue never reads them).
constexpr int SP_COLS = 128;
constexpr int SP_WAVES = 4;
static_assert(2 * SP_COLS == FOLD_THREADS && 64 * SP_WAVES == FOLD_THREADS,
              "a sparse-product workgroup can run the finishing step");

// Sum over the neighbour rows j of a of Y_s[j * ld] for S streams (pointers
// already offset to the lane's column); the row range [e0, e1) is uniform.
// Full groups of eight issue all their loads first.  The last, short group is
// either predicated (PRED: eight loads, the missing ones repeating the last
// neighbour and masked out) or taken one guarded load at a time (no extra
// requests; better where the memory system rather than latency is the limit).
template <int S, bool PRED, typename T = double>
__device__ __forceinline__ void gather_rows(const int* __restrict__ h_idx, int e0, int e1, int ld,
                                            const T* const (&base)[S], double (&out)[S]) {
  double acc[8][S];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int q = 0; q < S; ++q) acc[k][q] = 0.0;
  int e = e0;
  // the next full group's indices are fetched while the current group's rows
  // are in flight (one memory round trip per group, not two)
  int nx[8];
  if (e + 8 <= e1) {
#pragma unroll
    for (int k = 0; k < 8; ++k) nx[k] = h_idx[e + k];
  }
  for (; e + 8 <= e1; e += 8) {
    size_t off[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) off[k] = (size_t)nx[k] * ld;
    double v[8][S];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int q = 0; q < S; ++q) v[k][q] = (double)base[q][off[k]];
    if (e + 16 <= e1) {
#pragma unroll
      for (int k = 0; k < 8; ++k) nx[k] = h_idx[e + 8 + k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int q = 0; q < S; ++q) acc[k][q] += v[k][q];
  }
  if (e < e1) {
    if (PRED) {
      size_t off[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) off[k] = (size_t)h_idx[min(e + k, e1 - 1)] * ld;
      double v[8][S];
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int q = 0; q < S; ++q) v[k][q] = (double)base[q][off[k]];
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int q = 0; q < S; ++q) acc[k][q] += e + k < e1 ? v[k][q] : 0.0;
    } else {
#pragma unroll
      for (int k = 0; k < 7; ++k)
        if (e + k < e1) {
          const size_t o = (size_t)h_idx[e + k] * ld;
#pragma unroll
          for (int q = 0; q < S; ++q) acc[k][q] += (double)base[q][o];
        }
    }
  }
#pragma unroll
  for (int q = 0; q < S; ++q)
    out[q] = ((acc[0][q] + acc[1][q]) + (acc[2][q] + acc[3][q])) +
             ((acc[4][q] + acc[5][q]) + (acc[6][q] + acc[7][q]));
}

template <int W>
__device__ __forceinline__ void spmm_wave_row(const ProbView& pv, const double* __restrict__ yr,
                                              const double* __restrict__ yi,
                                              double* __restrict__ xr, double* __restrict__ xi,
                                              int a, int chunk) {
  const int l = threadIdx.x & 63;
  const int ld = pv.ld;
  const int e0 = pv.h_ptr[a], e1 = pv.h_ptr[a + 1];
  const double sg = (double)pv.hsign;
  const size_t row = (size_t)a * ld;
  if (W == 32) {
    const int c = chunk * 32 + (l & 31);
    const double* const b[1] = {(l < 32 ? yr : yi) + c};
    double o[1];
    gather_rows<1, true>(pv.h_idx, e0, e1, ld, b, o);
    (l < 32 ? xr : xi)[row + c] = sg * o[0];
  } else if (W == 64) {
    const int c = chunk * 64 + l;
    const double* const b[2] = {yr + c, yi + c};
    double o[2];
    gather_rows<2, true>(pv.h_idx, e0, e1, ld, b, o);
    xr[row + c] = sg * o[0];
    xi[row + c] = sg * o[1];
  } else {
    const int c = chunk * 128 + 2 * l;
    const double* const b[4] = {yr + c, yr + c + 1, yi + c, yi + c + 1};
    double o[4];
    gather_rows<4, true>(pv.h_idx, e0, e1, ld, b, o);
    *(double2*)(xr + row + c) = make_double2(sg * o[0], sg * o[1]);
    *(double2*)(xi + row + c) = make_double2(sg * o[2], sg * o[3]);
  }
}

// Workgroups per column chunk for the chunk-major variants.
template <int RPW>
__host__ __device__ __forceinline__ int spmm_cm_groups(int n) {
  return (n + SP_WAVES * RPW - 1) / (SP_WAVES * RPW);
}

// One logical workgroup (chunk, row group) of a chunk-major variant.
template <int W, int RPW>
__device__ __forceinline__ void spmm_cm_group(const ProbView& pv, const double* __restrict__ yr,
                                              const double* __restrict__ yi,
                                              double* __restrict__ xr, double* __restrict__ xi,
                                              int logical) {
  const int groups = spmm_cm_groups<RPW>(pv.n);
  const int chunk = logical / groups, g = logical - chunk * groups;
  // the row index is uniform over the wave: keep it (and the CSR reads) scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int a0 = (g * SP_WAVES + wave) * RPW;
#pragma unroll 1
  for (int r = 0; r < RPW; ++r) {
    const int a = a0 + r;
    if (a >= pv.n) return;
    spmm_wave_row<W>(pv, yr, yi, xr, xi, a, chunk);
  }
}


// The row-major and FP32 product launches may carry the finishing step of
// the previous stage as one extra workgroup, the first one dispatched
// (f.nb > 0), so that it overlaps the product: the product itself does not
// depend on the control block, and the next epilogue checks the flags that
// step sets.  The chunk-major FP64 kernels do not (FinishJob unused): at
// 124-128 VGPRs the call took the registers that keep a group's gathers in
// flight, and where they are the default (N >= 1536) a separate finishing
// launch costs < 0.5 % of a stage.
template <int W, int RPW>
__global__ void __launch_bounds__(64 * SP_WAVES)
    k_spmm_cm(ProbView pv, const double* __restrict__ yr, const double* __restrict__ yi,
              double* __restrict__ xr, double* __restrict__ xi, const DevState* __restrict__ st,
              int gate, FinishJob) {
  if (st->stop || (gate && st->hold)) return;
  spmm_cm_group<W, RPW>(pv, yr, yi, xr, xi, xcd_contiguous(blockIdx.x, gridDim.x));
}

__global__ void __launch_bounds__(2 * SP_COLS)
    k_spmm(ProbView pv, const double* __restrict__ yr, const double* __restrict__ yi,
           double* __restrict__ xr, double* __restrict__ xi, const DevState* __restrict__ st,
           int gate, FinishJob f) {
  const int extra = f.nb > 0;
  if (extra && blockIdx.x == 0) {
    run_finish(f);
    return;
  }
  if (st->stop || (gate && st->hold)) return;
  const int chunks = (pv.ld + SP_COLS - 1) / SP_COLS;
  const int bid = blockIdx.x - extra;
  const int a = __builtin_amdgcn_readfirstlane(bid / chunks);
  const int t = threadIdx.x, c = (bid % chunks) * SP_COLS + (t & (SP_COLS - 1));
  if (c >= pv.ld) return;
  const double* const b[1] = {(t < SP_COLS ? yr : yi) + c};
  double o[1];
  gather_rows<1, false>(pv.h_idx, pv.h_ptr[a], pv.h_ptr[a + 1], pv.ld, b, o);
  (t < SP_COLS ? xr : xi)[(size_t)a * pv.ld + c] = (double)pv.hsign * o[0];
}

// FP32 operand form for the mixed-precision steps: the gathered rows are the
// FP32 copy of the stage state (the defect delta), summed in FP64 in the order
// above and rounded once to FP32 for X.  Column chunks as in the FP64
// chunk-major variants: W = 32 (lanes 0-31 real plane, 32-63 imaginary),
// W = 64 (lane l: column l of both planes), W = 128 (lane l: columns 2l,
// 2l+1 of both planes).
template <int W>
__device__ __forceinline__ void spmm_f32_row(const ProbView& pv, const float* __restrict__ yr,
                                             const float* __restrict__ yi,
                                             float* __restrict__ xr, float* __restrict__ xi,
                                             int a, int chunk) {
  const int l = threadIdx.x & 63, ld = pv.ld;
  const int e0 = pv.h_ptr[a], e1 = pv.h_ptr[a + 1];
  const double sg = (double)pv.hsign;
  const size_t row = (size_t)a * ld;
  if (W == 32) {
    const int c = chunk * 32 + (l & 31);
    const float* const b[1] = {(l < 32 ? yr : yi) + c};
    double o[1];
    gather_rows<1, true, float>(pv.h_idx, e0, e1, ld, b, o);
    (l < 32 ? xr : xi)[row + c] = (float)(sg * o[0]);
  } else if (W == 64) {
    const int c = chunk * 64 + l;
    const float* const b[2] = {yr + c, yi + c};
    double o[2];
    gather_rows<2, true, float>(pv.h_idx, e0, e1, ld, b, o);
    xr[row + c] = (float)(sg * o[0]);
    xi[row + c] = (float)(sg * o[1]);
  } else {
    const int c = chunk * 128 + 2 * l;
    const float* const b[4] = {yr + c, yr + c + 1, yi + c, yi + c + 1};
    double o[4];
    gather_rows<4, true, float>(pv.h_idx, e0, e1, ld, b, o);
    *(float2*)(xr + row + c) = make_float2((float)(sg * o[0]), (float)(sg * o[1]));
    *(float2*)(xi + row + c) = make_float2((float)(sg * o[2]), (float)(sg * o[3]));
  }
}

// one logical workgroup (chunk, group of four rows) of the FP32 form
template <int W>
__device__ __forceinline__ void spmm_f32_group(const ProbView& pv, const float* yr,
                                               const float* yi, float* xr, float* xi,
                                               int logical) {
  const int groups = spmm_cm_groups<1>(pv.n);
  const int chunk = logical / groups, g = logical - chunk * groups;
  const int a = g * SP_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (a < pv.n) spmm_f32_row<W>(pv, yr, yi, xr, xi, a, chunk);
}

template <int W>
__global__ void __launch_bounds__(64 * SP_WAVES)
    k_spmm_f32(ProbView pv, const float* __restrict__ yr, const float* __restrict__ yi,
               float* __restrict__ xr, float* __restrict__ xi, const DevState* __restrict__ st,
               int gate, FinishJob f) {
  const int extra = f.nb > 0;
  if (extra && blockIdx.x == 0) {
    run_finish(f);
    return;
  }
  if (st->stop || (gate && st->hold)) return;
  spmm_f32_group<W>(pv, yr, yi, xr, xi, xcd_contiguous(blockIdx.x - extra, gridDim.x - extra));
}

// One row-major item (row a, 128-column chunk) of the sparse product for the
// batched kernels (the systems of a batch have N <= ~1000, where the row-major
// layout is fastest): thread t takes plane t / 128 and column c0 + t % 128.
template <typename T, typename TX>
__device__ __forceinline__ void spmm_row_item(const ProbView& pv, const T* __restrict__ yr,
                                              const T* __restrict__ yi, TX* __restrict__ xr,
                                              TX* __restrict__ xi, int item) {
  const int chunks = (pv.ld + SP_COLS - 1) / SP_COLS;
  const int a = __builtin_amdgcn_readfirstlane(item / chunks);
  const int t = threadIdx.x, c = (item % chunks) * SP_COLS + (t & (SP_COLS - 1));
  if (c >= pv.ld) return;
  const T* const b[1] = {(t < SP_COLS ? yr : yi) + c};
  double o[1];
  gather_rows<1, false, T>(pv.h_idx, pv.h_ptr[a], pv.h_ptr[a + 1], pv.ld, b, o);
  (t < SP_COLS ? xr : xi)[(size_t)a * pv.ld + c] = (TX)((double)pv.hsign * o[0]);
}

// Persistent FP32 form over (system, row * chunks + chunk) items; operand =
// the system's FP32 state copy (a.lor), result into its FP32 product planes.
__global__ void __launch_bounds__(2 * SP_COLS)
    k_spmm_f32_batch(const BatchEpi* __restrict__ args, const int2* __restrict__ items,
                     const int* __restrict__ nitems) {
  const int ni = *nitems;
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    const int2 item = items[it];
    const BatchEpi& e = args[item.x];
    if (e.st->stop || (e.a.gate && e.st->hold)) continue;
    spmm_row_item<float, float>(e.pv, e.a.lor, e.a.loi, (float*)e.a.xfr, (float*)e.a.xfi, item.y);
  }
}

// Persistent FP64 form over (system, row * chunks + chunk) items.
__global__ void __launch_bounds__(2 * SP_COLS)
    k_spmm_batch(const BatchEpi* __restrict__ args, const int2* __restrict__ items,
                 const int* __restrict__ nitems) {
  const int ni = *nitems;
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    const int2 item = items[it];
    const BatchEpi& e = args[item.x];
    if (e.st->stop || (e.a.gate && e.st->hold)) continue;
    spmm_row_item<double, double>(e.pv, e.a.ysr, e.a.ysi, (double*)e.a.xr, (double*)e.a.xi,
                                  item.y);
  }
}

// planar n x n (unpadded) -> ld x ld planes with zero padding, p = Re diag
__global__ void k_pad_in(const double* __restrict__ rho, int n, int ld, double* __restrict__ r,
                         double* __restrict__ im, double* __restrict__ p) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t tot = (size_t)ld * ld;
  if (idx >= tot) return;
  const int a = (int)(idx / ld), b = (int)(idx % ld);
  double vr = 0.0, vi = 0.0;
  if (a < n && b < n) {
    vr = rho[(size_t)a * n + b];
    vi = rho[(size_t)n * n + (size_t)a * n + b];
  }
  r[idx] = vr;
  im[idx] = vi;
  if (p && a == b && a < n) p[a] = vr;
}

__global__ void k_pad_out(const double* __restrict__ r, const double* __restrict__ im, int n,
                          int ld, double* __restrict__ rho) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t tot = (size_t)n * n;
  if (idx >= tot) return;
  const int a = (int)(idx / n), b = (int)(idx % n);
  rho[idx] = r[(size_t)a * ld + b];
  rho[tot + idx] = im[(size_t)a * ld + b];
}

__global__ void k_to_f32(const double* __restrict__ r, const double* __restrict__ im, size_t tot,
                         float* __restrict__ fr, float* __restrict__ fi) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  fr[idx] = (float)r[idx];
  fi[idx] = (float)im[idx];
}

__global__ void k_to_bf16x3(const double* __restrict__ r, const double* __restrict__ im,
                            size_t tot, uint16_t* __restrict__ sl) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  uint16_t s1, s2, s3;
  split3(r[idx], s1, s2, s3);
  sl[idx] = s1;
  sl[tot + idx] = s2;
  sl[2 * tot + idx] = s3;
  split3(-im[idx], s1, s2, s3);
  sl[3 * tot + idx] = s1;
  sl[4 * tot + idx] = s2;
  sl[5 * tot + idx] = s3;
}

__global__ void k_state_init(DevState* st, double tol, long long max_steps, int check) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->resid2 = 0.0;
  st->tol2 = tol * tol;
  st->step = 0;
  st->max_steps = max_steps;
  st->conv_step = -1;
  st->rhs_evals = 0;
  st->stop = 0;
  st->converged = 0;
  st->nonfinite = 0;
  st->check = check;
  st->ticket = 0u;
  st->hold = 0;
  st->judge2 = 0.0;
  st->folds = 0;
  for (int i = 0; i < 8; ++i) st->aux[i] = 0.0;
}

__global__ void k_state_rkf(DevState* st, double h0, double h_max, double tol_step) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->h = h0;
  st->h_max = h_max;
  st->tol_step = tol_step;
  st->t = 0.0;
  st->err = 0.0;
  st->accepted = 0;
  st->rejected = 0;
  st->accept = 0;
}

// st->aux[0] = sum_a p_a (one workgroup, fixed order); skipped once stopped
__global__ void __launch_bounds__(1024) k_trace(const double* __restrict__ p, int n,
                                                DevState* __restrict__ st) {
  __shared__ double red[16];
  if (st->stop) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += p[i];
  s = block_sum_1024(s, red);
  if (threadIdx.x == 0) st->aux[0] = s;
}

// Final-state diagnostics: trace, max |Y - Y^dag|, min diag, non-finite.
// Partial results per block, then the last block folds them into st->aux:
// aux[0] = tr, aux[1] = herm err, aux[2] = min diag, aux[3] = non-finite.
__global__ void __launch_bounds__(256) k_state_stats(const double* __restrict__ r,
                                                     const double* __restrict__ im,
                                                     const double* __restrict__ p, int n, int ld,
                                                     DevState* st, double* partials) {
  __shared__ double red[4];
  __shared__ int flag;
  const int tid = threadIdx.x;
  const size_t tot = (size_t)n * n;
  double herm = 0.0;
  int bad = 0;
  for (size_t idx = (size_t)blockIdx.x * 256 + tid; idx < tot; idx += (size_t)gridDim.x * 256) {
    const int a = (int)(idx / n), b = (int)(idx % n);
    const double xr = r[(size_t)a * ld + b], xi = im[(size_t)a * ld + b];
    const double yr = r[(size_t)b * ld + a], yi = im[(size_t)b * ld + a];
    herm = fmax(herm, fmax(fabs(xr - yr), fabs(xi + yi)));
    bad |= !(isfinite(xr) && isfinite(xi));
  }
  double tr = 0.0, mn = 1e300;
  for (int i = (int)blockIdx.x * 256 + tid; i < n; i += gridDim.x * 256) {
    tr += p[i];
    mn = fmin(mn, p[i]);
  }
  // block reductions (fixed order)
  tr = block_sum(tr, red, 4);
  herm = wave_max_d(herm);
  mn = wave_min_d(mn);
  __shared__ double hm[4], mm[4];
  if ((tid & 63) == 0) {
    hm[tid >> 6] = herm;
    mm[tid >> 6] = mn;
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) {
    double h = 0.0, m = 1e300;
    for (int w = 0; w < 4; ++w) {
      h = fmax(h, hm[w]);
      m = fmin(m, mm[w]);
    }
    partials[4 * blockIdx.x + 0] = tr;
    partials[4 * blockIdx.x + 1] = h;
    partials[4 * blockIdx.x + 2] = m;
    partials[4 * blockIdx.x + 3] = bad;
    __threadfence();
    const unsigned int t = atomicAdd(&st->ticket, 1u);
    flag = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (flag && tid == 0) {
    __threadfence();
    double T = 0.0, Hm = 0.0, Mn = 1e300, B = 0.0;
    for (unsigned int i = 0; i < gridDim.x; ++i) {
      T += partials[4 * i + 0];
      Hm = fmax(Hm, partials[4 * i + 1]);
      Mn = fmin(Mn, partials[4 * i + 2]);
      B = fmax(B, partials[4 * i + 3]);
    }
    st->aux[0] = T;
    st->aux[1] = Hm;
    st->aux[2] = Mn;
    st->aux[3] = B;
    st->ticket = 0u;
  }
}

// Rank by counting: position of i = #{j : p_j > p_i or (p_j == p_i and j < i)}.
__global__ void __launch_bounds__(256) k_rank(int n, const double* __restrict__ p,
                                              int* __restrict__ order) {
  __shared__ double ps[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double pi = i < n ? p[i] : 0.0;
  int cnt = 0;
  for (int j0 = 0; j0 < n; j0 += 256) {
    const int j = j0 + threadIdx.x;
    ps[threadIdx.x] = j < n ? p[j] : 0.0;
    __syncthreads();
    const int lim = min(256, n - j0);
    for (int t = 0; t < lim; ++t) {
      const double q = ps[t];
      cnt += (q > pi) || (q == pi && j0 + t < i);
    }
    __syncthreads();
  }
  if (i < n) order[cnt] = i;
}

// Hub classes of the results section: counts of p_i > c/N (main hubs) and
// 1/N < p_i <= c/N (secondary hubs); one workgroup, out[0..1] (device ints).
__global__ void __launch_bounds__(1024) k_hubs(int n, const double* __restrict__ p, double c,
                                               int* __restrict__ out) {
  __shared__ int red[2][1024];
  const int t = threadIdx.x;
  const double hi = c / (double)n, lo = 1.0 / (double)n;
  int m = 0, s2 = 0;
  for (int i = t; i < n; i += 1024) {
    const double v = p[i];
    m += v > hi;
    s2 += (v > lo) && (v <= hi);
  }
  red[0][t] = m;
  red[1][t] = s2;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) {
      red[0][t] += red[0][t + off];
      red[1][t] += red[1][t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

// Fehlberg: y <- candidate when the attempt was accepted (and not stopped)
__global__ void k_rkf_commit(double* __restrict__ yr, double* __restrict__ yi,
                             double* __restrict__ p, const double* __restrict__ cr,
                             const double* __restrict__ ci, const double* __restrict__ pc, int n,
                             int ld, const DevState* __restrict__ st) {
  if (st->stop || !st->accept) return;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ld * ld) return;
  yr[idx] = cr[idx];
  yi[idx] = ci[idx];
  if (idx < (size_t)n) p[idx] = pc[idx];
}

__global__ void k_axpy_planes(double* __restrict__ yr, double* __restrict__ yi,
                              const double* __restrict__ xr, const double* __restrict__ xi,
                              double alpha, int n, int ld, double* __restrict__ p,
                              const DevState* __restrict__ st) {
  if (st && st->stop) return;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ld * ld) return;
  const double vr = yr[idx] + alpha * xr[idx];
  yr[idx] = vr;
  yi[idx] = yi[idx] + alpha * xi[idx];
  const int a = (int)(idx / ld), b = (int)(idx % ld);
  if (p && a == b && a < n) p[a] = vr;
}

// y += alpha x with x FP32 planes (the fold of the FP32 defect)
__global__ void k_axpy_planes_f32(double* __restrict__ yr, double* __restrict__ yi,
                                  const float* __restrict__ xr, const float* __restrict__ xi,
                                  double alpha, int n, int ld, double* __restrict__ p,
                                  const DevState* __restrict__ st) {
  if (st && st->stop) return;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ld * ld) return;
  const double vr = yr[idx] + alpha * (double)xr[idx];
  yr[idx] = vr;
  yi[idx] = yi[idx] + alpha * (double)xi[idx];
  const int a = (int)(idx / ld), b = (int)(idx % ld);
  if (p && a == b && a < n) p[a] = vr;
}

// y <- y / tr, tr = st->aux[0]
__global__ void k_scale_planes(double* __restrict__ r, double* __restrict__ im,
                               double* __restrict__ p, int n, int ld,
                               const DevState* __restrict__ st) {
  if (st->stop) return;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ld * ld) return;
  const double inv = 1.0 / st->aux[0];
  const double vr = r[idx] * inv;
  r[idx] = vr;
  im[idx] = im[idx] * inv;
  const int a = (int)(idx / ld), b = (int)(idx % ld);
  if (p && a == b && a < n) p[a] = vr;
}

__global__ void k_fill16(uint4* dst, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = make_uint4(0u, 0u, 0u, 0u);
}
__global__ void k_fill1(unsigned char* dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = 0;
}

inline int blocks_for(size_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

ProbView view_of(const qpr_problem* P) {
  return ProbView{P->n,        P->ld,       P->teleport, P->alpha,
                  P->h_diag,   P->d,        P->inv_outdeg, P->dangling,
                  P->in_ptr,   P->in_idx,   P->hdiag == QPR_HDIAG_PAPER ? -1 : 1,
                  P->h_ptr,    P->h_idx,    -1};
}

FinishJob finish_job(const ProbView& pv, const EpiArgs& a, const Ws& w) {
  return FinishJob{w.partials, tri_tiles(pv.ld / TE), w.st, a.check, fehlberg_stage(a.mode), a.gate};
}

hipError_t launch_epilogue(const ProbView& pv, const EpiArgs& a, const Ws& w, hipStream_t s,
                           bool finish, const FinishJob* carry) {
  // non-temporal stage streams where the state outgrows the caches
  const bool nt = pv.ld >= 4096;
  const int grid = tri_tiles(pv.ld / TE);
  if (grid * 3 > w.max_partials) return hipErrorInvalidValue;
  if (carry && a.xkind != XS_FUSED64 && a.xkind != XS_FUSED32 && a.xkind != XS_FUSED32S)
    return hipErrorInvalidValue;
  if (a.xkind == XS_DENSE64 || a.xkind == XS_SPARSE64) {  // X written by the product
    if (nt)
      k_epilogue<XS_DENSE64, true><<<grid, ETHREADS, 0, s>>>(pv, a, w.st, w.partials);
    else
      k_epilogue<XS_DENSE64><<<grid, ETHREADS, 0, s>>>(pv, a, w.st, w.partials);
  } else if (a.xkind == XS_DENSE32) {
    if (nt)
      k_epilogue<XS_DENSE32, true><<<grid, ETHREADS, 0, s>>>(pv, a, w.st, w.partials);
    else
      k_epilogue<XS_DENSE32><<<grid, ETHREADS, 0, s>>>(pv, a, w.st, w.partials);
  }
  else if (a.xkind == XS_FUSED64 || a.xkind == XS_FUSED32 || a.xkind == XS_FUSED32S) {
    const FinishJob f = carry ? *carry : FinishJob{};
    const int g = grid + (f.nb > 0 ? 1 : 0), xcd = pv.ld < 4096 ? 1 : 0;
    if (a.xkind == XS_FUSED64 && nt)
      k_epilogue_fused<XS_FUSED64, true><<<g, ETHREADS, 0, s>>>(pv, a, w.st, w.partials, f, xcd);
    else if (a.xkind == XS_FUSED64)
      k_epilogue_fused<XS_FUSED64><<<g, ETHREADS, 0, s>>>(pv, a, w.st, w.partials, f, xcd);
    else if (a.xkind == XS_FUSED32 && nt)
      k_epilogue_fused<XS_FUSED32, true><<<g, ETHREADS, 0, s>>>(pv, a, w.st, w.partials, f, xcd);
    else if (a.xkind == XS_FUSED32)
      k_epilogue_fused<XS_FUSED32><<<g, ETHREADS, 0, s>>>(pv, a, w.st, w.partials, f, xcd);
    else if (nt)
      k_epilogue_fused<XS_FUSED32S, true><<<g, ETHREADS, 0, s>>>(pv, a, w.st, w.partials, f, xcd);
    else
      k_epilogue_fused<XS_FUSED32S><<<g, ETHREADS, 0, s>>>(pv, a, w.st, w.partials, f, xcd);
  } else {
    return hipErrorInvalidValue;
  }
  if (finish && reduces(a.mode)) k_finish<<<1, FOLD_THREADS, 0, s>>>(finish_job(pv, a, w));
  return hipGetLastError();
}

namespace {
typedef void (*SpmmFn)(ProbView, const double*, const double*, double*, double*, const DevState*,
                       int, FinishJob);
struct SpmmVariant {
  const char* name;
  SpmmFn fn;
  int cols, rpw;  // cols = 0: the legacy row-major kernel
};
const SpmmVariant kSpmm[] = {
    {"cm_w32_r1", k_spmm_cm<32, 1>, 32, 1},
    {"cm_w64_r1", k_spmm_cm<64, 1>, 64, 1},
    {"cm_w128_r1", k_spmm_cm<128, 1>, 128, 1},
    {"cm_w64_r2", k_spmm_cm<64, 2>, 64, 2},
    {"row128", k_spmm, 0, 0},
};
constexpr int kNumSpmm = (int)(sizeof(kSpmm) / sizeof(kSpmm[0]));
}  // namespace

int spmm_num_variants() { return kNumSpmm; }
const char* spmm_variant_name(int v) { return v >= 0 && v < kNumSpmm ? kSpmm[v].name : nullptr; }

// Default by size (measured, BA graphs): the row-major kernel up to N ~ 1000,
// 128-column chunks where ld is a multiple of 128 and the matrix is large.
int spmm_default_variant(const ProbView& pv) {
  int v;
  if (tuned_exact(kTuneSparseVariant, pv.ld, &v) && v >= 0 && v < kNumSpmm) return v;
  return pv.ld % 128 == 0 && pv.n >= 1536 ? 2 : 4;
}

hipError_t launch_spmm(const ProbView& pv, const double* yr, const double* yi, double* xr,
                       double* xi, const DevState* st, int gate, hipStream_t s, int variant,
                       const FinishJob* fin) {
  FinishJob f = fin ? *fin : FinishJob{};
  if (variant < 0) variant = pv.spmm_variant >= 0 ? pv.spmm_variant : spmm_default_variant(pv);
  if (variant >= kNumSpmm) return hipErrorInvalidValue;
  // ld is a multiple of 64 only: a 128-column chunk size that does not divide
  // it falls back to 64 columns (same sums, same bits)
  if (kSpmm[variant].cols == 128 && pv.ld % 128 != 0) variant = 1;  // cm_w64_r1
  const SpmmVariant& v = kSpmm[variant];
  if (v.cols != 0 && f.nb > 0) {  // chunk-major: finish in its own launch first
    k_finish<<<1, FOLD_THREADS, 0, s>>>(f);
    f = FinishJob{};
  }
  const int extra = f.nb > 0 ? 1 : 0;
  int grid;
  if (v.cols == 0) {
    grid = pv.n * ((pv.ld + SP_COLS - 1) / SP_COLS);
    v.fn<<<grid + extra, 2 * SP_COLS, 0, s>>>(pv, yr, yi, xr, xi, st, gate, f);
  } else {
    const int groups = (pv.n + SP_WAVES * v.rpw - 1) / (SP_WAVES * v.rpw);
    grid = (pv.ld / v.cols) * groups;
    v.fn<<<grid + extra, 64 * SP_WAVES, 0, s>>>(pv, yr, yi, xr, xi, st, gate, f);
  }
  return hipGetLastError();
}

hipError_t launch_spmm_f32_batch(const BatchEpi* args, const int2* items, const int* nitems,
                                 int grid, hipStream_t s) {
  k_spmm_f32_batch<<<grid, 2 * SP_COLS, 0, s>>>(args, items, nitems);
  return hipGetLastError();
}

hipError_t launch_spmm_f32(const ProbView& pv, const float* yr, const float* yi, float* xr,
                           float* xi, const DevState* st, int gate, hipStream_t s,
                           const FinishJob* fin) {
  const FinishJob f = fin ? *fin : FinishJob{};
  const int extra = f.nb > 0 ? 1 : 0;
  const int groups = (pv.n + SP_WAVES - 1) / SP_WAVES;
  if (pv.ld % 128 == 0)
    k_spmm_f32<128><<<(pv.ld / 128) * groups + extra, 64 * SP_WAVES, 0, s>>>(pv, yr, yi, xr, xi,
                                                                           st, gate, f);
  else
    k_spmm_f32<64><<<(pv.ld / 64) * groups + extra, 64 * SP_WAVES, 0, s>>>(pv, yr, yi, xr, xi,
                                                                         st, gate, f);
  return hipGetLastError();
}

int spmm_items_per_system(int n, int ld) { return n * ((ld + SP_COLS - 1) / SP_COLS); }

int epilogue_items_per_system(int ld) { return tri_tiles(ld / TE); }

hipError_t launch_spmm_batch(const BatchEpi* args, const int2* items, const int* nitems, int grid,
                             hipStream_t s) {
  k_spmm_batch<<<grid, 2 * SP_COLS, 0, s>>>(args, items, nitems);
  return hipGetLastError();
}

hipError_t launch_epilogue_batch(int xsource, const BatchEpi* args, const int2* items,
                                 const int* nitems, int grid, const int* sys_list,
                                 const int* nsys, bool finish, hipStream_t s) {
  if (xsource == XS_DENSE64)
    k_epilogue_batch<XS_DENSE64><<<grid, ETHREADS, 0, s>>>(args, items, nitems);
  else if (xsource == XS_DENSE32)
    k_epilogue_batch<XS_DENSE32><<<grid, ETHREADS, 0, s>>>(args, items, nitems);
  else if (xsource == XS_SPARSE64)
    k_epilogue_batch<XS_DENSE64><<<grid, ETHREADS, 0, s>>>(args, items, nitems);
  else if (xsource == XS_FUSED64)  // sparse gathers inside the tile kernel
    k_epilogue_batch<XS_FUSED64><<<grid, ETHREADS, 0, s>>>(args, items, nitems);
  else if (xsource == XS_FUSED32)
    k_epilogue_batch<XS_FUSED32><<<grid, ETHREADS, 0, s>>>(args, items, nitems);
  else if (xsource == XS_FUSED32S)  // the defect held in FP32
    k_epilogue_batch<XS_FUSED32S><<<grid, ETHREADS, 0, s>>>(args, items, nitems);
  else
    return hipErrorInvalidValue;
  if (finish) k_finish_batch<<<256, FOLD_THREADS, 0, s>>>(args, sys_list, nsys);
  return hipGetLastError();
}

hipError_t launch_pad_in(const double* rho, int n, int ld, double* r, double* i, double* p,
                         hipStream_t s) {
  const size_t tot = (size_t)ld * ld;
  k_pad_in<<<blocks_for(tot, 256), 256, 0, s>>>(rho, n, ld, r, i, p);
  return hipGetLastError();
}

hipError_t launch_pad_out(const double* r, const double* i, int n, int ld, double* rho,
                          hipStream_t s) {
  const size_t tot = (size_t)n * n;
  k_pad_out<<<blocks_for(tot, 256), 256, 0, s>>>(r, i, n, ld, rho);
  return hipGetLastError();
}

hipError_t launch_to_lowp(int kind, const double* r, const double* i, int n, int ld, const Ws& w,
                          hipStream_t s) {
  (void)n;
  const size_t tot = (size_t)ld * ld;
  if (kind == OP_F32)
    k_to_f32<<<blocks_for(tot, 256), 256, 0, s>>>(r, i, tot, w.lo_r, w.lo_i);
  else if (kind == OP_BF16X3)
    k_to_bf16x3<<<blocks_for(tot, 256), 256, 0, s>>>(r, i, tot, w.sl);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_state_init(DevState* st, double tol, long long max_steps, int check,
                             hipStream_t s) {
  k_state_init<<<1, 64, 0, s>>>(st, tol, max_steps, check);
  return hipGetLastError();
}

hipError_t launch_state_rkf(DevState* st, double h0, double h_max, double tol_step, hipStream_t s) {
  k_state_rkf<<<1, 64, 0, s>>>(st, h0, h_max, tol_step);
  return hipGetLastError();
}

hipError_t launch_state_stats(const double* r, const double* i, const double* p, int n, int ld,
                              const Ws& w, hipStream_t s) {
  int grid = blocks_for((size_t)n * n, 256);
  grid = grid > 1024 ? 1024 : grid;
  if (grid * 4 > w.max_partials) grid = w.max_partials / 4;
  k_state_stats<<<grid, 256, 0, s>>>(r, i, p, n, ld, w.st, w.partials);
  return hipGetLastError();
}

hipError_t launch_rank(int n, const double* p, int* order, hipStream_t s) {
  k_rank<<<blocks_for((size_t)n, 256), 256, 0, s>>>(n, p, order);
  return hipGetLastError();
}

hipError_t launch_rkf_commit(double* yr, double* yi, double* p, const double* cr,
                             const double* ci, const double* pc, int n, int ld,
                             const DevState* st, hipStream_t s) {
  k_rkf_commit<<<blocks_for((size_t)ld * ld, 256), 256, 0, s>>>(yr, yi, p, cr, ci, pc, n, ld, st);
  return hipGetLastError();
}

hipError_t launch_hubs(int n, const double* p, double c, int* out, hipStream_t s) {
  k_hubs<<<1, 1024, 0, s>>>(n, p, c, out);
  return hipGetLastError();
}

hipError_t launch_axpy_planes(double* yr, double* yi, const double* xr, const double* xi, double a,
                              int n, int ld, double* p, const DevState* st, hipStream_t s) {
  k_axpy_planes<<<blocks_for((size_t)ld * ld, 256), 256, 0, s>>>(yr, yi, xr, xi, a, n, ld, p, st);
  return hipGetLastError();
}

hipError_t launch_axpy_planes_f32(double* yr, double* yi, const float* xr, const float* xi,
                                  double a, int n, int ld, double* p, const DevState* st,
                                  hipStream_t s) {
  k_axpy_planes_f32<<<blocks_for((size_t)ld * ld, 256), 256, 0, s>>>(yr, yi, xr, xi, a, n, ld, p,
                                                                     st);
  return hipGetLastError();
}

hipError_t launch_trace(const double* p, int n, DevState* st, hipStream_t s) {
  k_trace<<<1, 1024, 0, s>>>(p, n, st);
  return hipGetLastError();
}

hipError_t launch_scale_planes(double* r, double* i, double* p, int n, int ld,
                               const DevState* st, hipStream_t s) {
  k_scale_planes<<<blocks_for((size_t)ld * ld, 256), 256, 0, s>>>(r, i, p, n, ld, st);
  return hipGetLastError();
}

hipError_t launch_fill(void* dst, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (((uintptr_t)dst % 16) == 0 && bytes % 16 == 0) {
    const size_t n16 = bytes / 16;
    int grid = blocks_for(n16, 256);
    grid = grid > 4096 ? 4096 : grid;
    k_fill16<<<grid, 256, 0, s>>>((uint4*)dst, n16);
  } else {
    int grid = blocks_for(bytes, 256);
    grid = grid > 4096 ? 4096 : grid;
    k_fill1<<<grid, 256, 0, s>>>((unsigned char*)dst, bytes);
  }
  return hipGetLastError();
}

}  // namespace qpr
