// Problem build: edge list -> Hamiltonian, Google-matrix pieces, PageRank.
//
// Supplementary Note 1 defines the adjacency (A_ij = 1 when j links to i), the
// out-degree, the hopping matrix F (Eq. (S2)), the Google matrix (Eq. (S4),
// read as the column-stochastic G = alpha S + (1 - alpha) T with dangling
// columns taken from T) and the Hamiltonian (Eq. (S6)).  G is never stored:
// the gain G p is evaluated from the in-link CSR, 1/outDeg, the dangling set
// and the two teleport sums (see gain_row in qpr_device.h).
#include <cstdio>
#include <vector>

#include "qpr_common.h"
#include "qpr_device.h"

namespace qpr {

namespace {

struct Summary {          // device -> host after the build
  long long nnz_a, nnz_h;
  int self_loops, dangling, pr_iters, pad;
  double h_lo, h_hi, h_norm;
};

struct ArenaLayout {
  size_t h64, h32, h16, a8, at8, hdiag, d, inv_out, pr, pr_tmp, dang, outdeg,
      indeg, degh, in_ptr, out_ptr, h_ptr, in_idx, out_idx, h_idx, edges, summary, total;
};

ArenaLayout arena_layout(int n, long long n_edges) {
  const size_t ld = (size_t)pad_n(n);
  const size_t e = (size_t)(n_edges > 0 ? n_edges : 1);
  ArenaLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  L.h64 = take(ld * ld * 8);
  L.h32 = take(ld * ld * 4);
  L.h16 = take(ld * ld * 2);
  L.a8 = take(ld * ld);
  L.at8 = take(ld * ld);
  L.hdiag = take(ld * 8);
  L.d = take(ld * 8);
  L.inv_out = take(ld * 8);
  L.pr = take(ld * 8);
  L.pr_tmp = take(ld * 8);
  L.dang = take(ld * 4);
  L.outdeg = take(ld * 4);
  L.indeg = take(ld * 4);
  L.degh = take(ld * 4);
  L.in_ptr = take((ld + 1) * 4);
  L.out_ptr = take((ld + 1) * 4);
  L.h_ptr = take((ld + 1) * 4);
  L.in_idx = take(e * 4);
  L.out_idx = take(e * 4);
  L.h_idx = take(2 * e * 4);
  L.edges = take(2 * e * 4);
  L.summary = take(sizeof(Summary));
  L.total = o;
  return L;
}

// Byte adjacency: A8[d][s] = 1 and AT8[s][d] = 1 for every edge s -> d, s != d.
__global__ void k_scatter(const int* __restrict__ edges, long long E, int ld,
                          unsigned char* A8, unsigned char* AT8, Summary* sm) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int s = edges[e], d = edges[E + e];
  if (s == d) {
    atomicAdd(&sm->self_loops, 1);
    return;
  }
  A8[(size_t)d * ld + s] = 1;
  AT8[(size_t)s * ld + d] = 1;
}

// One wave per row a: in/out degree, H row degree and the dense H rows in
// three precisions (padding written as zeros).
__global__ void __launch_bounds__(256) k_rows(const unsigned char* __restrict__ A8,
                                              const unsigned char* __restrict__ AT8,
                                              int n, int ld, int hsign, double* h64,
                                              float* h32, uint16_t* h16, int* indeg,
                                              int* outdeg, int* degh) {
  const int lane = threadIdx.x & 63;
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a >= ld) return;
  int cin = 0, cout = 0, ch = 0;
  const unsigned short one16 = hsign > 0 ? 0x3F80 : 0xBF80;  // bf16 +-1
  for (int b = lane; b < ld; b += 64) {
    int x = 0, y = 0;
    if (a < n && b < n) {
      x = A8[(size_t)a * ld + b];
      y = AT8[(size_t)a * ld + b];
    }
    const int h = (a != b) && (x | y);
    cin += x;
    cout += y;
    ch += h;
    const size_t o = (size_t)a * ld + b;
    h64[o] = h ? (double)hsign : 0.0;
    h32[o] = h ? (float)hsign : 0.0f;
    h16[o] = h ? one16 : (unsigned short)0;
  }
  cin = wave_sum_i(cin);
  cout = wave_sum_i(cout);
  ch = wave_sum_i(ch);
  if (lane == 0 && a < n) {
    indeg[a] = cin;
    outdeg[a] = cout;
    degh[a] = ch;
  }
}

// Exclusive scans of indeg and outdeg (one workgroup), totals into the summary.
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ indeg,
                                               const int* __restrict__ outdeg,
                                               const int* __restrict__ degh, int n,
                                               int* in_ptr, int* out_ptr, int* h_ptr,
                                               Summary* sm) {
  __shared__ long long buf[1024];
  const int t = threadIdx.x;
  for (int which = 0; which < 3; ++which) {
    const int* deg = which == 0 ? indeg : which == 1 ? outdeg : degh;
    int* ptr = which == 0 ? in_ptr : which == 1 ? out_ptr : h_ptr;
    long long carry = 0;
    for (int base = 0; base < n; base += 1024) {
      const int i = base + t;
      long long v = i < n ? deg[i] : 0;
      buf[t] = v;
      __syncthreads();
      for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
        long long add = t >= off ? buf[t - off] : 0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
      }
      if (i < n) ptr[i] = (int)(carry + buf[t] - v);
      const long long tot = buf[1023];
      __syncthreads();
      carry += tot;
    }
    if (t == 0) {
      ptr[n] = (int)carry;
      if (which == 0) sm->nnz_a = carry;
    }
    __syncthreads();
  }
  // nnz of H
  long long hsum = 0;
  for (int i = t; i < n; i += 1024) hsum += degh[i];
  buf[t] = hsum;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) buf[t] += buf[t + off];
    __syncthreads();
  }
  if (t == 0) sm->nnz_h = buf[0];
}

// One wave per row: ascending CSR fill of in-links (row a of A8), out-links
// (row a of AT8) and the off-diagonal Hamiltonian pattern (A8 | AT8 without
// the diagonal) by ballot compaction.
__global__ void __launch_bounds__(256) k_fill_csr(const unsigned char* __restrict__ A8,
                                                  const unsigned char* __restrict__ AT8,
                                                  int n, int ld, const int* __restrict__ in_ptr,
                                                  const int* __restrict__ out_ptr,
                                                  const int* __restrict__ h_ptr, int* in_idx,
                                                  int* out_idx, int* h_idx) {
  const int lane = threadIdx.x & 63;
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a >= n) return;
  for (int which = 0; which < 3; ++which) {
    int* idx = which == 0 ? in_idx : which == 1 ? out_idx : h_idx;
    int pos = which == 0 ? in_ptr[a] : which == 1 ? out_ptr[a] : h_ptr[a];
    for (int b0 = 0; b0 < n; b0 += 64) {
      const int b = b0 + lane;
      int x = 0;
      if (b < n) {
        const int u = A8[(size_t)a * ld + b], v = AT8[(size_t)a * ld + b];
        x = which == 0 ? u : which == 1 ? v : ((u | v) && b != a);
      }
      const unsigned long long mask = __ballot(x);
      const unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
      if (x) idx[pos + __popcll(below)] = b;
      pos += __popcll(mask);
    }
  }
}

// Per-node vectors: 1/outDeg, dangling flag, column sums d of G, diag of H,
// and the Gershgorin interval of H.
__global__ void __launch_bounds__(1024) k_vectors(const int* __restrict__ outdeg,
                                                  const int* __restrict__ degh, int n,
                                                  double alpha, int teleport, int hdiag,
                                                  double* inv_out, int* dang, double* d,
                                                  double* hdiag_out, Summary* sm) {
  __shared__ double lo_s[1024], hi_s[1024];
  __shared__ int dn_s[1024];
  const int t = threadIdx.x;
  double lo = 1e300, hi = -1e300;
  int dn = 0;
  const double tcol = teleport == QPR_TELEPORT_PAPER_F ? (double)(n - 1) * (1.0 / (double)(n - 1))
                                                       : (double)n * (1.0 / (double)n);
  for (int j = t; j < n; j += 1024) {
    const int od = outdeg[j];
    const int isd = od == 0;
    inv_out[j] = isd ? 0.0 : 1.0 / (double)od;
    dang[j] = isd;
    dn += isd;
    const double scol = isd ? tcol : (double)od * (1.0 / (double)od);
    d[j] = alpha * scol + (1.0 - alpha) * tcol;
    const double hd = hdiag == QPR_HDIAG_PAPER ? -(double)od : 0.0;
    hdiag_out[j] = hd;
    lo = fmin(lo, hd - (double)degh[j]);
    hi = fmax(hi, hd + (double)degh[j]);
  }
  lo_s[t] = lo;
  hi_s[t] = hi;
  dn_s[t] = dn;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) {
      lo_s[t] = fmin(lo_s[t], lo_s[t + off]);
      hi_s[t] = fmax(hi_s[t], hi_s[t + off]);
      dn_s[t] += dn_s[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    sm->h_lo = lo_s[0];
    sm->h_hi = hi_s[0];
    sm->dangling = dn_s[0];
  }
}

// PageRank by power iteration p <- G p / sum, from the uniform vector, until
// ||p_new - p||_1 < 1e-15 or max_it iterations (one workgroup).
__global__ void __launch_bounds__(1024) k_pagerank(GainView gv, double* p, double* q,
                                                   int max_it, Summary* sm) {
  __shared__ double red[1024];
  __shared__ double sums[2];
  const int t = threadIdx.x;
  const int n = gv.n;
  for (int i = t; i < n; i += 1024) p[i] = 1.0 / (double)n;
  __syncthreads();
  int it = 0;
  for (; it < max_it; ++it) {
    // teleport sums P = sum p, D = sum over dangling p
    double a = 0.0, b = 0.0;
    for (int i = t; i < n; i += 1024) {
      a += p[i];
      b += gv.dangling[i] ? p[i] : 0.0;
    }
    double P = block_sum_1024(a, red);
    double D = block_sum_1024(b, red);
    double s = 0.0;
    for (int i = t; i < n; i += 1024) {
      const double g = gain_row(gv, i, p, P, D);
      q[i] = g;
      s += g;
    }
    const double S = block_sum_1024(s, red);
    double diff = 0.0;
    for (int i = t; i < n; i += 1024) {
      const double v = q[i] / S;
      diff += fabs(v - p[i]);
      q[i] = v;
    }
    const double Dl = block_sum_1024(diff, red);
    for (int i = t; i < n; i += 1024) p[i] = q[i];
    __syncthreads();
    if (Dl < 1e-15) {
      ++it;
      break;
    }
  }
  if (t == 0) sm->pr_iters = it;
  (void)sums;
}

// Spectral radius estimate of H = diag(h) + H_off by power iteration (one
// workgroup, fixed start vector, `iters` products through the CSR of H_off).
// The Rayleigh quotients increase towards the spectral radius; the largest
// one seen is kept.
__global__ void __launch_bounds__(1024) k_spectral(int n, const int* __restrict__ h_ptr,
                                                   const int* __restrict__ h_idx, int hsign,
                                                   const double* __restrict__ hd, double* x,
                                                   double* y, int iters, Summary* sm) {
  __shared__ double red[1024];
  const int t = threadIdx.x;
  double nrm2 = 0.0;
  for (int i = t; i < n; i += 1024) {
    const double v = 1.0 + 0.5 * sin(0.7 * (double)i);
    x[i] = v;
    nrm2 += v * v;
  }
  nrm2 = block_sum_1024(nrm2, red);
  double best = 0.0;
  for (int it = 0; it < iters; ++it) {
    const double inv = 1.0 / sqrt(nrm2);
    double dot = 0.0, yy = 0.0;
    for (int i = t; i < n; i += 1024) {
      double acc = hd[i] * x[i];
      for (int e = h_ptr[i]; e < h_ptr[i + 1]; ++e) acc += (double)hsign * x[h_idx[e]];
      acc *= inv;
      y[i] = acc;
      dot += acc * x[i] * inv;
      yy += acc * acc;
    }
    dot = block_sum_1024(dot, red);   // Rayleigh quotient of x / |x|
    yy = block_sum_1024(yy, red);
    best = fmax(best, fabs(dot));
    for (int i = t; i < n; i += 1024) x[i] = y[i];
    __syncthreads();
    nrm2 = yy;
    if (!(nrm2 > 0.0)) break;
  }
  if (t == 0) sm->h_norm = best;
  // Rigorous upper bound on the spectral radius (Collatz-Wielandt): for any
  // positive u, rho(H) <= rho(|H|) <= max_i (|H| u)_i / u_i.  With u the
  // magnitude of the last iterate (near the Perron vector of |H| on the
  // dominant component), lifted by 1e-3 of its maximum so that it is positive
  // everywhere, the bound is close to rho(H).  The Gershgorin interval of the
  // spectrum (2 x the largest degree wide, loose on graphs with hubs) is
  // intersected with [-bound, bound]; the RK4 stability check uses it.
  double xm = 0.0;
  for (int i = t; i < n; i += 1024) xm = fmax(xm, fabs(x[i]));
  xm = block_max(xm, red, 1024 / 64);
  if (xm > 0.0 && isfinite(xm)) {
    const double lift = 1e-3 * xm;
    double bnd = 0.0;
    for (int i = t; i < n; i += 1024) {
      const double ui = fabs(x[i]) + lift;
      double z = fabs(hd[i]) * ui;
      for (int e = h_ptr[i]; e < h_ptr[i + 1]; ++e) z += fabs(x[h_idx[e]]) + lift;
      bnd = fmax(bnd, z / ui);
    }
    bnd = block_max(bnd, red, 1024 / 64);
    if (t == 0 && isfinite(bnd)) {
      sm->h_lo = fmax(sm->h_lo, -bnd);
      sm->h_hi = fmin(sm->h_hi, bnd);
    }
  }
}

}  // namespace

}  // namespace qpr

using namespace qpr;

extern "C" size_t qpr_problem_bytes(int32_t n, int64_t n_edges) {
  if (n < 2 || n_edges < 0) return 0;
  return arena_layout(n, n_edges).total;
}

extern "C" qpr_status qpr_build_google(int32_t n, int64_t n_edges, const int32_t* src,
                                       const int32_t* dst, double alpha, int32_t teleport,
                                       int32_t hdiag, void* arena, size_t arena_bytes,
                                       qpr_problem* out, qpr_stream_t stream) {
  clear_error();
  if (n < 2) return fail(QPR_E_ARG, "n must be >= 2 (got %d)", n);
  if (n > 65536) return fail(QPR_E_ARG, "n must be <= 65536 (got %d)", n);
  if (n_edges < 0 || n_edges > (int64_t)1 << 31)
    return fail(QPR_E_ARG, "n_edges out of range (%lld)", (long long)n_edges);
  if (n_edges > 0 && (!src || !dst)) return fail(QPR_E_ARG, "src/dst must not be NULL");
  if (!arena || !out) return fail(QPR_E_ARG, "arena and out must not be NULL");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(QPR_E_ARG, "alpha must be in [0,1] (got %g)", alpha);
  if (teleport != QPR_TELEPORT_PAPER_F && teleport != QPR_TELEPORT_UNIFORM)
    return fail(QPR_E_ARG, "unknown teleport %d", teleport);
  if (hdiag != QPR_HDIAG_ZERO && hdiag != QPR_HDIAG_PAPER)
    return fail(QPR_E_ARG, "unknown hdiag %d", hdiag);
  if (((uintptr_t)arena) % kAlign) return fail(QPR_E_ARG, "arena must be 256-byte aligned");
  for (int64_t e = 0; e < n_edges; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n)
      return fail(QPR_E_ARG, "edge %lld (%d -> %d) out of range for n=%d", (long long)e,
                  src[e], dst[e], n);
  const ArenaLayout L = arena_layout(n, n_edges);
  if (arena_bytes < L.total)
    return fail(QPR_E_WORKSPACE, "arena has %zu bytes, needs %zu", arena_bytes, L.total);

  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)arena;
  const int ld = pad_n(n);
  qpr_problem P{};
  P.n = n;
  P.ld = ld;
  P.n_edges_in = n_edges;
  P.alpha = alpha;
  P.teleport = teleport;
  P.hdiag = hdiag;
  P.h_off = (double*)(base + L.h64);
  P.h_off_f32 = (float*)(base + L.h32);
  P.h_off_bf16 = (uint16_t*)(base + L.h16);
  P.h_diag = (double*)(base + L.hdiag);
  P.d = (double*)(base + L.d);
  P.inv_outdeg = (double*)(base + L.inv_out);
  P.dangling = (int32_t*)(base + L.dang);
  P.outdeg = (int32_t*)(base + L.outdeg);
  P.indeg = (int32_t*)(base + L.indeg);
  P.in_ptr = (int32_t*)(base + L.in_ptr);
  P.out_ptr = (int32_t*)(base + L.out_ptr);
  P.in_idx = (int32_t*)(base + L.in_idx);
  P.out_idx = (int32_t*)(base + L.out_idx);
  P.h_ptr = (int32_t*)(base + L.h_ptr);
  P.h_idx = (int32_t*)(base + L.h_idx);
  P.pagerank = (double*)(base + L.pr);
  P.arena = arena;
  P.arena_bytes = arena_bytes;
  unsigned char* A8 = (unsigned char*)(base + L.a8);
  unsigned char* AT8 = (unsigned char*)(base + L.at8);
  int* edges = (int*)(base + L.edges);
  int* degh = (int*)(base + L.degh);
  Summary* sm = (Summary*)(base + L.summary);

  // Clear everything the scatter and the counters rely on (fill kernel, no memset).
  QPR_HIP(launch_fill(base + L.a8, L.hdiag - L.a8, s));
  QPR_HIP(launch_fill(sm, sizeof(Summary), s));
  if (n_edges > 0) {
    QPR_HIP(hipMemcpyAsync(edges, src, (size_t)n_edges * 4, hipMemcpyHostToDevice, s));
    QPR_HIP(hipMemcpyAsync(edges + n_edges, dst, (size_t)n_edges * 4, hipMemcpyHostToDevice, s));
    const int blocks = (int)((n_edges + 255) / 256);
    k_scatter<<<blocks, 256, 0, s>>>(edges, n_edges, ld, A8, AT8, sm);
    QPR_HIP(hipGetLastError());
  }
  const int hsign = hdiag == QPR_HDIAG_PAPER ? -1 : 1;
  k_rows<<<(ld + 3) / 4, 256, 0, s>>>(A8, AT8, n, ld, hsign, P.h_off, P.h_off_f32,
                                      P.h_off_bf16, P.indeg, P.outdeg, degh);
  QPR_HIP(hipGetLastError());
  k_scan<<<1, 1024, 0, s>>>(P.indeg, P.outdeg, degh, n, P.in_ptr, P.out_ptr, P.h_ptr, sm);
  QPR_HIP(hipGetLastError());
  k_fill_csr<<<(n + 3) / 4, 256, 0, s>>>(A8, AT8, n, ld, P.in_ptr, P.out_ptr, P.h_ptr,
                                         P.in_idx, P.out_idx, P.h_idx);
  QPR_HIP(hipGetLastError());
  k_vectors<<<1, 1024, 0, s>>>(P.outdeg, degh, n, alpha, teleport, hdiag, P.inv_outdeg,
                               P.dangling, P.d, P.h_diag, sm);
  QPR_HIP(hipGetLastError());
  GainView gv{n, teleport, alpha, P.inv_outdeg, P.dangling, P.in_ptr, P.in_idx};
  k_pagerank<<<1, 1024, 0, s>>>(gv, P.pagerank, (double*)(base + L.pr_tmp), 4000, sm);
  QPR_HIP(hipGetLastError());
  // scratch for the power iteration: the FP64 H plane is not touched, the
  // byte adjacency (no longer needed) is reused
  k_spectral<<<1, 1024, 0, s>>>(n, P.h_ptr, P.h_idx, hsign, P.h_diag, (double*)A8,
                                (double*)A8 + ld, 300, sm);
  QPR_HIP(hipGetLastError());
  Summary h{};
  QPR_HIP(hipMemcpyAsync(&h, sm, sizeof(Summary), hipMemcpyDeviceToHost, s));
  QPR_HIP(hipStreamSynchronize(s));
  P.nnz_a = h.nnz_a;
  P.nnz_h = h.nnz_h;
  P.n_self_loops = h.self_loops;
  P.n_dangling = h.dangling;
  P.h_lo = h.h_lo;
  P.h_hi = h.h_hi;
  P.h_norm = h.h_norm;
  P.pagerank_iters = h.pr_iters;
  *out = P;
  return QPR_OK;
}
