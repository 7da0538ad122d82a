// Warm-start message-passing network: forward, backward and Adam (FP32).
//
// The network predicts the steady-state populations diag(rho_ss) so the RK4
// integrator starts near its fixed point (it is always finished and judged by
// the plain FP64 solver).  Definition, per node i of a graph:
//   x_i   = [log(1+in_i), log(1+out_i), N * PR_i, omega]
//   h'_i  = ReLU(Ws h_i + Win mean_{j->i} h_j + Wout mean_{i->j} h_j + b), 3 layers, width 64
//   s_i   = w . h_i + c,   p_hat = softmax of s within each graph
//   loss  = mean over graphs of KL(p || p_hat)
// Graphs are batched block-diagonally; node ids are global.  Every reduction
// (softmax, loss, weight gradients) is a fixed-order two-level sum, and the
// transposed aggregations of the backward pass gather through the reverse
// CSR, so results are deterministic and no floating-point atomics are used.
#include <cmath>

#include "qpr_common.h"
#include "qpr_device.h"

namespace qpr {
namespace {

constexpr int HID = 64;
constexpr int FEAT = 4;
constexpr int LAYERS = 3;
constexpr int CHUNK = 64;  // nodes per partial-gradient block

__host__ __device__ constexpr int layer_in(int l) { return l == 0 ? FEAT : HID; }
// flat parameter offsets: [Ws_l | Win_l | Wout_l | b_l] for l = 0..2, then w, c
__host__ __device__ constexpr int layer_off(int l) {
  return l == 0 ? 0 : layer_off(l - 1) + 3 * HID * layer_in(l - 1) + HID;
}
constexpr int kReadoutOff = layer_off(LAYERS);
constexpr int kParams = kReadoutOff + HID + 1;

struct Acts {  // activations of one forward pass (node-major rows)
  float* H[LAYERS + 1];   // H[0] = features (n x 4), H[l] (n x 64)
  float* Ain[LAYERS];     // (n x F_l)
  float* Aout[LAYERS];
  float* Z[LAYERS];       // pre-activations (n x 64)
  float* s;               // scores (n)
  float* p_hat;           // (n)
  float* dH;              // (n x 64)
  float* dZ;              // (n x 64)
  float* Uin;             // (n x 64)
  float* Uout;            // (n x 64)
  float* V;               // (n x 64)
  float* partials;        // (n/CHUNK + 1) x kParams
  float* gloss;           // n_graphs
};

size_t acts_bytes(int n, int g, Acts* a, char* base) {
  size_t o = 0;
  auto take = [&](size_t count) {
    size_t r = o;
    o = align_up(o + count * 4);
    return base ? (float*)(base + r) : nullptr;
  };
  Acts t{};
  t.H[0] = take((size_t)n * FEAT);
  for (int l = 0; l < LAYERS; ++l) {
    t.Ain[l] = take((size_t)n * layer_in(l));
    t.Aout[l] = take((size_t)n * layer_in(l));
    t.Z[l] = take((size_t)n * HID);
    t.H[l + 1] = take((size_t)n * HID);
  }
  t.s = take(n);
  t.p_hat = take(n);
  t.dH = take((size_t)n * HID);
  t.dZ = take((size_t)n * HID);
  t.Uin = take((size_t)n * HID);
  t.Uout = take((size_t)n * HID);
  t.V = take((size_t)n * HID);
  t.partials = take((size_t)(n / CHUNK + 1) * kParams);
  t.gloss = take(g > 0 ? g : 1);
  if (a) *a = t;
  return o;
}

// ------------------------------------------------------------------ forward
// mean aggregation over in- and out-neighbours, thread per (node, feature)
__global__ void k_agg(int n, int F, const float* __restrict__ H, const int* __restrict__ in_ptr,
                      const int* __restrict__ in_idx, const float* __restrict__ inv_in,
                      const int* __restrict__ out_ptr, const int* __restrict__ out_idx,
                      const float* __restrict__ inv_out, float* __restrict__ Ain,
                      float* __restrict__ Aout) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * F) return;
  const int i = (int)(t / F), f = (int)(t % F);
  float si = 0.f, so = 0.f;
  for (int e = in_ptr[i]; e < in_ptr[i + 1]; ++e) si += H[(size_t)in_idx[e] * F + f];
  for (int e = out_ptr[i]; e < out_ptr[i + 1]; ++e) so += H[(size_t)out_idx[e] * F + f];
  Ain[t] = si * inv_in[i];
  Aout[t] = so * inv_out[i];
}

// Z = Ws h + Win a_in + Wout a_out + b ; H' = ReLU(Z); thread per (node, output)
__global__ void __launch_bounds__(256) k_dense(int n, int F, const float* __restrict__ W,
                                               const float* __restrict__ H,
                                               const float* __restrict__ Ain,
                                               const float* __restrict__ Aout,
                                               float* __restrict__ Z, float* __restrict__ Hn) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * HID) return;
  const int i = (int)(t / HID), o = (int)(t % HID);
  const float* Ws = W;
  const float* Wi = W + HID * F;
  const float* Wo = W + 2 * HID * F;
  const float* b = W + 3 * HID * F;
  float z = b[o];
  for (int k = 0; k < F; ++k) {
    const size_t x = (size_t)i * F + k;
    z += Ws[o * F + k] * H[x] + Wi[o * F + k] * Ain[x] + Wo[o * F + k] * Aout[x];
  }
  Z[t] = z;
  Hn[t] = z > 0.f ? z : 0.f;
}

// per-graph readout and softmax (one workgroup per graph)
__global__ void __launch_bounds__(256) k_readout(const int* __restrict__ gptr,
                                                 const float* __restrict__ H,
                                                 const float* __restrict__ Wr,
                                                 float* __restrict__ s, float* __restrict__ p) {
  __shared__ float red[256];
  const int g = blockIdx.x, t = threadIdx.x;
  const int i0 = gptr[g], i1 = gptr[g + 1];
  float mx = -INFINITY;
  for (int i = i0 + t; i < i1; i += 256) {
    float v = Wr[HID];
    for (int k = 0; k < HID; ++k) v += Wr[k] * H[(size_t)i * HID + k];
    s[i] = v;
    mx = fmaxf(mx, v);
  }
  red[t] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] = fmaxf(red[t], red[t + off]);
    __syncthreads();
  }
  mx = red[0];
  __syncthreads();
  float sum = 0.f;
  for (int i = i0 + t; i < i1; i += 256) sum += expf(s[i] - mx);
  red[t] = sum;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  sum = red[0];
  for (int i = i0 + t; i < i1; i += 256) p[i] = expf(s[i] - mx) / sum;
}

// ----------------------------------------------------------------- backward
// KL per graph and ds = (p_hat - p) / B (one workgroup per graph)
__global__ void __launch_bounds__(256) k_loss(const int* __restrict__ gptr, int B,
                                              const float* __restrict__ p_hat,
                                              const float* __restrict__ p_true,
                                              float* __restrict__ ds, float* __restrict__ gloss) {
  __shared__ float red[256];
  const int g = blockIdx.x, t = threadIdx.x;
  float kl = 0.f;
  for (int i = gptr[g] + t; i < gptr[g + 1]; i += 256) {
    const float pt = p_true[i], ph = p_hat[i];
    if (pt > 0.f) kl += pt * (logf(pt) - logf(ph));
    ds[i] = (ph - pt) / (float)B;
  }
  red[t] = kl;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0) gloss[g] = red[0] / (float)B;
}

__global__ void k_sum_loss(const float* __restrict__ gloss, int B, float* __restrict__ out) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  float s = 0.f;
  for (int g = t; g < B; g += 256) s += gloss[g];
  red[t] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0) out[0] = red[0];
}

// dH3 = ds (x) w
__global__ void k_readout_back(int n, const float* __restrict__ ds, const float* __restrict__ Wr,
                               float* __restrict__ dH) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * HID) return;
  dH[t] = ds[t / HID] * Wr[t % HID];
}

// Partial parameter gradients of one layer over a chunk of CHUNK nodes.
// dZ = dH * (Z > 0) is formed on the fly; the readout gradient (w, c) is
// taken in the same pass when layer == LAYERS-1.  Partials are written per
// chunk (block) for a fixed-order final sum.
__global__ void __launch_bounds__(256) k_layer_grad(int n, int layer, int F,
                                                    const float* __restrict__ dH,
                                                    const float* __restrict__ Z,
                                                    const float* __restrict__ H,
                                                    const float* __restrict__ Ain,
                                                    const float* __restrict__ Aout,
                                                    const float* __restrict__ ds,
                                                    const float* __restrict__ Hlast,
                                                    float* __restrict__ dZout,
                                                    float* __restrict__ partials) {
  __shared__ float sdz[CHUNK][HID + 1];
  __shared__ float sx[3][CHUNK][HID + 1];
  const int c = blockIdx.x, t = threadIdx.x;
  const int i0 = c * CHUNK;
  const int cnt = min(CHUNK, n - i0);
  for (int e = t; e < CHUNK * HID; e += 256) {
    const int r = e / HID, o = e % HID;
    float v = 0.f;
    if (r < cnt) {
      const size_t x = (size_t)(i0 + r) * HID + o;
      v = Z[x] > 0.f ? dH[x] : 0.f;
      dZout[x] = v;
    }
    sdz[r][o] = v;
  }
  for (int e = t; e < CHUNK * F; e += 256) {
    const int r = e / F, k = e % F;
    float a = 0.f, b = 0.f, d = 0.f;
    if (r < cnt) {
      const size_t x = (size_t)(i0 + r) * F + k;
      a = H[x];
      b = Ain[x];
      d = Aout[x];
    }
    sx[0][r][k] = a;
    sx[1][r][k] = b;
    sx[2][r][k] = d;
  }
  __syncthreads();
  float* out = partials + (size_t)c * kParams + layer_off(layer);
  // W blocks: [Ws | Win | Wout] each HID x F, then b (HID)
  for (int e = t; e < 3 * HID * F + HID; e += 256) {
    float acc = 0.f;
    if (e < 3 * HID * F) {
      const int m = e / (HID * F), rem = e % (HID * F), o = rem / F, k = rem % F;
      for (int r = 0; r < CHUNK; ++r) acc += sdz[r][o] * sx[m][r][k];
    } else {
      const int o = e - 3 * HID * F;
      for (int r = 0; r < CHUNK; ++r) acc += sdz[r][o];
    }
    out[e] = acc;
  }
  if (layer == LAYERS - 1) {
    float* ro = partials + (size_t)c * kParams + kReadoutOff;
    for (int k = t; k < HID + 1; k += 256) {
      float acc = 0.f;
      for (int r = 0; r < cnt; ++r) {
        const float d = ds[i0 + r];
        acc += k < HID ? d * Hlast[(size_t)(i0 + r) * HID + k] : d;
      }
      ro[k] = acc;
    }
  }
}

// V = Ws^T dZ, Uin = Win^T dZ, Uout = Wout^T dZ (rows of width F)
__global__ void k_back_mix(int n, int F, const float* __restrict__ W, const float* __restrict__ dZ,
                           float* __restrict__ V, float* __restrict__ Uin,
                           float* __restrict__ Uout) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * F) return;
  const int i = (int)(t / F), k = (int)(t % F);
  const float* Ws = W;
  const float* Wi = W + HID * F;
  const float* Wo = W + 2 * HID * F;
  float v = 0.f, a = 0.f, b = 0.f;
  for (int o = 0; o < HID; ++o) {
    const float d = dZ[(size_t)i * HID + o];
    v += Ws[o * F + k] * d;
    a += Wi[o * F + k] * d;
    b += Wo[o * F + k] * d;
  }
  V[t] = v;
  Uin[t] = a;
  Uout[t] = b;
}

// dH_prev_j = V_j + sum_{i: j->i} Uin_i / in_i + sum_{i: i->j} Uout_i / out_i
// (M_in^T gathers over out-links of j, M_out^T over its in-links)
__global__ void k_back_gather(int n, int F, const float* __restrict__ V,
                              const float* __restrict__ Uin, const float* __restrict__ Uout,
                              const int* __restrict__ in_ptr, const int* __restrict__ in_idx,
                              const float* __restrict__ inv_in, const int* __restrict__ out_ptr,
                              const int* __restrict__ out_idx, const float* __restrict__ inv_out,
                              float* __restrict__ dH) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * F) return;
  const int j = (int)(t / F), k = (int)(t % F);
  float acc = V[t];
  for (int e = out_ptr[j]; e < out_ptr[j + 1]; ++e) {
    const int i = out_idx[e];
    acc += Uin[(size_t)i * F + k] * inv_in[i];
  }
  for (int e = in_ptr[j]; e < in_ptr[j + 1]; ++e) {
    const int i = in_idx[e];
    acc += Uout[(size_t)i * F + k] * inv_out[i];
  }
  dH[t] = acc;
}

// grads[p] = sum over chunks of partials[c][p] (fixed order); entries a layer
// does not own are zero in every partial row of that chunk and are summed too
__global__ void k_reduce_partials(int nchunks, const float* __restrict__ partials,
                                  float* __restrict__ grads) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  float acc = 0.f;
  for (int c = 0; c < nchunks; ++c) acc += partials[(size_t)c * kParams + p];
  grads[p] = acc;
}

__global__ void k_adam(float* __restrict__ prm, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int count, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  prm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// features of one built problem: [log1p(in), log1p(out), N * PR, omega], 1/in, 1/out
__global__ void k_features(int n, const int* __restrict__ indeg, const int* __restrict__ outdeg,
                           const double* __restrict__ pr, double omega, float* __restrict__ x,
                           float* __restrict__ inv_in, float* __restrict__ inv_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = indeg[i], b = outdeg[i];
  x[4 * i + 0] = (float)log1p((double)a);
  x[4 * i + 1] = (float)log1p((double)b);
  x[4 * i + 2] = (float)((double)n * pr[i]);
  x[4 * i + 3] = (float)omega;
  inv_in[i] = a > 0 ? 1.f / (float)a : 0.f;
  inv_out[i] = b > 0 ? 1.f / (float)b : 0.f;
}

inline int nblk(long long n, int t) { return (int)((n + t - 1) / t); }

qpr_status check_batch(const qpr_mpnn_batch* b) {
  if (!b) return fail(QPR_E_ARG, "batch must not be NULL");
  if (b->n_nodes < 1 || b->n_graphs < 1) return fail(QPR_E_ARG, "empty batch");
  if (!b->x || !b->in_ptr || !b->out_ptr || !b->inv_in || !b->inv_out || !b->graph_ptr)
    return fail(QPR_E_ARG, "batch pointers must not be NULL");
  return QPR_OK;
}

}  // namespace
}  // namespace qpr

using namespace qpr;

extern "C" int32_t qpr_mpnn_param_count(void) { return kParams; }

extern "C" size_t qpr_mpnn_workspace_bytes(int32_t n_nodes, int32_t n_graphs) {
  if (n_nodes < 1 || n_graphs < 1) return 0;
  return acts_bytes(n_nodes, n_graphs, nullptr, nullptr);
}

extern "C" qpr_status qpr_mpnn_features(const qpr_problem* P, double omega, float* x,
                                        float* inv_in, float* inv_out, qpr_stream_t stream) {
  clear_error();
  if (!P || !P->indeg || !P->outdeg || !P->pagerank) return fail(QPR_E_ARG, "bad problem");
  if (!x || !inv_in || !inv_out) return fail(QPR_E_ARG, "outputs must not be NULL");
  k_features<<<nblk(P->n, 256), 256, 0, (hipStream_t)stream>>>(P->n, P->indeg, P->outdeg,
                                                               P->pagerank, omega, x, inv_in,
                                                               inv_out);
  QPR_HIP(hipGetLastError());
  return QPR_OK;
}

extern "C" qpr_status qpr_mpnn_forward(const qpr_mpnn_batch* b, const float* params,
                                       float* p_hat, void* ws, size_t ws_bytes,
                                       qpr_stream_t stream) {
  clear_error();
  qpr_status st = check_batch(b);
  if (st != QPR_OK) return st;
  if (!params || !ws) return fail(QPR_E_ARG, "params and ws must not be NULL");
  const int n = b->n_nodes;
  if (ws_bytes < acts_bytes(n, b->n_graphs, nullptr, nullptr))
    return fail(QPR_E_WORKSPACE, "mpnn workspace too small");
  Acts A;
  acts_bytes(n, b->n_graphs, &A, (char*)ws);
  hipStream_t s = (hipStream_t)stream;
  QPR_HIP(hipMemcpyAsync(A.H[0], b->x, (size_t)n * FEAT * 4, hipMemcpyDeviceToDevice, s));
  for (int l = 0; l < LAYERS; ++l) {
    const int F = layer_in(l);
    k_agg<<<nblk((long long)n * F, 256), 256, 0, s>>>(n, F, A.H[l], b->in_ptr, b->in_idx,
                                                      b->inv_in, b->out_ptr, b->out_idx,
                                                      b->inv_out, A.Ain[l], A.Aout[l]);
    k_dense<<<nblk((long long)n * HID, 256), 256, 0, s>>>(n, F, params + layer_off(l), A.H[l],
                                                          A.Ain[l], A.Aout[l], A.Z[l],
                                                          A.H[l + 1]);
  }
  k_readout<<<b->n_graphs, 256, 0, s>>>(b->graph_ptr, A.H[LAYERS], params + kReadoutOff, A.s,
                                        A.p_hat);
  QPR_HIP(hipGetLastError());
  if (p_hat) QPR_HIP(hipMemcpyAsync(p_hat, A.p_hat, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
  return QPR_OK;
}

extern "C" qpr_status qpr_mpnn_backward(const qpr_mpnn_batch* b, const float* params,
                                        const float* p_true, float* grads, float* loss,
                                        void* ws, size_t ws_bytes, qpr_stream_t stream) {
  clear_error();
  qpr_status st = check_batch(b);
  if (st != QPR_OK) return st;
  if (!params || !p_true || !grads || !ws) return fail(QPR_E_ARG, "NULL argument");
  const int n = b->n_nodes, B = b->n_graphs;
  if (ws_bytes < acts_bytes(n, B, nullptr, nullptr))
    return fail(QPR_E_WORKSPACE, "mpnn workspace too small");
  Acts A;
  acts_bytes(n, B, &A, (char*)ws);
  hipStream_t s = (hipStream_t)stream;
  const int nchunks = (n + CHUNK - 1) / CHUNK;
  float* ds = A.s;  // scores are not needed after the forward pass
  k_loss<<<B, 256, 0, s>>>(b->graph_ptr, B, A.p_hat, p_true, ds, A.gloss);
  if (loss) k_sum_loss<<<1, 256, 0, s>>>(A.gloss, B, loss);
  k_readout_back<<<nblk((long long)n * HID, 256), 256, 0, s>>>(n, ds, params + kReadoutOff, A.dH);
  QPR_HIP(launch_fill(A.partials, (size_t)nchunks * kParams * 4, s));
  for (int l = LAYERS - 1; l >= 0; --l) {
    const int F = layer_in(l);
    k_layer_grad<<<nchunks, 256, 0, s>>>(n, l, F, A.dH, A.Z[l], A.H[l], A.Ain[l], A.Aout[l], ds,
                                         A.H[LAYERS], A.dZ, A.partials);
    if (l > 0) {
      k_back_mix<<<nblk((long long)n * F, 256), 256, 0, s>>>(n, F, params + layer_off(l), A.dZ,
                                                            A.V, A.Uin, A.Uout);
      k_back_gather<<<nblk((long long)n * F, 256), 256, 0, s>>>(
          n, F, A.V, A.Uin, A.Uout, b->in_ptr, b->in_idx, b->inv_in, b->out_ptr, b->out_idx,
          b->inv_out, A.dH);
    }
  }
  k_reduce_partials<<<nblk(kParams, 256), 256, 0, s>>>(nchunks, A.partials, grads);
  QPR_HIP(hipGetLastError());
  return QPR_OK;
}

extern "C" qpr_status qpr_mpnn_adam(float* params, const float* grads, float* m, float* v,
                                    int32_t count, int32_t step, float lr, float b1, float b2,
                                    float eps, qpr_stream_t stream) {
  clear_error();
  if (!params || !grads || !m || !v) return fail(QPR_E_ARG, "NULL argument");
  if (count < 1 || step < 1) return fail(QPR_E_ARG, "count and step must be >= 1");
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  k_adam<<<nblk(count, 256), 256, 0, (hipStream_t)stream>>>(params, grads, m, v, count, lr, b1,
                                                            b2, eps, c1, c2);
  QPR_HIP(hipGetLastError());
  return QPR_OK;
}
