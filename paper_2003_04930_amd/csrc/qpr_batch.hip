// Many independent (graph, omega) systems in one set of launches.
//
// Every kernel of an RK4 stage is launched once for the whole batch over a
// device-side list of (system, tile) items -- the products with a persistent
// grid that strides over it, the epilogue with one workgroup per item -- and
// each item runs the same tile code as the single-system kernels.  A chunk of
// steps (plus, in mixed precision, the FP64 fold and judge) is captured once as
// a HIP graph and replayed; between replays the host reads every system's
// control block and rewrites the item lists to the systems still running
// (the lists live in device memory and their lengths are read by the kernels,
// so the graph is never re-captured).
//
// Precision: FP64 (sparse or dense product, as for one system) or FP32
// products with FP64 judging (the defect correction of the single solve).
// Integrator: classical RK4 with the fixed step dt, or (FP64) the adaptive
// Fehlberg 4(5) of the single solve, each system with its own step size and
// step control in its control block.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <vector>

#include "qpr_common.h"
#include "qpr_device.h"

namespace qpr {
namespace {

constexpr int TE = 32;  // epilogue tile edge (matches the epilogue kernels)

struct BatchFold {      // one system's fold: rho_a = (rho_a + delta) / tr, delta = 0
  double *an_r, *an_i, *dn_r, *dn_i, *p_a, *p_n;
  float *lo_r, *lo_i;
  int n, ld, renorm;
  DevState* st;
  float *d32_r, *d32_i;  // the defect held in FP32 (then dn_r / dn_i are unused), or null
};

// st->aux[0] = tr(rho_a + delta) from the two diagonals; one item per system
__global__ void __launch_bounds__(256) k_trace_batch(const BatchFold* __restrict__ f,
                                                     const int* __restrict__ sys_list,
                                                     const int* __restrict__ nsys) {
  __shared__ double red[4];
  const int ns = *nsys;
  for (int it = blockIdx.x; it < ns; it += gridDim.x) {
    const BatchFold& F = f[sys_list[it]];
    if (F.st->stop) continue;
    double s = 0.0;
    for (int j = threadIdx.x; j < F.n; j += 256) s += F.p_a[j] + F.p_n[j];
    s = block_sum(s, red, 4);
    if (threadIdx.x == 0) F.st->aux[0] = s;
    __syncthreads();
  }
}

// fold per (system, row block of 32 rows); skipped once the system stopped
__global__ void __launch_bounds__(256) k_fold_batch(const BatchFold* __restrict__ f,
                                                    const int2* __restrict__ items,
                                                    const int* __restrict__ nitems) {
  const int ni = *nitems;
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    const int2 item = items[it];
    const BatchFold& F = f[item.x];
    if (F.st->stop) continue;
    const double inv = F.renorm ? 1.0 / F.st->aux[0] : 1.0;
    const int r0 = item.y * TE;
    for (int e = threadIdx.x; e < TE * F.ld; e += 256) {
      const int a = r0 + e / F.ld, b = e % F.ld;
      const size_t o = (size_t)a * F.ld + b;
      double vr, vi;
      if (F.d32_r) {
        vr = (F.an_r[o] + (double)F.d32_r[o]) * inv;
        vi = (F.an_i[o] + (double)F.d32_i[o]) * inv;
        F.d32_r[o] = 0.f;
        F.d32_i[o] = 0.f;
      } else {
        vr = (F.an_r[o] + F.dn_r[o]) * inv;
        vi = (F.an_i[o] + F.dn_i[o]) * inv;
        F.dn_r[o] = 0.0;
        F.dn_i[o] = 0.0;
      }
      F.an_r[o] = vr;
      F.an_i[o] = vi;
      if (F.lo_r) {
        F.lo_r[o] = 0.f;
        F.lo_i[o] = 0.f;
      }
      if (a == b && a < F.n) {
        F.p_a[a] = vr;
        F.p_n[a] = 0.0;
      }
    }
  }
}

struct BatchCommit {    // one system's Fehlberg commit: y <- candidate when accepted
  double *yr, *yi, *p;
  const double *cr, *ci, *pc;
  int n, ld;
  const DevState* st;
};

// commit per (system, row block of 32 rows); skipped unless the attempt was
// accepted (and the system still runs)
__global__ void __launch_bounds__(256) k_commit_batch(const BatchCommit* __restrict__ c,
                                                      const int2* __restrict__ items,
                                                      const int* __restrict__ nitems) {
  const int ni = *nitems;
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    const int2 item = items[it];
    const BatchCommit& C = c[item.x];
    if (C.st->stop || !C.st->accept) continue;
    const size_t o0 = (size_t)item.y * TE * C.ld;
    for (int e = threadIdx.x; e < TE * C.ld; e += 256) {
      C.yr[o0 + e] = C.cr[o0 + e];
      C.yi[o0 + e] = C.ci[o0 + e];
    }
    for (int a = item.y * TE + threadIdx.x; a < item.y * TE + TE && a < C.n; a += 256)
      C.p[a] = C.pc[a];
  }
}

struct SysInfo {
  int n, ld;
  size_t ws_off, ws_size;
};

struct BatchLayout {
  std::vector<SysInfo> sys;
  size_t states, gemm_args, epi_args, fold_args, commit_args, items_g, items_e, items_f, items_s,
      sys_list, counts, total;
  size_t max_g, max_e, max_f, max_s;
};

// Stage argument slots per system: RK4 stages 0-3 and the judge (4), or the
// six Fehlberg stages.
constexpr int kSlots = 6;

BatchLayout batch_layout(int nsys, const int* ns, int prec, int gtile, bool rkf) {
  BatchLayout L;
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = align_up(o + b); return r; };
  L.max_g = L.max_e = L.max_f = L.max_s = 0;
  for (int s = 0; s < nsys; ++s) {
    SysInfo si;
    si.n = ns[s];
    si.ld = pad_n(ns[s]);
    si.ws_size = ws_bytes(ns[s], prec, rkf);
    si.ws_off = take(si.ws_size);
    L.sys.push_back(si);
    const size_t tg = (size_t)(si.ld / gtile) * (si.ld / gtile);
    L.max_g += std::max(tg, (size_t)(si.ld / 32) * (si.ld / 32));  // any batch tile size
    L.max_e += (size_t)epilogue_items_per_system(si.ld);
    L.max_f += (size_t)(si.ld / TE);
    L.max_s += (size_t)spmm_items_per_system(si.n, si.ld);
  }
  L.states = take((size_t)nsys * sizeof(DevState));
  L.gemm_args = take((size_t)nsys * kSlots * sizeof(BatchGemm));
  L.epi_args = take((size_t)nsys * kSlots * sizeof(BatchEpi));
  L.fold_args = take((size_t)nsys * sizeof(BatchFold));
  L.commit_args = take((size_t)nsys * sizeof(BatchCommit));
  L.items_g = take(L.max_g * sizeof(int2));
  L.items_e = take(L.max_e * sizeof(int2));
  L.items_f = take(L.max_f * sizeof(int2));
  L.items_s = take(L.max_s * sizeof(int2));
  L.sys_list = take((size_t)nsys * sizeof(int));
  L.counts = take(5 * sizeof(int));
  L.total = o;
  return L;
}

// Which form runs.  QPR_BATCH_AUTO takes the persistent form for FP32
// batches of eight or more systems whose defect may be held in FP32 (product
// QPR_PRODUCT_AUTO, delta_state not FP64): with the FP32 defect it runs
// 1.2-1.35x the concurrent form's solves/s from 10 to 1,280 family systems.
// Otherwise the concurrent form, faster on every FP64 batch and on three
// N = 922 systems.  Decided from what the workspace query also sees.
bool batch_concurrent(const qpr_opts* o, int prec, int nsys) {
  const int mode = o ? o->batch_mode : QPR_BATCH_AUTO;
  if (mode != QPR_BATCH_AUTO) return mode != QPR_BATCH_PERSISTENT;
  const bool fp32_state = prec == QPR_FP32 && nsys >= 8 &&
                          (!o || (o->product == QPR_PRODUCT_AUTO && o->delta_state != 1 &&
                                  o->integrator != QPR_RKF45));
  return !fp32_state;
}
// The concurrent form: its workers and the arena of one single-system
// workspace per worker.
int batch_workers(int nsys, const qpr_opts* o) {
  const int w = o && o->batch_workers > 0 ? o->batch_workers : 8;
  return std::max(1, std::min(std::min(w, nsys), kMaxWorkers));
}
size_t worker_ws_stride(int nsys, const int* n, int prec, bool rkf) {
  int nmax = 0;
  for (int s = 0; s < nsys; ++s) nmax = std::max(nmax, n[s]);
  return align_up(ws_bytes(nmax, prec, rkf));
}

}  // namespace
}  // namespace qpr

using namespace qpr;

extern "C" size_t qpr_batch_workspace_bytes(int32_t nsys, const int32_t* n, int32_t prec,
                                            const qpr_opts* opts) {
  if (nsys < 1 || !n || (prec != QPR_FP64 && prec != QPR_FP32)) return 0;
  for (int s = 0; s < nsys; ++s)
    if (n[s] < 2) return 0;
  const bool rkf = opts && opts->integrator == QPR_RKF45;
  if (rkf && prec != QPR_FP64) return 0;
  if (batch_concurrent(opts, prec, nsys))
    return batch_workers(nsys, opts) * worker_ws_stride(nsys, n, prec, rkf);
  return batch_layout(nsys, n, prec, 32, rkf).total;
}

extern "C" qpr_status qpr_batch_solve(int32_t nsys, const qpr_problem* const* probs,
                                      const double* omegas, double dt, double tol,
                                      int64_t max_steps, int32_t prec, double* const* rhos,
                                      int32_t* const* ranks, qpr_stats* stats,
                                      const qpr_opts* opts, int32_t* tuned_cfg,
                                      const char* tune_cache, void* ws, size_t ws_bytes_,
                                      qpr_stream_t stream) {
  const auto t0 = std::chrono::steady_clock::now();
  clear_error();
  if (nsys < 1) return fail(QPR_E_ARG, "nsys must be >= 1");
  if (!probs || !omegas || !rhos) return fail(QPR_E_ARG, "probs, omegas and rhos must not be NULL");
  if (prec != QPR_FP64 && prec != QPR_FP32)
    return fail(QPR_E_ARG, "batched solve supports QPR_FP64 and QPR_FP32 (got %d)", prec);
  if (!(tol > 0.0)) return fail(QPR_E_ARG, "tol must be positive");
  if (max_steps < 0) return fail(QPR_E_ARG, "max_steps must be >= 0");
  if (!ws || ((uintptr_t)ws) % kAlign) return fail(QPR_E_ARG, "workspace must be 256-byte aligned");
  if (tune_cache) {
    const qpr_status ts = qpr_load_tuning(tune_cache);
    if (ts != QPR_OK) return ts;  // its message names the cache
    clear_error();
  }
  qpr_opts o{};
  o.use_graph = 1;
  o.renorm = 1;
  o.gemm_cfg = -1;
  o.product = QPR_PRODUCT_AUTO;
  o.step_tol = 1e-4;
  if (opts) o = *opts;
  if (o.batch_mode < QPR_BATCH_AUTO || o.batch_mode > QPR_BATCH_CONCURRENT)
    return fail(QPR_E_ARG, "unknown batch_mode %d", o.batch_mode);
  const bool concurrent = batch_concurrent(&o, prec, nsys);
  if (!concurrent && o.product == QPR_PRODUCT_BLOCKSPARSE)
    return fail(QPR_E_ARG, "the persistent batch form has no block-sparse product");
  if (o.chunk <= 0) o.chunk = concurrent ? 64 : 32;
  const bool rkf = o.integrator == QPR_RKF45;
  if (rkf && prec != QPR_FP64) return fail(QPR_E_ARG, "the RKF45 integrator runs in FP64 only");
  if (rkf && !(o.step_tol > 0.0)) return fail(QPR_E_ARG, "step_tol must be positive");
  if (o.integrator != QPR_RK4 && !rkf) return fail(QPR_E_ARG, "unknown integrator %d", o.integrator);
  std::vector<int> ns(nsys);
  for (int s = 0; s < nsys; ++s) {
    const qpr_problem* P = probs[s];
    if (!P || P->n < 2 || P->ld != pad_n(P->n) || !P->h_off)
      return fail(QPR_E_ARG, "system %d: not a built problem", s);
    if (!(omegas[s] >= 0.0 && omegas[s] <= 1.0))
      return fail(QPR_E_ARG, "system %d: omega must be in [0,1]", s);
    if (!rhos[s]) return fail(QPR_E_ARG, "system %d: rho must not be NULL", s);
    const double reach = dt * ((1.0 - omegas[s]) * (P->h_hi - P->h_lo) + 2.0 * omegas[s]);
    if (!(dt > 0.0)) return fail(QPR_E_ARG, "dt must be positive (got %g)", dt);
    if (!rkf && reach >= 2.8)
      return fail(QPR_E_UNSTABLE, "system %d: dt=%g outside the RK4 stability bound", s, dt);
    ns[s] = P->n;
  }
  hipStream_t s = (hipStream_t)stream;
  if (concurrent) {
    // one workspace and one stream per worker, the streams ordered after the
    // caller's stream (where the initial states were written)
    const int nw = batch_workers(nsys, &o);
    const size_t stride = worker_ws_stride(nsys, ns.data(), prec, rkf);
    if (ws_bytes_ < stride * nw)
      return fail(QPR_E_WORKSPACE, "batch workspace has %zu bytes, needs %zu", ws_bytes_,
                  stride * nw);
    std::vector<void*> wsp(nw);
    std::vector<size_t> wsb(nw, stride);
    std::vector<HipStream> streams(nw);
    std::vector<qpr_stream_t> hs(nw);
    HipEvent ready;
    QPR_HIP(hipEventCreateWithFlags(&ready.h, hipEventDisableTiming));
    QPR_HIP(hipEventRecord(ready.h, s));
    for (int w = 0; w < nw; ++w) {
      wsp[w] = (char*)ws + stride * w;
      QPR_HIP(hipStreamCreateWithFlags(&streams[w].h, hipStreamNonBlocking));
      QPR_HIP(hipStreamWaitEvent(streams[w].h, ready.h, 0));
      hs[w] = (qpr_stream_t)streams[w].h;
    }
    if (tuned_cfg) *tuned_cfg = -1;
    return run_many(nsys, probs, omegas, dt, tol, max_steps, prec, rhos, ranks, stats, &o, nw,
                    wsp.data(), wsb.data(), hs.data());
  }
  const BatchLayout L = batch_layout(nsys, ns.data(), prec, 32, rkf);
  if (ws_bytes_ < L.total)
    return fail(QPR_E_WORKSPACE, "batch workspace has %zu bytes, needs %zu", ws_bytes_, L.total);
  char* base = (char*)ws;
  DevState* states = (DevState*)(base + L.states);
  BatchGemm* d_gemm = (BatchGemm*)(base + L.gemm_args);
  BatchEpi* d_epi = (BatchEpi*)(base + L.epi_args);
  BatchFold* d_fold = (BatchFold*)(base + L.fold_args);
  BatchCommit* d_commit = (BatchCommit*)(base + L.commit_args);
  int2* d_items_g = (int2*)(base + L.items_g);
  int2* d_items_e = (int2*)(base + L.items_e);
  int2* d_items_f = (int2*)(base + L.items_f);
  int* d_sys_list = (int*)(base + L.sys_list);
  int2* d_items_s = (int2*)(base + L.items_s);
  int* d_counts = (int*)(base + L.counts);  // [gemm, epilogue, fold, systems, sparse]

  const bool mixed = prec == QPR_FP32;
  const int xk = mixed ? OP_F32 : OP_F64;
  // products: sparse gathers (FP64 operands, or the FP32 delta copy in FP32
  // mode) below 5 % density unless opts->product says otherwise
  auto sparse_for = [&](const qpr_problem* P) {
    if (o.product == QPR_PRODUCT_DENSE) return false;
    if (o.product == QPR_PRODUCT_SPARSE || o.product == QPR_PRODUCT_FUSED) return true;
    return (double)P->nnz_h < 0.05 * (double)P->n * (double)P->n;
  };
  // one product form for all systems of the shared launches, decided on the
  // largest system (the one whose stages cost the most); the small ones of a
  // mixed-size batch may be denser than the threshold, which only changes
  // their speed, never their result
  int big = 0;
  for (int k = 1; k < nsys; ++k)
    if (probs[k]->n > probs[big]->n) big = k;
  const bool step_sparse = sparse_for(probs[big]);
  const bool judge_sparse = step_sparse;
  // FP64 sparse stages as fused epilogues (the gathers inside the tile
  // kernel, bitwise the same sums): the FP64 steps and the judge; the FP32
  // steps of the mixed solve keep their FP32 product.  AUTO fuses: over 160
  // family systems (N 50..922) the fused stages give 5.46 against 3.88
  // solves/s with RK4 and 17.2 against 13.5 with RKF45.
  const bool fuse = o.product == QPR_PRODUCT_FUSED || o.product == QPR_PRODUCT_AUTO;
  // the FP32 steps fused too (gathers of the FP32 state copy inside the tile
  // kernel): 5.85 against 4.07 solves/s over the same 160 systems
  const bool fuse32 = fuse;
  // the defect held in FP32 (every state plane of the FP32 steps single
  // precision), as the lone mixed solve does by default with the sparse
  // product: half the bytes per stage
  if (mixed && (o.delta_state < 0 || o.delta_state > 2))
    return fail(QPR_E_ARG, "delta_state must be 0, 1 or 2 (got %d)", o.delta_state);
  if (mixed && o.delta_state == 2 && !step_sparse)
    return fail(QPR_E_ARG, "an FP32 defect needs the sparse product");
  const bool state32 = mixed && step_sparse &&
                       (o.delta_state == 2 || (o.delta_state == 0 && o.product == QPR_PRODUCT_AUTO));
  const int xs_step = state32 ? XS_FUSED32S
                      : mixed ? (step_sparse && fuse32 ? XS_FUSED32 : XS_DENSE32)
                      : step_sparse ? (fuse ? XS_FUSED64 : XS_SPARSE64) : XS_DENSE64;
  const int xs_judge = judge_sparse ? (fuse ? XS_FUSED64 : XS_SPARSE64) : XS_DENSE64;
  // the dense product's tile configurations at this precision
  int cands[8];
  const int ncand = batch_gemm_cfgs(xk, cands, 8);
  if (!step_sparse && o.gemm_cfg >= ncand)
    return fail(QPR_E_ARG, "gemm_cfg %d: the batched product has %d tile configurations at "
                "this precision", o.gemm_cfg, ncand);

  // host argument tables: slots 0..3 = RK4 stages, 4 = judge / RHS; or the six
  // Fehlberg stages
  std::vector<Ws> W(nsys);
  std::vector<BatchGemm> hg((size_t)nsys * kSlots);
  std::vector<BatchEpi> he((size_t)nsys * kSlots);
  std::vector<BatchFold> hf(nsys);
  std::vector<BatchCommit> hc(nsys);
  std::vector<double> hmax(nsys, 0.0);
  for (int k = 0; k < nsys; ++k) {
    const qpr_problem* P = probs[k];
    Ws& w = W[k];
    if (!ws_carve(base + L.sys[k].ws_off, L.sys[k].ws_size, P->n, prec, &w, rkf))
      return fail(QPR_E_WORKSPACE, "system %d: workspace carve failed", k);
    w.st = states + k;
    const ProbView pv = view_of(P);
    if (rkf) {
      hmax[k] = o.dt_max > 0.0 ? o.dt_max : rkf_step_cap(omegas[k], P->h_norm);
      if (!(hmax[k] > 0.0))
        return fail(QPR_E_UNSTABLE, "system %d: no stable Fehlberg step at omega=%g", k, omegas[k]);
      for (int q = 0; q < 6; ++q) {
        BatchGemm& g = hg[(size_t)q * nsys + k];
        BatchEpi& e = he[(size_t)q * nsys + k];
        e = BatchEpi{};
        e.pv = pv;
        e.st = w.st;
        e.partials = w.partials;
        e.a = rkf_stage_args(w, q, omegas[k], xs_step);
        g = BatchGemm{};
        g.H = P->h_off;
        g.yr = e.a.ysr;
        g.yi = e.a.ysi;
        g.xr = w.x_r;
        g.xi = w.x_i;
        g.ld = P->ld;
        g.gate = 0;
        g.st = w.st;
      }
      hc[k] = BatchCommit{w.yn_r, w.yn_i, w.p_n, w.cand_r, w.cand_i, w.p_c, P->n, P->ld, w.st};
      continue;
    }
    struct St {
      double *inr, *ini, *pin, *outr, *outi, *pout, cdt;
    };
    const St stg[4] = {{w.yn_r, w.yn_i, w.p_n, w.y1_r, w.y1_i, w.p_1, 0.5 * dt},
                       {w.y1_r, w.y1_i, w.p_1, w.y2_r, w.y2_i, w.p_2, 0.5 * dt},
                       {w.y2_r, w.y2_i, w.p_2, w.y1_r, w.y1_i, w.p_1, dt},
                       {w.y1_r, w.y1_i, w.p_1, w.yn_r, w.yn_i, w.p_n, dt / 6.0}};
    for (int q = 0; q < 5; ++q) {
      BatchGemm& g = hg[(size_t)q * nsys + k];
      BatchEpi& e = he[(size_t)q * nsys + k];
      g = BatchGemm{};
      e = BatchEpi{};
      e.pv = pv;
      e.st = w.st;
      e.partials = w.partials;
      EpiArgs& a = e.a;
      a.xr = w.x_r;
      a.xi = w.x_i;
      a.xfr = w.xf_r;
      a.xfi = w.xf_i;
      a.omega = omegas[k];
      if (q < 4) {
        const St& sg = stg[q];
        g.H = mixed ? (const void*)P->h_off_f32 : (const void*)P->h_off;
        g.yr = mixed ? (const void*)w.lo_r : (const void*)sg.inr;
        g.yi = mixed ? (const void*)w.lo_i : (const void*)sg.ini;
        g.xr = mixed ? (void*)w.xf_r : (void*)w.x_r;
        g.xi = mixed ? (void*)w.xf_i : (void*)w.x_i;
        g.ld = P->ld;
        g.gate = mixed ? 1 : 0;
        g.st = w.st;
        a.ysr = sg.inr;
        a.ysi = sg.ini;
        a.ps = sg.pin;
        a.ynr = w.yn_r;
        a.yni = w.yn_i;
        a.accr = w.acc_r;
        a.acci = w.acc_i;
        a.outr = sg.outr;
        a.outi = sg.outi;
        a.pout = sg.pout;
        a.rar = mixed ? w.ra_r : nullptr;
        a.rai = mixed ? w.ra_i : nullptr;
        a.lor = mixed ? w.lo_r : nullptr;
        a.loi = mixed ? w.lo_i : nullptr;
        a.cdt = sg.cdt;
        a.mode = EPI_S1 + q;
        a.xkind = xs_step;
        if (xs_step == XS_FUSED32) {  // FP32 copies alternate between lo and the X planes
          a.xfr = q % 2 ? w.xf_r : w.lo_r;
          a.xfi = q % 2 ? w.xf_i : w.lo_i;
          a.lor = q % 2 ? w.lo_r : w.xf_r;
          a.loi = q % 2 ? w.lo_i : w.xf_i;
        }
        a.check = q == 0 ? (mixed ? CHK_DELTA : CHK_PLAIN) : CHK_NONE;
        a.gate = mixed ? 1 : 0;
        if (state32) a = rk4_stage_args_f32s(w, q, omegas[k], dt, CHK_DELTA, 1);
      } else {  // judge: r_a = L(rho_a) with the FP64 product
        g.H = P->h_off;
        g.yr = w.an_r;
        g.yi = w.an_i;
        g.xr = w.x_r;
        g.xi = w.x_i;
        g.ld = P->ld;
        g.gate = 0;
        g.st = w.st;
        a.ysr = w.an_r;
        a.ysi = w.an_i;
        a.ps = w.p_a;
        a.outr = w.ra_r;
        a.outi = w.ra_i;
        a.mode = EPI_RHS;
        a.xkind = xs_judge;
        a.check = CHK_JUDGE;
        if (state32) {  // and the FP32 copy of r_a the FP32 steps add
          a.lor = w.ra32_r;
          a.loi = w.ra32_i;
        }
      }
    }
    hf[k] = BatchFold{w.an_r, w.an_i, w.yn_r, w.yn_i, w.p_a, w.p_n,
                      mixed && !state32 ? w.lo_r : nullptr, mixed && !state32 ? w.lo_i : nullptr,
                      P->n, P->ld, o.renorm ? 1 : 0, w.st,
                      state32 ? w.dn_r : nullptr, state32 ? w.dn_i : nullptr};
  }
  QPR_HIP(hipMemcpyAsync(d_gemm, hg.data(), hg.size() * sizeof(BatchGemm), hipMemcpyHostToDevice, s));
  QPR_HIP(hipMemcpyAsync(d_epi, he.data(), he.size() * sizeof(BatchEpi), hipMemcpyHostToDevice, s));
  QPR_HIP(hipMemcpyAsync(d_fold, hf.data(), hf.size() * sizeof(BatchFold), hipMemcpyHostToDevice, s));
  QPR_HIP(hipMemcpyAsync(d_commit, hc.data(), hc.size() * sizeof(BatchCommit), hipMemcpyHostToDevice, s));

  // initial state of every system
  for (int k = 0; k < nsys; ++k) {
    const qpr_problem* P = probs[k];
    Ws& w = W[k];
    QPR_HIP(launch_state_init(w.st, tol, max_steps, rkf ? CHK_RKF : mixed ? CHK_DELTA : CHK_PLAIN, s));
    if (rkf) QPR_HIP(launch_state_rkf(w.st, std::min(dt, hmax[k]), hmax[k], o.step_tol, s));
    if (mixed) {
      const size_t plane = (size_t)P->ld * P->ld;
      QPR_HIP(launch_pad_in(rhos[k], P->n, P->ld, w.an_r, w.an_i, w.p_a, s));
      QPR_HIP(launch_fill(w.yn_r, 2 * plane * 8, s));
      QPR_HIP(launch_fill(w.p_n, (size_t)P->ld * 8, s));
      QPR_HIP(launch_fill(w.lo_r, 2 * plane * 4, s));
    } else {
      QPR_HIP(launch_pad_in(rhos[k], P->n, P->ld, w.yn_r, w.yn_i, w.p_n, s));
    }
  }

  // work lists, largest systems first
  std::vector<int> order(nsys);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ns[a] > ns[b]; });
  int gtile = 64;
  int gcfg = -1;  // index into the batch kernel table
  int gpick = -1; // the same as an index into this precision's candidates (what
                  // opts->gemm_cfg takes and tuned_cfg reports)
  std::vector<int2> ig, ie, iff, isp;
  std::vector<int> sl;
  std::vector<char> active(nsys, 1);
  auto build_lists = [&]() {
    ig.clear();
    ie.clear();
    iff.clear();
    isp.clear();
    sl.clear();
    for (int k : order) {
      if (!active[k]) continue;
      const int ld = pad_n(ns[k]);
      const int tg = (ld / gtile) * (ld / gtile), te = epilogue_items_per_system(ld);
      for (int t = 0; t < tg; ++t) ig.push_back(make_int2(k, t));
      for (int t = 0; t < te; ++t) ie.push_back(make_int2(k, t));
      for (int t = 0; t < ld / TE; ++t) iff.push_back(make_int2(k, t));
      const int ts = spmm_items_per_system(ns[k], ld);
      for (int t = 0; t < ts; ++t) isp.push_back(make_int2(k, t));
      sl.push_back(k);
    }
  };
  HostPinned counts_buf;
  QPR_HIP(hipHostMalloc(&counts_buf.h, 5 * sizeof(int), hipHostMallocDefault));
  int* h_counts = (int*)counts_buf.h;
  auto upload_lists = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(d_items_g, ig.data(), ig.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_items_e, ie.data(), ie.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_items_f, iff.data(), iff.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_sys_list, sl.data(), sl.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_items_s, isp.data(), isp.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    h_counts[0] = (int)ig.size();
    h_counts[1] = (int)ie.size();
    h_counts[2] = (int)iff.size();
    h_counts[3] = (int)sl.size();
    h_counts[4] = (int)isp.size();
    if (e == hipSuccess) e = hipMemcpyAsync(d_counts, h_counts, 5 * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host vectors are reused
    return e;
  };

  const bool use_gemm = !step_sparse;
  const int grid_g = 1024, grid_e = 2048, grid_f = 1024;
  // the epilogue takes one work item per workgroup: its grid covers the whole
  // initial list (all systems running); later, workgroups past the live count
  // exit at once
  build_lists();
  const int grid_e1 = std::max(1, (int)ie.size());
  // tile configuration: tuned on this batch's own work list unless given
  if (use_gemm) {
    if (o.gemm_cfg >= 0) {
      gpick = o.gemm_cfg;
      gcfg = cands[gpick];
    } else {
      HipEvent ev0, ev1;
      QPR_HIP(hipEventCreate(&ev0.h));
      QPR_HIP(hipEventCreate(&ev1.h));
      hipEvent_t e0 = ev0.h, e1 = ev1.h;
      float best = 1e30f;
      for (int c = 0; c < ncand; ++c) {
        // a dense FP64 judge shares the item list, so it needs 64-wide tiles
        if (mixed && !judge_sparse && batch_gemm_tile(cands[c]) != 64) continue;
        gtile = batch_gemm_tile(cands[c]);
        build_lists();
        QPR_HIP(upload_lists());
        QPR_HIP(launch_gemm_batch(cands[c], d_gemm, d_items_g, d_counts, grid_g, s));
        QPR_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r)
          QPR_HIP(launch_gemm_batch(cands[c], d_gemm, d_items_g, d_counts, grid_g, s));
        QPR_HIP(hipEventRecord(e1, s));
        QPR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        QPR_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          gcfg = cands[c];
          gpick = c;
        }
      }
    }
    gtile = batch_gemm_tile(gcfg);
  }
  if (tuned_cfg) *tuned_cfg = gpick;
  build_lists();
  QPR_HIP(upload_lists());

  auto enqueue_stage = [&](int q, hipStream_t qs) -> hipError_t {
    hipError_t e = hipSuccess;
    const bool judge = !rkf && q == 4;
    const bool gemm = judge ? !judge_sparse : use_gemm;
    const int xs = judge ? xs_judge : xs_step;
    // the fused kinds gather inside the epilogue: no product launch (the FP32
    // product would read the FP32 copy, which the FP32-state stages do not keep)
    const bool spmm = (judge ? judge_sparse : step_sparse) && xs != XS_FUSED64 &&
                      xs != XS_FUSED32 && xs != XS_FUSED32S;
    if (spmm) {
      e = mixed && !judge
              ? launch_spmm_f32_batch(d_epi + (size_t)q * nsys, d_items_s, d_counts + 4, grid_e, qs)
              : launch_spmm_batch(d_epi + (size_t)q * nsys, d_items_s, d_counts + 4, grid_e, qs);
      if (e != hipSuccess) return e;
    }
    if (gemm) {
      // the judge always takes the FP64 product (configuration 0 of the FP64 batch table)
      const int cfg = judge ? 0 : gcfg;
      e = launch_gemm_batch(cfg, d_gemm + (size_t)q * nsys, d_items_g, d_counts, grid_g, qs);
      if (e != hipSuccess) return e;
    }
    const bool finish = rkf ? (q == 0 || q == 5) : (q == 0 || q == 4);
    return launch_epilogue_batch(xs, d_epi + (size_t)q * nsys, d_items_e, d_counts + 1, grid_e1,
                                 d_sys_list, d_counts + 3, finish, qs);
  };
  auto enqueue_fold_judge = [&](hipStream_t qs) -> hipError_t {
    k_trace_batch<<<256, 256, 0, qs>>>(d_fold, d_sys_list, d_counts + 3);
    k_fold_batch<<<grid_f, 256, 0, qs>>>(d_fold, d_items_f, d_counts + 2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return enqueue_stage(4, qs);
  };
  if (mixed && !judge_sparse && gtile != 64)
    return fail(QPR_E_ARG, "dense FP64 judging needs a 64-wide product tile configuration");
  if (mixed) QPR_HIP(enqueue_fold_judge(s));  // fold of delta = 0: renormalise + judge rho0

  auto enqueue_chunk = [&](hipStream_t qs) -> hipError_t {
    for (int k = 0; k < o.chunk; ++k) {
      for (int q = 0; q < (rkf ? 6 : 4); ++q) {
        hipError_t e = enqueue_stage(q, qs);
        if (e != hipSuccess) return e;
      }
      if (rkf) {
        k_commit_batch<<<grid_f, 256, 0, qs>>>(d_commit, d_items_f, d_counts + 2);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    return mixed ? enqueue_fold_judge(qs) : hipSuccess;
  };
  HipStream cap_stream;
  HipGraph graph_h;
  HipGraphExec exec_h;
  if (o.use_graph) {
    QPR_HIP(hipStreamCreateWithFlags(&cap_stream.h, hipStreamNonBlocking));
    QPR_HIP(hipStreamBeginCapture(cap_stream.h, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_chunk(cap_stream.h);
    hipError_t e2 = hipStreamEndCapture(cap_stream.h, &graph_h.h);
    QPR_HIP(e);
    QPR_HIP(e2);
    QPR_HIP(hipGraphInstantiate(&exec_h.h, graph_h.h, nullptr, nullptr, 0));
  }
  hipGraphExec_t exec = exec_h.h;
  std::vector<DevState> hs(nsys);
  qpr_status rc = QPR_OK;
  Progress progress("persistent batch");
  for (;;) {
    hipError_t e = o.use_graph ? hipGraphLaunch(exec, s) : enqueue_chunk(s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hs.data(), states, nsys * sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      rc = fail(QPR_E_HIP, "batched chunk failed: %s", hipGetErrorString(e));
      break;
    }
    int running = 0;
    bool changed = false;
    for (int k = 0; k < nsys; ++k) {
      const bool a = hs[k].stop == 0;
      if (!a && active[k]) {
        active[k] = 0;
        changed = true;
      }
      running += a;
    }
    progress.report(nsys - running, nsys, "stopped");
    if (!running) break;
    if (changed) {
      build_lists();
      e = upload_lists();
      if (e != hipSuccess) {
        rc = fail(QPR_E_HIP, "work-list upload failed: %s", hipGetErrorString(e));
        break;
      }
    }
  }
  if (rc != QPR_OK) return rc;

  // results: state, ranking and diagnostics per system
  int n_bad = 0, n_unconv = 0;
  for (int k = 0; k < nsys; ++k) {
    const qpr_problem* P = probs[k];
    Ws& w = W[k];
    double* outr = mixed ? w.an_r : w.yn_r;
    double* outi = mixed ? w.an_i : w.yn_i;
    double* outp = mixed ? w.p_a : w.p_n;
    const DevState& f = hs[k];
    if (!f.nonfinite) {
      QPR_HIP(launch_state_stats(outr, outi, outp, P->n, P->ld, w, s));
      QPR_HIP(launch_pad_out(outr, outi, P->n, P->ld, rhos[k], s));
      if (ranks && ranks[k] && f.converged) QPR_HIP(launch_rank(P->n, outp, ranks[k], s));
    }
  }
  QPR_HIP(hipMemcpyAsync(hs.data(), states, nsys * sizeof(DevState), hipMemcpyDeviceToHost, s));
  QPR_HIP(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int k = 0; k < nsys; ++k) {
    const DevState& f = hs[k];
    n_bad += f.nonfinite != 0;
    n_unconv += !f.converged;
    if (!stats) continue;
    qpr_stats& S = stats[k];
    S = qpr_stats{};
    if (rkf) {
      S.steps = f.accepted;
      S.rejected = f.rejected;
      S.rhs_evals = 6 * (f.accepted + f.rejected) + 1;
      S.rhs_evals_fp64 = S.rhs_evals;
      S.t = f.t;
      S.last_step = f.h;
      S.residual = std::sqrt(f.resid2);
      S.trace_err = std::fabs(f.aux[0] - 1.0);
      S.herm_err = f.aux[1];
      S.min_diag = f.aux[2];
      S.seconds = secs;
      S.converged = f.converged;
      S.status = f.nonfinite ? QPR_E_NONFINITE : f.converged ? QPR_OK : QPR_E_NOT_CONVERGED;
      continue;
    }
    S.steps = f.converged ? f.conv_step : f.step;
    S.folds = f.folds;
    S.rhs_evals_fp64 = mixed ? f.folds : 4 * S.steps + 1;
    S.rhs_evals = 4 * S.steps + (mixed ? f.folds : 1);
    S.t = (double)S.steps * dt;
    S.residual = std::sqrt(mixed ? f.judge2 : f.resid2);
    S.trace_err = std::fabs(f.aux[0] - 1.0);
    S.herm_err = f.aux[1];
    S.min_diag = f.aux[2];
    S.seconds = secs;
    S.converged = f.converged;
    S.status = f.nonfinite ? QPR_E_NONFINITE : f.converged ? QPR_OK : QPR_E_NOT_CONVERGED;
  }
  if (n_bad) return fail(QPR_E_NONFINITE, "%d systems met non-finite values", n_bad);
  if (n_unconv) return fail(QPR_E_NOT_CONVERGED, "%d systems did not converge", n_unconv);
  return QPR_OK;
}
