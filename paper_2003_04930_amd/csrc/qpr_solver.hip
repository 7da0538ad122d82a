// Host drivers of the C ABI: right-hand side, fixed RK4 steps and the
// steady-state solve (plain FP64, or defect correction with a low-precision
// product judged in FP64).
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "qpr_common.h"

namespace qpr {

namespace {
thread_local char g_err[512] = "";

constexpr double kRk4Limit = 2.8;  // inside RK4's stability region on both axes
}  // namespace

qpr_status fail(qpr_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}
void clear_error() { g_err[0] = 0; }

// Sparse gathers for the FP64 product when H_off is sparse enough (or forced).
// The sparse product serves the FP64 and the FP32-operand products (there is
// no three-slice bf16 form: its point is the MFMA throughput of dense tiles).
// The fused mode asks for the same gathers, so it implies the sparse product
// wherever the fused epilogue does not apply (the FP32 product).
static bool use_sparse(const qpr_problem* P, int product, int xk) {
  if (xk == OP_BF16X3 || product == QPR_PRODUCT_DENSE || product == QPR_PRODUCT_BLOCKSPARSE)
    return false;
  if (product == QPR_PRODUCT_SPARSE || product == QPR_PRODUCT_FUSED) return true;
  return (double)P->nnz_h < 0.05 * (double)P->n * (double)P->n;
}

// Where the epilogue takes X from: the FP32 X of a low-precision product, the
// FP64 X a separate product launch wrote (sparse or dense), or the epilogue's
// own gathers (fused: no product launch).
// AUTO takes the FP64 fused epilogue from a padded size of 4096 on: there a
// stage is 13 % faster than product + epilogue; at 922 and 2048 the two
// kernels win when a solve runs alone (the fused tile pairs run their gathers
// and the epilogue back to back, with too few workgroups per CU to hide
// either).  The FP32 steps of the mixed solve take the fused form at every
// size: it gathers half the bytes (N = 922 solve 0.546 against 0.568 s,
// N = 4096 stage 314 against 349 us).
static int x_source(const qpr_problem* P, int product, int xk) {
  if (xk == OP_BF16X3) return XS_DENSE32;
  const bool sparse = use_sparse(P, product, xk);
  if (xk == OP_F32)
    return sparse && (product == QPR_PRODUCT_FUSED || product == QPR_PRODUCT_AUTO) ? XS_FUSED32
                                                                                  : XS_DENSE32;
  if (product == QPR_PRODUCT_FUSED) return XS_FUSED64;
  if (!sparse) return XS_DENSE64;
  if (product != QPR_PRODUCT_AUTO) return XS_SPARSE64;
  int fused;  // the autotuner's choice for this padded size, else the measured rule
  if (tuned_exact(kTuneFusedStage, P->ld, &fused)) return fused ? XS_FUSED64 : XS_SPARSE64;
  return P->ld >= 4096 ? XS_FUSED64 : XS_SPARSE64;
}

// The problem view with the sparse-product variant the options ask for.
static qpr_status view_for(const qpr_problem* P, const qpr_opts& o, ProbView* pv) {
  *pv = view_of(P);
  if (o.sparse_variant < 0 || o.sparse_variant > spmm_num_variants())
    return fail(QPR_E_ARG, "sparse_variant must be in [0, %d]", spmm_num_variants());
  pv->spmm_variant = o.sparse_variant - 1;
  return QPR_OK;
}

// X = H_off Y for a stage: the sparse gathers (FP64 operand, or the FP32 copy
// of the state in FP32 mode) or the dense MFMA product.
// A sparse launch may carry the finishing step `fin` of the previous stage.
static hipError_t launch_product(const qpr_problem* P, const Ws& w, const ProbView& pv, int xk,
                                 int cfg, bool sparse, const double* yr, const double* yi,
                                 int gate, hipStream_t s, int spv = -1,
                                 const FinishJob* fin = nullptr) {
  if (!sparse) return launch_gemm(xk, cfg, P, w, yr, yi, gate, s);
  if (xk == OP_F32) return launch_spmm_f32(pv, w.lo_r, w.lo_i, w.xf_r, w.xf_i, w.st, gate, s, fin);
  return launch_spmm(pv, yr, yi, w.x_r, w.x_i, w.st, gate, s, spv, fin);
}

static int op_kind(int prec) {
  return prec == QPR_FP32 ? OP_F32 : prec == QPR_BF16X3 ? OP_BF16X3 : OP_F64;
}

// QPR_PRODUCT_BLOCKSPARSE: build the slab lists of H_off in the workspace and
// route every product of the call to the tile-skipping kernels (the dense
// product's role: use_sparse() is false for it).
static qpr_status setup_product(const qpr_problem* P, const Ws& w, int prec, qpr_opts* o,
                                hipStream_t s) {
  if (o->product < QPR_PRODUCT_AUTO || o->product > QPR_PRODUCT_BLOCKSPARSE)
    return fail(QPR_E_ARG, "unknown product %d", o->product);
  if (o->product != QPR_PRODUCT_BLOCKSPARSE) return QPR_OK;
  if (prec == QPR_BF16X3)
    return fail(QPR_E_ARG, "the block-sparse product serves QPR_FP64 and QPR_FP32");
  QPR_HIP(launch_block_pattern(P, w, s));
  o->gemm_cfg = kCfgBlockSparse;
  return QPR_OK;
}

// ---------------------------------------------------------------- workspace
namespace {
struct WsLayout {
  size_t yn, y1, y2, acc, x, ra, an, xf, lo, sl, pv, kf, cand, pc, partials, st, scal, bs, total;
  int max_partials;
};

WsLayout ws_layout(int n, int prec, bool rkf) {
  const size_t ld = (size_t)pad_n(n);
  const size_t pd = ld * ld * 8, pf = ld * ld * 4, ph = ld * ld * 2;
  WsLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = align_up(o + b); return r; };
  L.yn = take(2 * pd);
  L.y1 = take(2 * pd);
  L.y2 = take(2 * pd);
  const size_t pk = packed_values((int)ld) * 8;  // Hermitian-packed, by tile pair
  L.acc = take(pk);
  L.x = take(2 * pd);
  if (prec != QPR_FP64) {
    L.ra = take(2 * pd);
    L.an = take(2 * pd);
    L.xf = take(2 * pf);
    if (prec == QPR_FP32) L.lo = take(2 * pf);
    if (prec == QPR_BF16X3) L.sl = take(6 * ph);
  }
  L.pv = take(4 * ld * 8);
  if (prec == QPR_FP64 && rkf) {  // Fehlberg: K_1..K_5, candidate state and its diagonal
    L.kf = take(5 * pk);
    L.cand = take(2 * pd);
    L.pc = take(ld * 8);
  }
  const size_t tiles = (ld / 32) * (ld / 32);
  L.max_partials = (int)std::max<size_t>(3 * tiles, 4 * 1024);
  L.partials = take((size_t)L.max_partials * 8);
  L.st = take(sizeof(DevState));
  L.scal = take(16 * 8);
  // block-sparse product: a slab count per 32-row block and a list of up to
  // ld / 16 slabs each
  L.bs = take((ld / kBsM) * 4 + (ld / kBsM) * (ld / kBsK) * 4);
  L.total = o;
  return L;
}
}  // namespace

size_t ws_bytes(int n, int prec, bool rkf) { return ws_layout(n, prec, rkf).total; }

bool ws_carve(void* base, size_t bytes, int n, int prec, Ws* w, bool rkf) {
  const WsLayout L = ws_layout(n, prec, rkf);
  if (bytes < L.total) return false;
  char* b = (char*)base;
  const size_t ld = (size_t)pad_n(n);
  const size_t pl = ld * ld;
  w->n = n;
  w->ld = (int)ld;
  w->prec = prec;
  w->yn_r = (double*)(b + L.yn);
  w->yn_i = w->yn_r + pl;
  w->y1_r = (double*)(b + L.y1);
  w->y1_i = w->y1_r + pl;
  w->y2_r = (double*)(b + L.y2);
  w->y2_i = w->y2_r + pl;
  w->acc_r = (double*)(b + L.acc);
  w->acc_i = w->acc_r + 32 * 32;
  w->x_r = (double*)(b + L.x);
  w->x_i = w->x_r + pl;
  if (prec != QPR_FP64) {
    w->ra_r = (double*)(b + L.ra);
    w->ra_i = w->ra_r + pl;
    w->an_r = (double*)(b + L.an);
    w->an_i = w->an_r + pl;
    w->xf_r = (float*)(b + L.xf);
    w->xf_i = w->xf_r + pl;
    if (prec == QPR_FP32) {
      w->lo_r = (float*)(b + L.lo);
      w->lo_i = w->lo_r + pl;
      // the FP32 defect planes, in FP64 regions the FP32-state solve leaves unused
      w->dn_r = (float*)(b + L.yn);
      w->dn_i = w->dn_r + pl;
      w->d1_r = (float*)(b + L.y1);
      w->d1_i = w->d1_r + pl;
      w->d2_r = (float*)(b + L.y2);
      w->d2_i = w->d2_r + pl;
      w->dac_r = (float*)(b + L.acc);  // packed as the FP64 accumulator
      w->dac_i = w->dac_r + 32 * 32;
      w->ra32_r = (float*)(b + L.x);
      w->ra32_i = w->ra32_r + pl;
    }
    if (prec == QPR_BF16X3) w->sl = (uint16_t*)(b + L.sl);
  }
  double* pv = (double*)(b + L.pv);
  w->p_n = pv;
  w->p_1 = pv + ld;
  w->p_2 = pv + 2 * ld;
  w->p_a = pv + 3 * ld;
  if (prec == QPR_FP64 && rkf) {
    double* kf = (double*)(b + L.kf);
    const size_t pk = packed_values((int)ld);
    for (int j = 0; j < 5; ++j) {
      w->k_r[j] = kf + j * pk;
      w->k_i[j] = w->k_r[j] + 32 * 32;
    }
    w->cand_r = (double*)(b + L.cand);
    w->cand_i = w->cand_r + pl;
    w->p_c = (double*)(b + L.pc);
  }
  w->partials = (double*)(b + L.partials);
  w->max_partials = L.max_partials;
  w->st = (DevState*)(b + L.st);
  w->scal = (double*)(b + L.scal);
  w->bs_cnt = (int*)(b + L.bs);
  w->bs_idx = w->bs_cnt + ld / kBsM;
  return true;
}

// ------------------------------------------------------------- validation
static qpr_status check_problem(const qpr_problem* P) {
  if (!P) return fail(QPR_E_ARG, "problem must not be NULL");
  if (P->n < 2 || P->ld != pad_n(P->n) || !P->h_off || !P->d)
    return fail(QPR_E_ARG, "problem struct is not a built problem");
  return QPR_OK;
}

// rkf: the solve may run the Fehlberg integrator, so the workspace must hold
// its stage planes (RK4 solves and single right-hand sides do without them)
static qpr_status check_common(const qpr_problem* P, double omega, int prec, void* ws,
                               size_t ws_bytes_, Ws* w, bool rkf = false) {
  qpr_status st = check_problem(P);
  if (st != QPR_OK) return st;
  if (!(omega >= 0.0 && omega <= 1.0)) return fail(QPR_E_ARG, "omega must be in [0,1] (got %g)", omega);
  if (prec != QPR_FP64 && prec != QPR_FP32 && prec != QPR_BF16X3)
    return fail(QPR_E_ARG, "unknown precision %d", prec);
  if (!ws) return fail(QPR_E_ARG, "workspace must not be NULL");
  if (((uintptr_t)ws) % kAlign) return fail(QPR_E_ARG, "workspace must be 256-byte aligned");
  if (!ws_carve(ws, ws_bytes_, P->n, prec, w, rkf))
    return fail(QPR_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes_,
                ws_bytes(P->n, prec, rkf));
  return QPR_OK;
}

static qpr_status check_dt(const qpr_problem* P, double omega, double dt) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(QPR_E_ARG, "dt must be positive (got %g)", dt);
  const double reach = dt * ((1.0 - omega) * (P->h_hi - P->h_lo) + 2.0 * omega);
  if (reach >= kRk4Limit)
    return fail(QPR_E_UNSTABLE,
                "dt=%g outside the RK4 stability bound: dt*((1-w)*spread(H)+2w)=%.3f >= %.1f", dt,
                reach, kRk4Limit);
  return QPR_OK;
}

// ------------------------------------------------------------ one RK4 step
// Enqueue the four stages of one step on the state (yn, p_n).  `xk` selects
// the product; with a low-precision product the stage inputs are read from
// the low-precision copies the previous epilogue wrote, and `ra` (the FP64
// anchor residual) is added to every stage's right-hand side.
// Epilogue arguments of classical RK4 stage k (0..3) on the workspace: the
// stage inputs rotate y_n -> Y_1 -> Y_2 -> Y_1 and the last stage writes y_n.
static EpiArgs rk4_stage_args(const Ws& w, int k, double omega, double dt, int xk, int xs,
                              int check, int gate, bool with_ra) {
  struct Stage {
    double *inr, *ini, *pin, *outr, *outi, *pout;
    double cdt;
  };
  const Stage stages[4] = {
      {w.yn_r, w.yn_i, w.p_n, w.y1_r, w.y1_i, w.p_1, 0.5 * dt},
      {w.y1_r, w.y1_i, w.p_1, w.y2_r, w.y2_i, w.p_2, 0.5 * dt},
      {w.y2_r, w.y2_i, w.p_2, w.y1_r, w.y1_i, w.p_1, dt},
      {w.y1_r, w.y1_i, w.p_1, w.yn_r, w.yn_i, w.p_n, dt / 6.0},
  };
  const Stage& sg = stages[k];
  EpiArgs a{};
  a.xr = w.x_r;
  a.xi = w.x_i;
  a.xfr = w.xf_r;
  a.xfi = w.xf_i;
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
  a.rar = with_ra ? w.ra_r : nullptr;
  a.rai = with_ra ? w.ra_i : nullptr;
  a.lor = xk == OP_F32 ? w.lo_r : nullptr;
  a.loi = xk == OP_F32 ? w.lo_i : nullptr;
  a.slices = xk == OP_BF16X3 ? w.sl : nullptr;
  a.omega = omega;
  a.cdt = sg.cdt;
  a.mode = EPI_S1 + k;
  a.xkind = xs;
  if (xs == XS_FUSED32) {
    // no FP32 X: the X planes hold the second FP32 state copy; stage k
    // gathers from one copy and writes the other (lo at even stages), so lo
    // again holds the copy of y_n after stage 4
    float *in_r = k % 2 ? w.xf_r : w.lo_r, *in_i = k % 2 ? w.xf_i : w.lo_i;
    a.xfr = in_r;
    a.xfi = in_i;
    a.lor = k % 2 ? w.lo_r : w.xf_r;
    a.loi = k % 2 ? w.lo_i : w.xf_i;
  }
  a.check = k == 0 ? check : CHK_NONE;
  a.gate = gate;
  return a;
}

static hipError_t enqueue_step(const qpr_problem* P, const Ws& w, const ProbView& pv, double omega,
                               double dt, int xk, int cfg, int product, int check, bool with_ra,
                               hipStream_t s) {
  const int gate = check == CHK_DELTA ? 1 : 0;
  const bool sparse = use_sparse(P, product, xk);
  const int xs = x_source(P, product, xk);
  const bool fused = xs == XS_FUSED64 || xs == XS_FUSED32;
  // with the sparse product the stage-2 launch (product, or fused epilogue)
  // carries stage 1's finishing step; not a gated fused launch, whose tiles
  // would have to see the hold that step may set
  FinishJob pending{};
  for (int k = 0; k < 4; ++k) {
    const EpiArgs a = rk4_stage_args(w, k, omega, dt, xk, xs, check, gate, with_ra);
    hipError_t e = hipSuccess;
    if (!fused) {
      e = launch_product(P, w, pv, xk, cfg, sparse, a.ysr, a.ysi, gate, s, -1,
                         k == 1 ? &pending : nullptr);
      if (e != hipSuccess) return e;
    }
    const bool carry = sparse && k == 0 && !(fused && gate);
    // (pending is empty when stage 1 finished on its own: no extra workgroup)
    e = launch_epilogue(pv, a, w, s, !carry, fused && k == 1 ? &pending : nullptr);
    if (e != hipSuccess) return e;
    if (carry) pending = finish_job(pv, a, w);
  }
  return hipSuccess;
}

// L(Y) for Y in (inr, ini, pin) into (outr, outi); FP64 product unless xk says otherwise.
static hipError_t enqueue_rhs(const qpr_problem* P, const Ws& w, const ProbView& pv, double omega,
                              double* inr, double* ini, double* pin, double* outr, double* outi,
                              int xk, int cfg, int product, int check, hipStream_t s,
                              float* lor = nullptr, float* loi = nullptr) {
  const bool sparse = use_sparse(P, product, xk);
  const int xs = x_source(P, product, xk);
  if (xk != OP_F64) {
    hipError_t e = launch_to_lowp(xk, inr, ini, P->n, P->ld, w, s);
    if (e != hipSuccess) return e;
  }
  if (xs != XS_FUSED64 && xs != XS_FUSED32) {
    hipError_t e = launch_product(P, w, pv, xk, cfg, sparse, inr, ini, 0, s);
    if (e != hipSuccess) return e;
  }
  EpiArgs a{};
  a.xr = w.x_r;
  a.xi = w.x_i;
  a.xfr = w.xf_r;
  a.xfi = w.xf_i;
  a.ysr = inr;
  a.ysi = ini;
  a.ps = pin;
  a.outr = outr;
  a.outi = outi;
  a.omega = omega;
  a.mode = EPI_RHS;
  a.xkind = xs;
  if (xs == XS_FUSED32) {  // gathers from the FP32 copy of the input
    a.xfr = w.lo_r;
    a.xfi = w.lo_i;
  }
  a.lor = lor;  // also store the result rounded to FP32 (the FP32-state defect's r_a)
  a.loi = loi;
  a.check = check;
  return launch_epilogue(pv, a, w, s);
}

// Classical RK4 stage k of the defect step with the defect held in FP32
// (XS_FUSED32S): d delta/dt = r_a + L(delta), every state plane FP32 (delta_n,
// the ping-pong stage states, the accumulator, the FP32 copy of r_a); the
// stage gathers X from its FP32 input; arithmetic in FP64.  Same rotation as
// rk4_stage_args: delta_n -> D_1 -> D_2 -> D_1 -> delta_n.
EpiArgs rk4_stage_args_f32s(const Ws& w, int k, double omega, double dt, int check, int gate) {
  float* in_r[4] = {w.dn_r, w.d1_r, w.d2_r, w.d1_r};
  float* in_i[4] = {w.dn_i, w.d1_i, w.d2_i, w.d1_i};
  float* out_r[4] = {w.d1_r, w.d2_r, w.d1_r, w.dn_r};
  float* out_i[4] = {w.d1_i, w.d2_i, w.d1_i, w.dn_i};
  double* pin[4] = {w.p_n, w.p_1, w.p_2, w.p_1};
  double* pout[4] = {w.p_1, w.p_2, w.p_1, w.p_n};
  const double cdt[4] = {0.5 * dt, 0.5 * dt, dt, dt / 6.0};
  EpiArgs a{};
  a.xfr = in_r[k];  // the gathers read the FP32 stage input itself
  a.xfi = in_i[k];
  a.ysr = (const double*)in_r[k];  // FP32 planes (XS_FUSED32S reads them as such)
  a.ysi = (const double*)in_i[k];
  a.ps = pin[k];
  a.ynr = (const double*)w.dn_r;
  a.yni = (const double*)w.dn_i;
  a.accr = (double*)w.dac_r;
  a.acci = (double*)w.dac_i;
  a.outr = (double*)out_r[k];
  a.outi = (double*)out_i[k];
  a.pout = pout[k];
  a.rar = (const double*)w.ra32_r;
  a.rai = (const double*)w.ra32_i;
  a.omega = omega;
  a.cdt = cdt[k];
  a.mode = EPI_S1 + k;
  a.xkind = XS_FUSED32S;
  a.check = k == 0 ? check : CHK_NONE;
  a.gate = gate;
  return a;
}

// One RK4 step of the FP32-state defect: four fused launches (gated by the
// hold of the defect correction, so stage 1 keeps its own finishing launch).
static hipError_t enqueue_step_f32s(const ProbView& pv, const Ws& w, double omega, double dt,
                                    int check, hipStream_t s) {
  const int gate = check == CHK_DELTA ? 1 : 0;
  for (int k = 0; k < 4; ++k) {
    hipError_t e = launch_epilogue(pv, rk4_stage_args_f32s(w, k, omega, dt, check, gate), w, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Fehlberg 4(5) tableau (Supplementary Note 2, Eq. (S10)-(S12)), the two
// 4101 denominators read as 4104 (the order conditions require it).
static const double kFa[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 4, 0, 0, 0, 0},
    {3.0 / 32, 9.0 / 32, 0, 0, 0},
    {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197, 0, 0},
    {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104, 0},
    {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40},
};
static const double kFb4[6] = {25.0 / 216, 0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0};
static const double kFb5[6] = {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55};

// Stability cap for the Fehlberg fourth-order solution.  Its stability
// polynomial is R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/104 (b4 A^k 1
// from the tableau above); because of the z^5/104 term |R(i y)| > 1 for every
// y != 0 on the imaginary axis, so steps are only stable for modes with
// enough damping.  The Liouvillian's fast modes are coherences between
// eigenstates of H, eigenvalues ~ -omega + i beta with
// |beta| <= (1 - omega) 2 rho(H); the classical part lies within radius
// 2 omega.  The cap is the largest h (bisection) with |R(h z)| <= 1 on that
// set, taking half the dephasing rate as the damping, times 0.9.
double rkf_step_cap(double omega, double rho_h) {
  const double bmax = (1.0 - omega) * 2.0 * 1.02 * rho_h;
  const double gamma = 0.5 * omega;
  auto R = [](std::complex<double> z) {
    return 1.0 + z * (1.0 + z * (0.5 + z * (1.0 / 6 + z * (1.0 / 24 + z / 104.0))));
  };
  auto ok = [&](double h) {
    if (std::abs(R(std::complex<double>(-2.0 * omega * h, 0.0))) > 1.0) return false;
    for (int k = 0; k <= 2000; ++k) {
      const double b = bmax * k / 2000.0;
      if (std::abs(R(std::complex<double>(-gamma * h, b * h))) > 1.0) return false;
    }
    return true;
  };
  double lo = 0.0, hi = 4.0;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    (ok(mid) ? lo : hi) = mid;
  }
  return 0.9 * lo;
}

// One Fehlberg attempt on y = (yn, p_n): six stages (product + epilogue),
// then the commit of the candidate if the step control accepted it.
// Epilogue arguments of Fehlberg stage st (0..5) on the workspace: stage
// inputs y_n -> Y_1 -> Y_2 -> Y_1 -> Y_2 -> Y_1 (stage s + 1 reads what stage s
// wrote), K_s kept for the later stages, and the sixth stage writing the
// fourth-order candidate and the error estimate.
EpiArgs rkf_stage_args(const Ws& w, int st, double omega, int xs) {
  double* in_r[6] = {w.yn_r, w.y1_r, w.y2_r, w.y1_r, w.y2_r, w.y1_r};
  double* in_i[6] = {w.yn_i, w.y1_i, w.y2_i, w.y1_i, w.y2_i, w.y1_i};
  double* in_p[6] = {w.p_n, w.p_1, w.p_2, w.p_1, w.p_2, w.p_1};
  EpiArgs a{};
  a.xr = w.x_r;
  a.xi = w.x_i;
  a.ysr = in_r[st];
  a.ysi = in_i[st];
  a.ps = in_p[st];
  a.ynr = w.yn_r;
  a.yni = w.yn_i;
  a.omega = omega;
  a.mode = EPI_F1 + st;
  a.xkind = xs;
  a.check = st == 0 ? CHK_RKF : CHK_NONE;
  for (int j = 0; j < 5; ++j) {
    a.kr[j] = w.k_r[j];
    a.ki[j] = w.k_i[j];
  }
  if (st < 5) {
    a.kwr = w.k_r[st];
    a.kwi = w.k_i[st];
    a.outr = in_r[st + 1];
    a.outi = in_i[st + 1];
    a.pout = in_p[st + 1];
    for (int j = 0; j <= st; ++j) a.cf[j] = kFa[st + 1][j];
  } else {
    a.outr = w.cand_r;
    a.outi = w.cand_i;
    a.pout = w.p_c;
    for (int j = 0; j < 6; ++j) {
      a.cf[j] = kFb4[j];
      a.ce[j] = kFb5[j] - kFb4[j];
    }
  }
  return a;
}

// One Fehlberg attempt on y = (yn, p_n): six stages (product + epilogue),
// then the commit of the candidate if the step control accepted it.
static hipError_t enqueue_rkf_attempt(const qpr_problem* P, const Ws& w, const ProbView& pv,
                                      double omega, int cfg, int product, hipStream_t s) {
  const bool sparse = use_sparse(P, product, OP_F64);
  const int xs = x_source(P, product, OP_F64);
  const bool fused = xs == XS_FUSED64;
  FinishJob pending{};  // stage 1's finishing step rides on the stage-2 sparse launch
  for (int st = 0; st < 6; ++st) {
    const EpiArgs a = rkf_stage_args(w, st, omega, xs);
    hipError_t e = hipSuccess;
    if (!fused) {
      e = launch_product(P, w, pv, OP_F64, cfg, sparse, a.ysr, a.ysi, 0, s, -1,
                         st == 1 ? &pending : nullptr);
      if (e != hipSuccess) return e;
    }
    const bool carry = sparse && st == 0;
    e = launch_epilogue(pv, a, w, s, !carry, fused && st == 1 ? &pending : nullptr);
    if (e != hipSuccess) return e;
    if (carry) pending = finish_job(pv, a, w);
  }
  return launch_rkf_commit(w.yn_r, w.yn_i, w.p_n, w.cand_r, w.cand_i, w.p_c, P->n, P->ld, w.st, s);
}

}  // namespace qpr

using namespace qpr;

extern "C" const char* qpr_last_error(void) { return g_err; }
extern "C" const char* qpr_version(void) { return "qpr 0.1 (gfx950)"; }

extern "C" size_t qpr_workspace_bytes(int32_t n, int32_t prec, int32_t integrator) {
  if (n < 2 || (prec != QPR_FP64 && prec != QPR_FP32 && prec != QPR_BF16X3)) return 0;
  if (integrator != QPR_RK4 && integrator != QPR_RKF45) return 0;
  if (integrator == QPR_RKF45 && prec != QPR_FP64) return 0;
  return ws_bytes(n, prec, integrator == QPR_RKF45);
}

static qpr_opts default_opts() {
  qpr_opts o{};
  o.chunk = 64;
  o.use_graph = 1;
  o.fold_every = 0;
  o.renorm = 1;
  o.gemm_cfg = -1;
  o.product = QPR_PRODUCT_AUTO;
  o.integrator = QPR_RK4;
  o.step_tol = 1e-4;
  o.dt_max = 0.0;
  o.delta_state = 0;
  return o;
}

extern "C" qpr_status qpr_rhs(const qpr_problem* P, double omega, const double* rho, double* out,
                              int32_t prec, const qpr_opts* opts, void* ws, size_t wsb,
                              qpr_stream_t stream) {
  qpr_opts o = opts ? *opts : default_opts();
  clear_error();
  Ws w;
  qpr_status st = check_common(P, omega, prec, ws, wsb, &w);
  if (st != QPR_OK) return st;
  if (!rho || !out) return fail(QPR_E_ARG, "rho and out must not be NULL");
  if (rho == out) return fail(QPR_E_ARG, "rho and out must not alias");
  hipStream_t s = (hipStream_t)stream;
  ProbView pv;
  if ((st = view_for(P, o, &pv)) != QPR_OK) return st;
  if ((st = setup_product(P, w, prec, &o, s)) != QPR_OK) return st;
  QPR_HIP(launch_state_init(w.st, 0.0, 0, 0, s));
  QPR_HIP(launch_pad_in(rho, P->n, P->ld, w.y1_r, w.y1_i, w.p_1, s));
  QPR_HIP(enqueue_rhs(P, w, pv, omega, w.y1_r, w.y1_i, w.p_1, w.y2_r, w.y2_i, op_kind(prec), o.gemm_cfg,
                        o.product, CHK_NONE, s));
  QPR_HIP(launch_pad_out(w.y2_r, w.y2_i, P->n, P->ld, out, s));
  return QPR_OK;
}

extern "C" qpr_status qpr_rk4_step(const qpr_problem* P, double omega, double dt, int32_t nsteps,
                                   double* rho, int32_t prec, double* diag_out,
                                   const qpr_opts* opts, void* ws, size_t wsb,
                                   qpr_stream_t stream) {
  qpr_opts o = opts ? *opts : default_opts();
  clear_error();
  Ws w;
  qpr_status st = check_common(P, omega, prec, ws, wsb, &w);
  if (st != QPR_OK) return st;
  if (!rho) return fail(QPR_E_ARG, "rho must not be NULL");
  if (nsteps < 0) return fail(QPR_E_ARG, "nsteps must be >= 0");
  if ((st = check_dt(P, omega, dt)) != QPR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  ProbView pv;
  if ((st = view_for(P, o, &pv)) != QPR_OK) return st;
  if ((st = setup_product(P, w, prec, &o, s)) != QPR_OK) return st;
  const int xk = op_kind(prec);
  QPR_HIP(launch_state_init(w.st, 0.0, nsteps, 0, s));
  QPR_HIP(launch_pad_in(rho, P->n, P->ld, w.yn_r, w.yn_i, w.p_n, s));
  if (xk != OP_F64) QPR_HIP(launch_to_lowp(xk, w.yn_r, w.yn_i, P->n, P->ld, w, s));
  for (int k = 0; k < nsteps; ++k)
    QPR_HIP(enqueue_step(P, w, pv, omega, dt, xk, o.gemm_cfg, o.product, CHK_NONE, false, s));
  if (diag_out) {
    QPR_HIP(launch_state_stats(w.yn_r, w.yn_i, w.p_n, P->n, P->ld, w, s));
    // diag_out = [resid2, trace, herm, nonfinite]
    QPR_HIP(hipMemcpyAsync(diag_out, &w.st->resid2, 8, hipMemcpyDeviceToDevice, s));
    QPR_HIP(hipMemcpyAsync(diag_out + 1, &w.st->aux[0], 16, hipMemcpyDeviceToDevice, s));
    QPR_HIP(hipMemcpyAsync(diag_out + 3, &w.st->aux[3], 8, hipMemcpyDeviceToDevice, s));
  }
  QPR_HIP(launch_pad_out(w.yn_r, w.yn_i, P->n, P->ld, rho, s));
  return QPR_OK;
}

namespace {

// Run chunks of `chunk` steps (eager or as a replayed graph) until the device
// control block says stop.  Returns the final host copy of the block.  With
// `alt` set, each chunk is either enqueue_chunk or alt->enqueue, as
// alt->choose() says just before it is launched (both captured once).
struct AltChunk {
  std::function<hipError_t(hipStream_t)> enqueue;
  std::function<bool()> choose;
};
// `pinned` is two pinned host copies of the control block (a worker of a
// concurrent solve passes the pair it owns for all its systems); NULL: this
// call allocates its own (hipHostFree synchronises the device, so a worker
// must not pay it per system).
qpr_status run_chunks(const std::function<hipError_t(hipStream_t)>& enqueue_chunk,
                      DevState* dev_st, bool use_graph, hipStream_t s, DevState* final_state,
                      long long* chunks_run, const AltChunk* alt = nullptr,
                      DevState* pinned = nullptr) {
  HostPinned own;
  if (!pinned) {
    if (hipHostMalloc(&own.h, 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess)
      return fail(QPR_E_HIP, "hipHostMalloc of the control-block copies failed");
    pinned = (DevState*)own.h;
  }
  DevState* hs = pinned;
  hipGraphExec_t exec = nullptr, exec_alt = nullptr;
  hipGraph_t graph = nullptr, graph_alt = nullptr;
  hipStream_t cs = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  qpr_status rc = QPR_OK;
  auto cleanup = [&]() {
    // nothing of this call may still be in flight (copies into `pinned`)
    (void)hipStreamSynchronize(s);
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (exec_alt) hipGraphExecDestroy(exec_alt);
    if (graph_alt) hipGraphDestroy(graph_alt);
    if (cs) hipStreamDestroy(cs);
    for (auto& e : ev)
      if (e) hipEventDestroy(e);
  };
#define QPR_HIP_C(call)                                                                 \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      rc = fail(QPR_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));              \
      cleanup();                                                                        \
      return rc;                                                                        \
    }                                                                                   \
  } while (0)
  if (use_graph) {
    QPR_HIP_C(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    QPR_HIP_C(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_chunk(cs);
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    QPR_HIP_C(e);
    QPR_HIP_C(e2);
    QPR_HIP_C(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    if (alt) {
      QPR_HIP_C(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      hipError_t ea = alt->enqueue(cs);
      hipError_t ea2 = hipStreamEndCapture(cs, &graph_alt);
      QPR_HIP_C(ea);
      QPR_HIP_C(ea2);
      QPR_HIP_C(hipGraphInstantiate(&exec_alt, graph_alt, nullptr, nullptr, 0));
    }
  }
  QPR_HIP_C(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  QPR_HIP_C(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  auto launch = [&](int slot) -> hipError_t {
    const bool a = alt && alt->choose();
    hipError_t e = use_graph ? hipGraphLaunch(a ? exec_alt : exec, s)
                             : (a ? alt->enqueue(s) : enqueue_chunk(s));
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&hs[slot], dev_st, sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipEventRecord(ev[slot], s);
  };
  long long c = 0;
  QPR_HIP_C(launch(0));
  for (;;) {
    QPR_HIP_C(launch((int)((c + 1) & 1)));  // keep one chunk in flight
    QPR_HIP_C(hipEventSynchronize(ev[c & 1]));
    const DevState cur = hs[c & 1];
    ++c;
    if (cur.stop) break;
  }
  QPR_HIP_C(hipStreamSynchronize(s));
  *final_state = hs[c & 1];  // state after the in-flight chunk (a no-op once stopped)
  *chunks_run = c + 1;
  cleanup();
#undef QPR_HIP_C
  return QPR_OK;
}

}  // namespace

// Systems of a qpr_steady_state_many call not yet finished, and its workers:
// min of the two is how many run at once.
struct Concurrency {
  std::atomic<int> remaining{0};
  int workers = 1;
  int in_flight() const {
    return std::min(remaining.load(std::memory_order_relaxed), workers);
  }
};

// The single-system solve.  `conc` is NULL for a lone solve; in a concurrent
// call, while two or more systems run, the FP64 stages that AUTO gives the
// two-kernel sparse stage take the fused epilogue instead (bitwise the same
// sums; with the other systems' kernels beside it, the one launch per stage
// is the faster one), and a system left running alone goes back to the two
// kernels.
static qpr_status steady_state_impl(const qpr_problem* P, double omega, double dt, double tol,
                                    int64_t max_steps, int32_t prec, double* rho, int32_t* rank,
                                    qpr_stats* stats, const qpr_opts* opts, void* ws, size_t wsb,
                                    qpr_stream_t stream, const Concurrency* conc,
                                    DevState* pinned = nullptr) {
  const auto t0 = std::chrono::steady_clock::now();
  clear_error();
  qpr_opts o = opts ? *opts : default_opts();
  if (o.integrator != QPR_RK4 && o.integrator != QPR_RKF45)
    return fail(QPR_E_ARG, "unknown integrator %d", o.integrator);
  Ws w;
  qpr_status st = check_common(P, omega, prec, ws, wsb, &w, o.integrator == QPR_RKF45);
  if (st != QPR_OK) return st;
  if (!rho) return fail(QPR_E_ARG, "rho must not be NULL");
  if (!(tol > 0.0)) return fail(QPR_E_ARG, "tol must be positive (got %g)", tol);
  if (max_steps < 0) return fail(QPR_E_ARG, "max_steps must be >= 0");
  if (o.integrator == QPR_RKF45) {
    if (!(dt > 0.0)) return fail(QPR_E_ARG, "dt must be positive (got %g)", dt);
  } else if ((st = check_dt(P, omega, dt)) != QPR_OK) {
    return st;
  }
  if (o.chunk <= 0) o.chunk = 64;
  if (o.fold_every <= 0) o.fold_every = o.chunk;
  hipStream_t s = (hipStream_t)stream;
  ProbView pv;
  if ((st = view_for(P, o, &pv)) != QPR_OK) return st;
  if ((st = setup_product(P, w, prec, &o, s)) != QPR_OK) return st;
  const int n = P->n, ld = P->ld;
  qpr_stats S{};
  qpr_status result = QPR_OK;
  const bool switch_fused = conc && conc->workers >= 2 && o.product == QPR_PRODUCT_AUTO &&
                            x_source(P, o.product, OP_F64) == XS_SPARSE64;
  const int product = o.product;
  AltChunk alt;
  const AltChunk* altp = nullptr;
  auto set_alt = [&](std::function<hipError_t(hipStream_t)> f) {
    if (!switch_fused) return;
    alt.enqueue = std::move(f);
    alt.choose = [conc]() { return conc->in_flight() >= 2; };
    altp = &alt;
  };

  const bool graph = o.use_graph != 0;
  DevState fs{};
  long long chunks = 0;
  double* out_r = w.yn_r;
  double* out_i = w.yn_i;
  double* out_p = w.p_n;
  if (o.integrator == QPR_RKF45) {
    if (prec != QPR_FP64) return fail(QPR_E_ARG, "the RKF45 integrator runs in FP64 only");
    if (!(o.step_tol > 0.0)) return fail(QPR_E_ARG, "step_tol must be positive");
    double hmax = o.dt_max;
    if (!(hmax > 0.0)) hmax = rkf_step_cap(omega, P->h_norm);
    if (!(hmax > 0.0)) return fail(QPR_E_UNSTABLE, "no stable Fehlberg step at omega=%g", omega);
    QPR_HIP(launch_state_init(w.st, tol, max_steps, CHK_RKF, s));
    QPR_HIP(launch_state_rkf(w.st, std::min(dt, hmax), hmax, o.step_tol, s));
    QPR_HIP(launch_pad_in(rho, n, ld, w.yn_r, w.yn_i, w.p_n, s));
    auto chunk_of = [&](int pr) {
      return [&, pr](hipStream_t q) -> hipError_t {
        for (int k = 0; k < o.chunk; ++k) {
          hipError_t e = enqueue_rkf_attempt(P, w, pv, omega, o.gemm_cfg, pr, q);
          if (e != hipSuccess) return e;
        }
        return hipSuccess;
      };
    };
    set_alt(chunk_of(QPR_PRODUCT_FUSED));
    st = run_chunks(chunk_of(product), w.st, graph, s, &fs, &chunks, altp, pinned);
    if (st != QPR_OK) return st;
    S.steps = fs.accepted;
    S.rejected = fs.rejected;
    S.rhs_evals = 6 * (fs.accepted + fs.rejected) + 1;
    S.rhs_evals_fp64 = S.rhs_evals;
    S.residual = std::sqrt(fs.resid2);
    S.last_step = fs.h;
  } else if (prec == QPR_FP64) {
    QPR_HIP(launch_state_init(w.st, tol, max_steps, CHK_PLAIN, s));
    QPR_HIP(launch_pad_in(rho, n, ld, w.yn_r, w.yn_i, w.p_n, s));
    auto chunk_of = [&](int pr) {
      return [&, pr](hipStream_t q) -> hipError_t {
        for (int k = 0; k < o.chunk; ++k) {
          hipError_t e =
              enqueue_step(P, w, pv, omega, dt, OP_F64, o.gemm_cfg, pr, CHK_PLAIN, false, q);
          if (e != hipSuccess) return e;
        }
        return hipSuccess;
      };
    };
    set_alt(chunk_of(QPR_PRODUCT_FUSED));
    st = run_chunks(chunk_of(product), w.st, graph, s, &fs, &chunks, altp, pinned);
    if (st != QPR_OK) return st;
    S.steps = fs.converged ? fs.conv_step : fs.step;
    S.rhs_evals = 4 * S.steps + 1;
    S.rhs_evals_fp64 = S.rhs_evals;
    S.residual = std::sqrt(fs.resid2);
  } else {
    // Defect correction: anchor rho_a (FP64) with residual r_a = L(rho_a) in
    // FP64; delta follows d delta/dt = r_a + L_lowp(delta) from delta = 0 and
    // is folded into the anchor every fold_every steps (or as soon as the
    // running estimate meets the tolerance), after which r_a is recomputed in
    // FP64 and judged.
    const int xk = op_kind(prec);
    out_r = w.an_r;
    out_i = w.an_i;
    out_p = w.p_a;
    const size_t plane = (size_t)ld * ld;
    // Where the defect is stored: FP32 (every state plane of the steps single
    // precision, half the bytes per stage) by default wherever the FP32 steps
    // take the fused sparse stage, else FP64 (the stage writes an FP32 copy
    // of its output for the next product).
    const bool sparse32 = xk == OP_F32 && use_sparse(P, product, OP_F32);
    if (o.delta_state < 0 || o.delta_state > 2)
      return fail(QPR_E_ARG, "delta_state must be 0, 1 or 2 (got %d)", o.delta_state);
    if (o.delta_state == 2 && !sparse32)
      return fail(QPR_E_ARG, "an FP32 defect needs prec QPR_FP32 with the sparse product");
    const bool state32 =
        o.delta_state == 2 || (o.delta_state == 0 && sparse32 && product == QPR_PRODUCT_AUTO);
    if (state32) {
      auto reset32 = [&](hipStream_t q) -> hipError_t {
        hipError_t e = launch_fill(w.dn_r, 2 * plane * 4, q);
        if (e == hipSuccess) e = launch_fill(w.p_n, (size_t)ld * 8, q);
        return e;
      };
      // fold the FP32 defect into the FP64 anchor, renormalise, judge in FP64
      // (fused sparse stage) and keep r_a in FP64 and as the FP32 copy the
      // steps add
      auto fold_judge32 = [&](hipStream_t q, bool first) -> hipError_t {
        hipError_t e = hipSuccess;
        if (!first)
          e = launch_axpy_planes_f32(w.an_r, w.an_i, w.dn_r, w.dn_i, 1.0, n, ld, w.p_a, w.st, q);
        if (e == hipSuccess && o.renorm) e = launch_trace(w.p_a, n, w.st, q);
        if (e == hipSuccess && o.renorm) e = launch_scale_planes(w.an_r, w.an_i, w.p_a, n, ld, w.st, q);
        if (e == hipSuccess)
          e = enqueue_rhs(P, w, pv, omega, w.an_r, w.an_i, w.p_a, w.ra_r, w.ra_i, OP_F64,
                          o.gemm_cfg, QPR_PRODUCT_FUSED, CHK_JUDGE, q, w.ra32_r, w.ra32_i);
        if (e == hipSuccess) e = reset32(q);
        return e;
      };
      QPR_HIP(launch_state_init(w.st, tol, max_steps, CHK_DELTA, s));
      QPR_HIP(launch_pad_in(rho, n, ld, w.an_r, w.an_i, w.p_a, s));
      QPR_HIP(fold_judge32(s, true));
      auto chunk32 = [&](hipStream_t q) -> hipError_t {
        for (int k = 0; k < o.fold_every; ++k) {
          hipError_t e = enqueue_step_f32s(pv, w, omega, dt, CHK_DELTA, q);
          if (e != hipSuccess) return e;
        }
        return fold_judge32(q, false);
      };
      st = run_chunks(chunk32, w.st, graph, s, &fs, &chunks, nullptr, pinned);
      if (st != QPR_OK) return st;
      S.steps = fs.converged ? fs.conv_step : fs.step;
      S.folds = fs.folds;
      S.rhs_evals_fp64 = fs.folds;
      S.rhs_evals = 4 * S.steps + fs.folds;
      S.residual = std::sqrt(fs.judge2);
    } else {
    auto reset_delta = [&](hipStream_t q) -> hipError_t {
      hipError_t e = launch_fill(w.yn_r, 2 * plane * 8, q);
      if (e == hipSuccess) e = launch_fill(w.p_n, (size_t)ld * 8, q);
      if (e == hipSuccess && xk == OP_F32) e = launch_fill(w.lo_r, 2 * plane * 4, q);
      if (e == hipSuccess && xk == OP_BF16X3) e = launch_fill(w.sl, 6 * plane * 2, q);
      return e;
    };
    auto fold_judge = [&](hipStream_t q, bool first, int pr) -> hipError_t {
      hipError_t e = hipSuccess;
      if (!first) e = launch_axpy_planes(w.an_r, w.an_i, w.yn_r, w.yn_i, 1.0, n, ld, w.p_a, w.st, q);
      if (e == hipSuccess && o.renorm) e = launch_trace(w.p_a, n, w.st, q);
      if (e == hipSuccess && o.renorm) e = launch_scale_planes(w.an_r, w.an_i, w.p_a, n, ld, w.st, q);
      if (e == hipSuccess)
        e = enqueue_rhs(P, w, pv, omega, w.an_r, w.an_i, w.p_a, w.ra_r, w.ra_i, OP_F64,
                        o.gemm_cfg, pr, CHK_JUDGE, q);
      if (e == hipSuccess) e = reset_delta(q);
      return e;
    };
    QPR_HIP(launch_state_init(w.st, tol, max_steps, CHK_DELTA, s));
    QPR_HIP(launch_pad_in(rho, n, ld, w.an_r, w.an_i, w.p_a, s));
    QPR_HIP(fold_judge(s, true, product));
    auto chunk_of = [&](int pr) {
      return [&, pr](hipStream_t q) -> hipError_t {
        for (int k = 0; k < o.fold_every; ++k) {
          hipError_t e =
              enqueue_step(P, w, pv, omega, dt, xk, o.gemm_cfg, pr, CHK_DELTA, true, q);
          if (e != hipSuccess) return e;
        }
        return fold_judge(q, false, pr);
      };
    };
    set_alt(chunk_of(QPR_PRODUCT_FUSED));
    st = run_chunks(chunk_of(product), w.st, graph, s, &fs, &chunks, altp, pinned);
    if (st != QPR_OK) return st;
    S.steps = fs.converged ? fs.conv_step : fs.step;
    S.folds = fs.folds;
    S.rhs_evals_fp64 = fs.folds;
    S.rhs_evals = 4 * S.steps + fs.folds;
    S.residual = std::sqrt(fs.judge2);
    }
  }
  S.converged = fs.converged;
  if (fs.nonfinite) result = fail(QPR_E_NONFINITE, "non-finite value in the state or L(rho)");
  else if (!fs.converged)
    result = fail(QPR_E_NOT_CONVERGED, "not converged after %lld steps (residual %.3e)",
                  (long long)S.steps, S.residual);

  if (result == QPR_OK || result == QPR_E_NOT_CONVERGED) {
    QPR_HIP(launch_state_stats(out_r, out_i, out_p, n, ld, w, s));
    DevState hs{};
    QPR_HIP(hipMemcpyAsync(&hs, w.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    QPR_HIP(launch_pad_out(out_r, out_i, n, ld, rho, s));
    if (rank && result == QPR_OK) QPR_HIP(launch_rank(n, out_p, rank, s));
    QPR_HIP(hipStreamSynchronize(s));
    S.trace_err = std::fabs(hs.aux[0] - 1.0);
    S.herm_err = hs.aux[1];
    S.min_diag = hs.aux[2];
  }
  S.t = o.integrator == QPR_RKF45 ? fs.t : (double)S.steps * dt;
  S.status = result;
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = S;
  return result;
}

extern "C" qpr_status qpr_steady_state(const qpr_problem* P, double omega, double dt, double tol,
                                       int64_t max_steps, int32_t prec, double* rho, int32_t* rank,
                                       qpr_stats* stats, const qpr_opts* opts, void* ws,
                                       size_t wsb, qpr_stream_t stream) {
  return steady_state_impl(P, omega, dt, tol, max_steps, prec, rho, rank, stats, opts, ws, wsb,
                           stream, nullptr);
}

// A pool of host threads: worker w solves on streams[w] with workspace ws[w],
// each taking the next unsolved system (index order) until none is left; the
// calling thread waits for all of them.  Error messages live in thread-local
// storage, so each worker copies its own out.
qpr_status qpr::run_many(int count, const qpr_problem* const* probs, const double* omegas,
                         double dt, double tol, int64_t max_steps, int prec, double* const* rhos,
                         int32_t* const* ranks, qpr_stats* stats, const qpr_opts* opts,
                         int nworkers, void* const* ws, const size_t* wsb,
                         const qpr_stream_t* streams) {
  if (count < 1) return fail(QPR_E_ARG, "count must be >= 1 (got %d)", count);
  if (nworkers < 1 || nworkers > kMaxWorkers)
    return fail(QPR_E_ARG, "nworkers must be in [1, %d] (got %d)", kMaxWorkers, nworkers);
  if (!probs || !omegas || !rhos || !ws || !wsb || !streams)
    return fail(QPR_E_ARG, "probs, omegas, rhos, ws, ws_bytes and streams must not be NULL");
  for (int w = 0; w < nworkers; ++w)
    for (int j = 0; j < w; ++j)
      if (streams[j] == streams[w]) return fail(QPR_E_ARG, "workers %d and %d share a stream", j, w);
  int nmax = 0;
  for (int k = 0; k < count; ++k) {
    if (!probs[k]) return fail(QPR_E_ARG, "probs[%d] is NULL", k);
    nmax = std::max(nmax, probs[k]->n);
  }
  const size_t need =
      qpr_workspace_bytes(nmax, prec, opts ? opts->integrator : (int32_t)QPR_RK4);
  if (need == 0) return fail(QPR_E_ARG, "invalid problem size %d or precision %d", nmax, prec);
  for (int w = 0; w < nworkers; ++w)
    if (!ws[w] || wsb[w] < need)
      return fail(QPR_E_WORKSPACE, "workspace %d has %zu bytes, the largest system needs %zu", w,
                  ws[w] ? wsb[w] : (size_t)0, need);
  nworkers = std::min(nworkers, count);
  int dev = 0;
  QPR_HIP(hipGetDevice(&dev));
  std::vector<qpr_status> status(count, QPR_OK);
  std::vector<std::string> msg(count);
  std::vector<qpr_stats> local(count);
  Concurrency conc;
  conc.remaining.store(count);
  conc.workers = nworkers;
  std::atomic<int> next(0);
  Progress progress("concurrent batch");
  auto work = [&](int w) {
    bool dev_ok = hipSetDevice(dev) == hipSuccess;
    // this worker's pinned control-block copies, for all of its systems
    HostPinned pin;
    if (dev_ok && hipHostMalloc(&pin.h, 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess)
      pin.h = nullptr;
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= count) break;
      if (!dev_ok || !pin.h) {
        status[k] = QPR_E_HIP;
        msg[k] = dev_ok ? "hipHostMalloc of the control-block copies failed in the worker thread"
                        : "hipSetDevice failed in the worker thread";
      } else {
        status[k] = steady_state_impl(probs[k], omegas[k], dt, tol, max_steps, prec, rhos[k],
                                      ranks ? ranks[k] : nullptr, &local[k], opts, ws[w], wsb[w],
                                      streams[w], &conc, (DevState*)pin.h);
        if (status[k] != QPR_OK) msg[k] = qpr_last_error();
      }
      const int left = conc.remaining.fetch_sub(1, std::memory_order_relaxed) - 1;
      local[k].status = status[k];
      progress.report(count - left, count, "solved");
    }
  };
  // a worker that cannot be started runs on the calling thread
  std::vector<std::thread> threads;
  std::vector<int> here;
  threads.reserve(nworkers);
  for (int w = 0; w < nworkers; ++w) {
    try {
      threads.emplace_back(work, w);
    } catch (const std::system_error&) {
      here.push_back(w);
    }
  }
  for (int w : here) work(w);
  for (auto& t : threads) t.join();
  if (stats)
    for (int k = 0; k < count; ++k) stats[k] = local[k];
  for (int k = 0; k < count; ++k)
    if (status[k] != QPR_OK) return fail(status[k], "system %d: %s", k, msg[k].c_str());
  return QPR_OK;
}

extern "C" qpr_status qpr_steady_state_many(int32_t count, const qpr_problem* const* probs,
                                            const double* omegas, double dt, double tol,
                                            int64_t max_steps, int32_t prec, double* const* rhos,
                                            int32_t* const* ranks, qpr_stats* stats,
                                            const qpr_opts* opts, int32_t nworkers,
                                            void* const* ws, const size_t* wsb,
                                            const qpr_stream_t* streams) {
  clear_error();
  return run_many(count, probs, omegas, dt, tol, max_steps, prec, rhos, ranks, stats, opts,
                  nworkers, ws, wsb, streams);
}

extern "C" qpr_status qpr_hub_counts(int32_t n, const double* p, double c, int32_t* counts,
                                      qpr_stream_t stream) {
  clear_error();
  if (n < 1) return fail(QPR_E_ARG, "n must be >= 1");
  if (!p || !counts) return fail(QPR_E_ARG, "p and counts must not be NULL");
  if (!(c > 1.0)) return fail(QPR_E_ARG, "c must be > 1 (got %g)", c);
  QPR_HIP(launch_hubs(n, p, c, counts, (hipStream_t)stream));
  return QPR_OK;
}

extern "C" qpr_status qpr_rank(int32_t n, const double* p, int32_t* order, qpr_stream_t stream) {
  clear_error();
  if (n < 1) return fail(QPR_E_ARG, "n must be >= 1");
  if (!p || !order) return fail(QPR_E_ARG, "p and order must not be NULL");
  QPR_HIP(launch_rank(n, p, order, (hipStream_t)stream));
  return QPR_OK;
}

extern "C" qpr_status qpr_time_kernels(const qpr_problem* P, double omega, int32_t prec,
                                       int32_t cfg, int32_t reps, const double* rho,
                                       double* ms_out, void* ws, size_t wsb,
                                       qpr_stream_t stream) {
  clear_error();
  Ws w;
  qpr_status st = check_common(P, omega, prec, ws, wsb, &w);
  if (st != QPR_OK) return st;
  if (!rho || !ms_out) return fail(QPR_E_ARG, "rho and ms_out must not be NULL");
  if (reps < 1) return fail(QPR_E_ARG, "reps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  const ProbView pv = view_of(P);
  const int xk = op_kind(prec);
  // tol 0 and an unreachable step budget: stage 1 runs its reductions and the
  // control block never stops the launches
  QPR_HIP(launch_state_init(w.st, 0.0, 1ll << 60, CHK_PLAIN, s));
  QPR_HIP(launch_pad_in(rho, P->n, P->ld, w.y1_r, w.y1_i, w.p_1, s));
  QPR_HIP(launch_pad_in(rho, P->n, P->ld, w.yn_r, w.yn_i, w.p_n, s));
  QPR_HIP(launch_fill(w.acc_r, packed_values(P->ld) * 8, s));
  if (xk != OP_F64) QPR_HIP(launch_to_lowp(xk, w.y1_r, w.y1_i, P->n, P->ld, w, s));
  // cfg = -2: time the sparse product (default variant) instead; cfg = -3 - v: sparse variant v;
  // v = nvar (the number of variants): the fused epilogue (no product launch);
  // v = nvar + 1: the block-sparse MFMA product; v = nvar + 2 (QPR_FP32): the
  // fused stages of the FP32-state defect (no product launch)
  const int nvar = spmm_num_variants();
  const int spv = cfg <= -3 ? -3 - cfg : -1;
  if (spv > nvar + 2) return fail(QPR_E_ARG, "no such sparse-product variant");
  const bool bsp = spv == nvar + 1;
  const bool f32s = spv == nvar + 2;
  if (bsp && xk == OP_BF16X3) return fail(QPR_E_ARG, "no block-sparse bf16 product");
  if (f32s && xk != OP_F32) return fail(QPR_E_ARG, "the FP32-state stages need QPR_FP32");
  const bool sparse = cfg <= -2 && xk != OP_BF16X3 && !bsp;
  const bool fused = sparse && (spv == nvar || f32s);
  if (bsp) {
    QPR_HIP(launch_block_pattern(P, w, s));
    cfg = kCfgBlockSparse;
  }
  const int xs = f32s ? XS_FUSED32S
                      : fused ? (xk == OP_F64 ? XS_FUSED64 : XS_FUSED32)
                              : xk != OP_F64 ? XS_DENSE32 : sparse ? XS_SPARSE64 : XS_DENSE64;
  // the FP32 fused stages gather from both FP32 copies in turn (the X planes
  // hold the second one)
  if (fused && xk == OP_F32 && !f32s)
    QPR_HIP(launch_fill(w.xf_r, 2 * (size_t)P->ld * P->ld * 4, s));
  if (f32s) {  // FP32 state planes: the operand (as the FP32 copy) and zeros
    const size_t pl4 = 2 * (size_t)P->ld * P->ld * 4;
    QPR_HIP(launch_to_lowp(OP_F32, w.y1_r, w.y1_i, P->n, P->ld, w, s));
    QPR_HIP(launch_fill(w.dac_r, packed_values(P->ld) * 4, s));
    QPR_HIP(launch_fill(w.ra32_r, pl4, s));
    QPR_HIP(hipMemcpyAsync(w.dn_r, w.lo_r, pl4, hipMemcpyDeviceToDevice, s));
    QPR_HIP(hipMemcpyAsync(w.d1_r, w.lo_r, pl4, hipMemcpyDeviceToDevice, s));
    QPR_HIP(hipMemcpyAsync(w.d2_r, w.lo_r, pl4, hipMemcpyDeviceToDevice, s));
  }
  HipEvent evh[3];
  for (auto& e : evh) QPR_HIP(hipEventCreate(&e.h));
  hipEvent_t ev[3] = {evh[0].h, evh[1].h, evh[2].h};
  auto product = [&]() {
    return fused ? hipSuccess : launch_product(P, w, pv, xk, cfg, sparse, w.y1_r, w.y1_i, 0, s, spv);
  };
  for (int r = 0; r < 3; ++r) QPR_HIP(product());
  QPR_HIP(hipEventRecord(ev[0], s));
  for (int r = 0; r < reps; ++r) QPR_HIP(product());
  QPR_HIP(hipEventRecord(ev[1], s));
  // the epilogues of `reps` RK4 steps with dt = 0.01 (X held fixed); stage 1
  // computes its reductions, the finishing kernel that folds them is not timed
  for (int r = 0; r < reps; ++r)
    for (int k = 0; k < 4; ++k)
      QPR_HIP(launch_epilogue(pv,
                              f32s ? rk4_stage_args_f32s(w, k, omega, 0.01, CHK_PLAIN, 0)
                                   : rk4_stage_args(w, k, omega, 0.01, xk, xs, CHK_PLAIN, 0, false),
                              w, s, false));
  QPR_HIP(hipEventRecord(ev[2], s));
  QPR_HIP(hipEventSynchronize(ev[2]));
  float t0 = 0.f, t1 = 0.f;
  QPR_HIP(hipEventElapsedTime(&t0, ev[0], ev[1]));
  QPR_HIP(hipEventElapsedTime(&t1, ev[1], ev[2]));
  ms_out[0] = (double)t0 / reps;
  ms_out[1] = (double)t1 / (4.0 * reps);
  return QPR_OK;
}

static bool known_prec(int32_t prec) {
  return prec == QPR_FP64 || prec == QPR_FP32 || prec == QPR_BF16X3;
}

extern "C" int32_t qpr_product_configs(int32_t prec) {
  return known_prec(prec) ? gemm_num_cfgs(op_kind(prec)) : 0;
}

extern "C" int32_t qpr_sparse_variants(void) { return spmm_num_variants(); }

extern "C" const char* qpr_sparse_variant_name(int32_t v) { return spmm_variant_name(v); }

extern "C" const char* qpr_product_config_name(int32_t prec, int32_t cfg) {
  return known_prec(prec) ? gemm_cfg_name(op_kind(prec), cfg) : "?";
}

extern "C" qpr_status qpr_autotune(const qpr_problem* P, int32_t prec, int32_t reps,
                                   const char* cache_path, int32_t* best_cfg, double* us_out,
                                   void* ws, size_t wsb, qpr_stream_t stream) {
  clear_error();
  Ws w;
  qpr_status st = check_common(P, 0.5, prec, ws, wsb, &w);
  if (st != QPR_OK) return st;
  if (reps < 1) return fail(QPR_E_ARG, "reps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  const int xk = op_kind(prec);
  const int ncfg = gemm_num_cfgs(xk);
  const size_t plane = (size_t)P->ld * P->ld;
  QPR_HIP(launch_state_init(w.st, 0.0, 0, CHK_NONE, s));
  QPR_HIP(launch_fill(w.y1_r, 2 * plane * 8, s));
  if (xk == OP_F32) QPR_HIP(launch_fill(w.lo_r, 2 * plane * 4, s));
  if (xk == OP_BF16X3) QPR_HIP(launch_fill(w.sl, 6 * plane * 2, s));
  HipEvent ev0, ev1;
  QPR_HIP(hipEventCreate(&ev0.h));
  QPR_HIP(hipEventCreate(&ev1.h));
  hipEvent_t e0 = ev0.h, e1 = ev1.h;
  int best = -1;
  double best_us = 1e300;
  for (int c = 0; c < ncfg; ++c) {
    double us = -1.0;
    // a configuration whose tile does not divide ld cannot run at this size
    if (gemm_cfg_fits(xk, c, P->ld)) {
      QPR_HIP(launch_gemm(xk, c, P, w, w.y1_r, w.y1_i, 0, s));
      QPR_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) QPR_HIP(launch_gemm(xk, c, P, w, w.y1_r, w.y1_i, 0, s));
      QPR_HIP(hipEventRecord(e1, s));
      QPR_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      QPR_HIP(hipEventElapsedTime(&ms, e0, e1));
      us = 1e3 * (double)ms / reps;
      if (us < best_us) {
        best_us = us;
        best = c;
      }
    }
    if (us_out) us_out[c] = us;
  }
  if (best < 0) return fail(QPR_E_HIP, "no product configuration ran");
  gemm_set_tuned(xk, P->ld, best);
  if (best_cfg) *best_cfg = best;
  // FP64: also the sparse-product variant and the form of a lone solve's
  // sparse stage (product + epilogue, or the fused epilogue), timed as RK4
  // steps (the four stage epilogues, finishing steps not included)
  int sv = -1, fused = -1;
  double sv_us = 0.0, stage_us[2] = {0.0, 0.0};
  if (xk == OP_F64) {
    const ProbView pv = view_of(P);
    auto time_us = [&](const std::function<hipError_t()>& f, double* us) -> qpr_status {
      QPR_HIP(f());
      QPR_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) QPR_HIP(f());
      QPR_HIP(hipEventRecord(e1, s));
      QPR_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      QPR_HIP(hipEventElapsedTime(&ms, e0, e1));
      *us = 1e3 * (double)ms / reps;
      return QPR_OK;
    };
    QPR_HIP(launch_fill(w.acc_r, packed_values(P->ld) * 8, s));
    QPR_HIP(launch_fill(w.yn_r, 2 * plane * 8, s));
    double best_v = 1e300;
    for (int v = 0; v < spmm_num_variants(); ++v) {
      double us = 0.0;
      st = time_us([&]() { return launch_spmm(pv, w.y1_r, w.y1_i, w.x_r, w.x_i, w.st, 0, s, v); },
                   &us);
      if (st != QPR_OK) return st;
      if (us < best_v) {
        best_v = us;
        sv = v;
      }
    }
    sv_us = best_v;
    for (int form = 0; form < 2; ++form) {
      const int xs = form ? XS_FUSED64 : XS_SPARSE64;
      st = time_us(
          [&]() -> hipError_t {
            for (int k = 0; k < 4; ++k) {
              const EpiArgs a = rk4_stage_args(w, k, 0.5, 0.01, OP_F64, xs, CHK_NONE, 0, false);
              if (!form) {
                hipError_t e = launch_spmm(pv, a.ysr, a.ysi, w.x_r, w.x_i, w.st, 0, s, sv);
                if (e != hipSuccess) return e;
              }
              hipError_t e = launch_epilogue(pv, a, w, s, false);
              if (e != hipSuccess) return e;
            }
            return hipSuccess;
          },
          &stage_us[form]);
      if (st != QPR_OK) return st;
    }
    fused = stage_us[1] < stage_us[0] ? 1 : 0;
    gemm_set_tuned(kTuneSparseVariant, P->ld, sv);
    gemm_set_tuned(kTuneFusedStage, P->ld, fused);
  }
  if (cache_path && cache_path[0]) {
    FILE* f = fopen(cache_path, "a");
    if (!f) return fail(QPR_E_ARG, "cannot open tuning cache %s", cache_path);
    fprintf(f, "%d %d %d %.3f %s\n", prec, P->ld, best, best_us, gemm_cfg_name(xk, best));
    if (sv >= 0) {
      fprintf(f, "%d %d %d %.3f %s\n", kTuneSparseVariant, P->ld, sv, sv_us, spmm_variant_name(sv));
      fprintf(f, "%d %d %d %.3f %s\n", kTuneFusedStage, P->ld, fused, stage_us[fused] / 4.0,
              fused ? "fused_epilogue" : "product+epilogue");
    }
    fclose(f);
  }
  return QPR_OK;
}

extern "C" qpr_status qpr_load_tuning(const char* cache_path) {
  clear_error();
  if (!cache_path) return fail(QPR_E_ARG, "cache_path must not be NULL");
  FILE* f = fopen(cache_path, "r");
  if (!f) return fail(QPR_E_ARG, "cannot open tuning cache %s", cache_path);
  int prec, ld, cfg;
  double us;
  char name[128];
  int loaded = 0;
  while (fscanf(f, "%d %d %d %lf %127s", &prec, &ld, &cfg, &us, name) == 5) {
    if (ld <= 0 || ld % kPad != 0) continue;
    if (prec == kTuneSparseVariant || prec == kTuneFusedStage) {
      const bool ok = prec == kTuneSparseVariant ? cfg >= 0 && cfg < spmm_num_variants()
                                                 : cfg == 0 || cfg == 1;
      if (ok) {
        gemm_set_tuned(prec, ld, cfg);
        ++loaded;
      }
      continue;
    }
    if (prec != QPR_FP64 && prec != QPR_FP32 && prec != QPR_BF16X3) continue;
    const int xk = op_kind(prec);
    if (cfg >= 0 && cfg < gemm_num_cfgs(xk)) {
      gemm_set_tuned(xk, ld, cfg);  // later lines win
      ++loaded;
    }
  }
  fclose(f);
  return loaded > 0 ? QPR_OK : fail(QPR_E_ARG, "no entries in tuning cache %s", cache_path);
}

// ------------------------------------------------- no-allocation RK4 steps
// qpr_rk4_step_noalloc: qpr_rk4_step with its workspace in a file-scope
// device array instead of a caller buffer, for callers that cannot allocate
// (graph capture, tight serving loops).  FP64 products only, n <= 1024: the
// workspace of an FP64 RK4 call at n = 1024 (y_n, two stage states and X,
// 2 x 1024^2 doubles each, the tile-pair packed accumulator, the diagonals,
// partials, slab lists and control block) is 75,834,112 bytes.  Every GPU the library runs on
// holds one such array for the life of the process; calls on one GPU share
// it, so calls that overlap on one GPU race.  Everything a call reads is
// written earlier in the same call (the padded state planes by the pad-in
// kernel, the control block by the init kernel, the stage planes, the
// accumulator and the partials by the stage kernels), so nothing left by a
// previous call, of whatever size, is read.
namespace {
constexpr int kNoAllocMaxN = 1024;
constexpr size_t kScratchBytes = 73 * 1024 * 1024;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's `scratch` (the host-side name is only
// a stand-in), taken once per device with that device current.
qpr_status scratch_for_current_device(void** out) {
  int dev = -1;
  QPR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(QPR_E_HIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    QPR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(QPR_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QPR_OK;
}
}  // namespace

extern "C" qpr_status qpr_rk4_step_noalloc(const qpr_problem* P, double omega, double dt,
                                           int32_t nsteps, double* rho, int32_t prec,
                                           double* diag_out, const qpr_opts* opts,
                                           qpr_stream_t stream) {
  clear_error();
  qpr_status st = check_problem(P);
  if (st != QPR_OK) return st;
  if (P->n > kNoAllocMaxN)
    return fail(QPR_E_ARG, "qpr_rk4_step_noalloc serves n <= %d (got n = %d)", kNoAllocMaxN,
                P->n);
  if (prec != QPR_FP64)
    return fail(QPR_E_ARG, "qpr_rk4_step_noalloc runs FP64 products only (got prec %d)", prec);
  const size_t need = ws_bytes(P->n, prec, false);
  if (need > kScratchBytes)
    return fail(QPR_E_WORKSPACE, "static scratch of %zu bytes, n = %d needs %zu", kScratchBytes,
                P->n, need);
  void* ws = nullptr;
  if ((st = scratch_for_current_device(&ws)) != QPR_OK) return st;
  return qpr_rk4_step(P, omega, dt, nsteps, rho, prec, diag_out, opts, ws, kScratchBytes, stream);
}
