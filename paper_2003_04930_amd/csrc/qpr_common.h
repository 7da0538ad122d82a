// Internal declarations shared by the libqpr sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>

#include "../../include/qpr.h"

namespace qpr {

constexpr int kPad = 64;          // internal planes are padded to a multiple of this
// block-sparse product: slab lists per 32-row block of H_off, slabs 16 wide
constexpr int kBsM = 32, kBsK = 16;
// product configuration value that selects the block-sparse product
constexpr int kCfgBlockSparse = -1000;
constexpr size_t kAlign = 256;    // every carved region starts on this boundary

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }
inline int pad_n(int n) { return (n + kPad - 1) / kPad * kPad; }
// Values of a Hermitian-packed tile-pair array (the accumulator, the Fehlberg
// stage derivatives): a real and an imaginary 32 x 32 block per tile pair of
// the upper triangle, (ld/32)(ld/32 + 1)/2 pairs -- ld^2 + 32 ld values, about
// one plane instead of two.
inline size_t packed_values(int ld) {
  const size_t t = (size_t)ld / 32;
  return t * (t + 1) / 2 * 2 * 32 * 32;
}

// Error reporting: sets this thread's last message and returns the status.
qpr_status fail(qpr_status s, const char* fmt, ...);
void clear_error();

#define QPR_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return ::qpr::fail(QPR_E_HIP, "%s failed: %s (%s:%d)", #call,            \
                         hipGetErrorString(e_), __FILE__, __LINE__);           \
  } while (0)

// Owners of HIP runtime objects, released on every return path (locals are
// destroyed in reverse order: declare a graph before its executable).
struct HipEvent {
  hipEvent_t h = nullptr;
  HipEvent() = default;
  HipEvent(const HipEvent&) = delete;
  HipEvent& operator=(const HipEvent&) = delete;
  ~HipEvent() { if (h) (void)hipEventDestroy(h); }
};
struct HipStream {
  hipStream_t h = nullptr;
  HipStream() = default;
  HipStream(const HipStream&) = delete;
  HipStream& operator=(const HipStream&) = delete;
  ~HipStream() { if (h) (void)hipStreamDestroy(h); }
};
struct HipGraph {
  hipGraph_t h = nullptr;
  HipGraph() = default;
  HipGraph(const HipGraph&) = delete;
  HipGraph& operator=(const HipGraph&) = delete;
  ~HipGraph() { if (h) (void)hipGraphDestroy(h); }
};
struct HipGraphExec {
  hipGraphExec_t h = nullptr;
  HipGraphExec() = default;
  HipGraphExec(const HipGraphExec&) = delete;
  HipGraphExec& operator=(const HipGraphExec&) = delete;
  ~HipGraphExec() { if (h) (void)hipGraphExecDestroy(h); }
};
struct HostPinned {
  void* h = nullptr;
  HostPinned() = default;
  HostPinned(const HostPinned&) = delete;
  HostPinned& operator=(const HostPinned&) = delete;
  ~HostPinned() { if (h) (void)hipHostFree(h); }
};

// Device-resident control block of one solve.  Written by one lane of the
// finishing step of a reducing stage (and of the final-state statistics
// kernel), with vector stores, and read by every later launch on the stream.
struct DevState {
  double resid2;        // ||L(y_n)||_F^2 measured by the latest stage-1 pass
  double tol2;          // tol^2
  long long step;       // RK4 steps whose stage 1 has been started
  long long max_steps;  // stop (not converged) once step reaches this
  long long conv_step;  // step index whose state met the tolerance
  long long rhs_evals;  // product launches that ran (counted by stage-1 and RHS passes)
  int stop;             // non-zero: every solver launch returns at once
  int converged;
  int nonfinite;
  int check;            // 1: stage 1 tests the tolerance
  unsigned int ticket;  // last-workgroup counter of the final-state statistics
  int hold;             // non-zero: low-precision step launches return at once
  double judge2;        // mixed precision: latest FP64 ||L(rho_a)||_F^2
  long long folds;      // mixed precision: FP64 judge evaluations
  double aux[8];        // final-state diagnostics (trace, herm, min diag, ...)
  // adaptive Fehlberg 4(5) integration
  double h;             // current step size
  double h_max;         // cap on the step size
  double tol_step;      // local error tolerance per unit step
  double t;             // integrated time of the accepted state
  double err;           // latest max |z - y|
  long long accepted;   // accepted steps
  long long rejected;   // rejected steps
  int accept;           // the latest attempt was accepted
  int pad1;
};

// Values of EpiArgs::check
enum CheckMode {
  CHK_NONE = 0,   // record ||k||^2 only
  CHK_PLAIN = 1,  // stage 1 of the FP64 solve: converge / count steps
  CHK_DELTA = 2,  // stage 1 of a low-precision delta step: hold when the estimate meets tol
  CHK_JUDGE = 3,  // FP64 residual of the anchor: converge, or release the hold
  CHK_RKF = 4     // stage 1 of a Fehlberg attempt: converge / count attempts
};

// Workspace carved from the caller's buffer.  Planes are ld*ld.
struct Ws {
  int n = 0, ld = 0, prec = 0;
  double *yn_r = nullptr, *yn_i = nullptr;   // y_n (or the anchor delta in mixed mode)
  double *y1_r = nullptr, *y1_i = nullptr;   // stage states (ping)
  double *y2_r = nullptr, *y2_i = nullptr;   // stage states (pong)
  double *acc_r = nullptr, *acc_i = nullptr; // RK4 accumulator (Hermitian-packed by tile pair:
                                             // acc_i = acc_r + 32 * 32)
  double *x_r = nullptr, *x_i = nullptr;     // X = H_off * Y (FP64 products)
  double *ra_r = nullptr, *ra_i = nullptr;   // mixed: FP64 anchor residual L(rho_a)
  double *an_r = nullptr, *an_i = nullptr;   // mixed: FP64 anchor rho_a
  float *xf_r = nullptr, *xf_i = nullptr;    // FP32 products (mixed modes)
  float *lo_r = nullptr, *lo_i = nullptr;    // FP32 operand copy (QPR_FP32)
  // QPR_FP32 with the defect held in FP32 (each pair of FP32 planes lives in
  // the bytes of an FP64 plane pair that this mode leaves unused): delta_n,
  // the two stage states, the accumulator, and the FP32 copy of r_a
  float *dn_r = nullptr, *dn_i = nullptr, *d1_r = nullptr, *d1_i = nullptr;
  float *d2_r = nullptr, *d2_i = nullptr, *dac_r = nullptr, *dac_i = nullptr;
  float *ra32_r = nullptr, *ra32_i = nullptr;
  uint16_t* sl = nullptr;                    // bf16 slices: [plane][slice][ld*ld]
  double *p_n = nullptr, *p_1 = nullptr, *p_2 = nullptr, *p_a = nullptr; // diagonals (n)
  double *k_r[5] = {}, *k_i[5] = {};         // Fehlberg stage derivatives (FP64 only; packed
                                             // as the accumulator)
  double *cand_r = nullptr, *cand_i = nullptr, *p_c = nullptr;  // Fehlberg candidate state
  double* partials = nullptr;                // per-workgroup partial sums
  int max_partials = 0;
  int *bs_cnt = nullptr, *bs_idx = nullptr;  // block-sparse product: slab lists per block row
  DevState* st = nullptr;
  double* scal = nullptr;                    // small scratch (16 doubles)
};

// rkf: include the Fehlberg planes (single solves); the batched solve omits them
size_t ws_bytes(int n, int prec, bool rkf = true);
bool ws_carve(void* base, size_t bytes, int n, int prec, Ws* out, bool rkf = true);

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return hipGetLastError().

// Problem view handed to the epilogue.
struct ProbView {
  int n, ld, teleport;
  double alpha;
  const double *h, *d, *inv_outdeg;
  const int *dangling, *in_ptr, *in_idx;
  int hsign;                 // value of every nonzero of H_off (+1 or -1)
  const int *h_ptr, *h_idx;  // CSR pattern of H_off
  int spmm_variant;          // sparse-product variant, -1 = the default one
};
ProbView view_of(const qpr_problem* P);

// The finishing step of a reducing stage (fold the tile partials, update the
// control block), run by k_finish or by one extra workgroup of the next
// sparse-product launch.  nb = 0: nothing to finish.
struct FinishJob {
  const double* partials;
  int nb;
  DevState* st;
  int check, fstage, gate;
};

// Epilogue modes: the right-hand side alone, the four classical RK4 stages,
// and the six Fehlberg 4(5) stages (EPI_F1 + s - 1 for stage s).
enum EpiMode { EPI_RHS = 0, EPI_S1 = 1, EPI_S2 = 2, EPI_S3 = 3, EPI_S4 = 4, EPI_F1 = 11 };

// Which buffer kind the epilogue reads X from and what lowp copy it writes.
enum OpKind { OP_F64 = 0, OP_F32 = 1, OP_BF16X3 = 2 };

// Where the epilogue gets X = H_off Y from.
enum XSource {
  XS_DENSE64 = 0,   // FP64 X written by the dense product
  XS_DENSE32 = 1,   // FP32 X written by a low-precision dense product
  XS_SPARSE64 = 2,  // FP64 X written by the sparse product (k_spmm)
  XS_FUSED64 = 3,   // FP64 X gathered inside the epilogue tile (no product launch)
  XS_FUSED32 = 4,   // the same from the FP32 copy of Y_s (xfr/xfi), X rounded to FP32
  XS_FUSED32S = 5   // FP32 state: every state plane of the stage is FP32 (the defect of
                    // the mixed solve); gathers and X as XS_FUSED32, xfr/xfi = Y_s
};

struct EpiArgs {
  const double *xr, *xi;      // FP64 X (OP_F64)
  const float *xfr, *xfi;     // FP32 X (OP_F32 / OP_BF16X3); XS_FUSED32: FP32 copy of Y_s
  const double *ysr, *ysi;    // stage input Y_s
  const double* ps;           // diag of Y_s
  const double *ynr, *yni;    // y_n
  double *accr, *acci;        // accumulator
  double *outr, *outi;        // stage output (y_{s+1}, y_n at stage 4, or L(Y) for RHS)
  double* pout;               // diag of the output state
  const double *rar, *rai;    // mixed mode: FP64 anchor residual added to L (or null)
  float *lor, *loi;           // FP32 copy of the output state (or null)
  uint16_t* slices;           // bf16 slices of the output state (or null)
  double omega, cdt;          // cdt: c_s * dt for stages 1..3, dt/6 for stage 4
  int mode, xkind;             // xkind: XSource
  int check;                  // CheckMode
  int gate;                   // 1: also return when DevState::hold is set
  // Fehlberg stages (mode EPI_F1 .. EPI_F1 + 5)
  const double *kr[5], *ki[5];  // K_1 .. K_5 (upper triangle)
  double *kwr, *kwi;            // where this stage stores its K (stages 1..5)
  double cf[6];                 // stage s < 6: a_{s+1, 1..s}; stage 6: b4
  double ce[6];                 // stage 6: b5 - b4
};

// cfg = kCfgBlockSparse: the block-sparse product over the slab lists in w
hipError_t launch_gemm(int kind, int cfg, const qpr_problem* P, const Ws& w,
                       const double* yr, const double* yi, int gate, hipStream_t s);
// slab lists of the block-sparse product for P into w.bs_cnt / w.bs_idx
hipError_t launch_block_pattern(const qpr_problem* P, const Ws& w, hipStream_t s);
// finish = false leaves a reducing stage's partials unfolded (kernel timing,
// or a finishing step carried by the next launch); `carry` (fused epilogue
// only) is the previous stage's finishing step, run as one extra workgroup
hipError_t launch_epilogue(const ProbView& pv, const EpiArgs& a, const Ws& w, hipStream_t s,
                           bool finish = true, const FinishJob* carry = nullptr);
hipError_t launch_pad_in(const double* rho, int n, int ld, double* r, double* i,
                         double* p, hipStream_t s);
hipError_t launch_pad_out(const double* r, const double* i, int n, int ld,
                          double* rho, hipStream_t s);
hipError_t launch_to_lowp(int kind, const double* r, const double* i, int n,
                          int ld, const Ws& w, hipStream_t s);
hipError_t launch_state_init(DevState* st, double tol, long long max_steps,
                             int check, hipStream_t s);
hipError_t launch_state_rkf(DevState* st, double h0, double h_max, double tol_step,
                            hipStream_t s);
hipError_t launch_state_stats(const double* r, const double* i, const double* p,
                              int n, int ld, const Ws& w, hipStream_t s);
hipError_t launch_rank(int n, const double* p, int* order, hipStream_t s);
hipError_t launch_hubs(int n, const double* p, double c, int* out, hipStream_t s);
hipError_t launch_axpy_planes(double* yr, double* yi, const double* xr,
                              const double* xi, double a, int n, int ld,
                              double* p, const DevState* st, hipStream_t s);
hipError_t launch_axpy_planes_f32(double* yr, double* yi, const float* xr, const float* xi,
                                  double a, int n, int ld, double* p, const DevState* st,
                                  hipStream_t s);
hipError_t launch_trace(const double* p, int n, DevState* st, hipStream_t s);
hipError_t launch_rkf_commit(double* yr, double* yi, double* p, const double* cr,
                             const double* ci, const double* pc, int n, int ld,
                             const DevState* st, hipStream_t s);
hipError_t launch_fill(void* dst, size_t bytes, hipStream_t s);
hipError_t launch_scale_planes(double* r, double* i, double* p, int n, int ld,
                               const DevState* st, hipStream_t s);

// One system's operands for a batched product launch (pointer types per kind).
struct BatchGemm {
  const void *H, *yr, *yi;
  void *xr, *xi;
  int ld, gate;
  const DevState* st;
};
// One system's arguments for a batched epilogue launch.
struct BatchEpi {
  ProbView pv;
  EpiArgs a;
  DevState* st;
  double* partials;
};
int batch_gemm_cfgs(int kind, int* out, int max);
int batch_gemm_tile(int cfg);
hipError_t launch_gemm_batch(int cfg, const BatchGemm* args, const int2* items,
                             const int* nitems, int grid, hipStream_t s);
// finish: the stage reduces (stage 1, judge, Fehlberg stages 1 and 6), so the
// finishing kernel folds each running system's partials (sys_list, nsys)
hipError_t launch_epilogue_batch(int xsource, const BatchEpi* args, const int2* items,
                                 const int* nitems, int grid, const int* sys_list,
                                 const int* nsys, bool finish, hipStream_t s);
// Fehlberg 4(5): epilogue arguments of stage st (0..5) on a workspace, and the
// largest step whose fourth-order update is stable for the spectrum bound of
// the Liouvillian at omega (rho_h = spectral radius of H).
EpiArgs rkf_stage_args(const Ws& w, int st, double omega, int xs);
// classical RK4 stage k of the mixed solve's defect step with the defect held
// in FP32 (XS_FUSED32S, every state plane single precision)
EpiArgs rk4_stage_args_f32s(const Ws& w, int k, double omega, double dt, int check, int gate);

// Concurrent single-system solves: `nworkers` host threads, worker w on
// streams[w] with workspace ws[w] (each large enough for the largest system),
// taking systems in index order (qpr_steady_state_many).
constexpr int kMaxWorkers = 64;
qpr_status run_many(int count, const qpr_problem* const* probs, const double* omegas, double dt,
                    double tol, int64_t max_steps, int prec, double* const* rhos,
                    int32_t* const* ranks, qpr_stats* stats, const qpr_opts* opts, int nworkers,
                    void* const* ws, const size_t* wsb, const qpr_stream_t* streams);
double rkf_step_cap(double omega, double rho_h);

// variant: index into the sparse-product variants (-1 = pv.spmm_variant);
// fin: the finishing step of the previous stage, run by one extra workgroup
hipError_t launch_spmm(const ProbView& pv, const double* yr, const double* yi, double* xr,
                       double* xi, const DevState* st, int gate, hipStream_t s, int variant = -1,
                       const FinishJob* fin = nullptr);
// FP32 operand form (mixed-precision steps): X (FP32) = H_off Y (FP32 copy)
hipError_t launch_spmm_f32(const ProbView& pv, const float* yr, const float* yi, float* xr,
                           float* xi, const DevState* st, int gate, hipStream_t s,
                           const FinishJob* fin = nullptr);
// The finishing step of a reducing epilogue launch with these arguments.
FinishJob finish_job(const ProbView& pv, const EpiArgs& a, const Ws& w);
int spmm_num_variants();
const char* spmm_variant_name(int v);
int spmm_items_per_system(int n, int ld);
int epilogue_items_per_system(int ld);
hipError_t launch_spmm_batch(const BatchEpi* args, const int2* items, const int* nitems, int grid,
                             hipStream_t s);
// FP32 operand form over the same items: a.lor / a.loi -> a.xfr / a.xfi
hipError_t launch_spmm_f32_batch(const BatchEpi* args, const int2* items, const int* nitems,
                                 int grid, hipStream_t s);

// Tuned choices beside the dense tiles (qpr_autotune, qpr_load_tuning), per
// padded size, looked up exactly: the sparse-product variant, and whether
// a lone FP64 solve takes the fused epilogue (1) or product + epilogue (0).
constexpr int kTuneSparseVariant = 10, kTuneFusedStage = 11;
bool tuned_exact(int kind, int ld, int* cfg);
int gemm_num_cfgs(int kind);
const char* gemm_cfg_name(int kind, int cfg);
int gemm_default_cfg(int kind, int n);
void gemm_set_tuned(int kind, int ld, int cfg);
bool gemm_cfg_fits(int kind, int cfg, int ld);

// Progress of a long batch on stderr, for callers that watch a run's output:
// with QPR_PROGRESS=<seconds> set, report() prints "done of total" at most
// once per that interval, and the final count when the run has lasted at
// least that long; unset, it prints nothing.  Safe to call from several
// worker threads.
class Progress {
 public:
  explicit Progress(const char* what) : what_(what), t0_(std::chrono::steady_clock::now()) {
    const char* e = std::getenv("QPR_PROGRESS");
    every_ = e ? std::atof(e) : 0.0;
  }
  void report(int done, int total, const char* unit) {
    if (every_ <= 0.0) return;
    std::lock_guard<std::mutex> lk(mu_);
    const double t =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
    if (done < total ? t - last_ < every_ : t < every_) return;
    last_ = t;
    std::fprintf(stderr, "[qpr] %s: %d of %d systems %s after %.0f s\n", what_, done, total, unit,
                 t);
    std::fflush(stderr);
  }

 private:
  const char* what_;
  std::chrono::steady_clock::time_point t0_;
  double every_ = 0.0, last_ = 0.0;
  std::mutex mu_;
};

}  // namespace qpr
