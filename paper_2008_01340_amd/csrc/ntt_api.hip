// ntt_api.hip -- plan, workspace layout, stage executor and the C ABI of ntt.h.
//
// The executor runs the sweep of Alg.2 with MU as the NMF, or the BCD of Alg.3
// (ntt_bcd.hip); the ranks are given, or chosen per stage by the singular-value rule of
// Alg.2.  Stage l factors X_l, an (r_{l-1} n_l) x (n_{l+1}...n_d) row-major matrix that
// is a zero-copy view of the input (l = 1) or of the previous stage's H; with host input
// (stream_cols > 0) stage 1 reads X_1 in column blocks copied from host memory.  W is updated in place inside the caller's core buffer l (its C-order
// layout r_{l-1} x n_l x r_l is exactly W, m x r_l); H lives in one of two workspace
// buffers (ping-pong, so X_l and H_l never alias), except that the last stage's H is
// written straight into core d.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "ntt_internal.h"

using namespace ntt;

namespace {

thread_local std::string g_last_error;

ntt_status fail(ntt_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(NTT_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

constexpr int kGraphIters = 25;     // MU iterations per replayed graph
constexpr size_t kMaxGraphs = 64;

}  // namespace

// A plan: the host layout (ntt_host.h) and the device-side objects created on first use.
struct ntt_plan_s : PlanLayout {
  rocblas_handle rb = nullptr;  // created on first use by the rank rule
  std::vector<hipEvent_t> prof_events;
  hipEvent_t stage_ev[2 * NTT_MAX_DIMS] = {};
  bool events_ready = false;
  // stages may run as one grid-synchronised launch (standalone plans; batched and served
  // problems run concurrently on several streams and keep one launch per pass)
  bool coop_allowed = true;
  // replayable blocks of MU iterations, one per (stage, block length, buffers)
  struct GraphEntry {
    int stage, iters;
    bool bf;
    int variant;  // 0: pass + W-update; 1, 2: prologue mode from the first / a later iteration
    const void *X, *H, *W, *ws;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  ~ntt_plan_s() {
    if (rb) (void)rocblas_destroy_handle(rb);
    for (auto e : prof_events) (void)hipEventDestroy(e);
    if (events_ready)
      for (auto e : stage_ev) (void)hipEventDestroy(e);
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
  }
};

extern "C" {

const char* ntt_version(void) { return "ntt-mi355x 0.1 gfx950"; }

const char* ntt_last_error(void) { return g_last_error.c_str(); }

const char* ntt_status_string(ntt_status s) {
  switch (s) {
    case NTT_OK: return "ok";
    case NTT_ERR_INVALID_ARG: return "invalid argument";
    case NTT_ERR_RANK_INFEASIBLE: return "rank infeasible";
    case NTT_ERR_NEGATIVE_INPUT: return "negative, NaN or Inf input";
    case NTT_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case NTT_ERR_ZERO_NORM: return "zero norm";
    case NTT_ERR_DEVICE: return "device error";
  }
  return "unknown status";
}

double ntt_compression_ratio(int32_t d, const int64_t* dims, const int64_t* ranks) {
  if (d < 1 || d > NTT_MAX_DIMS || !dims || !ranks) return 0.0;
  return compression_of(d, dims, ranks);
}

ntt_status ntt_plan(const ntt_config* cfg, ntt_plan_t* out) {
  if (!cfg || !out) return fail(NTT_ERR_INVALID_ARG, "null config or output");
  *out = nullptr;
  auto* p = new ntt_plan_s();
  std::string err;
  const ntt_status st = plan_layout(cfg, p, &err);
  if (st != NTT_OK) {
    delete p;
    return fail(st, err);
  }
  *out = p;
  return NTT_OK;
}

ntt_status ntt_plan_workspace(ntt_plan_t p, size_t* bytes, int64_t* eff_ranks, double* compression) {
  if (!p) return fail(NTT_ERR_INVALID_ARG, "null plan");
  if (bytes) *bytes = p->total;
  if (eff_ranks)
    for (int i = 0; i <= p->d; ++i) eff_ranks[i] = p->cap[i];
  if (compression) *compression = compression_of(p->d, p->dims, p->cap);
  return NTT_OK;
}

void ntt_plan_destroy(ntt_plan_t p) { delete p; }

}  // extern "C"

namespace {


// Workspace views of one problem.
struct Ctx {
  ntt_plan_s* p;
  hipStream_t s;
  char* ws;
  float* part() const { return reinterpret_cast<float*>(ws + p->off_part); }
  double* rpart() const { return reinterpret_cast<double*>(ws + p->off_rpart); }
  double* red() const { return reinterpret_cast<double*>(ws + p->off_red); }
  float* gw() const { return reinterpret_cast<float*>(ws + p->off_gw); }
  double* scal(int l) const {  // FP64 scalars of stage l (1-based)
    return reinterpret_cast<double*>(ws + p->off_scal) + (size_t)SCAL_COUNT * (l - 1);
  }
  // [0] input flags, [8] cooperative-stage status, [32] W-update arrival counter
  int* ints() const { return reinterpret_cast<int*>(ws + p->off_ints); }
  uint16_t* xb() const { return reinterpret_cast<uint16_t*>(ws + p->off_xb); }
  float* xt() const { return reinterpret_cast<float*>(ws + p->off_xt); }
  float* wp() const { return reinterpret_cast<float*>(ws + p->off_wp); }
  float* hp() const { return reinterpret_cast<float*>(ws + p->off_hp); }
  float* sbuf() const { return reinterpret_cast<float*>(ws + p->off_s); }
  float* wb() const { return reinterpret_cast<float*>(ws + p->off_wb); }
  double* gpart() const { return reinterpret_cast<double*>(ws + p->off_gpart); }
  double* grp() const { return reinterpret_cast<double*>(ws + p->off_grp); }
  double* gram() const { return reinterpret_cast<double*>(ws + p->off_gram); }
  double* eig() const { return reinterpret_cast<double*>(ws + p->off_eig); }
  void* eigws() const { return ws + p->off_eigws; }
  template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

PassArgs pass_args(const Ctx& c, const Stage& s, const float* X, float* H, const float* W, float eps) {
  PassArgs a{};  // every field set below; Xb (BF16 copy) stays NULL unless set by the caller
  a.X = X;
  a.Xb = nullptr;
  a.H = H;
  a.W = W;
  a.GW = c.gw();
  a.part = c.part();
  a.part_stride = (int64_t)s.part_stride;
  a.rpart = c.rpart();
  a.m = (int)s.m;
  a.r = s.r;
  a.k = s.k;
  a.eps = eps;
  a.S = s.kind == PASS_C ? c.sbuf() : nullptr;
  a.nchunks = s.nch;
  a.Hs = s.kind == PASS_C ? c.sbuf() + (size_t)s.nch * s.r * s.k : nullptr;
  a.pair_groups = s.pairs ? 1 : 0;
  return a;
}

hipError_t run_pass(hipStream_t q, const Stage& s, const PassArgs& a, bool update, bool resid) {
  if (s.kind == PASS_S && s.tiny && update) {
    // a residual with the update: the 16-row-block pass first, on the incoming (W, H)
    if (resid) {
      const hipError_t e = launch_pass_fused(a, s.rp, s.mb, s.G, false, true, false, q);
      if (e != hipSuccess) return e;
    }
    return launch_pass_tiny(a, s.G, q);
  }
  if (s.kind == PASS_S) return launch_pass_fused(a, s.rp, s.mb, s.G, update, resid, s.wide, q);
  if (s.kind == PASS_L) return launch_pass_L(a, s.rp, s.cls, s.G, update, resid, s.wide, q);
  if (s.kind == PASS_C) return launch_pass_C(a, s.rp, s.G, update, resid, q);
  return launch_pass_generic(a, s.rp, s.G, s.chunk, update, resid, q);
}

int resid_blocks(const Stage& s) {
  if (s.kind == PASS_C) return s.G * s.nch;
  return s.fused ? s.G : (int)((s.k + 255) / 256);
}

}  // namespace

// One decomposition in flight: the sweep as a resumable state machine (stage l,
// iteration t), so that it can run to completion (ntt_decompose), in lock-step with
// other problems (batched mode), or a block of iterations at a time (serving).
struct NttJob {
  ntt_plan_s* p = nullptr;
  Ctx c{};
  const float* A = nullptr;
  std::vector<float*> cores;
  std::vector<const float*> initW, initH;
  double* trace = nullptr;
  bool record = false, profile = false, want_final = false;
  int l = 1, t = 0;
  bool prepared = false, done = false;
  int64_t trace_off = 0;
  int iters[NTT_MAX_DIMS] = {};
  int bf_planned[NTT_MAX_DIMS] = {};  // per stage: leading iterations on the BF16 copy of X
  // state of the current stage
  const float* X = nullptr;
  float* H = nullptr;
  float* W = nullptr;
  PassArgs pa{}, pa_bf{};
  FinArgs fa{}, fa_pre{};
  int bf_iters = 0;
  bool one_wg = false, final_known = false;
  bool trans = false;  // the stage iterates on X^T ~ H^T W^T (pa, fa refer to it)
  // prologue mode: each pass applies the previous iteration's W-update (W_j alternates
  // between the core buffer, j even, and the workspace buffer, j odd); one W-update
  // launch at the end of the stage puts W_T into the core
  bool pro = false, pro_done = false;
  double nx = 0.0;
  std::vector<double> fhist;
  bool bcd = false;  // the stage runs Alg.3 (BCD) instead of MU
  BcdArgs ba{};
  bool streamed = false;  // stage 1 with X in host memory, passed over in column blocks
  bool coop = false;      // the stage's iterations run in cooperative whole-stage launches

  // column block b of the streamed stage: width, shape, staging copies
  int64_t blk_w(int64_t b) const { return std::min(p->kblk, st().k - b * p->kblk); }
  const Stage& blk_stage(int64_t b) const { return b == p->nblk - 1 ? p->sst[1] : p->sst[0]; }
  float* xs() const { return c.at<float>(p->off_xs); }
  float* hs() const { return c.at<float>(p->off_hs); }
  hipError_t stage_in(int64_t b, bool with_h) {
    const int64_t j0 = b * p->kblk, w = blk_w(b), k = st().k;
    hipError_t e = hipMemcpy2DAsync(xs(), (size_t)w * 4, A + j0, (size_t)k * 4, (size_t)w * 4,
                                    (size_t)st().m, hipMemcpyHostToDevice, c.s);
    if (e != hipSuccess || !with_h) return e;
    return hipMemcpy2DAsync(hs(), (size_t)w * 4, H + j0, (size_t)k * 4, (size_t)w * 4, (size_t)st().r,
                            hipMemcpyDeviceToDevice, c.s);
  }
  hipError_t stage_out_h(int64_t b) {
    const int64_t j0 = b * p->kblk, w = blk_w(b), k = st().k;
    return hipMemcpy2DAsync(H + j0, (size_t)k * 4, hs(), (size_t)w * 4, (size_t)w * 4, (size_t)st().r,
                            hipMemcpyDeviceToDevice, c.s);
  }
  PassArgs blk_args(int64_t b) const { return pass_args(c, blk_stage(b), xs(), hs(), W, (float)p->cfg.eps); }

  const Stage& st() const { return p->st[l - 1]; }
  const Stage& es() const { return trans ? p->tst[l - 1] : p->st[l - 1]; }  // as iterated
  int d() const { return p->d; }

  ntt_status start(ntt_plan_s* plan, hipStream_t s, void* workspace, const float* A_,
                   float* const* cores_, const float* const* iW, const float* const* iH,
                   double* trace_, bool want_report) {
    p = plan;
    c = Ctx{plan, s, reinterpret_cast<char*>(workspace)};
    A = A_;
    cores.assign(cores_, cores_ + plan->d);
    initW.assign(plan->d, nullptr);
    initH.assign(plan->d, nullptr);
    if (iW)
      for (int i = 0; i < plan->d - 1; ++i) initW[i] = iW[i];
    if (iH)
      for (int i = 0; i < plan->d - 1; ++i) initH[i] = iH[i];
    trace = trace_;
    record = (plan->cfg.flags & NTT_RECORD_OBJECTIVE) && trace_;
    profile = (plan->cfg.flags & NTT_PROFILE) && want_report && plan->cfg.nmf == NTT_NMF_MU &&
              plan->cfg.stream_cols == 0;
    want_final = record || want_report || plan->cfg.tol > 0.0;
    l = 1;
    t = 0;
    prepared = done = false;
    trace_off = 0;
    if (plan->cfg.rank_eps > 0.0)
      for (int i = 0; i <= plan->d; ++i) plan->eff[i] = plan->cap[i];
    HIP_TRY(launch_zero_ints(c.ints(), 64, s));
    return NTT_OK;
  }

  // The rank rule of Alg.2 for stage l: the squared singular values of X_l are the
  // eigenvalues of its FP64 Gram on the shorter side (rocSOLVER syevd, eigenvalues
  // only, in the plan's workspace); r_l is the smallest k whose tail ratio
  // sqrt(sum_{i>k} s_i^2 / sum_i s_i^2) is at most rank_eps (tails added from the
  // smallest value up), capped by the planned rank.  The stage is then re-planned at
  // that rank.
  ntt_status select_rank() {
    const ntt_config& cfg = p->cfg;
    hipStream_t q = c.s;
    const int64_t m = p->eff[l - 1] * p->dims[l - 1];
    int64_t k = 1;
    for (int j = l; j < d(); ++j) k *= p->dims[j];
    const bool blocks = l == 1 && cfg.stream_cols > 0;  // X_1 in host memory
    int n = (int)std::min(m, k);
    if (blocks) {  // the m x m Gram as the sum of the column blocks' row Grams
      double* g2 = c.at<double>(p->off_gram2);
      for (int64_t b = 0; b < p->nblk; ++b) {
        HIP_TRY(stage_in(b, false));
        HIP_TRY(launch_gram_rows(xs(), m, blk_w(b), c.grp(), g2, q));
        HIP_TRY(launch_add_doubles(c.gram(), g2, m * m, b == 0 ? 1 : 0, q));
      }
      n = (int)m;
    } else {
      const float* Xl = (l == 1) ? A : reinterpret_cast<const float*>(c.ws + p->off_h[(l - 2) & 1]);
      HIP_TRY(launch_gram(Xl, m, k, c.grp(), c.gram(), q));
    }
    if (!p->rb && rocblas_create_handle(&p->rb) != rocblas_status_success) {
      p->rb = nullptr;
      return fail(NTT_ERR_DEVICE, "rocblas_create_handle failed");
    }
    if (rocblas_set_stream(p->rb, q) != rocblas_status_success)
      return fail(NTT_ERR_DEVICE, "rocblas_set_stream failed");
    double* D = c.eig();
    double* E = D + n;
    rocblas_int* info = reinterpret_cast<rocblas_int*>(E + n);
    size_t need = 0;
    if (rocblas_start_device_memory_size_query(p->rb) != rocblas_status_success)
      return fail(NTT_ERR_DEVICE, "rocblas memory size query failed");
    (void)rocsolver_dsyevd(p->rb, rocblas_evect_none, rocblas_fill_upper, n, c.gram(), n, D, E, info);
    if (rocblas_stop_device_memory_size_query(p->rb, &need) != rocblas_status_success)
      return fail(NTT_ERR_DEVICE, "rocblas memory size query failed");
    if (need > p->eigws_size)
      return fail(NTT_ERR_WORKSPACE_TOO_SMALL, "eigensolver needs " + std::to_string(need) + " bytes");
    if (rocblas_set_workspace(p->rb, c.eigws(), p->eigws_size) != rocblas_status_success)
      return fail(NTT_ERR_DEVICE, "rocblas_set_workspace failed");
    if (rocsolver_dsyevd(p->rb, rocblas_evect_none, rocblas_fill_upper, n, c.gram(), n, D, E, info) !=
        rocblas_status_success)
      return fail(NTT_ERR_DEVICE, "rocsolver_dsyevd failed");
    std::vector<double> ev((size_t)n);
    rocblas_int hinfo = 0;
    HIP_TRY(hipMemcpyAsync(ev.data(), D, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, q));
    HIP_TRY(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, q));
    HIP_TRY(hipStreamSynchronize(q));
    if (hinfo != 0) return fail(NTT_ERR_DEVICE, "eigensolver did not converge");
    // eigenvalues ascending; pre[j] = sum of the j smallest (negative rounding -> 0)
    std::vector<double> pre((size_t)n + 1, 0.0);
    for (int j = 0; j < n; ++j) pre[j + 1] = pre[j] + std::max(ev[j], 0.0);
    const double total = pre[n];
    int64_t rk = 1;
    if (total > 0.0) {
      rk = n;
      for (int kk = 1; kk <= n; ++kk)
        if (std::sqrt(pre[n - kk] / total) <= cfg.rank_eps) {
          rk = kk;
          break;
        }
    }
    const int64_t r = std::min(std::min(p->cap[l], rk), std::min(m, k));
    p->eff[l] = r;
    stage_shape(cfg, m, k, (int)r, p->st[l - 1], p->tst[l - 1]);
    if (blocks) {  // the column blocks' shapes at the chosen rank
      Stage tt{};
      stage_shape(cfg, m, p->kblk, (int)r, p->sst[0], tt);
      stage_shape(cfg, m, k - (p->nblk - 1) * p->kblk, (int)r, p->sst[1], tt);
    }
    p->compression = compression_of(d(), p->dims, p->eff);
    // graphs captured for an earlier shape of this stage
    for (size_t i = 0; i < p->graphs.size();) {
      if (p->graphs[i].stage == l) {
        (void)hipGraphExecDestroy(p->graphs[i].exec);
        p->graphs.erase(p->graphs.begin() + (long)i);
      } else {
        ++i;
      }
    }
    return NTT_OK;
  }

  // a1 (norm, input check), a2 (initial factors), W^T W, and the BF16 copy (a8)
  ntt_status prepare_stage(bool validate_now) {
    const ntt_config& cfg = p->cfg;
    if (cfg.rank_eps > 0.0) {
      const ntt_status rs = select_rank();
      if (rs != NTT_OK) return rs;
    }
    const Stage& s = st();
    hipStream_t q = c.s;
    const int dd = d();
    X = (l == 1) ? A : reinterpret_cast<const float*>(c.ws + p->off_h[(l - 2) & 1]);
    H = (l == dd - 1) ? cores[dd - 1] : reinterpret_cast<float*>(c.ws + p->off_h[(l - 1) & 1]);
    W = cores[l - 1];
    const int64_t mr = s.m * s.r, rk = (int64_t)s.r * s.k;
    const bool validate = (l == 1) && (cfg.flags & NTT_VALIDATE_INPUT);
    streamed = (l == 1) && cfg.stream_cols > 0;
    if (streamed) {  // ||X||^2 (and the input check) over the column blocks
      double* bsum = c.at<double>(p->off_bsum);
      for (int64_t b = 0; b < p->nblk; ++b) {
        HIP_TRY(stage_in(b, false));
        HIP_TRY(launch_sumsq(xs(), s.m * blk_w(b), c.rpart(), kSumsqBlocks, c.ints(), validate ? 1 : 0,
                             bsum + b, q));
      }
      HIP_TRY(launch_sum_doubles(bsum, (int)p->nblk, 1.0, c.scal(l) + SCAL_NX2, q));
    } else {
      HIP_TRY(launch_sumsq(X, s.m * s.k, c.rpart(), kSumsqBlocks, c.ints(), validate ? 1 : 0,
                           c.scal(l) + SCAL_NX2, q));
    }
    if (validate && validate_now) {
      int flag = 0;
      HIP_TRY(hipMemcpyAsync(&flag, c.ints(), sizeof(int), hipMemcpyDeviceToHost, q));
      HIP_TRY(hipStreamSynchronize(q));
      if (flag) return fail(NTT_ERR_NEGATIVE_INPUT, "input holds a negative, NaN or Inf entry");
    }
    if (initW[l - 1]) HIP_TRY(launch_copy(W, initW[l - 1], mr, q));
    else HIP_TRY(launch_init_uniform(W, mr, cfg.seed, 2ull * l, q));
    if (initH[l - 1]) HIP_TRY(launch_copy(H, initH[l - 1], rk, q));
    else HIP_TRY(launch_init_uniform(H, rk, cfg.seed, 2ull * l + 1, q));
    bcd = cfg.nmf == NTT_NMF_BCD;
    trans = !bcd && !streamed && s.trans_ok && !record && !profile && cfg.tol == 0.0 && cfg.max_iters >= 1;
    const Stage& e = es();
    one_wg = !bcd && !streamed && !trans && !record && !profile && stage_1wg_ok(s.m, s.k, s.r);
    coop = p->coop_allowed && !(cfg.flags & NTT_NO_COOP) && s.coop_ok && !bcd && !streamed && !trans &&
           !one_wg && !record && !profile && cfg.tol == 0.0 && cfg.max_iters >= 1 &&
           s.coop_G <= stage_coop_max_grid(s.coop_ng);
    pro = !bcd && !streamed && !coop && s.pro_ok && !trans && !one_wg && !record && !profile && cfg.tol == 0.0 && cfg.max_iters >= 1;
    pro_done = false;
    const float eps = (float)cfg.eps;
    if (trans) {
      // X' = X^T (k x m), W' = H^T (k x r), H' = W^T (r x m); W'^T W' comes from the
      // first W'-update
      HIP_TRY(launch_transpose(X, c.xt(), s.m, s.k, q));
      HIP_TRY(launch_transpose(W, c.hp(), s.m, s.r, q));
      HIP_TRY(launch_transpose(H, c.wp(), s.r, s.k, q));
      pa = pass_args(c, e, c.xt(), c.hp(), c.wp(), eps);
    } else {
      if (!one_wg) HIP_TRY(launch_gram_w(W, (int)s.m, s.r, s.rp, c.gw(), q));
      pa = pass_args(c, s, X, H, W, eps);
    }
    pa_bf = pa;
    // (a cooperative stage keeps X on chip: it reads X once per launch, in FP32)
    bf_iters = (e.bf16 && !bcd && !streamed && !coop) ? std::max(0, cfg.max_iters - cfg.fp32_tail_iters) : 0;
    bf_planned[l - 1] = bf_iters;
    if (bf_iters > 0) {
      HIP_TRY(launch_cast_bf16(c.xb(), pa.X, s.m * s.k, q));
      pa_bf.Xb = c.xb();
    }
    fa = FinArgs{};
    fa.part = c.part();
    fa.part_stride = (int64_t)e.part_stride;
    fa.G = e.G;
    fa.m = (int)e.m;
    fa.r = e.r;
    fa.red = c.red();
    fa.gpart = c.gpart();
    fa.arrive = reinterpret_cast<unsigned*>(c.ints() + 32);  // zeroed with the ints at job start
    fa.W = trans ? c.wp() : W;
    fa.GW = c.gw();
    fa.scal = c.scal(l);
    fa.eps = eps;
    fa_pre = fa;
    fa_pre.G = e.G_pre;
    t = 0;
    final_known = false;
    fhist.clear();
    if (bcd) {
      ba = BcdArgs{};
      ba.X = X;
      ba.Hb[0] = H;
      ba.Hb[1] = c.at<float>(p->off_bh[0]);
      ba.Hb[2] = c.at<float>(p->off_bh[1]);
      ba.W = W;
      ba.Wp = c.at<float>(p->off_bwp);
      ba.Wn = c.at<float>(p->off_bwn);
      ba.XHc = c.at<double>(p->off_bxh);
      ba.HHc = c.at<double>(p->off_bhh);
      ba.GWn = c.at<float>(p->off_bgw);
      ba.st = c.at<BcdState>(p->off_bst);
      ba.part = c.part();
      ba.part_stride = (int64_t)bcd_part_stride(s.m, s.r);
      bcd_chunks(s.m, s.k, s.r, &ba.G, &ba.chunk);
      ba.red = c.red();
      ba.rpart = c.rpart();
      ba.scal = c.scal(l);
      ba.trace = nullptr;
      ba.m = (int)s.m;
      ba.r = s.r;
      ba.k = s.k;
      ba.delta = cfg.bcd_delta;
      HIP_TRY(launch_bcd_prepare(ba, q));
    }
    if (cfg.tol > 0.0) {
      HIP_TRY(residual_now(nullptr));
      double h2[2];
      HIP_TRY(hipMemcpyAsync(h2, c.scal(l), 2 * sizeof(double), hipMemcpyDeviceToHost, q));
      HIP_TRY(hipStreamSynchronize(q));
      nx = std::sqrt(h2[SCAL_NX2]);
      fhist.push_back(h2[SCAL_OBJ]);
    }
    prepared = true;
    return NTT_OK;
  }

  hipError_t residual_now(double* slot) {
    hipError_t e = run_pass(c.s, es(), pa, false, true);
    if (e != hipSuccess) return e;
    return launch_resid_sum(c.rpart(), resid_blocks(es()), c.scal(l) + SCAL_OBJ, slot, c.s);
  }

  float* wbuf(int j) const { return (j & 1) ? c.wb() : W; }

  // one prologue-mode iteration (0-based `it`): the pass, then the reduction of its partials
  hipError_t pro_iter(hipStream_t q, int it, bool bf) {
    PassArgs a = bf ? pa_bf : pa;
    if (it > 0) {
      a.Wprev = wbuf(it - 1);
      a.Wout = wbuf(it);
      a.red = c.red();
    }
    hipError_t e = run_pass(q, st(), a, true, false);
    if (e != hipSuccess) return e;
    return launch_reduce(fa, q);
  }

  hipError_t graph_for(int n, bool bf, int it0, hipGraphExec_t* out) {
    const PassArgs& pg = bf ? pa_bf : pa;
    const int variant = bcd ? 3 : (pro ? (it0 == 0 ? 1 : 2) : 0);
    const void* wkey = variant == 2 ? (const void*)wbuf(it0 - 1) : (const void*)pg.W;
    for (auto& g : p->graphs)
      if (g.stage == l && g.iters == n && g.bf == bf && g.variant == variant && g.X == pg.X &&
          g.H == pg.H && g.W == wkey && g.ws == c.ws) {
        *out = g.exec;
        return hipSuccess;
      }
    // capture on one library-wide stream (graphs are then launched on any stream)
    static std::mutex cap_mu;
    static hipStream_t cap_stream = nullptr;
    std::lock_guard<std::mutex> lock(cap_mu);
    hipError_t e;
    if (!cap_stream) {
      e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int i = 0; i < n && le == hipSuccess; ++i) {
      if (bcd) {
        le = launch_bcd_iter(ba, cap_stream);
        continue;
      }
      if (pro) {
        le = pro_iter(cap_stream, it0 + i, bf);
        continue;
      }
      le = run_pass(cap_stream, es(), pg, true, false);
      if (le == hipSuccess) {
        FinArgs f2 = fa;
        f2.rpart = nullptr;
        f2.trace = nullptr;
        le = launch_finalize(f2, es().rp, cap_stream);
      }
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap_stream, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return le;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    if (p->graphs.size() >= kMaxGraphs) {
      (void)hipGraphExecDestroy(p->graphs.front().exec);
      p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back({l, n, bf, variant, pg.X, pg.H, wkey, c.ws, exec});
    *out = exec;
    return hipSuccess;
  }

  // a3 + a4: up to `budget` MU iterations of the current stage (a stopping check of a5
  // may end the stage early); *stage_done is set when no iterations remain.
  ntt_status iterate(int budget, bool* stage_done) {
    if (bcd) return iterate_bcd(budget, stage_done);
    if (coop) return iterate_coop(budget, stage_done);
    if (streamed) return iterate_streamed(budget, stage_done);
    if (trans) return iterate_transposed(budget, stage_done);
    if (pro) return iterate_prologue(budget, stage_done);
    const ntt_config& cfg = p->cfg;
    const Stage& s = st();
    hipStream_t q = c.s;
    const bool use_graph = !record && !profile && cfg.max_iters > 1;
    bool stop = false;
    while (budget > 0 && t < cfg.max_iters && !stop) {
      int block = std::min(budget, cfg.max_iters - t);
      if (cfg.tol > 0.0) block = std::min(block, cfg.check_every - (t % cfg.check_every));
      const bool bf = t < bf_iters;  // this block reads the BF16 copy of X
      if (bf) block = std::min(block, bf_iters - t);
      const PassArgs& pcur = bf ? pa_bf : pa;
      int n_done = 0;
      if (one_wg) {
        StageArgs sa{};
        sa.X = X;
        sa.W = W;
        sa.H = H;
        sa.m = (int)s.m;
        sa.r = s.r;
        sa.k = (int)s.k;
        sa.iters = block;
        sa.eps = (float)cfg.eps;
        HIP_TRY(launch_stage_1wg(sa, q));
        n_done = block;
      } else {
        if (use_graph) {
          while (block - n_done >= kGraphIters || (block - n_done > 1 && cfg.tol > 0.0)) {
            const int n = std::min(block - n_done, kGraphIters);
            hipGraphExec_t ex = nullptr;
            HIP_TRY(graph_for(n, bf, t + n_done, &ex));
            HIP_TRY(hipGraphLaunch(ex, q));
            n_done += n;
          }
        }
        for (; n_done < block; ++n_done) {
          const int tt = t + n_done + 1;
          const bool resid = record;  // f_{tt-1} of the incoming iterate
          double* slot = (resid && tt >= 2) ? trace + trace_off + (tt - 2) : nullptr;
          if (profile) HIP_TRY(hipEventRecord(p->prof_events[2 * (tt - 1)], q));
          HIP_TRY(run_pass(q, s, resid ? pa : pcur, true, resid));
          if (profile) HIP_TRY(hipEventRecord(p->prof_events[2 * (tt - 1) + 1], q));
          FinArgs f2 = fa;
          if (resid && !s.fused) {
            HIP_TRY(launch_resid_sum(c.rpart(), resid_blocks(s), c.scal(l) + SCAL_OBJ, slot, q));
            f2.rpart = nullptr;
            f2.trace = nullptr;
          } else {
            f2.rpart = resid ? c.rpart() : nullptr;
            f2.trace = resid ? slot : nullptr;
          }
          HIP_TRY(launch_finalize(f2, s.rp, q));
        }
      }
      t += block;
      budget -= block;
      final_known = false;
      if (cfg.tol > 0.0 && t % cfg.check_every == 0) {
        HIP_TRY(residual_now(record ? trace + trace_off + (t - 1) : nullptr));
        double ft = 0.0;
        HIP_TRY(hipMemcpyAsync(&ft, c.scal(l) + SCAL_OBJ, sizeof(double), hipMemcpyDeviceToHost, q));
        HIP_TRY(hipStreamSynchronize(q));
        fhist.resize(t + 1, 0.0);
        fhist[t] = ft;
        final_known = true;
        const double fprev = fhist[t - cfg.check_every];
        if (std::sqrt(2.0 * std::max(ft, 0.0)) / nx <= cfg.tol || (fprev - ft) <= cfg.tol * fprev)
          stop = true;
      }
    }
    *stage_done = stop || t >= cfg.max_iters;
    if (stop) iters[l - 1] = t;
    return NTT_OK;
  }

  // MU iterations of a stage in cooperative whole-stage launches (X, H and W on chip);
  // W, H and W^T W are read at the start of a launch and written at its end, so launches
  // of a few iterations each continue one another.  A barrier time-out sets ints[8].
  ntt_status iterate_coop(int budget, bool* stage_done) {
    const ntt_config& cfg = p->cfg;
    const Stage& s = st();
    const int block = std::min(budget, cfg.max_iters - t);
    if (block > 0) {
      CoopArgs a{};
      a.X = X;
      a.W = W;
      a.H = H;
      a.GW = c.gw();
      a.part = c.part();
      a.red = c.red();
      a.flags = c.at<unsigned>(p->off_coop);
      a.status = c.ints() + 8;
      a.m = (int)s.m;
      a.r = s.r;
      a.k = s.k;
      a.iters = block;
      a.eps = (float)cfg.eps;
      HIP_TRY(launch_stage_coop(a, s.coop_ng, s.coop_G, c.s));
      t += block;
      final_known = false;
    }
    *stage_done = t >= cfg.max_iters;
    return NTT_OK;
  }

  // Alg.3: up to `budget` of the stage's T iterations (fixed count).  With a trace, the
  // objective of candidate j (1-based) is stored when iteration j + 1 (or the end of the
  // stage) decides on it, at trace slot j - 1.
  ntt_status iterate_bcd(int budget, bool* stage_done) {
    const ntt_config& cfg = p->cfg;
    hipStream_t q = c.s;
    const int T = cfg.max_iters;
    while (budget > 0 && t < T) {
      const int block = std::min(budget, T - t);
      int n_done = 0;
      if (!record) {
        while (block - n_done >= kGraphIters) {
          hipGraphExec_t ex = nullptr;
          HIP_TRY(graph_for(kGraphIters, false, t + n_done, &ex));
          HIP_TRY(hipGraphLaunch(ex, q));
          n_done += kGraphIters;
        }
      }
      for (; n_done < block; ++n_done) {
        BcdArgs b = ba;
        const int it = t + n_done + 1;
        b.trace = (record && it >= 2) ? trace + trace_off + (it - 2) : nullptr;
        HIP_TRY(launch_bcd_iter(b, q));
      }
      t += block;
      budget -= block;
      final_known = false;
    }
    *stage_done = t >= T;
    return NTT_OK;
  }

  // Stage 1 out of core: per MU iteration, every column block is copied in (X from host
  // memory, its H columns from H_1), its pass updates H and writes its X H^T, H H^T
  // partials, which are reduced and added in block order; H goes back; then one
  // W-update from the sums.
  ntt_status iterate_streamed(int budget, bool* stage_done) {
    const ntt_config& cfg = p->cfg;
    hipStream_t q = c.s;
    const Stage& s = st();
    const int64_t E = s.m * s.r + (int64_t)s.r * s.r;
    double* redtmp = c.at<double>(p->off_redtmp);
    FinArgs fw = fa;
    fw.rpart = nullptr;
    fw.trace = nullptr;
    fw.Wout = nullptr;
    while (budget > 0 && t < cfg.max_iters) {
      for (int64_t b = 0; b < p->nblk; ++b) {
        const Stage& sb = blk_stage(b);
        HIP_TRY(stage_in(b, true));
        HIP_TRY(run_pass(q, sb, blk_args(b), true, false));
        FinArgs fb = fa;
        fb.part_stride = (int64_t)sb.part_stride;
        fb.G = sb.G;
        fb.red = redtmp;
        HIP_TRY(launch_reduce(fb, q));
        HIP_TRY(launch_add_doubles(c.red(), redtmp, E, b == 0 ? 1 : 0, q));
        HIP_TRY(stage_out_h(b));
      }
      HIP_TRY(launch_wupdate_red(fw, q));
      ++t;
      --budget;
      final_known = false;
    }
    *stage_done = t >= cfg.max_iters;
    return NTT_OK;
  }

  // The stage's T iterations in prologue mode (no stopping checks), then W_T.
  ntt_status iterate_prologue(int budget, bool* stage_done) {
    const ntt_config& cfg = p->cfg;
    hipStream_t q = c.s;
    const int T = cfg.max_iters;
    while (budget > 0 && t < T) {
      const bool bf = t < bf_iters;
      int block = std::min(budget, T - t);
      if (bf) block = std::min(block, bf_iters - t);
      int n_done = 0;
      while (block - n_done >= kGraphIters) {
        hipGraphExec_t ex = nullptr;
        HIP_TRY(graph_for(kGraphIters, bf, t + n_done, &ex));
        HIP_TRY(hipGraphLaunch(ex, q));
        n_done += kGraphIters;
      }
      for (; n_done < block; ++n_done) HIP_TRY(pro_iter(q, t + n_done, bf));
      t += block;
      budget -= block;
      final_known = false;
    }
    if (t >= T && !pro_done) {
      FinArgs ff = fa;
      ff.W = wbuf(T - 1);
      ff.Wout = ff.W == W ? nullptr : W;
      ff.rpart = nullptr;
      ff.trace = nullptr;
      HIP_TRY(launch_wupdate_red(ff, q));
      pro_done = true;
    }
    *stage_done = t >= T;
    return NTT_OK;
  }

  // The stage's T iterations on X' = X^T: H'-update of X' is the W-update of X and its
  // W'-update the H-update, so H_1 is the W'-update of (W'_0, H'_0), each of the next
  // T - 1 transposed iterations gives (W_t, H_{t+1}), and an H'-update alone gives W_T.
  ntt_status iterate_transposed(int budget, bool* stage_done) {
    const ntt_config& cfg = p->cfg;
    const Stage& e = es();
    hipStream_t q = c.s;
    const int T = cfg.max_iters;
    while (budget > 0 && t < T) {
      if (t == 0) {
        PassArgs pre = pa;
        pre.part_stride = (int64_t)e.part_stride;
        HIP_TRY(launch_xht_partials(pre, e.rp, e.G_pre, e.chunk_pre, q));
        HIP_TRY(launch_finalize(fa_pre, e.rp, q));
      }
      const bool bf = t < bf_iters;
      const PassArgs& pcur = bf ? pa_bf : pa;
      if (t < T - 1) {
        int block = std::min(budget, T - 1 - t);
        if (bf) block = std::min(block, bf_iters - t);
        int n_done = 0;
        while (block - n_done >= kGraphIters) {
          hipGraphExec_t ex = nullptr;
          HIP_TRY(graph_for(kGraphIters, bf, t + n_done, &ex));
          HIP_TRY(hipGraphLaunch(ex, q));
          n_done += kGraphIters;
        }
        for (; n_done < block; ++n_done) {
          HIP_TRY(run_pass(q, e, pcur, true, false));
          HIP_TRY(launch_finalize(fa, e.rp, q));
        }
        t += block;
        budget -= block;
      } else {
        HIP_TRY(run_pass(q, e, pcur, true, false));
        t = T;
        budget -= 1;
      }
      final_known = false;
    }
    *stage_done = t >= T;
    return NTT_OK;
  }

  // a5 at the end of the stage (explicit objective of the final iterate), then a6:
  // W is already core l; H becomes the next unfolding (or is core d).
  ntt_status finish_stage() {
    const ntt_config& cfg = p->cfg;
    if (iters[l - 1] == 0) iters[l - 1] = t;
    if (streamed) {  // the final objective over the column blocks
      if (want_final) {
        double* bsum = c.at<double>(p->off_bsum);
        for (int64_t b = 0; b < p->nblk; ++b) {
          const Stage& sb = blk_stage(b);
          HIP_TRY(stage_in(b, true));
          HIP_TRY(run_pass(c.s, sb, blk_args(b), false, true));
          HIP_TRY(launch_resid_sum(c.rpart(), resid_blocks(sb), bsum + b, nullptr, c.s));
        }
        HIP_TRY(launch_sum_doubles(bsum, (int)p->nblk, 1.0, c.scal(l) + SCAL_OBJ, c.s));
        final_known = true;
      }
      streamed = false;
    }
    // the trace slot of the last iterate: with BCD it holds the last candidate's objective
    // (written by the decision on it), which need not be the kept pair's
    double* last_slot = (record && t >= 1) ? trace + trace_off + (t - 1) : nullptr;
    if (bcd) {  // decision on the last candidate; the kept H into the stage's buffer
      BcdArgs b = ba;
      b.trace = last_slot;
      HIP_TRY(launch_bcd_finish(b, c.s));
      bcd = false;
      last_slot = nullptr;
    }
    if (want_final && !final_known) HIP_TRY(residual_now(last_slot));
    if (trans) {  // W = H'^T, H = W'^T
      const Stage& s = st();
      HIP_TRY(launch_transpose(c.hp(), W, s.r, s.m, c.s));
      HIP_TRY(launch_transpose(c.wp(), H, s.k, s.r, c.s));
      trans = false;
    }
    trace_off += cfg.max_iters;
    prepared = false;
    if (l + 1 >= d()) done = true;
    else ++l;
    return NTT_OK;
  }

  // one stage from start to end on the job's stream
  ntt_status run_stage() {
    ntt_status e = prepare_stage(true);
    if (e != NTT_OK) return e;
    bool sd = false;
    e = iterate(p->cfg.max_iters, &sd);
    if (e != NTT_OK) return e;
    return finish_stage();
  }

  // per-stage FP64 scalars (asynchronous copy; valid after the stream has synchronised)
  hipError_t fetch_scalars(double* host) {
    return hipMemcpyAsync(host, c.scal(1), sizeof(double) * SCAL_COUNT * (d() - 1),
                          hipMemcpyDeviceToHost, c.s);
  }

  void fill_report(const double* sc, ntt_report* rep) const {
    memset(rep, 0, sizeof(*rep));
    for (int i = 0; i <= d(); ++i) rep->eff_ranks[i] = p->eff[i];
    rep->compression_ratio = p->compression;
    for (int ll = 1; ll < d(); ++ll) {
      const Stage& s = p->st[ll - 1];
      const double* v = sc + (size_t)SCAL_COUNT * (ll - 1);
      rep->iters[ll - 1] = iters[ll - 1];
      if (p->cfg.nmf == NTT_NMF_BCD) rep->corrections[ll - 1] = (int32_t)v[SCAL_BCD_CORR];
      rep->bf16_iters[ll - 1] = std::min(bf_planned[ll - 1], iters[ll - 1]);
      rep->norm_x[ll - 1] = std::sqrt(v[SCAL_NX2]);
      rep->objective[ll - 1] = v[SCAL_OBJ];
      rep->stage_rel_err[ll - 1] =
          rep->norm_x[ll - 1] > 0 ? std::sqrt(2.0 * std::max(v[SCAL_OBJ], 0.0)) / rep->norm_x[ll - 1] : 0.0;
      rep->gflop[ll - 1] = (double)iters[ll - 1] *
                           (4.0 * s.m * s.k * s.r + 4.0 * (s.m + s.k) * s.r * s.r) * 1e-9;
      rep->total_gflop += rep->gflop[ll - 1];
    }
  }
};

static ntt_status check_decompose_args(ntt_plan_s* p, void* workspace, const float* A,
                                       float* const* cores) {
  if (!p) return fail(NTT_ERR_INVALID_ARG, "null plan");
  if (!workspace) return fail(NTT_ERR_WORKSPACE_TOO_SMALL, "null workspace");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(NTT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (!A || !cores) return fail(NTT_ERR_INVALID_ARG, "null A or cores");
  for (int i = 0; i < p->d; ++i)
    if (!cores[i]) return fail(NTT_ERR_INVALID_ARG, "null core pointer");
  return NTT_OK;
}

extern "C" ntt_status ntt_decompose(ntt_plan_t p, void* stream, void* workspace, const float* A,
                                    float* const* cores, const float* const* init_W,
                                    const float* const* init_H, double* objective_trace,
                                    ntt_report* report) {
  ntt_status st = check_decompose_args(p, workspace, A, cores);
  if (st != NTT_OK) return st;
  const ntt_config& cfg = p->cfg;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!p->events_ready) {
    for (auto& e : p->stage_ev) HIP_TRY(hipEventCreate(&e));
    p->events_ready = true;
  }
  const bool profile = (cfg.flags & NTT_PROFILE) && report && cfg.nmf == NTT_NMF_MU &&
                       cfg.stream_cols == 0;
  if (profile && (int64_t)p->prof_events.size() < 2 * (int64_t)cfg.max_iters) {
    while (p->prof_events.size() < 2 * (size_t)cfg.max_iters) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      p->prof_events.push_back(e);
    }
  }
  NttJob job;
  st = job.start(p, s, workspace, A, cores, init_W, init_H, objective_trace, report != nullptr);
  if (st != NTT_OK) return st;
  const int d = p->d;
  std::vector<double> pass_ms(d, 0.0);
  while (!job.done) {
    const int l = job.l;
    HIP_TRY(hipEventRecord(p->stage_ev[2 * (l - 1)], s));
    st = job.run_stage();
    if (st != NTT_OK) return st;
    HIP_TRY(hipEventRecord(p->stage_ev[2 * (l - 1) + 1], s));
    if (profile && job.iters[l - 1] > 0) {
      HIP_TRY(hipStreamSynchronize(s));
      double sum = 0.0;
      for (int t = 0; t < job.iters[l - 1]; ++t) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p->prof_events[2 * t], p->prof_events[2 * t + 1]));
        sum += ms;
      }
      pass_ms[l - 1] = sum / job.iters[l - 1];
    }
  }
  std::vector<double> sc((size_t)SCAL_COUNT * (d - 1), 0.0);
  if (report) HIP_TRY(job.fetch_scalars(sc.data()));
  int coop_status = 0;
  HIP_TRY(hipMemcpyAsync(&coop_status, job.c.ints() + 8, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (coop_status != 0) return fail(NTT_ERR_DEVICE, "a cooperative stage's grid barrier timed out");
  if (report) {
    ntt_report rep;
    job.fill_report(sc.data(), &rep);
    for (int l = 1; l < d; ++l) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, p->stage_ev[2 * (l - 1)], p->stage_ev[2 * (l - 1) + 1]));
      rep.ms[l - 1] = ms;
      rep.total_ms += ms;
      rep.pass_ms[l - 1] = pass_ms[l - 1];
    }
    *report = rep;
  }
  return NTT_OK;
}

// ------------------------------------------------------------------ TT expansion entry points
static ntt_status tt_args(int32_t d, const int64_t* dims, const int64_t* ranks,
                          const float* const* cores, TTArgs* t) {
  if (d < 2 || d > NTT_MAX_DIMS) return fail(NTT_ERR_INVALID_ARG, "d must be in 2..16");
  if (!dims || !ranks || !cores) return fail(NTT_ERR_INVALID_ARG, "null dims, ranks or cores");
  if (ranks[0] != 1 || ranks[d] != 1) return fail(NTT_ERR_INVALID_ARG, "r_0 and r_d must be 1");
  memset(t, 0, sizeof(*t));
  t->d = d;
  int64_t rows = 1;
  for (int i = 0; i < d; ++i) {
    if (dims[i] < 1) return fail(NTT_ERR_INVALID_ARG, "dims must be >= 1");
    if (!cores[i]) return fail(NTT_ERR_INVALID_ARG, "null core pointer");
    t->dims[i] = dims[i];
    t->cores[i] = cores[i];
    if (i < d - 1) {
      if (rows > ((int64_t)1 << 62) / dims[i]) return fail(NTT_ERR_INVALID_ARG, "tensor too large");
      rows *= dims[i];
    }
  }
  if (rows > ((int64_t)1 << 62) / dims[d - 1]) return fail(NTT_ERR_INVALID_ARG, "tensor too large");
  for (int i = 0; i <= d; ++i) {
    if (ranks[i] < 1 || ranks[i] > NTT_MAX_RANK) return fail(NTT_ERR_INVALID_ARG, "ranks must be in 1..32");
    t->ranks[i] = (int)ranks[i];
  }
  t->rows = rows;
  return NTT_OK;
}

extern "C" ntt_status ntt_tt_workspace(int32_t d, const int64_t* dims, const int64_t* ranks, size_t* bytes) {
  TTArgs t{};
  std::vector<const float*> dummy(NTT_MAX_DIMS, reinterpret_cast<const float*>(16));
  ntt_status st = tt_args(d, dims, ranks, dummy.data(), &t);
  if (st != NTT_OK) return st;
  if (!bytes) return fail(NTT_ERR_INVALID_ARG, "null bytes");
  const int64_t nb = tt_blocks(t.rows, t.dims[d - 1]);
  *bytes = align_up((size_t)(2 * nb + 2) * sizeof(double), 256);
  return NTT_OK;
}

extern "C" ntt_status ntt_reconstruct(int32_t d, const int64_t* dims, const int64_t* ranks,
                                      const float* const* cores, float* A_out, void* stream) {
  TTArgs t{};
  ntt_status st = tt_args(d, dims, ranks, cores, &t);
  if (st != NTT_OK) return st;
  if (!A_out) return fail(NTT_ERR_INVALID_ARG, "null output");
  t.out = A_out;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(launch_tt_expand(t, 0, s));
  HIP_TRY(hipStreamSynchronize(s));
  return NTT_OK;
}

extern "C" ntt_status ntt_rel_error(int32_t d, const int64_t* dims, const int64_t* ranks, const float* A,
                                    const float* const* cores, void* workspace, size_t workspace_bytes,
                                    double* rel_err, void* stream) {
  TTArgs t{};
  ntt_status st = tt_args(d, dims, ranks, cores, &t);
  if (st != NTT_OK) return st;
  if (!A || !rel_err) return fail(NTT_ERR_INVALID_ARG, "null A or rel_err");
  size_t need = 0;
  ntt_tt_workspace(d, dims, ranks, &need);
  if (!workspace || workspace_bytes < need) return fail(NTT_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  t.A = A;
  t.part = reinterpret_cast<double*>(workspace);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(launch_tt_expand(t, 1, s));
  const int64_t nb = tt_blocks(t.rows, t.dims[d - 1]);
  double tot[2];
  HIP_TRY(hipMemcpyAsync(tot, t.part + 2 * nb, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!(tot[1] > 0.0)) return fail(NTT_ERR_ZERO_NORM, "||A||_F = 0");
  *rel_err = std::sqrt(tot[0] / tot[1]);
  return NTT_OK;
}

// ------------------------------------------------------------------ Eq.(3) without allocation
// The per-block partial sums of ntt_rel_error_static live in a file-scope device array
// (each GPU holds its own copy for the life of the process).  Host code never passes the
// array's name to a kernel or a copy: its device address is taken once per device with
// hipGetSymbolAddress, with that device current, and that address is used instead.
namespace {
constexpr size_t kStaticScratchDoubles = NTT_REL_ERROR_STATIC_BYTES / sizeof(double);
__device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

ntt_status static_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(NTT_ERR_DEVICE, "no current HIP device (or device index beyond 63)");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(NTT_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return NTT_OK;
}
}  // namespace

extern "C" ntt_status ntt_rel_error_static(int32_t d, const int64_t* dims, const int64_t* ranks,
                                           const float* A, const float* const* cores, double* rel_err,
                                           void* stream) {
  size_t need = 0;
  ntt_status st = ntt_tt_workspace(d, dims, ranks, &need);
  if (st != NTT_OK) return st;
  // the limit in rows: (8 MiB / 8 - 2) / 2 blocks of 64 rows; the partials of every tensor
  // within it fit the array whatever n_d (fewer blocks for n_d < 64, column ranges only
  // below 2048 row blocks)
  constexpr int64_t kStaticRows = (int64_t)((NTT_REL_ERROR_STATIC_BYTES / sizeof(double) - 2) / 2) * 64;
  int64_t rows = 1;
  for (int i = 0; i < d - 1; ++i) rows *= dims[i];
  if (rows > kStaticRows || need > NTT_REL_ERROR_STATIC_BYTES)
    return fail(NTT_ERR_WORKSPACE_TOO_SMALL,
                "tensor too large for ntt_rel_error_static: n_1...n_{d-1} must be at most " +
                    std::to_string(kStaticRows) + " (use ntt_rel_error with a workspace)");
  double* ws = nullptr;
  st = static_scratch(&ws);
  if (st != NTT_OK) return st;
  return ntt_rel_error(d, dims, ranks, A, cores, ws, NTT_REL_ERROR_STATIC_BYTES, rel_err, stream);
}

// ------------------------------------------------------------------ batched mode (a9)
// Independent decompositions of uneven shape and rank, advanced stage level by stage
// level.  At each level, unfoldings small enough for one workgroup (m <= 256, k <= 64,
// r <= 16) run all their iterations in grouped launches (one workgroup per problem,
// read from a device work-list); the others replay their per-problem iteration graphs
// on a small pool of streams so that they overlap on the device.  Problems never share
// a reduction, so each result is the same as when decomposed alone.
struct ntt_batch_s {
  std::vector<ntt_plan_s*> plans;
  std::vector<size_t> ws_off;
  size_t list_off = 0, total = 0;
  std::vector<hipStream_t> pool;
  hipEvent_t ev_prep = nullptr;
  std::vector<hipEvent_t> ev_done;
  ~ntt_batch_s() {
    for (auto* p : plans) delete p;
    for (auto q : pool) (void)hipStreamDestroy(q);
    if (ev_prep) (void)hipEventDestroy(ev_prep);
    for (auto e : ev_done) (void)hipEventDestroy(e);
  }
};

// Streams of the batched pool, problems dealt to them in order.  Measured on the 256-problem
// mix (MI355X): 4 streams 3.25 s, 8 2.97 s, 16 2.80 s, 32 2.72 s; dealing the largest
// problems first to the least-loaded stream was no faster than dealing in order.
constexpr int kBatchStreams = 16;

extern "C" ntt_status ntt_batch_plan(int32_t count, const ntt_config* cfgs, ntt_batch_t* out) {
  if (!out || !cfgs || count < 1) return fail(NTT_ERR_INVALID_ARG, "bad batch arguments");
  *out = nullptr;
  auto* b = new ntt_batch_s();
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    ntt_plan_t p = nullptr;
    if (cfgs[i].flags & (NTT_RECORD_OBJECTIVE | NTT_PROFILE | NTT_VALIDATE_INPUT)) {
      delete b;
      return fail(NTT_ERR_INVALID_ARG, "batched mode takes no RECORD/PROFILE/VALIDATE flags");
    }
    if (cfgs[i].stream_cols != 0) {
      delete b;
      return fail(NTT_ERR_INVALID_ARG, "batched mode takes device inputs (stream_cols = 0)");
    }
    if (cfgs[i].rank_eps != 0.0) {
      delete b;
      return fail(NTT_ERR_INVALID_ARG, "batched mode takes given ranks (rank_eps = 0)");
    }
    ntt_status st = ntt_plan(&cfgs[i], &p);
    if (st != NTT_OK) {
      delete b;
      return st;
    }
    p->coop_allowed = false;  // problems run concurrently on several streams
    b->plans.push_back(p);
    b->ws_off.push_back(off);
    off = align_up(off + p->total, 256);
  }
  b->list_off = off;
  off = align_up(off + (size_t)count * sizeof(StageArgs), 256);
  b->total = off;
  *out = b;
  return NTT_OK;
}

extern "C" ntt_status ntt_batch_workspace(ntt_batch_t b, size_t* bytes) {
  if (!b || !bytes) return fail(NTT_ERR_INVALID_ARG, "null batch or bytes");
  *bytes = b->total;
  return NTT_OK;
}

extern "C" ntt_status ntt_batch_eff_ranks(ntt_batch_t b, int32_t i, int64_t* eff_ranks) {
  if (!b || !eff_ranks) return fail(NTT_ERR_INVALID_ARG, "null batch or eff_ranks");
  if (i < 0 || (size_t)i >= b->plans.size()) return fail(NTT_ERR_INVALID_ARG, "problem index out of range");
  return ntt_plan_workspace(b->plans[(size_t)i], nullptr, eff_ranks, nullptr);
}

extern "C" void ntt_batch_destroy(ntt_batch_t b) { delete b; }

extern "C" ntt_status ntt_decompose_batch(ntt_batch_t b, void* stream, void* workspace,
                                          const float* const* A, float* const* const* cores,
                                          ntt_report* reports) {
  if (!b) return fail(NTT_ERR_INVALID_ARG, "null batch");
  if (!workspace) return fail(NTT_ERR_WORKSPACE_TOO_SMALL, "null workspace");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(NTT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (!A || !cores) return fail(NTT_ERR_INVALID_ARG, "null A or cores");
  const int n = (int)b->plans.size();
  char* ws = reinterpret_cast<char*>(workspace);
  hipStream_t main = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < n; ++i) {
    ntt_status st = check_decompose_args(b->plans[i], ws + b->ws_off[i], A[i], cores ? cores[i] : nullptr);
    if (st != NTT_OK) return st;
  }
  if (b->pool.empty()) {
    for (int i = 0; i < kBatchStreams; ++i) {
      hipStream_t q;
      HIP_TRY(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
      b->pool.push_back(q);
      hipEvent_t e;
      HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->ev_done.push_back(e);
    }
    HIP_TRY(hipEventCreateWithFlags(&b->ev_prep, hipEventDisableTiming));
  }
  std::vector<NttJob> jobs(n);
  int max_level = 0;
  for (int i = 0; i < n; ++i) {
    ntt_status st = jobs[i].start(b->plans[i], main, ws + b->ws_off[i], A[i], cores[i], nullptr,
                                  nullptr, nullptr, reports != nullptr);
    if (st != NTT_OK) return st;
    max_level = std::max(max_level, b->plans[i]->d - 1);
  }
  StageArgs* list_dev = reinterpret_cast<StageArgs*>(ws + b->list_off);
  std::vector<StageArgs> lists[3];
  for (int level = 1; level <= max_level; ++level) {
    std::vector<int> active;
    for (int i = 0; i < n; ++i)
      if (!jobs[i].done && jobs[i].l == level) active.push_back(i);
    if (active.empty()) continue;
    for (int i : active) {
      jobs[i].c.s = main;
      ntt_status st = jobs[i].prepare_stage(false);
      if (st != NTT_OK) return st;
    }
    HIP_TRY(hipEventRecord(b->ev_prep, main));
    // small unfoldings: grouped single-workgroup launches, all iterations
    for (auto& v : lists) v.clear();
    for (int i : active) {
      NttJob& j = jobs[i];
      if (!j.one_wg || j.p->cfg.max_iters < 1 || j.p->cfg.tol > 0.0) continue;
      const Stage& s = j.st();
      StageArgs sa{};
      sa.X = j.X;
      sa.W = j.W;
      sa.H = j.H;
      sa.m = (int)s.m;
      sa.r = s.r;
      sa.k = (int)s.k;
      sa.iters = j.p->cfg.max_iters;
      sa.eps = (float)j.p->cfg.eps;
      const int ng = stage_1wg_ng(s.k);
      lists[ng == 1 ? 0 : (ng == 2 ? 1 : 2)].push_back(sa);
      j.t = j.p->cfg.max_iters;
    }
    size_t at = 0;
    for (int g = 0; g < 3; ++g) {
      if (lists[g].empty()) continue;
      HIP_TRY(hipMemcpyAsync(list_dev + at, lists[g].data(), lists[g].size() * sizeof(StageArgs),
                             hipMemcpyHostToDevice, main));
      HIP_TRY(launch_stage_1wg_grouped(list_dev + at, (int)lists[g].size(), g == 0 ? 1 : (g == 1 ? 2 : 4), main));
      at += lists[g].size();
    }
    // the rest: per-problem iteration graphs, spread over the stream pool
    int slot = 0;
    for (int i : active) {
      NttJob& j = jobs[i];
      if (j.t >= j.p->cfg.max_iters) continue;
      hipStream_t q = b->pool[slot++ % kBatchStreams];
      HIP_TRY(hipStreamWaitEvent(q, b->ev_prep, 0));
      j.c.s = q;
      bool sd = false;
      ntt_status st = j.iterate(j.p->cfg.max_iters, &sd);
      if (st != NTT_OK) return st;
    }
    for (int i : active) {
      ntt_status st = jobs[i].finish_stage();
      if (st != NTT_OK) return st;
    }
    for (int q = 0; q < kBatchStreams; ++q) {
      HIP_TRY(hipEventRecord(b->ev_done[q], b->pool[q]));
      HIP_TRY(hipStreamWaitEvent(main, b->ev_done[q], 0));
    }
  }
  std::vector<std::vector<double>> sc(n);
  if (reports) {
    for (int i = 0; i < n; ++i) {
      sc[i].assign((size_t)SCAL_COUNT * (b->plans[i]->d - 1), 0.0);
      jobs[i].c.s = main;
      HIP_TRY(jobs[i].fetch_scalars(sc[i].data()));
    }
  }
  HIP_TRY(hipStreamSynchronize(main));
  if (reports)
    for (int i = 0; i < n; ++i) jobs[i].fill_report(sc[i].data(), &reports[i]);
  return NTT_OK;
}

// ------------------------------------------------------------------ serving (a10)
// A persistent request engine with continuous batching.  Requests wait in a FIFO queue;
// a scheduler tick (non-blocking) admits the head request when a slot is free and its
// input, cores and workspace fit in the HBM arena (first-fit), copies its input on a
// copy stream, and advances every admitted request whose previous block of work has
// finished by `iters_per_tick` MU iterations: small unfoldings of all such requests in
// one grouped single-workgroup launch, the rest as per-request graph replays on slot
// streams.  Factors stay on the device between ticks and after completion, until the
// client releases the request.  Each request's arithmetic is independent of the mix.
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  int state = NTT_REQ_QUEUED;
  ntt_plan_s* plan = nullptr;
  std::vector<int64_t> dims;
  const float* host_A = nullptr;
  size_t bytes_A = 0, bytes_cores = 0, bytes_ws = 0;
  size_t off_c = 0, total_c = 0;  // cores: held until the client releases the request
  size_t off_w = 0, total_w = 0;  // input + workspace: freed when the request finishes
  std::vector<float*> cores;
  float* A = nullptr;
  NttJob job;
  int slot = -1;
  hipEvent_t ev = nullptr;  // completion of the last block of work issued for this request
  bool started = false;
  double t_submit = 0, t_admit = 0, t_start = 0, t_finish = 0;
  int64_t iters_total = 0;
  double gflop = 0.0;
};

}  // namespace

struct ntt_server_s {
  ntt_server_config cfg;
  Admission adm;  // arena offsets and slots (ntt_host.h)
  char* base = nullptr;  // the arena's device memory
  std::vector<hipStream_t> streams;  // slot streams, then the copy stream, then the grouped stream
  hipStream_t copy_stream = nullptr, group_stream = nullptr;
  hipEvent_t group_ev = nullptr;
  std::deque<Request*> queue;
  std::vector<Request*> active;  // admitted, not yet released
  std::map<int64_t, Request*> all;
  int64_t next_id = 1;
  double t0 = 0;
  std::vector<StageArgs> list_host;
  // the grouped launches of a tick as one graph: one kernel node per register class, its
  // work-list (a kernel argument by value) and grid set before each replay.  A ring of
  // executable instances, each reused only once its previous replay has completed, so an
  // update never touches the arguments of a replay still queued or running.
  static const int kRing = 4;
  hipGraph_t group_graph = nullptr;
  hipGraphNode_t group_node[3] = {};
  hipGraphExec_t group_exec[kRing] = {};
  hipEvent_t ring_ev[kRing] = {};
  bool ring_used[kRing] = {};
  int ring_next = 0;
  ~ntt_server_s() {
    for (auto& kv : all) {
      if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
      delete kv.second->plan;
      delete kv.second;
    }
    for (int i = 0; i < kRing; ++i) {
      if (group_exec[i]) (void)hipGraphExecDestroy(group_exec[i]);
      if (ring_ev[i]) (void)hipEventDestroy(ring_ev[i]);
    }
    if (group_graph) (void)hipGraphDestroy(group_graph);
    for (auto q : streams) (void)hipStreamDestroy(q);
    if (group_ev) (void)hipEventDestroy(group_ev);
  }
};

static const int kGroupNG[3] = {1, 2, 4};

// kernel-node parameters of register class c running list L (one workgroup per entry,
// at least one)
static hipKernelNodeParams group_params(int c, StageList* L, void** args) {
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(stage_1wg_list_kernel(kGroupNG[c]));
  kp.gridDim = dim3((unsigned)std::max(1, L->count));
  kp.blockDim = dim3(256);
  kp.sharedMemBytes = 0;
  args[0] = L;
  kp.kernelParams = args;
  kp.extra = nullptr;
  return kp;
}

// the grouped-launch graph (three independent kernel nodes) and its ring of instances,
// built on first use
static hipError_t server_group_graph(ntt_server_s* sv) {
  if (sv->group_graph) return hipSuccess;
  hipError_t e = hipGraphCreate(&sv->group_graph, 0);
  if (e != hipSuccess) return e;
  for (int c = 0; c < 3; ++c) {
    StageList empty{};
    empty.count = 0;
    void* args[1];
    hipKernelNodeParams kp = group_params(c, &empty, args);
    e = hipGraphAddKernelNode(&sv->group_node[c], sv->group_graph, nullptr, 0, &kp);
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < ntt_server_s::kRing; ++i) {
    e = hipGraphInstantiate(&sv->group_exec[i], sv->group_graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return e;
    e = hipEventCreateWithFlags(&sv->ring_ev[i], hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// an instance whose previous replay has completed: the first idle one from the ring's
// cursor, else the cursor's own once its replay ends (the host waits for that replay only)
static hipError_t server_ring_slot(ntt_server_s* sv, int* slot) {
  const int R = ntt_server_s::kRing;
  for (int d = 0; d < R; ++d) {
    const int i = (sv->ring_next + d) % R;
    if (!sv->ring_used[i]) { *slot = i; return hipSuccess; }
    const hipError_t q = hipEventQuery(sv->ring_ev[i]);
    if (q == hipSuccess) { *slot = i; return hipSuccess; }
    if (q != hipErrorNotReady) return q;
  }
  *slot = sv->ring_next;
  return hipEventSynchronize(sv->ring_ev[sv->ring_next]);
}

// input + workspace and the slot go back when a request finishes; cores on release
static void server_release_work(ntt_server_s* sv, Request* q) {
  if (q->total_w) sv->adm.arena.release(q->off_w, q->total_w);
  q->total_w = 0;
  if (q->slot >= 0) sv->adm.slot_used[q->slot] = 0;
  q->slot = -1;
}

static void server_release_memory(ntt_server_s* sv, Request* q) {
  server_release_work(sv, q);
  if (q->total_c) sv->adm.arena.release(q->off_c, q->total_c);
  q->total_c = 0;
}

extern "C" ntt_status ntt_server_create(const ntt_server_config* cfg, ntt_server_t* out) {
  if (!cfg || !out) return fail(NTT_ERR_INVALID_ARG, "null config or output");
  *out = nullptr;
  if (!cfg->arena || cfg->arena_bytes < 4096 || cfg->max_slots < 1 || cfg->max_slots > NTT_STAGE_LIST ||
      cfg->iters_per_tick < 1)
    return fail(NTT_ERR_INVALID_ARG, "bad server config");
  if ((reinterpret_cast<uintptr_t>(cfg->arena) & 255) != 0)
    return fail(NTT_ERR_INVALID_ARG, "arena must be 256-byte aligned");
  auto* sv = new ntt_server_s();
  sv->cfg = *cfg;
  sv->base = reinterpret_cast<char*>(cfg->arena);
  sv->adm.init(cfg->arena_bytes, cfg->max_slots);
  const int nstreams = std::min(cfg->max_slots, 16);  // slot streams (as the batched pool)
  for (int i = 0; i < nstreams + 2; ++i) {
    hipStream_t q;
    hipError_t e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete sv;
      return fail(NTT_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    sv->streams.push_back(q);
  }
  sv->copy_stream = sv->streams[nstreams];
  sv->group_stream = sv->streams[nstreams + 1];
  if (hipEventCreateWithFlags(&sv->group_ev, hipEventDisableTiming) != hipSuccess) {
    delete sv;
    return fail(NTT_ERR_DEVICE, "hipEventCreate failed");
  }
  sv->t0 = now_s();
  *out = sv;
  return NTT_OK;
}

extern "C" void ntt_server_destroy(ntt_server_t sv) {
  if (!sv) return;
  for (auto q : sv->streams) (void)hipStreamSynchronize(q);
  delete sv;
}

extern "C" ntt_status ntt_server_submit(ntt_server_t sv, const ntt_request* rq, int64_t* id) {
  if (!sv || !rq || !id) return fail(NTT_ERR_INVALID_ARG, "null server, request or id");
  if (!rq->host_A) return fail(NTT_ERR_INVALID_ARG, "null input");
  ntt_config c{};
  c.d = rq->d;
  c.dims = rq->dims;
  c.ranks = rq->ranks;
  c.max_iters = rq->max_iters;
  c.tol = 0.0;
  c.check_every = 10;
  c.eps = rq->eps;
  c.seed = rq->seed;
  c.precision = rq->precision;
  c.fp32_tail_iters = rq->fp32_tail_iters;
  c.flags = 0;
  c.nmf = rq->nmf;
  c.bcd_delta = rq->bcd_delta;
  ntt_plan_t p = nullptr;
  ntt_status st = ntt_plan(&c, &p);
  if (st != NTT_OK) return st;
  p->coop_allowed = false;  // requests run concurrently on several streams
  auto* q = new Request();
  q->id = sv->next_id++;
  q->plan = p;
  q->dims.assign(rq->dims, rq->dims + rq->d);
  q->host_A = rq->host_A;
  int64_t n = 1;
  for (int i = 0; i < rq->d; ++i) n *= rq->dims[i];
  q->bytes_A = align_up((size_t)n * sizeof(float), 256);
  size_t cb = 0;
  for (int i = 0; i < rq->d; ++i)
    cb += align_up((size_t)p->eff[i] * (size_t)p->dims[i] * (size_t)p->eff[i + 1] * sizeof(float), 256);
  q->bytes_cores = cb;
  q->bytes_ws = align_up(p->total, 256);
  q->t_submit = now_s() - sv->t0;
  for (int l = 1; l < p->d; ++l) {
    const Stage& s = p->st[l - 1];
    q->iters_total += c.max_iters;
    q->gflop += (double)c.max_iters * (4.0 * s.m * s.k * s.r + 4.0 * (s.m + s.k) * s.r * s.r) * 1e-9;
  }
  if (q->bytes_A + q->bytes_cores + q->bytes_ws > sv->adm.arena.size) q->state = NTT_REQ_REJECTED;
  else sv->queue.push_back(q);
  sv->all[q->id] = q;
  *id = q->id;
  return NTT_OK;
}

extern "C" ntt_status ntt_server_tick(ntt_server_t sv, int32_t* n_active, int32_t* n_queued) {
  if (!sv) return fail(NTT_ERR_INVALID_ARG, "null server");
  const int K = sv->cfg.iters_per_tick;
  // 1. admission: FIFO while a slot is free and the head request fits in the arena
  while (!sv->queue.empty()) {
    Request* q = sv->queue.front();
    int slot = -1;
    size_t off_c = 0, off_w = 0;
    if (!sv->adm.admit(q->bytes_cores, q->bytes_A + q->bytes_ws, &slot, &off_c, &off_w)) break;
    sv->queue.pop_front();
    q->off_c = off_c;
    q->total_c = q->bytes_cores;
    q->off_w = off_w;
    q->total_w = q->bytes_A + q->bytes_ws;
    q->slot = slot;
    char* base = sv->base + off_w;
    q->A = reinterpret_cast<float*>(base);
    char* cp = sv->base + off_c;
    q->cores.clear();
    for (int i = 0; i < q->plan->d; ++i) {
      q->cores.push_back(reinterpret_cast<float*>(cp));
      cp += align_up((size_t)q->plan->eff[i] * (size_t)q->plan->dims[i] * (size_t)q->plan->eff[i + 1] *
                         sizeof(float), 256);
    }
    char* ws = base + q->bytes_A;
    int64_t n = 1;
    for (auto v : q->dims) n *= v;
    hipStream_t qs = sv->streams[slot % (sv->streams.size() - 2)];
    if (!q->ev) HIP_TRY(hipEventCreateWithFlags(&q->ev, hipEventDisableTiming));
    HIP_TRY(hipMemcpyAsync(q->A, q->host_A, (size_t)n * sizeof(float), hipMemcpyHostToDevice,
                           sv->copy_stream));
    HIP_TRY(hipEventRecord(q->ev, sv->copy_stream));
    HIP_TRY(hipStreamWaitEvent(qs, q->ev, 0));
    ntt_status st = q->job.start(q->plan, qs, ws, q->A, q->cores.data(), nullptr, nullptr, nullptr,
                                 true);
    if (st != NTT_OK) return st;
    HIP_TRY(hipEventRecord(q->ev, qs));
    q->state = NTT_REQ_RUNNING;
    q->t_admit = now_s() - sv->t0;
    sv->active.push_back(q);
  }
  // 2. advance every running request whose previous block has completed
  sv->list_host.clear();
  std::vector<Request*> grouped;
  for (Request* q : sv->active) {
    if (q->state != NTT_REQ_RUNNING) continue;
    const hipError_t qe = hipEventQuery(q->ev);
    if (qe == hipErrorNotReady) continue;
    if (qe != hipSuccess) return fail(NTT_ERR_DEVICE, std::string("hipEventQuery: ") + hipGetErrorString(qe));
    NttJob& j = q->job;
    if (j.done) {
      q->state = NTT_REQ_DONE;
      q->t_finish = now_s() - sv->t0;
      server_release_work(sv, q);  // the cores stay until the client releases them
      continue;
    }
    if (!q->started) {
      q->started = true;
      q->t_start = now_s() - sv->t0;
    }
    if (!j.prepared) {
      ntt_status st = j.prepare_stage(false);
      if (st != NTT_OK) return st;
    }
    const int budget = std::min(K, j.p->cfg.max_iters - j.t);
    if (j.one_wg && budget > 0) {
      const Stage& s = j.st();
      StageArgs sa{};
      sa.X = j.X;
      sa.W = j.W;
      sa.H = j.H;
      sa.m = (int)s.m;
      sa.r = s.r;
      sa.k = (int)s.k;
      sa.iters = budget;
      sa.eps = (float)j.p->cfg.eps;
      sv->list_host.push_back(sa);
      grouped.push_back(q);
      j.t += budget;
      HIP_TRY(hipEventRecord(q->ev, j.c.s));  // the grouped launch waits for this stream
    } else {
      bool sd = false;
      if (budget > 0) {
        ntt_status st = j.iterate(budget, &sd);
        if (st != NTT_OK) return st;
      }
      if (j.t >= j.p->cfg.max_iters) {
        ntt_status st = j.finish_stage();
        if (st != NTT_OK) return st;
      }
      HIP_TRY(hipEventRecord(q->ev, j.c.s));
    }
  }
  if (!grouped.empty()) {
    // one grouped launch per register class for the small stages of all requests; the
    // work-list travels as a kernel argument, so nothing on the host outlives the call
    for (Request* q : grouped) HIP_TRY(hipStreamWaitEvent(sv->group_stream, q->ev, 0));
    StageList lists[3];
    for (auto& L : lists) L.count = 0;
    for (size_t i = 0; i < grouped.size(); ++i) {
      const int ng = stage_1wg_ng(sv->list_host[i].k);
      StageList& L = lists[ng == 1 ? 0 : (ng == 2 ? 1 : 2)];
      L.a[L.count++] = sv->list_host[i];
    }
    for (int c = 0; c < 3; ++c)
      if (lists[c].count > NTT_STAGE_LIST) return fail(NTT_ERR_INVALID_ARG, "too many grouped stages");
    // one graph replay: each node's work-list and grid set for this tick
    HIP_TRY(server_group_graph(sv));
    int slot = 0;
    HIP_TRY(server_ring_slot(sv, &slot));
    for (int c = 0; c < 3; ++c) {
      void* args[1];
      hipKernelNodeParams kp = group_params(c, &lists[c], args);
      HIP_TRY(hipGraphExecKernelNodeSetParams(sv->group_exec[slot], sv->group_node[c], &kp));
    }
    HIP_TRY(hipGraphLaunch(sv->group_exec[slot], sv->group_stream));
    HIP_TRY(hipEventRecord(sv->ring_ev[slot], sv->group_stream));
    sv->ring_used[slot] = true;
    sv->ring_next = (slot + 1) % ntt_server_s::kRing;
    HIP_TRY(hipEventRecord(sv->group_ev, sv->group_stream));
    for (Request* q : grouped) {
      NttJob& j = q->job;
      HIP_TRY(hipStreamWaitEvent(j.c.s, sv->group_ev, 0));
      if (j.t >= j.p->cfg.max_iters) {
        ntt_status st = j.finish_stage();
        if (st != NTT_OK) return st;
      }
      HIP_TRY(hipEventRecord(q->ev, j.c.s));
    }
  }
  sv->active.erase(std::remove_if(sv->active.begin(), sv->active.end(),
                                  [](Request* q) { return q->state != NTT_REQ_RUNNING; }),
                   sv->active.end());
  int na = (int)sv->active.size();
  if (n_active) *n_active = na;
  if (n_queued) *n_queued = (int32_t)sv->queue.size();
  return NTT_OK;
}

extern "C" ntt_status ntt_server_info(ntt_server_t sv, int64_t id, ntt_request_info* info) {
  if (!sv || !info) return fail(NTT_ERR_INVALID_ARG, "null server or info");
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return fail(NTT_ERR_INVALID_ARG, "unknown request id");
  const Request* q = it->second;
  memset(info, 0, sizeof(*info));
  info->id = q->id;
  info->state = q->state;
  info->t_submit = q->t_submit;
  info->t_admit = q->t_admit;
  info->t_start = q->t_start;
  info->t_finish = q->t_finish;
  info->device_bytes = q->bytes_A + q->bytes_cores + q->bytes_ws;
  info->gflop = q->gflop;
  info->d = q->plan->d;
  for (int i = 0; i <= q->plan->d; ++i) info->eff_ranks[i] = q->plan->eff[i];
  return NTT_OK;
}

extern "C" ntt_status ntt_server_cores(ntt_server_t sv, int64_t id, float** core_ptrs) {
  if (!sv || !core_ptrs) return fail(NTT_ERR_INVALID_ARG, "null server or output");
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return fail(NTT_ERR_INVALID_ARG, "unknown request id");
  const Request* q = it->second;
  if (q->state != NTT_REQ_DONE) return fail(NTT_ERR_INVALID_ARG, "request not finished");
  for (int i = 0; i < q->plan->d; ++i) core_ptrs[i] = q->cores[i];
  return NTT_OK;
}

extern "C" ntt_status ntt_server_release(ntt_server_t sv, int64_t id) {
  if (!sv) return fail(NTT_ERR_INVALID_ARG, "null server");
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return fail(NTT_ERR_INVALID_ARG, "unknown request id");
  Request* q = it->second;
  if (q->state == NTT_REQ_RUNNING) {
    // cancellation: wait for the work already issued for it, then drop it
    if (q->ev) HIP_TRY(hipEventSynchronize(q->ev));
    HIP_TRY(hipStreamSynchronize(sv->group_stream));
    HIP_TRY(hipStreamSynchronize(sv->streams[q->slot % (sv->streams.size() - 2)]));
    q->state = NTT_REQ_CANCELLED;
  }
  if (q->state == NTT_REQ_QUEUED) {
    for (auto qi = sv->queue.begin(); qi != sv->queue.end(); ++qi)
      if (*qi == q) {
        sv->queue.erase(qi);
        break;
      }
    q->state = NTT_REQ_CANCELLED;
  }
  server_release_memory(sv, q);
  for (auto ai = sv->active.begin(); ai != sv->active.end(); ++ai)
    if (*ai == q) {
      sv->active.erase(ai);
      break;
    }
  if (q->ev) (void)hipEventDestroy(q->ev);
  q->ev = nullptr;
  delete q->plan;
  q->plan = nullptr;
  sv->all.erase(it);
  delete q;
  return NTT_OK;
}

extern "C" ntt_status ntt_server_free_bytes(ntt_server_t sv, size_t* bytes) {
  if (!sv || !bytes) return fail(NTT_ERR_INVALID_ARG, "null server or bytes");
  *bytes = sv->adm.arena.free_bytes();
  return NTT_OK;
}
