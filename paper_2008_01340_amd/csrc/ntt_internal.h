// ntt_internal.h -- kernel argument blocks and launchers shared by the library sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ntt.h"
#include "ntt_host.h"

namespace ntt {

// One MU pass over the columns of an m x k unfolding.
struct PassArgs {
  const float* X;       // m x k, row stride k
  const uint16_t* Xb;   // BF16 shadow of X (read instead of X when not NULL)
  float* H;             // r x k, row stride k (updated in place)
  const float* W;       // m x r
  const float* GW;      // RP x RP, W^T W zero padded
  float* part;          // per-workgroup partials: [m][r] X H^T, then [r][r] H H^T
  int64_t part_stride;  // floats between workgroups' partials
  double* rpart;        // per-workgroup residual sums (FP64)
  int m, r;
  int64_t k;
  float eps;
  float* S;             // row-chunked pass: W^T X of each row chunk, nchunks x r x k floats
  int nchunks;          // row-chunked pass: number of row chunks
  float* Hs;            // row-chunked pass: copy of H taken in phase 1, read in phase 2 (r x k)
  int pair_groups;      // row-split and row-chunked passes: take column groups in pairs
  // W-update in the prologue (r <= 8 pass): when Wprev is not NULL, the pass first forms
  // W = max(0, Wprev .* N_W ./ (Wprev G_H + eps)) and G_W = W^T W from red (N_W = X H^T as
  // m x r, then G_H = H H^T as r x r, FP64) and uses them instead of W and GW; workgroup 0
  // also stores W to Wout.
  const float* Wprev;
  float* Wout;
  const double* red;
};

// Reduction of the pass partials and the W-update.
struct FinArgs {
  const float* part;
  int64_t part_stride;
  int G;           // number of partials
  int m, r;
  double* red;     // reduced X H^T (m x r) then H H^T (r x r), FP64
  float* W;        // m x r, updated in place
  float* GW;       // RP x RP, receives W'^T W'
  double* scal;    // SCAL_* scalars
  const double* rpart;  // residual partials of this pass (NULL when none)
  double* trace;   // where to store the residual objective (NULL: do not store)
  float eps;
  float* Wout;     // where the new W goes (NULL: W is updated in place)
  double* gpart;   // m > 256: per-block parts of W'^T W' and <W', X H^T>, ceil(m/256) x (32*32+1)
  unsigned* arrive;  // m > 256: arrival counter of the W-update's blocks (zero between launches)
};

// A whole stage of MU iterations in one workgroup (small unfoldings).
struct StageArgs {
  const float* X;  // m x k
  float* W;        // m x r, read at entry, written at exit
  float* H;        // r x k, read at entry, written at exit
  int m, r, k, iters;
  float eps;
};

// A whole stage of MU iterations in one grid-synchronised launch (m <= 256, r <= 16, k <= 32768):
// G workgroups of 16 NG columns each, X and H on chip for all iterations.
struct CoopArgs {
  const float* X;    // m x k
  float* W;          // m x r, read at entry, written at exit
  float* H;          // r x k, read at entry, written at exit
  float* GW;         // 16 x 16 W^T W (FP32), read at entry, written at exit
  float* part;       // G x (m r + r r) partials
  double* red;       // m r + r r sums (FP64)
  unsigned* flags;   // barrier flags, 32 per workgroup (zeroed by the launcher)
  int* status;       // set to 1 when a barrier timed out
  int m, r;
  int64_t k;
  int iters;
  float eps;
};

// Work-list of up to NTT_STAGE_LIST small stages passed by value as a kernel argument.
#define NTT_STAGE_LIST 64
struct StageList {
  int count;
  StageArgs a[NTT_STAGE_LIST];
};
static_assert(sizeof(StageList) <= 4096, "work-list must fit the kernel argument segment");

// TT expansion (Eq.(2)) over the rows of the (n_1...n_{d-1}) x n_d matrix.
struct TTArgs {
  int d;
  int64_t rows;
  int64_t dims[NTT_MAX_DIMS];
  int ranks[NTT_MAX_DIMS + 1];
  const float* cores[NTT_MAX_DIMS];
  const float* A;  // MODE 1 input
  float* out;      // MODE 0 output
  double* part;    // MODE 1 per-block (err, ref) pairs, then the two totals
};

struct BcdArgs {
  const float* X;    // m x k, row stride k
  float* Hb[3];      // three r x k buffers; Hb[0] is the stage's H (the result goes there)
  float* W;          // m x r, the kept W (the stage's core buffer)
  float* Wp;         // m x r, the kept W before it
  float* Wn;         // m x r, the candidate W
  double* XHc;       // m x r, X H^T of the kept H
  double* HHc;       // r x r, H H^T of the kept H
  float* GWn;        // 32 x 32 zero padded, W_n^T W_n (FP32, for the H step)
  BcdState* st;
  float* part;       // X H^T, H H^T partials per column chunk ([m][r] then [r][r])
  int64_t part_stride;
  int G;             // column chunks
  int64_t chunk;     // columns per chunk (multiple of 64)
  double* red;       // the reduced partials (m r + r r), FP64
  double* rpart;     // residual partials, G x ceil(m / 64)
  double* scal;      // the stage's SCAL_* scalars
  double* trace;     // where the step stores the candidate's objective (NULL: nowhere)
  int m, r;
  int64_t k;
  double delta;      // extrapolation cap
};
// Stage set-up: scale W and Hb[0] to Frobenius norm sqrt(||X||_F) (scal[SCAL_NX2] must
// hold ||X||^2), reset the state and form X H^T, H H^T of the initial H.
hipError_t launch_bcd_prepare(const BcdArgs& b, hipStream_t s);
// One iteration: decision on the previous candidate and the W step, the H step, the
// products of the new candidate and their reduction.
hipError_t launch_bcd_iter(const BcdArgs& b, hipStream_t s);
// End of the stage: decision on the last candidate; the kept H goes to Hb[0] and the
// number of dropped iterations to scal[SCAL_BCD_CORR].
hipError_t launch_bcd_finish(const BcdArgs& b, hipStream_t s);

hipError_t launch_init_uniform(float* out, int64_t n, uint64_t seed, uint64_t tag, hipStream_t s);
hipError_t launch_copy(float* dst, const float* src, int64_t n, hipStream_t s);
hipError_t launch_cast_bf16(uint16_t* dst, const float* src, int64_t n, hipStream_t s);
hipError_t launch_transpose(const float* src, float* dst, int64_t rows, int64_t cols, hipStream_t s);
hipError_t launch_sumsq(const float* x, int64_t n, double* part, int nblocks, int* flags,
                        int validate, double* out, hipStream_t s);
hipError_t launch_gram_w(const float* W, int m, int r, int rp, float* G, hipStream_t s);
hipError_t launch_pass_fused(const PassArgs& a, int rp, int mb, int grid, bool update, bool resid,
                             bool wide, hipStream_t s);
// Update pass for m <= 4 rows (one column per lane, no MFMA); grid: any number of
// workgroups, each taking pass_tiny_cols(m) columns per round.
hipError_t launch_pass_tiny(const PassArgs& a, int grid, hipStream_t s);
// wide: update passes by the wide pass (a residual with them runs the per-group pass
// first); otherwise every pass by the per-group row-split pass
hipError_t launch_pass_L(const PassArgs& a, int rp, int cls, int grid, bool update, bool resid,
                         bool wide, hipStream_t s);
// Row-chunked pass (m beyond one workgroup; rows per chunk in ntt_host.h): the launches of one
// iteration (phase 1, chunk sum, phase 2) or of the residual (phase 0) on a
// (G, nchunks) grid.  S holds nchunks x r x k floats, Hs r x k.
hipError_t launch_pass_C(const PassArgs& a, int rp, int G, bool update, bool resid, hipStream_t s);
hipError_t launch_stage_1wg(const StageArgs& a, hipStream_t s);
hipError_t launch_stage_1wg_grouped(const StageArgs* list_dev, int count, int ng, hipStream_t s);
hipError_t launch_stage_1wg_list(const StageList& L, int ng, hipStream_t s);
// the grouped kernel instance for ng groups (a graph kernel node's function); its list
// may be empty (the node then runs one workgroup that returns at once)
const void* stage_1wg_list_kernel(int ng);
// Cooperative whole-stage kernel (eligibility and grid in ntt_host.h): the largest grid the
// device holds at once for an instance (0 when unknown), and the launch.
int stage_coop_max_grid(int ng);
hipError_t launch_stage_coop(const CoopArgs& c, int ng, int G, hipStream_t s);
hipError_t launch_pass_generic(const PassArgs& a, int rp, int gxht, int64_t chunk, bool update,
                               bool resid, hipStream_t s);
// X H^T and H H^T partials alone (column chunks of `chunk`), as the generic pass writes them
hipError_t launch_xht_partials(const PassArgs& a, int rp, int gxht, int64_t chunk, hipStream_t s);
hipError_t launch_finalize(const FinArgs& f, int rp, hipStream_t s);
// The partial reduction of launch_finalize alone (into f.red), for passes that apply the
// W-update in their prologue.
hipError_t launch_reduce(const FinArgs& f, hipStream_t s);
// The W-update of launch_finalize alone, from the reduced partials in f.red.
hipError_t launch_wupdate_red(const FinArgs& f, hipStream_t s);
hipError_t launch_zero_ints(int* p, int64_t n, hipStream_t s);
// acc = src (first != 0) or acc += src over n doubles
hipError_t launch_add_doubles(double* acc, const double* src, int64_t n, int first, hipStream_t s);
// out[0] = scale * (fixed-order sum of part[0..n))
hipError_t launch_sum_doubles(const double* part, int n, double scale, double* out, hipStream_t s);
hipError_t launch_resid_sum(const double* rpart, int G, double* obj, double* trace, hipStream_t s);
hipError_t launch_tt_expand(const TTArgs& t, int mode, hipStream_t s);

// Rank rule of Alg.2: FP64 Gram of the shorter side of X (m x k, row-major): G = X X^T
// (n = m) when m <= k, else X^T X (n = k); G is n x n, row-major, both triangles.  The
// long dimension is split into nsplit chunks whose partials (npairs x nsplit blocks of
// 64 x 64 doubles in `part`) are added in chunk order (gram_plan: the split and the
// partial size in doubles for an m x k matrix).
hipError_t launch_gram(const float* X, int64_t m, int64_t k, double* part, double* G, hipStream_t s);
// The m x m Gram X X^T whatever the shape (a column block of a streamed unfolding; the
// blocks' Grams are added by the caller; split and partial size by gram_rows_plan).
hipError_t launch_gram_rows(const float* X, int64_t m, int64_t k, double* part, double* G, hipStream_t s);

}  // namespace ntt
