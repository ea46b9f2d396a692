// ntt_host.h -- the host-only logic of the library: kernel-class rules of a stage shape,
// the plan's workspace layout, the server's arena allocator and its admission table.
// Nothing here touches a device or includes a HIP header, so this part also builds and
// runs as plain C++ (the sanitizer build of the host checks compiles it with g++).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "ntt.h"

namespace ntt {

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// FP64 scalars kept on the device per stage
enum { SCAL_NX2 = 0, SCAL_OBJ = 1, SCAL_MONITOR = 2, SCAL_OBJ0 = 3, SCAL_BCD_W2 = 4,
       SCAL_BCD_H2 = 5, SCAL_BCD_CORR = 6, SCAL_BCD_OBJ = 7, SCAL_COUNT = 8 };

// BCD NMF (Alg.3): state of one stage, in device memory, read and written by the kernels
// only (so that iterations replay from a captured graph).  Hb[cur] holds the kept H,
// Hb[prev] the kept H before it, Hb[nxt] receives the candidate; the three indices are
// always a permutation of 0, 1, 2.
struct BcdState {
  double t, obj;   // extrapolation sequence and the objective of the kept pair
  double wW, wH;   // extrapolation weights of the next iteration
  double gH, gW;   // ||H H^T||_F and ||W^T W||_F of the kept pair
  double gWn;      // ||W_n^T W_n||_F of the candidate W (the H step size 1/gWn)
  double pad0;
  int cur, prev, nxt, first, corrections, pad1[3];
};

// ---- kernel-class rules (which kernel takes an m x k, rank-r unfolding, and its grid)
int pass_L_class(int64_t m, int rp);  // -1 when m is beyond the row-split variant
int pass_L_waves(int cls);
// 16-column groups per step of the wide row-split update pass for a row class (0: the
// class has no wide pass); a wide stage's grid takes ceil(groups / 4) steps.
int pass_L_batch(int cls, int rp);
// Pass for m <= 4 rows: columns one workgroup takes per round.
int pass_tiny_cols(int64_t m);
// Row-chunked pass (m beyond one workgroup): rows per chunk.
int pass_C_rows(int rp);
// Whole stage in one workgroup (small unfoldings), and the 16-column groups its kernel
// instance holds (1, 2 or 4).
bool stage_1wg_ok(int64_t m, int64_t k, int r);
int stage_1wg_ng(int64_t k);
// Cooperative whole-stage kernel: eligibility, 16-column groups per workgroup, grid.
bool stage_coop_ok(int64_t m, int64_t k, int r);
int stage_coop_ng(int64_t k);
int stage_coop_grid(int64_t k, int ng);
// Column chunks of the BCD products for an m x k unfolding at rank r (G <= 1024).
void bcd_chunks(int64_t m, int64_t k, int r, int* G, int64_t* chunk);
// floats between the column chunks' partials of the BCD products
size_t bcd_part_stride(int64_t m, int r);
// Rank rule of Alg.2: split of the long side of the FP64 Gram of an m x k matrix (the
// shorter side's Gram) and the partials' size in doubles; the same for the m x m Gram of
// the rows whatever the shape.
void gram_plan(int64_t m, int64_t k, int* nsplit, size_t* part_doubles);
void gram_rows_plan(int64_t m, int64_t k, int* nsplit, size_t* part_doubles);

enum PassKind { PASS_S = 0, PASS_L = 1, PASS_GENERIC = 2, PASS_C = 3 };

struct Stage {
  int64_t m = 0, k = 0;
  int r = 0, rp = 16;
  bool fused = true;  // one X pass per iteration whose workgroups also sum the residual
                      // (PASS_S or PASS_L)
  int kind = PASS_S;
  int cls = 0;      // PASS_L: row class
  int mb = 1;       // PASS_S: 16-row blocks
  int nch = 0;      // PASS_C: row chunks
  bool pro_ok = false;  // the update pass can apply the W-update in its prologue (r <= 8 pass)
  bool pairs = false;  // PASS_L, PASS_C: column groups taken in pairs
  bool wide = false;   // PASS_L, PASS_S (r <= 8): update passes in 64-column steps
  bool tiny = false;   // PASS_S, m <= 4: update passes one column per lane (no MFMA)
  int G = 1;        // number of partials (pass workgroups or column chunks)
  int64_t chunk = 0;  // generic: columns per chunk
  bool bf16 = false;  // BF16 mode: this stage's X passes read a BF16 copy of X
  size_t part_stride = 0;  // floats between the per-workgroup partials of this stage
  // generic stages whose transposed problem (X^T = H^T W^T) fits the fused passes
  bool trans_ok = false;
  // the whole stage in one grid-synchronised launch (m <= 256, r <= 16, 64 < k <= 32768):
  // 16-column groups per workgroup and workgroups
  bool coop_ok = false;
  int coop_ng = 0, coop_G = 0;
  int G_pre = 1;          // transposed problem: column chunks of its first X H^T pass
  int64_t chunk_pre = 0;
};

void classify_stage(Stage& s, int precision);
// Classes of an m x k, rank-r stage (s) and of its transposed problem (t, when the stage
// iterates transposed: s.trans_ok).
void stage_shape(const ntt_config& cfg, int64_t m, int64_t k, int r, Stage& s, Stage& t);
// Column chunks of the generic X H^T partials.
void generic_chunks(const Stage& s, int* G, int64_t* chunk);

// Eq.(1)-(3) kernels: rows per block of the n_1...n_{d-1} x n_d matrix (64, or 128 for
// n_d < 64), column ranges per row block (more than one when there are few row blocks),
// and the blocks' FP64 partial pairs.
int tt_rows_per_block(int64_t nd);
int64_t tt_col_splits(int64_t rows, int64_t nd);
int64_t tt_blocks(int64_t rows, int64_t nd);

// ---- the plan: validated config, effective ranks, stage classes, workspace layout
struct Region {
  const char* name;
  size_t off, bytes;
};

struct PlanLayout {
  ntt_config cfg;
  int d = 0;
  int64_t dims[NTT_MAX_DIMS] = {};
  int64_t eff[NTT_MAX_DIMS + 1] = {};
  int64_t cap[NTT_MAX_DIMS + 1] = {};  // eff as planned (rank_eps > 0: the caps of the rule)
  Stage st[NTT_MAX_DIMS];
  Stage tst[NTT_MAX_DIMS];  // transposed problems of the stages with trans_ok
  double compression = 0.0;
  int64_t total_iters = 0;
  // workspace layout (bytes)
  size_t off_h[2] = {0, 0};
  size_t off_part = 0, part_stride = 0, off_rpart = 0, off_red = 0, off_gw = 0;
  size_t off_scal = 0, off_ints = 0, off_xb = 0, total = 0;
  size_t off_xt = 0, off_wp = 0, off_hp = 0;  // X^T, H^T, W^T of a transposed stage
  size_t off_s = 0;  // row-chunked stages: W^T X per row chunk, then a copy of H
  size_t off_wb = 0;  // prologue-mode stages: the second W buffer
  size_t off_gpart = 0;  // W-update over row blocks: per-block Gram parts
  // rank rule (rank_eps > 0): Gram partials, the Gram, eigenvalues, eigensolver workspace
  size_t off_grp = 0, off_gram = 0, off_eig = 0, off_eigws = 0, eigws_size = 0;
  // BCD (Alg.3): the two other H buffers, W before and candidate, X H^T and H H^T of the
  // kept H, W_n^T W_n, the state block
  size_t off_bh[2] = {0, 0}, off_bwp = 0, off_bwn = 0, off_bxh = 0, off_bhh = 0, off_bgw = 0, off_bst = 0;
  // stage 1 streamed from host memory (stream_cols > 0): column blocks of kblk columns,
  // their shapes (full blocks, last block), the staging buffers of X and H, the reduced
  // products of one block, and per-block sums
  int64_t kblk = 0, nblk = 0;
  Stage sst[2];
  size_t off_xs = 0, off_hs = 0, off_redtmp = 0, off_bsum = 0, off_gram2 = 0;
  size_t off_coop = 0;  // barrier flags of the cooperative stage (32 per workgroup)
  std::vector<Region> regions;  // every workspace region in layout order
};

// Fixed-order sum of the first workgroups' residual partials needs at least this many
// slots (the norm of X uses them too).
constexpr int kSumsqBlocks = 1024;

// Validate cfg (the rules of ntt_plan in ntt.h), fix the effective ranks, classify every
// stage and lay out the workspace.  On an error, *err gets the reason.
ntt_status plan_layout(const ntt_config* cfg, PlanLayout* p, std::string* err);
// Eq.(4): prod n_i / sum n_i r_{i-1} r_i
double compression_of(int d, const int64_t* dims, const int64_t* ranks);

// ---- serving: first-fit allocator over the device arena (offsets only; 256-byte units)
struct Arena {
  size_t size = 0;
  std::vector<std::pair<size_t, size_t>> free_list;  // (offset, bytes), sorted by offset
  void init(size_t n);
  bool alloc(size_t n, size_t* off);
  void release(size_t off, size_t n);
  size_t free_bytes() const;
};

// The admission rule of a server tick: the head request is admitted while a slot is free
// and both of its arena blocks (cores; input + workspace) fit, FIFO.
struct Admission {
  Arena arena;
  std::vector<char> slot_used;
  void init(size_t arena_bytes, int slots);
  // true with a slot and both offsets taken; false with nothing taken
  bool admit(size_t bytes_cores, size_t bytes_work, int* slot, size_t* off_c, size_t* off_w);
};

}  // namespace ntt
