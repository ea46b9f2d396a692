// ntt_host.cpp -- host-only logic: kernel-class rules, the plan's validation and workspace
// layout, the serving arena and admission.  Plain C++ (no device calls, no HIP headers).

#include "ntt_host.h"

#include <algorithm>
#include <cmath>

namespace ntt {

namespace {

constexpr int kMaxPassBlocks = 1024;  // persistent grid of the fused pass
// grid cap of the row-split pass over at most 64 rows (three 256-thread workgroups per CU
// are resident at its register use: one full round on 256 CUs); the classes of 65..256
// rows (two 4-wave workgroups per CU) and the 8-wave classes take one round of 512
constexpr int kMaxLBlocks = 768;
// grid cap of the r <= 8 pass in 64-column steps over 32 rows (two workgroups per CU at
// its register use)
constexpr int kR8WCap = 512;
// fewest 64-column steps (four 16-column groups) for the batched row-split update pass
constexpr int64_t kLWMinSteps = 256;


}  // namespace

// ------------------------------------------------------------------ kernel-class rules
int pass_L_class(int64_t m, int rp) {
  if (m <= 64) return 0;
  if (m <= 128) return 1;
  if (m <= 256) return 2;
  if (m <= 512) return 3;
  if (m <= 1024 && rp == 16) return 4;
  return -1;
}

int pass_L_waves(int cls) { return cls <= 2 ? 4 : 8; }

int pass_L_batch(int cls, int rp) { return (rp == 16 && cls >= 0 && cls <= 3) ? 4 : 0; }

// 256 threads, one column each, 4 columns per thread
int pass_tiny_cols(int64_t m) {
  (void)m;
  return 1024;
}

// chunks of 512 rows, 8 waves of 64 rows (both paddings)
int pass_C_rows(int rp) {
  (void)rp;
  return 512;
}

bool stage_1wg_ok(int64_t m, int64_t k, int r) { return m <= 256 && k <= 64 && r <= 16; }

int stage_1wg_ng(int64_t k) { return k <= 16 ? 1 : (k <= 32 ? 2 : 4); }

int stage_coop_ng(int64_t k) {
  const int64_t per = (k + 127) / 128;  // workgroups at 8 groups each
  if (per <= 16) return (k + 15) / 16 <= 128 ? 1 : 2;
  if (per <= 32) return 2;
  if (per <= 64) return 4;
  return 8;
}

int stage_coop_grid(int64_t k, int ng) { return (int)((k + 16 * ng - 1) / (16 * ng)); }

bool stage_coop_ok(int64_t m, int64_t k, int r) {
  return m >= 1 && m <= 256 && r >= 1 && r <= 16 && k > 64 && k <= 256 * 128;
}

void bcd_chunks(int64_t m, int64_t k, int r, int* G, int64_t* chunk) {
  // about a quarter of X's size in partials at most; up to 1024 chunks of >= 64 columns
  const double E = (double)m * r + (double)r * r;
  const int64_t cap = std::max<int64_t>(1, (int64_t)(0.25 * (double)m * (double)k / E));
  const int64_t want = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>((k + 63) / 64, 1024), cap));
  int64_t c = (k + want - 1) / want;
  c = (c + 63) / 64 * 64;
  *chunk = c;
  *G = (int)((k + c - 1) / c);
}

void gram_plan(int64_t m, int64_t k, int* nsplit, size_t* part_doubles) {
  const int64_t n = std::min(m, k), L = std::max(m, k);
  const int64_t nb = (n + 63) / 64;
  const int64_t npairs = nb * (nb + 1) / 2;
  // about 1024 workgroups, each chunk at least 1024 long-side indices
  int64_t ns = std::max<int64_t>(1, std::min<int64_t>(1024 / npairs, (L + 1023) / 1024));
  *nsplit = (int)ns;
  *part_doubles = (size_t)npairs * (size_t)ns * 4096;
}

void gram_rows_plan(int64_t m, int64_t k, int* nsplit, size_t* part_doubles) {
  const int64_t nb = (m + 63) / 64;
  const int64_t npairs = nb * (nb + 1) / 2;
  int64_t ns = std::max<int64_t>(1, std::min<int64_t>(1024 / npairs, (k + 1023) / 1024));
  *nsplit = (int)ns;
  *part_doubles = (size_t)npairs * (size_t)ns * 4096;
}

int tt_rows_per_block(int64_t nd) { return nd < 64 ? 128 : 64; }

// about 2048 blocks in all when the rows alone give fewer, each column range at least
// 1024 columns
int64_t tt_col_splits(int64_t rows, int64_t nd) {
  const int rpb = tt_rows_per_block(nd);
  const int64_t rb = (rows + rpb - 1) / rpb;
  if (rb >= 2048 || nd <= 1024) return 1;
  return std::max<int64_t>(1, std::min<int64_t>({(2048 + rb - 1) / rb, (nd + 1023) / 1024, 65535}));
}

int64_t tt_blocks(int64_t rows, int64_t nd) {
  const int rpb = tt_rows_per_block(nd);
  return (rows + rpb - 1) / rpb * tt_col_splits(rows, nd);
}

// ------------------------------------------------------------------ stage classes
// Pass kind, row class and workgroup count of an m x k, rank-r problem.
void classify_stage(Stage& s, int precision) {
  s.rp = s.r <= 16 ? 16 : 32;
  const int64_t ngroups = (s.k + 15) / 16;
  const double Ed = (double)s.m * s.r + (double)s.r * s.r;
  // partials cost G E floats per iteration: keep them within ~10% of the X bytes,
  // but use at least 256 workgroups when there are that many groups
  const int64_t gcap = std::max<int64_t>(
      256, std::min<int64_t>(kMaxPassBlocks, (int64_t)(0.1 * (double)s.m * (double)s.k / Ed)));
  s.cls = pass_L_class(s.m, s.rp);
  if (s.m <= 32) {
    // one wavefront per 16-column group with all rows in registers (one or two 16-row
    // blocks): no per-group barrier or cross-wave sum
    s.kind = PASS_S;
    s.mb = s.m <= 16 ? 1 : 2;
    // a grid of one resident round (workgroups per CU x 256 CUs) avoids a partly filled
    // second round: three per CU for the r <= 8 pass
    int64_t cap = gcap;
    if (s.r <= 8) cap = std::min<int64_t>(gcap, 768);
    // the r <= 8 pass in 64-column steps (one per wave) once there are enough of them
    s.wide = s.r <= 8 && ngroups >= 4 * 4 * 256;
    const int64_t units = s.wide ? ((ngroups + 3) / 4 + 3) / 4 : (ngroups + 3) / 4;
    if (s.wide && s.mb == 2) cap = std::min<int64_t>(cap, kR8WCap);
    s.G = (int)std::max<int64_t>(1, std::min<int64_t>(units, cap));
    // at most 4 rows (then r <= 4): the update passes take one column per lane on the
    // VALU once there are enough columns; the partials (m r + r r <= 32 floats per
    // workgroup) stay far below the X bytes at up to 1024 workgroups
    if (s.m <= 4 && ngroups >= 256) {
      s.tiny = true;
      s.wide = false;
      s.G = (int)std::max<int64_t>(
          1, std::min<int64_t>(kMaxPassBlocks, (s.k + pass_tiny_cols(s.m) - 1) / pass_tiny_cols(s.m)));
    }
  } else if (s.cls >= 0) {
    s.kind = PASS_L;
    // the batched update pass takes B whole groups per step; otherwise column groups
    // in pairs once there are enough of them
    // (the wide pass's 64-column steps leave too few workgroups below ~256 steps)
    const int nb = ngroups >= 4 * kLWMinSteps ? pass_L_batch(s.cls, s.rp) : 0;
    s.wide = nb > 0;
    s.pairs = nb == 0 && ngroups >= 512;
    const int64_t units = nb > 0 ? (ngroups + nb - 1) / nb : (s.pairs ? (ngroups + 1) / 2 : ngroups);
    // one resident round of workgroups; partials up to ~25% of the X bytes
    // (65..256 rows: two workgroups per CU; 768 workgroups left a half-filled second
    // round: the 256^4 stage 1 took 446 ms at 768, 425 ms at 512)
    const int64_t gcap_l = std::max<int64_t>(
        256, std::min<int64_t>(s.cls == 0 ? kMaxLBlocks : 512,
                               (int64_t)(0.25 * (double)s.m * (double)s.k / Ed)));
    s.G = (int)std::max<int64_t>(1, std::min<int64_t>(units, gcap_l));
  } else if ((s.m + pass_C_rows(s.rp) - 1) / pass_C_rows(s.rp) <= 65535) {
    s.kind = PASS_C;
    s.nch = (int)((s.m + pass_C_rows(s.rp) - 1) / pass_C_rows(s.rp));
    s.pairs = ngroups >= 512;
    // the (G, nchunks) grid has enough workgroups at G = 128, or at G nchunks >= 1024
    // when there are many row chunks; more only adds partials (G (m r + r r) floats
    // written and reduced per iteration, kept near 10% of the X bytes above that floor)
    const int64_t gfloor = std::min<int64_t>(128, (1024 + s.nch - 1) / s.nch);
    int64_t gcap_c = std::max<int64_t>(
        gfloor, std::min<int64_t>(1024, (int64_t)(0.1 * (double)s.m * (double)s.k / Ed)));
    // up to 64 partials are reduced one thread per entry with every load in flight; a grid
    // of 65..128 column chunks gains less in the pass than its slower reduction costs
    // (128^4 stage 2, 2048 x 16384: 64 chunks 18.1 ms, 101 21.4 ms, 128 20.4 ms), while
    // far larger grids pay off (256^4 stage 2, 2560 x 65536: 652 chunks 41.6 ms, 64 57.2
    // ms); the (64, chunks) grid keeps at least 256 workgroups from 4 chunks on
    if (gcap_c <= 128 && s.nch >= 4) gcap_c = std::min<int64_t>(gcap_c, 64);
    s.G = (int)std::max<int64_t>(1, std::min<int64_t>(s.pairs ? (ngroups + 1) / 2 : ngroups, gcap_c));
  } else {
    s.kind = PASS_GENERIC;
  }
  s.fused = s.kind == PASS_S || s.kind == PASS_L;
  // (a prologue in the wide row-split pass was measured slower than the separate
  // W-update launch: every workgroup waits for it before its first load)
  s.pro_ok = s.kind == PASS_S && s.r <= 8 && s.m <= 32 && !s.tiny;
  // BF16 X is read by the S passes at rank padding 16, the row-split and the row-chunked
  // passes; stages the single-workgroup kernel takes (small unfoldings), the S pass at
  // padding 32 and the generic path stay FP32
  s.bf16 = precision == NTT_PREC_BF16_MIXED && !stage_1wg_ok(s.m, s.k, s.r) &&
           (s.kind == PASS_L || s.kind == PASS_C || (s.kind == PASS_S && s.rp == 16));
  const size_t E = (size_t)s.m * s.r + (size_t)s.r * s.r;
  s.part_stride = align_up(E, 64);
}

void stage_shape(const ntt_config& cfg, int64_t m, int64_t k, int r, Stage& s, Stage& t) {
  s = Stage{};
  t = Stage{};
  s.m = m;
  s.k = k;
  s.r = r;
  classify_stage(s, cfg.precision);
  if (s.kind == PASS_GENERIC) generic_chunks(s, &s.G, &s.chunk);
  s.coop_ok = stage_coop_ok(m, k, r);
  if (s.coop_ok) {
    s.coop_ng = stage_coop_ng(k);
    s.coop_G = stage_coop_grid(k, s.coop_ng);
  }
  if (!s.fused) {
    // X^T (k x m) ~ H^T W^T: the MU iterations of the transposed problem are those of
    // this one shifted by half a step, and its rows (k) may fit the fused passes
    Stage u{};
    u.m = s.k;
    u.k = s.m;
    u.r = s.r;
    classify_stage(u, cfg.precision);
    if (u.fused && cfg.tol == 0.0 && cfg.max_iters >= 1 && !stage_1wg_ok(u.m, u.k, u.r)) {
      generic_chunks(u, &u.G_pre, &u.chunk_pre);
      s.trans_ok = true;
      t = u;
    }
  }
}

// Column chunks of the generic X H^T partials: enough for parallelism, while their
// G (m r + r r) floats stay within ~1/4 of the X bytes.
size_t bcd_part_stride(int64_t m, int r) { return align_up((size_t)m * r + (size_t)r * r, 64); }

void generic_chunks(const Stage& s, int* G, int64_t* chunk) {
  const double Ed = (double)s.m * s.r + (double)s.r * s.r;
  const int64_t gcap_gen = std::max<int64_t>(1, (int64_t)(0.25 * (double)s.m * (double)s.k / Ed));
  const int64_t want = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>((s.k + 255) / 256, 256), gcap_gen));
  *chunk = (int64_t)align_up((size_t)((s.k + want - 1) / want), 64);
  *G = (int)((s.k + *chunk - 1) / *chunk);
}


// ------------------------------------------------------------------ plan layout
double compression_of(int d, const int64_t* dims, const int64_t* ranks) {
  double num = 1.0, den = 0.0;
  for (int i = 0; i < d; ++i) {
    num *= (double)dims[i];
    den += (double)dims[i] * (double)ranks[i] * (double)ranks[i + 1];
  }
  return num / den;
}

ntt_status plan_layout(const ntt_config* cfg, PlanLayout* p, std::string* err) {
  auto fail = [&](ntt_status st, const std::string& msg) {
    *err = msg;
    return st;
  };
  if (!cfg) return fail(NTT_ERR_INVALID_ARG, "null config");
  const int d = cfg->d;
  if (d < 2 || d > NTT_MAX_DIMS) return fail(NTT_ERR_INVALID_ARG, "d must be in 2..16");
  if (!cfg->dims || !cfg->ranks) return fail(NTT_ERR_INVALID_ARG, "null dims or ranks");
  if (cfg->max_iters < 0) return fail(NTT_ERR_INVALID_ARG, "max_iters < 0");
  if (cfg->check_every < 1) return fail(NTT_ERR_INVALID_ARG, "check_every < 1");
  if (!(cfg->eps >= 0.0) || !std::isfinite(cfg->eps)) return fail(NTT_ERR_INVALID_ARG, "eps must be finite and >= 0");
  if (!(cfg->tol >= 0.0) || !std::isfinite(cfg->tol)) return fail(NTT_ERR_INVALID_ARG, "tol must be finite and >= 0");
  if (cfg->precision != NTT_PREC_FP32 && cfg->precision != NTT_PREC_BF16_MIXED)
    return fail(NTT_ERR_INVALID_ARG, "unknown precision");
  if (cfg->fp32_tail_iters < 0) return fail(NTT_ERR_INVALID_ARG, "fp32_tail_iters < 0");
  if (!(cfg->rank_eps >= 0.0) || !std::isfinite(cfg->rank_eps))
    return fail(NTT_ERR_INVALID_ARG, "rank_eps must be finite and >= 0");
  const bool eps_mode = cfg->rank_eps > 0.0;
  if (cfg->nmf != NTT_NMF_MU && cfg->nmf != NTT_NMF_BCD) return fail(NTT_ERR_INVALID_ARG, "unknown nmf");
  const bool bcd = cfg->nmf == NTT_NMF_BCD;
  if (bcd) {
    if (cfg->precision != NTT_PREC_FP32) return fail(NTT_ERR_INVALID_ARG, "BCD runs in FP32 only");
    if (cfg->tol != 0.0) return fail(NTT_ERR_INVALID_ARG, "BCD runs a fixed iteration count (tol = 0)");
    if (!(cfg->bcd_delta >= 0.0 && cfg->bcd_delta < 1.0))
      return fail(NTT_ERR_INVALID_ARG, "bcd_delta must be in [0, 1)");
  }
  if (cfg->stream_cols < 0) return fail(NTT_ERR_INVALID_ARG, "stream_cols < 0");
  const bool streamed = cfg->stream_cols > 0;
  if (streamed && (bcd || cfg->precision != NTT_PREC_FP32 || cfg->tol != 0.0 ||
                   (cfg->flags & NTT_RECORD_OBJECTIVE)))
    return fail(NTT_ERR_INVALID_ARG, "stream_cols: MU in FP32, tol = 0 and no objective trace");
  int64_t total = 1;
  for (int i = 0; i < d; ++i) {
    if (cfg->dims[i] < 1) return fail(NTT_ERR_INVALID_ARG, "dims must be >= 1");
    // at most 2^44 entries (64 TiB of floats): every workspace size below stays far from
    // the range of size_t
    if (total > ((int64_t)1 << 44) / cfg->dims[i])
      return fail(NTT_ERR_INVALID_ARG, "tensor too large (more than 2^44 entries)");
    total *= cfg->dims[i];
  }
  if (cfg->ranks[0] != 1 || cfg->ranks[d] != 1) return fail(NTT_ERR_INVALID_ARG, "r_0 and r_d must be 1");
  for (int i = 1; i < d; ++i)
    if (cfg->ranks[i] < 1) return fail(NTT_ERR_INVALID_ARG, "inner ranks must be >= 1");

  p->cfg = *cfg;
  p->cfg.dims = nullptr;
  p->cfg.ranks = nullptr;
  p->d = d;
  for (int i = 0; i < d; ++i) p->dims[i] = cfg->dims[i];
  // effective ranks: r_l <= min(r_{l-1} n_l, n_{l+1}...n_d), left to right
  p->eff[0] = 1;
  for (int l = 1; l < d; ++l) {
    const int64_t m = p->eff[l - 1] * p->dims[l - 1];
    int64_t k = 1;
    for (int j = l; j < d; ++j) k *= p->dims[j];
    const int64_t r = std::min(cfg->ranks[l], std::min(m, k));
    if (r != cfg->ranks[l] && (cfg->flags & NTT_STRICT_RANKS))
      return fail(NTT_ERR_RANK_INFEASIBLE, "rank " + std::to_string(l) + " exceeds min(r_{l-1} n_l, n_{l+1}..n_d)");
    if (r > NTT_MAX_RANK)
      return fail(NTT_ERR_INVALID_ARG, "effective rank above NTT_MAX_RANK (32)");
    p->eff[l] = r;
  }
  p->eff[d] = 1;
  for (int i = 0; i <= d; ++i) p->cap[i] = p->eff[i];
  p->compression = compression_of(d, p->dims, p->eff);

  // stages and workspace
  size_t hsize[2] = {0, 0};
  size_t xb_size = 0;
  size_t part_floats = 0;
  int gmax = 1, gfin = 1;
  int64_t gres = 1;  // residual partial slots (doubles)
  size_t red_max = 0;
  size_t xt_size = 0, wp_size = 0, hp_size = 0, s_size = 0, wb_size = 0;
  int64_t m_max = 1;
  size_t grp_max = 0, gram_max = 0;
  int64_t n_max = 0;
  size_t bh_size = 0, bm_size = 0;  // BCD: one H buffer, one m x r factor (elements)
  // one stage shape: its classes (kept in s, t) and its share of the workspace maxima
  auto plan_stage = [&](int l, int64_t m, int64_t k, int r, Stage& s, Stage& t_out) {
    stage_shape(*cfg, m, k, r, s, t_out);
    if (s.kind == PASS_GENERIC) gres = std::max<int64_t>(gres, (s.k + 255) / 256);  // residual blocks
    if (s.kind == PASS_C) {
      gres = std::max<int64_t>(gres, (int64_t)s.G * s.nch);
      s_size = std::max(s_size, (size_t)(s.nch + 1) * (size_t)s.r * (size_t)s.k * sizeof(float));
    }
    if (s.trans_ok) {
      const Stage& t = t_out;
      {
        part_floats = std::max(part_floats, (size_t)std::max(t.G, t.G_pre) * t.part_stride);
        red_max = std::max(red_max, (size_t)t.m * t.r + (size_t)t.r * t.r);
        gres = std::max<int64_t>(gres, t.G);
        gfin = std::max(gfin, std::max(t.G, t.G_pre));
        xt_size = std::max(xt_size, (size_t)s.m * (size_t)s.k * sizeof(float));
        wp_size = std::max(wp_size, (size_t)s.k * (size_t)s.r * sizeof(float));
        hp_size = std::max(hp_size, (size_t)s.r * (size_t)s.m * sizeof(float));
        if (t.bf16) xb_size = std::max(xb_size, (size_t)s.m * (size_t)s.k * sizeof(uint16_t));
      }
    }
    const size_t E = (size_t)s.m * s.r + (size_t)s.r * s.r;
    red_max = std::max(red_max, E);
    m_max = std::max(m_max, s.m);
    if (s.trans_ok) m_max = std::max(m_max, t_out.m);
    gmax = std::max(gmax, s.G);
    gfin = std::max(gfin, s.G);
    part_floats = std::max(part_floats, (size_t)s.G * s.part_stride);
    if (s.coop_ok) part_floats = std::max(part_floats, (size_t)s.coop_G * E);
    if (l < d - 1) {
      const size_t hb = (size_t)s.r * (size_t)s.k * sizeof(float);
      hsize[(l - 1) & 1] = std::max(hsize[(l - 1) & 1], hb);
    }
    if (s.bf16) xb_size = std::max(xb_size, (size_t)s.m * (size_t)s.k * sizeof(uint16_t));
    if (s.pro_ok) wb_size = std::max(wb_size, (size_t)s.m * (size_t)s.r * sizeof(float));
    if (bcd) {
      int G = 1;
      int64_t chunk = 64;
      bcd_chunks(s.m, s.k, s.r, &G, &chunk);
      part_floats = std::max(part_floats, (size_t)G * bcd_part_stride(s.m, s.r));
      gres = std::max<int64_t>(gres, (int64_t)G * ((s.m + 63) / 64));
      gfin = std::max(gfin, G);
      bh_size = std::max(bh_size, (size_t)s.r * (size_t)s.k);
      bm_size = std::max(bm_size, (size_t)s.m * (size_t)s.r);
    }
    if (eps_mode) {
      int ns = 1;
      size_t pd = 0;
      gram_plan(s.m, s.k, &ns, &pd);
      const int64_t n = std::min(s.m, s.k);
      grp_max = std::max(grp_max, pd);
      gram_max = std::max(gram_max, (size_t)n * (size_t)n);
      n_max = std::max(n_max, n);
    }
  };
  for (int l = 1; l < d; ++l) {
    int64_t k = 1;
    for (int j = l; j < d; ++j) k *= p->dims[j];
    plan_stage(l, p->eff[l - 1] * p->dims[l - 1], k, (int)p->eff[l], p->st[l - 1], p->tst[l - 1]);
    if (eps_mode) {
      // the rule may choose any r_{l-1} <= cap and r_l <= cap: plan the workspace for all
      for (int64_t rp_ = 1; rp_ <= p->eff[l - 1]; ++rp_)
        for (int64_t r_ = 1; r_ <= p->eff[l]; ++r_) {
          const int64_t m_ = rp_ * p->dims[l - 1];
          if (r_ > std::min(m_, k)) continue;
          Stage s2{}, t2{};
          plan_stage(l, m_, k, (int)r_, s2, t2);
        }
    }
    p->total_iters += cfg->max_iters;
  }
  if (streamed) {
    // stage 1 in column blocks: the full blocks' shape and the last block's
    const int64_t m1 = p->dims[0], k1 = total / p->dims[0];
    const int64_t kb = std::min<int64_t>(cfg->stream_cols, k1);
    p->kblk = kb;
    p->nblk = (k1 + kb - 1) / kb;
    Stage tt{};
    const int64_t last = k1 - (p->nblk - 1) * kb;
    plan_stage(1, m1, kb, (int)p->eff[1], p->sst[0], tt);
    plan_stage(1, m1, last, (int)p->eff[1], p->sst[1], tt);
    if (eps_mode) {
      // the rule may choose any r_1 up to the cap: the block stages at every rank; the
      // Gram of X_1 is the n_1 x n_1 sum of the blocks' row Grams
      for (int64_t r_ = 1; r_ < p->eff[1]; ++r_) {
        Stage s2{};
        plan_stage(1, m1, kb, (int)r_, s2, tt);
        plan_stage(1, m1, last, (int)r_, s2, tt);
      }
      for (int64_t w : {kb, last}) {
        int ns = 1;
        size_t pd = 0;
        gram_rows_plan(m1, w, &ns, &pd);
        grp_max = std::max(grp_max, pd);
      }
      gram_max = std::max(gram_max, (size_t)m1 * (size_t)m1);
      n_max = std::max(n_max, m1);
    }
  }
  if (bcd && m_max > 64 * 65535)
      return fail(NTT_ERR_INVALID_ARG, "BCD: an unfolding has more than 4194240 rows");
  if (eps_mode && n_max > 2048)
      return fail(NTT_ERR_INVALID_ARG, "rank_eps: an unfolding's shorter side exceeds 2048");
  gres = std::max<int64_t>(std::max<int64_t>(gres, gmax), kSumsqBlocks);
  size_t off = 0;
  p->regions.clear();
  auto place = [&](const char* name, size_t bytes) {
    const size_t at = off;
    p->regions.push_back(Region{name, at, bytes});
    off = align_up(off + bytes, 256);
    return at;
  };
  p->off_h[0] = place("off_h[0]", hsize[0]);
  p->off_h[1] = place("off_h[1]", hsize[1]);
  p->off_part = place("off_part", part_floats * sizeof(float));
  p->off_rpart = place("off_rpart", (size_t)gres * sizeof(double));
  p->off_red = place("off_red", red_max * sizeof(double));
  if (gfin > 1024)
      return fail(NTT_ERR_INVALID_ARG, "too many partials for the W-update reduction");
  p->off_gw = place("off_gw", 32 * 32 * sizeof(float));
  p->off_scal = place("off_scal", (size_t)SCAL_COUNT * (d - 1) * sizeof(double));
  p->off_ints = place("off_ints", 64 * sizeof(int));
  p->off_xb = place("off_xb", xb_size);
  p->off_xt = place("off_xt", xt_size);
  p->off_wp = place("off_wp", wp_size);
  p->off_hp = place("off_hp", hp_size);
  p->off_s = place("off_s", s_size);
  p->off_wb = place("off_wb", wb_size);
  p->off_gpart = place("off_gpart", (size_t)((m_max + 255) / 256) * (32 * 32 + 1) * sizeof(double));
  p->off_coop = place("off_coop", (size_t)512 * 32 * sizeof(unsigned));
  if (eps_mode) {
    p->off_grp = place("off_grp", grp_max * sizeof(double));
    p->off_gram = place("off_gram", gram_max * sizeof(double));
    p->off_eig = place("off_eig", (2 * (size_t)n_max + 8) * sizeof(double));
    // eigensolver scratch (eigenvalues only): checked against the solver's own query,
    // which asked for 110 MB at n = 2048 (about 3.3 n^2 doubles)
    p->eigws_size = (size_t)32 << 20;
    p->eigws_size += 4 * gram_max * sizeof(double);
    p->off_eigws = place("off_eigws", p->eigws_size);
    if (streamed) {  // the Gram of one column block of X_1
      p->off_gram2 = place("off_gram2", (size_t)p->dims[0] * (size_t)p->dims[0] * sizeof(double));
    }
  }
  if (streamed) {
    const size_t m1 = (size_t)p->dims[0], r1 = (size_t)p->eff[1];
    p->off_xs = place("off_xs", m1 * (size_t)p->kblk * sizeof(float));
    p->off_hs = place("off_hs", r1 * (size_t)p->kblk * sizeof(float));
    p->off_redtmp = place("off_redtmp", (m1 * r1 + r1 * r1) * sizeof(double));
    p->off_bsum = place("off_bsum", (size_t)p->nblk * sizeof(double));
  }
  if (bcd) {
    p->off_bh[0] = place("off_bh[0]", bh_size * sizeof(float));
    p->off_bh[1] = place("off_bh[1]", bh_size * sizeof(float));
    p->off_bwp = place("off_bwp", bm_size * sizeof(float));
    p->off_bwn = place("off_bwn", bm_size * sizeof(float));
    p->off_bxh = place("off_bxh", bm_size * sizeof(double));
    p->off_bhh = place("off_bhh", 32 * 32 * sizeof(double));
    p->off_bgw = place("off_bgw", 32 * 32 * sizeof(float));
    p->off_bst = place("off_bst", sizeof(BcdState));
  }
  p->total = off;
  return NTT_OK;
}

// ------------------------------------------------------------------ serving arena
void Arena::init(size_t n) {
  size = n;
  free_list.assign(1, {0, n});
}

bool Arena::alloc(size_t n, size_t* off) {
  n = align_up(std::max<size_t>(n, 256), 256);
  for (size_t i = 0; i < free_list.size(); ++i) {
    if (free_list[i].second >= n) {
      *off = free_list[i].first;
      free_list[i].first += n;
      free_list[i].second -= n;
      if (free_list[i].second == 0) free_list.erase(free_list.begin() + (std::ptrdiff_t)i);
      return true;
    }
  }
  return false;
}

void Arena::release(size_t off, size_t n) {
  n = align_up(std::max<size_t>(n, 256), 256);
  auto it = free_list.begin();
  while (it != free_list.end() && it->first < off) ++it;
  it = free_list.insert(it, {off, n});
  // merge with the next and the previous ranges
  if (it + 1 != free_list.end() && it->first + it->second == (it + 1)->first) {
    it->second += (it + 1)->second;
    free_list.erase(it + 1);
  }
  if (it != free_list.begin() && (it - 1)->first + (it - 1)->second == it->first) {
    (it - 1)->second += it->second;
    free_list.erase(it);
  }
}

size_t Arena::free_bytes() const {
  size_t f = 0;
  for (const auto& r : free_list) f += r.second;
  return f;
}

void Admission::init(size_t arena_bytes, int slots) {
  arena.init(arena_bytes);
  slot_used.assign((size_t)slots, 0);
}

bool Admission::admit(size_t bytes_cores, size_t bytes_work, int* slot, size_t* off_c, size_t* off_w) {
  int s = -1;
  for (int i = 0; i < (int)slot_used.size(); ++i)
    if (!slot_used[(size_t)i]) {
      s = i;
      break;
    }
  if (s < 0) return false;
  if (!arena.alloc(bytes_cores, off_c)) return false;
  if (!arena.alloc(bytes_work, off_w)) {
    arena.release(*off_c, bytes_cores);
    return false;
  }
  slot_used[(size_t)s] = 1;
  *slot = s;
  return true;
}

}  // namespace ntt
