// Host-logic checks of the library's plain C++ part (ntt_host.cpp): the plan's validation
// and workspace layout over many random configurations, the serving arena against a
// bitmap model, and the admission rule.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py; prints "ok" and exits 0
// when every check holds, else names the first failure and exits 1.

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../paper_2008_01340_amd/csrc/ntt_host.h"

using namespace ntt;

namespace {

int g_fail = 0;

#define CHECK(cond, ...)                                      \
  do {                                                        \
    if (!(cond)) {                                            \
      fprintf(stderr, "check failed (%s:%d): %s: ", __FILE__, __LINE__, #cond); \
      fprintf(stderr, __VA_ARGS__);                           \
      fprintf(stderr, "\n");                                  \
      if (++g_fail > 20) exit(1);                             \
    }                                                         \
  } while (0)

// SplitMix64: the checks' own generator (seeded, reproducible)
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1)); }
  double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  // log-uniform integer in [1, hi]
  int64_t logint(int64_t hi) {
    double v = std::exp(unit() * std::log((double)hi));
    return std::max<int64_t>(1, std::min<int64_t>(hi, (int64_t)v));
  }
};

const Region* region(const PlanLayout& p, const char* name) {
  for (const Region& r : p.regions)
    if (std::string(r.name) == name) return &r;
  return nullptr;
}

void check_stage(const PlanLayout& p, const Stage& s, int l, const char* what) {
  const size_t E = (size_t)s.m * s.r + (size_t)s.r * s.r;
  CHECK(s.m >= 1 && s.k >= 1 && s.r >= 1 && s.r <= NTT_MAX_RANK, "%s %d: m %lld k %lld r %d", what, l,
        (long long)s.m, (long long)s.k, s.r);
  CHECK(s.rp == (s.r <= 16 ? 16 : 32), "%s %d: padding", what, l);
  CHECK(s.part_stride >= E, "%s %d: part stride", what, l);
  CHECK(s.G >= 1, "%s %d: G", what, l);
  switch (s.kind) {
    case PASS_S:
      CHECK(s.m <= 32 && (s.mb == 1 || s.mb == 2) && 16 * s.mb >= s.m, "%s %d: S pass rows", what, l);
      CHECK(!s.tiny || (s.m <= 4 && s.r <= s.m && !s.wide && !s.pro_ok && s.G <= 1024 &&
                        (int64_t)s.G * pass_tiny_cols(s.m) >= std::min<int64_t>(s.k, 1024LL * pass_tiny_cols(s.m))),
            "%s %d: pass for at most 4 rows", what, l);
      break;
    case PASS_L:
      CHECK(s.cls >= 0 && s.m <= (s.rp == 16 ? 1024 : 512), "%s %d: row-split class", what, l);
      break;
    case PASS_C:
      CHECK(s.nch >= 1 && s.nch <= 65535 && (int64_t)s.nch * pass_C_rows(s.rp) >= s.m,
            "%s %d: row chunks", what, l);
      break;
    case PASS_GENERIC:
      CHECK(s.chunk >= 64 && s.chunk % 64 == 0 && (int64_t)s.G * s.chunk >= s.k, "%s %d: generic chunks",
            what, l);
      break;
    default:
      CHECK(false, "%s %d: unknown kind %d", what, l, s.kind);
  }
  const Region* part = region(p, "off_part");
  const Region* red = region(p, "off_red");
  CHECK(part && red, "regions");
  if (!part || !red) return;
  if (s.kind != PASS_GENERIC) CHECK(part->bytes >= (size_t)s.G * s.part_stride * 4, "%s %d: partials", what, l);
  CHECK(red->bytes >= E * 8, "%s %d: reduced partials", what, l);
  if (s.coop_ok) {
    CHECK(s.m <= 256 && s.r <= 16 && s.k > 64, "%s %d: cooperative shape", what, l);
    CHECK((int64_t)s.coop_G * s.coop_ng * 16 >= s.k && s.coop_G <= 512, "%s %d: cooperative grid", what, l);
    CHECK(part->bytes >= (size_t)s.coop_G * E * 4, "%s %d: cooperative partials", what, l);
  }
  if (s.bf16) CHECK(region(p, "off_xb")->bytes >= (size_t)s.m * (size_t)s.k * 2, "%s %d: BF16 copy", what, l);
  if (s.kind == PASS_C)
    CHECK(region(p, "off_s")->bytes >= (size_t)(s.nch + 1) * s.r * (size_t)s.k * 4, "%s %d: chunk sums", what, l);
}

void check_plans(int n) {
  Rng g{12345};
  int ok = 0, refused = 0;
  for (int it = 0; it < n; ++it) {
    ntt_config c{};
    const int d = g.uniform(0, 40) == 0 ? 1 : (int)g.uniform(2, 8);
    int64_t dims[NTT_MAX_DIMS + 1] = {}, ranks[NTT_MAX_DIMS + 2] = {};
    // total entries up to ~2^36, now and then up to ~2^52 (beyond the 2^44 limit): layouts
    // only, nothing is allocated
    const double budget = std::log(g.uniform(0, 50) == 0 ? 4503599627370496.0 : 68719476736.0) * g.unit();
    for (int i = 0; i < d; ++i) dims[i] = std::max<int64_t>(1, (int64_t)std::exp(budget / d * (0.3 + 1.4 * g.unit())));
    ranks[0] = 1;
    for (int i = 1; i < d; ++i) ranks[i] = g.uniform(1, 32);
    if (g.uniform(0, 20) == 0) ranks[g.uniform(1, std::max(1, d - 1))] = g.uniform(33, 40);  // above the cap
    ranks[d] = 1;
    if (g.uniform(0, 30) == 0) ranks[g.uniform(0, d)] = 0;  // invalid on purpose
    c.d = d;
    c.dims = dims;
    c.ranks = ranks;
    c.max_iters = (int32_t)g.uniform(-1, 600);
    c.tol = g.uniform(0, 6) == 0 ? 1e-4 : 0.0;
    c.check_every = (int32_t)g.uniform(g.uniform(0, 20) == 0 ? 0 : 1, 20);
    c.eps = g.uniform(0, 20) == 0 ? -1.0 : 1e-12;
    c.seed = g.next();
    c.precision = g.uniform(0, 20) == 0 ? 2 : (int32_t)g.uniform(0, 1);
    c.fp32_tail_iters = (int32_t)g.uniform(0, 30);
    c.flags = (uint32_t)(g.uniform(0, 4) == 0 ? NTT_STRICT_RANKS : 0);
    c.rank_eps = g.uniform(0, 4) == 0 ? 0.05 : 0.0;
    c.nmf = g.uniform(0, 3) == 0 ? 1 : 0;
    c.bcd_delta = 0.9999;
    c.stream_cols = g.uniform(0, 5) == 0 ? g.uniform(1, 100000) : 0;
    PlanLayout p;
    std::string err;
    const ntt_status st = plan_layout(&c, &p, &err);
    if (st != NTT_OK) {
      ++refused;
      CHECK(!err.empty(), "config %d refused without a reason", it);
      CHECK(st == NTT_ERR_INVALID_ARG || st == NTT_ERR_RANK_INFEASIBLE, "config %d: status %d", it, (int)st);
      continue;
    }
    ++ok;
    // regions: 256-byte aligned, in order, disjoint, inside the total
    size_t end = 0;
    for (const Region& r : p.regions) {
      CHECK(r.off % 256 == 0, "config %d: %s misaligned", it, r.name);
      CHECK(r.off >= end, "config %d: %s overlaps the region before it", it, r.name);
      end = r.off + r.bytes;
    }
    CHECK(end <= p.total && p.total % 256 == 0, "config %d: total %zu below the end %zu", it, p.total, end);
    // effective ranks
    CHECK(p.eff[0] == 1 && p.eff[d] == 1, "config %d: boundary ranks", it);
    int64_t left = 1;
    for (int l = 1; l < d; ++l) {
      int64_t right = 1;
      for (int j = l; j < d; ++j) right *= dims[j];
      left = p.eff[l - 1] * dims[l - 1];
      CHECK(p.eff[l] >= 1 && p.eff[l] <= ranks[l] && p.eff[l] <= left && p.eff[l] <= right &&
                p.eff[l] <= NTT_MAX_RANK,
            "config %d: rank %d", it, l);
      const Stage& s = p.st[l - 1];
      CHECK(s.m == left && s.k == right && s.r == (int)p.eff[l], "config %d: stage %d shape", it, l);
      check_stage(p, s, l, "stage");
      if (s.trans_ok) {
        const Stage& t = p.tst[l - 1];
        CHECK(t.m == s.k && t.k == s.m && t.r == s.r && t.fused, "config %d: transposed stage %d", it, l);
        check_stage(p, t, l, "transposed stage");
        CHECK(region(p, "off_xt")->bytes >= (size_t)s.m * (size_t)s.k * 4, "config %d: X^T", it);
      }
      if (l < d - 1)
        CHECK(region(p, (l - 1) % 2 ? "off_h[1]" : "off_h[0]")->bytes >= (size_t)s.r * (size_t)s.k * 4,
              "config %d: H buffer of stage %d", it, l);
    }
    if (c.stream_cols > 0) {
      CHECK(p.kblk >= 1 && p.nblk >= 1 && p.kblk * p.nblk >= p.st[0].k && p.kblk * (p.nblk - 1) < p.st[0].k,
            "config %d: column blocks", it);
      CHECK(region(p, "off_xs")->bytes >= (size_t)dims[0] * (size_t)p.kblk * 4, "config %d: staging", it);
    }
    CHECK(p.compression > 0.0, "config %d: compression", it);
    double entries = 1.0;
    for (int i = 0; i < d; ++i) entries *= (double)dims[i];
    CHECK(entries <= 17592186044416.0, "config %d: a tensor above 2^44 entries was planned", it);
  }
  printf("plans: %d laid out, %d refused\n", ok, refused);
  CHECK(ok > n / 4 && refused > n / 50, "too few of one outcome (%d, %d)", ok, refused);
}

void check_arena(int rounds) {
  Rng g{777};
  for (int round = 0; round < rounds; ++round) {
    const size_t units = (size_t)g.uniform(1, 4096);
    Arena a;
    a.init(units * 256);
    std::vector<char> used(units, 0);
    std::vector<std::pair<size_t, size_t>> live;  // (offset, bytes as asked)
    for (int op = 0; op < 400; ++op) {
      if (live.empty() || g.uniform(0, 2) > 0) {
        const size_t n = (size_t)g.logint((int64_t)units * 256 / 4 + 1);
        const size_t nu = (std::max<size_t>(n, 256) + 255) / 256;
        size_t off = 0;
        if (a.alloc(n, &off)) {
          CHECK(off % 256 == 0 && off / 256 + nu <= units, "arena: range [%zu, +%zu) outside", off, n);
          for (size_t u = off / 256; u < off / 256 + nu && u < units; ++u) {
            CHECK(!used[u], "arena: unit %zu handed out twice", u);
            used[u] = 1;
          }
          live.push_back({off, n});
        } else {
          // first fit fails only when no free run is long enough
          size_t run = 0, best = 0;
          for (size_t u = 0; u < units; ++u) {
            run = used[u] ? 0 : run + 1;
            best = std::max(best, run);
          }
          CHECK(best < nu, "arena: %zu units refused with a free run of %zu", nu, best);
        }
      } else {
        const size_t i = (size_t)g.uniform(0, (int64_t)live.size() - 1);
        const size_t off = live[i].first, n = live[i].second;
        const size_t nu = (std::max<size_t>(n, 256) + 255) / 256;
        a.release(off, n);
        for (size_t u = off / 256; u < off / 256 + nu; ++u) used[u] = 0;
        live.erase(live.begin() + (std::ptrdiff_t)i);
      }
      // the free list: sorted, disjoint, merged, and exactly the unused units
      size_t free_units = 0, prev_end = 0;
      for (size_t j = 0; j < a.free_list.size(); ++j) {
        const auto& r = a.free_list[j];
        CHECK(r.first % 256 == 0 && r.second % 256 == 0 && r.second > 0, "arena: free range shape");
        CHECK(j == 0 || r.first > prev_end, "arena: free ranges unsorted, overlapping or unmerged");
        for (size_t u = r.first / 256; u < (r.first + r.second) / 256 && u < units; ++u)
          CHECK(!used[u], "arena: unit %zu both free and live", u);
        prev_end = r.first + r.second;
        free_units += r.second / 256;
      }
      size_t live_units = 0;
      for (char c : used) live_units += (size_t)c;
      CHECK(free_units + live_units == units, "arena: %zu free + %zu live != %zu", free_units, live_units, units);
      CHECK(a.free_bytes() == free_units * 256, "arena: free_bytes");
    }
  }
  printf("arena: %d rounds\n", rounds);
}

void check_admission(int rounds) {
  Rng g{4242};
  for (int round = 0; round < rounds; ++round) {
    const int slots = (int)g.uniform(1, 64);
    const size_t bytes = (size_t)g.uniform(16, 2048) * 256;
    Admission ad;
    ad.init(bytes, slots);
    struct Held { int slot; size_t oc, nc, ow, nw; };
    std::vector<Held> held;
    for (int op = 0; op < 300; ++op) {
      if (held.empty() || g.uniform(0, 2) > 0) {
        const size_t nc = (size_t)g.logint((int64_t)bytes / 8), nw = (size_t)g.logint((int64_t)bytes / 3);
        const size_t free_before = ad.arena.free_bytes();
        int slot = -1;
        size_t oc = 0, ow = 0;
        if (ad.admit(nc, nw, &slot, &oc, &ow)) {
          CHECK(slot >= 0 && slot < slots, "admission: slot %d", slot);
          for (const Held& h : held) CHECK(h.slot != slot, "admission: slot %d given twice", slot);
          held.push_back({slot, oc, nc, ow, nw});
        } else {
          CHECK(ad.arena.free_bytes() == free_before, "admission: a refused request kept memory");
          CHECK(slot == -1, "admission: a refused request got a slot");
          int busy = 0;
          for (char c : ad.slot_used) busy += c;
          CHECK(busy == (int)held.size(), "admission: slot table out of step");
        }
      } else {
        const size_t i = (size_t)g.uniform(0, (int64_t)held.size() - 1);
        const Held h = held[i];
        ad.arena.release(h.oc, h.nc);
        ad.arena.release(h.ow, h.nw);
        ad.slot_used[(size_t)h.slot] = 0;
        held.erase(held.begin() + (std::ptrdiff_t)i);
      }
    }
    for (const Held& h : held) {
      ad.arena.release(h.oc, h.nc);
      ad.arena.release(h.ow, h.nw);
    }
    CHECK(ad.arena.free_bytes() == bytes && ad.arena.free_list.size() == 1, "admission: arena not whole at the end");
  }
  printf("admission: %d rounds\n", rounds);
}

// Eq.(3) partial blocks: at least one column range, at most 65535, and the fixed 8 MiB
// array of ntt_rel_error_static holds the partials of every tensor of up to 33,554,368
// rows n_1...n_{d-1}, whatever n_d
void check_tt_blocks(int n) {
  Rng g{99};
  for (int it = 0; it < n; ++it) {
    const int64_t rows = g.logint(g.uniform(0, 3) == 0 ? 33554368 : (1LL << 40));
    const int64_t nd = g.logint(1LL << 34);
    const int64_t cs = tt_col_splits(rows, nd);
    const int rpb = tt_rows_per_block(nd);
    CHECK((rpb == 64 || rpb == 128) && cs >= 1 && cs <= 65535 && (cs == 1 || (rows + rpb - 1) / rpb < 2048),
          "tt splits %lld for %lld x %lld", (long long)cs, (long long)rows, (long long)nd);
    CHECK(tt_blocks(rows, nd) == (rows + rpb - 1) / rpb * cs, "tt blocks");
    if (rows <= 33554368)
      CHECK((size_t)(2 * tt_blocks(rows, nd) + 2) * sizeof(double) <= NTT_REL_ERROR_STATIC_BYTES,
            "static Eq.(3) array too small for %lld x %lld", (long long)rows, (long long)nd);
  }
  printf("tt blocks: %d shapes\n", n);
}

}  // namespace

int main(int argc, char** argv) {
  const int n = argc > 1 ? atoi(argv[1]) : 20000;
  check_plans(n);
  check_arena(n / 100 + 1);
  check_admission(n / 100 + 1);
  check_tt_blocks(n);
  if (g_fail) {
    printf("%d checks failed\n", g_fail);
    return 1;
  }
  printf("ok\n");
  return 0;
}
