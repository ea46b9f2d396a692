// ntt_kernels.hip -- CDNA4 (gfx950) kernels of the nTT multiplicative-update sweep.
//
// One MU iteration on an m x k unfolding X at rank r (paper: Alg.2 sweep; the MU rule
// the experiments time; the products of Alg.4-6 on one GPU):
//   H <- max(0, H .* (W^T X) ./ ((W^T W) H + eps))          (W^T X: Alg.6, W^T W: Alg.4)
//   W <- max(0, W .* (X H^T) ./ (W (H H^T) + eps))          (X H^T: Alg.5, H H^T: Alg.4)
//
// The H-update of a column j needs only W, W^T W, X[:,j] and H[:,j].  So one pass over
// the columns of X does the whole H-update and, while X[:,j] is still in registers,
// accumulates X[:,j] H_new[:,j]^T and H_new[:,j] H_new[:,j]^T: X is read from HBM once
// per iteration.  Per-workgroup partial sums are reduced in a fixed order (no float
// atomics) by separate launches (k_reduce_partials, then k_wupdate_t over blocks of 256
// rows), which apply the W-update and form the next W^T W;
// the r <= 8 passes can instead take that W-update in their own prologue.  Small stages
// run whole in one workgroup (k_stage_1wg) or in one grid-synchronised launch (ntt_coop.hip).
// The result equals the two-pass MU up to summation order.
//
// Rank r is padded to RP = 16 or 32 (zero rows/columns) to fit the MFMA 16x16x4 f32
// tiles.  All shapes are runtime values; ragged edges are masked to zero, which is
// exact: a zero column of X with a zero column of H stays zero and adds nothing.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ntt_device.h"
#include "ntt_internal.h"

namespace ntt {

// ------------------------------------------------------------------ SplitMix64 init
// Value i of stream `tag`: SplitMix64 finaliser of seed + GAMMA (tag 2^32 + i + 1);
// uniform = top 24 bits * 2^-24 (exact in FP32).
__device__ __forceinline__ float splitmix_uniform(uint64_t seed, uint64_t tag, uint64_t i) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * ((tag << 32) + i + 1ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (float)(z >> 40) * (1.0f / 16777216.0f);
}

__global__ void k_init_uniform(float* __restrict__ out, int64_t n, uint64_t seed, uint64_t tag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = splitmix_uniform(seed, tag, (uint64_t)i);
}

// ------------------------------------------------------------------ ||X||^2 + validation
// Per-block FP64 sum of squares; flags |= 1 when an entry is negative, NaN or Inf.
__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ x, int64_t n,
                                               double* __restrict__ part, int* __restrict__ flags,
                                               int validate) {
  __shared__ double red[4];
  double acc = 0.0;
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  const bool vec = ((reinterpret_cast<uintptr_t>(x) & 15) == 0);
  if (vec) {
    const int64_t n4 = n >> 2;
    const float4* x4 = reinterpret_cast<const float4*>(x);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
      float4 v = x4[i];
      acc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
      if (validate) {
        bad |= !(v.x >= 0.f && v.x <= 3.4028235e38f) | !(v.y >= 0.f && v.y <= 3.4028235e38f) |
               !(v.z >= 0.f && v.z <= 3.4028235e38f) | !(v.w >= 0.f && v.w <= 3.4028235e38f);
      }
    }
    for (int64_t i = (n4 << 2) + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
      float v = x[i];
      acc += (double)v * v;
      if (validate) bad |= !(v >= 0.f && v <= 3.4028235e38f);
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
      float v = x[i];
      acc += (double)v * v;
      if (validate) bad |= !(v >= 0.f && v <= 3.4028235e38f);
    }
  }
  acc = wave_sum(acc);
  if (validate && __any(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, 1);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Fixed-order sum of n doubles by one wavefront: out[0] = scale * sum (optionally also
// out2 = out).  Used for ||X||^2 and residual objectives.
__global__ __launch_bounds__(64) void k_sum_doubles(const double* __restrict__ part, int n,
                                                    double scale, double* __restrict__ out,
                                                    double* __restrict__ out2) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) acc += part[i];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) {
    out[0] = scale * acc;
    if (out2) out2[0] = scale * acc;
  }
}

// ------------------------------------------------------------------ Gram W^T W
// Accumulate sum over rows of a 256-row chunk held in LDS (sW[256][RP+1], zero padded)
// into acc[] (pairs p = tid + 256 t of the RP x RP Gram), FP64.
template <int RP>
__device__ __forceinline__ void gram_chunk(const float (*sW)[RP + 1], int nrows, double* acc) {
  constexpr int NP = (RP * RP + 255) / 256;
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    const int pidx = threadIdx.x + 256 * t;
    if (pidx < RP * RP) {
      const int c = pidx / RP, q = pidx % RP;
      double s = 0.0;
      for (int i = 0; i < nrows; ++i) s += (double)sW[i][c] * (double)sW[i][q];
      acc[t] += s;
    }
  }
}

// G (RP x RP floats, zero padded) = W^T W for W m x r; one block of 256 threads, rows
// staged through LDS 256 at a time, FP64 accumulation.
template <int RP>
__global__ __launch_bounds__(256) void k_gram_w(const float* __restrict__ W, int m, int r,
                                                float* __restrict__ G) {
  __shared__ float sW[256][RP + 1];
  constexpr int NP = (RP * RP + 255) / 256;
  double acc[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) acc[t] = 0.0;
  for (int i0 = 0; i0 < m; i0 += 256) {
    __syncthreads();
    for (int e = threadIdx.x; e < 256 * RP; e += 256) {
      const int i = e / RP, c = e % RP;
      sW[i][c] = zmask(W[(int64_t)min(i0 + i, m - 1) * r + min(c, r - 1)], i0 + i < m && c < r);
    }
    __syncthreads();
    gram_chunk<RP>(sW, min(256, m - i0), acc);
  }
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    const int pidx = threadIdx.x + 256 * t;
    if (pidx < RP * RP) G[pidx] = (float)acc[t];
  }
}

// ------------------------------------------------------------------ fused MU pass
// X element loads: FP32 storage, or the BF16 shadow (widened exactly to FP32).
__device__ __forceinline__ float bf16_to_f32(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

// A non-temporal 16-byte store (H_new: written once per pass, read by the next one)
__device__ __forceinline__ void st_nt4(float* dst, const float4& v) {
  __builtin_nontemporal_store(v4f{v.x, v.y, v.z, v.w}, reinterpret_cast<v4f*>(dst));
}

template <bool XBF, bool NT = false>
__device__ __forceinline__ float4 ldx4(const PassArgs& p, int64_t off) {
  // NT: non-temporal loads (an X far larger than the last-level cache streams past it)
  if (XBF) {
    uint2 u;
    if constexpr (NT) {
      typedef uint32_t u2v __attribute__((ext_vector_type(2)));
      const u2v v = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(p.Xb + off));
      u = make_uint2(v.x, v.y);
    } else {
      u = *reinterpret_cast<const uint2*>(p.Xb + off);
    }
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                       __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
  }
  if constexpr (NT) {
    const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p.X + off));
    return make_float4(v[0], v[1], v[2], v[3]);
  }
  return *reinterpret_cast<const float4*>(p.X + off);
}

template <bool XBF>
__device__ __forceinline__ float ldx(const PassArgs& p, int64_t off) {
  return XBF ? bf16_to_f32(p.Xb[off]) : p.X[off];
}

template <bool XBF>
__device__ __forceinline__ bool x_aligned(const PassArgs& p) {
  return XBF ? ((reinterpret_cast<uintptr_t>(p.Xb) & 7) == 0)
             : ((reinterpret_cast<uintptr_t>(p.X) & 15) == 0);
}

// Variant for m <= 16*MB (MB 16-row blocks held in registers) and r <= RP.
// Each wavefront takes 16-column groups (group g = global wave id + s * total waves).
// UPDATE: do the H-update and accumulate X H_new^T and H_new H_new^T partials.
// RESID : accumulate sum (X - W H_in)^2 in FP64 over the incoming W, H.
// Per-workgroup partial (written when UPDATE): X H_new^T as m x r, then H_new H_new^T
// as r x r, both row-major and compact.
template <int RP, int MB, bool UPDATE, bool RESID, bool XBF = false>
__global__ __launch_bounds__(256) void k_mu_pass(PassArgs p) {
  constexpr int NH = RP / 16;  // 16-row halves of the padded rank
  constexpr int MPAD = 16 * MB;
  constexpr int SX = 20;       // LDS row stride of 16-wide transposition tiles
  __shared__ __attribute__((aligned(16))) float sWt[RP][MPAD + 4];   // W^T, zero padded
  __shared__ __attribute__((aligned(16))) float sW[RESID ? MPAD : 1][RP + 4];  // W rows
  __shared__ __attribute__((aligned(16))) float sX[4][16 * SX];      // per-wave 16x16 X block
  __shared__ __attribute__((aligned(16))) float sHn[4][RP * SX];     // per-wave H_new block
  __shared__ double sRes[4];

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;

  // stage W and W^T in LDS (all loads first, then the stores)
  {
    constexpr int NWL = (RP * MPAD + 255) / 256;
    float wtmp[NWL];
#pragma unroll
    for (int t = 0; t < NWL; ++t) {
      const int e = tid + 256 * t;
      const int i = e / RP, c = e % RP;
      const float v = p.W[(int64_t)min(i, m - 1) * r + min(c, r - 1)];
      wtmp[t] = zmask(v, e < RP * MPAD && i < m && c < r);
    }
#pragma unroll
    for (int t = 0; t < NWL; ++t) {
      const int e = tid + 256 * t;
      if (e < RP * MPAD) {
        const int i = e / RP, c = e % RP;
        sWt[c][i] = wtmp[t];
        if (RESID) sW[i][c] = wtmp[t];
      }
    }
  }
  // G_W as the A operand of (W^T W) H: lane (a,b), half h, K step (q,kk) -> G[16h+a][16q+4b+kk]
  float gw[NH][NH][4];
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int q = 0; q < NH; ++q)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) gw[h][q][kk] = p.GW[(16 * h + a) * RP + 16 * q + 4 * b + kk];
  __syncthreads();

  v4f accW[MB][NH];      // X H_new^T: lane (a,b) reg i -> row 16*blk+4b+i, rank 16h+a
  v4f accG[NH][NH];      // H_new H_new^T
  double res = 0.0;
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int h = 0; h < NH; ++h) accW[i][h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int q = 0; q < NH; ++q) accG[h][q] = v4f{0.f, 0.f, 0.f, 0.f};

  const int64_t ngroups = (k + 15) >> 4;
  const int64_t wstride = (int64_t)gridDim.x * 4;
  const bool vec_ok = ((k & 3) == 0) && x_aligned<XBF>(p) &&
                      ((reinterpret_cast<uintptr_t>(p.H) & 15) == 0);
  float* sXw = sX[w];
  float* sHw = sHn[w];

  // Loads of a 16-column group: X rows 16*blk + a, columns j0+4b .. j0+4b+3 (the A
  // operand of X H^T) and H[16h+4b+kk][j0+a].  Addresses are clamped into the arrays, so
  // interior groups need no branches; their values are stored as loaded and the entries
  // out of range are zeroed only when the group is processed (mask_group), so that no
  // instruction waits on a prefetch still in flight.  (The two load paths must differ:
  // identical plain loads in both would let the compiler merge them into one path of
  // scalar loads.)
  auto load_group = [&](int64_t g, float (&xr)[MB][4], float (&hv)[NH][4]) {
    const int64_t j0 = g << 4;
    if (vec_ok && (j0 + 16 <= k)) {
#pragma unroll
      for (int blk = 0; blk < MB; ++blk) {
        const int row = 16 * blk + a;
        const float4 v = ldx4<XBF>(p, (int64_t)min(row, m - 1) * k + j0 + 4 * b);
        xr[blk][0] = v.x;
        xr[blk][1] = v.y;
        xr[blk][2] = v.z;
        xr[blk][3] = v.w;
      }
    } else {  // ragged or unaligned group (rare): masked here
#pragma unroll
      for (int blk = 0; blk < MB; ++blk) {
        const int row = 16 * blk + a;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t col = j0 + 4 * b + q;
          const float v = ldx<XBF>(p, (int64_t)min(row, m - 1) * k + min(col, k - 1));
          xr[blk][q] = zmask(v, row < m && col < k);
        }
      }
    }
    const int64_t colc = min(j0 + a, k - 1);
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int c = 16 * h + 4 * b + kk;
        hv[h][kk] = p.H[(int64_t)min(c, r - 1) * k + colc];
      }
  };
  // zero the entries of a loaded group that lie outside X (rows >= m; a ragged group is
  // masked as it is loaded) or H (rows >= r, columns >= k)
  auto mask_group = [&](int64_t j0, bool full, float (&xr)[MB][4], float (&hv)[NH][4]) {
    if (full) {
#pragma unroll
      for (int blk = 0; blk < MB; ++blk)
#pragma unroll
        for (int q = 0; q < 4; ++q) xr[blk][q] = zmask(xr[blk][q], 16 * blk + a < m);
    }
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        hv[h][kk] = zmask(hv[h][kk], 16 * h + 4 * b + kk < r && (full || j0 + a < k));
  };

  auto process_group = [&](int64_t g, const float (&xin)[MB][4], const float (&hin)[NH][4]) {
    const int64_t j0 = g << 4;
    const bool full = vec_ok && (j0 + 16 <= k);
    float xr[MB][4], hv[NH][4];
#pragma unroll
    for (int blk = 0; blk < MB; ++blk)
#pragma unroll
      for (int q = 0; q < 4; ++q) xr[blk][q] = xin[blk][q];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) hv[h][q] = hin[h][q];
    mask_group(j0, full, xr, hv);
    // N_H = W^T X (M = rank, N = column, K = row) and the residual X - W H
    v4f nh[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) nh[h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int blk = 0; blk < MB; ++blk) {
      wave_sync();
      *reinterpret_cast<float4*>(&sXw[a * SX + 4 * b]) =
          make_float4(xr[blk][0], xr[blk][1], xr[blk][2], xr[blk][3]);
      wave_sync();
      float xt[4];  // X[16blk + 4b + kk][j0 + a]
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) xt[kk] = sXw[(4 * b + kk) * SX + a];
      if (UPDATE) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const float4 wt = *reinterpret_cast<const float4*>(&sWt[16 * h + a][16 * blk + 4 * b]);
          nh[h] = mfma16(wt.x, xt[0], nh[h]);
          nh[h] = mfma16(wt.y, xt[1], nh[h]);
          nh[h] = mfma16(wt.z, xt[2], nh[h]);
          nh[h] = mfma16(wt.w, xt[3], nh[h]);
        }
      }
      if (RESID) {
        // (W H)[16blk + 4b + i][j0 + a]: M = row, N = column, K = rank
        v4f wh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NH; ++q) {
          const float4 wa = *reinterpret_cast<const float4*>(&sW[16 * blk + a][16 * q + 4 * b]);
          wh = mfma16(wa.x, hv[q][0], wh);
          wh = mfma16(wa.y, hv[q][1], wh);
          wh = mfma16(wa.z, hv[q][2], wh);
          wh = mfma16(wa.w, hv[q][3], wh);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double dlt = (double)xt[i] - (double)wh[i];
          res += dlt * dlt;
        }
      }
    }
    if (!UPDATE) return;
    // D_H = G_W H (M = rank, N = column, K = rank)
    v4f dh[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      dh[h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < NH; ++q)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) dh[h] = mfma16(gw[h][q][kk], hv[q][kk], dh[h]);
    }
    // epilogue: lane (a,b) reg i -> H_new[16h + 4b + i][j0 + a]
    wave_sync();
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * h + 4 * b + i;
        const float q = fmaxf(0.f, fast_div(hv[h][i] * nh[h][i], dh[h][i] + p.eps));
        sHw[c * SX + a] = (c < r) ? q : 0.f;
      }
    wave_sync();
    // transposed read: lane (a,b) -> H_new[16h + a][j0 + 4b .. 4b+3]
    float4 hn4[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) hn4[h] = *reinterpret_cast<const float4*>(&sHw[(16 * h + a) * SX + 4 * b]);
    // store H_new (in place)
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int c = 16 * h + a;
      if (c < r) {
        float* dst = p.H + (int64_t)c * k + j0 + 4 * b;
        if (full) {
          st_nt4(dst, hn4[h]);
        } else {
          const float vv[4] = {hn4[h].x, hn4[h].y, hn4[h].z, hn4[h].w};
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (j0 + 4 * b + q < k) dst[q] = vv[q];
        }
      }
    }
    // X H_new^T (M = row, N = rank, K = column) and H_new H_new^T
#pragma unroll
    for (int blk = 0; blk < MB; ++blk)
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        accW[blk][h] = mfma16(xr[blk][0], hn4[h].x, accW[blk][h]);
        accW[blk][h] = mfma16(xr[blk][1], hn4[h].y, accW[blk][h]);
        accW[blk][h] = mfma16(xr[blk][2], hn4[h].z, accW[blk][h]);
        accW[blk][h] = mfma16(xr[blk][3], hn4[h].w, accW[blk][h]);
      }
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int q = 0; q < NH; ++q) {
        accG[h][q] = mfma16(hn4[h].x, hn4[q].x, accG[h][q]);
        accG[h][q] = mfma16(hn4[h].y, hn4[q].y, accG[h][q]);
        accG[h][q] = mfma16(hn4[h].z, hn4[q].z, accG[h][q]);
        accG[h][q] = mfma16(hn4[h].w, hn4[q].w, accG[h][q]);
      }
  };

  // two register sets: the next group's loads are in flight while one is processed
  float xa[MB][4], ha[NH][4], xb[MB][4], hb[NH][4];
  int64_t g = (int64_t)blockIdx.x * 4 + w;
  if (g < ngroups) load_group(g, xa, ha);
  while (g < ngroups) {
    const int64_t g2 = g + wstride;
    if (g2 < ngroups) load_group(g2, xb, hb);
    process_group(g, xa, ha);
    if (g2 >= ngroups) break;
    const int64_t g3 = g2 + wstride;
    if (g3 < ngroups) load_group(g3, xa, ha);
    process_group(g2, xb, hb);
    g = g3;
  }

  // ---- per-workgroup partials, waves combined in the fixed order 3, 2, 1, 0
  if (RESID) {
    res = wave_sum(res);
    if (lane == 0) sRes[w] = res;
  }
  if (UPDATE) {
    float* dst = p.part + (int64_t)blockIdx.x * p.part_stride;
    float* buf = &sWt[0][0];
    static_assert(RP * (MPAD + 4) >= MPAD * RP, "reduction buffer");
    __syncthreads();
    for (int turn = 3; turn >= 0; --turn) {
      if (w == turn) {
#pragma unroll
        for (int blk = 0; blk < MB; ++blk)
#pragma unroll
          for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int idx = (16 * blk + 4 * b + i) * RP + 16 * h + a;
              buf[idx] = (turn == 3) ? accW[blk][h][i] : buf[idx] + accW[blk][h][i];
            }
      }
      __syncthreads();
    }
    for (int e = tid; e < m * r; e += 256) dst[e] = buf[(e / r) * RP + (e % r)];
    float* gbuf = &sHn[0][0];
    static_assert(4 * RP * SX >= RP * RP, "gram reduction buffer");
    __syncthreads();
    for (int turn = 3; turn >= 0; --turn) {
      if (w == turn) {
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
          for (int q = 0; q < NH; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int idx = (16 * h + 4 * b + i) * RP + 16 * q + a;
              gbuf[idx] = (turn == 3) ? accG[h][q][i] : gbuf[idx] + accG[h][q][i];
            }
      }
      __syncthreads();
    }
    for (int e = tid; e < r * r; e += 256) dst[m * r + e] = gbuf[(e / r) * RP + (e % r)];
  } else {
    __syncthreads();
  }
  if (RESID && tid == 0) p.rpart[blockIdx.x] = ((sRes[0] + sRes[1]) + sRes[2]) + sRes[3];
}

// W^T (zero padded, 16 x MPAD) and G_W (8 x 8) of the r <= 8 passes in LDS: from W and
// W^T W, or, in prologue mode (p.Wprev set), by applying the previous iteration's
// W-update first (the entries of the W-update kernel, one thread per entry (row tid / 8,
// column tid % 8); the Gram by wavefront 0, which holds every row since m <= 32);
// workgroup 0 then stores W to p.Wout.
template <int MPAD>
__device__ __forceinline__ void r8_w_setup(const PassArgs& p, float (*sWt)[MPAD + 4], float (*sG)[8],
                                           int tid, int w, int a, int b) {
  static_assert(8 * MPAD <= 256, "one thread per entry");
  const int m = p.m, r = p.r;
  if (p.Wprev) {
    __shared__ float sWc[MPAD][9];
    __shared__ double sGH[8][9];
    __shared__ double sGW[8][9];
    const int i = tid >> 3, c = tid & 7;
    const int64_t mr = (int64_t)m * r;
    float wv = 0.f;
    double nv = 0.0;
    if (i < MPAD) {
      const int64_t idx = (int64_t)min(i, m - 1) * r + min(c, r - 1);
      wv = zmask(p.Wprev[idx], i < m && c < r);
      nv = zmask(p.red[idx], i < m && c < r);
    }
    if (tid < 64) {
      const int gc = tid >> 3, gq = tid & 7;
      sGH[gc][gq] = zmask(p.red[mr + min(gc, r - 1) * r + min(gq, r - 1)], gc < r && gq < r);
    }
    if (i < MPAD) sWc[i][c] = wv;
    __syncthreads();
    float wf = 0.f;
    if (i < MPAD) {
      const float v = wupdate_entry<8>(sWc[i], nv, sGH, c, p.eps);
      wf = (c < r && i < m) ? v : 0.f;
    }
    __syncthreads();  // every row has been read before it is replaced
    if (i < MPAD) {
      sWc[i][c] = wf;
      if (blockIdx.x == 0 && i < m && c < r) p.Wout[(int64_t)i * r + c] = wf;
    }
    __syncthreads();
    if (w == 0) {
      v4d acc[1][1] = {{v4d{0.0, 0.0, 0.0, 0.0}}};
      gram_rows_f64<8, 1, MPAD>(sWc, acc, 0, a, b);
      // (the W-update kernel's wavefront 0 forms the same sums over its 64 rows, the other
      // wavefronts add exact zeros); value i of lane (a, b) is row 4 i + b, column a
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 * i + b < 8 && a < 8) sGW[4 * i + b][a] = acc[0][0][i];
    }
    __syncthreads();
    for (int e = tid; e < 16 * MPAD; e += 256) {
      const int i = e / 16, c = e % 16;
      sWt[c][i] = c < 8 ? sWc[i][c < 8 ? c : 0] : 0.f;
    }
    if (tid < 64) {
      const int c = tid >> 3, q = tid & 7;
      sG[c][q] = (c < r && q < r) ? (float)sGW[c][q] : 0.f;
    }
  } else {
    constexpr int NWL = (16 * MPAD + 255) / 256;
    float wtmp[NWL];
#pragma unroll
    for (int t = 0; t < NWL; ++t) {
      const int e = tid + 256 * t;
      const int i = e / 16, c = e % 16;
      const float v = p.W[(int64_t)min(i, m - 1) * r + min(c, r - 1)];
      wtmp[t] = zmask(v, e < 16 * MPAD && i < m && c < r);
    }
#pragma unroll
    for (int t = 0; t < NWL; ++t) {
      const int e = tid + 256 * t;
      if (e < 16 * MPAD) sWt[e % 16][e / 16] = wtmp[t];
    }
    if (tid < 64) {
      const int c = tid >> 3, q = tid & 7;
      sG[c][q] = p.GW[c * 16 + q];  // zero beyond r
    }
  }
}

// ------------------------------------------------------------------ fused MU pass, r <= 8
// Specialisation of k_mu_pass (UPDATE only) for r <= 8.  The two 16-wide MFMA products
// (W^T X and X H_new^T) keep the MFMA path; the r x r products (W^T W) H and
// H_new H_new^T, which would fill only a quarter of a 16x16 MFMA tile at r = 8, run on
// the VALU from LDS copies of the H tiles:
//   D_H[c][j] = sum_{q<8} G[c][q] H[q][j]   : lane (a, b<2) forms rows 4b..4b+3 of column a
//   G_H[c][q] += H_new[c][j] H_new[q][j]     : lane (a, b) accumulates the 4x4 block
//                                              (rows 4(b&1).., cols 4(b>>1)..) of column a
// Rows and columns beyond r are zero in G and H_new, so the 8-wide sums are exact for any
// r <= 8.
template <int MB, bool XBF>
__global__ __launch_bounds__(256, 1) void k_mu_pass_r8(PassArgs p) {
  constexpr int MPAD = 16 * MB;
  constexpr int SX = 20;
  __shared__ __attribute__((aligned(16))) float sWt[16][MPAD + 4];  // W^T, zero padded
  __shared__ __attribute__((aligned(16))) float sG[8][8];           // W^T W (8 x 8)
  __shared__ __attribute__((aligned(16))) float sX[4][16 * SX];     // per-wave X block
  __shared__ __attribute__((aligned(16))) float sHn[4][16 * SX];    // per-wave H_new [rank][col]
  __shared__ __attribute__((aligned(16))) float sHc[4][16 * SX];    // per-wave H columns [col][rank]
  __shared__ __attribute__((aligned(16))) float sHnc[4][16 * SX];   // per-wave H_new [col][rank]

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;

  // first group's loads go out before the W set-up, whose latency they then overlap
  const int64_t ngroups = (k + 15) >> 4;
  const int64_t wstride = (int64_t)gridDim.x * 4;
  const bool vec_ok = ((k & 3) == 0) && x_aligned<XBF>(p) &&
                      ((reinterpret_cast<uintptr_t>(p.H) & 15) == 0);
  float* sXw = sX[w];
  float* sHw = sHn[w];
  float* sHcw = sHc[w];
  float* sHncw = sHnc[w];
  const int rq = 4 * (b & 1), cq = 4 * (b >> 1);  // G_H block of this lane
  // row pointers of this lane (clamped into the matrix)
  int64_t xrow[MB];  // row offsets of this lane (clamped into the matrix)
#pragma unroll
  for (int blk = 0; blk < MB; ++blk) xrow[blk] = (int64_t)min(16 * blk + a, m - 1) * k;
  const float* hrow[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) hrow[kk] = p.H + (int64_t)min(4 * b + kk, r - 1) * k;

  auto load_group = [&](int64_t g, float (&xr)[MB][4], float (&hv)[4]) {
    const int64_t j0 = g << 4;
    if (vec_ok && (j0 + 16 <= k)) {
#pragma unroll
      for (int blk = 0; blk < MB; ++blk) {
        const float4 v = ldx4<XBF>(p, xrow[blk] + j0 + 4 * b);
        xr[blk][0] = v.x; xr[blk][1] = v.y; xr[blk][2] = v.z; xr[blk][3] = v.w;
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) hv[kk] = hrow[kk][j0 + a];
    } else {
#pragma unroll
      for (int blk = 0; blk < MB; ++blk)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t col = j0 + 4 * b + q;
          const float v = ldx<XBF>(p, xrow[blk] + min(col, k - 1));
          xr[blk][q] = zmask(v, col < k);
        }
      const int64_t col = j0 + a;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const float v = hrow[kk][min(col, k - 1)];
        hv[kk] = zmask(v, col < k);
      }
    }
  };

  int64_t g = (int64_t)blockIdx.x * 4 + w;
  float xn[MB][4], hn_[4];  // next group's loads, in flight while one is processed
  if (g < ngroups) load_group(g, xn, hn_);
  r8_w_setup<MPAD>(p, sWt, sG, tid, w, a, b);
  __syncthreads();

  v4f accW[MB];     // X H_new^T: lane (a,b) reg i -> row 16*blk+4b+i, rank a
  float pg[4][4];   // G_H block of this lane
#pragma unroll
  for (int i = 0; i < MB; ++i) accW[i] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) pg[i][q] = 0.f;

  for (; g < ngroups; g += wstride) {
    const int64_t j0 = g << 4;
    const bool full = vec_ok && (j0 + 16 <= k);
    float xr[MB][4], hv[4];
#pragma unroll
    for (int blk = 0; blk < MB; ++blk)
#pragma unroll
      for (int q = 0; q < 4; ++q) xr[blk][q] = xn[blk][q];
#pragma unroll
    for (int q = 0; q < 4; ++q) hv[q] = hn_[q];
    if (g + wstride < ngroups) load_group(g + wstride, xn, hn_);

    // H tile to LDS as [column][rank]; rows >= r of the loads hold copies of row r-1,
    // so they are zeroed here
    wave_sync();
    {
      float4 hz;
      hz.x = (4 * b + 0 < r) ? hv[0] : 0.f;
      hz.y = (4 * b + 1 < r) ? hv[1] : 0.f;
      hz.z = (4 * b + 2 < r) ? hv[2] : 0.f;
      hz.w = (4 * b + 3 < r) ? hv[3] : 0.f;
      *reinterpret_cast<float4*>(&sHcw[a * SX + 4 * b]) = hz;
    }
    // N_H = W^T X (M = rank, N = column, K = row)
    v4f nh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int blk = 0; blk < MB; ++blk) {
      if (blk > 0) wave_sync();
      *reinterpret_cast<float4*>(&sXw[a * SX + 4 * b]) =
          make_float4(xr[blk][0], xr[blk][1], xr[blk][2], xr[blk][3]);
      wave_sync();
      float xt[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) xt[kk] = sXw[(4 * b + kk) * SX + a];
      const float4 wt = *reinterpret_cast<const float4*>(&sWt[a][16 * blk + 4 * b]);
      nh = mfma16(wt.x, xt[0], nh);
      nh = mfma16(wt.y, xt[1], nh);
      nh = mfma16(wt.z, xt[2], nh);
      nh = mfma16(wt.w, xt[3], nh);
    }
    // D_H on the VALU: lane (a, b < 2) -> rows 4b..4b+3 of column a
    const float4 hc0 = *reinterpret_cast<const float4*>(&sHcw[a * SX]);
    const float4 hc1 = *reinterpret_cast<const float4*>(&sHcw[a * SX + 4]);
    const float hc[8] = {hc0.x, hc0.y, hc0.z, hc0.w, hc1.x, hc1.y, hc1.z, hc1.w};
    float hnew[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int c = rq + kk;  // = 4b + kk for b < 2
      const float4 g0 = *reinterpret_cast<const float4*>(&sG[c][0]);
      const float4 g1 = *reinterpret_cast<const float4*>(&sG[c][4]);
      float dh = g0.x * hc[0];
      dh = fmaf(g0.y, hc[1], dh);
      dh = fmaf(g0.z, hc[2], dh);
      dh = fmaf(g0.w, hc[3], dh);
      dh = fmaf(g1.x, hc[4], dh);
      dh = fmaf(g1.y, hc[5], dh);
      dh = fmaf(g1.z, hc[6], dh);
      dh = fmaf(g1.w, hc[7], dh);
      const float q = fmaxf(0.f, fast_div(hv[kk] * nh[kk], dh + p.eps));
      hnew[kk] = (b < 2 && 4 * b + kk < r) ? q : 0.f;
    }
    // H_new to LDS in both layouts: [rank][col] (X H^T operand) and [col][rank] (G_H)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) sHw[(4 * b + kk) * SX + a] = hnew[kk];
    *reinterpret_cast<float4*>(&sHncw[a * SX + 4 * b]) = make_float4(hnew[0], hnew[1], hnew[2], hnew[3]);
    wave_sync();
    const float4 hn4 = *reinterpret_cast<const float4*>(&sHw[a * SX + 4 * b]);  // H_new[a][j0+4b..]
    if (a < r) {
      float* dst = p.H + (int64_t)a * k + j0 + 4 * b;
      if (full) {
        st_nt4(dst, hn4);
      } else {
        const float vv[4] = {hn4.x, hn4.y, hn4.z, hn4.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (j0 + 4 * b + q < k) dst[q] = vv[q];
      }
    }
    // X H_new^T (M = row, N = rank, K = column)
#pragma unroll
    for (int blk = 0; blk < MB; ++blk) {
      accW[blk] = mfma16(xr[blk][0], hn4.x, accW[blk]);
      accW[blk] = mfma16(xr[blk][1], hn4.y, accW[blk]);
      accW[blk] = mfma16(xr[blk][2], hn4.z, accW[blk]);
      accW[blk] = mfma16(xr[blk][3], hn4.w, accW[blk]);
    }
    // G_H block on the VALU
    const float4 hr = *reinterpret_cast<const float4*>(&sHncw[a * SX + rq]);
    const float4 hq = *reinterpret_cast<const float4*>(&sHncw[a * SX + cq]);
    const float hrv[4] = {hr.x, hr.y, hr.z, hr.w}, hqv[4] = {hq.x, hq.y, hq.z, hq.w};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) pg[i][q] = fmaf(hrv[i], hqv[q], pg[i][q]);
  }

  // ---- per-workgroup partials
  // G_H: sum the lane blocks over the 16 columns a (fixed butterfly), then waves in order
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float v = pg[i][q];
      v += __shfl_xor(v, 8, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 1, 64);
      pg[i][q] = v;
    }
  float* dst = p.part + (int64_t)blockIdx.x * p.part_stride;
  float* buf = &sWt[0][0];
  static_assert(16 * (MPAD + 4) >= MPAD * 16, "reduction buffer");
  float* gbuf = &sHn[0][0];
  __syncthreads();
  for (int turn = 3; turn >= 0; --turn) {
    if (w == turn) {
#pragma unroll
      for (int blk = 0; blk < MB; ++blk)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int idx = (16 * blk + 4 * b + i) * 16 + a;
          buf[idx] = (turn == 3) ? accW[blk][i] : buf[idx] + accW[blk][i];
        }
      if (a == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int idx = (rq + i) * 8 + cq + q;
            gbuf[idx] = (turn == 3) ? pg[i][q] : gbuf[idx] + pg[i][q];
          }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < m * r; e += 256) dst[e] = buf[(e / r) * 16 + (e % r)];
  for (int e = tid; e < r * r; e += 256) dst[m * r + e] = gbuf[(e / r) * 8 + (e % r)];
}

// ------------------------------------------------------------------ r <= 8 pass on 4 x 4 MFMA blocks
// The wide r <= 8 update pass (FP32 X) on the 16-block form of the matrix cores,
// v_mfma_f32_4x4x1_16b_f32: block b = lane / 4 multiplies a 4 x 1 A (lanes 4b .. 4b + 3, or,
// with the broadcast controls cbsz = 4 / abid = a, the lanes 4a .. 4a + 3 for every block)
// by a 1 x 4 B (lanes 4b .. 4b + 3), and lane 4b + j holds column j of the block's 4 x 4
// sum in its four registers (checked on the GPU against host products).  These blocks do
// not pad rank 8 to 16, so the MFMA work per column is less than half that of the 16 x 16
// tiles.  Per 64-column step of a wave, with one column per lane (lane L <-> column j0 + L):
//   - each lane loads X[R][j0 + L] (rows R < MPAD) and H[c][j0 + L] (c < 8): every load
//     instruction reads 256 contiguous bytes of one row;
//   - W^T X (K = rows): for each row R and rank quad g one MFMA, B = the lanes' X[R], A =
//     W[R][4g .. 4g + 3] broadcast from slot 2R + g of the W registers (lane 4s + i of
//     register v holds W[R][4g + i] for slot 16v + s = 2R + g); lane L then holds ranks
//     4g .. 4g + 3 of its own column, which is what the epilogue needs;
//   - D_H = G_W H and the epilogue of the lane's column (VALU, as in k_mu_pass_r8w), H_new
//     stored;
//   - X and H_new go to per-wave LDS tiles ([row][column]) for X H_new^T and
//     H_new H_new^T (K = columns): block b = 4u + s takes the columns 16s .. 16s + 15 of
//     the step, one per MFMA; for X H_new^T, u = (rank quad kq, row half rh) of each 8-row
//     group; for H_new H_new^T, u = (rank quads cg, qg).  The four column slots s of a
//     block are added at the end of the pass.
// Partials as in k_mu_pass_r8w (X H_new^T as m x r, then H_new H_new^T as r x r, the waves
// added in the order 3, 2, 1, 0).
__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}
// the same with A taken from block `abid` for every block (abid folds to a constant when
// the caller's loops are unrolled)
__device__ __forceinline__ v4f mfma4_bc(float a, float b, v4f c, int abid) {
  switch (abid) {
    case 0: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 0, 0);
    case 1: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 1, 0);
    case 2: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 2, 0);
    case 3: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 3, 0);
    case 4: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 4, 0);
    case 5: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 5, 0);
    case 6: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 6, 0);
    case 7: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 7, 0);
    case 8: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 8, 0);
    case 9: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 9, 0);
    case 10: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 10, 0);
    case 11: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 11, 0);
    case 12: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 12, 0);
    case 13: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 13, 0);
    case 14: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 14, 0);
    default: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 15, 0);
  }
}

template <int MPAD>
__global__ __launch_bounds__(256) void k_mu_pass_r8m(PassArgs p) {
  constexpr int NP = MPAD / 8;  // 8-row groups
  constexpr int NV = MPAD / 8;  // W registers: 2 MPAD slots of four lanes, 16 per register
  constexpr int SX = 68;        // row stride of the per-wave tiles (floats)
  __shared__ __attribute__((aligned(16))) float sWt[16][MPAD + 4];
  __shared__ __attribute__((aligned(16))) float sG[8][8];
  __shared__ __attribute__((aligned(16))) float sX[4][MPAD * SX];
  __shared__ __attribute__((aligned(16))) float sHn[4][8 * SX];

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = p.m, r = p.r;
  const int64_t k = p.k;
  const int64_t nsteps = (k + 63) >> 6;

  r8_w_setup<MPAD>(p, sWt, sG, tid, tid >> 6, lane & 15, lane >> 4);
  __syncthreads();
  float wab[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int slot = 16 * v + (lane >> 2);
    wab[v] = sWt[4 * (slot & 1) + (lane & 3)][slot >> 1];  // W[R][4g + i], zero past m and r
  }
  // roles in the K = columns products: block blk = 4u + s, lane index i4 within the block
  const int blk = lane >> 2, i4 = lane & 3, cs = blk & 3, u = blk >> 2;
  const int kq = u & 1, rh = u >> 1;  // X H^T: rank quad, row half; H H^T: qg = kq, cg = rh

  v4f accX[NP];
  v4f accG = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) accX[pp] = v4f{0.f, 0.f, 0.f, 0.f};
  float* sXw = sX[w];
  float* sHw = sHn[w];

  // X and H through buffer loads: a row's byte offset (below 2^32, checked at launch) in
  // the scalar offset, the lane's column in the vector offset, so no per-load address
  // arithmetic.  Rows past m and columns past k read clamped (valid) addresses: W is zero
  // there and G_W past r, so they add exact zeros, and H_new is masked to zero past k.
  const __amdgpu_buffer_rsrc_t rsX =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p.X), (short)0, -1, 0x00020000);
  const __amdgpu_buffer_rsrc_t rsH = __builtin_amdgcn_make_buffer_rsrc(p.H, (short)0, -1, 0x00020000);
  const uint32_t k4 = (uint32_t)k * 4u;

  // every wave takes a contiguous run of steps: at any moment the waves of the GPU then
  // read few, long runs of each row of X (DRAM page locality), rather than 256-byte pieces
  // spread over whole rows
  const int64_t spw = (nsteps + 4 * (int64_t)gridDim.x - 1) / (4 * (int64_t)gridDim.x);
  const int64_t sw0 = ((int64_t)blockIdx.x * 4 + w) * spw, sw1 = min(nsteps, sw0 + spw);
  for (int64_t st = sw0; st < sw1; ++st) {
    const int64_t j0 = st << 6;
    const bool colok = j0 + lane < k;
    const int lc4 = 4 * (colok ? lane : (int)(k - 1 - j0));  // clamped column (ragged last step)
    const uint32_t j04 = (uint32_t)j0 * 4u;
    float x[MPAD], hv[8];
#pragma unroll
    for (int R = 0; R < MPAD; ++R)
      x[R] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsX, lc4, (int)((uint32_t)min(R, m - 1) * k4 + j04), 0));
#pragma unroll
    for (int c = 0; c < 8; ++c)
      hv[c] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsH, lc4, (int)((uint32_t)min(c, r - 1) * k4 + j04), 0));

    // W^T X: ranks 4g .. 4g + 3 of the lane's column, the even and the odd rows in separate
    // sums (four independent MFMA chains), added at the end
    v4f n2[2][2] = {{v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}},
                    {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}}};
#pragma unroll
    for (int R = 0; R < MPAD; ++R)
#pragma unroll
      for (int g = 0; g < 2; ++g)
        n2[R & 1][g] = mfma4_bc(wab[(2 * R + g) >> 4], x[R], n2[R & 1][g], (2 * R + g) & 15);
    const v4f n[2] = {n2[0][0] + n2[1][0], n2[0][1] + n2[1][1]};

    // D_H = G_W H and the epilogue of the lane's column (ranks 0..7)
    float hnew[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float4 g0 = *reinterpret_cast<const float4*>(&sG[c][0]);
      const float4 g1 = *reinterpret_cast<const float4*>(&sG[c][4]);
      float dh = g0.x * hv[0];
      dh = fmaf(g0.y, hv[1], dh);
      dh = fmaf(g0.z, hv[2], dh);
      dh = fmaf(g0.w, hv[3], dh);
      dh = fmaf(g1.x, hv[4], dh);
      dh = fmaf(g1.y, hv[5], dh);
      dh = fmaf(g1.z, hv[6], dh);
      dh = fmaf(g1.w, hv[7], dh);
      const float q = fmaxf(0.f, fast_div(hv[c] * n[c >> 2][c & 3], dh + p.eps));
      hnew[c] = (c < r && colok) ? q : 0.f;
    }
    if (colok) {
      float* hd = p.H + j0 + lane;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < r) __builtin_nontemporal_store(hnew[c], hd + (int64_t)c * k);
    }
    // X and H_new to the wave's tiles, then X H_new^T and H_new H_new^T (K = columns)
    wave_sync();
#pragma unroll
    for (int R = 0; R < MPAD; ++R) sXw[R * SX + lane] = x[R];
#pragma unroll
    for (int c = 0; c < 8; ++c) sHw[c * SX + lane] = hnew[c];
    wave_sync();
#pragma unroll
    for (int mq = 0; mq < 4; ++mq) {
      const int c0 = 16 * cs + 4 * mq;
      const float4 hb4 = *reinterpret_cast<const float4*>(&sHw[(4 * kq + i4) * SX + c0]);
      const float4 ha4 = *reinterpret_cast<const float4*>(&sHw[(4 * rh + i4) * SX + c0]);
      float4 xa4[NP];
#pragma unroll
      for (int pp = 0; pp < NP; ++pp)
        xa4[pp] = *reinterpret_cast<const float4*>(&sXw[(8 * pp + 4 * rh + i4) * SX + c0]);
      const float hb[4] = {hb4.x, hb4.y, hb4.z, hb4.w};
      const float ha[4] = {ha4.x, ha4.y, ha4.z, ha4.w};
      // column by column, the NP + 1 accumulators interleaved (independent chains)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        accG = mfma4(ha[q], hb[q], accG);
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
          const float xq = q == 0 ? xa4[pp].x : q == 1 ? xa4[pp].y : q == 2 ? xa4[pp].z : xa4[pp].w;
          accX[pp] = mfma4(xq, hb[q], accX[pp]);
        }
      }
    }
  }

  // the four column slots of every block added (lanes 16u + 4s + j, s = 0..3): lane s = 0
  // then holds X H^T[8pp + 4rh + i][4kq + j] and H H^T[4rh + i][4kq + j] in register i
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int pp = 0; pp < NP; ++pp) {
      float v = accX[pp][q];
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      accX[pp][q] = v;
    }
    float v = accG[q];
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    accG[q] = v;
  }
  // per-workgroup partials, waves added in the order 3, 2, 1, 0
  float* dst = p.part + (int64_t)blockIdx.x * p.part_stride;
  float* buf = &sX[0][0];    // MPAD x 8 floats
  float* gbuf = &sHn[0][0];  // 8 x 8 floats
  __syncthreads();
  for (int turn = 3; turn >= 0; --turn) {
    if (w == turn && cs == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int pp = 0; pp < NP; ++pp) {
          const int idx = (8 * pp + 4 * rh + q) * 8 + 4 * kq + i4;
          buf[idx] = (turn == 3) ? accX[pp][q] : buf[idx] + accX[pp][q];
        }
        const int gi = (4 * rh + q) * 8 + 4 * kq + i4;
        gbuf[gi] = (turn == 3) ? accG[q] : gbuf[gi] + accG[q];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < m * r; e += 256) dst[e] = buf[(e / r) * 8 + (e % r)];
  for (int e = tid; e < r * r; e += 256) dst[m * r + e] = gbuf[(e / r) * 8 + (e % r)];
}

// ------------------------------------------------------------------ pass for at most 4 rows
// Update pass for unfoldings of m <= MP <= 4 rows (so r <= 4 too), where a 16-row MFMA
// tile would be mostly padding: one column per lane on the VALU.  Per column j:
// x = X[:, j], h = H[:, j] (coalesced across the workgroup, U columns per lane with all
// their loads issued together); N = W^T x and D = G_W h (rows and ranks in order, FP32),
// H_new = max(0, h N / (D + eps)) stored; x H_new^T and H_new H_new^T accumulated per
// lane.  At the end each accumulator is summed over the wave's 64 lanes by a fixed
// butterfly and over the 4 waves in order: one partial per workgroup (m x r, then r x r).
// Rows >= m and ranks >= r: W, G_W and H beyond them are zero, so they add nothing.
// (At 8 rows the loop-invariant W and G_W held in registers next to 128 accumulators
// take all 256 VGPRs, one wave per SIMD; 5..8 rows stay on the 16-row-block pass.)
template <int MP, int U, bool XBF>
__global__ __launch_bounds__(256) void k_mu_pass_tiny(PassArgs p) {
  __shared__ float sW[MP][MP];  // W (m x r), zero padded
  __shared__ float sG[MP][MP];  // W^T W, zero padded
  __shared__ float sAcc[4][2 * MP * MP];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;
  if (tid < MP * MP) {
    const int i = tid / MP, q = tid % MP;
    sW[i][q] = zmask(p.W[(int64_t)min(i, m - 1) * r + min(q, r - 1)], i < m && q < r);
    sG[i][q] = zmask(p.GW[i * 16 + q], i < r && q < r);
  }
  __syncthreads();
  float axh[MP][MP], ahh[MP][MP];
#pragma unroll
  for (int i = 0; i < MP; ++i)
#pragma unroll
    for (int q = 0; q < MP; ++q) {
      axh[i][q] = 0.f;
      ahh[i][q] = 0.f;
    }
  const int64_t span = (int64_t)256 * U;
  for (int64_t base = (int64_t)blockIdx.x * span; base < k; base += (int64_t)gridDim.x * span) {
    float x[U][MP], h[U][MP];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t cc = min(base + 256 * u + tid, k - 1);
#pragma unroll
      for (int i = 0; i < MP; ++i) x[u][i] = ldx<XBF>(p, (int64_t)min(i, m - 1) * k + cc);
#pragma unroll
      for (int q = 0; q < MP; ++q) h[u][q] = p.H[(int64_t)min(q, r - 1) * k + cc];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t c = base + 256 * u + tid;
      const bool ok = c < k;
      float hn[MP];
#pragma unroll
      for (int q = 0; q < MP; ++q) {
        float nq = 0.f, dq = 0.f;
#pragma unroll
        for (int i = 0; i < MP; ++i) nq = fmaf(sW[i][q], x[u][i], nq);
#pragma unroll
        for (int pp = 0; pp < MP; ++pp) dq = fmaf(sG[q][pp], h[u][pp], dq);
        const float hq = zmask(h[u][q], ok && q < r);
        hn[q] = fmaxf(0.f, fast_div(hq * nq, dq + p.eps));
      }
      if (ok) {
#pragma unroll
        for (int q = 0; q < MP; ++q)
          if (q < r) p.H[(int64_t)q * k + c] = hn[q];
      }
#pragma unroll
      for (int i = 0; i < MP; ++i)
#pragma unroll
        for (int q = 0; q < MP; ++q) axh[i][q] = fmaf(x[u][i], hn[q], axh[i][q]);
#pragma unroll
      for (int q = 0; q < MP; ++q)
#pragma unroll
        for (int pp = 0; pp < MP; ++pp) ahh[q][pp] = fmaf(hn[q], hn[pp], ahh[q][pp]);
    }
  }
  // the 64 lanes by a fixed butterfly, then the waves in order
#pragma unroll
  for (int i = 0; i < MP; ++i)
#pragma unroll
    for (int q = 0; q < MP; ++q) {
      float v = axh[i][q], g = ahh[i][q];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        v += __shfl_xor(v, off, 64);
        g += __shfl_xor(g, off, 64);
      }
      if (lane == 0) {
        sAcc[w][i * MP + q] = v;
        sAcc[w][MP * MP + i * MP + q] = g;
      }
    }
  __syncthreads();
  float* dst = p.part + (int64_t)blockIdx.x * p.part_stride;
  if (tid < 2 * MP * MP) {
    const float v = ((sAcc[0][tid] + sAcc[1][tid]) + sAcc[2][tid]) + sAcc[3][tid];
    if (tid < MP * MP) {
      const int i = tid / MP, q = tid % MP;
      if (i < m && q < r) dst[i * r + q] = v;
    } else {
      const int e = tid - MP * MP, q = e / MP, pp = e % MP;
      if (q < r && pp < r) dst[m * r + q * r + pp] = v;
    }
  }
}

// ------------------------------------------------------------------ wide r <= 8 pass
// The r <= 8 pass over 64-column steps, one step per wave, X read as in the wide
// row-split pass: lane (a, b) loads X[4i + b][j0 + 4a .. 4a + 3] for row quads i (4 rows
// x 256 bytes per load instruction), which is directly the B operand of W^T X for the
// column sets q = 0..3 (columns j0 + 4a + q).  Per step:
//   - the W^T X values of ranks < 8 and the H tile go to LDS as [column][rank], and each
//     lane takes one column (lane l: column j0 + l) for D_H = G_W H (VALU, 8 x 8) and the
//     epilogue of its 8 ranks;
//   - H_new goes to LDS as [rank][column] and to HBM (rows of 256 bytes);
//   - X H_new^T per 16-row block (X through a per-wave transposition tile) and
//     H_new H_new^T, both with MFMA (K = columns).
// Partials as in k_mu_pass_r8 (waves added in the order 3, 2, 1, 0).
template <int NQ, bool XBF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1)))
void k_mu_pass_r8w(PassArgs p) {
  constexpr int MPAD = 4 * NQ;  // 16 or 32 rows
  constexpr int NB = NQ / 4;    // 16-row blocks
  constexpr int ST = 68;        // row stride of the 64-column tiles
  constexpr int SC = 9;         // row stride of the [column][rank] tiles
  __shared__ __attribute__((aligned(16))) float sWt[16][MPAD + 4];
  __shared__ __attribute__((aligned(16))) float sG[8][8];
  __shared__ __attribute__((aligned(16))) float sT[4][16 * ST];  // per-wave X block
  __shared__ __attribute__((aligned(16))) float sHn[4][8 * ST];  // per-wave H_new [rank][col]
  __shared__ float sNc[4][64 * SC];                              // per-wave W^T X [col][rank]
  __shared__ float sHc[4][64 * SC];                              // per-wave H [col][rank]

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;
  const int64_t nsteps = (k + 63) >> 6;
  const int64_t wstride = (int64_t)gridDim.x * 4;
  const bool vec_ok = ((k & 3) == 0) && x_aligned<XBF>(p) &&
                      ((reinterpret_cast<uintptr_t>(p.H) & 15) == 0);
  const float* hrow0 = p.H + (int64_t)min(b, r - 1) * k;      // H rows b and b + 4 (clamped)
  const float* hrow1 = p.H + (int64_t)min(b + 4, r - 1) * k;

  auto load_step = [&](int64_t st, float4 (&x)[NQ], float4 (&h)[2]) {
    const int64_t j0 = st << 6;
    if (vec_ok && (j0 + 64 <= k)) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) x[i] = ldx4<XBF>(p, (int64_t)min(4 * i + b, m - 1) * k + j0 + 4 * a);
      h[0] = *reinterpret_cast<const float4*>(hrow0 + j0 + 4 * a);
      h[1] = *reinterpret_cast<const float4*>(hrow1 + j0 + 4 * a);
    } else {  // ragged or unaligned step (rare): masked here
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t col = j0 + 4 * a + q;
          v[q] = zmask(ldx<XBF>(p, (int64_t)min(4 * i + b, m - 1) * k + min(col, k - 1)), col < k);
        }
        x[i] = make_float4(v[0], v[1], v[2], v[3]);
      }
      float v0[4], v1[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = j0 + 4 * a + q;
        v0[q] = zmask(hrow0[min(col, k - 1)], col < k);
        v1[q] = zmask(hrow1[min(col, k - 1)], col < k);
      }
      h[0] = make_float4(v0[0], v0[1], v0[2], v0[3]);
      h[1] = make_float4(v1[0], v1[1], v1[2], v1[3]);
    }
  };

  int64_t st = (int64_t)blockIdx.x * 4 + w;
  r8_w_setup<MPAD>(p, sWt, sG, tid, w, a, b);
  __syncthreads();
  float wa[NQ];  // W^T as the A operand of W^T X: W[4i + b][a] (zero past m and r)
#pragma unroll
  for (int i = 0; i < NQ; ++i) wa[i] = sWt[a][4 * i + b];

  v4f accW[NB];
  v4f accG = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int blk = 0; blk < NB; ++blk) accW[blk] = v4f{0.f, 0.f, 0.f, 0.f};
  float* sN = sNc[w];
  float* sH = sHc[w];
  float* sHw = sHn[w];
  float* sTw = sT[w];

  // every wave takes a contiguous run of steps (DRAM page locality)
  const int64_t spw = (nsteps + wstride - 1) / wstride;
  const int64_t sw0 = ((int64_t)blockIdx.x * 4 + w) * spw, sw1 = min(nsteps, sw0 + spw);
  for (st = sw0; st < sw1; ++st) {
    const int64_t j0 = st << 6;
    float4 x[NQ], h[2];
    load_step(st, x, h);

    // W^T X of the four column sets: lane (a, b) value i of set q is rank 4b + i, column
    // j0 + 4a + q
    v4f nh[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) nh[q] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      nh[0] = mfma16(wa[i], x[i].x, nh[0]);
      nh[1] = mfma16(wa[i], x[i].y, nh[1]);
      nh[2] = mfma16(wa[i], x[i].z, nh[2]);
      nh[3] = mfma16(wa[i], x[i].w, nh[3]);
    }
    wave_sync();
    if (b < 2) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) sN[(4 * a + q) * SC + 4 * b + i] = nh[q][i];
    }
    {
      const float h0v[4] = {h[0].x, h[0].y, h[0].z, h[0].w};
      const float h1v[4] = {h[1].x, h[1].y, h[1].z, h[1].w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        sH[(4 * a + q) * SC + b] = (b < r) ? h0v[q] : 0.f;
        sH[(4 * a + q) * SC + b + 4] = (b + 4 < r) ? h1v[q] : 0.f;
      }
    }
    wave_sync();
    // one column per lane: D_H = G_W H and the epilogue of ranks 0..7
    const int64_t colg = j0 + lane;
    float hc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) hc[c] = sH[lane * SC + c];
    float hnew[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float4 g0 = *reinterpret_cast<const float4*>(&sG[c][0]);
      const float4 g1 = *reinterpret_cast<const float4*>(&sG[c][4]);
      float dh = g0.x * hc[0];
      dh = fmaf(g0.y, hc[1], dh);
      dh = fmaf(g0.z, hc[2], dh);
      dh = fmaf(g0.w, hc[3], dh);
      dh = fmaf(g1.x, hc[4], dh);
      dh = fmaf(g1.y, hc[5], dh);
      dh = fmaf(g1.z, hc[6], dh);
      dh = fmaf(g1.w, hc[7], dh);
      const float q = fmaxf(0.f, fast_div(hc[c] * sN[lane * SC + c], dh + p.eps));
      hnew[c] = (c < r && colg < k) ? q : 0.f;
    }
    // H_new to LDS as [rank][column] and to HBM
#pragma unroll
    for (int c = 0; c < 8; ++c) sHw[c * ST + lane] = hnew[c];
    if (colg < k) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < r) __builtin_nontemporal_store(hnew[c], p.H + (int64_t)c * k + colg);
    }
    wave_sync();
    // B operands H_new[a][j0 + 16g + 4b .. 4b + 3] (ranks 8.. are zero)
    float4 hb[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 v = *reinterpret_cast<const float4*>(&sHw[min(a, 7) * ST + 16 * g + 4 * b]);
      hb[g] = (a < 8) ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // H_new H_new^T (K = columns)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      accG = mfma16(hb[g].x, hb[g].x, accG);
      accG = mfma16(hb[g].y, hb[g].y, accG);
      accG = mfma16(hb[g].z, hb[g].z, accG);
      accG = mfma16(hb[g].w, hb[g].w, accG);
    }
    // X H_new^T per 16-row block (M = row, N = rank, K = column)
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
      wave_sync();
#pragma unroll
      for (int j = 0; j < 4; ++j) *reinterpret_cast<float4*>(&sTw[(4 * j + b) * ST + 4 * a]) = x[4 * blk + j];
      wave_sync();
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 xa = *reinterpret_cast<const float4*>(&sTw[a * ST + 16 * g + 4 * b]);
        accW[blk] = mfma16(xa.x, hb[g].x, accW[blk]);
        accW[blk] = mfma16(xa.y, hb[g].y, accW[blk]);
        accW[blk] = mfma16(xa.z, hb[g].z, accW[blk]);
        accW[blk] = mfma16(xa.w, hb[g].w, accW[blk]);
      }
    }
  }

  // ---- per-workgroup partials, waves added in the order 3, 2, 1, 0
  float* dst = p.part + (int64_t)blockIdx.x * p.part_stride;
  float* buf = &sT[0][0];   // MPAD x 16 floats
  float* gbuf = &sHn[0][0];  // 8 x 8 floats
  __syncthreads();
  for (int turn = 3; turn >= 0; --turn) {
    if (w == turn) {
#pragma unroll
      for (int blk = 0; blk < NB; ++blk)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int idx = (16 * blk + 4 * b + i) * 16 + a;
          buf[idx] = (turn == 3) ? accW[blk][i] : buf[idx] + accW[blk][i];
        }
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 * b + i < 8 && a < 8) {
          const int idx = (4 * b + i) * 8 + a;
          gbuf[idx] = (turn == 3) ? accG[i] : gbuf[idx] + accG[i];
        }
    }
    __syncthreads();
  }
  for (int e = tid; e < m * r; e += 256) dst[e] = buf[(e / r) * 16 + (e % r)];
  for (int e = tid; e < r * r; e += 256) dst[m * r + e] = gbuf[(e / r) * 8 + (e % r)];
}

// ------------------------------------------------------------------ fused MU pass, rows split over waves
// Variant for larger m: the workgroup's NW wavefronts share each 16-column group, wave w
// owning rows [16 MBW w, 16 MBW (w+1)).  Per group: every wave forms its rows' part of
// W^T X (MFMA, K = rows); the parts are summed across waves in the fixed order 0..NW-1
// through LDS (double-buffered by group parity, one barrier per group); every wave then
// applies the same epilogue to the full sum (so all hold the same H_new); wave 0 stores
// H_new and accumulates H_new H_new^T; each wave accumulates X H_new^T for its own rows,
// so that partial needs no cross-wave reduction.  W stays in registers as MFMA operands.
template <int RP, int MBW, int NW, bool UPDATE, bool RESID, bool XBF>
__global__ __launch_bounds__(64 * NW) void k_mu_pass_L(PassArgs p) {
  constexpr int NH = RP / 16;
  constexpr int SX = 20;
  __shared__ __attribute__((aligned(16))) float sX[NW][16 * SX];
  __shared__ __attribute__((aligned(16))) float sNH[UPDATE ? 2 : 1][UPDATE ? NW : 1][RP * 16];
  __shared__ __attribute__((aligned(16))) float sHn[NW][RP * SX];
  __shared__ double sRes[NW];

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;
  const int row0 = w * 16 * MBW;

  // W^T as the A operand of W^T X: wa[blk][h][kk] = W[row0 + 16 blk + 4b + kk][16h + a]
  float wa[MBW][NH][4];
  // W as the A operand of W H (residual): wr[blk][q][kk] = W[row0 + 16 blk + a][16q + 4b + kk]
  float wr[RESID ? MBW : 1][NH][4];
#pragma unroll
  for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int i = row0 + 16 * blk + 4 * b + kk, c = 16 * h + a;
        const float v = p.W[(int64_t)min(i, m - 1) * r + min(c, r - 1)];
        wa[blk][h][kk] = zmask(v, i < m && c < r);
        if (RESID) {
          const int i2 = row0 + 16 * blk + a, c2 = 16 * h + 4 * b + kk;
          const float v2 = p.W[(int64_t)min(i2, m - 1) * r + min(c2, r - 1)];
          wr[blk][h][kk] = zmask(v2, i2 < m && c2 < r);
        }
      }
  float gw[NH][NH][4];
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int q = 0; q < NH; ++q)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) gw[h][q][kk] = p.GW[(16 * h + a) * RP + 16 * q + 4 * b + kk];

  v4f accW[MBW][NH];
  v4f accG[NH][NH];
  double res = 0.0;
#pragma unroll
  for (int i = 0; i < MBW; ++i)
#pragma unroll
    for (int h = 0; h < NH; ++h) accW[i][h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int q = 0; q < NH; ++q) accG[h][q] = v4f{0.f, 0.f, 0.f, 0.f};

  const int64_t ngroups = (k + 15) >> 4;
  const bool vec_ok = ((k & 3) == 0) && x_aligned<XBF>(p) &&
                      ((reinterpret_cast<uintptr_t>(p.H) & 15) == 0);
  float* sXw = sX[w];
  float* sHw = sHn[w];
  int64_t xrow[MBW];  // row offsets of this lane (clamped into the matrix)
#pragma unroll
  for (int blk = 0; blk < MBW; ++blk) xrow[blk] = (int64_t)min(row0 + 16 * blk + a, m - 1) * k;

  // loads of one 16-column group: this wave's X rows and the H tile, at clamped
  // addresses; the values are kept as loaded until the group is processed (mask_group
  // zeroes the out-of-range ones), so that no instruction waits on a prefetch in flight
  auto load_group = [&](int64_t g, float (&xr)[MBW][4], float (&hv)[NH][4]) {
    const int64_t j0 = g << 4;
    if (vec_ok && (j0 + 16 <= k)) {
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk) {
        const float4 v = ldx4<XBF>(p, xrow[blk] + j0 + 4 * b);
        xr[blk][0] = v.x;
        xr[blk][1] = v.y;
        xr[blk][2] = v.z;
        xr[blk][3] = v.w;
      }
    } else {  // ragged or unaligned group (rare): masked here, so the two paths differ
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t col = j0 + 4 * b + q;
          const float v = ldx<XBF>(p, xrow[blk] + min(col, k - 1));
          xr[blk][q] = zmask(v, col < k && row0 + 16 * blk + a < m);
        }
    }
    const int64_t colc = min(j0 + a, k - 1);
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) hv[h][kk] = p.H[(int64_t)min(16 * h + 4 * b + kk, r - 1) * k + colc];
  };
  // Out-of-range X rows reach a result only through the residual (a ragged group is
  // masked as it is loaded); H entries past r or k are zeroed always.
  auto mask_group = [&](int64_t j0, bool full, float (&xr)[MBW][4], float (&hv)[NH][4]) {
    if (RESID && full) {
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
        for (int q = 0; q < 4; ++q) xr[blk][q] = zmask(xr[blk][q], row0 + 16 * blk + a < m);
    }
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        hv[h][kk] = zmask(hv[h][kk], 16 * h + 4 * b + kk < r && (full || j0 + a < k));
  };

  float xn[MBW][4], hn_[NH][4];  // next group, loaded while the current one is processed
  // with pair_groups, groups in pairs (2p, 2p + 1), one after the other: both halves of a
  // 128-byte line of X (and H) are then read by the same workgroup, so the line is
  // fetched once; small stages keep one group per workgroup for parallelism
  const bool pairs = p.pair_groups != 0;
  auto group_of = [&](int64_t it) -> int64_t {
    return pairs ? 2 * ((int64_t)blockIdx.x + (it >> 1) * (int64_t)gridDim.x) + (it & 1)
                 : (int64_t)blockIdx.x + it * (int64_t)gridDim.x;
  };
  int64_t it = 0;
  if (group_of(0) < ngroups) load_group(group_of(0), xn, hn_);
  int par = 0;
  for (int64_t g = group_of(0); g < ngroups; g = group_of(++it), par ^= 1) {
    const int64_t j0 = g << 4;
    const bool full = vec_ok && (j0 + 16 <= k);
    float xr[MBW][4], hv[NH][4];
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
      for (int q = 0; q < 4; ++q) xr[blk][q] = xn[blk][q];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) hv[h][q] = hn_[h][q];
    if (group_of(it + 1) < ngroups) load_group(group_of(it + 1), xn, hn_);
    mask_group(j0, full, xr, hv);
    v4f nh[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) nh[h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk) {
      wave_sync();
      *reinterpret_cast<float4*>(&sXw[a * SX + 4 * b]) =
          make_float4(xr[blk][0], xr[blk][1], xr[blk][2], xr[blk][3]);
      wave_sync();
      float xt[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) xt[kk] = sXw[(4 * b + kk) * SX + a];
      if (UPDATE) {
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) nh[h] = mfma16(wa[blk][h][kk], xt[kk], nh[h]);
      }
      if (RESID) {
        v4f wh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NH; ++q)
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) wh = mfma16(wr[blk][q][kk], hv[q][kk], wh);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double dlt = (double)xt[i] - (double)wh[i];
          res += dlt * dlt;
        }
      }
    }
    if (!UPDATE) continue;
    // sum the waves' parts of W^T X in order
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) sNH[par][w][(16 * h + 4 * b + i) * 16 + a] = nh[h][i];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float s = sNH[par][0][(16 * h + 4 * b + i) * 16 + a];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww) s += sNH[par][ww][(16 * h + 4 * b + i) * 16 + a];
        nh[h][i] = s;
      }
    // D_H = G_W H and the epilogue (identical in every wave)
    v4f dh[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      dh[h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < NH; ++q)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) dh[h] = mfma16(gw[h][q][kk], hv[q][kk], dh[h]);
    }
    wave_sync();
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * h + 4 * b + i;
        const float q = fmaxf(0.f, fast_div(hv[h][i] * nh[h][i], dh[h][i] + p.eps));
        sHw[c * SX + a] = (c < r) ? q : 0.f;
      }
    wave_sync();
    float4 hn4[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) hn4[h] = *reinterpret_cast<const float4*>(&sHw[(16 * h + a) * SX + 4 * b]);
    if (w == 0) {
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int c = 16 * h + a;
        if (c < r) {
          float* dst = p.H + (int64_t)c * k + j0 + 4 * b;
          if (full) {
            st_nt4(dst, hn4[h]);
          } else {
            const float vv[4] = {hn4[h].x, hn4[h].y, hn4[h].z, hn4[h].w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (j0 + 4 * b + q < k) dst[q] = vv[q];
          }
        }
      }
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int q = 0; q < NH; ++q) {
          accG[h][q] = mfma16(hn4[h].x, hn4[q].x, accG[h][q]);
          accG[h][q] = mfma16(hn4[h].y, hn4[q].y, accG[h][q]);
          accG[h][q] = mfma16(hn4[h].z, hn4[q].z, accG[h][q]);
          accG[h][q] = mfma16(hn4[h].w, hn4[q].w, accG[h][q]);
        }
    }
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        accW[blk][h] = mfma16(xr[blk][0], hn4[h].x, accW[blk][h]);
        accW[blk][h] = mfma16(xr[blk][1], hn4[h].y, accW[blk][h]);
        accW[blk][h] = mfma16(xr[blk][2], hn4[h].z, accW[blk][h]);
        accW[blk][h] = mfma16(xr[blk][3], hn4[h].w, accW[blk][h]);
      }
  }

  if (UPDATE) {
    // this wave's rows of X H_new^T, and (wave 0) H_new H_new^T: compact m x r, r x r
    float* dst = p.part + (int64_t)blockIdx.x * p.part_stride;
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = row0 + 16 * blk + 4 * b + i, c = 16 * h + a;
          if (row < m && c < r) dst[(int64_t)row * r + c] = accW[blk][h][i];
        }
    if (w == 0) {
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int q = 0; q < NH; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = 16 * h + 4 * b + i, cc = 16 * q + a;
            if (c < r && cc < r) dst[(int64_t)m * r + c * r + cc] = accG[h][q][i];
          }
    }
  }
  if (RESID) {
    res = wave_sum(res);
    if (lane == 0) sRes[w] = res;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int ww = 0; ww < NW; ++ww) s += sRes[ww];
      p.rpart[blockIdx.x] = s;
    }
  }
}

// ------------------------------------------------------------------ wide row-split pass
// UPDATE-only row-split pass (rank padding 16) that reads X in steps of 64 columns with
// every load instruction covering 4 rows x 256 contiguous bytes.  (Loads of 16 rows x
// 64 bytes, the layout the MFMA A operand of X H^T wants, reach well under half of the
// HBM bandwidth that 256-byte row runs do.)  Lane (a, b) of wave w loads
// X[row0 + 4i + b][j0 + 4a .. 4a+3] for row quads i, which is directly the B operand of
// W^T X (K = row, N = column) for the four column sets {j0 + 4a + q}, q = 0..3; only the
// X H^T product needs X transposed, through a per-wave LDS tile.  Per step:
//   A: each wave forms its rows' part of W^T X for the 4 column sets; parts to LDS;
//   B: wave q < 4 sums the NW parts of column set q in the order 0..NW-1, forms
//      D_H = G_W H (MFMA) and H_new, and writes H_new to an LDS tile of the step;
//   C: the workgroup stores H_new (rows of 256 bytes); wave g < 4 accumulates
//      H_new H_new^T over columns 16g..16g+15; each wave accumulates X H_new^T for its
//      rows (X from registers through the transposition tile).
// Partials as in k_mu_pass_L (the H H^T parts of waves 0..3 summed in that order).
template <int MBW, int NW, bool XBF, bool NT>
__global__ __launch_bounds__(64 * NW) void k_mu_pass_LW(PassArgs p) {
  constexpr int NQ = 4 * MBW;  // row quads per wave
  constexpr int SN = 20;       // row stride of the W^T X parts: [column index][rank]
  constexpr int ST = 68;       // row stride of the 64-column LDS tiles
  static_assert(NW >= 4, "four waves take the four column sets of the epilogue");
  __shared__ __attribute__((aligned(16))) float sNH[4][NW][16 * SN];
  __shared__ __attribute__((aligned(16))) float sHn[16 * ST];
  __shared__ __attribute__((aligned(16))) float sT[NW][16 * ST];

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;
  const int row0 = w * 16 * MBW;

  const int64_t nsteps = (k + 63) >> 6;
  const int64_t nblk = gridDim.x;
  const bool vec_ok = ((k & 3) == 0) && x_aligned<XBF>(p) &&
                      ((reinterpret_cast<uintptr_t>(p.H) & 15) == 0);
  int64_t xrow[NQ];  // row offsets of this lane (clamped into the matrix)
#pragma unroll
  for (int i = 0; i < NQ; ++i) xrow[i] = (int64_t)min(row0 + 4 * i + b, m - 1) * k;
  const float* hrow[4];  // H rows 4b + kk (clamped), read by the epilogue waves
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) hrow[kk] = p.H + (int64_t)min(4 * b + kk, r - 1) * k;
  float* sTw = sT[w];

  // loads of a step: X[row0 + 4i + b][j0 + 4a .. 4a + 3]; wave q < 4 also
  // H[4b + kk][j0 + 4a + q] (values as loaded; the ragged path masks X here)
  auto load_step = [&](int64_t st, float4 (&x)[NQ], float (&hv)[4]) {
    const int64_t j0 = st << 6;
    if (vec_ok && (j0 + 64 <= k)) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) x[i] = ldx4<XBF, NT>(p, xrow[i] + j0 + 4 * a);
    } else {  // ragged or unaligned step (rare)
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t col = j0 + 4 * a + q;
          v[q] = zmask(ldx<XBF>(p, xrow[i] + min(col, k - 1)), col < k && row0 + 4 * i + b < m);
        }
        x[i] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
    if (w < 4) {
      const int64_t colc = min(j0 + 4 * a + w, k - 1);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) hv[kk] = hrow[kk][colc];
    }
  };

  // W^T as the A operand of W^T X: wa[i] = W[row0 + 4i + b][a]; G_W as that of G_W H
  float wa[NQ];
  float gw[4];
  {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int row = row0 + 4 * i + b;
      wa[i] = zmask(p.W[(int64_t)min(row, m - 1) * r + min(a, r - 1)], row < m && a < r);
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) gw[kk] = p.GW[a * 16 + 4 * b + kk];
  }

  v4f accW[MBW];
  v4f accG = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int blk = 0; blk < MBW; ++blk) accW[blk] = v4f{0.f, 0.f, 0.f, 0.f};

  // (steps taken cyclically: measured slightly faster here than contiguous runs per
  // workgroup, unlike the 32-row pass, whose waves read only 32 rows per step)
  // 65..128 rows (MBW = 2): the next step's loads are issued before the current step is
  // processed (two waves per SIMD then; one resident round of 512 workgroups).  Measured
  // on the 128 x 2,097,152 stage: 60.7 -> 58.8 ms for 200 iterations; the 256-row class
  // was slower with it (the 256^4 stage 1 446 -> 510 ms) and keeps single-step loads.
  constexpr bool PF = MBW == 2;
  float4 xn[PF ? NQ : 1];
  float hn[PF ? 4 : 1];
  if constexpr (PF) {
    if (blockIdx.x < nsteps) load_step(blockIdx.x, xn, hn);
  }
  for (int64_t st = blockIdx.x; st < nsteps; st += nblk) {
    const int64_t j0 = st << 6;
    const bool full = vec_ok && (j0 + 64 <= k);
    float4 x[NQ];
    float hv[4];
    if constexpr (PF) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) x[q] = xn[q];
#pragma unroll
      for (int q = 0; q < 4; ++q) hv[q] = hn[q];
      if (st + nblk < nsteps) load_step(st + nblk, xn, hn);
    } else {
      load_step(st, x, hv);
    }

    // A: parts of W^T X of the four column sets, stored as [a][rank 4b + i]
    {
      v4f nh[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) nh[q] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        nh[0] = mfma16(wa[i], x[i].x, nh[0]);
        nh[1] = mfma16(wa[i], x[i].y, nh[1]);
        nh[2] = mfma16(wa[i], x[i].z, nh[2]);
        nh[3] = mfma16(wa[i], x[i].w, nh[3]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<float4*>(&sNH[q][w][a * SN + 4 * b]) =
            make_float4(nh[q][0], nh[q][1], nh[q][2], nh[q][3]);
    }
    __syncthreads();

    // B: the epilogue of column set q = w: columns j0 + 4a + q
    if (w < 4) {
      float4 n4 = *reinterpret_cast<const float4*>(&sNH[w][0][a * SN + 4 * b]);
#pragma unroll
      for (int ww = 1; ww < NW; ++ww) {
        const float4 v = *reinterpret_cast<const float4*>(&sNH[w][ww][a * SN + 4 * b]);
        n4.x += v.x;
        n4.y += v.y;
        n4.z += v.z;
        n4.w += v.w;
      }
      const float nv[4] = {n4.x, n4.y, n4.z, n4.w};
      const int64_t col = j0 + 4 * a + w;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) hv[kk] = zmask(hv[kk], 4 * b + kk < r && col < k);
      v4f dh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) dh = mfma16(gw[kk], hv[kk], dh);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 4 * b + i;
        const float q = fmaxf(0.f, fast_div(hv[i] * nv[i], dh[i] + p.eps));
        sHn[c * ST + 4 * a + w] = (c < r) ? q : 0.f;
      }
    }
    __syncthreads();

    // C: store H_new; H_new H_new^T (wave g < 4: columns 16g ..); X H_new^T per row block
    if (tid < 256) {
      const int c = tid >> 4, cq = 4 * (tid & 15);
      if (c < r) {
        const float4 v = *reinterpret_cast<const float4*>(&sHn[c * ST + cq]);
        float* dst = p.H + (int64_t)c * k + j0 + cq;
        if (full) {
          st_nt4(dst, v);
        } else {
          const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (j0 + cq + q < k) dst[q] = vv[q];
        }
      }
    }
    float4 hn4[4];  // H_new[a][16g + 4b .. 4b + 3]: the B operand of X H_new^T
#pragma unroll
    for (int g = 0; g < 4; ++g) hn4[g] = *reinterpret_cast<const float4*>(&sHn[a * ST + 16 * g + 4 * b]);
    if (w < 4) {  // (read from LDS: indexing hn4 by the wave would put it in scratch)
      const float4 h = *reinterpret_cast<const float4*>(&sHn[a * ST + 16 * w + 4 * b]);
      accG = mfma16(h.x, h.x, accG);
      accG = mfma16(h.y, h.y, accG);
      accG = mfma16(h.z, h.z, accG);
      accG = mfma16(h.w, h.w, accG);
    }
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk) {
      // tile rows 4j + b <- row quad 4 blk + j: X[row0 + 16 blk + rho][j0 + col]
      wave_sync();
#pragma unroll
      for (int j = 0; j < 4; ++j)
        *reinterpret_cast<float4*>(&sTw[(4 * j + b) * ST + 4 * a]) = x[4 * blk + j];
      wave_sync();
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 xa = *reinterpret_cast<const float4*>(&sTw[a * ST + 16 * g + 4 * b]);
        accW[blk] = mfma16(xa.x, hn4[g].x, accW[blk]);
        accW[blk] = mfma16(xa.y, hn4[g].y, accW[blk]);
        accW[blk] = mfma16(xa.z, hn4[g].z, accW[blk]);
        accW[blk] = mfma16(xa.w, hn4[g].w, accW[blk]);
      }
    }
    // the next step's phase B rewrites sHn only after its first barrier, which every
    // wave reaches after these reads
  }

  // partials: this wave's rows of X H_new^T; H_new H_new^T summed over waves 0..3
  float* dst = p.part + (int64_t)blockIdx.x * p.part_stride;
#pragma unroll
  for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = row0 + 16 * blk + 4 * b + i;
      if (row < m && a < r) dst[(int64_t)row * r + a] = accW[blk][i];
    }
  __syncthreads();
  float* gbuf = &sNH[0][0][0];  // 4 x 256 floats, free after the last step
  if (w < 4) {
#pragma unroll
    for (int i = 0; i < 4; ++i) gbuf[w * 256 + (4 * b + i) * 16 + a] = accG[i];
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += 64 * NW) {
    const int c = e / r, cc = e % r;
    dst[(int64_t)m * r + e] = ((gbuf[c * 16 + cc] + gbuf[256 + c * 16 + cc]) + gbuf[512 + c * 16 + cc]) +
                              gbuf[768 + c * 16 + cc];
  }
}

// ------------------------------------------------------------------ wide row-split pass, BF16 MFMA
// The wide row-split update pass for a BF16 copy of X (precision mode) on BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  X stays BF16 as loaded; the
// FP32 factors enter each product as two BF16 terms, f = hi + lo with hi = bf16(f) and
// lo = bf16(f - hi) (round to nearest even), so that W^T X and X H_new^T carry the
// rounding of X alone (every BF16 x BF16 product is exact in FP32).  D_H = G_W H, the
// epilogue and H_new H_new^T stay FP32 as in k_mu_pass_LW, whose structure and partials
// this pass shares, in steps of 128 columns so that every load still covers 4 rows x
// 256 contiguous bytes:
//   lane (a, b) holds X[row0 + 4i + b][j0 + 8a .. 8a + 7] for the row quads i;
//   W^T X (K = rows): for column set q (columns j0 + 8a + q, q = 0..7) the K slot 8b + u
//   of an MFMA is row row0 + 32 gq + 4u + b (u = 0..7, row quads 8 gq .. 8 gq + 7), so
//   the lane's own values of eight row quads are its B operand; W^T is laid out to match;
//   epilogue: wave q' < 4 takes column sets q' and q' + 4;
//   X H_new^T (K = columns): each 16-row block goes through a per-wave BF16 tile; lane
//   (a, b) reads X[row a][c0 + 8b .. 8b + 7] and H_new[a][c0 + 8b ..] (c0 = 0, 32, 64, 96).
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// hi and lo BF16 parts of eight FP32 values, packed two per 32-bit word, by the
// conversion instruction (round to nearest even)
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_bf8(const float (&f)[8], bf8& hi, bf8& lo) {
  u4v h, l;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bf2 hv = {(__bf16)f[2 * j], (__bf16)f[2 * j + 1]};
    const uint32_t hb = __builtin_bit_cast(uint32_t, hv);
    const bf2 lv = {(__bf16)(f[2 * j] - __uint_as_float(hb << 16)),
                    (__bf16)(f[2 * j + 1] - __uint_as_float(hb & 0xffff0000u))};
    h[j] = hb;
    l[j] = __builtin_bit_cast(uint32_t, lv);
  }
  hi = __builtin_bit_cast(bf8, h);
  lo = __builtin_bit_cast(bf8, l);
}
__device__ __forceinline__ v4f mfma32bf(const bf8& a, const bf8& b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// BF16 values q (0..7) of two raw 8 x BF16 loads, packed as lo | hi << 16 (one byte
// permute: selector bytes 0-3 pick bytes of the second source, 4-7 of the first)
__device__ __forceinline__ uint32_t bf_pair(const uint4& lo, const uint4& hi, int q) {
  const uint32_t wl = (q < 2) ? lo.x : (q < 4) ? lo.y : (q < 6) ? lo.z : lo.w;
  const uint32_t wh = (q < 2) ? hi.x : (q < 4) ? hi.y : (q < 6) ? hi.z : hi.w;
  return __builtin_amdgcn_perm(wh, wl, (q & 1) ? 0x07060302u : 0x05040100u);
}

template <int MBW, int NW, bool NT>
__global__ __launch_bounds__(64 * NW) void k_mu_pass_LWB(PassArgs p) {
  constexpr int NQ = 4 * MBW;  // row quads per wave
  constexpr int NG8 = NQ / 8;  // MFMA row groups (eight row quads each) per wave
  constexpr int SN = 20;       // row stride of the W^T X parts: [column index][rank]
  constexpr int ST = 132;      // row stride of the 128-column H_new tile (floats)
  constexpr int SB = 136;      // row stride of the per-wave BF16 X tile (halves, 16-byte rows)
  static_assert(NW >= 4 && NQ % 8 == 0, "four epilogue waves; whole row groups");
  __shared__ __attribute__((aligned(16))) float sNH[8][NW][16 * SN];
  __shared__ __attribute__((aligned(16))) float sHn[16 * ST];
  __shared__ __attribute__((aligned(16))) uint16_t sT[NW][16 * SB];

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;
  const int row0 = w * 16 * MBW;

  const int64_t nsteps = (k + 127) >> 7;
  const int64_t nblk = gridDim.x;
  const bool vec_ok = ((k & 7) == 0) && ((reinterpret_cast<uintptr_t>(p.Xb) & 15) == 0) &&
                      ((reinterpret_cast<uintptr_t>(p.H) & 15) == 0);
  int64_t xrow[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) xrow[i] = (int64_t)min(row0 + 4 * i + b, m - 1) * k;
  const float* hrow[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) hrow[kk] = p.H + (int64_t)min(4 * b + kk, r - 1) * k;
  uint16_t* sTw = sT[w];

  // raw BF16 loads of a step: X[row0 + 4i + b][j0 + 8a .. 8a + 7]; wave q' < 4 also
  // H[4b + kk][j0 + 8a + q' + 4s] (the ragged path masks X here)
  auto load_step = [&](int64_t st, uint4 (&x)[NQ], float (&hv)[2][4]) {
    const int64_t j0 = st << 7;
    if (vec_ok && (j0 + 128 <= k)) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        if constexpr (NT) {
          const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(p.Xb + xrow[i] + j0 + 8 * a));
          x[i] = make_uint4(v[0], v[1], v[2], v[3]);
        } else {
          x[i] = *reinterpret_cast<const uint4*>(p.Xb + xrow[i] + j0 + 8 * a);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        uint32_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int64_t col = j0 + 8 * a + q;
          const uint32_t raw = p.Xb[xrow[i] + min(col, k - 1)];
          v[q] = (col < k && row0 + 4 * i + b < m) ? raw : 0u;
        }
        x[i] = make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16), v[6] | (v[7] << 16));
      }
    }
    if (w < 4) {
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const int64_t colc = min(j0 + 8 * a + w + 4 * sx, k - 1);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) hv[sx][kk] = hrow[kk][colc];
      }
    }
  };

  // W^T as the A operand of W^T X: row group gq, K slot 8b + u <-> row row0 + 32 gq + 4u + b
  bf8 wa_hi[NG8], wa_lo[NG8];
#pragma unroll
  for (int gq = 0; gq < NG8; ++gq) {
    float f[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = row0 + 32 * gq + 4 * u + b;
      f[u] = zmask(p.W[(int64_t)min(row, m - 1) * r + min(a, r - 1)], row < m && a < r);
    }
    split_bf8(f, wa_hi[gq], wa_lo[gq]);
  }
  float gw[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) gw[kk] = p.GW[a * 16 + 4 * b + kk];

  v4f accW[MBW];
  v4f accG = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int blk = 0; blk < MBW; ++blk) accW[blk] = v4f{0.f, 0.f, 0.f, 0.f};

  // the next step's loads are issued before the current step is processed
  uint4 xn[NQ];
  float hn_[2][4];
  if (blockIdx.x < nsteps) load_step(blockIdx.x, xn, hn_);
  for (int64_t st = blockIdx.x; st < nsteps; st += nblk) {
    const int64_t j0 = st << 7;
    const bool full = vec_ok && (j0 + 128 <= k);
    uint4 x[NQ];
    float hv[2][4];
#pragma unroll
    for (int i = 0; i < NQ; ++i) x[i] = xn[i];
#pragma unroll
    for (int sx = 0; sx < 2; ++sx)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) hv[sx][kk] = hn_[sx][kk];
    if (st + nblk < nsteps) load_step(st + nblk, xn, hn_);

    // A: parts of W^T X of the eight column sets, stored as [a][rank 4b + i]
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      v4f nh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int gq = 0; gq < NG8; ++gq) {
        u4v xb;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          xb[j] = bf_pair(x[8 * gq + 2 * j], x[8 * gq + 2 * j + 1], q);
        const bf8 xv = __builtin_bit_cast(bf8, xb);
        nh = mfma32bf(wa_hi[gq], xv, nh);
        nh = mfma32bf(wa_lo[gq], xv, nh);
      }
      *reinterpret_cast<float4*>(&sNH[q][w][a * SN + 4 * b]) = make_float4(nh[0], nh[1], nh[2], nh[3]);
    }
    __syncthreads();

    // B: the epilogue of column sets q = w and w + 4: columns j0 + 8a + q
    if (w < 4) {
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const int q = w + 4 * sx;
        float4 n4 = *reinterpret_cast<const float4*>(&sNH[q][0][a * SN + 4 * b]);
#pragma unroll
        for (int ww = 1; ww < NW; ++ww) {
          const float4 v = *reinterpret_cast<const float4*>(&sNH[q][ww][a * SN + 4 * b]);
          n4.x += v.x;
          n4.y += v.y;
          n4.z += v.z;
          n4.w += v.w;
        }
        const float nv[4] = {n4.x, n4.y, n4.z, n4.w};
        const int64_t col = j0 + 8 * a + q;
        float hq[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) hq[kk] = zmask(hv[sx][kk], 4 * b + kk < r && col < k);
        v4f dh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) dh = mfma16(gw[kk], hq[kk], dh);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 4 * b + i;
          const float qv = fmaxf(0.f, fast_div(hq[i] * nv[i], dh[i] + p.eps));
          sHn[c * ST + 8 * a + q] = (c < r) ? qv : 0.f;
        }
      }
    }
    __syncthreads();

    // C: store H_new; H_new H_new^T (FP32, wave g < 4: columns 32g .. 32g + 31); X H_new^T
    // per row block on BF16 matrix cores
    for (int e = tid; e < 16 * 32; e += 64 * NW) {
      const int c = e >> 5, cq = 4 * (e & 31);
      if (c < r) {
        const float4 v = *reinterpret_cast<const float4*>(&sHn[c * ST + cq]);
        float* dst = p.H + (int64_t)c * k + j0 + cq;
        if (full) {
          st_nt4(dst, v);
        } else {
          const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (j0 + cq + q < k) dst[q] = vv[q];
        }
      }
    }
    if (w < 4) {
#pragma unroll
      for (int t2 = 0; t2 < 2; ++t2) {
        const float4 h = *reinterpret_cast<const float4*>(&sHn[a * ST + 32 * w + 16 * t2 + 4 * b]);
        accG = mfma16(h.x, h.x, accG);
        accG = mfma16(h.y, h.y, accG);
        accG = mfma16(h.z, h.z, accG);
        accG = mfma16(h.w, h.w, accG);
      }
    }
    // H_new[a][c0 + 8b .. 8b + 7] as hi + lo BF16, the B operand of X H_new^T
    bf8 hn_hi[4], hn_lo[4];
#pragma unroll
    for (int h2 = 0; h2 < 4; ++h2) {
      const float4 f0 = *reinterpret_cast<const float4*>(&sHn[a * ST + 32 * h2 + 8 * b]);
      const float4 f1 = *reinterpret_cast<const float4*>(&sHn[a * ST + 32 * h2 + 8 * b + 4]);
      const float f[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
      split_bf8(f, hn_hi[h2], hn_lo[h2]);
    }
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk) {
      // tile row 4j + b <- row quad 4 blk + j: X[row0 + 16 blk + rho][j0 + col] (BF16)
      wave_sync();
#pragma unroll
      for (int j = 0; j < 4; ++j)
        *reinterpret_cast<uint4*>(&sTw[(4 * j + b) * SB + 8 * a]) = x[4 * blk + j];
      wave_sync();
#pragma unroll
      for (int h2 = 0; h2 < 4; ++h2) {
        const uint4 t = *reinterpret_cast<const uint4*>(&sTw[a * SB + 32 * h2 + 8 * b]);
        const bf8 xa = __builtin_bit_cast(bf8, u4v{t.x, t.y, t.z, t.w});
        accW[blk] = mfma32bf(xa, hn_hi[h2], accW[blk]);
        accW[blk] = mfma32bf(xa, hn_lo[h2], accW[blk]);
      }
    }
  }

  // partials: this wave's rows of X H_new^T; H_new H_new^T summed over waves 0..3
  float* dst = p.part + (int64_t)blockIdx.x * p.part_stride;
#pragma unroll
  for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = row0 + 16 * blk + 4 * b + i;
      if (row < m && a < r) dst[(int64_t)row * r + a] = accW[blk][i];
    }
  __syncthreads();
  float* gbuf = &sNH[0][0][0];  // 4 x 256 floats, free after the last step
  if (w < 4) {
#pragma unroll
    for (int i = 0; i < 4; ++i) gbuf[w * 256 + (4 * b + i) * 16 + a] = accG[i];
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += 64 * NW) {
    const int c = e / r, cc = e % r;
    dst[(int64_t)m * r + e] = ((gbuf[c * 16 + cc] + gbuf[256 + c * 16 + cc]) + gbuf[512 + c * 16 + cc]) +
                              gbuf[768 + c * 16 + cc];
  }
}

// ------------------------------------------------------------------ row-chunked MU pass
// For m beyond one workgroup: rows are cut into chunks of CR = 16 MBW NW rows, chunk y
// taken by the workgroups with blockIdx.y = y, which visit the same 16-column groups for
// every chunk.  One MU iteration is two launches, each reading X once:
//   phase 1: per group, the chunk's part of W^T X (waves as in the row-split pass, summed
//            over the workgroup's waves in order) is stored to S[y] (r x k); chunk 0
//            also copies the group's H to Hs;
//   (k_sum_chunks between them: S[0] <- S[0] + S[1] + ..., in chunk order;)
//   phase 2: per group, N_H = S[0], the H-update epilogue in every wave (H read from Hs:
//            the workgroups of the other chunks may still be reading a group whose H
//            chunk 0 has already replaced), H_new stored and H_new H_new^T accumulated by
//            wave 0 of chunk 0, X H_new^T accumulated for each wave's own rows.  Workgroup (x, y) writes the chunk-y rows of partial x
//            (chunk 0 also its H H^T part), so the gridDim.x partials are complete, as
//            after the fused passes;
//   phase 0: the residual of the wave's rows, to rpart[y gridDim.x + x].
template <int RP, int MBW, int NW, int PH, bool XBF, int PD = 1>
__global__ __launch_bounds__(64 * NW) void k_mu_pass_C(PassArgs p) {
  constexpr int NH = RP / 16;
  constexpr int SX = 20;
  constexpr int CR = 16 * MBW * NW;
  __shared__ __attribute__((aligned(16))) float sX[NW][16 * SX];
  __shared__ __attribute__((aligned(16))) float sNH[PH == 1 ? 2 : 1][PH == 1 ? NW : 1][RP * 16];
  __shared__ __attribute__((aligned(16))) float sHn[NW][RP * SX];
  __shared__ double sRes[NW];

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;
  const int y = blockIdx.y;
  const int row0 = y * CR + w * 16 * MBW;
  const int64_t ngroups = (k + 15) >> 4;
  const bool vec_ok = ((k & 3) == 0) && x_aligned<XBF>(p) &&
                      ((reinterpret_cast<uintptr_t>(p.H) & 15) == 0);

  // phase 1: W^T as the A operand of W^T X; phase 0: W as the A operand of W H
  float wa[PH == 1 ? MBW : 1][NH][4];
  float wr[PH == 0 ? MBW : 1][NH][4];
#pragma unroll
  for (int blk = 0; blk < (PH == 2 ? 0 : MBW); ++blk)
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        if (PH == 1) {
          const int i = row0 + 16 * blk + 4 * b + kk, c = 16 * h + a;
          wa[blk][h][kk] = zmask(p.W[(int64_t)min(i, m - 1) * r + min(c, r - 1)], i < m && c < r);
        } else {
          const int i2 = row0 + 16 * blk + a, c2 = 16 * h + 4 * b + kk;
          wr[blk][h][kk] = zmask(p.W[(int64_t)min(i2, m - 1) * r + min(c2, r - 1)], i2 < m && c2 < r);
        }
      }
  float gw[PH == 2 ? NH : 1][PH == 2 ? NH : 1][4];
  if (PH == 2) {
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int q = 0; q < NH; ++q)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) gw[h][q][kk] = p.GW[(16 * h + a) * RP + 16 * q + 4 * b + kk];
  }
  v4f accW[PH == 2 ? MBW : 1][NH];
  v4f accG[NH][NH];
#pragma unroll
  for (int i = 0; i < (PH == 2 ? MBW : 1); ++i)
#pragma unroll
    for (int h = 0; h < NH; ++h) accW[i][h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int q = 0; q < NH; ++q) accG[h][q] = v4f{0.f, 0.f, 0.f, 0.f};
  double res = 0.0;

  float* sXw = sX[w];
  float* sHw = sHn[w];
  int64_t xrow[MBW];
#pragma unroll
  for (int blk = 0; blk < MBW; ++blk) xrow[blk] = (int64_t)min(row0 + 16 * blk + a, m - 1) * k;

  // X rows of the wave (rows past m: zero in phase 0, unused otherwise), the H tile
  // (phases 0 and 2) and the summed W^T X (phase 2) of group g
  // (loaded values are kept as they are until the group is processed: mask_group then
  // zeroes the out-of-range ones, so no instruction waits on a prefetch in flight)
  auto load_group = [&](int64_t g, float (&xr)[MBW][4], float (&hv)[NH][4], float (&sv)[NH][4]) {
    const int64_t j0 = g << 4;
    if (vec_ok && (j0 + 16 <= k)) {
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk) {
        const float4 v = ldx4<XBF>(p, xrow[blk] + j0 + 4 * b);
        xr[blk][0] = v.x;
        xr[blk][1] = v.y;
        xr[blk][2] = v.z;
        xr[blk][3] = v.w;
      }
    } else {  // ragged or unaligned group (rare): masked here, so the two paths differ
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t col = j0 + 4 * b + q;
          const float v = ldx<XBF>(p, xrow[blk] + min(col, k - 1));
          xr[blk][q] = zmask(v, col < k && row0 + 16 * blk + a < m);
        }
    }
    const int64_t colc = min(j0 + a, k - 1);
    if (PH != 1 || (y == 0 && w == 0)) {
      const float* Hsrc = PH == 2 ? p.Hs : p.H;
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) hv[h][kk] = Hsrc[(int64_t)min(16 * h + 4 * b + kk, r - 1) * k + colc];
    }
    if (PH == 2) {
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) sv[h][kk] = p.S[(int64_t)min(16 * h + 4 * b + kk, r - 1) * k + colc];
    }
  };
  // X rows >= m matter to the residual (phase 0; a ragged group is masked as it is
  // loaded); the H and S tiles past r or k are zeroed always
  auto mask_group = [&](int64_t j0, bool full, float (&xr)[MBW][4], float (&hv)[NH][4], float (&sv)[NH][4]) {
    if (PH == 0 && full) {
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
        for (int q = 0; q < 4; ++q) xr[blk][q] = zmask(xr[blk][q], row0 + 16 * blk + a < m);
    }
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const bool ok = 16 * h + 4 * b + kk < r && (full || j0 + a < k);
        if (PH != 1 || (y == 0 && w == 0)) hv[h][kk] = zmask(hv[h][kk], ok);
        if (PH == 2) sv[h][kk] = zmask(sv[h][kk], ok);
      }
  };

  // with pair_groups, groups in pairs (2p, 2p + 1), one after the other: both halves of a
  // 128-byte line of X (and H) are then read by the same workgroup, so the line is
  // fetched once; small stages keep one group per workgroup for parallelism
  const bool pairs = p.pair_groups != 0;
  // on the BF16 copy each workgroup takes a contiguous run of groups instead (measured on
  // the 2048 x 16,384 stage: 19.4 -> 18.0 ms in BF16, but 16.6 -> 18.4 ms in FP32)
  const int64_t gpb = (ngroups + gridDim.x - 1) / gridDim.x;
  auto group_of = [&](int64_t it) -> int64_t {
    if (XBF) return it < gpb ? (int64_t)blockIdx.x * gpb + it : ngroups;
    return pairs ? 2 * ((int64_t)blockIdx.x + (it >> 1) * (int64_t)gridDim.x) + (it & 1)
                 : (int64_t)blockIdx.x + it * (int64_t)gridDim.x;
  };
  // PD groups in flight: with PD = 2 the loop is unrolled by two over buffers A and B, so
  // taking a group out of its buffer waits only for that group's loads
  static_assert(PD == 1 || PD == 2, "one or two groups in flight");
  auto step = [&](int64_t g, int64_t it, int par, float (&xn)[MBW][4], float (&hn_)[NH][4], float (&sn)[NH][4]) {
    const int64_t j0 = g << 4;
    const bool full = vec_ok && (j0 + 16 <= k);
    float xr[MBW][4], hv[NH][4], sv[NH][4];
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
      for (int q = 0; q < 4; ++q) xr[blk][q] = xn[blk][q];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) hv[h][q] = hn_[h][q];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) sv[h][q] = sn[h][q];
    if (group_of(it + PD) < ngroups) load_group(group_of(it + PD), xn, hn_, sn);
    mask_group(j0, full, xr, hv, sv);

    if (PH != 2) {
      v4f nh[NH];
#pragma unroll
      for (int h = 0; h < NH; ++h) nh[h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk) {
        wave_sync();
        *reinterpret_cast<float4*>(&sXw[a * SX + 4 * b]) =
            make_float4(xr[blk][0], xr[blk][1], xr[blk][2], xr[blk][3]);
        wave_sync();
        float xt[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) xt[kk] = sXw[(4 * b + kk) * SX + a];
        if (PH == 1) {
#pragma unroll
          for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) nh[h] = mfma16(wa[blk][h][kk], xt[kk], nh[h]);
        } else {
          v4f wh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < NH; ++q)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) wh = mfma16(wr[blk][q][kk], hv[q][kk], wh);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double dlt = (double)xt[i] - (double)wh[i];
            res += dlt * dlt;
          }
        }
      }
      if (PH == 1) {
        if (y == 0 && w == 0) {  // H of the group, for phase 2
#pragma unroll
          for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
              const int c = 16 * h + 4 * b + kk;
              if (c < r && j0 + a < k) p.Hs[(int64_t)c * k + j0 + a] = hv[h][kk];
            }
        }
        // sum the waves' parts in order; wave 0 stores the chunk's W^T X of the group
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
          for (int i = 0; i < 4; ++i) sNH[par][w][(16 * h + 4 * b + i) * 16 + a] = nh[h][i];
        __syncthreads();
        if (w == 0) {
#pragma unroll
          for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              float sum = sNH[par][0][(16 * h + 4 * b + i) * 16 + a];
#pragma unroll
              for (int ww = 1; ww < NW; ++ww) sum += sNH[par][ww][(16 * h + 4 * b + i) * 16 + a];
              const int c = 16 * h + 4 * b + i;
              if (c < r && j0 + a < k) p.S[((int64_t)y * r + c) * k + j0 + a] = sum;
            }
        }
      }
      return;
    }

    // phase 2: N_H, D_H = G_W H, the epilogue (identical in every wave)
    v4f nh[NH], dh[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
#pragma unroll
      for (int i = 0; i < 4; ++i) nh[h][i] = sv[h][i];
      dh[h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < NH; ++q)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) dh[h] = mfma16(gw[h][q][kk], hv[q][kk], dh[h]);
    }
    wave_sync();
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * h + 4 * b + i;
        const float q = fmaxf(0.f, fast_div(hv[h][i] * nh[h][i], dh[h][i] + p.eps));
        sHw[c * SX + a] = (c < r) ? q : 0.f;
      }
    wave_sync();
    float4 hn4[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) hn4[h] = *reinterpret_cast<const float4*>(&sHw[(16 * h + a) * SX + 4 * b]);
    if (y == 0 && w == 0) {
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int c = 16 * h + a;
        if (c < r) {
          float* dst = p.H + (int64_t)c * k + j0 + 4 * b;
          if (full) {
            st_nt4(dst, hn4[h]);
          } else {
            const float vv[4] = {hn4[h].x, hn4[h].y, hn4[h].z, hn4[h].w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (j0 + 4 * b + q < k) dst[q] = vv[q];
          }
        }
      }
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int q = 0; q < NH; ++q) {
          accG[h][q] = mfma16(hn4[h].x, hn4[q].x, accG[h][q]);
          accG[h][q] = mfma16(hn4[h].y, hn4[q].y, accG[h][q]);
          accG[h][q] = mfma16(hn4[h].z, hn4[q].z, accG[h][q]);
          accG[h][q] = mfma16(hn4[h].w, hn4[q].w, accG[h][q]);
        }
    }
#pragma unroll
    for (int blk = 0; blk < (PH == 2 ? MBW : 0); ++blk)
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        accW[blk][h] = mfma16(xr[blk][0], hn4[h].x, accW[blk][h]);
        accW[blk][h] = mfma16(xr[blk][1], hn4[h].y, accW[blk][h]);
        accW[blk][h] = mfma16(xr[blk][2], hn4[h].z, accW[blk][h]);
        accW[blk][h] = mfma16(xr[blk][3], hn4[h].w, accW[blk][h]);
      }
  };
  float xA[MBW][4], hA[NH][4], sA[NH][4];
  if (group_of(0) < ngroups) load_group(group_of(0), xA, hA, sA);
  if constexpr (PD == 2) {
    float xB[MBW][4], hB[NH][4], sB[NH][4];
    if (group_of(1) < ngroups) load_group(group_of(1), xB, hB, sB);
    for (int64_t it = 0;; it += 2) {
      if (group_of(it) >= ngroups) break;
      step(group_of(it), it, 0, xA, hA, sA);
      if (group_of(it + 1) >= ngroups) break;
      step(group_of(it + 1), it + 1, 1, xB, hB, sB);
    }
  } else {
    int par = 0;
    for (int64_t it = 0, g = group_of(0); g < ngroups; g = group_of(++it), par ^= 1) step(g, it, par, xA, hA, sA);
  }

  if (PH == 2) {
    float* dst = p.part + (int64_t)blockIdx.x * p.part_stride;
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = row0 + 16 * blk + 4 * b + i, c = 16 * h + a;
          if (row < m && c < r) dst[(int64_t)row * r + c] = accW[blk][h][i];
        }
    if (y == 0 && w == 0) {
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int q = 0; q < NH; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = 16 * h + 4 * b + i, cc = 16 * q + a;
            if (c < r && cc < r) dst[(int64_t)m * r + c * r + cc] = accG[h][q][i];
          }
    }
  }
  if (PH == 0) {
    res = wave_sum(res);
    if (lane == 0) sRes[w] = res;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int ww = 0; ww < NW; ++ww) s += sRes[ww];
      p.rpart[(int64_t)y * gridDim.x + blockIdx.x] = s;
    }
  }
}

// S[0][e] <- S[0][e] + S[1][e] + ... + S[n-1][e] (chunk order), e < r k.
__global__ __launch_bounds__(256) void k_sum_chunks(float* __restrict__ S, int64_t n_el, int nch) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_el) return;
  float s = S[e];
  for (int y = 1; y < nch; ++y) s += S[(int64_t)y * n_el + e];
  S[e] = s;
}

// ------------------------------------------------------------------ whole stage in one workgroup
// For small unfoldings (m <= 256, k <= 16 NG <= 64, r <= 16) one workgroup of four
// wavefronts runs `iters` MU iterations without leaving the kernel.  X stays in
// registers (wave w owns rows 64w..64w+63, in both MFMA operand layouts), H lives in
// LDS, W in registers.  Per iteration, for each 16-column group: W^T X by MFMA (rows
// split over waves, parts summed in LDS in wave order), (W^T W) H and the H epilogue,
// then X H_new^T for the wave's own rows and H_new H_new^T; after the last group the
// wave's rows of X H^T are complete, so the W-update
//   W <- max(0, W .* (X H^T) ./ (W (H H^T) + eps))
// is local to each wave (W (H H^T) by MFMA), followed by W^T W summed over the waves.
// All arithmetic is FP32 with FP32 accumulation; results are deterministic.
template <int NG>
__device__ __forceinline__ void stage_1wg_body(const StageArgs& s);

template <int NG>
__global__ __launch_bounds__(256) void k_stage_1wg(StageArgs s) {
  stage_1wg_body<NG>(s);
}

// grouped launch: workgroup i runs the stage described by list[i] (uneven shapes)
template <int NG>
__global__ __launch_bounds__(256) void k_stage_1wg_grouped(const StageArgs* __restrict__ list) {
  const StageArgs s = list[blockIdx.x];
  stage_1wg_body<NG>(s);
}

// grouped launch with the work-list passed by value (at most NTT_STAGE_LIST entries)
template <int NG>
__global__ __launch_bounds__(256) void k_stage_1wg_list(StageList L) {
  if ((int)blockIdx.x >= L.count) return;  // a graph node may be launched with an empty list
  const StageArgs s = L.a[blockIdx.x];
  stage_1wg_body<NG>(s);
}

template <int NG>
__device__ __forceinline__ void stage_1wg_body(const StageArgs& s) {
  constexpr int MBW = 4, SX = 20, KC = 16 * NG;
  __shared__ __attribute__((aligned(16))) float sX[4][16 * SX];
  __shared__ __attribute__((aligned(16))) float sNH[2][4][256];
  __shared__ __attribute__((aligned(16))) float sH[16][KC + 4];   // H, zero padded
  __shared__ __attribute__((aligned(16))) float sHn[4][16 * SX];  // per-wave H_new tile
  __shared__ __attribute__((aligned(16))) float sWr[4][16 * SX];  // per-wave W transpose tile
  __shared__ __attribute__((aligned(16))) float sG[4][256];       // Gram partials per wave
  __shared__ __attribute__((aligned(16))) float sGW[16][17];
  __shared__ __attribute__((aligned(16))) float sGH[16][17];

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = s.m, r = s.r, k = s.k;
  const int row0 = 64 * w;

  // X in both operand layouts: xa[g][blk][q] = X[row0+16blk+a][16g+4b+q] (A of X H^T),
  // xt[g][blk][kk] = X[row0+16blk+4b+kk][16g+a] (B of W^T X)
  float xa[NG][MBW][4], xt[NG][MBW][4];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i1 = row0 + 16 * blk + a, c1 = 16 * g + 4 * b + q;
        const float v1 = s.X[(int64_t)min(i1, m - 1) * k + min(c1, k - 1)];
        xa[g][blk][q] = zmask(v1, i1 < m && c1 < k);
        const int i2 = row0 + 16 * blk + 4 * b + q, c2 = 16 * g + a;
        const float v2 = s.X[(int64_t)min(i2, m - 1) * k + min(c2, k - 1)];
        xt[g][blk][q] = zmask(v2, i2 < m && c2 < k);
      }
  // W in the C layout of the 16x16 tiles: wc[blk][i] = W[row0+16blk+4b+i][a]
  float wc[MBW][4];
#pragma unroll
  for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = row0 + 16 * blk + 4 * b + i;
      const float v = s.W[(int64_t)min(row, m - 1) * r + min(a, r - 1)];
      wc[blk][i] = zmask(v, row < m && a < r);
    }
  for (int e = tid; e < 16 * (KC + 4); e += 256) {
    const int c = e / (KC + 4), j = e % (KC + 4);
    const float v = s.H[(int64_t)min(c, r - 1) * k + min(j, k - 1)];
    sH[c][j] = zmask(v, c < r && j < k);
  }

  // G_W = sum over waves of sum_rows W^T W (M = N = rank, K = row): both operands are wc
  auto gram_w = [&]() {
    v4f gp = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) gp = mfma16(wc[blk][kk], wc[blk][kk], gp);
#pragma unroll
    for (int i = 0; i < 4; ++i) sG[w][(4 * b + i) * 16 + a] = gp[i];
    __syncthreads();
    for (int e = tid; e < 256; e += 256) {
      sGW[e / 16][e % 16] = ((sG[0][e] + sG[1][e]) + sG[2][e]) + sG[3][e];
    }
    __syncthreads();
  };
  gram_w();

  for (int it = 0; it < s.iters; ++it) {
    // G_W as the A operand of (W^T W) H
    float gw[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) gw[kk] = sGW[a][4 * b + kk];
    v4f accW[MBW];
    v4f accG = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk) accW[blk] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int par = g & 1;
      float hv[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) hv[kk] = sH[4 * b + kk][16 * g + a];
      v4f nh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) nh = mfma16(wc[blk][kk], xt[g][blk][kk], nh);
#pragma unroll
      for (int i = 0; i < 4; ++i) sNH[par][w][(4 * b + i) * 16 + a] = nh[i];
      __syncthreads();  // every wave has also read its hv for this group
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = (4 * b + i) * 16 + a;
        nh[i] = ((sNH[par][0][e] + sNH[par][1][e]) + sNH[par][2][e]) + sNH[par][3][e];
      }
      v4f dh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) dh = mfma16(gw[kk], hv[kk], dh);
      float hn[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 4 * b + i;
        const float q = fmaxf(0.f, fast_div(hv[i] * nh[i], dh[i] + s.eps));
        hn[i] = (c < r && 16 * g + a < k) ? q : 0.f;
      }
      wave_sync();
#pragma unroll
      for (int i = 0; i < 4; ++i) sHn[w][(4 * b + i) * SX + a] = hn[i];
      if (w == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) sH[4 * b + i][16 * g + a] = hn[i];
      }
      wave_sync();
      const float4 hn4 = *reinterpret_cast<const float4*>(&sHn[w][a * SX + 4 * b]);
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk) {
        accW[blk] = mfma16(xa[g][blk][0], hn4.x, accW[blk]);
        accW[blk] = mfma16(xa[g][blk][1], hn4.y, accW[blk]);
        accW[blk] = mfma16(xa[g][blk][2], hn4.z, accW[blk]);
        accW[blk] = mfma16(xa[g][blk][3], hn4.w, accW[blk]);
      }
      accG = mfma16(hn4.x, hn4.x, accG);
      accG = mfma16(hn4.y, hn4.y, accG);
      accG = mfma16(hn4.z, hn4.z, accG);
      accG = mfma16(hn4.w, hn4.w, accG);
    }
    // G_H (every wave accumulated the same H_new, so any one copy is the full sum)
    if (w == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) sGH[4 * b + i][a] = accG[i];
    }
    // W rows of this wave in the A layout of W (H H^T): W[row0+16blk+a][4b+kk]
    wave_sync();
    float wr[MBW][4];
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk) {
#pragma unroll
      for (int i = 0; i < 4; ++i) sWr[w][(4 * b + i) * SX + a] = wc[blk][i];
      wave_sync();
      const float4 t4 = *reinterpret_cast<const float4*>(&sWr[w][a * SX + 4 * b]);
      wr[blk][0] = t4.x; wr[blk][1] = t4.y; wr[blk][2] = t4.z; wr[blk][3] = t4.w;
      wave_sync();
    }
    __syncthreads();
    float gh[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) gh[kk] = sGH[4 * b + kk][a];
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk) {
      v4f dw = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) dw = mfma16(wr[blk][kk], gh[kk], dw);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row0 + 16 * blk + 4 * b + i;
        const float q = fmaxf(0.f, fast_div(wc[blk][i] * accW[blk][i], dw[i] + s.eps));
        wc[blk][i] = (row < m && a < r) ? q : 0.f;
      }
    }
    gram_w();
  }

  // write W and H back
#pragma unroll
  for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = row0 + 16 * blk + 4 * b + i;
      if (row < m && a < r) s.W[(int64_t)row * r + a] = wc[blk][i];
    }
  for (int e = tid; e < 16 * KC; e += 256) {
    const int c = e / KC, j = e % KC;
    if (c < r && j < k) s.H[(int64_t)c * k + j] = sH[c][j];
  }
}

// ------------------------------------------------------------------ generic path (any m)
// H-update with one thread per column; W streamed through LDS in 64-row chunks.
template <int RP, bool UPDATE, bool RESID>
__global__ __launch_bounds__(256) void k_gen_hupdate(PassArgs p) {
  __shared__ float sW[64][RP + 1];
  __shared__ double sRes[4];
  const int tid = threadIdx.x;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;
  const int64_t j = (int64_t)blockIdx.x * 256 + tid;
  const bool act = j < k;
  float h[RP];
  const int64_t jc = act ? j : k - 1;
#pragma unroll
  for (int c = 0; c < RP; ++c) h[c] = zmask(p.H[(int64_t)min(c, r - 1) * k + jc], act && c < r);
  float acc[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) acc[c] = 0.f;
  double res = 0.0;
  for (int i0 = 0; i0 < m; i0 += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * RP; e += 256) {
      const int i = e / RP, c = e % RP;
      sW[i][c] = zmask(p.W[(int64_t)min(i0 + i, m - 1) * r + min(c, r - 1)], i0 + i < m && c < r);
    }
    __syncthreads();
    const int iend = min(64, m - i0);
#pragma unroll 8
    for (int i = 0; i < iend; ++i) {
      const float x = zmask(p.X[(int64_t)(i0 + i) * k + jc], act);
      if (UPDATE) {
#pragma unroll
        for (int c = 0; c < RP; ++c) acc[c] = fmaf(sW[i][c], x, acc[c]);
      }
      if (RESID) {
        float wh = 0.f;
#pragma unroll
        for (int c = 0; c < RP; ++c) wh = fmaf(sW[i][c], h[c], wh);
        const double dlt = (double)x - (double)wh;
        res += dlt * dlt;
      }
    }
  }
  if (UPDATE && act) {
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      if (c < r) {
        float dh = 0.f;
#pragma unroll
        for (int q = 0; q < RP; ++q) dh = fmaf(p.GW[c * RP + q], h[q], dh);
        p.H[(int64_t)c * k + j] = fmaxf(0.f, h[c] * acc[c] / (dh + p.eps));
      }
    }
  }
  if (RESID) {
    res = wave_sum(res);
    if ((tid & 63) == 0) sRes[tid >> 6] = res;
    __syncthreads();
    if (tid == 0) p.rpart[blockIdx.x] = ((sRes[0] + sRes[1]) + sRes[2]) + sRes[3];
  }
}

// X H^T and H H^T partials: block (g, rb) covers column chunk g and rows 64rb..64rb+63.
// Partial layout per chunk g: [m][r] then [r][r], compact (H H^T written by rb == 0).
template <int RP>
__global__ __launch_bounds__(256) void k_gen_xht(PassArgs p, int64_t chunk) {
  __shared__ float sX[64][65];
  __shared__ float sH[RP][65];
  const int tid = threadIdx.x;
  const int m = p.m, r = p.r;
  const int64_t k = p.k;
  const int g = blockIdx.x, rb = blockIdx.y;
  const int64_t c0 = (int64_t)g * chunk, c1 = min(k, c0 + chunk);
  const int row = tid >> 2, qd = tid & 3;
  float acc[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) acc[c] = 0.f;
  float accg[RP * RP / 256 > 0 ? RP * RP / 256 : 1];
  constexpr int NG = RP * RP / 256 > 0 ? RP * RP / 256 : 1;
#pragma unroll
  for (int t = 0; t < NG; ++t) accg[t] = 0.f;
  for (int64_t j0 = c0; j0 < c1; j0 += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
      const int i = e >> 6, jj = e & 63;
      const int gi = 64 * rb + i;
      const int64_t gj = j0 + jj;
      sX[i][jj] = zmask(p.X[(int64_t)min(gi, m - 1) * k + min(gj, c1 - 1)], gi < m && gj < c1);
    }
    for (int e = tid; e < RP * 64; e += 256) {
      const int c = e >> 6, jj = e & 63;
      const int64_t gj = j0 + jj;
      sH[c][jj] = zmask(p.H[(int64_t)min(c, r - 1) * k + min(gj, c1 - 1)], c < r && gj < c1);
    }
    __syncthreads();
#pragma unroll 1
    for (int jj = qd * 16; jj < qd * 16 + 16; ++jj) {
      const float x = sX[row][jj];
#pragma unroll
      for (int c = 0; c < RP; ++c) acc[c] = fmaf(x, sH[c][jj], acc[c]);
    }
    if (rb == 0) {
#pragma unroll
      for (int t = 0; t < NG; ++t) {
        const int pidx = tid + 256 * t;
        if (pidx < RP * RP) {
          const int c = pidx / RP, q = pidx % RP;
          float s = accg[t];
#pragma unroll 4
          for (int jj = 0; jj < 64; ++jj) s = fmaf(sH[c][jj], sH[q][jj], s);
          accg[t] = s;
        }
      }
    }
  }
  // combine the four column quarters of each row in order
  __syncthreads();
  float* red = &sX[0][0];  // 64 rows x 4 quarters x RP needs 256*RP floats <= 64*65 when RP<=16
  float* dst = p.part + (int64_t)g * p.part_stride;
  for (int c = 0; c < RP; ++c) {
    __syncthreads();
    red[tid] = acc[c];
    __syncthreads();
    if (qd == 0) {
      const int gi = 64 * rb + row;
      const float s = ((red[tid] + red[tid + 1]) + red[tid + 2]) + red[tid + 3];
      if (gi < m && c < r) dst[(int64_t)gi * r + c] = s;
    }
  }
  if (rb == 0) {
#pragma unroll
    for (int t = 0; t < NG; ++t) {
      const int pidx = tid + 256 * t;
      if (pidx < RP * RP && pidx / RP < r && pidx % RP < r)
        dst[(int64_t)m * r + (pidx / RP) * r + (pidx % RP)] = accg[t];
    }
  }
}

// ------------------------------------------------------------------ W-update
// Two launches after each pass with G > 4 partials, free of cross-block waits:
// (1) k_reduce_partials, grid ceil(E / 16): block eb sums entries [16 eb, 16 eb + 16)
//     of the E = m r + r r partial entries (X H^T then H H^T) over all G <= 1024
//     partials: 64 lanes per entry, lane l taking partials l, l + 64, ... (all loads
//     issued at once), then lanes in groups of eight and the groups in order, in FP64;
// (2) k_wupdate_t reads the sums and updates W.
// With G <= 4, k_wupdate_t sums the FP32 partials itself (g = 0..G-1 in order).
// The summation order is fixed, so results do not depend on scheduling.
constexpr int kReduceLanes = 64;
constexpr int kMaxReduceG = 16 * kReduceLanes;

// The same sums for G <= 64 with one thread per entry (consecutive threads, consecutive
// entries: every load is coalesced), NQ = ceil(G / 8) groups of eight partials, all loads
// issued at once: partial g goes into group g / 8 in order, the groups in order, each sum
// starting from 0.0 -- the operations and their order are those of k_reduce_partials for
// G <= 64 (there lane g holds partial g alone, and zeros for the missing ones), so the
// results are bitwise the same with far fewer threads.
template <int NQ>
__global__ __launch_bounds__(256) void k_reduce_partials_small(const float* __restrict__ part,
                                                               int64_t stride, int G, int64_t E,
                                                               double* __restrict__ red) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= E) return;
  float v[8 * NQ];
#pragma unroll
  for (int g = 0; g < 8 * NQ; ++g) v[g] = zmask(part[(int64_t)min(g, G - 1) * stride + e], g < G);
  double tot = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double sq = 0.0;
#pragma unroll
    for (int l = 0; l < 8; ++l) sq += (double)v[8 * q + l];
    tot += sq;
  }
  red[e] = tot;
}

__global__ __launch_bounds__(1024) void k_reduce_partials(const float* __restrict__ part,
                                                          int64_t stride, int G, int64_t E,
                                                          double* __restrict__ red) {
  __shared__ double sP[kReduceLanes][17];
  __shared__ double sQ[8][17];
  const int tid = threadIdx.x, el = tid & 15, lane = tid >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + el;
  float v[kMaxReduceG / kReduceLanes];
#pragma unroll
  for (int i = 0; i < kMaxReduceG / kReduceLanes; ++i) {
    const int g = lane + kReduceLanes * i;
    v[i] = zmask(part[(int64_t)min(g, G - 1) * stride + min(e, E - 1)], e < E && g < G);
  }
  double a = 0.0;
#pragma unroll
  for (int i = 0; i < kMaxReduceG / kReduceLanes; ++i) a += (double)v[i];
  sP[lane][el] = a;
  __syncthreads();
  if (tid < 128) {
    const int q = tid >> 4;
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < 8; ++l) s += sP[8 * q + l][el];
    sQ[q][el] = s;
  }
  __syncthreads();
  if (tid < 16 && (int64_t)blockIdx.x * 16 + tid < E) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += sQ[q][tid];
    red[(int64_t)blockIdx.x * 16 + tid] = s;
  }
}


// k_wupdate_t: W <- max(0, W .* N_W ./ (W G_H + eps)) with N_W = X H^T and G_H = H H^T,
//     over blocks of 256 rows (block j: rows [256 j, 256 j + 256)) of 1024 threads, one
//     thread per entry: thread t takes entries t, t + 1024, ... of the block's 256 x RB
//     (row, column) grid.  Rows are independent, so the update is in place; each thread
//     loads its entries, and the block its rows into LDS, before any is replaced.  FP64
//     arithmetic on FP32 data, rounded to FP32 (wupdate_entry).  The new rows go to LDS,
//     from where each of four wavefronts accumulates its 64 rows of the block's part of
//     G_W' = W'^T W' with FP64 MFMA (16 x 16 x 4 tiles; four rows per step, in row order);
//     the four wavefront sums are added in order, and the block parts in block order.
//     With one block (m <= 256) the block writes G_W and the Gram-identity monitor
//       f = 1/2 (||X||^2 - 2 <W', X H^T> + <W'^T W', H H^T>)
//     and, when this iteration accumulated one, the explicit residual objective.  With
//     several, each block stores its parts (G_W' and <W', N_W>) to gpart[j] with
//     device-scope stores, waits for them to complete and counts itself in at `arrive`
//     (a device-scope atomic add); the block that arrives last adds the parts, writes
//     G_W and the monitor, and sets the counter back to zero for the next launch.  No
//     block waits for another and no fence is needed: the parts are written and read past
//     the XCDs' non-coherent L2s.  RB >= r bounds the loops.  Entries are read from `red`
//     or, when FUSED (G <= 4), summed from the FP32 partials in order.
template <int RB, bool FUSED>
__global__ __launch_bounds__(1024) void k_wupdate_t(FinArgs f) {
  constexpr int NT = (RB + 15) / 16;  // 16 x 16 tiles per side of the Gram
  constexpr int EPT = RB / 4;         // entries per thread: 256 RB / 1024
  __shared__ double sGH[RB][RB + 1];
  __shared__ double sGW[RB][RB + 1];
  __shared__ float sW[256][RB + 1];
  __shared__ double sGp[4][NT * NT][64][4];
  __shared__ double sRed[16];
  __shared__ int sLast;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = f.m, r = f.r;
  const int64_t mr = (int64_t)m * r;
  const int i0 = blockIdx.x * 256;
  auto entry = [&](int64_t e) -> double {
    if (FUSED) {
      double v = 0.0;
#pragma unroll
      for (int g = 0; g < 4; ++g)
        v += (double)zmask(f.part[(int64_t)min(g, f.G - 1) * f.part_stride + e], g < f.G);
      return v;
    }
    return f.red[e];
  };
  // one round of loads: this thread's entries of W and N_W, and G_H
  float wv[EPT];
  double nv[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + 1024 * u, row = e / RB, c = e % RB;
    const int i = i0 + row;
    const int64_t idx = (int64_t)min(i, m - 1) * r + min(c, r - 1);
    const bool ok = i < m && c < r;
    wv[u] = zmask(f.W[idx], ok);
    nv[u] = zmask(entry(idx), ok);
  }
  if (tid < RB * RB) {
    const int c = tid / RB, q = tid % RB;
    sGH[c][q] = zmask(entry(mr + min(c, r - 1) * r + min(q, r - 1)), c < r && q < r);
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + 1024 * u;
    sW[e / RB][e % RB] = wv[u];
  }
  __syncthreads();
  float wn[EPT];
  double dot = 0.0;
  constexpr int kUnroll = RB == 32 ? 2 : EPT;  // RB = 32: bounded register use (1024 threads)
#pragma unroll kUnroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + 1024 * u, row = e / RB, c = e % RB;
    const float v = wupdate_entry<RB>(sW[row], nv[u], sGH, c, f.eps);
    wn[u] = (c < r && i0 + row < m) ? v : 0.f;
    dot += (double)wn[u] * nv[u];
  }
  __syncthreads();  // every row has been read before it is replaced
  float* wdst = f.Wout ? f.Wout : f.W;
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + 1024 * u, row = e / RB, c = e % RB;
    sW[row][c] = wn[u];
    if (c < r && i0 + row < m) wdst[(int64_t)(i0 + row) * r + c] = wn[u];
  }
  dot = wave_sum(dot);
  if (lane == 0) sRed[w] = dot;
  __syncthreads();
  if (w < 4) {  // wavefront w's 64 rows of the block's Gram
    v4d acc[NT][NT];
#pragma unroll
    for (int h = 0; h < NT; ++h)
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[h][q] = v4d{0.0, 0.0, 0.0, 0.0};
    gram_rows_f64<RB, NT, 256>(sW, acc, w, a, b);
#pragma unroll
    for (int h = 0; h < NT; ++h)
#pragma unroll
      for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) sGp[w][h * NT + q][lane][ii] = acc[h][q][ii];
  }
  __syncthreads();
  if (tid < NT * NT * 256) {
    const int tq = tid >> 8, l = (tid >> 2) & 63, ii = tid & 3;
    const double sg = ((sGp[0][tq][l][ii] + sGp[1][tq][l][ii]) + sGp[2][tq][l][ii]) + sGp[3][tq][l][ii];
    // FP64 16 x 16 x 4 result layout: value ii of lane (a, b) is row 4 ii + b, column a
    const int row = 16 * (tq / NT) + 4 * ii + (l >> 4), col = 16 * (tq % NT) + (l & 15);
    if (row < RB && col < RB) sGW[row][col] = sg;
  }
  double dot_wn = 0.0;  // thread 0: <W', N_W> of the block, wavefronts in order
  if (tid == 0) {
    dot_wn = sRed[0];
#pragma unroll
    for (int ww = 1; ww < 16; ++ww) dot_wn += sRed[ww];
  }
  __syncthreads();
  if (gridDim.x > 1) {
    constexpr int PS = 32 * 32 + 1;  // gpart stride per block: G_W' part, then <W', N_W>
    const int nb = gridDim.x;
    double* dst = f.gpart + (int64_t)blockIdx.x * PS;
    if (tid < RB * RB) st_dev(dst + tid, sGW[tid / RB][tid % RB]);
    if (tid == 0) st_dev(dst + RB * RB, dot_wn);
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed
    __syncthreads();
    if (tid == 0)
      sLast = __hip_atomic_fetch_add(f.arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
              (unsigned)(nb - 1);
    __syncthreads();
    if (!sLast) return;
    // the last block: entry e of every part added in block order (from 0.0), eight loads
    // in flight; entry RB RB is <W', N_W>
    for (int e = tid; e <= RB * RB; e += 1024) {
      double acc = 0.0;
      for (int j0 = 0; j0 < nb; j0 += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = ld_dev(f.gpart + (int64_t)min(j0 + u, nb - 1) * PS + e);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += zmask(x[u], j0 + u < nb);
      }
      if (e < RB * RB) sGW[e / RB][e % RB] = acc;
      else sRed[0] = acc;
    }
    if (tid == 0) __hip_atomic_store(f.arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (tid == 0) dot_wn = sRed[0];
  }
  // next G_W, zero padded to the pass kernels' RP x RP layout
  const int rp = r <= 16 ? 16 : 32;
  if (tid < rp * rp) {
    const int c = tid / rp, q = tid % rp;
    f.GW[tid] = (c < RB && q < RB && c < r && q < r) ? (float)sGW[c < RB ? c : 0][q < RB ? q : 0] : 0.f;
  }
  // monitor: <W'^T W', H H^T> over the first wavefront, residual partials over the second
  double gg = 0.0, rsum = 0.0;
  if (w == 0) {
    for (int pidx = lane; pidx < r * r; pidx += 64) gg += sGW[pidx / r][pidx % r] * sGH[pidx / r][pidx % r];
    gg = wave_sum(gg);
    if (lane == 0) sRed[1] = gg;
  } else if (w == 1 && f.rpart) {
    for (int g = lane; g < f.G; g += 64) rsum += f.rpart[g];
    rsum = wave_sum(rsum);
    if (lane == 0) sRed[2] = rsum;
  }
  __syncthreads();
  if (tid == 0) {
    f.scal[SCAL_MONITOR] = 0.5 * (f.scal[SCAL_NX2] - 2.0 * dot_wn + sRed[1]);
    if (f.rpart) {
      const double obj = 0.5 * sRed[2];
      f.scal[SCAL_OBJ] = obj;
      if (f.trace) f.trace[0] = obj;
    }
  }
}

__global__ void k_zero_ints(int* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// BF16 shadow of X: round to nearest, ties to even (NaN stays NaN).
__global__ void k_cast_bf16(uint16_t* __restrict__ dst, const float* __restrict__ src, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const uint32_t u = __float_as_uint(src[i]);
    uint16_t o;
    if ((u & 0x7fffffffu) > 0x7f800000u) o = (uint16_t)((u >> 16) | 0x40u);
    else o = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    dst[i] = o;
  }
}

// Coalesced transpose: dst (cols x rows) = src (rows x cols)^T, both row-major, through
// 32 x 33 LDS tiles (the padding keeps the column reads free of bank conflicts).  One
// workgroup per tile, tiles numbered row-major over a 1-D grid.
__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ src, float* __restrict__ dst,
                                                   int64_t rows, int64_t cols, int64_t tiles_c) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  const int64_t t = blockIdx.x;
  const int64_t c0 = (t % tiles_c) * 32, r0 = (t / tiles_c) * 32;
  for (int i = ty; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < rows && c < cols) tile[i][tx] = src[r * cols + c];
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + tx;  // dst row c, column r
    if (c < cols && r < rows) dst[c * rows + r] = tile[tx][i];
  }
}

// copy helper: dst[i] = src[i]
__global__ void k_copy(float* __restrict__ dst, const float* __restrict__ src, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

// ------------------------------------------------------------------ Gram for the rank rule
// FP64 Gram of the shorter side of X (Alg.2 rank rule: the squared singular values of X
// are the eigenvalues of X X^T or X^T X).  Workgroup (pair, split) forms the 64 x 64
// block (bi, bj), bi <= bj, of the Gram over one chunk of the long dimension: tiles of
// 64 short-side indices x 16 long-side indices of both blocks are staged in LDS as FP32
// (exact in FP64) and multiplied with v_mfma_f64_16x16x4f64, each wave owning a 32 x 32
// quarter.  The partial goes to part[pair][split]; k_gram_reduce adds the splits in
// order and writes both triangles.
struct GramArgs {
  const float* X;
  int64_t m, k;     // X is m x k, row-major
  int n;            // Gram side: min(m, k)
  int trans;        // 0: G = X X^T (n = m); 1: G = X^T X (n = k)
  int nb;           // 64-blocks per side
  int nsplit;
  int64_t chunk;    // long-side indices per split (multiple of 16)
  double* part;
  double* G;
};

__device__ __forceinline__ void gram_pair(int p, int nb, int* bi, int* bj) {
  int i = 0;
  while (p >= nb - i) {  // row i of the upper triangle holds nb - i blocks
    p -= nb - i;
    ++i;
  }
  *bi = i;
  *bj = i + p;
}

__global__ __launch_bounds__(256) void k_gram(GramArgs g) {
  __shared__ float sA[64][17];
  __shared__ float sB[64][17];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  int bi, bj;
  gram_pair(blockIdx.x, g.nb, &bi, &bj);
  const int split = blockIdx.y;
  const int64_t L = g.trans ? g.m : g.k;  // long side
  const int64_t c_begin = (int64_t)split * g.chunk;
  const int64_t c_end = min(L, c_begin + g.chunk);
  const int n = g.n;
  v4d acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  for (int64_t c0 = c_begin; c0 < c_end; c0 += 16) {
    // element (p, c) of the short x long view: X[p][c] (trans 0) or X[c][p] (trans 1);
    // entries past n or past the chunk are zero
    for (int e = tid; e < 2 * 64 * 16; e += 256) {
      const int which = e >> 10, q = e & 1023;
      int pl, cl;
      if (g.trans) {  // consecutive threads along p: rows of X are contiguous in p
        cl = q >> 6;
        pl = q & 63;
      } else {        // consecutive threads along c
        pl = q >> 4;
        cl = q & 15;
      }
      const int pg = (which ? bj : bi) * 64 + pl;
      const int64_t cg = c0 + cl;
      const int pc = min(pg, n - 1);
      const int64_t cc = min(cg, c_end - 1);
      const float v = g.trans ? g.X[cc * g.k + pc] : g.X[(int64_t)pc * g.k + cc];
      const float z = zmask(v, pg < n && cg < c_end);
      if (which) sB[pl][cl] = z;
      else sA[pl][cl] = z;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) {
        const double av = (double)sA[wi + 16 * ti + a][4 * kk + b];
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          const double bv = (double)sB[wj + 16 * tj + a][4 * kk + b];
          acc[ti][tj] = mfma16_f64(av, bv, acc[ti][tj]);
        }
      }
    __syncthreads();
  }
  // FP64 16 x 16 x 4 result layout: value i of lane (a, b) is row 4 i + b, column a
  double* dst = g.part + ((size_t)blockIdx.x * g.nsplit + split) * 4096;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[(wi + 16 * ti + 4 * i + b) * 64 + wj + 16 * tj + a] = acc[ti][tj][i];
}

__global__ __launch_bounds__(256) void k_gram_reduce(GramArgs g) {
  int bi, bj;
  gram_pair(blockIdx.x, g.nb, &bi, &bj);
  const double* src = g.part + (size_t)blockIdx.x * g.nsplit * 4096;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    double s = 0.0;
    for (int sp = 0; sp < g.nsplit; ++sp) s += src[(size_t)sp * 4096 + e];
    const int gi = bi * 64 + (e >> 6), gj = bj * 64 + (e & 63);
    if (gi < g.n && gj < g.n) {
      g.G[(size_t)gi * g.n + gj] = s;
      g.G[(size_t)gj * g.n + gi] = s;
    }
  }
}

// ------------------------------------------------------------------ TT expand (Eq.(2))
// Rows of the (n_1...n_{d-1}) x n_d matrix of the full tensor, ROWS per block (blockIdx.x),
// columns split into gridDim.y ranges (blockIdx.y) when there are few row blocks.  Each
// row's left factor P[row,:] = G_1[i_1,:] G_2[:,i_2,:] ... G_{d-1}[:,i_{d-1},:] is formed
// in LDS (FP32, zero beyond the rank), then Ahat[row, col] = P[row,:] . G_d[:, col]
// (ranks in order, RLP >= r_{d-1} terms, the padding adding exact zeros): each thread
// takes CPT adjacent columns at a time, holds their G_d columns in registers and runs down
// a share of the block's rows.  MODE 0 writes Ahat; MODE 1 accumulates sum (A - Ahat)^2
// and sum A^2 in FP64 (thread order, a fixed butterfly, the waves in order) into
// part[2 b], part[2 b + 1] with b = blockIdx.x + gridDim.x blockIdx.y.
template <int MODE, int ROWS, int RLP, int CPT>
__global__ __launch_bounds__(256) void k_tt_expand(TTArgs t) {
  constexpr int PW = NTT_MAX_RANK + 1;
  __shared__ float sP[2][ROWS][PW];
  __shared__ int sIdx[ROWS][NTT_MAX_DIMS];
  __shared__ double sRed[2][4];
  const int tid = threadIdx.x;
  const int d = t.d;
  const int64_t rows = t.rows;
  const int64_t r0 = (int64_t)blockIdx.x * ROWS;
  const int nrow = (int)min((int64_t)ROWS, rows - r0);
  for (int rr = tid; rr < nrow; rr += 256) {
    int64_t rem = r0 + rr;
    for (int kx = d - 2; kx >= 0; --kx) {
      sIdx[rr][kx] = (int)(rem % t.dims[kx]);
      rem /= t.dims[kx];
    }
  }
  for (int e = tid; e < 2 * ROWS * PW; e += 256) (&sP[0][0][0])[e] = 0.f;
  __syncthreads();
  // P_1 = G_1[i_1, :]
  int cur = 0;
  {
    const int rk = t.ranks[1];
    for (int e = tid; e < ROWS * rk; e += 256) {
      const int rr = e / rk, c = e % rk;
      sP[0][rr][c] = zmask(t.cores[0][(int64_t)sIdx[min(rr, nrow - 1)][0] * rk + c], rr < nrow);
    }
  }
  __syncthreads();
  for (int kx = 1; kx < d - 1; ++kx) {
    const int ra = t.ranks[kx], rb = t.ranks[kx + 1];
    const int64_t nk = t.dims[kx];
    const float* G = t.cores[kx];
    for (int e = tid; e < ROWS * rb; e += 256) {
      const int rr = e / rb, c = e % rb;
      float s = 0.f;
      if (rr < nrow) {
        const int64_t base = (int64_t)sIdx[rr][kx] * rb + c;
        for (int q = 0; q < ra; ++q) s = fmaf(sP[cur][rr][q], G[(int64_t)q * nk * rb + base], s);
      }
      sP[cur ^ 1][rr][c] = s;
    }
    cur ^= 1;
    __syncthreads();
  }
  // last contraction, fused with the output or the error sums
  const int rl = t.ranks[d - 1];
  const int64_t nd = t.dims[d - 1];
  const float* Gd = t.cores[d - 1];
  const int64_t span = ((nd + gridDim.y - 1) / gridDim.y + CPT - 1) / CPT * CPT;
  const int64_t c0 = (int64_t)blockIdx.y * span, c1 = min(nd, c0 + span);
  // W threads across the range's CPT-column groups (rounded up to a power of two, at most
  // 256) times 256 / W across rows
  const int64_t ngrp = c1 > c0 ? (c1 - c0 + CPT - 1) / CPT : 0;
  int W = 256;
  while (W > 1 && W / 2 >= ngrp) W >>= 1;
  const int lanes = 256 / W;
  double s_err = 0.0, s_ref = 0.0;
  for (int64_t gi = tid % W; gi < ngrp; gi += W) {
    const int64_t col = c0 + CPT * gi;
    float g[CPT][RLP];
#pragma unroll
    for (int u = 0; u < CPT; ++u)
#pragma unroll
      for (int q = 0; q < RLP; ++q)
        g[u][q] = zmask(Gd[(int64_t)min(q, rl - 1) * nd + min(col + u, c1 - 1)], q < rl);
    for (int rr = tid / W; rr < nrow; rr += lanes) {
      float sv[CPT];
#pragma unroll
      for (int u = 0; u < CPT; ++u) sv[u] = 0.f;
#pragma unroll
      for (int q = 0; q < RLP; ++q) {
        const float pq = sP[cur][rr][q];
#pragma unroll
        for (int u = 0; u < CPT; ++u) sv[u] = fmaf(pq, g[u][q], sv[u]);
      }
      const int64_t at = (r0 + rr) * nd + col;
      if (CPT == 4 && col + 4 <= c1) {
        if (MODE == 0) {
          *reinterpret_cast<float4*>(t.out + at) = make_float4(sv[0], sv[1], sv[2], sv[3]);
        } else {
          const float4 a4 = *reinterpret_cast<const float4*>(t.A + at);
          const float av[4] = {a4.x, a4.y, a4.z, a4.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double dv = (double)av[u] - (double)sv[u];
            s_err += dv * dv;
            s_ref += (double)av[u] * (double)av[u];
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
          if (col + u < c1) {
            if (MODE == 0) {
              t.out[at + u] = sv[u];
            } else {
              const double av = (double)t.A[at + u];
              const double dv = av - (double)sv[u];
              s_err += dv * dv;
              s_ref += av * av;
            }
          }
        }
      }
    }
  }
  if (MODE == 1) {
    s_err = wave_sum(s_err);
    s_ref = wave_sum(s_ref);
    if ((tid & 63) == 0) {
      sRed[0][tid >> 6] = s_err;
      sRed[1][tid >> 6] = s_ref;
    }
    __syncthreads();
    if (tid == 0) {
      const int64_t b = (int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
      t.part[2 * b] = ((sRed[0][0] + sRed[0][1]) + sRed[0][2]) + sRed[0][3];
      t.part[2 * b + 1] = ((sRed[1][0] + sRed[1][1]) + sRed[1][2]) + sRed[1][3];
    }
  }
}

__global__ __launch_bounds__(64) void k_sum_pairs(const double* __restrict__ part, int64_t n,
                                                  double* __restrict__ out) {
  double a = 0.0, c = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 64) {
    a += part[2 * i];
    c += part[2 * i + 1];
  }
  a = wave_sum(a);
  c = wave_sum(c);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = c;
  }
}

// ------------------------------------------------------------------ host launchers
#define NTT_CHECK_LAUNCH()                          \
  do {                                              \
    hipError_t e_ = hipGetLastError();              \
    if (e_ != hipSuccess) return e_;                \
  } while (0)

hipError_t launch_init_uniform(float* out, int64_t n, uint64_t seed, uint64_t tag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  k_init_uniform<<<(int)blocks, 256, 0, s>>>(out, n, seed, tag);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_cast_bf16(uint16_t* dst, const float* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  k_cast_bf16<<<(int)blocks, 256, 0, s>>>(dst, src, n);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_transpose(const float* src, float* dst, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t tc = (cols + 31) / 32, tr = (rows + 31) / 32;
  if (tc * tr > 0x7fffffffLL) return hipErrorInvalidValue;
  k_transpose<<<(unsigned)(tc * tr), 256, 0, s>>>(src, dst, rows, cols, tc);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_copy(float* dst, const float* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  k_copy<<<(int)blocks, 256, 0, s>>>(dst, src, n);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_sumsq(const float* x, int64_t n, double* part, int nblocks, int* flags,
                        int validate, double* out, hipStream_t s) {
  k_sumsq<<<nblocks, 256, 0, s>>>(x, n, part, flags, validate);
  NTT_CHECK_LAUNCH();
  k_sum_doubles<<<1, 64, 0, s>>>(part, nblocks, 1.0, out, nullptr);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_gram_w(const float* W, int m, int r, int rp, float* G, hipStream_t s) {
  if (rp == 16) k_gram_w<16><<<1, 256, 0, s>>>(W, m, r, G);
  else k_gram_w<32><<<1, 256, 0, s>>>(W, m, r, G);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

template <int RP, int MB>
static hipError_t pass_fused_mb(const PassArgs& a, int grid, bool update, bool resid, hipStream_t s) {
  if (a.Xb != nullptr) {
    if constexpr (RP == 16) {
      if (!update || resid) return hipErrorInvalidValue;  // BF16 X: update passes only
      k_mu_pass<RP, MB, true, false, true><<<grid, 256, 0, s>>>(a);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (update && resid) k_mu_pass<RP, MB, true, true><<<grid, 256, 0, s>>>(a);
  else if (update) k_mu_pass<RP, MB, true, false><<<grid, 256, 0, s>>>(a);
  else k_mu_pass<RP, MB, false, true><<<grid, 256, 0, s>>>(a);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

template <int RP>
static hipError_t pass_fused_rp(const PassArgs& a, int mb, int grid, bool update, bool resid,
                                hipStream_t s) {
  switch (mb) {
    case 1: return pass_fused_mb<RP, 1>(a, grid, update, resid, s);
    case 2: return pass_fused_mb<RP, 2>(a, grid, update, resid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pass_tiny(const PassArgs& a, int grid, hipStream_t s) {
  if (a.m < 1 || a.m > 4 || a.r < 1 || a.r > a.m || a.Wprev != nullptr || grid < 1) return hipErrorInvalidValue;
  const bool xb = a.Xb != nullptr;
  if (a.m <= 2) {
    if (xb) k_mu_pass_tiny<2, 4, true><<<grid, 256, 0, s>>>(a);
    else k_mu_pass_tiny<2, 4, false><<<grid, 256, 0, s>>>(a);
  } else {
    if (xb) k_mu_pass_tiny<4, 4, true><<<grid, 256, 0, s>>>(a);
    else k_mu_pass_tiny<4, 4, false><<<grid, 256, 0, s>>>(a);
  }
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_pass_fused(const PassArgs& a, int rp, int mb, int grid, bool update, bool resid,
                             bool wide, hipStream_t s) {
  if (rp == 16 && a.r <= 8 && mb <= 2 && update && !resid) {
    const bool xb = a.Xb != nullptr;
    if (wide) {
      // FP32 X: the 4 x 4-block pass; the BF16 copy: the 16 x 16-tile pass
      // (the 4 x 4-block pass addresses X and H by 32-bit byte offsets)
      const bool small = 4.0 * (double)std::max(a.m, 8) * (double)a.k < 4294967296.0;
      if (mb == 1) {
        if (xb || !small) { if (xb) k_mu_pass_r8w<4, true><<<grid, 256, 0, s>>>(a);
                            else k_mu_pass_r8w<4, false><<<grid, 256, 0, s>>>(a); }
        else k_mu_pass_r8m<16><<<grid, 256, 0, s>>>(a);
      } else {
        if (xb || !small) { if (xb) k_mu_pass_r8w<8, true><<<grid, 256, 0, s>>>(a);
                            else k_mu_pass_r8w<8, false><<<grid, 256, 0, s>>>(a); }
        else k_mu_pass_r8m<32><<<grid, 256, 0, s>>>(a);
      }
      NTT_CHECK_LAUNCH();
      return hipSuccess;
    }
    switch (mb) {
      case 1:
        if (xb) k_mu_pass_r8<1, true><<<grid, 256, 0, s>>>(a);
        else k_mu_pass_r8<1, false><<<grid, 256, 0, s>>>(a);
        break;
      case 2:
        if (xb) k_mu_pass_r8<2, true><<<grid, 256, 0, s>>>(a);
        else k_mu_pass_r8<2, false><<<grid, 256, 0, s>>>(a);
        break;
      default: return hipErrorInvalidValue;
    }
    NTT_CHECK_LAUNCH();
    return hipSuccess;
  }
  if (a.Wprev != nullptr) return hipErrorInvalidValue;  // W-update prologue: r <= 8 pass only
  if (rp == 16) return pass_fused_rp<16>(a, mb, grid, update, resid, s);
  if (a.Xb != nullptr) return hipErrorInvalidValue;  // BF16 X: rank padding 16 only
  return pass_fused_rp<32>(a, mb, grid, update, resid, s);
}

template <int RP, int MBW, int NW>
static hipError_t pass_L3(const PassArgs& a, int grid, bool update, bool resid, hipStream_t s) {
  if (a.Xb != nullptr) {
    if (!update || resid) return hipErrorInvalidValue;  // BF16 X: update passes only
    k_mu_pass_L<RP, MBW, NW, true, false, true><<<grid, 64 * NW, 0, s>>>(a);
  } else if (update && resid) {
    k_mu_pass_L<RP, MBW, NW, true, true, false><<<grid, 64 * NW, 0, s>>>(a);
  } else if (update) {
    k_mu_pass_L<RP, MBW, NW, true, false, false><<<grid, 64 * NW, 0, s>>>(a);
  } else {
    k_mu_pass_L<RP, MBW, NW, false, true, false><<<grid, 64 * NW, 0, s>>>(a);
  }
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

template <int RP>
static hipError_t pass_L_rp(const PassArgs& a, int cls, int grid, bool update, bool resid, hipStream_t s) {
  switch (cls) {
    case 0: return pass_L3<RP, 1, 4>(a, grid, update, resid, s);   // m <= 64
    case 1: return pass_L3<RP, 2, 4>(a, grid, update, resid, s);   // m <= 128
    case 2: return pass_L3<RP, 4, 4>(a, grid, update, resid, s);   // m <= 256
    case 3: return pass_L3<RP, 4, 8>(a, grid, update, resid, s);   // m <= 512
    case 4:  // m <= 1024 (RP = 16 only: the RP = 32 instance would spill)
      if (RP == 16) return pass_L3<16, 8, 8>(a, grid, update, resid, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int MBW, int NW, bool NT>
static void pass_LW_nt(const PassArgs& a, int grid, hipStream_t s) {
  // BF16 X: BF16 matrix cores for waves of 32 rows (wider waves would spill registers)
  if (a.Xb != nullptr) {
    if constexpr (MBW == 2) k_mu_pass_LWB<MBW, NW, NT><<<grid, 64 * NW, 0, s>>>(a);
    else k_mu_pass_LW<MBW, NW, true, NT><<<grid, 64 * NW, 0, s>>>(a);
  } else {
    k_mu_pass_LW<MBW, NW, false, NT><<<grid, 64 * NW, 0, s>>>(a);
  }
}

template <int MBW, int NW>
static hipError_t pass_LW(const PassArgs& a, int grid, hipStream_t s) {
  // An X of more bytes than the last-level cache (256 MB) is read with non-temporal loads:
  // it cannot stay cached from one pass to the next, and streaming it past the cache keeps
  // H there (measured on the 128 x 2,097,152 pass: 4-5% faster; slower where X fits)
  const bool nt = (double)a.m * (double)a.k * (a.Xb != nullptr ? 2.0 : 4.0) > 268435456.0;
  if (nt) pass_LW_nt<MBW, NW, true>(a, grid, s);
  else pass_LW_nt<MBW, NW, false>(a, grid, s);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_pass_L(const PassArgs& a, int rp, int cls, int grid, bool update, bool resid,
                         bool wide, hipStream_t s) {
  if (wide && pass_L_batch(cls, rp) == 0) return hipErrorInvalidValue;
  if (a.Wprev != nullptr) return hipErrorInvalidValue;  // W-update prologue: r <= 8 pass only
  if (update && wide) {
    // the residual of the incoming (W, H) first, by the per-group pass, then the update
    if (resid) {
      const hipError_t e = pass_L_rp<16>(a, cls, grid, false, true, s);
      if (e != hipSuccess) return e;
    }
    switch (cls) {
      case 0: return pass_LW<1, 4>(a, grid, s);
      case 1: return pass_LW<2, 4>(a, grid, s);
      case 2: return pass_LW<4, 4>(a, grid, s);
      case 3: return pass_LW<4, 8>(a, grid, s);
      default: return hipErrorInvalidValue;
    }
  }
  return rp == 16 ? pass_L_rp<16>(a, cls, grid, update, resid, s)
                  : pass_L_rp<32>(a, cls, grid, update, resid, s);
}

constexpr int kNumCUs = 256;  // MI355X: 8 XCDs of 32 CUs

template <int RP>
static hipError_t pass_C_rp(const PassArgs& a, int G, bool update, bool resid, hipStream_t s) {
  dim3 grid((unsigned)G, (unsigned)a.nchunks);
  if (resid) {
    k_mu_pass_C<RP, 4, 8, 0, false><<<grid, 512, 0, s>>>(a);
    NTT_CHECK_LAUNCH();
  }
  if (update) {
    const int64_t n_el = (int64_t)a.r * a.k;
    // at most one workgroup per CU (8 waves): two groups in flight per wave, which the
    // registers allow at rank 16 (at three waves per SIMD, too many for two workgroups)
    constexpr int PD = RP == 16 ? 2 : 1;
    const bool deep = PD == 2 && (int64_t)G * a.nchunks <= kNumCUs;
    if (a.Xb != nullptr) {
      if (deep) k_mu_pass_C<RP, 4, 8, 1, true, PD><<<grid, 512, 0, s>>>(a);
      else k_mu_pass_C<RP, 4, 8, 1, true><<<grid, 512, 0, s>>>(a);
    } else {
      if (deep) k_mu_pass_C<RP, 4, 8, 1, false, PD><<<grid, 512, 0, s>>>(a);
      else k_mu_pass_C<RP, 4, 8, 1, false><<<grid, 512, 0, s>>>(a);
    }
    NTT_CHECK_LAUNCH();
    k_sum_chunks<<<(unsigned)((n_el + 255) / 256), 256, 0, s>>>(a.S, n_el, a.nchunks);
    NTT_CHECK_LAUNCH();
    if (a.Xb != nullptr) {
      if (deep) k_mu_pass_C<RP, 4, 8, 2, true, PD><<<grid, 512, 0, s>>>(a);
      else k_mu_pass_C<RP, 4, 8, 2, true><<<grid, 512, 0, s>>>(a);
    } else {
      if (deep) k_mu_pass_C<RP, 4, 8, 2, false, PD><<<grid, 512, 0, s>>>(a);
      else k_mu_pass_C<RP, 4, 8, 2, false><<<grid, 512, 0, s>>>(a);
    }
    NTT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

hipError_t launch_pass_C(const PassArgs& a, int rp, int G, bool update, bool resid, hipStream_t s) {
  if (a.nchunks < 1 || a.nchunks > 65535 || !a.S || !a.Hs ||
      (int64_t)a.nchunks * pass_C_rows(rp) < a.m || G < 1)
    return hipErrorInvalidValue;
  if (a.Xb != nullptr && resid) return hipErrorInvalidValue;  // BF16 X: update passes only
  return rp == 16 ? pass_C_rp<16>(a, G, update, resid, s) : pass_C_rp<32>(a, G, update, resid, s);
}

hipError_t launch_stage_1wg(const StageArgs& a, hipStream_t s) {
  if (!stage_1wg_ok(a.m, a.k, a.r) || a.iters <= 0) return hipErrorInvalidValue;
  const int ng = stage_1wg_ng(a.k);
  if (ng == 1) k_stage_1wg<1><<<1, 256, 0, s>>>(a);
  else if (ng == 2) k_stage_1wg<2><<<1, 256, 0, s>>>(a);
  else k_stage_1wg<4><<<1, 256, 0, s>>>(a);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_stage_1wg_grouped(const StageArgs* list_dev, int count, int ng, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (ng == 1) k_stage_1wg_grouped<1><<<count, 256, 0, s>>>(list_dev);
  else if (ng == 2) k_stage_1wg_grouped<2><<<count, 256, 0, s>>>(list_dev);
  else if (ng == 4) k_stage_1wg_grouped<4><<<count, 256, 0, s>>>(list_dev);
  else return hipErrorInvalidValue;
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_stage_1wg_list(const StageList& L, int ng, hipStream_t s) {
  if (L.count <= 0) return hipSuccess;
  if (L.count > NTT_STAGE_LIST) return hipErrorInvalidValue;
  if (ng == 1) k_stage_1wg_list<1><<<L.count, 256, 0, s>>>(L);
  else if (ng == 2) k_stage_1wg_list<2><<<L.count, 256, 0, s>>>(L);
  else if (ng == 4) k_stage_1wg_list<4><<<L.count, 256, 0, s>>>(L);
  else return hipErrorInvalidValue;
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

const void* stage_1wg_list_kernel(int ng) {
  if (ng == 1) return reinterpret_cast<const void*>(k_stage_1wg_list<1>);
  if (ng == 2) return reinterpret_cast<const void*>(k_stage_1wg_list<2>);
  if (ng == 4) return reinterpret_cast<const void*>(k_stage_1wg_list<4>);
  return nullptr;
}

hipError_t launch_pass_generic(const PassArgs& a, int rp, int gxht, int64_t chunk, bool update,
                               bool resid, hipStream_t s) {
  const int gh = (int)((a.k + 255) / 256);
  if (rp == 16) {
    if (update && resid) k_gen_hupdate<16, true, true><<<gh, 256, 0, s>>>(a);
    else if (update) k_gen_hupdate<16, true, false><<<gh, 256, 0, s>>>(a);
    else k_gen_hupdate<16, false, true><<<gh, 256, 0, s>>>(a);
  } else {
    if (update && resid) k_gen_hupdate<32, true, true><<<gh, 256, 0, s>>>(a);
    else if (update) k_gen_hupdate<32, true, false><<<gh, 256, 0, s>>>(a);
    else k_gen_hupdate<32, false, true><<<gh, 256, 0, s>>>(a);
  }
  NTT_CHECK_LAUNCH();
  if (update) return launch_xht_partials(a, rp, gxht, chunk, s);
  return hipSuccess;
}

hipError_t launch_xht_partials(const PassArgs& a, int rp, int gxht, int64_t chunk, hipStream_t s) {
  dim3 grid(gxht, (a.m + 63) / 64);
  if (rp == 16) k_gen_xht<16><<<grid, 256, 0, s>>>(a, chunk);
  else k_gen_xht<32><<<grid, 256, 0, s>>>(a, chunk);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

template <int RB>
static hipError_t launch_wupdate(const FinArgs& f, bool fused, hipStream_t s) {
  const int nb = (f.m + 255) / 256;
  if (f.m < 1 || (nb > 1 && (!f.gpart || !f.arrive))) return hipErrorInvalidValue;
  if (fused) k_wupdate_t<RB, true><<<nb, 1024, 0, s>>>(f);
  else k_wupdate_t<RB, false><<<nb, 1024, 0, s>>>(f);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_finalize(const FinArgs& f, int rp, hipStream_t s) {
  (void)rp;
  const bool fused = f.G <= 4;  // the W-update sums the partials itself
  if (!fused) {
    if (f.G > kMaxReduceG) return hipErrorInvalidValue;
    const hipError_t e = launch_reduce(f, s);
    if (e != hipSuccess) return e;
  }
  if (f.r <= 8) return launch_wupdate<8>(f, fused, s);
  if (f.r <= 16) return launch_wupdate<16>(f, fused, s);
  return launch_wupdate<32>(f, fused, s);
}

hipError_t launch_wupdate_red(const FinArgs& f, hipStream_t s) {
  if (f.r <= 8) return launch_wupdate<8>(f, false, s);
  if (f.r <= 16) return launch_wupdate<16>(f, false, s);
  return launch_wupdate<32>(f, false, s);
}

hipError_t launch_reduce(const FinArgs& f, hipStream_t s) {
  if (f.G < 1 || f.G > kMaxReduceG) return hipErrorInvalidValue;
  const int64_t E = (int64_t)f.m * f.r + (int64_t)f.r * f.r;
  const unsigned gs = (unsigned)((E + 255) / 256);
  switch ((f.G + 7) / 8) {
    case 1: k_reduce_partials_small<1><<<gs, 256, 0, s>>>(f.part, f.part_stride, f.G, E, f.red); break;
    case 2: k_reduce_partials_small<2><<<gs, 256, 0, s>>>(f.part, f.part_stride, f.G, E, f.red); break;
    case 3: k_reduce_partials_small<3><<<gs, 256, 0, s>>>(f.part, f.part_stride, f.G, E, f.red); break;
    case 4: k_reduce_partials_small<4><<<gs, 256, 0, s>>>(f.part, f.part_stride, f.G, E, f.red); break;
    case 5: k_reduce_partials_small<5><<<gs, 256, 0, s>>>(f.part, f.part_stride, f.G, E, f.red); break;
    case 6: k_reduce_partials_small<6><<<gs, 256, 0, s>>>(f.part, f.part_stride, f.G, E, f.red); break;
    case 7: k_reduce_partials_small<7><<<gs, 256, 0, s>>>(f.part, f.part_stride, f.G, E, f.red); break;
    case 8: k_reduce_partials_small<8><<<gs, 256, 0, s>>>(f.part, f.part_stride, f.G, E, f.red); break;
    default:
      k_reduce_partials<<<(unsigned)((E + 15) / 16), 1024, 0, s>>>(f.part, f.part_stride, f.G, E, f.red);
  }
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

// acc = src (first) or acc + src, elementwise, FP64: the column blocks of a streamed
// stage add their reduced products in block order.
__global__ void k_add_doubles(double* __restrict__ acc, const double* __restrict__ src, int64_t n,
                              int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) acc[i] = first ? src[i] : acc[i] + src[i];
}

hipError_t launch_add_doubles(double* acc, const double* src, int64_t n, int first, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_add_doubles<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(acc, src, n, first);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_sum_doubles(const double* part, int n, double scale, double* out, hipStream_t s) {
  k_sum_doubles<<<1, 64, 0, s>>>(part, n, scale, out, nullptr);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_zero_ints(int* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_zero_ints<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_resid_sum(const double* rpart, int G, double* obj, double* trace, hipStream_t s) {
  k_sum_doubles<<<1, 64, 0, s>>>(rpart, G, 0.5, obj, trace);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

template <int MODE, int ROWS, int RLP>
static void tt_launch(const TTArgs& t, dim3 grid, bool vec4, hipStream_t s) {
  if (vec4) k_tt_expand<MODE, ROWS, RLP, 4><<<grid, 256, 0, s>>>(t);
  else k_tt_expand<MODE, ROWS, RLP, 1><<<grid, 256, 0, s>>>(t);
}

template <int MODE, int ROWS>
static void tt_launch_rl(const TTArgs& t, int rl, dim3 grid, bool vec4, hipStream_t s) {
  if (rl <= 8) tt_launch<MODE, ROWS, 8>(t, grid, vec4, s);
  else if (rl <= 16) tt_launch<MODE, ROWS, 16>(t, grid, vec4, s);
  else tt_launch<MODE, ROWS, 32>(t, grid, vec4, s);
}

hipError_t launch_tt_expand(const TTArgs& t, int mode, hipStream_t s) {
  const int64_t nd = t.dims[t.d - 1];
  const int rpb = tt_rows_per_block(nd);
  const int64_t rb = (t.rows + rpb - 1) / rpb;
  if (rb <= 0) return hipSuccess;
  const int64_t cs = tt_col_splits(t.rows, nd);
  if (rb > 0x7fffffffLL || cs > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)rb, (unsigned)cs);
  const int rl = t.ranks[t.d - 1];
  // four adjacent columns per thread (16-byte accesses) on rows of whole float4s
  const void* io = mode == 0 ? static_cast<const void*>(t.out) : static_cast<const void*>(t.A);
  const bool vec4 = nd % 4 == 0 && nd >= 256 && (reinterpret_cast<uintptr_t>(io) & 15) == 0;
  if (mode == 0) {
    if (rpb == 128) tt_launch_rl<0, 128>(t, rl, grid, vec4, s);
    else tt_launch_rl<0, 64>(t, rl, grid, vec4, s);
  } else {
    if (rpb == 128) tt_launch_rl<1, 128>(t, rl, grid, vec4, s);
    else tt_launch_rl<1, 64>(t, rl, grid, vec4, s);
  }
  NTT_CHECK_LAUNCH();
  if (mode == 1) {
    k_sum_pairs<<<1, 64, 0, s>>>(t.part, rb * cs, t.part + 2 * rb * cs);
    NTT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

static hipError_t launch_gram_impl(const float* X, int64_t m, int64_t k, bool rows, double* part,
                                   double* G, hipStream_t s) {
  if (m < 1 || k < 1) return hipErrorInvalidValue;
  GramArgs g{};
  g.X = X;
  g.m = m;
  g.k = k;
  g.trans = (!rows && m > k) ? 1 : 0;
  g.n = (int)(g.trans ? k : m);
  g.nb = (g.n + 63) / 64;
  size_t pd = 0;
  if (rows) gram_rows_plan(m, k, &g.nsplit, &pd);
  else gram_plan(m, k, &g.nsplit, &pd);
  const int64_t L = g.trans ? m : k;
  g.chunk = ((L + g.nsplit - 1) / g.nsplit + 15) / 16 * 16;
  g.part = part;
  g.G = G;
  const int npairs = g.nb * (g.nb + 1) / 2;
  k_gram<<<dim3((unsigned)npairs, (unsigned)g.nsplit), 256, 0, s>>>(g);
  NTT_CHECK_LAUNCH();
  k_gram_reduce<<<(unsigned)npairs, 256, 0, s>>>(g);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_gram(const float* X, int64_t m, int64_t k, double* part, double* G, hipStream_t s) {
  return launch_gram_impl(X, m, k, false, part, G, s);
}

hipError_t launch_gram_rows(const float* X, int64_t m, int64_t k, double* part, double* G, hipStream_t s) {
  return launch_gram_impl(X, m, k, true, part, G, s);
}

}  // namespace ntt
