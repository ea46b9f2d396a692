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
// atomics) by the finalize kernel, whose last workgroup applies the W-update and forms
// the next W^T W.  The result equals the two-pass MU up to summation order.
//
// Rank r is padded to RP = 16 or 32 (zero rows/columns) to fit the MFMA 16x16x4 f32
// tiles.  All shapes are runtime values; ragged edges are masked to zero, which is
// exact: a zero column of X with a zero column of H stays zero and adds nothing.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntt_internal.h"

namespace ntt {

typedef float v4f __attribute__((ext_vector_type(4)));

// D[4*(l/16)+i][l%16] += sum_s A[l%16][s] * B[s][l%16]; A from lane a+16s, B from lane n+16s.
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Order LDS accesses of one wavefront (LDS is in order per wave; this stops the
// compiler from moving accesses across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

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
      sW[i][c] = (i0 + i < m && c < r) ? W[(int64_t)(i0 + i) * r + c] : 0.f;
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
// x / y by the hardware reciprocal and one Newton-Raphson correction
// (q0 = x r, e = x - y q0, q = q0 + e r): within about 1 ulp for normal y.
__device__ __forceinline__ float fast_div(float x, float y) {
  const float r = __builtin_amdgcn_rcpf(y);
  const float q0 = x * r;
  const float e = fmaf(-y, q0, x);
  return fmaf(e, r, q0);
}

// Variant for m <= 16*MB (MB 16-row blocks held in registers) and r <= RP.
// Each wavefront takes 16-column groups (group g = global wave id + s * total waves).
// UPDATE: do the H-update and accumulate X H_new^T and H_new H_new^T partials.
// RESID : accumulate sum (X - W H_in)^2 in FP64 over the incoming W, H.
// Per-workgroup partial (written when UPDATE): X H_new^T as m x r, then H_new H_new^T
// as r x r, both row-major and compact.
template <int RP, int MB, bool UPDATE, bool RESID>
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
      wtmp[t] = (e < RP * MPAD && i < m && c < r) ? v : 0.f;
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
  const bool vec_ok = ((k & 3) == 0) && ((reinterpret_cast<uintptr_t>(p.X) & 15) == 0) &&
                      ((reinterpret_cast<uintptr_t>(p.H) & 15) == 0);
  float* sXw = sX[w];
  float* sHw = sHn[w];

  // Loads of a 16-column group: X rows 16*blk + a, columns j0+4b .. j0+4b+3 (the A
  // operand of X H^T) and H[16h+4b+kk][j0+a].  Addresses are clamped into the arrays
  // and out-of-range values replaced by zero, so interior groups need no branches.
  auto load_group = [&](int64_t g, float (&xr)[MB][4], float (&hv)[NH][4]) {
    const int64_t j0 = g << 4;
    if (vec_ok && (j0 + 16 <= k)) {
#pragma unroll
      for (int blk = 0; blk < MB; ++blk) {
        const int row = 16 * blk + a;
        const float4 v = *reinterpret_cast<const float4*>(p.X + (int64_t)min(row, m - 1) * k + j0 + 4 * b);
        const bool ok = row < m;
        xr[blk][0] = ok ? v.x : 0.f;
        xr[blk][1] = ok ? v.y : 0.f;
        xr[blk][2] = ok ? v.z : 0.f;
        xr[blk][3] = ok ? v.w : 0.f;
      }
    } else {
#pragma unroll
      for (int blk = 0; blk < MB; ++blk) {
        const int row = 16 * blk + a;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t col = j0 + 4 * b + q;
          const float v = p.X[(int64_t)min(row, m - 1) * k + min(col, k - 1)];
          xr[blk][q] = (row < m && col < k) ? v : 0.f;
        }
      }
    }
    const int64_t col = j0 + a;
    const int64_t colc = min(col, k - 1);
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int c = 16 * h + 4 * b + kk;
        const float v = p.H[(int64_t)min(c, r - 1) * k + colc];
        hv[h][kk] = (c < r && col < k) ? v : 0.f;
      }
  };

  auto process_group = [&](int64_t g, const float (&xr)[MB][4], const float (&hv)[NH][4]) {
    const int64_t j0 = g << 4;
    const bool full = vec_ok && (j0 + 16 <= k);
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
          *reinterpret_cast<float4*>(dst) = hn4[h];
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
#pragma unroll
  for (int c = 0; c < RP; ++c) h[c] = (act && c < r) ? p.H[(int64_t)c * k + j] : 0.f;
  float acc[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) acc[c] = 0.f;
  double res = 0.0;
  for (int i0 = 0; i0 < m; i0 += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * RP; e += 256) {
      const int i = e / RP, c = e % RP;
      sW[i][c] = (i0 + i < m && c < r) ? p.W[(int64_t)(i0 + i) * r + c] : 0.f;
    }
    __syncthreads();
    const int iend = min(64, m - i0);
    for (int i = 0; i < iend; ++i) {
      const float x = act ? p.X[(int64_t)(i0 + i) * k + j] : 0.f;
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
      sX[i][jj] = (gi < m && gj < c1) ? p.X[(int64_t)gi * k + gj] : 0.f;
    }
    for (int e = tid; e < RP * 64; e += 256) {
      const int c = e >> 6, jj = e & 63;
      const int64_t gj = j0 + jj;
      sH[c][jj] = (c < r && gj < c1) ? p.H[(int64_t)c * k + gj] : 0.f;
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
// (1) k_reduce_partials: red[e] = sum over g of part[g][e] in FP64, for the E = m r + r r
//     entries of the partials (X H^T then H H^T); 16 entries per block, 16 chunk
//     threads per entry, four interleaved accumulators per thread, then chunks 0..15
//     in order: a fixed summation order, so results do not depend on scheduling.
__global__ __launch_bounds__(256) void k_reduce_partials(const float* __restrict__ part,
                                                         int64_t stride, int G, int64_t E,
                                                         double* __restrict__ red) {
  __shared__ double sPart[16][17];
  const int tid = threadIdx.x;
  const int e_loc = tid & 15, ch = tid >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + e_loc;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (e < E) {
    int g = ch;
    for (; g + 48 < G; g += 64) {
      a0 += (double)part[(int64_t)g * stride + e];
      a1 += (double)part[(int64_t)(g + 16) * stride + e];
      a2 += (double)part[(int64_t)(g + 32) * stride + e];
      a3 += (double)part[(int64_t)(g + 48) * stride + e];
    }
    for (; g < G; g += 16) a0 += (double)part[(int64_t)g * stride + e];
  }
  sPart[ch][e_loc] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (tid < 16 && (int64_t)blockIdx.x * 16 + tid < E) {
    double s = 0.0;
    for (int c = 0; c < 16; ++c) s += sPart[c][tid];
    red[(int64_t)blockIdx.x * 16 + tid] = s;
  }
}

// (2) k_wupdate: one block.  W <- max(0, W .* N_W ./ (W G_H + eps)) with N_W = X H^T
//     and G_H = H H^T from `red`, 256 rows at a time, one thread per row (rows are
//     independent, so the update is in place; each thread reads its whole row before
//     writing it).  FP64 arithmetic on FP32 data, rounded to FP32.  The new rows also
//     go to LDS, where the block accumulates G_W' = W'^T W' (FP64) for the next
//     H-update.  It also writes the Gram-identity monitor
//       f = 1/2 (||X||^2 - 2 <W', X H^T> + <W'^T W', H H^T>)
//     and, when this iteration accumulated one, the explicit residual objective.
template <int RP>
__global__ __launch_bounds__(256) void k_wupdate(FinArgs f) {
  __shared__ double sGH[RP][RP + 1];
  __shared__ double sGW[RP][RP + 1];
  __shared__ float sWc[256][RP + 1];
  __shared__ double sRed[4];
  const int tid = threadIdx.x;
  const int m = f.m, r = f.r;
  const double* NW = f.red;
  const double* GH = f.red + (int64_t)m * r;
  for (int pidx = tid; pidx < RP * RP; pidx += 256) {
    const int c = pidx / RP, q = pidx % RP;
    sGH[c][q] = (c < r && q < r) ? GH[c * r + q] : 0.0;
  }
  double rsum = 0.0;
  if (f.rpart && tid < 64) {
    for (int g = tid; g < f.G; g += 64) rsum += f.rpart[g];
    rsum = wave_sum(rsum);
  }
  __syncthreads();
  constexpr int NP = (RP * RP + 255) / 256;
  double gacc[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) gacc[t] = 0.0;
  double dot_wn = 0.0;
  for (int i0 = 0; i0 < m; i0 += 256) {
    const int i = i0 + tid;
    if (i < m) {
      float wrow[RP];
      double nrow[RP];
      const int64_t base = (int64_t)i * r;
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        const int qc = min(q, r - 1);
        const float wv = f.W[base + qc];
        const double nv = NW[base + qc];
        wrow[q] = (q < r) ? wv : 0.f;
        nrow[q] = (q < r) ? nv : 0.0;
      }
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        double dw = 0.0;
#pragma unroll
        for (int q = 0; q < RP; ++q) dw += (double)wrow[q] * sGH[q][c];
        const double wn = fmax(0.0, (double)wrow[c] * nrow[c] / (dw + (double)f.eps));
        const float wf = (c < r) ? (float)wn : 0.f;
        sWc[tid][c] = wf;
        dot_wn += (double)wf * nrow[c];
      }
#pragma unroll
      for (int c = 0; c < RP; ++c)
        if (c < r) f.W[base + c] = sWc[tid][c];
    } else {
#pragma unroll
      for (int c = 0; c < RP; ++c) sWc[tid][c] = 0.f;
    }
    __syncthreads();
    gram_chunk<RP>(sWc, min(256, m - i0), gacc);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    const int pidx = tid + 256 * t;
    if (pidx < RP * RP) {
      sGW[pidx / RP][pidx % RP] = gacc[t];
      f.GW[pidx] = (float)gacc[t];
    }
  }
  dot_wn = wave_sum(dot_wn);
  if ((tid & 63) == 0) sRed[tid >> 6] = dot_wn;
  __syncthreads();
  if (tid == 0) {
    const double wn = ((sRed[0] + sRed[1]) + sRed[2]) + sRed[3];
    double gg = 0.0;
    for (int c = 0; c < r; ++c)
      for (int q = 0; q < r; ++q) gg += sGW[c][q] * sGH[c][q];
    f.scal[SCAL_MONITOR] = 0.5 * (f.scal[SCAL_NX2] - 2.0 * wn + gg);
    if (f.rpart) {
      const double obj = 0.5 * rsum;
      f.scal[SCAL_OBJ] = obj;
      if (f.trace) f.trace[0] = obj;
    }
  }
}

// copy helper: dst[i] = src[i]
__global__ void k_copy(float* __restrict__ dst, const float* __restrict__ src, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

// ------------------------------------------------------------------ TT expand (Eq.(2))
// Rows of the (n_1...n_{d-1}) x n_d matrix of the full tensor, 64 per block.  Each row's
// left factor P[row,:] = G_1[i_1,:] G_2[:,i_2,:] ... G_{d-1}[:,i_{d-1},:] is formed in
// LDS (FP32), then Ahat[row, col] = P[row,:] . G_d[:, col].  MODE 0 writes Ahat; MODE 1
// accumulates sum (A - Ahat)^2 and sum A^2 in FP64 per block.
template <int MODE>
__global__ __launch_bounds__(256) void k_tt_expand(TTArgs t) {
  __shared__ float sP[2][64][NTT_MAX_RANK + 1];
  __shared__ int sIdx[64][NTT_MAX_DIMS];
  __shared__ double sRed[2][4];
  const int tid = threadIdx.x;
  const int d = t.d;
  const int64_t rows = t.rows;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int nrow = (int)min((int64_t)64, rows - r0);
  if (tid < nrow) {
    int64_t rem = r0 + tid;
    for (int kx = d - 2; kx >= 0; --kx) {
      sIdx[tid][kx] = (int)(rem % t.dims[kx]);
      rem /= t.dims[kx];
    }
  }
  __syncthreads();
  // P_1 = G_1[i_1, :]
  int cur = 0;
  {
    const int rk = t.ranks[1];
    for (int e = tid; e < 64 * rk; e += 256) {
      const int rr = e / rk, c = e % rk;
      sP[0][rr][c] = (rr < nrow) ? t.cores[0][(int64_t)sIdx[rr][0] * rk + c] : 0.f;
    }
  }
  __syncthreads();
  for (int kx = 1; kx < d - 1; ++kx) {
    const int ra = t.ranks[kx], rb = t.ranks[kx + 1];
    const int64_t nk = t.dims[kx];
    const float* G = t.cores[kx];
    for (int e = tid; e < 64 * rb; e += 256) {
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
  const int64_t base = r0 * nd;
  const int64_t cnt = (int64_t)nrow * nd;
  double s_err = 0.0, s_ref = 0.0;
  for (int64_t e = tid; e < cnt; e += 256) {
    const int rr = (int)(e / nd);
    const int64_t col = e - (int64_t)rr * nd;
    float s = 0.f;
    for (int q = 0; q < rl; ++q) s = fmaf(sP[cur][rr][q], Gd[(int64_t)q * nd + col], s);
    if (MODE == 0) {
      t.out[base + e] = s;
    } else {
      const double av = (double)t.A[base + e];
      const double dv = av - (double)s;
      s_err += dv * dv;
      s_ref += av * av;
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
      t.part[2 * blockIdx.x] = ((sRed[0][0] + sRed[0][1]) + sRed[0][2]) + sRed[0][3];
      t.part[2 * blockIdx.x + 1] = ((sRed[1][0] + sRed[1][1]) + sRed[1][2]) + sRed[1][3];
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
  if (update && resid) k_mu_pass<RP, MB, true, true><<<grid, 256, 0, s>>>(a);
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
    case 4: return pass_fused_mb<RP, 4>(a, grid, update, resid, s);
    case 8: return pass_fused_mb<RP, 8>(a, grid, update, resid, s);
    case 16: return pass_fused_mb<RP, 16>(a, grid, update, resid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pass_fused(const PassArgs& a, int rp, int mb, int grid, bool update, bool resid,
                             hipStream_t s) {
  return rp == 16 ? pass_fused_rp<16>(a, mb, grid, update, resid, s)
                  : pass_fused_rp<32>(a, mb, grid, update, resid, s);
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
  if (update) {
    dim3 grid(gxht, (a.m + 63) / 64);
    if (rp == 16) k_gen_xht<16><<<grid, 256, 0, s>>>(a, chunk);
    else k_gen_xht<32><<<grid, 256, 0, s>>>(a, chunk);
    NTT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

hipError_t launch_finalize(const FinArgs& f, int rp, hipStream_t s) {
  const int64_t E = (int64_t)f.m * f.r + (int64_t)f.r * f.r;
  const int nb = (int)((E + 15) / 16);
  k_reduce_partials<<<nb, 256, 0, s>>>(f.part, f.part_stride, f.G, E, f.red);
  NTT_CHECK_LAUNCH();
  if (rp == 16) k_wupdate<16><<<1, 256, 0, s>>>(f);
  else k_wupdate<32><<<1, 256, 0, s>>>(f);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_resid_sum(const double* rpart, int G, double* obj, double* trace, hipStream_t s) {
  k_sum_doubles<<<1, 64, 0, s>>>(rpart, G, 0.5, obj, trace);
  NTT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_tt_expand(const TTArgs& t, int mode, hipStream_t s) {
  const int64_t nb = (t.rows + 63) / 64;
  if (nb <= 0) return hipSuccess;
  if (mode == 0) k_tt_expand<0><<<(unsigned)nb, 256, 0, s>>>(t);
  else k_tt_expand<1><<<(unsigned)nb, 256, 0, s>>>(t);
  NTT_CHECK_LAUNCH();
  if (mode == 1) {
    k_sum_pairs<<<1, 64, 0, s>>>(t.part, nb, t.part + 2 * nb);
    NTT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

}  // namespace ntt
