// ntt_bcd.hip -- the BCD NMF of Alg.3 for one stage of the sweep: projected-gradient
// steps on the two blocks (W first, then H), each from an extrapolated point, with the
// objective test keeping the new pair ("extrapolation") or dropping it ("correction").
//
// One iteration is four launches whose arguments never change, so blocks of iterations
// can be captured into a graph and replayed; every data-dependent choice is made on the
// device and kept in a small state block (BcdState):
//   k_bcd_step   one workgroup.  (a) Decides on the previous iteration's candidate: it is
//                kept when its objective is below the kept one; then the kept pair, its
//                products X H^T, H H^T and the extrapolation weights move on, else they
//                stay and the next steps start from the kept pair without extrapolation.
//                (b) W_m = W + w_W (W - W_prev) and the W step
//                W_n = max(0, W_m - (W_m H H^T - X H^T) / ||H H^T||_F), in FP64 on FP32
//                data, then W_n /= sum(W_n) (the L1 normalisation the W block of Alg.3
//                ends with; W_n >= 0, and a zero W_n is left as it is), and
//                G = W_n^T W_n of the normalised W_n (FP64, rows in order).
//   k_bcd_h      one thread per column: H_m = H + w_H (H - H_prev), W_n^T X, and the H step
//                H_n = max(0, H_m - (G H_m - W_n^T X) / ||G||_F) into the candidate buffer.
//   k_bcd_xht    X H_n^T and H_n H_n^T partials per column chunk, and per workgroup the
//                FP64 residual sum ||X - W_n H_n||^2 of its tile (the objective of the test).
//   k_reduce_partials (the MU reduction) adds the partials in a fixed order.
// The three r x k H buffers change roles by index (kept, kept before, candidate), so no
// H is ever copied during the iterations; W, its earlier values and the products are
// small and are copied.  Every sum has a fixed order: results do not depend on scheduling.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "ntt_internal.h"

namespace ntt {
namespace {

// `v` where `ok`, else 0, for a value loaded from a clamped (always valid) address
// (a multiply keeps the load unconditional).
__device__ __forceinline__ float bmask(float v, bool ok) { return v * (ok ? 1.f : 0.f); }
__device__ __forceinline__ double bmask(double v, bool ok) { return v * (ok ? 1.0 : 0.0); }

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double bcd_wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Scale a factor to Frobenius norm sqrt(||X||_F): a *= ||X||^(1/2) / ||a|| (a zero factor
// is left as it is).
__global__ void k_bcd_scale(float* __restrict__ a, int64_t n, const double* __restrict__ nx2,
                            const double* __restrict__ na2) {
  const double s2 = *na2;
  const double f = s2 > 0.0 ? std::sqrt(std::sqrt(*nx2)) / std::sqrt(s2) : 1.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    a[i] = (float)((double)a[i] * f);
}

// t = 1, the objective of W = H = 0 (1/2 ||X||^2), no extrapolation, the initial H kept
// in Hb[0].
__global__ void k_bcd_state_init(BcdState* st, const double* __restrict__ scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  BcdState s{};
  s.t = 1.0;
  s.obj = 0.5 * scal[SCAL_NX2];
  s.cur = 0;
  s.prev = 2;
  s.nxt = 1;
  s.first = 1;
  st[0] = s;
}

// X H^T and H H^T partials of H (Hb[0] when `init`, else the candidate Hb[nxt]), as
// block (g, rb) covers column chunk g and rows 64 rb .. 64 rb + 63; with RESID also the
// FP64 sum of (x - (W_n H)_ij)^2 over the tile.  Partial layout per chunk: [m][r] then
// [r][r] (H H^T by the rb = 0 blocks).  XV: X rows are read as float4 (k % 4 == 0 and a
// 16-byte aligned X).
template <int RP, bool RESID, bool XV>
__global__ __launch_bounds__(256) void k_bcd_xht(BcdArgs b, int init) {
  // rows of 68 floats: 16-byte aligned, so the tile is written and read as float4
  __shared__ __attribute__((aligned(16))) float sX[64][68];
  __shared__ __attribute__((aligned(16))) float sH[RP][68];
  __shared__ double sRes[4];
  const int tid = threadIdx.x;
  const int m = b.m, r = b.r;
  const int64_t k = b.k;
  const float* __restrict__ H = init ? b.Hb[0] : b.Hb[b.st->nxt];
  const int g = blockIdx.x, rb = blockIdx.y;
  const int64_t c0 = (int64_t)g * b.chunk, c1 = min(k, c0 + b.chunk);
  const int mrows = min(64, m - 64 * rb);  // rows of this block inside X
  // threads per row: 4 (16 columns of a 64-column tile each), 8 when the block holds at
  // most 32 rows, 16 when at most 16
  const int tpr = mrows <= 16 ? 16 : (mrows <= 32 ? 8 : 4);
  const int cpt = 64 / tpr;
  const int row = tid / tpr, part = tid % tpr;
  const int gi = 64 * rb + row;
  float acc[RP];
  float w[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) {
    acc[c] = 0.f;
    w[c] = RESID ? bmask(b.Wn[(int64_t)min(gi, m - 1) * r + min(c, r - 1)], gi < m && c < r) : 0.f;
  }
  // the Gram: GT threads per pair while there are fewer pairs than threads
  constexpr int GT = RP * RP >= 256 ? 1 : 256 / (RP * RP);
  constexpr int NG = RP * RP / 256 > 0 ? RP * RP / 256 : 1;
  float accg[NG];
#pragma unroll
  for (int t = 0; t < NG; ++t) accg[t] = 0.f;
  double res = 0.0;
  // Tiles go through registers two deep: the loads of tile t + 2 are issued before
  // tile t is computed, and each tile is stored to LDS (masked there) when its turn comes.
  constexpr int HPT = (RP * 64 + 255) / 256;  // H tile entries per thread
  float4 xr0[4], xr1[4];
  float hr0[HPT], hr1[HPT];
  auto issue = [&](float4 (&xr)[4], float (&hr)[HPT], int64_t j0) {
    if (XV) {
      // 16 float4 per tile row: each load instruction of a wave covers 4 rows x 256
      // bytes; groups of 16 rows wholly beyond m are not loaded
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (16 * q < mrows) {
          const int e = tid + 256 * q;
          const int i = e >> 4, j4 = (e & 15) * 4;
          const int xi = 64 * rb + i;
          const int64_t gj = j0 + j4;
          const bool ok = xi < m && gj < c1;
          xr[q] = *reinterpret_cast<const float4*>(b.X + (int64_t)min(xi, m - 1) * k + (ok ? gj : c0));
        }
      }
    }
#pragma unroll
    for (int t = 0; t < HPT; ++t) {
      const int e = tid + 256 * t;
      const int c = min(e >> 6, RP - 1), jj = e & 63;
      const int64_t gj = j0 + jj;
      hr[t] = H[(int64_t)min(c, r - 1) * k + min(gj, c1 - 1)];
    }
  };
  auto store = [&](const float4 (&xr)[4], const float (&hr)[HPT], int64_t j0) {
    if (XV) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q;
        const int i = e >> 4, j4 = (e & 15) * 4;
        const int xi = 64 * rb + i;
        const bool ok = 16 * q < mrows && xi < m && j0 + j4 < c1;
        *reinterpret_cast<float4*>(&sX[i][j4]) = ok ? xr[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    } else {
      for (int e = tid; e < 64 * 64; e += 256) {
        const int i = e >> 6, jj = e & 63;
        const int xi = 64 * rb + i;
        const int64_t gj = j0 + jj;
        sX[i][jj] = bmask(b.X[(int64_t)min(xi, m - 1) * k + min(gj, c1 - 1)], xi < m && gj < c1);
      }
    }
#pragma unroll
    for (int t = 0; t < HPT; ++t) {
      const int e = tid + 256 * t;
      if (e < RP * 64) {
        const int c = e >> 6, jj = e & 63;
        sH[c][jj] = (c < r && j0 + jj < c1) ? hr[t] : 0.f;
      }
    }
  };
  auto compute = [&]() {
    // four columns per LDS read; the columns are still taken in order
#pragma unroll 1
    for (int j4 = part * cpt; j4 < part * cpt + cpt; j4 += 4) {
      const float4 xv = *reinterpret_cast<const float4*>(&sX[row][j4]);
      float wh0 = 0.f, wh1 = 0.f, wh2 = 0.f, wh3 = 0.f;
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        const float4 hv = *reinterpret_cast<const float4*>(&sH[c][j4]);
        float a = acc[c];
        a = fmaf(xv.x, hv.x, a);
        a = fmaf(xv.y, hv.y, a);
        a = fmaf(xv.z, hv.z, a);
        a = fmaf(xv.w, hv.w, a);
        acc[c] = a;
        if (RESID) {
          wh0 = fmaf(w[c], hv.x, wh0);
          wh1 = fmaf(w[c], hv.y, wh1);
          wh2 = fmaf(w[c], hv.z, wh2);
          wh3 = fmaf(w[c], hv.w, wh3);
        }
      }
      if (RESID) {  // 0 outside the matrix
        const double d0 = (double)xv.x - (double)wh0, d1 = (double)xv.y - (double)wh1;
        const double d2 = (double)xv.z - (double)wh2, d3 = (double)xv.w - (double)wh3;
        res += d0 * d0;
        res += d1 * d1;
        res += d2 * d2;
        res += d3 * d3;
      }
    }
    if (rb == 0) {
      // H H^T: pair p of the RP x RP Gram, GT threads per pair over 64 / GT columns each
#pragma unroll
      for (int t = 0; t < NG; ++t) {
        const int pidx = tid / GT + (256 / GT) * t;
        if (pidx < RP * RP) {
          const int c = pidx / RP, q = pidx % RP;
          const int j1 = (tid % GT) * (64 / GT);
          float s = accg[t];
#pragma unroll 4
          for (int jj = j1; jj < j1 + 64 / GT; jj += 4) {
            const float4 u = *reinterpret_cast<const float4*>(&sH[c][jj]);
            const float4 v = *reinterpret_cast<const float4*>(&sH[q][jj]);
            s = fmaf(u.x, v.x, s);
            s = fmaf(u.y, v.y, s);
            s = fmaf(u.z, v.z, s);
            s = fmaf(u.w, v.w, s);
          }
          accg[t] = s;
        }
      }
    }
  };
  // two tiles in flight: tile t + 2 is issued while tile t is computed
  issue(xr0, hr0, c0);
  if (c0 + 64 < c1) issue(xr1, hr1, c0 + 64);
  for (int64_t j0 = c0; j0 < c1; j0 += 128) {
    __syncthreads();
    store(xr0, hr0, j0);
    __syncthreads();
    if (j0 + 128 < c1) issue(xr0, hr0, j0 + 128);
    compute();
    if (j0 + 64 < c1) {
      __syncthreads();
      store(xr1, hr1, j0 + 64);
      __syncthreads();
      if (j0 + 192 < c1) issue(xr1, hr1, j0 + 192);
      compute();
    }
  }
  // the column parts of each row, added in order
  __syncthreads();
  float* red = &sX[0][0];
  float* dst = b.part + (int64_t)g * b.part_stride;
  for (int c = 0; c < RP; ++c) {
    __syncthreads();
    red[tid] = acc[c];
    __syncthreads();
    if (part == 0) {
      float s = red[tid];
      for (int p2 = 1; p2 < tpr; ++p2) s += red[tid + p2];
      if (gi < m && c < r) dst[(int64_t)gi * r + c] = s;
    }
  }
  if (rb == 0) {
#pragma unroll
    for (int t = 0; t < NG; ++t) {
      __syncthreads();
      red[tid] = accg[t];
      __syncthreads();
      const int pidx = tid / GT + (256 / GT) * t;
      if (tid % GT == 0 && pidx < RP * RP && pidx / RP < r && pidx % RP < r) {
        float s = red[tid];
        for (int p2 = 1; p2 < GT; ++p2) s += red[tid + p2];
        dst[(int64_t)m * r + (pidx / RP) * r + (pidx % RP)] = s;
      }
    }
  }
  if (RESID) {
    res = bcd_wave_sum(res);
    if ((tid & 63) == 0) sRes[tid >> 6] = res;
    __syncthreads();
    if (tid == 0) b.rpart[(int64_t)g * gridDim.y + rb] = ((sRes[0] + sRes[1]) + sRes[2]) + sRes[3];
  }
}

// The same products with FP32 MFMA (16 x 16 x 4) when X rows are float4-readable
// (k % 4 == 0, 16-byte aligned X).  Tiles hold RT rows x CT = 4096 / RT columns (RT = 64
// for more than 32 rows, else 32 or 16, so that short unfoldings keep every wave busy);
// block (g, rb) covers column chunk g and tile rows RT rb ...  Wave w owns rows
// 16 (w % WR) .. + 15 and the 64 columns 64 (w / WR) .. + 63 of each tile (WR = RT / 16).
// Lane l = (a, q4) with a = l % 16, q4 = l / 16; output register i of an MFMA is
// D[4 q4 + i][a].  Per tile:
//   X H^T: A = X[row0 + a][col0 + 4 s + q4], B = H[16 n + a][col0 + 4 s + q4], s = 0..15;
//   W_n H (residual): A = W_n[row0 + a][4 s + q4] (registers), B = H[4 s + q4][col0 + 16 cb + a],
//     lined up with X[row0 + 4 q4 + i][col0 + 16 cb + a] read from LDS;
//   H H^T (rb = 0): the CT / 4 column steps split over the four waves.
// Partials of waves that share rows, and the waves' H H^T parts, are added in wave order.
template <int RP, bool RESID, int RT>
__global__ __launch_bounds__(256) void k_bcd_xhtm(BcdArgs b, int init) {
  constexpr int NB = (RP + 15) / 16;  // 16-wide rank blocks
  constexpr int RQ = NB * 16;         // ranks padded to a multiple of 16
  constexpr int CT = 4096 / RT;       // tile columns
  constexpr int WR = RT / 16;         // waves along the rows
  constexpr int WC = 4 / WR;          // waves along the columns
  constexpr int HPT = RQ * CT / 256;  // H tile entries per thread
  constexpr int RPQ = RT / 4;         // tile rows per float4 load instruction group
  __shared__ __attribute__((aligned(16))) float sX[RT][CT + 4];
  __shared__ __attribute__((aligned(16))) float sH[RQ][CT + 4];
  __shared__ double sRes[4];
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63, la = ln & 15, lq = ln >> 4;
  const int wr = wv % WR, wc = wv / WR;
  const int row0 = 16 * wr, col0 = 64 * wc;
  const int m = b.m, r = b.r;
  const int64_t k = b.k;
  const float* __restrict__ H = init ? b.Hb[0] : b.Hb[b.st->nxt];
  const int g = blockIdx.x, rb = blockIdx.y;
  const int64_t c0 = (int64_t)g * b.chunk, c1 = min(k, c0 + b.chunk);
  const int mrows = min(RT, m - RT * rb);
  float wop[RQ / 4];
#pragma unroll
  for (int s4 = 0; s4 < RQ / 4; ++s4) {
    const int row = RT * rb + row0 + la, c = 4 * s4 + lq;
    wop[s4] = RESID ? bmask(b.Wn[(int64_t)min(row, m - 1) * r + min(c, r - 1)], row < m && c < r) : 0.f;
  }
  v4f accx[NB];
  v4f accg[NB][NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    accx[n] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NB; ++q) accg[n][q] = v4f{0.f, 0.f, 0.f, 0.f};
  }
  double res = 0.0;
  float4 xr0[4], xr1[4];
  float hr0[HPT], hr1[HPT];
  auto issue = [&](float4 (&xr)[4], float (&hr)[HPT], int64_t j0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (RPQ * q < mrows) {  // load groups wholly beyond m are skipped
        const int e = tid + 256 * q;
        const int i = e / (CT / 4), j4 = (e % (CT / 4)) * 4;
        const int xi = RT * rb + i;
        const int64_t gj = j0 + j4;
        const bool ok = xi < m && gj < c1;
        xr[q] = *reinterpret_cast<const float4*>(b.X + (int64_t)min(xi, m - 1) * k + (ok ? gj : c0));
      }
    }
#pragma unroll
    for (int t = 0; t < HPT; ++t) {
      const int e = tid + 256 * t;
      const int c = e / CT, jj = e % CT;
      hr[t] = H[(int64_t)min(c, r - 1) * k + min(j0 + jj, c1 - 1)];
    }
  };
  auto store = [&](const float4 (&xr)[4], const float (&hr)[HPT], int64_t j0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int i = e / (CT / 4), j4 = (e % (CT / 4)) * 4;
      const bool ok = RPQ * q < mrows && RT * rb + i < m && j0 + j4 < c1;
      *reinterpret_cast<float4*>(&sX[i][j4]) = ok ? xr[q] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int t = 0; t < HPT; ++t) {
      const int e = tid + 256 * t;
      const int c = e / CT, jj = e % CT;
      sH[c][jj] = (c < r && j0 + jj < c1) ? hr[t] : 0.f;
    }
  };
  auto compute = [&]() {
#pragma unroll 4
    for (int s4 = 0; s4 < 16; ++s4) {
      const float av = sX[row0 + la][col0 + 4 * s4 + lq];
#pragma unroll
      for (int n = 0; n < NB; ++n)
        accx[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sH[16 * n + la][col0 + 4 * s4 + lq], accx[n], 0, 0, 0);
    }
    if (rb == 0) {
#pragma unroll
      for (int s4 = wv * (CT / 16); s4 < (wv + 1) * (CT / 16); ++s4) {
        float op[NB];
#pragma unroll
        for (int n = 0; n < NB; ++n) op[n] = sH[16 * n + la][4 * s4 + lq];
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
          for (int q = 0; q < NB; ++q)
            accg[n][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(op[n], op[q], accg[n][q], 0, 0, 0);
      }
    }
    if (RESID) {
      // the lane's 16 squared residuals of the tile in FP32 (each difference carries the
      // rounding of the FP32 product d already), their sum added to the FP64 total
      float tsum = 0.f;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        v4f d = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s4 = 0; s4 < RQ / 4; ++s4)
          d = __builtin_amdgcn_mfma_f32_16x16x4f32(wop[s4], sH[4 * s4 + lq][col0 + 16 * cb + la], d, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float dl = sX[row0 + 4 * lq + i][col0 + 16 * cb + la] - d[i];
          tsum = fmaf(dl, dl, tsum);  // 0 outside the matrix
        }
      }
      res += (double)tsum;
    }
  };
  issue(xr0, hr0, c0);
  if (c0 + CT < c1) issue(xr1, hr1, c0 + CT);
  for (int64_t j0 = c0; j0 < c1; j0 += 2 * CT) {
    __syncthreads();
    store(xr0, hr0, j0);
    __syncthreads();
    if (j0 + 2 * CT < c1) issue(xr0, hr0, j0 + 2 * CT);
    compute();
    if (j0 + CT < c1) {
      __syncthreads();
      store(xr1, hr1, j0 + CT);
      __syncthreads();
      if (j0 + 3 * CT < c1) issue(xr1, hr1, j0 + 3 * CT);
      compute();
    }
  }
  // LDS scratch for the wave sums (sX is free now): [4 waves][NB * NB][64 lanes][4]
  float* sG = &sX[0][0];
  float* dst = b.part + (int64_t)g * b.part_stride;
  if (WC > 1) {
    __syncthreads();
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
      for (int i = 0; i < 4; ++i) sG[((wv * NB + n) * 64 + ln) * 4 + i] = accx[n][i];
    __syncthreads();
  }
  if (wc == 0) {
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = accx[n][i];
        for (int c2 = 1; c2 < WC; ++c2) v += sG[(((c2 * WR + wr) * NB + n) * 64 + ln) * 4 + i];
        const int row = RT * rb + row0 + 4 * lq + i, c = 16 * n + la;
        if (row < m && c < r) dst[(int64_t)row * r + c] = v;
      }
  }
  if (rb == 0) {
    __syncthreads();
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) sG[(((wv * NB * NB) + n * NB + q) * 64 + ln) * 4 + i] = accg[n][q][i];
    __syncthreads();
    for (int e = tid; e < RQ * RQ; e += 256) {
      const int c = e / RQ, q = e % RQ;
      if (c < r && q < r) {
        // FP32 16 x 16 x 4 output: register i of lane l is row 4 (l / 16) + i, column l % 16
        const int n = c / 16, i = c % 4, lane = ((c % 16) / 4) * 16 + q % 16, qq = q / 16;
        float v = 0.f;
        for (int w4 = 0; w4 < 4; ++w4) v += sG[(((w4 * NB * NB) + n * NB + qq) * 64 + lane) * 4 + i];
        dst[(int64_t)m * r + c * r + q] = v;
      }
    }
  }
  if (RESID) {
    res = bcd_wave_sum(res);
    if (ln == 0) sRes[wv] = res;
    __syncthreads();
    if (tid == 0) b.rpart[(int64_t)g * gridDim.y + rb] = ((sRes[0] + sRes[1]) + sRes[2]) + sRes[3];
  }
}

// The decision on the previous candidate (unless this is the stage's first step), then,
// unless `final_step`, the W step, its L1 normalisation and G = W_n^T W_n.  One workgroup;
// thread tid owns rows tid, tid + 256, ... in every phase, so it only re-reads global data
// it wrote itself.
// The kernel is latency-bound: every load it needs for the decision and for its first
// 256 rows is issued at once, the sums go through one barrier, and every thread then
// takes the (identical) decision itself.
template <int RP>
__global__ __launch_bounds__(256) void k_bcd_step(BcdArgs b, int final_step) {
  __shared__ float sWn[256][RP + 1];
  __shared__ double sHH[RP][RP + 1];
  __shared__ double sPart[4][4];  // per-wave sums: objective, ||H_n H_n^T||^2, ||G||^2, sum(W_n)
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const int m = b.m, r = b.r;
  const int64_t mr = (int64_t)m * r;
  BcdState* st = b.st;
  const BcdState s0 = *st;
  // rows of one 256-row chunk: kept W, W before it, candidate W, X H^T kept and candidate
  float wc[RP], wp[RP], wn[RP];
  double xc[RP], xn[RP];
  auto load_rows = [&](int i0) {
    const int i = i0 + tid;
    const bool ok = i < m;
    const int ic = ok ? i : m - 1;
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      const int64_t e = (int64_t)ic * r + min(c, r - 1);
      const bool v = ok && c < r;
      wc[c] = bmask(b.W[e], v);
      wp[c] = bmask(b.Wp[e], v);
      wn[c] = bmask(b.Wn[e], v);
      xc[c] = bmask(b.XHc[e], v);
      xn[c] = bmask(b.red[e], v);
    }
  };
  load_rows(0);
  const int nres = b.G * ((m + 63) / 64);
  double fpart = 0.0;
  if (!s0.first)
    for (int i0 = tid; i0 < nres; i0 += 256 * 8) {  // eight independent loads at a time
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = bmask(b.rpart[min(i0 + 256 * u, nres - 1)], i0 + 256 * u < nres);
#pragma unroll
      for (int u = 0; u < 8; ++u) fpart += v[u];
    }
  constexpr int NG = (RP * RP + 255) / 256;
  double hn[NG], hc[NG];
  double g2 = 0.0;
#pragma unroll
  for (int t = 0; t < NG; ++t) {
    const int e = tid + 256 * t;
    const int c = e / RP, q = e % RP;
    const bool ok = e < RP * RP && c < r && q < r;
    const int64_t ee = ok ? (int64_t)c * r + q : 0;
    hn[t] = bmask(b.red[mr + ee], ok);
    hc[t] = bmask(b.HHc[ee], ok);
    g2 += hn[t] * hn[t];
  }
  fpart = bcd_wave_sum(fpart);
  g2 = bcd_wave_sum(g2);
  if (ln == 0) {
    sPart[0][wv] = fpart;
    sPart[1][wv] = g2;
  }
  __syncthreads();  // also: every wave has read the state before thread 0 rewrites it
  const double f = 0.5 * (((sPart[0][0] + sPart[0][1]) + sPart[0][2]) + sPart[0][3]);
  const double gHn = std::sqrt(((sPart[1][0] + sPart[1][1]) + sPart[1][2]) + sPart[1][3]);
  BcdState s = s0;
  int mode;  // 0: candidate dropped, 1: kept, 2: first step
  if (s0.first) {
    mode = 2;
    s.first = 0;
    s.gH = gHn;
    s.wW = s.wH = 0.0;
  } else if (f < s0.obj) {
    mode = 1;
    const double tp = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * s0.t * s0.t));
    const double w = (s0.t - 1.0) / tp;
    s.wW = gHn > 0.0 ? std::min(w, b.delta * std::sqrt(s0.gH / gHn)) : w;
    s.wH = s0.gWn > 0.0 ? std::min(w, b.delta * std::sqrt(s0.gW / s0.gWn)) : w;
    s.gH = gHn;
    s.gW = s0.gWn;
    s.t = tp;
    s.obj = f;
    s.prev = s0.cur;
    s.cur = s0.nxt;
    s.nxt = s0.prev;
  } else {
    mode = 0;
    s.wW = s.wH = 0.0;
    s.corrections += 1;
  }
  if (tid == 0) {
    if (b.trace && !s0.first) b.trace[0] = f;
    *st = s;
  }
  // H H^T of the kept H into LDS (and into HHc when it changed)
#pragma unroll
  for (int t = 0; t < NG; ++t) {
    const int e = tid + 256 * t;
    if (e < RP * RP) {
      const int c = e / RP, q = e % RP;
      const double v = mode ? hn[t] : hc[t];
      sHH[c][q] = v;
      if (mode && c < r && q < r) b.HHc[c * r + q] = v;
    }
  }
  if (final_step) {
    for (int i0 = 0; i0 < m; i0 += 256) {
      if (i0 > 0) load_rows(i0);
      const int i = i0 + tid;
      if (mode == 1 && i < m)
#pragma unroll
        for (int c = 0; c < RP; ++c)
          if (c < r) {
            const int64_t e = (int64_t)i * r + c;
            b.Wp[e] = wc[c];
            b.W[e] = wn[c];
            b.XHc[e] = xn[c];
          }
    }
    if (tid == 0) {
      b.scal[SCAL_BCD_CORR] = (double)s.corrections;
      b.scal[SCAL_BCD_OBJ] = s.obj;
    }
    return;
  }
  __syncthreads();
  const double wW = s.wW, LW = s.gH;
  // accumulators of G = W_n^T W_n
  constexpr int NT = (RP + 15) / 16;
  v4d gm[NT][NT];
#pragma unroll
  for (int h = 0; h < NT; ++h)
#pragma unroll
    for (int q = 0; q < NT; ++q) gm[h][q] = v4d{0.0, 0.0, 0.0, 0.0};
  const int la = ln & 15, lb = ln >> 4;
  // (1) the W step from the extrapolated point, row by row; the entry sum of W_n for its
  // L1 norm.  With one 256-row chunk the unnormalised rows stay in registers (FP64);
  // with more they go to Wn as FP32 and are read back by the same thread in (2).
  const bool one_chunk = m <= 256;
  double wd[RP];
  double wsum = 0.0;
  for (int i0 = 0; i0 < m; i0 += 256) {
    if (i0 > 0) load_rows(i0);
    const int i = i0 + tid;
#pragma unroll
    for (int c = 0; c < RP; ++c) wd[c] = 0.0;
    if (i < m) {
      double wm[RP], xh[RP];
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        // the kept W (and the kept W before it) after the decision
        const double cur = mode == 1 ? (double)wn[c] : (double)wc[c];
        const double prv = mode == 1 ? (double)wc[c] : (double)wp[c];
        xh[c] = mode ? xn[c] : xc[c];
        wm[c] = wW != 0.0 ? cur + wW * (cur - prv) : cur;
        if (c < r) {
          const int64_t e = (int64_t)i * r + c;
          if (mode == 1) {
            b.Wp[e] = wc[c];
            b.W[e] = wn[c];
          }
          if (mode) b.XHc[e] = xh[c];
        }
      }
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        if (c < r) {
          double gr = -xh[c];
#pragma unroll
          for (int q = 0; q < RP; ++q) gr += wm[q] * sHH[q][c];
          const double v = LW > 0.0 ? wm[c] - gr / LW : wm[c];
          wd[c] = std::max(0.0, v);
          wsum += wd[c];
          if (!one_chunk) b.Wn[(int64_t)i * r + c] = (float)wd[c];
        }
      }
    }
  }
  wsum = bcd_wave_sum(wsum);
  if (ln == 0) sPart[3][wv] = wsum;
  __syncthreads();
  const double l1 = ((sPart[3][0] + sPart[3][1]) + sPart[3][2]) + sPart[3][3];
  const double l1d = l1 > 0.0 ? l1 : 1.0;  // a zero W_n stays as it is
  // (2) W_n / ||W_n||_1 into Wn, and G = W_n^T W_n with FP64 MFMA (16 x 16 x 4): wave wv
  // takes rows 64 wv .. 64 wv + 63 of each 256-row chunk, four rows a step, the lane
  // (a, bq) feeding W_n[row 4 st + bq][a] as both operands; output register i of lane l is
  // G[4 i + l / 16][l % 16]
  for (int i0 = 0; i0 < m; i0 += 256) {
    const int i = i0 + tid;
    float wo[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) wo[c] = 0.f;
    if (i < m) {
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        if (c < r) {
          const int64_t e = (int64_t)i * r + c;
          const double v = one_chunk ? wd[c] : (double)b.Wn[e];
          wo[c] = (float)(v / l1d);
          b.Wn[e] = wo[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < RP; ++c) sWn[tid][c] = wo[c];
    __syncthreads();
    const int nst = min(16, (m - i0 - 64 * wv + 3) / 4);  // steps holding rows < m
    for (int st4 = 0; st4 < nst; ++st4) {
      const int row = 64 * wv + 4 * st4 + lb;
      double op[NT];
#pragma unroll
      for (int h = 0; h < NT; ++h) {
        const int c = 16 * h + la;
        op[h] = c < RP ? (double)sWn[row][c < RP ? c : 0] : 0.0;
      }
#pragma unroll
      for (int h = 0; h < NT; ++h)
#pragma unroll
        for (int q = 0; q < NT; ++q) gm[h][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[h], op[q], gm[h][q], 0, 0, 0);
    }
    __syncthreads();
  }
  // the four waves' sums, added in wave order (sWn is free now)
  double* sGp = reinterpret_cast<double*>(&sWn[0][0]);  // [4][NT * NT][64][4]
#pragma unroll
  for (int h = 0; h < NT; ++h)
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) sGp[(((size_t)wv * NT * NT + h * NT + q) * 64 + ln) * 4 + i] = gm[h][q][i];
  __syncthreads();
  double gg = 0.0;
  for (int e = tid; e < RP * RP; e += 256) {
    const int c = e / RP, q = e % RP;
    const int h = c / 16, i = (c % 16) / 4, lane = (c % 4) * 16 + q % 16, qq = q / 16;
    double v = 0.0;
    for (int w4 = 0; w4 < 4; ++w4) v += sGp[(((size_t)w4 * NT * NT + h * NT + qq) * 64 + lane) * 4 + i];
    b.GWn[c * 32 + q] = (float)v;
    gg += v * v;
  }
  gg = bcd_wave_sum(gg);
  if (ln == 0) sPart[2][wv] = gg;
  __syncthreads();
  if (tid == 0) st->gWn = std::sqrt(((sPart[2][0] + sPart[2][1]) + sPart[2][2]) + sPart[2][3]);
}

// The H step, CPT adjacent columns per thread (vector loads and stores; k % CPT == 0 and
// 4 CPT-byte aligned rows): H_m from the kept H (and, with extrapolation, the kept H
// before it), W_n^T X with W_n streamed through LDS in 64-row chunks, then
// H_n = max(0, H_m - (G H_m - W_n^T X) / ||G||_F) into Hb[nxt].
template <int N> struct BVec { typedef float __attribute__((ext_vector_type(N))) T; };
template <> struct BVec<1> { typedef float T; };

template <int N>
__device__ __forceinline__ float bget(const typename BVec<N>::T& v, int u) {
  if constexpr (N == 1) return v;
  else return v[u];
}

template <int N>
__device__ __forceinline__ void bset(typename BVec<N>::T& v, int u, float x) {
  if constexpr (N == 1) v = x;
  else v[u] = x;
}

template <int RP, int CPT>
__global__ __launch_bounds__(256) void k_bcd_h(BcdArgs b) {
  typedef typename BVec<CPT>::T VT;
  __shared__ float sW[64][RP + 1];
  __shared__ float sG[RP][RP + 1];
  const int tid = threadIdx.x;
  const int m = b.m, r = b.r;
  const int64_t k = b.k;
  const BcdState* st = b.st;
  const float* __restrict__ Hc = b.Hb[st->cur];
  const float* __restrict__ Hp = b.Hb[st->prev];
  float* __restrict__ Hn = b.Hb[st->nxt];
  const float wH = (float)st->wH;
  const double LH = st->gWn;
  const float Lf = (float)LH;
  const int64_t j = ((int64_t)blockIdx.x * 256 + tid) * CPT;
  const bool act = j < k;
  const int64_t jc = act ? j : k - CPT;
  float hm[CPT][RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) {
    const int64_t e = (int64_t)min(c, r - 1) * k + jc;
    const bool ok = act && c < r;
    const VT hc = *reinterpret_cast<const VT*>(Hc + e);
    if (wH != 0.f) {
      const VT hp = *reinterpret_cast<const VT*>(Hp + e);
#pragma unroll
      for (int u = 0; u < CPT; ++u)
        hm[u][c] = bmask(fmaf(wH, bget<CPT>(hc, u) - bget<CPT>(hp, u), bget<CPT>(hc, u)), ok);
    } else {
#pragma unroll
      for (int u = 0; u < CPT; ++u) hm[u][c] = bmask(bget<CPT>(hc, u), ok);
    }
  }
  for (int e = tid; e < RP * RP; e += 256) sG[e / RP][e % RP] = b.GWn[(e / RP) * 32 + e % RP];
  float acc[CPT][RP];
#pragma unroll
  for (int u = 0; u < CPT; ++u)
#pragma unroll
    for (int c = 0; c < RP; ++c) acc[u][c] = 0.f;
  for (int i0 = 0; i0 < m; i0 += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * RP; e += 256) {
      const int i = e / RP, c = e % RP;
      sW[i][c] = bmask(b.Wn[(int64_t)min(i0 + i, m - 1) * r + min(c, r - 1)], i0 + i < m && c < r);
    }
    __syncthreads();
    const int iend = min(64, m - i0);
#pragma unroll 8
    for (int i = 0; i < iend; ++i) {
      const VT x = *reinterpret_cast<const VT*>(b.X + (int64_t)(i0 + i) * k + jc);
#pragma unroll
      for (int u = 0; u < CPT; ++u)
#pragma unroll
        for (int c = 0; c < RP; ++c) acc[u][c] = fmaf(sW[i][c], bget<CPT>(x, u), acc[u][c]);
    }
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      if (c < r) {
        VT out;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
          float gr = -acc[u][c];
#pragma unroll
          for (int q = 0; q < RP; ++q) gr = fmaf(sG[c][q], hm[u][q], gr);
          const float v = LH > 0.0 ? hm[u][c] - gr / Lf : hm[u][c];
          bset<CPT>(out, u, fmaxf(0.f, v));
        }
        *reinterpret_cast<VT*>(Hn + (int64_t)c * k + j) = out;
      }
    }
  }
}

// The H step with the rows of W_n^T X split over RG thread groups (short unfoldings, where
// one thread per column gives too few workgroups): a workgroup takes CT = 256 / RG
// columns; thread (g, col) sums rows i = g, g + RG, ... of each chunk of W_n (256 rows at
// RG = 16, so one round of loads for m <= 256; 64 rows at RG = 4, where 16 loads per
// thread in flight already cover the latency); the RG partial sums are added in order in
// LDS and CT threads apply the step to their column.
template <int RP, int RG>
__global__ __launch_bounds__(256) void k_bcd_hs(BcdArgs b) {
  constexpr int CT = 256 / RG;
  constexpr int CH = RG >= 16 ? 256 : 64;  // rows of W_n per chunk (measured best)
  __shared__ float sW[CH][RP + 1];
  __shared__ float sG[RP][RP + 1];
  __shared__ float sAcc[RG][CT][RP + 1];
  const int tid = threadIdx.x;
  const int m = b.m, r = b.r;
  const int64_t k = b.k;
  const BcdState* st = b.st;
  const int grp = tid / CT, col = tid % CT;
  const int64_t j = (int64_t)blockIdx.x * CT + col;
  const bool act = j < k;
  const int64_t jc = act ? j : k - 1;
  for (int e = tid; e < RP * RP; e += 256) sG[e / RP][e % RP] = b.GWn[(e / RP) * 32 + e % RP];
  float acc[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) acc[c] = 0.f;
  for (int i0 = 0; i0 < m; i0 += CH) {
    // the chunk's X loads go out first, unconditionally: rows past m are clamped and
    // meet zero rows of sW
    constexpr int NU = CH / RG;
    float xs[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) xs[u] = b.X[(int64_t)min(i0 + grp + u * RG, m - 1) * k + jc];
    __syncthreads();
    for (int e = tid; e < CH * RP; e += 256) {
      const int i = e / RP, c = e % RP;
      sW[i][c] = bmask(b.Wn[(int64_t)min(i0 + i, m - 1) * r + min(c, r - 1)], i0 + i < m && c < r);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const float x = act ? xs[u] : 0.f;
#pragma unroll
      for (int c = 0; c < RP; ++c) acc[c] = fmaf(sW[grp + u * RG][c], x, acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < RP; ++c) sAcc[grp][col][c] = acc[c];
  __syncthreads();
  if (tid < CT && act) {
    const float* __restrict__ Hc = b.Hb[st->cur];
    const float* __restrict__ Hp = b.Hb[st->prev];
    float* __restrict__ Hn = b.Hb[st->nxt];
    const float wH = (float)st->wH;
    const double LH = st->gWn;
    const float Lf = (float)LH;
    float hm[RP], wx[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      float a = 0.f;
      for (int g2 = 0; g2 < RG; ++g2) a += sAcc[g2][tid][c];
      wx[c] = a;
      const int64_t e = (int64_t)min(c, r - 1) * k + j;
      const float hc = Hc[e];
      hm[c] = c < r ? (wH != 0.f ? fmaf(wH, hc - Hp[e], hc) : hc) : 0.f;
    }
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      if (c < r) {
        float gr = -wx[c];
#pragma unroll
        for (int q = 0; q < RP; ++q) gr = fmaf(sG[c][q], hm[q], gr);
        const float v = LH > 0.0 ? hm[c] - gr / Lf : hm[c];
        Hn[(int64_t)c * k + j] = fmaxf(0.f, v);
      }
    }
  }
}

// The kept H into Hb[0] (nothing to do when it is there already).
__global__ void k_bcd_commit(BcdArgs b) {
  const int cur = b.st->cur;
  if (cur == 0) return;
  const float* __restrict__ src = b.Hb[cur];
  float* __restrict__ dst = b.Hb[0];
  const int64_t n = (int64_t)b.r * b.k;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

#define NTT_BCD_CHECK()                \
  do {                                 \
    hipError_t e_ = hipGetLastError(); \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

int bcd_rp(int r) { return r <= 8 ? 8 : (r <= 16 ? 16 : 32); }

bool aligned(const void* p, int bytes) { return (reinterpret_cast<uintptr_t>(p) % bytes) == 0; }

template <int RP>
hipError_t bcd_xht(const BcdArgs& b, bool resid, hipStream_t s) {
  const dim3 grid((unsigned)b.G, (unsigned)((b.m + 63) / 64));
  const bool xv = b.k % 4 == 0 && aligned(b.X, 16);
  if (xv) {  // MFMA products; tiles of 64, 32 or 16 rows (grid.y is 1 below 64 rows)
    if (b.m > 32) {
      if (resid) k_bcd_xhtm<RP, true, 64><<<grid, 256, 0, s>>>(b, 0);
      else k_bcd_xhtm<RP, false, 64><<<grid, 256, 0, s>>>(b, 1);
    } else if (b.m > 16) {
      if (resid) k_bcd_xhtm<RP, true, 32><<<grid, 256, 0, s>>>(b, 0);
      else k_bcd_xhtm<RP, false, 32><<<grid, 256, 0, s>>>(b, 1);
    } else {
      if (resid) k_bcd_xhtm<RP, true, 16><<<grid, 256, 0, s>>>(b, 0);
      else k_bcd_xhtm<RP, false, 16><<<grid, 256, 0, s>>>(b, 1);
    }
    NTT_BCD_CHECK();
    return hipSuccess;
  }
  if (resid) {
    if (xv) k_bcd_xht<RP, true, true><<<grid, 256, 0, s>>>(b, 0);
    else k_bcd_xht<RP, true, false><<<grid, 256, 0, s>>>(b, 0);
  } else {
    if (xv) k_bcd_xht<RP, false, true><<<grid, 256, 0, s>>>(b, 1);
    else k_bcd_xht<RP, false, false><<<grid, 256, 0, s>>>(b, 1);
  }
  NTT_BCD_CHECK();
  return hipSuccess;
}

// columns per thread of the H step: 4 at r <= 8, 2 at r <= 16, else 1, when the rows
// allow vector access
int bcd_cpt(const BcdArgs& b) {
  int c = b.r <= 8 ? 4 : (b.r <= 16 ? 2 : 1);
  while (c > 1 && !(b.k % c == 0 && aligned(b.X, 4 * c) && aligned(b.Hb[0], 4 * c) &&
                    aligned(b.Hb[1], 4 * c) && aligned(b.Hb[2], 4 * c)))
    c >>= 1;
  return c;
}

template <int RP, int CPT>
hipError_t bcd_h(const BcdArgs& b, hipStream_t s) {
  const int64_t nb = (b.k + 256 * CPT - 1) / (256 * CPT);
  k_bcd_h<RP, CPT><<<(unsigned)nb, 256, 0, s>>>(b);
  NTT_BCD_CHECK();
  return hipSuccess;
}

template <int RP, int RG>
hipError_t bcd_hs(const BcdArgs& b, hipStream_t s) {
  const int64_t nb = (b.k + 256 / RG - 1) / (256 / RG);
  k_bcd_hs<RP, RG><<<(unsigned)nb, 256, 0, s>>>(b);
  NTT_BCD_CHECK();
  return hipSuccess;
}

hipError_t bcd_h_any(const BcdArgs& b, hipStream_t s) {
  const int cpt = bcd_cpt(b);
  // short unfoldings: rows split over 4 (64 columns per workgroup) or 16 thread groups
  if ((b.k + 256 * cpt - 1) / (256 * cpt) < 512) {
    const bool rg4 = (b.k + 63) / 64 >= 256;
    switch (bcd_rp(b.r)) {
      case 8: return rg4 ? bcd_hs<8, 4>(b, s) : bcd_hs<8, 16>(b, s);
      case 16: return rg4 ? bcd_hs<16, 4>(b, s) : bcd_hs<16, 16>(b, s);
      default: return rg4 ? bcd_hs<32, 4>(b, s) : bcd_hs<32, 16>(b, s);
    }
  }
  switch (bcd_rp(b.r)) {
    case 8:
      return cpt == 4 ? bcd_h<8, 4>(b, s) : (cpt == 2 ? bcd_h<8, 2>(b, s) : bcd_h<8, 1>(b, s));
    case 16: return cpt == 2 ? bcd_h<16, 2>(b, s) : bcd_h<16, 1>(b, s);
    default: return bcd_h<32, 1>(b, s);
  }
}

hipError_t bcd_xht_any(const BcdArgs& b, bool resid, hipStream_t s) {
  switch (bcd_rp(b.r)) {
    case 8: return bcd_xht<8>(b, resid, s);
    case 16: return bcd_xht<16>(b, resid, s);
    default: return bcd_xht<32>(b, resid, s);
  }
}

hipError_t bcd_step(const BcdArgs& b, int final_step, hipStream_t s) {
  switch (bcd_rp(b.r)) {
    case 8: k_bcd_step<8><<<1, 256, 0, s>>>(b, final_step); break;
    case 16: k_bcd_step<16><<<1, 256, 0, s>>>(b, final_step); break;
    default: k_bcd_step<32><<<1, 256, 0, s>>>(b, final_step); break;
  }
  NTT_BCD_CHECK();
  return hipSuccess;
}

hipError_t bcd_reduce(const BcdArgs& b, hipStream_t s) {
  FinArgs f{};
  f.part = b.part;
  f.part_stride = b.part_stride;
  f.G = b.G;
  f.m = b.m;
  f.r = b.r;
  f.red = b.red;
  return launch_reduce(f, s);
}

bool bcd_args_ok(const BcdArgs& b) {
  return b.m >= 1 && b.r >= 1 && b.r <= 32 && b.k >= 1 && b.G >= 1 && b.G <= 1024 &&
         b.chunk >= 64 && b.chunk % 64 == 0 && (int64_t)b.G * b.chunk >= b.k &&
         b.part_stride >= (int64_t)b.m * b.r + (int64_t)b.r * b.r;
}

}  // namespace

hipError_t launch_bcd_prepare(const BcdArgs& b, hipStream_t s) {
  if (!bcd_args_ok(b)) return hipErrorInvalidValue;
  const int64_t mr = (int64_t)b.m * b.r, rk = (int64_t)b.r * b.k;
  hipError_t e = launch_sumsq(b.W, mr, b.rpart, 1024, nullptr, 0, b.scal + SCAL_BCD_W2, s);
  if (e != hipSuccess) return e;
  e = launch_sumsq(b.Hb[0], rk, b.rpart, 1024, nullptr, 0, b.scal + SCAL_BCD_H2, s);
  if (e != hipSuccess) return e;
  k_bcd_scale<<<(unsigned)std::min<int64_t>((mr + 255) / 256, 4096), 256, 0, s>>>(
      b.W, mr, b.scal + SCAL_NX2, b.scal + SCAL_BCD_W2);
  NTT_BCD_CHECK();
  k_bcd_scale<<<(unsigned)std::min<int64_t>((rk + 255) / 256, 8192), 256, 0, s>>>(
      b.Hb[0], rk, b.scal + SCAL_NX2, b.scal + SCAL_BCD_H2);
  NTT_BCD_CHECK();
  e = launch_copy(b.Wp, b.W, mr, s);
  if (e != hipSuccess) return e;
  k_bcd_state_init<<<1, 64, 0, s>>>(b.st, b.scal);
  NTT_BCD_CHECK();
  e = bcd_xht_any(b, false, s);
  if (e != hipSuccess) return e;
  return bcd_reduce(b, s);
}

hipError_t launch_bcd_iter(const BcdArgs& b, hipStream_t s) {
  if (!bcd_args_ok(b)) return hipErrorInvalidValue;
  hipError_t e = bcd_step(b, 0, s);
  if (e != hipSuccess) return e;
  e = bcd_h_any(b, s);
  if (e != hipSuccess) return e;
  e = bcd_xht_any(b, true, s);
  if (e != hipSuccess) return e;
  return bcd_reduce(b, s);
}

hipError_t launch_bcd_finish(const BcdArgs& b, hipStream_t s) {
  if (!bcd_args_ok(b)) return hipErrorInvalidValue;
  hipError_t e = bcd_step(b, 1, s);
  if (e != hipSuccess) return e;
  const int64_t rk = (int64_t)b.r * b.k;
  k_bcd_commit<<<(unsigned)std::min<int64_t>((rk + 255) / 256, 8192), 256, 0, s>>>(b);
  NTT_BCD_CHECK();
  return hipSuccess;
}

}  // namespace ntt
