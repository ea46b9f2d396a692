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
//                data, and G = W_n^T W_n (FP64, rows in order).
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
// [r][r] (H H^T by the rb = 0 blocks).
template <int RP, bool RESID>
__global__ __launch_bounds__(256) void k_bcd_xht(BcdArgs b, int init) {
  __shared__ float sX[64][65];
  __shared__ float sH[RP][65];
  __shared__ double sRes[4];
  const int tid = threadIdx.x;
  const int m = b.m, r = b.r;
  const int64_t k = b.k;
  const float* __restrict__ H = init ? b.Hb[0] : b.Hb[b.st->nxt];
  const int g = blockIdx.x, rb = blockIdx.y;
  const int64_t c0 = (int64_t)g * b.chunk, c1 = min(k, c0 + b.chunk);
  const int row = tid >> 2, qd = tid & 3;
  const int gi = 64 * rb + row;
  float acc[RP];
  float w[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) {
    acc[c] = 0.f;
    w[c] = RESID ? bmask(b.Wn[(int64_t)min(gi, m - 1) * r + min(c, r - 1)], gi < m && c < r) : 0.f;
  }
  constexpr int NG = RP * RP / 256 > 0 ? RP * RP / 256 : 1;
  float accg[NG];
#pragma unroll
  for (int t = 0; t < NG; ++t) accg[t] = 0.f;
  double res = 0.0;
  for (int64_t j0 = c0; j0 < c1; j0 += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
      const int i = e >> 6, jj = e & 63;
      const int xi = 64 * rb + i;
      const int64_t gj = j0 + jj;
      sX[i][jj] = bmask(b.X[(int64_t)min(xi, m - 1) * k + min(gj, c1 - 1)], xi < m && gj < c1);
    }
    for (int e = tid; e < RP * 64; e += 256) {
      const int c = e >> 6, jj = e & 63;
      const int64_t gj = j0 + jj;
      sH[c][jj] = bmask(H[(int64_t)min(c, r - 1) * k + min(gj, c1 - 1)], c < r && gj < c1);
    }
    __syncthreads();
#pragma unroll 1
    for (int jj = qd * 16; jj < qd * 16 + 16; ++jj) {
      const float x = sX[row][jj];
      float wh = 0.f;
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        acc[c] = fmaf(x, sH[c][jj], acc[c]);
        if (RESID) wh = fmaf(w[c], sH[c][jj], wh);
      }
      if (RESID) {
        const double dl = (double)x - (double)wh;  // 0 outside the matrix
        res += dl * dl;
      }
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
  // the four column quarters of each row, added in order
  __syncthreads();
  float* red = &sX[0][0];
  float* dst = b.part + (int64_t)g * b.part_stride;
  for (int c = 0; c < RP; ++c) {
    __syncthreads();
    red[tid] = acc[c];
    __syncthreads();
    if (qd == 0) {
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
  if (RESID) {
    res = bcd_wave_sum(res);
    if ((tid & 63) == 0) sRes[tid >> 6] = res;
    __syncthreads();
    if (tid == 0) b.rpart[(int64_t)g * gridDim.y + rb] = ((sRes[0] + sRes[1]) + sRes[2]) + sRes[3];
  }
}

// The decision on the previous candidate (unless this is the stage's first step), then,
// unless `final_step`, the W step and G = W_n^T W_n.  One workgroup; thread tid owns rows
// tid, tid + 256, ... in every phase, so it only re-reads global data it wrote itself.
template <int RP>
__global__ __launch_bounds__(256) void k_bcd_step(BcdArgs b, int final_step) {
  __shared__ float sWn[256][RP + 1];
  __shared__ double sHH[RP][RP + 1];
  __shared__ double sRed[256];
  __shared__ double sPar[3];  // w_W, w_H, ||H H^T||_F of the kept H
  __shared__ int sMode;       // 0: candidate dropped, 1: kept, 2: first step
  const int tid = threadIdx.x;
  const int m = b.m, r = b.r;
  const int64_t mr = (int64_t)m * r;
  BcdState* st = b.st;
  const int first = st->first;
  __syncthreads();  // every wave has read the state before thread 0 rewrites it
  if (first) {
    if (tid == 0) {
      double g2 = 0.0;
      for (int e = 0; e < r * r; ++e) g2 += b.red[mr + e] * b.red[mr + e];
      BcdState s = *st;
      s.first = 0;
      s.gH = std::sqrt(g2);
      s.wW = s.wH = 0.0;
      *st = s;
      sMode = 2;
      sPar[0] = 0.0;
      sPar[1] = 0.0;
      sPar[2] = s.gH;
    }
  } else {
    double a = 0.0;
    for (int i = tid; i < b.G * ((m + 63) / 64); i += 256) a += b.rpart[i];
    sRed[tid] = a;
    __syncthreads();
    if (tid == 0) {
      double f = 0.0;
      for (int i = 0; i < 256; ++i) f += sRed[i];
      f *= 0.5;
      if (b.trace) b.trace[0] = f;
      BcdState s = *st;
      if (f < s.obj) {
        const double tp = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * s.t * s.t));
        const double w = (s.t - 1.0) / tp;
        double g2 = 0.0;
        for (int e = 0; e < r * r; ++e) g2 += b.red[mr + e] * b.red[mr + e];
        const double gHn = std::sqrt(g2), gWn = s.gWn;
        s.wW = gHn > 0.0 ? std::min(w, b.delta * std::sqrt(s.gH / gHn)) : w;
        s.wH = gWn > 0.0 ? std::min(w, b.delta * std::sqrt(s.gW / gWn)) : w;
        s.gH = gHn;
        s.gW = gWn;
        s.t = tp;
        s.obj = f;
        const int old_prev = s.prev;
        s.prev = s.cur;
        s.cur = s.nxt;
        s.nxt = old_prev;
        sMode = 1;
      } else {
        s.wW = s.wH = 0.0;
        s.corrections += 1;
        sMode = 0;
      }
      *st = s;
      sPar[0] = s.wW;
      sPar[1] = s.wH;
      sPar[2] = s.gH;
    }
  }
  __syncthreads();
  const int mode = sMode;
  const double wW = sPar[0], LW = sPar[2];
  // H H^T of the kept H into LDS (and into HHc when it changed)
  for (int e = tid; e < RP * RP; e += 256) {
    const int c = e / RP, q = e % RP;
    double v = 0.0;
    if (c < r && q < r) {
      v = mode ? b.red[mr + c * r + q] : b.HHc[c * r + q];
      if (mode) b.HHc[c * r + q] = v;
    }
    sHH[c][q] = v;
  }
  if (final_step) {
    for (int64_t e = tid; e < mr; e += 256)
      if (mode == 1) {
        b.Wp[e] = b.W[e];
        b.W[e] = b.Wn[e];
        b.XHc[e] = b.red[e];
      }
    if (tid == 0) {
      b.scal[SCAL_BCD_CORR] = (double)st->corrections;
      b.scal[SCAL_BCD_OBJ] = st->obj;
    }
    return;
  }
  __syncthreads();
  constexpr int NG = (RP * RP + 255) / 256;
  double gacc[NG];
#pragma unroll
  for (int t = 0; t < NG; ++t) gacc[t] = 0.0;
  for (int i0 = 0; i0 < m; i0 += 256) {
    const int i = i0 + tid;
    float wn[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) wn[c] = 0.f;
    if (i < m) {
      double wm[RP], xh[RP];
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        wm[c] = 0.0;
        xh[c] = 0.0;
        if (c < r) {
          const int64_t e = (int64_t)i * r + c;
          double wc, wp;
          if (mode == 1) {
            wp = b.W[e];
            wc = b.Wn[e];
            b.Wp[e] = (float)wp;
            b.W[e] = (float)wc;
            xh[c] = b.red[e];
            b.XHc[e] = xh[c];
          } else {
            wc = b.W[e];
            wp = wW != 0.0 ? (double)b.Wp[e] : wc;
            xh[c] = mode == 2 ? b.red[e] : b.XHc[e];
            if (mode == 2) b.XHc[e] = xh[c];
          }
          wm[c] = wW != 0.0 ? wc + wW * (wc - wp) : wc;
        }
      }
#pragma unroll
      for (int c = 0; c < RP; ++c) {
        if (c < r) {
          double gr = -xh[c];
#pragma unroll
          for (int q = 0; q < RP; ++q) gr += wm[q] * sHH[q][c];
          const double v = LW > 0.0 ? wm[c] - gr / LW : wm[c];
          wn[c] = (float)std::max(0.0, v);
          b.Wn[(int64_t)i * r + c] = wn[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < RP; ++c) sWn[tid][c] = wn[c];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NG; ++t) {
      const int pidx = tid + 256 * t;
      if (pidx < RP * RP) {
        const int c = pidx / RP, q = pidx % RP;
        double s = gacc[t];
        const int rows = min(256, m - i0);
        for (int j = 0; j < rows; ++j) s += (double)sWn[j][c] * (double)sWn[j][q];
        gacc[t] = s;
      }
    }
    __syncthreads();
  }
  double g2 = 0.0;
#pragma unroll
  for (int t = 0; t < NG; ++t) {
    const int pidx = tid + 256 * t;
    if (pidx < RP * RP) {
      const int c = pidx / RP, q = pidx % RP;
      b.GWn[c * 32 + q] = (float)gacc[t];
      g2 += gacc[t] * gacc[t];
    }
  }
  sRed[tid] = g2;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += sRed[i];
    st->gWn = std::sqrt(s);
  }
}

// The H step, one thread per column: H_m from the kept H (and, with extrapolation, the
// kept H before it), W_n^T X with W_n streamed through LDS in 64-row chunks, then
// H_n = max(0, H_m - (G H_m - W_n^T X) / ||G||_F) into Hb[nxt].
template <int RP>
__global__ __launch_bounds__(256) void k_bcd_h(BcdArgs b) {
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
  const int64_t j = (int64_t)blockIdx.x * 256 + tid;
  const bool act = j < k;
  const int64_t jc = act ? j : k - 1;
  float hm[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) {
    const int64_t e = (int64_t)min(c, r - 1) * k + jc;
    const float hc = bmask(Hc[e], act && c < r);
    if (wH != 0.f) {
      const float hp = bmask(Hp[e], act && c < r);
      hm[c] = fmaf(wH, hc - hp, hc);
    } else {
      hm[c] = hc;
    }
  }
  for (int e = tid; e < RP * RP; e += 256) sG[e / RP][e % RP] = b.GWn[(e / RP) * 32 + e % RP];
  float acc[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) acc[c] = 0.f;
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
      const float x = bmask(b.X[(int64_t)(i0 + i) * k + jc], act);
#pragma unroll
      for (int c = 0; c < RP; ++c) acc[c] = fmaf(sW[i][c], x, acc[c]);
    }
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < RP; ++c) {
      if (c < r) {
        float gr = -acc[c];
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

template <int RP>
hipError_t bcd_xht(const BcdArgs& b, bool resid, hipStream_t s) {
  const dim3 grid((unsigned)b.G, (unsigned)((b.m + 63) / 64));
  if (resid) k_bcd_xht<RP, true><<<grid, 256, 0, s>>>(b, 0);
  else k_bcd_xht<RP, false><<<grid, 256, 0, s>>>(b, 1);
  NTT_BCD_CHECK();
  return hipSuccess;
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
  const int64_t nb = (b.k + 255) / 256;
  switch (bcd_rp(b.r)) {
    case 8: k_bcd_h<8><<<(unsigned)nb, 256, 0, s>>>(b); break;
    case 16: k_bcd_h<16><<<(unsigned)nb, 256, 0, s>>>(b); break;
    default: k_bcd_h<32><<<(unsigned)nb, 256, 0, s>>>(b); break;
  }
  NTT_BCD_CHECK();
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
