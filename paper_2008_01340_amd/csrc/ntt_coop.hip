// ntt_coop.hip -- a whole MU stage in one grid-synchronised launch, for unfoldings of at most
// 256 rows at rank <= 16 whose columns fit the registers of the GPU's workgroups
// (k <= 256 x 128).  It runs the same iteration as the pass + reduction + W-update
// launches (paper: the MU update the experiments time; W^T X, W^T W, X H^T, H H^T of
// Alg.4-6 on one GPU), but keeps X, H and W on chip for all iterations:
//
//   * workgroup g owns CW = 16 NG columns of X: its X columns stay in registers for the
//     whole launch (both MFMA operand layouts), its H columns in LDS; every workgroup
//     holds the whole W (LDS) and W^T W;
//   * per iteration (A) the H-update of the workgroup's columns and its X H_new^T,
//     H_new H_new^T partials; (B) after a grid barrier, workgroup g adds entries
//     [g E/G, (g+1) E/G) of the E = m r + r r partial entries over all G workgroups in a
//     fixed order (FP64); (C) after a second barrier, every workgroup reads all sums and
//     applies the W-update to all m rows and forms the next W^T W itself (the same code
//     and inputs in every workgroup, so every copy of W holds the same bits).
//
// Data crossing workgroups (partials, sums, barrier flags) is written and read with
// device-scope relaxed atomic accesses, which go past the non-coherent caches of the
// XCDs; each wave waits for its stores to complete before the workgroup raises its
// flag.  The barrier is a flag per workgroup (its own 128-byte line) holding the last
// epoch it reached; waiting means reading all flags.  A bounded wait: a barrier that is
// not reached in about a quarter of a second sets `status` and every workgroup leaves.
//
// The barrier needs every workgroup of the grid resident at once.  The launch checks the
// grid against the device's occupancy for the kernel (workgroups per CU x CUs) and uses
// an ordinary launch rather than the cooperative-launch API, whose only service here
// would be that same guarantee: measured on MI355X, after one cooperative launch the
// process's later multi-stream work ran about 40% slower (256 batched problems on four
// streams: 3.24 s before, 4.5 s after), and the next sweep's first stage 2.5% slower.
// With an ordinary launch a workgroup that is not yet resident (another stream's kernel
// holding CUs) only delays the barrier; it fails with `status` set if that lasts past the
// bounded wait, and NTT_NO_COOP then selects the per-pass launches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntt_device.h"
#include "ntt_internal.h"

namespace ntt {
namespace {

constexpr int kCoopWaves = 8;           // 512 threads, wave w owns rows 32 w .. 32 w + 31
constexpr long kCoopMaxPolls = 1L << 18;

// Grid barrier at `epoch` (1, 2, ...): false when it timed out (then every thread of the
// workgroup returns false and the caller leaves).
__device__ __forceinline__ bool coop_barrier(const CoopArgs& c, unsigned epoch, int* sAbort) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's global stores have completed
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid == 0) __hip_atomic_store(c.flags + 32 * blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (tid < (int)gridDim.x) {
    long polls = 0;
    while (__hip_atomic_load(c.flags + 32 * tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      if (++polls > kCoopMaxPolls) {
        *sAbort = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  return *sAbort == 0;
}

template <int NG>
__global__ __launch_bounds__(64 * kCoopWaves) void k_stage_coop(CoopArgs c) {
  constexpr int NW = kCoopWaves, MBW = 2, RB = 16, CW = 16 * NG;
  static_assert(NG <= NW, "one wave per 16-column group in the epilogue");
  // phase A: the waves' parts of W^T X of every group; phase C: the sums of X H^T by row
  constexpr int kBig = NG * NW * 256 * 4 > 256 * (RB + 1) * 8 ? NG * NW * 256 * 4 : 256 * (RB + 1) * 8;
  __shared__ __attribute__((aligned(16))) char sBig[kBig];
  __shared__ __attribute__((aligned(16))) float sH[16][CW + 4];    // H columns of this workgroup
  __shared__ float sWc[256][RB + 1];                               // W, zero padded
  __shared__ double sGH[RB][RB + 1];
  __shared__ double sGp[NW][64][4];
  __shared__ double sAcc[64 * NW];
  __shared__ float sGW[16][17];
  __shared__ int sAbort;
  float (*sNH)[NW][256] = reinterpret_cast<float (*)[NW][256]>(sBig);
  double (*sN)[RB + 1] = reinterpret_cast<double (*)[RB + 1]>(sBig);

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int a = lane & 15, b = lane >> 4;
  const int m = c.m, r = c.r, G = gridDim.x;
  const int64_t k = c.k;
  const int64_t col0 = (int64_t)blockIdx.x * CW;
  const int row0 = 32 * w;
  const int E = m * r + r * r;
  if (tid == 0) sAbort = 0;

  // X columns in both operand layouts, loaded once:
  //   xt[g][blk][q] = X[row0 + 16 blk + 4b + q][col0 + 16g + a]  (B of W^T X, K = rows)
  //   xa[g][blk][q] = X[row0 + 16 blk + a][col0 + 16g + 4b + q]  (A of X H^T, K = columns)
  float xt[NG][MBW][4], xa[NG][MBW][4];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i1 = row0 + 16 * blk + 4 * b + q;
        const int64_t j1 = col0 + 16 * g + a;
        xt[g][blk][q] = zmask(c.X[(int64_t)min(i1, m - 1) * k + min(j1, k - 1)], i1 < m && j1 < k);
        const int i2 = row0 + 16 * blk + a;
        const int64_t j2 = col0 + 16 * g + 4 * b + q;
        xa[g][blk][q] = zmask(c.X[(int64_t)min(i2, m - 1) * k + min(j2, k - 1)], i2 < m && j2 < k);
      }
  for (int e = tid; e < 16 * (CW + 4); e += 64 * NW) {
    const int cc = e / (CW + 4), j = e % (CW + 4);
    const int64_t col = col0 + j;
    sH[cc][j] = zmask(c.H[(int64_t)min(cc, r - 1) * k + min(col, k - 1)], cc < r && j < CW && col < k);
  }
  for (int e = tid; e < 256 * RB; e += 64 * NW) {
    const int i = e / RB, cc = e % RB;
    sWc[i][cc] = zmask(c.W[(int64_t)min(i, m - 1) * r + min(cc, r - 1)], i < m && cc < r);
  }
  if (tid < 256) sGW[tid / 16][tid % 16] = c.GW[tid];
  __syncthreads();

  unsigned epoch = 0;
  for (int it = 0; it < c.iters; ++it) {
    // ---- (A1) every wave's rows' part of W^T X for every group of this workgroup
    {
      float wa[MBW][4];
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
        for (int q = 0; q < 4; ++q) wa[blk][q] = sWc[row0 + 16 * blk + 4 * b + q][a];
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        v4f nh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
          for (int q = 0; q < 4; ++q) nh = mfma16(wa[blk][q], xt[g][blk][q], nh);
#pragma unroll
        for (int i = 0; i < 4; ++i) sNH[g][w][(4 * b + i) * 16 + a] = nh[i];
      }
    }
    __syncthreads();
    // ---- (A2) wave g < NG: group g's sum over the waves (in wave order), D_H = G_W H and
    // the epilogue H_new = max(0, H .* N_H ./ (D_H + eps)) into sH
    if (w < NG) {
      const int g = w;
      float gw[4], hv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        gw[q] = sGW[a][4 * b + q];
        hv[q] = sH[4 * b + q][16 * g + a];
      }
      v4f nh;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = (4 * b + i) * 16 + a;
        float sum = sNH[g][0][e];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww) sum += sNH[g][ww][e];
        nh[i] = sum;
      }
      v4f dh = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) dh = mfma16(gw[q], hv[q], dh);
      const bool colok = col0 + 16 * g + a < k;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float q = fmaxf(0.f, fast_div(hv[i] * nh[i], dh[i] + c.eps));
        sH[4 * b + i][16 * g + a] = (4 * b + i < r && colok) ? q : 0.f;
      }
    }
    __syncthreads();
    // ---- (A3) X H_new^T for every wave's rows and (wave 0) H_new H_new^T, over all groups;
    // the B operand H_new[a][16g + 4b + q] is read straight from sH
    v4f accW[MBW], accG = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk) accW[blk] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const float4 hn4 = *reinterpret_cast<const float4*>(&sH[a][16 * g + 4 * b]);
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk) {
        accW[blk] = mfma16(xa[g][blk][0], hn4.x, accW[blk]);
        accW[blk] = mfma16(xa[g][blk][1], hn4.y, accW[blk]);
        accW[blk] = mfma16(xa[g][blk][2], hn4.z, accW[blk]);
        accW[blk] = mfma16(xa[g][blk][3], hn4.w, accW[blk]);
      }
      if (w == 0) {
        accG = mfma16(hn4.x, hn4.x, accG);
        accG = mfma16(hn4.y, hn4.y, accG);
        accG = mfma16(hn4.z, hn4.z, accG);
        accG = mfma16(hn4.w, hn4.w, accG);
      }
    }
    // partials of this workgroup: [m][r] X H^T (each wave its rows), [r][r] H H^T
    float* dst = c.part + (int64_t)blockIdx.x * E;
#pragma unroll
    for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row0 + 16 * blk + 4 * b + i;
        if (row < m && a < r) st_dev(dst + row * r + a, accW[blk][i]);
      }
    if (w == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int cc = 4 * b + i;
        if (cc < r && a < r) st_dev(dst + m * r + cc * r + a, accG[i]);
      }
    }
    if (!coop_barrier(c, ++epoch, &sAbort)) break;

    // ---- (B) entries [e0, e0 + ne) summed over the G partials.  With few entries per
    // thread, S threads per entry: thread (s, e) adds partials s, s + S, ... in order,
    // then the S sums are added in order; else (S = 1) each thread adds all G partials of
    // entries e, e + 512, ... in order
    {
      const int chunk = (E + G - 1) / G;
      const int e0 = blockIdx.x * chunk;
      const int ne = max(0, min(chunk, E - e0));
      int S = 1;
      while (2 * S <= G && 2 * S * ne <= 64 * NW) S *= 2;
      // partials are read eight at a time from clamped addresses (masked after the load)
      // so that the loads of a round are all in flight together
      if (S == 1) {
        for (int e = tid; e < ne; e += 64 * NW) {
          double v = 0.0;
          for (int p0 = 0; p0 < G; p0 += 8) {
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = ld_dev(c.part + (int64_t)min(p0 + u, G - 1) * E + e0 + e);
#pragma unroll
            for (int u = 0; u < 8; ++u) v += (double)zmask(x[u], p0 + u < G);
          }
          st_dev(c.red + e0 + e, v);
        }
      } else {
        if (tid < S * ne) {
          const int e = tid % ne, sidx = tid / ne;
          double acc = 0.0;
          for (int p0 = sidx; p0 < G; p0 += 8 * S) {
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = ld_dev(c.part + (int64_t)min(p0 + u * S, G - 1) * E + e0 + e);
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += (double)zmask(x[u], p0 + u * S < G);
          }
          sAcc[tid] = acc;
        }
        __syncthreads();
        if (tid < ne) {
          double v = 0.0;
          for (int sidx = 0; sidx < S; ++sidx) v += sAcc[sidx * ne + tid];
          st_dev(c.red + e0 + tid, v);
        }
      }
    }
    if (!coop_barrier(c, ++epoch, &sAbort)) break;

    // ---- (C) the W-update of all rows and W^T W, in every workgroup
    {  // thread (h, i) loads half h of row i of the sums of X H^T and one sum of H H^T,
       // all nine loads in flight together (clamped addresses, masked after the load)
      const int i = tid & 255, h = tid >> 8;
      const int cg = (tid & 255) / RB, qg = tid % RB;
      double nv[RB / 2];
#pragma unroll
      for (int u = 0; u < RB / 2; ++u)
        nv[u] = ld_dev(c.red + min(i, m - 1) * r + min(RB / 2 * h + u, r - 1));
      const double gv = ld_dev(c.red + m * r + min(cg, r - 1) * r + min(qg, r - 1));
#pragma unroll
      for (int u = 0; u < RB / 2; ++u) sN[i][RB / 2 * h + u] = zmask(nv[u], i < m && RB / 2 * h + u < r);
      if (h == 0) sGH[cg][qg] = zmask(gv, cg < r && qg < r);
    }
    __syncthreads();
    // D_W = W G_H by FP64 MFMA (16 x 16 x 4), wave w its two 16-row tiles: lane (a, b)
    // feeds A = W[r0 + a][4s + b] and B = G_H[4s + b][a]; value v of the result is
    // D_W[r0 + 4v + b][a].  Then W <- max(0, W .* N_W ./ (D_W + eps)) in FP64 on FP32 data.
    {
      v4d dw[MBW];
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk) {
        const int r0 = row0 + 16 * blk;
        dw[blk] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int st4 = 0; st4 < RB / 4; ++st4)
          dw[blk] = mfma16_f64((double)sWc[r0 + a][4 * st4 + b], sGH[4 * st4 + b][a], dw[blk]);
      }
      float wn[MBW][4];
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + 16 * blk + 4 * v + b;
          const double q = fmax(0.0, (double)sWc[row][a] * sN[row][a] / (dw[blk][v] + (double)c.eps));
          wn[blk][v] = (row < m && a < r) ? (float)q : 0.f;
        }
      wave_sync();  // the wave's reads of its old rows are done before they are replaced
#pragma unroll
      for (int blk = 0; blk < MBW; ++blk)
#pragma unroll
        for (int v = 0; v < 4; ++v) sWc[row0 + 16 * blk + 4 * v + b][a] = wn[blk][v];
      wave_sync();
      // this wave's 32 rows of G_W = W^T W (FP64 MFMA, four rows a step, in row order)
      v4d gacc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st4 = 0; st4 < 8; ++st4) {
        const double o = (double)sWc[row0 + 4 * st4 + b][a];
        gacc = mfma16_f64(o, o, gacc);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) sGp[w][lane][q] = gacc[q];
    }
    __syncthreads();
    if (tid < 256) {  // the waves' Grams added in wave order
      const int l = tid >> 2, q = tid & 3;
      double s = sGp[0][l][q];
#pragma unroll
      for (int ww = 1; ww < NW; ++ww) s += sGp[ww][l][q];
      // FP64 16 x 16 x 4 result layout: value q of lane (a, b) is row 4 q + b, column a
      sGW[4 * q + (l >> 4)][l & 15] = (float)s;
    }
    __syncthreads();
  }
  if (sAbort) {
    if (tid == 0) atomicExch(c.status, 1);
    return;
  }
  // write back: W and W^T W (workgroup 0), this workgroup's H columns
  if (blockIdx.x == 0) {
    for (int e = tid; e < m * r; e += 64 * NW) c.W[e] = sWc[e / r][e % r];
    if (tid < 256) c.GW[tid] = sGW[tid / 16][tid % 16];
  }
  for (int e = tid; e < 16 * CW; e += 64 * NW) {
    const int cc = e / CW, j = e % CW;
    const int64_t col = col0 + j;
    if (cc < r && col < k) c.H[(int64_t)cc * k + col] = sH[cc][j];
  }
}

template <int NG>
hipError_t launch_ng(const CoopArgs& c, int G, hipStream_t s) {
  k_stage_coop<NG><<<G, 64 * kCoopWaves, 0, s>>>(c);
  return hipGetLastError();
}

template <int NG>
int max_blocks_ng() {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_stage_coop<NG>),
                                                   64 * kCoopWaves, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

}  // namespace

int stage_coop_max_grid(int ng) {
  switch (ng) {
    case 1: { static const int v = max_blocks_ng<1>(); return v; }
    case 2: { static const int v = max_blocks_ng<2>(); return v; }
    case 4: { static const int v = max_blocks_ng<4>(); return v; }
    case 8: { static const int v = max_blocks_ng<8>(); return v; }
    default: return 0;
  }
}

hipError_t launch_stage_coop(const CoopArgs& c, int ng, int G, hipStream_t s) {
  if (c.m < 1 || c.m > 256 || c.r < 1 || c.r > 16 || G < 1 || G > 64 * kCoopWaves ||
      (int64_t)G * 16 * ng < c.k)
    return hipErrorInvalidValue;
  // every workgroup must be resident at once for the grid barrier
  const int cap = stage_coop_max_grid(ng);
  if (cap <= 0 || G > cap) return hipErrorInvalidValue;
  hipError_t e = launch_zero_ints(reinterpret_cast<int*>(c.flags), (int64_t)32 * G, s);
  if (e != hipSuccess) return e;
  switch (ng) {
    case 1: return launch_ng<1>(c, G, s);
    case 2: return launch_ng<2>(c, G, s);
    case 4: return launch_ng<4>(c, G, s);
    case 8: return launch_ng<8>(c, G, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ntt
