// ntt_device.h -- device helpers shared by the kernel sources: MFMA wrappers, wave-level
// synchronisation and sums, masked loads, the FP32 divide of the MU epilogues, the
// W-update entry, device-scope accesses and the FP64 Gram of W's rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ntt {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

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

// `v` where `ok`, else 0, for a value loaded from a clamped (always valid) address.
// Written as a multiply rather than a select so that the load stays unconditional: a
// select lets the compiler sink the load into a branch that waits for every memory
// operation in flight, which serialises loads and defeats prefetching.
__device__ __forceinline__ float zmask(float v, bool ok) { return v * (ok ? 1.f : 0.f); }
__device__ __forceinline__ double zmask(double v, bool ok) { return v * (ok ? 1.0 : 0.0); }

__device__ __forceinline__ v4d mfma16_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Entry c of a row of the W-update in FP64 on FP32 data (shared by the W-update kernel and
// the pass prologues, so that both give the same bits): with D = sum_{q < RB} w[q] G_H[q][c]
// (q in order; w and G_H zero padded past r), max(0, w[c] n / (D + eps)) rounded to FP32.
// The caller masks columns c >= r.
template <int RB>
__device__ __forceinline__ float wupdate_entry(const float* wrow, double n, const double (*sGH)[RB + 1],
                                               int c, float eps) {
  double dw = 0.0;
#pragma unroll
  for (int q = 0; q < RB; ++q) dw += (double)wrow[q] * sGH[q][c];
  return (float)fmax(0.0, (double)wrow[c] * n / (dw + (double)eps));
}

// Device-scope relaxed accesses for data that crosses workgroups within one launch: they go
// past the XCDs' non-coherent L2s, so a value stored by one workgroup (after the storing
// wave's s_waitcnt) is what another workgroup loads, without a fence.
__device__ __forceinline__ void st_dev(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_dev(const float* p) {
  return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront w's part of the Gram of the rows in LDS (FP64 MFMA, 16 x 16 x 4 tiles): rows
// 64 w + 4 st + (0..3) for st = 0, 1, ..., in order, stopping at NROWS (rows from the
// first zero row on contribute exact zeros, so stopping early does not change the bits).
template <int RB, int NT, int NROWS>
__device__ __forceinline__ void gram_rows_f64(const float (*sWc)[RB + 1], v4d (&acc)[NT][NT],
                                              int w, int a, int b) {
#pragma unroll 4
  for (int st = 0; st < 16; ++st) {
    if (64 * w + 4 * st >= NROWS) break;
    const int row = 64 * w + 4 * st + b;
    double opnd[NT];
#pragma unroll
    for (int h = 0; h < NT; ++h) {
      const int c = 16 * h + a;
      opnd[h] = (c < RB) ? (double)sWc[row][c < RB ? c : 0] : 0.0;
    }
#pragma unroll
    for (int h = 0; h < NT; ++h)
#pragma unroll
      for (int q = 0; q < NT; ++q) acc[h][q] = mfma16_f64(opnd[h], opnd[q], acc[h][q]);
  }
}


// x / y by the hardware reciprocal and one Newton-Raphson correction
// (q0 = x r, e = x - y q0, q = q0 + e r): within about 1 ulp for normal y.
__device__ __forceinline__ float fast_div(float x, float y) {
  const float r = __builtin_amdgcn_rcpf(y);
  const float q0 = x * r;
  const float e = fmaf(-y, q0, x);
  return fmaf(e, r, q0);
}

}  // namespace ntt
