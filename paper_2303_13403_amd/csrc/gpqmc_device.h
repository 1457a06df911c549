// Device helpers shared by the HIP kernels: XCD-aware workgroup mapping,
// wave/workgroup reductions, and the MFMA wave tiles of the GEMM kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "gpqmc_internal.h"

namespace gpqmc {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Pointers into device memory typed in the global address space.  The buffers
// reach the kernels through descriptor structs, so the compiler cannot tell
// that they are not LDS and would emit flat loads; those count on the LDS
// counter too, and every wait for an LDS read would then also wait for the
// global loads in flight (the prefetch of the next k-tile).  Reads and writes
// through a GLOBAL pointer are global_load / global_store.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL T* gp(T* p) {
  return (GLOBAL T*)p;
}

// 16-byte vector loads through a GLOBAL pointer (as builtin vector types: the
// float4 / double2 classes have no constructor from a global-space lvalue)
__device__ __forceinline__ float4 gload4(const GLOBAL float* p) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  const v4 v = *(const GLOBAL v4*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 gload2(const GLOBAL double* p) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(const GLOBAL v2*)p;
  return make_double2(v.x, v.y);
}

constexpr int BK = 16;        // GEMM k-tile
constexpr int LDS_PAD = 4;    // LDS row padding of the GEMM tiles (elements)

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Map hardware id b (of n) to a logical index so that every XCD receives one
// contiguous range of logical indices: consecutive tiles of one chain/spin,
// and the per-chain kernels of the same chain, then share an L2.
__device__ inline int xcd_remap(int b, int n) {
  if (n < 16) return b;
  const int per = n / 8, rem = n % 8;
  const int x = b % 8, idx = b / 8;
  return (x < rem) ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

// Orders LDS traffic between the lanes of one wave (no instruction is emitted
// for a single wave; it stops the compiler from moving memory operations).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the 256-thread workgroup; result returned to every thread.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// D_l diagonal for one site with exponent m: exp(sigma c_b m); the inverse is
// the value at -m.
__device__ inline double dfac(const double (&dv)[2][2 * kMexp + 1], int b, int8_t m,
                              bool inverse) {
  return dv[b][kMexp + (inverse ? -(int)m : (int)m)];
}

// ---------------------------------------------------------------------------
// MFMA wave tiles: every wave computes a 32 x 32 block of the 64 x 64 tile.
// ---------------------------------------------------------------------------
template <typename T>
struct WaveTile;

// FP32: one v_mfma_f32_32x32x2f32 per k-pair.  Lane l supplies A[l%32][k0+l/32]
// and B[k0+l/32][l%32]; result element (i, j) lives in lane j + 32*((i/4)%2),
// register (i%4) + 4*(i/8).
template <>
struct WaveTile<float> {
  floatx16 acc;
  __device__ void zero() {
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  }
  __device__ void mac(const float* As, const float* Bs, int ld, int wm, int wn, int lane) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const float a = As[(kk + (lane >> 5)) * ld + wm + (lane & 31)];
      const float b = Bs[(kk + (lane >> 5)) * ld + wn + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
  }
  template <class F>
  __device__ void each(int wm, int wn, int lane, F f) const {
#pragma unroll
    for (int r = 0; r < 16; ++r)
      f(wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), wn + (lane & 31), acc[r]);
  }
};

// FP64: 2 x 2 blocks of v_mfma_f64_16x16x4f64.  Lane l supplies A[l%16][k0+l/16]
// and B[k0+l/16][l%16]; result element (i, j) of a block lives in lane
// j + 16*(i%4), register i/4 (measured on gfx950).
template <>
struct WaveTile<double> {
  doublex4 acc[2][2];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[a][b][r] = 0.0;
  }
  __device__ void mac(const double* As, const double* Bs, int ld, int wm, int wn, int lane) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = (kk + (lane >> 4)) * ld;
      const double a0 = As[kr + wm + (lane & 15)];
      const double a1 = As[kr + wm + 16 + (lane & 15)];
      const double b0 = Bs[kr + wn + (lane & 15)];
      const double b1 = Bs[kr + wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  template <class F>
  __device__ void each(int wm, int wn, int lane, F f) const {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          f(wm + 16 * a + 4 * r + (lane >> 4), wn + 16 * b + (lane & 15), acc[a][b][r]);
  }
};

}  // namespace gpqmc
