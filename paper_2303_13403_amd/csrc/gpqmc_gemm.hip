// Batched MFMA GEMM of the PQMC sweep (gfx950), one 64 x 64 output tile per
// workgroup, with the epilogues that fuse the sweep's elementwise work:
//   the kinetic wrap                    G <- D_{l+1} (Gtmp e^{dtau K}) D_{l+1}^{-1}
//   the basis propagation               U <- e^{-dtau K} (D_l U)   /  D_l (e^{-dtau K} U)
//   the checkpoint products (FP64)      U^T U, U R^{-1}, L^T R, (L R)^{-1} L, 1 - R Y
// The tile list maps every workgroup to (entry, tile); entries are one chain
// and one spin, so a launch covers the whole batch, uneven lattices included.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gpqmc_device.h"

namespace gpqmc {

template <typename T, int MODE, bool TRANSA, bool TRANSB, typename Tb>
__global__ __launch_bounds__(kThreads) void k_gemm(const GemmEntry* __restrict__ ents,
                                                   const TileRef* __restrict__ tiles,
                                                   int n_tiles, GemmArgs args) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid >= n_tiles) return;
  const TileRef tr = tiles[bid];
  const GemmEntry& e = ents[tr.entry];
  const int M = e.M, N = e.N, K = e.K;
  const int m0 = tr.tm * kTile, n0 = tr.tn * kTile;
  if (m0 >= M || n0 >= N) return;

  const int p = args.parity;
  const T* A = (const T*)e.A[0];
  const T* B = (const T*)e.B[0];
  T* C = (T*)e.C[0];
  if (MODE == GM_PROPB || MODE == GM_PROPR) {
    B = (const T*)e.B[p];
    C = (T*)e.C[p ^ 1];
  } else if (MODE == GM_GRAM) {
    A = (const T*)e.A[p];
    B = A;
  } else if (MODE == GM_APPLY) {
    A = (const T*)e.A[p];
  } else if (MODE == GM_XMAT || MODE == GM_YMAT || MODE == GM_GFRESH) {
    const double* slotp = e.stack + (size_t)args.slot * e.slot_stride;
    const double* R = args.dir == 0 ? e.Qc : slotp;
    const double* Lt = args.dir == 0 ? slotp : e.Qc;
    if (MODE == GM_XMAT) {
      A = (const T*)Lt;
      B = (const T*)R;
    } else if (MODE == GM_YMAT) {
      B = (const T*)Lt;
    } else {
      A = (const T*)R;
    }
  }
  const int lda = e.lda, ldb = e.ldb, ldc = e.ldc;

  constexpr int LDS_LD = kTile + LDS_PAD;
  __shared__ T As[BK * LDS_LD];
  __shared__ T Bs[BK * LDS_LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

  // B-row scaling by the diagonal of D_l (basis propagation A (D B))
  const int8_t* bfield = nullptr;
  int bbnd = 1;
  if (MODE == GM_PROPB && args.bscale_slice >= 0) {
    bfield = e.field + (size_t)args.bscale_slice * e.n_sites;
    bbnd = (args.bscale_slice == 0 || args.bscale_slice == args.n_bulk_last + 1) ? 0 : 1;
  }

  T ra[4], rb[4];
  auto load_regs = [&](int kbase) {
    if (!TRANSA) {
      const int i = m0 + (tid >> 2), k = kbase + (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        ra[q] = (i < M && k + q < K) ? A[(size_t)i * lda + k + q] : T(0);
    } else {
      const int k = kbase + (tid >> 4), i = m0 + (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        ra[q] = (k < K && i + q < M) ? A[(size_t)k * lda + i + q] : T(0);
    }
    if (!TRANSB) {
      const int k = kbase + (tid >> 4), j = n0 + (tid & 15) * 4;
      T sc = T(1);
      if (bfield && k < K) sc = (T)dfac(e.dval, bbnd, bfield[k], false);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rb[q] = (k < K && j + q < N) ? B[(size_t)k * ldb + j + q] * sc : T(0);
    } else {
      const int j = n0 + (tid >> 2), k = kbase + (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rb[q] = (j < N && k + q < K) ? B[(size_t)j * ldb + k + q] : T(0);
    }
  };
  auto store_lds = [&]() {
    if (!TRANSA) {
      const int i = tid >> 2, k = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) As[(k + q) * LDS_LD + i] = ra[q];
    } else {
      const int k = tid >> 4, i = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) As[k * LDS_LD + i + q] = ra[q];
    }
    if (!TRANSB) {
      const int k = tid >> 4, j = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) Bs[k * LDS_LD + j + q] = rb[q];
    } else {
      const int j = tid >> 2, k = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) Bs[(k + q) * LDS_LD + j] = rb[q];
    }
  };

  WaveTile<T> wt;
  wt.zero();
  const int nk = (K + BK - 1) / BK;
  if (nk > 0) {
    load_regs(0);
    store_lds();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      if (kt + 1 < nk) load_regs((kt + 1) * BK);
      wt.mac(As, Bs, LDS_LD, wm, wn, lane);
      __syncthreads();
      if (kt + 1 < nk) {
        store_lds();
        __syncthreads();
      }
    }
  }

  // ---- epilogue ----
  const int8_t* sfield = nullptr;
  int sbnd = 1;
  if (args.scale_slice >= 0) {
    sfield = e.field + (size_t)args.scale_slice * e.n_sites;
    sbnd = (args.scale_slice == 0 || args.scale_slice == args.n_bulk_last + 1) ? 0 : 1;
  }
  const bool inv = args.scale_inverse != 0;
  float dmax = 0.f;
  // the drift check reads the wrapped Green's function it replaces: all of
  // those loads are issued before the first store of the tile
  Tb prev[16];
  int ix = 0;
  if (MODE == GM_GFRESH && args.check_drift) {
    const Tb* Cb = (const Tb*)e.C[1];
    wt.each(wm, wn, lane, [&](int li, int lj, T) {
      const int i = m0 + li, j = n0 + lj;
      prev[ix++] = (i < M && j < N) ? Cb[(size_t)i * e.ldc2 + j] : Tb(0);
    });
  }
  ix = 0;
  wt.each(wm, wn, lane, [&](int li, int lj, T acc) {
    const int i = m0 + li, j = n0 + lj;
    const int k = ix++;
    if (i >= M || j >= N) return;
    const size_t o = (size_t)i * ldc + j;
    if (MODE == GM_PROPR) {
      T v = acc;
      if (sfield) v *= (T)dfac(e.dval, sbnd, sfield[i], false);
      C[o] = v;
    } else if (MODE == GM_WRAP) {
      T v = acc;
      if (sfield)
        v *= (T)(dfac(e.dval, sbnd, sfield[i], inv) * dfac(e.dval, sbnd, sfield[j], !inv));
      C[o] = v;
    } else if (MODE == GM_GFRESH) {
      const double g = (i == j ? 1.0 : 0.0) - (double)acc;
      C[o] = (T)g;
      Tb* Cb = (Tb*)e.C[1];
      const size_t o2 = (size_t)i * e.ldc2 + j;
      if (args.check_drift) {
        const float d = (float)fabs((double)prev[k] - g);
        dmax = (d != d) ? __builtin_inff() : fmaxf(dmax, d);
      }
      double v = g;
      if (sfield) v *= dfac(e.dval, sbnd, sfield[i], inv) * dfac(e.dval, sbnd, sfield[j], !inv);
      Cb[o2] = (Tb)v;
    } else {
      C[o] = acc;
    }
  });
  if (MODE == GM_GFRESH && args.check_drift) {
    __shared__ float red[4];
    dmax = wave_max(dmax);
    if (lane == 0) red[wave] = dmax;
    __syncthreads();
    if (tid == 0) {
      const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
      atomicMax(&e.st->drift_bits, __float_as_uint(m));
    }
  }
}

template <typename T, int MODE, bool TA, bool TB, typename Tb>
static hipError_t gemm_t(const GemmEntry* e, const TileRef* t, int n, GemmArgs a, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemm<T, MODE, TA, TB, Tb>), dim3(n), dim3(kThreads), 0, s, e, t, n, a);
  return hipGetLastError();
}

// fp32: arithmetic type of the modes that follow the Green's function or the
// basis precision (STORE/WRAP/PROP*); the checkpoint modes are FP64
// and write their bulk copy (GFRESH) in the Green's-function precision g_fp32.
hipError_t launch_gemm(int fp32, int g_fp32, int mode, const GemmEntry* e, const TileRef* t, int n,
                       GemmArgs a, hipStream_t s) {
  switch (mode) {
    case GM_GRAM: return gemm_t<double, GM_GRAM, true, false, double>(e, t, n, a, s);
    case GM_APPLY: return gemm_t<double, GM_APPLY, false, false, double>(e, t, n, a, s);
    case GM_XMAT: return gemm_t<double, GM_XMAT, true, false, double>(e, t, n, a, s);
    case GM_YMAT: return gemm_t<double, GM_YMAT, false, true, double>(e, t, n, a, s);
    case GM_GFRESH:
      return g_fp32 ? gemm_t<double, GM_GFRESH, false, false, float>(e, t, n, a, s)
                    : gemm_t<double, GM_GFRESH, false, false, double>(e, t, n, a, s);
    default: break;
  }
  if (fp32) {
    switch (mode) {
      case GM_STORE: return gemm_t<float, GM_STORE, false, false, float>(e, t, n, a, s);
      case GM_WRAP: return gemm_t<float, GM_WRAP, false, false, float>(e, t, n, a, s);
      case GM_PROPB: return gemm_t<float, GM_PROPB, false, false, float>(e, t, n, a, s);
      case GM_PROPR: return gemm_t<float, GM_PROPR, false, false, float>(e, t, n, a, s);
    }
  } else {
    switch (mode) {
      case GM_STORE: return gemm_t<double, GM_STORE, false, false, double>(e, t, n, a, s);
      case GM_WRAP: return gemm_t<double, GM_WRAP, false, false, double>(e, t, n, a, s);
      case GM_PROPB: return gemm_t<double, GM_PROPB, false, false, double>(e, t, n, a, s);
      case GM_PROPR: return gemm_t<double, GM_PROPR, false, false, double>(e, t, n, a, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_plain(int fp32, int transA, const GemmEntry* e, const TileRef* t, int n,
                             GemmArgs a, hipStream_t s) {
  if (fp32) return transA ? gemm_t<float, GM_STORE, true, false, float>(e, t, n, a, s)
                          : gemm_t<float, GM_STORE, false, false, float>(e, t, n, a, s);
  return transA ? gemm_t<double, GM_STORE, true, false, double>(e, t, n, a, s)
                : gemm_t<double, GM_STORE, false, false, double>(e, t, n, a, s);
}

}  // namespace gpqmc
