// Batched MFMA GEMM of the PQMC sweep (gfx950), one 64 x 64 output tile per
// workgroup, with the epilogues that fuse the sweep's elementwise work:
//   the kinetic wrap                    G <- D_{l+1} (Gtmp e^{dtau K}) D_{l+1}^{-1}
//   the slice's delayed update          G <- D (G - Xa Ya) D^{-1}
//   the basis propagation               U <- e^{-dtau K} (D_l U)   /  D_l (e^{-dtau K} U)
//   the checkpoint products (FP64)      U^T U, U R^{-1}, L^T R, (L R)^{-1} L, 1 - R Y
// and, for the factored engine (G = 1 - A B^T, FP64), the propagation of both
// factors with the frame change fused (A <- D^{+-1} K^{-+} A, B likewise), the
// segment update Q <- Q - (Q Mf^T) Wf of the dual factor, and the checkpoint
// products 1 - A B^T, L^T (L R)^{-T}, R (L R)^{-1}.
// The tile list maps every workgroup to (entry, tile); entries are one chain
// and one spin, so a launch covers the whole batch, uneven lattices included.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gpqmc_device.h"

namespace gpqmc {

// Four consecutive elements from global memory: one 16-byte (FP32) or two
// 16-byte (FP64) loads when all four are in range and aligned, else element
// by element with zeros past the end.
__device__ inline void ld4(const GLOBAL float* __restrict__ p, int valid, bool aligned, float (&r)[4]) {
  if (aligned && valid >= 4) {
    const float4 v = gload4(p);
    r[0] = v.x, r[1] = v.y, r[2] = v.z, r[3] = v.w;
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = q < valid ? p[q] : 0.f;
}
__device__ inline void ld4(const GLOBAL double* __restrict__ p, int valid, bool aligned, double (&r)[4]) {
  if (aligned && valid >= 4) {
    const double2 a = gload2(p), b = gload2(p + 2);
    r[0] = a.x, r[1] = a.y, r[2] = b.x, r[3] = b.y;
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = q < valid ? p[q] : 0.0;
}

template <typename T, int MODE, bool TRANSA, bool TRANSB, typename Tb>
__global__ __launch_bounds__(kThreads) void k_gemm(const GemmEntry* __restrict__ ents,
                                                   const TileRef* __restrict__ tiles,
                                                   int n_tiles, GemmArgs args) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid >= n_tiles) return;
  const TileRef tr = tiles[bid];
  const GemmEntry& e = ents[tr.entry];
  const int M = e.M, N = e.dynN ? *e.dynN : e.N, K = e.dynK ? *e.dynK : e.K;
  const int m0 = tr.tm * kTile, n0 = tr.tn * kTile;
  if (m0 >= M || n0 >= N) return;
  if (MODE == GM_SEGF && K == 0) return;   // no flip accepted: Q unchanged

  const int p = args.parity;
  const GLOBAL T* A = gp((const T*)e.A[0]);
  const GLOBAL T* B = gp((const T*)e.B[0]);
  GLOBAL T* C = gp((T*)e.C[0]);
  // factored checkpoint operands: 0 = the new orthonormal basis Qc, 1 = the
  // stack slot, 2 = the active factor of this entry
  const double* slot_base = e.stack ? e.stack + (size_t)args.slot * e.slot_stride : nullptr;
  auto fsel = [&](int sel, const void* fac) -> const GLOBAL T* {
    return gp((const T*)(sel == 0 ? (const void*)e.Qc : sel == 1 ? (const void*)slot_base : fac));
  };
  if (MODE == GM_IMABT) {
    A = gp((const T*)e.A[p]);
    B = gp((const T*)e.B[p]);
  } else if (MODE == GM_SEGP) {
    A = gp((const T*)e.A[p]);
  } else if (MODE == GM_SEGF) {
    C = gp((T*)e.C[p]);
  } else if (MODE == GM_BMAT) {
    A = fsel(args.lsel, nullptr);
    C = gp((T*)e.C[p]);
  } else if (MODE == GM_AMAT) {
    A = fsel(args.rsel, nullptr);
    C = gp((T*)e.C[p]);
  } else if (MODE == GM_GFRESH2) {
    A = fsel(args.rsel, e.A[p]);
    B = fsel(args.lsel, e.B[p]);
  }
  if (MODE == GM_PROPB || MODE == GM_PROPR) {
    B = gp((const T*)e.B[p]);
    C = gp((T*)e.C[p ^ 1]);
  } else if (MODE == GM_GRAM) {
    A = gp((const T*)e.A[p]);
    B = A;
  } else if (MODE == GM_APPLY) {
    A = gp((const T*)e.A[p]);
  } else if (MODE == GM_XMAT || MODE == GM_YMAT || MODE == GM_GFRESH) {
    const double* slotp = e.stack + (size_t)args.slot * e.slot_stride;
    const double* R = args.dir == 0 ? e.Qc : slotp;
    const double* Lt = args.dir == 0 ? slotp : e.Qc;
    if (MODE == GM_XMAT) {
      A = gp((const T*)Lt);
      B = gp((const T*)R);
    } else if (MODE == GM_YMAT) {
      B = gp((const T*)Lt);
    } else {
      A = gp((const T*)R);
    }
  }
  const int lda = e.lda, ldb = e.ldb, ldc = e.ldc;
  // 16-byte alignment of every row start (the four-element groups start at
  // multiples of four)
  constexpr int VA = 16 / sizeof(T) - 1;
  const bool a_al = (lda & VA) == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
  const bool b_al = (ldb & VA) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;

  constexpr int LDS_LD = kTile + LDS_PAD;
  __shared__ T As[BK * LDS_LD];
  __shared__ T Bs[BK * LDS_LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

  // B-row scaling by the diagonal of D_l (basis propagation A (D B))
  const GLOBAL int8_t* bfield = nullptr;
  int bbnd = 1;
  if (MODE == GM_PROPB && args.bscale_slice >= 0) {
    bfield = gp(e.field + (size_t)args.bscale_slice * e.n_sites);
    bbnd = (args.bscale_slice == 0 || args.bscale_slice == args.n_bulk_last + 1) ? 0 : 1;
  }

  // the two possible B-row factors, read once; a prefetched row carries only
  // its field value, the factor is applied when it is stored to LDS
  const T bsc_p = bfield ? (T)dfac(e.dval, bbnd, 1, false) : T(1);
  const T bsc_m = bfield ? (T)dfac(e.dval, bbnd, -1, false) : T(1);
  int8_t bf = 1;
  T ra[4], rb[4];
  auto load_regs = [&](int kbase) {
    if (!TRANSA) {
      const int i = m0 + (tid >> 2), k = kbase + (tid & 3) * 4;
      ld4(A + (size_t)i * lda + k, i < M ? K - k : 0, a_al, ra);
    } else {
      const int k = kbase + (tid >> 4), i = m0 + (tid & 15) * 4;
      ld4(A + (size_t)k * lda + i, k < K ? M - i : 0, a_al, ra);
    }
    if (!TRANSB) {
      const int k = kbase + (tid >> 4), j = n0 + (tid & 15) * 4;
      bf = (bfield && k < K) ? bfield[k] : (int8_t)1;
      ld4(B + (size_t)k * ldb + j, k < K ? N - j : 0, b_al, rb);
    } else {
      const int j = n0 + (tid >> 2), k = kbase + (tid & 3) * 4;
      ld4(B + (size_t)j * ldb + k, j < N ? K - k : 0, b_al, rb);
    }
  };
  auto store_lds = [&]() {
    T* as = As;
    T* bs = Bs;
    if (!TRANSA) {
      const int i = tid >> 2, k = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) as[(k + q) * LDS_LD + i] = ra[q];
    } else {
      const int k = tid >> 4, i = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) as[k * LDS_LD + i + q] = ra[q];
    }
    if (!TRANSB) {
      const int k = tid >> 4, j = (tid & 15) * 4;
      const T sc = bf > 0 ? bsc_p : bsc_m;
#pragma unroll
      for (int q = 0; q < 4; ++q) bs[k * LDS_LD + j + q] = rb[q] * sc;
    } else {
      const int j = tid >> 2, k = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) bs[(k + q) * LDS_LD + j] = rb[q];
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
  const GLOBAL int8_t* sfield = nullptr;
  int sbnd = 1;
  if (args.scale_slice >= 0) {
    sfield = gp(e.field + (size_t)args.scale_slice * e.n_sites);
    sbnd = (args.scale_slice == 0 || args.scale_slice == args.n_bulk_last + 1) ? 0 : 1;
  }
  const bool inv = (args.scale_inverse != 0) != (e.sinv != 0);
  // the tile's row factors d(i) and column factors 1/d(j) of the frame
  // change, staged once (PROPR scales rows only, by d(i), or by 1/d(i) for an
  // entry marked sinv)
  __shared__ double drow[kTile], dcol[kTile];
  if (sfield) {
    if (tid < kTile) {
      const int i = m0 + tid;
      drow[tid] = i < M ? dfac(e.dval, sbnd, sfield[i], inv) : 0.0;
    } else if (tid < 2 * kTile) {
      const int j = n0 + tid - kTile;
      dcol[tid - kTile] = j < N ? dfac(e.dval, sbnd, sfield[j], !inv) : 0.0;
    }
    __syncthreads();
  }
  float dmax = 0.f, gmx = 0.f;
  // the drift check reads the wrapped Green's function it replaces: all of
  // those loads are issued before the first store of the tile
  Tb prev[16];
  int ix = 0;
  if ((MODE == GM_GFRESH || MODE == GM_GFRESH2) && args.check_drift) {
    const GLOBAL Tb* Cb = gp((const Tb*)e.C[1]);
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
      if (sfield) v *= (T)drow[li];
      C[o] = v;
    } else if (MODE == GM_WRAP || MODE == GM_FLUSH) {
      T v = (MODE == GM_FLUSH) ? gp((const T*)e.C[0])[o] - acc : acc;
      if (sfield) v *= (T)(drow[li] * dcol[lj]);
      if (MODE == GM_FLUSH)
        gp((T*)e.C[1])[o] = v;
      else
        C[o] = v;
    } else if (MODE == GM_GFRESH) {
      const double g = (i == j ? 1.0 : 0.0) - (double)acc;
      C[o] = (T)g;
      GLOBAL Tb* Cb = gp((Tb*)e.C[1]);
      const size_t o2 = (size_t)i * e.ldc2 + j;
      if (args.check_drift) {
        const float d = (float)fabs((double)prev[k] - g);
        dmax = (d != d) ? __builtin_inff() : fmaxf(dmax, d);
        gmx = fmaxf(gmx, (float)fabs(g));
      }
      double v = g;
      if (sfield) v *= drow[li] * dcol[lj];
      Cb[o2] = (Tb)v;
    } else if (MODE == GM_GFRESH2) {
      const double g = (i == j ? 1.0 : 0.0) - (double)acc;
      C[o] = (T)g;
      if (args.check_drift) {
        const float d = (float)fabs((double)prev[k] - g);
        dmax = (d != d) ? __builtin_inff() : fmaxf(dmax, d);
        gmx = fmaxf(gmx, (float)fabs(g));
      }
    } else if (MODE == GM_IMABT) {
      C[o] = (T)((i == j ? 1.0 : 0.0) - (double)acc);
    } else if (MODE == GM_SEGF) {
      C[o] = C[o] - acc;
    } else {
      C[o] = acc;
    }
  });
  if ((MODE == GM_GFRESH || MODE == GM_GFRESH2) && args.check_drift) {
    __shared__ float red[2][4];
    dmax = wave_max(dmax);
    gmx = wave_max(gmx);
    if (lane == 0) {
      red[0][wave] = dmax;
      red[1][wave] = gmx;
    }
    __syncthreads();
    if (tid == 0) {
      // non-negative floats order as their bit patterns
      const float m = fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3]));
      const float gm = fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3]));
      atomicMax(&e.st->drift_bits, __float_as_uint(m));
      atomicMax(&e.st->gmax_bits, __float_as_uint(gm));
    }
  }
}

// ---------------------------------------------------------------------------
// Large-tile FP32 GEMM for the N x N x N products of the kinetic wrap (modes
// STORE and WRAP) and the slice's delayed update (FLUSH, K = accepted flips): 128 x 128 output tile per workgroup, 64 x 64 per wave as
// 2 x 2 blocks of v_mfma_f32_32x32x2f32, k-tiles of 16 double-buffered in LDS
// with the next k-tile prefetched into registers (one barrier per k-tile).
// A is kept in LDS with each row's k values split by parity (k = 2 kk + h at
// [row][h][kk]), so a lane fetches the A operand of four MFMA k-steps with one
// 128-bit read; B stays row-major ([k][j]), read one float per k-step.
// ---------------------------------------------------------------------------
constexpr int kTileL = 128, BKL = 16;
constexpr int LDAL = BKL + 4;        // A tile row: BKL / 2 even-k, BKL / 2 odd-k, 4 pad
constexpr int LDBL = kTileL + 4;     // B tile row

__device__ inline float4 load4(const GLOBAL float* __restrict__ p, int valid, bool aligned) {
  if (aligned && valid >= 4) return gload4(p);
  float4 v;
  v.x = valid > 0 ? p[0] : 0.f;
  v.y = valid > 1 ? p[1] : 0.f;
  v.z = valid > 2 ? p[2] : 0.f;
  v.w = valid > 3 ? p[3] : 0.f;
  return v;
}

// FLUSH keeps four workgroups per CU like STORE: the old values of C are
// loaded in the epilogue rather than held through the k-loop
template <int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MODE == GM_FLUSH ? 4 : 1))) void k_gemm_l(const GemmEntry* __restrict__ ents,
                                                     const TileRef* __restrict__ tiles,
                                                     int n_tiles, GemmArgs args) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid >= n_tiles) return;
  const TileRef tr = tiles[bid];
  const GemmEntry& e = ents[tr.entry];
  const int M = e.M, N = e.N, K = e.dynK ? *e.dynK : e.K;
  const int m0 = tr.tm * kTileL, n0 = tr.tn * kTileL;
  if (m0 >= M || n0 >= N) return;
  const GLOBAL float* __restrict__ A = gp((const float*)e.A[0]);
  const GLOBAL float* __restrict__ B = gp((const float*)e.B[0]);
  GLOBAL float* __restrict__ C = gp((float*)e.C[0]);
  const int lda = e.lda, ldb = e.ldb, ldc = e.ldc;
  const bool a_al = (lda & 3) == 0, b_al = (ldb & 3) == 0;
  // a tile inside the matrices with aligned rows loads its whole k-tiles
  // without bounds checks
  const bool interior = a_al && b_al && m0 + kTileL <= M && n0 + kTileL <= N;

  __shared__ __align__(16) float As[2][kTileL * LDAL];
  __shared__ __align__(16) float Bs[2][BKL * LDBL];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  // global -> register mapping: A row am, BKL / 2 k values from ak; B k-row
  // bk, BKL / 2 columns from bj (NQ float4 loads of each per thread)
  constexpr int NQ = BKL / 8, TPR = kThreads / BKL;
  static_assert(NQ % 2 == 0, "A rows are stored as pairs of float4");
  const int am = tid >> 1, ak = (tid & 1) * (BKL / 2);
  const int bk = tid / TPR, bj = (tid % TPR) * (BKL / 2);
  float4 ra[NQ], rb[NQ];
  auto gload = [&](int k0) {
    const int i = m0 + am, kb = k0 + bk;
    if (interior && k0 + BKL <= K) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        ra[q] = gload4(A + (size_t)i * lda + k0 + ak + 4 * q);
        rb[q] = gload4(B + (size_t)kb * ldb + n0 + bj + 4 * q);
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = k0 + ak + 4 * q;
      ra[q] = load4(A + (size_t)i * lda + k, i < M ? K - k : 0, a_al);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = n0 + bj + 4 * q;
      rb[q] = load4(B + (size_t)kb * ldb + j, kb < K ? N - j : 0, b_al);
    }
  };
  auto sstore = [&](int buf) {
    // k = ak + 4 q + {0, 1, 2, 3}: even k to [row][0][kk], odd k to [row][1][kk]
    float* a = &As[buf][am * LDAL + ak / 2];
#pragma unroll
    for (int q = 0; q < NQ; q += 2) {
      *reinterpret_cast<float4*>(a + 2 * q) =
          make_float4(ra[q].x, ra[q].z, ra[q + 1].x, ra[q + 1].z);
      *reinterpret_cast<float4*>(a + BKL / 2 + 2 * q) =
          make_float4(ra[q].y, ra[q].w, ra[q + 1].y, ra[q + 1].w);
    }
    float* b = &Bs[buf][bk * LDBL + bj];
#pragma unroll
    for (int q = 0; q < NQ; ++q) *reinterpret_cast<float4*>(b + 4 * q) = rb[q];
  };

  floatx16 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.f;

  const int h = lane >> 5, l32 = lane & 31;
  const int nk = (K + BKL - 1) / BKL;
  if (nk > 0) {
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) gload((kt + 1) * BKL);
      const float* as = As[buf];
      const float* bs = Bs[buf];
#pragma unroll
      for (int c = 0; c < BKL / 8; ++c) {          // four k-steps (k = 8c .. 8c + 7)
        float4 av[2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
          av[x] = *reinterpret_cast<const float4*>(&as[(wm + 32 * x + l32) * LDAL + (BKL / 2) * h + 4 * c]);
#pragma unroll
        for (int pp = 0; pp < 4; ++pp) {
          const int kr = 2 * (4 * c + pp) + h;
          float bv[2];
#pragma unroll
          for (int y = 0; y < 2; ++y) bv[y] = bs[kr * LDBL + wn + 32 * y + l32];
#pragma unroll
          for (int x = 0; x < 2; ++x) {
            const float a = pp == 0 ? av[x].x : pp == 1 ? av[x].y : pp == 2 ? av[x].z : av[x].w;
#pragma unroll
            for (int y = 0; y < 2; ++y)
              acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv[y], acc[x][y], 0, 0, 0);
          }
        }
      }
      if (kt + 1 < nk) sstore(buf ^ 1);
      __syncthreads();
    }
  }

  // epilogue: element (i, j) of a 32 x 32 block lives in lane j + 32 ((i / 4) % 2),
  // register (i % 4) + 4 (i / 8)
  const GLOBAL int8_t* sfield = nullptr;
  int sbnd = 1;
  if ((MODE == GM_WRAP || MODE == GM_FLUSH) && args.scale_slice >= 0) {
    sfield = gp(e.field + (size_t)args.scale_slice * e.n_sites);
    sbnd = (args.scale_slice == 0 || args.scale_slice == args.n_bulk_last + 1) ? 0 : 1;
  }
  const bool inv = args.scale_inverse != 0;
  // the tile's row factors d(i) and column factors 1/d(j), staged once in LDS
  // (the A buffer is free after the last k-tile's barrier)
  float* drow = As[0];
  float* dcol = As[0] + kTileL;
  if (sfield) {
    if (tid < kTileL) {
      const int i = m0 + tid;
      drow[tid] = i < M ? (float)dfac(e.dval, sbnd, sfield[i], inv) : 0.f;
    } else {
      const int j = n0 + tid - kTileL;
      dcol[tid - kTileL] = j < N ? (float)dfac(e.dval, sbnd, sfield[j], !inv) : 0.f;
    }
    __syncthreads();
  }
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const int jl = wn + 32 * y + l32, j = n0 + jl;
    const float dj = sfield ? dcol[jl] : 1.f;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      // FLUSH: the block's old values of C, all sixteen loads in flight
      float cold[16];
      if (MODE == GM_FLUSH) {
        const GLOBAL float* __restrict__ C0 = gp((const float*)e.C[0]);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = m0 + wm + 32 * x + 8 * (r >> 2) + 4 * h + (r & 3);
          cold[r] = (i < M && j < N) ? C0[(size_t)i * ldc + j] : 0.f;
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int il = wm + 32 * x + 8 * (r >> 2) + 4 * h + (r & 3), i = m0 + il;
        if (i < M && j < N) {
          const size_t o = (size_t)i * ldc + j;
          float v = MODE == GM_FLUSH ? cold[r] - acc[x][y][r] : acc[x][y][r];
          if (sfield) v *= drow[il] * dj;
          if (MODE == GM_FLUSH)
            gp((float*)e.C[1])[o] = v;
          else
            C[o] = v;
        }
      }
    }
  }
}

hipError_t launch_gemm_l(int mode, const GemmEntry* e, const TileRef* t, int n, GemmArgs a,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (mode == GM_STORE)
    hipLaunchKernelGGL(k_gemm_l<GM_STORE>, dim3(n), dim3(kThreads), 0, s, e, t, n, a);
  else if (mode == GM_WRAP)
    hipLaunchKernelGGL(k_gemm_l<GM_WRAP>, dim3(n), dim3(kThreads), 0, s, e, t, n, a);
  else if (mode == GM_FLUSH)
    hipLaunchKernelGGL(k_gemm_l<GM_FLUSH>, dim3(n), dim3(kThreads), 0, s, e, t, n, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Large-tile FP64 GEMM (modes STORE and WRAP; it serves the FP64 scaled wrap,
// where it measured faster than the 64 x 64 kernel): 128 x 128 output tile per
// workgroup, 64 x 64 per wave as 4 x 4 blocks of
// v_mfma_f64_16x16x4f64, k-tiles of 16 double-buffered in LDS with the next
// k-tile prefetched into registers.  A is kept in LDS with each row's k values
// split by k mod 4 (k = 4 s + kq at [row][kq][s]), so a lane fetches the A
// operand of two MFMA k-steps with one 128-bit read; B stays row-major.
// ---------------------------------------------------------------------------
constexpr int BKD = 16;
// the factor staging is ordered by the k-loop's first barrier; with no k-loop
// (K = 0) an explicit barrier is needed
__device__ inline bool nk_zero_guard(int K) { return K <= 0; }
constexpr int LDAD = BKD + 2;        // A tile row: 4 groups of 4 (k mod 4), 2 pad
constexpr int LDBD = kTileL + 2;     // B tile row

__device__ inline double2 load2(const GLOBAL double* __restrict__ p, int valid, bool aligned) {
  if (aligned && valid >= 2) return gload2(p);
  double2 v;
  v.x = valid > 0 ? p[0] : 0.0;
  v.y = valid > 1 ? p[1] : 0.0;
  return v;
}

template <int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm_l64(const GemmEntry* __restrict__ ents,
                                                       const TileRef* __restrict__ tiles,
                                                       int n_tiles, GemmArgs args) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid >= n_tiles) return;
  const TileRef tr = tiles[bid];
  const GemmEntry& e = ents[tr.entry];
  const int M = e.M, N = e.N, K = e.dynK ? *e.dynK : e.K;
  const int m0 = tr.tm * kTileL, n0 = tr.tn * kTileL;
  if (m0 >= M || n0 >= N) return;
  const GLOBAL double* __restrict__ A = gp((const double*)e.A[0]);
  const GLOBAL double* __restrict__ B = gp((const double*)e.B[0]);
  GLOBAL double* __restrict__ C = gp((double*)e.C[0]);
  const int lda = e.lda, ldb = e.ldb, ldc = e.ldc;
  const bool a_al = (lda & 1) == 0, b_al = (ldb & 1) == 0;
  // a tile inside the matrices with aligned rows loads its whole k-tiles
  // without bounds checks
  const bool interior = a_al && b_al && m0 + kTileL <= M && n0 + kTileL <= N;

  __shared__ __align__(16) double As[2][kTileL * LDAD];
  __shared__ __align__(16) double Bs[2][BKD * LDBD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  // output scaling (frame change): the tile's row and column factors, staged
  // once (ordered by the first barrier)
  const GLOBAL int8_t* sfield = nullptr;
  int sbnd = 1;
  if (MODE == GM_WRAP && args.scale_slice >= 0) {
    sfield = gp(e.field + (size_t)args.scale_slice * e.n_sites);
    sbnd = (args.scale_slice == 0 || args.scale_slice == args.n_bulk_last + 1) ? 0 : 1;
  }
  const bool inv = args.scale_inverse != 0;
  __shared__ double drow[kTileL], dcol[kTileL];
  if (sfield) {
    if (tid < kTileL) {
      const int i = m0 + tid;
      drow[tid] = i < M ? dfac(e.dval, sbnd, sfield[i], inv) : 0.0;
    } else {
      const int j = n0 + tid - kTileL;
      dcol[tid - kTileL] = j < N ? dfac(e.dval, sbnd, sfield[j], !inv) : 1.0;
    }
  }
  if (nk_zero_guard(K)) __syncthreads();

  // global -> register mapping: A row am, k from ak (8 values); B k-row bk, columns from bj
  const int am = tid >> 1, ak = (tid & 1) * 8;
  const int bk = tid >> 4, bj = (tid & 15) * 8;
  double2 ra[4], rb[4];
  auto gload = [&](int k0) {
    const int i = m0 + am;
    const int kb = k0 + bk;
    if (interior && k0 + BKD <= K) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ra[q] = gload2(A + (size_t)i * lda + k0 + ak + 2 * q);
        rb[q] = gload2(B + (size_t)kb * ldb + n0 + bj + 2 * q);
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + ak + 2 * q;
      ra[q] = load2(A + (size_t)i * lda + k, i < M ? K - k : 0, a_al);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = n0 + bj + 2 * q;
      rb[q] = load2(B + (size_t)kb * ldb + j, kb < K ? N - j : 0, b_al);
    }
  };
  auto sstore = [&](int buf) {
    // k = ak + e, e = 0..7: kq = k & 3, s = k >> 2 (ak is 0 or 8)
    double* a = &As[buf][am * LDAD + ak / 4];
    const double v[8] = {ra[0].x, ra[0].y, ra[1].x, ra[1].y, ra[2].x, ra[2].y, ra[3].x, ra[3].y};
#pragma unroll
    for (int kq = 0; kq < 4; ++kq)
      *reinterpret_cast<double2*>(a + 4 * kq) = make_double2(v[kq], v[4 + kq]);
    double* b = &Bs[buf][bk * LDBD + bj];
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<double2*>(b + 2 * q) = rb[q];
  };

  doublex4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[x][y][r] = 0.0;

  const int kq = lane >> 4, l16 = lane & 15;
  const int nk = (K + BKD - 1) / BKD;
  if (nk > 0) {
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) gload((kt + 1) * BKD);
      const double* as = As[buf];
      const double* bs = Bs[buf];
#pragma unroll
      for (int s = 0; s < BKD / 4; s += 2) {          // two k-steps (k = 4 s + kq, 4 s + 4 + kq)
        double2 av[4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
          av[x] = *reinterpret_cast<const double2*>(&as[(wm + 16 * x + l16) * LDAD + 4 * kq + s]);
#pragma unroll
        for (int ss = 0; ss < 2; ++ss) {
          const int kr = 4 * (s + ss) + kq;
          double bv[4];
#pragma unroll
          for (int y = 0; y < 4; ++y) bv[y] = bs[kr * LDBD + wn + 16 * y + l16];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            const double a = ss == 0 ? av[x].x : av[x].y;
#pragma unroll
            for (int y = 0; y < 4; ++y)
              acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[y], acc[x][y], 0, 0, 0);
          }
        }
      }
      if (kt + 1 < nk) sstore(buf ^ 1);
      __syncthreads();
    }
  }

  // epilogue: element (i, j) of a 16 x 16 block lives in lane j + 16 (i % 4),
  // register i / 4
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    const int jl = wn + 16 * y + l16, j = n0 + jl;
    const double dj = sfield ? dcol[jl] : 1.0;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int il = wm + 16 * x + 4 * r + kq, i = m0 + il;
        if (i < M && j < N) {
          const size_t o = (size_t)i * ldc + j;
          double v = acc[x][y][r];
          if (sfield) v *= drow[il] * dj;
          C[o] = v;
        }
        if (r == 3) __builtin_amdgcn_sched_barrier(0);   // one 16 x 16 block at a time
      }
  }
}

hipError_t launch_gemm_l64(int mode, const GemmEntry* e, const TileRef* t, int n, GemmArgs a,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (mode) {
    case GM_STORE: hipLaunchKernelGGL(k_gemm_l64<GM_STORE>, dim3(n), dim3(kThreads), 0, s, e, t, n, a); break;
    case GM_WRAP: hipLaunchKernelGGL(k_gemm_l64<GM_WRAP>, dim3(n), dim3(kThreads), 0, s, e, t, n, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Basis propagation of the factored engine, C[p^1] = D (A B[p]): A is the
// lattice exponential e^{-+dtau K} (N x N, one copy shared by the chains of a
// lattice, so it stays in L2) and B[p] a factor (N x n, n <= 16 NBC).  One
// workgroup of W waves (8, or 4 for a batch where 128-row tiles would pad
// more rows than 64-row ones) per 16 W rows of the output and all of its n
// columns (no column tiles padded past n); wave w owns rows 16 w .. 16 w + 15
// and the NBC 16-column blocks, MFMA k-steps of 4 over k-tiles of 16.
//
// With every row 16-byte aligned (even N and n), both operands of a k-tile
// go to LDS by direct loads (global_load_lds_dwordx4: no registers, no LDS
// store instructions), two stages, the next k-tile's loads in flight during
// the current one's MFMAs, one barrier per k-tile.  Each load instruction
// places 64 chunks of 16 bytes side by side; the lanes pick their chunks so
// that the operand reads are conflict-free:
//   A stage: [8 pairs of k][16 W rows] (a half-wave reads 16 rows x one pair);
//   B stage: [16 k][8 NBC pairs], rows of 16 NBC doubles (odd NBC:
//   consecutive rows land on opposite bank halves; even NBC: the pair index of
//   odd rows XOR 8).
// Rows past M and k past K load clamped in-range addresses; the A operand is
// zeroed past K and rows past M are not stored.  Otherwise the A operand is
// read straight into registers (k slot g of step s taking k = k0 + 4 g + s)
// and the B k-tiles go through registers into a double-buffered LDS tile.
// ---------------------------------------------------------------------------
#define GLOBAL_V __attribute__((address_space(1))) void
#define LOCAL_V __attribute__((address_space(3))) void
constexpr int kPropSB = 1024 * 2;                     // doubles of a B stage (1024 chunks)

// FULL: every entry of the launch has NBC column blocks (no per-block guard)
template <int NBC, bool FULL, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(W == 8 ? 4 : 3)))
void k_prop(const GemmEntry* __restrict__ ents, const TileRef* __restrict__ tiles, int n_tiles,
            GemmArgs args) {
  constexpr int kPropThreads = 64 * W;
  constexpr int kPropRows = 16 * W;      // output rows per workgroup
  constexpr int kPropSA = 8 * kPropRows * 2;   // doubles of an A stage
  constexpr int kPropStage = kPropSA + kPropSB;
  constexpr int PK = 16;                 // k-tile
  constexpr int LDB = 16 * NBC + 4;      // register path: LDS row of a B k-tile
  constexpr int NPR = 8 * NBC;           // pairs of columns per k row
  constexpr int NPAIR = PK * NPR;        // pairs of a k-tile
  constexpr int PER = (NPAIR + kPropThreads - 1) / kPropThreads;
  constexpr int BI = (NPAIR + kPropThreads - 1) / kPropThreads;   // direct loads of a B stage per wave
  constexpr bool SWZ = (NBC & 1) == 0;
  static_assert(NPAIR <= 1024 && 2 * PK * LDB <= 2 * kPropStage, "stages hold the tiles");
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid >= n_tiles) return;
  const TileRef tr = tiles[bid];
  const GemmEntry& e = ents[tr.entry];
  const int M = e.M, n = e.N, K = e.K, m0 = tr.tm * kPropRows;
  if (m0 >= M) return;
  const int p = args.parity;
  const double* Ap = (const double*)e.A[0];
  const double* Bp = (const double*)e.B[p];
  const GLOBAL double* __restrict__ A = gp(Ap);
  const GLOBAL double* __restrict__ B = gp(Bp);
  GLOBAL double* __restrict__ C = gp((double*)e.C[p ^ 1]);
  const int lda = e.lda, ldb = e.ldb, ldc = e.ldc;
  typedef double v2 __attribute__((ext_vector_type(2)));
  const bool avec = (lda & 1) == 0 && (reinterpret_cast<uintptr_t>(Ap) & 15) == 0;
  const bool bvec = (ldb & 1) == 0 && (reinterpret_cast<uintptr_t>(Bp) & 15) == 0;
  __shared__ __align__(16) double ring[2 * kPropStage];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, g = lane >> 4;
  const int nbc = FULL ? NBC : (n + 15) / 16;
  const int nk = (K + PK - 1) / PK;
  doublex4 acc[NBC];
#pragma unroll
  for (int c = 0; c < NBC; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[c][i] = 0.0;

  if (avec && bvec && (K & 1) == 0 && (n & 1) == 0) {
    // ---- direct-to-LDS path ----
    auto issue = [&](int kt) {
      const int k0 = kt * PK;
      double* st = ring + (kt & 1) * kPropStage;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int c = (wave * 2 + u) * 64;   // chunk base: pair c / 128, rows c % 128 + lane
        const int kp = c / kPropRows, arow = min(m0 + c % kPropRows + lane, M - 1);
        const int kk = min(k0 + 2 * kp, K - 2);
        __builtin_amdgcn_global_load_lds((const GLOBAL_V*)(Ap + (size_t)arow * lda + kk),
                                         (LOCAL_V*)(st + c * 2), 16, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < BI; ++u) {
        const int base = (wave * BI + u) * 64, c = base + lane;
        const int k = c / NPR;
        const int pd = c - k * NPR;
        const int ps = SWZ ? (pd ^ ((k & 1) << 3)) : pd;   // source pair of this slot
        const int kk = min(k0 + k, K - 1), jj = min(2 * ps, n - 2);
        __builtin_amdgcn_global_load_lds((const GLOBAL_V*)(Bp + (size_t)kk * ldb + jj),
                                         (LOCAL_V*)(st + kPropSA + base * 2), 16, 0, 0);
      }
    };
    issue(0);
    for (int kt = 0; kt < nk; ++kt) {
      // this wave's loads of stage kt have landed, then every wave's have; the
      // barrier also ends every wave's reads of the stage the next loads fill
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      if (kt + 1 < nk) issue(kt + 1);
      const double* st = ring + (kt & 1) * kPropStage;
      const int k0 = kt * PK;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = 4 * s4 + g;
        double a = st[((k >> 1) * kPropRows + 16 * wave + l16) * 2 + (k & 1)];
        a = k0 + k < K ? a : 0.0;
        const int bx = SWZ ? ((k & 1) << 4) : 0;
#pragma unroll
        for (int c = 0; c < NBC; ++c)
          if (FULL || c < nbc)
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                a, st[kPropSA + k * 2 * NPR + ((16 * c + l16) ^ bx)], acc[c], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    // ---- register path ----
    double* Bs0 = ring;
    double* Bs1 = ring + PK * LDB;
    const int row = m0 + 16 * wave + l16;
    const bool rok = row < M;
    const GLOBAL double* __restrict__ Ar = A + (size_t)(rok ? row : 0) * lda;
    v2 rbv[PER];
    auto load_b = [&](int kb) {
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * kPropThreads, k = idx / NPR, j = 2 * (idx - k * NPR), kk = kb + k;
        const bool ok = idx < NPAIR && kk < K;
        const GLOBAL double* src = B + (ok ? (size_t)kk * ldb + j : 0);
        if (bvec && ok && j + 1 < n) {
          rbv[u] = *reinterpret_cast<const GLOBAL v2*>(src);
        } else {
          rbv[u] = v2{(ok && j < n) ? src[0] : 0.0, (ok && j + 1 < n) ? src[1] : 0.0};
        }
      }
    };
    auto store_b = [&](double* bs) {
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * kPropThreads, k = idx / NPR, j = 2 * (idx - k * NPR);
        if (idx < NPAIR) *reinterpret_cast<v2*>(&bs[k * LDB + j]) = rbv[u];
      }
    };
    v2 ra[2], rn[2];
    auto load_a = [&](int kb, v2 (&r)[2]) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = kb + 4 * g + 2 * h;
        if (avec && rok && k + 1 < K) {
          r[h] = *reinterpret_cast<const GLOBAL v2*>(Ar + k);
        } else {
          r[h] = v2{(rok && k < K) ? Ar[k] : 0.0, (rok && k + 1 < K) ? Ar[k + 1] : 0.0};
        }
      }
    };
    load_b(0);
    load_a(0, ra);
    store_b(Bs0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      if (kt + 1 < nk) {
        load_b((kt + 1) * PK);
        load_a((kt + 1) * PK, rn);
      }
      const double* bs = (kt & 1) ? Bs1 : Bs0;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const double a = st == 0 ? ra[0].x : st == 1 ? ra[0].y : st == 2 ? ra[1].x : ra[1].y;
#pragma unroll
        for (int c = 0; c < NBC; ++c)
          if (FULL || c < nbc)
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bs[(4 * g + st) * LDB + 16 * c + l16],
                                                          acc[c], 0, 0, 0);
      }
      if (kt + 1 < nk) {
        store_b((kt & 1) ? Bs0 : Bs1);
        ra[0] = rn[0];
        ra[1] = rn[1];
      }
      __syncthreads();
    }
  }
  // epilogue: rows scaled by the slice's D (or D^{-1} for an entry marked sinv)
  const GLOBAL int8_t* sfield =
      args.scale_slice >= 0 ? gp(e.field + (size_t)args.scale_slice * e.n_sites) : nullptr;
  const int sbnd = (args.scale_slice == 0 || args.scale_slice == args.n_bulk_last + 1) ? 0 : 1;
  const bool inv = (args.scale_inverse != 0) != (e.sinv != 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = m0 + 16 * wave + g + 4 * i;
    if (r >= M) continue;
    const double d = sfield ? dfac(e.dval, sbnd, sfield[r], inv) : 1.0;
#pragma unroll
    for (int c = 0; c < NBC; ++c) {
      const int j = 16 * c + l16;
      if (c < nbc && j < n) C[(size_t)r * ldc + j] = acc[c][i] * d;
    }
  }
}

// the factored engine's propagation over a tile list of (entry, row tile);
// nmin, nmax: the fewest and most columns of the launch's factors; rows: the
// output rows of a tile (64 or 128, as the tile list was built)
hipError_t launch_prop(int nmin, int nmax, int rows, const GemmEntry* e, const TileRef* t, int n,
                       GemmArgs a, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nb = (nmax + 15) / 16;
#define LAUNCH_PROP(B, F)                                                                    \
  do {                                                                                       \
    if (rows == 128)                                                                         \
      hipLaunchKernelGGL((k_prop<B, F, 8>), dim3(n), dim3(512), 0, s, e, t, n, a);           \
    else                                                                                     \
      hipLaunchKernelGGL((k_prop<B, F, 4>), dim3(n), dim3(256), 0, s, e, t, n, a);           \
  } while (0)
  if ((nmin + 15) / 16 == nb) {   // every factor has nb column blocks
    switch (nb) {
#define GPQMC_PROP_FULL(B) \
  case B:                  \
    LAUNCH_PROP(B, true);  \
    return hipGetLastError();
      GPQMC_PROP_FULL(1)
      GPQMC_PROP_FULL(2)
      GPQMC_PROP_FULL(3)
      GPQMC_PROP_FULL(4)
      GPQMC_PROP_FULL(5)
      GPQMC_PROP_FULL(6)
      GPQMC_PROP_FULL(7)
      GPQMC_PROP_FULL(8)
#undef GPQMC_PROP_FULL
      default: break;
    }
  }
  if (nb <= 7)
    LAUNCH_PROP(7, false);
  else
    LAUNCH_PROP(8, false);
#undef LAUNCH_PROP
  return hipGetLastError();
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
    case GM_IMABT: return gemm_t<double, GM_IMABT, false, true, double>(e, t, n, a, s);
    case GM_SEGP: return gemm_t<double, GM_SEGP, false, true, double>(e, t, n, a, s);
    case GM_SEGF: return gemm_t<double, GM_SEGF, false, false, double>(e, t, n, a, s);
    case GM_BMAT: return gemm_t<double, GM_BMAT, false, true, double>(e, t, n, a, s);
    case GM_AMAT: return gemm_t<double, GM_AMAT, false, false, double>(e, t, n, a, s);
    case GM_GFRESH2: return gemm_t<double, GM_GFRESH2, false, true, double>(e, t, n, a, s);
    default: break;
  }
  if (fp32) {
    switch (mode) {
      case GM_STORE: return gemm_t<float, GM_STORE, false, false, float>(e, t, n, a, s);
      case GM_WRAP: return gemm_t<float, GM_WRAP, false, false, float>(e, t, n, a, s);
      case GM_FLUSH: return gemm_t<float, GM_FLUSH, false, false, float>(e, t, n, a, s);
      case GM_PROPB: return gemm_t<float, GM_PROPB, false, false, float>(e, t, n, a, s);
      case GM_PROPR: return gemm_t<float, GM_PROPR, false, false, float>(e, t, n, a, s);
    }
  } else {
    switch (mode) {
      case GM_STORE: return gemm_t<double, GM_STORE, false, false, double>(e, t, n, a, s);
      case GM_WRAP: return gemm_t<double, GM_WRAP, false, false, double>(e, t, n, a, s);
      case GM_FLUSH: return gemm_t<double, GM_FLUSH, false, false, double>(e, t, n, a, s);
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
