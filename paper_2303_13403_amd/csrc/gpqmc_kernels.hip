// HIP kernels (gfx950 / CDNA4) of the Gutzwiller-projection PQMC sweep
// (Chang & Li, arXiv:2303.13403: Method section and the Hubbard section).
//
// Kernels of one imaginary-time slice, batched over chains and spins:
//   k_scan        Metropolis proposals for every site of the slice with the
//                 ratio 1 + Delta (1 - G_ii), processed in submatrix blocks of
//                 k sites and accumulated as G0 - G0[:,F] Z (1 - G0)[F,:]
//                 (delayed updates over the whole slice; one workgroup per chain).
//   k_gemm        batched MFMA GEMM with fused epilogues: the delayed-update
//                 flush, the kinetic wrap e^{-dtau K} G e^{dtau K} with the next
//                 slice's diagonal wrap fused, the basis propagation with
//                 e^{V(s_l)} fused, L R, and the fresh Green's function.
//   k_qr          FP64 Householder QR of the propagated N x n basis.
//   k_lu_solve    FP64 LU (partial pivoting) of L R and (L R)^{-1} L.
//   k_finalize    checkpoint bookkeeping: log|det| and sign, drift, stack
//                 store, measurement of E/N and double occupancy at tau = Theta.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gpqmc_internal.h"

namespace gpqmc {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16;        // GEMM k-tile
constexpr int LDS_PAD = 4;    // LDS row padding (elements)

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Map a hardware workgroup id to a logical tile so that consecutive logical
// tiles (the tiles of one chain/spin) land on the same XCD: workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2.
__device__ inline int xcd_remap(int b, int n) {
  if (n < 16) return b;
  const int per = n / 8, rem = n % 8;
  const int x = b % 8, idx = b / 8;
  return (x < rem) ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
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

// D_l diagonal for one site: d = exp(sigma c_b s); inverse uses the flipped field.
__device__ inline double dfac(const double (&dv)[2][2], int b, int8_t s, bool inverse) {
  const int si = (s > 0) ? 0 : 1;
  return dv[b][inverse ? 1 - si : si];
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

// ---------------------------------------------------------------------------
// batched GEMM: C(M x N) = op(A)(M x K) B(K x N), 64 x 64 tile per workgroup,
// k-tiles of 16 staged through LDS with a one-tile register prefetch.
// T: arithmetic type; Tb: bulk type of the secondary output (GM_GFRESH).
// ---------------------------------------------------------------------------
template <typename T, int MODE, bool TRANSA, typename Tb>
__global__ __launch_bounds__(kThreads) void k_gemm(const GemmEntry* __restrict__ ents,
                                                   const TileRef* __restrict__ tiles,
                                                   int n_tiles, GemmArgs args) {
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  if (bid >= n_tiles) return;
  const TileRef tr = tiles[bid];
  const GemmEntry& e = ents[tr.entry];
  int M = e.M, N = e.N, K = e.K;
  if (e.dynMK) {
    const int f = *e.dynMK;
    K = f;
    if (MODE == GM_T1) M = f;
  }
  const int m0 = tr.tm * kTile, n0 = tr.tn * kTile;
  if (m0 >= M || n0 >= N) return;

  const T* A = (const T*)e.A;
  const T* B = (const T*)e.B;
  T* C = (T*)e.C;
  if (MODE == GM_PROPB || MODE == GM_PROPR) {
    B = (const T*)e.Bpp[args.parity];
    C = (T*)e.Cpp[args.parity ^ 1];
  }
  if (MODE == GM_XMAT || MODE == GM_GFRESH) {
    const double* slotp = e.stack + (size_t)args.slot * e.slot_stride;
    const double* R = args.dir == 0 ? e.Qc : slotp;
    const double* Lt = args.dir == 0 ? slotp : e.Qc;
    if (MODE == GM_XMAT) {
      A = (const T*)Lt;
      B = (const T*)R;
    } else {
      A = (const T*)R;
      B = (const T*)e.Ym;
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
    {
      const int k = kbase + (tid >> 4), j = n0 + (tid & 15) * 4;
      T sc = T(1);
      if (bfield && k < K) sc = (T)dfac(e.dval, bbnd, bfield[k], false);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rb[q] = (k < K && j + q < N) ? B[(size_t)k * ldb + j + q] * sc : T(0);
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
    const int k = tid >> 4, j = (tid & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[k * LDS_LD + j + q] = rb[q];
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
  wt.each(wm, wn, lane, [&](int li, int lj, T acc) {
    const int i = m0 + li, j = n0 + lj;
    if (i >= M || j >= N) return;
    const size_t o = (size_t)i * ldc + j;
    if (MODE == GM_STORE || MODE == GM_T1 || MODE == GM_PROPB || MODE == GM_XMAT) {
      C[o] = acc;
    } else if (MODE == GM_PROPR) {
      T v = acc;
      if (sfield) v *= (T)dfac(e.dval, sbnd, sfield[i], false);
      C[o] = v;
    } else if (MODE == GM_WRAP || MODE == GM_FLUSH) {
      T v = (MODE == GM_FLUSH) ? C[o] - acc : acc;
      if (sfield)
        v *= (T)(dfac(e.dval, sbnd, sfield[i], inv) * dfac(e.dval, sbnd, sfield[j], !inv));
      C[o] = v;
    } else if (MODE == GM_GFRESH) {
      const double g = (i == j ? 1.0 : 0.0) - (double)acc;
      C[o] = (T)g;
      Tb* Cb = (Tb*)e.C2;
      const size_t o2 = (size_t)i * e.ldc2 + j;
      if (args.check_drift) {
        const float d = (float)fabs((double)Cb[o2] - g);
        dmax = (d != d) ? __builtin_inff() : fmaxf(dmax, d);
      }
      double v = g;
      if (sfield) v *= dfac(e.dval, sbnd, sfield[i], inv) * dfac(e.dval, sbnd, sfield[j], !inv);
      Cb[o2] = (Tb)v;
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

// ---------------------------------------------------------------------------
// Metropolis scan of one slice (one workgroup per chain, both spins).
//
// G0 is the Green's function in the frame where D_l acts.  The sites are
// visited in ascending order in blocks S of kblk sites.  With F the sites
// accepted so far in this slice (nonzero Delta), the current Green's function
// is G0 - G0[:,F] Z (1 - G0)[F,:]; only the block G[S,S] is formed, the
// proposals of the block are taken with rank-1 updates of that block, and the
// block's coefficient matrix Zb is merged into Z.  The full update is applied
// afterwards by the T1 and FLUSH GEMMs.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan(const ChainDev* __restrict__ chains,
                                                   const Ctl* __restrict__ ctl, int l, int M,
                                                   int kblk) {
  const ChainDev& C = chains[blockIdx.x];
  ChainState* st = C.st;
  const int N = C.N;
  const int tid = threadIdx.x;
  constexpr int KP = kMaxBlock + 1;

  __shared__ double u_s[kMaxSites];
  __shared__ int8_t fs[kMaxSites];
  __shared__ int Fs[kMaxSites];
  __shared__ T Hs[2][kMaxBlock][KP];
  __shared__ T Gt[2][kMaxBlock][KP];
  __shared__ T Zb[2][kMaxBlock][KP];
  __shared__ T colb[2][kMaxBlock], rowb[2][kMaxBlock];
  __shared__ T uvec[2][kMaxBlock + 1], vvec[2][kMaxBlock + 1];
  __shared__ int Fb[kMaxBlock];
  __shared__ int sh_f, sh_fb, sh_sign, sh_acc;

  const int bnd = (l == 0 || l == M + 1) ? 0 : 1;
  int8_t* frow = C.field + (size_t)l * N;
  const uint32_t sweep = (uint32_t)st->sweep;
  const bool force_reject = ctl->force_reject != 0;
  for (int i = tid; i < N; i += kThreads) {
    uint32_t c[4] = {C.chain_id, sweep, (uint32_t)l, (uint32_t)i};
    philox4x32_10(c, C.key0, C.key1);
    u_s[i] = uniform53(c[0], c[1]);
    fs[i] = frow[i];
  }
  if (tid == 0) {
    sh_f = 0;
    sh_sign = st->sign;
    sh_acc = 0;
  }
  const bool zero_delta = C.delta[bnd][0][0] == 0.0 && C.delta[bnd][0][1] == 0.0;
  const T* G0[2] = {(const T*)C.G[0], (const T*)C.G[1]};
  T* Z[2] = {(T*)C.Z[0], (T*)C.Z[1]};
  T* W1[2];
  T* Pm[2];
  T* Qm[2];
  T* PZ[2];
  T* ZQ[2];
  for (int s = 0; s < 2; ++s) {
    T* w = (T*)C.scan_ws[s];
    W1[s] = w;
    Pm[s] = w + (size_t)kMaxBlock * N;
    Qm[s] = w + (size_t)2 * kMaxBlock * N;
    PZ[s] = w + (size_t)3 * kMaxBlock * N;
    ZQ[s] = w + (size_t)4 * kMaxBlock * N;
  }
  __syncthreads();

  for (int b0 = 0; b0 < N; b0 += kblk) {
    const int kb = min(kblk, N - b0);
    const int f = sh_f;
    // W1 = G0[S, F] Z  (kb x f)
    if (f > 0) {
      const int tot = kb * f;
      for (int idx = tid; idx < 2 * tot; idx += kThreads) {
        const int s = idx / tot, r = idx - s * tot, a = r / f, q = r - a * f;
        const T* row = G0[s] + (size_t)(b0 + a) * N;
        const T* zc = Z[s] + q;
        T acc = 0;
        for (int p = 0; p < f; ++p) acc += row[Fs[p]] * zc[(size_t)p * N];
        W1[s][r] = acc;
      }
      __syncthreads();
    }
    // block of the current Green's function: G[S,S] = G0[S,S] + W1 G0[F,S]
    for (int idx = tid; idx < 2 * kb * kb; idx += kThreads) {
      const int s = idx / (kb * kb), r = idx - s * kb * kb, a = r / kb, bb = r - a * kb;
      T acc = G0[s][(size_t)(b0 + a) * N + b0 + bb];
      for (int q = 0; q < f; ++q) acc += W1[s][a * f + q] * G0[s][(size_t)Fs[q] * N + b0 + bb];
      Gt[s][a][bb] = acc;
      Hs[s][a][bb] = acc;
    }
    if (tid == 0) sh_fb = 0;
    __syncthreads();

    for (int j = 0; j < kb; ++j) {
      const int i = b0 + j;
      const int si = fs[i] > 0 ? 0 : 1;
      const double du = C.delta[bnd][0][si], dd = C.delta[bnd][1][si];
      const double ru = 1.0 + du * (1.0 - (double)Gt[0][j][j]);
      const double rd = 1.0 + dd * (1.0 - (double)Gt[1][j][j]);
      const double prob = fabs(ru * rd);
      const bool accept = !force_reject && (u_s[i] < prob);
      if (tid == 0 && C.trace_ratio) {
        C.trace_ratio[((size_t)l * N + i) * 2 + 0] = ru;
        C.trace_ratio[((size_t)l * N + i) * 2 + 1] = rd;
      }
      if (!accept) continue;
      if (!zero_delta) {
        const int fb = sh_fb;
        if (tid < 2 * kb) {
          const int s = tid / kb, a = tid - s * kb;
          colb[s][a] = Gt[s][a][j];
          rowb[s][a] = (a == j ? T(1) : T(0)) - Gt[s][j][a];
        } else if (tid >= 64 && tid < 64 + 2 * (fb + 1)) {
          const int t = tid - 64, s = t / (fb + 1), p = t - s * (fb + 1);
          T uu = (p == fb) ? T(1) : T(0), vv = uu;
          if (p < fb) {
            for (int c = 0; c < fb; ++c) {
              uu += Zb[s][p][c] * Hs[s][Fb[c]][j];
              vv += Zb[s][c][p] * Hs[s][j][Fb[c]];
            }
          }
          uvec[s][p] = uu;
          vvec[s][p] = vv;
        }
        __syncthreads();
        const T coef[2] = {(T)(du / ru), (T)(dd / rd)};
        for (int idx = tid; idx < 2 * kb * kb; idx += kThreads) {
          const int s = idx / (kb * kb), r = idx - s * kb * kb, a = r / kb, bb = r - a * kb;
          Gt[s][a][bb] -= coef[s] * colb[s][a] * rowb[s][bb];
        }
        const int fb1 = fb + 1;
        for (int idx = tid; idx < 2 * fb1 * fb1; idx += kThreads) {
          const int s = idx / (fb1 * fb1), r = idx - s * fb1 * fb1, p = r / fb1, q = r - p * fb1;
          const T base = (p < fb && q < fb) ? Zb[s][p][q] : T(0);
          Zb[s][p][q] = base + coef[s] * uvec[s][p] * vvec[s][q];
        }
        if (tid == 0) {
          Fb[fb] = j;
          sh_fb = fb1;
        }
      }
      if (tid == 0) {
        fs[i] = (int8_t)(-fs[i]);
        if (ru * rd < 0) sh_sign = -sh_sign;
        sh_acc += 1;
      }
      __syncthreads();
    }
    __syncthreads();

    // merge the block's Zb into Z:
    //   Z <- [[Z + P Zb Q, P Zb], [Zb Q, Zb]],  P = Z G0[F,Fb], Q = G0[Fb,F] Z
    const int fb = sh_fb;
    if (fb > 0) {
      if (f > 0) {
        const int tot = f * fb;
        for (int idx = tid; idx < 4 * tot; idx += kThreads) {
          const int s = idx / (2 * tot), r0 = idx - s * 2 * tot;
          if (r0 < tot) {  // P[p][c]
            const int p = r0 / fb, c = r0 - p * fb;
            const int col = b0 + Fb[c];
            T acc = 0;
            for (int q = 0; q < f; ++q) acc += Z[s][(size_t)p * N + q] * G0[s][(size_t)Fs[q] * N + col];
            Pm[s][p * fb + c] = acc;
          } else {         // Q[c][q]
            const int r = r0 - tot, c = r / f, q = r - c * f;
            const T* row = G0[s] + (size_t)(b0 + Fb[c]) * N;
            T acc = 0;
            for (int p = 0; p < f; ++p) acc += row[Fs[p]] * Z[s][(size_t)p * N + q];
            Qm[s][c * f + q] = acc;
          }
        }
        __syncthreads();
        for (int idx = tid; idx < 4 * tot; idx += kThreads) {
          const int s = idx / (2 * tot), r0 = idx - s * 2 * tot;
          if (r0 < tot) {  // PZb[p][c]
            const int p = r0 / fb, c = r0 - p * fb;
            T acc = 0;
            for (int d = 0; d < fb; ++d) acc += Pm[s][p * fb + d] * Zb[s][d][c];
            PZ[s][p * fb + c] = acc;
          } else {         // ZbQ[c][q]
            const int r = r0 - tot, c = r / f, q = r - c * f;
            T acc = 0;
            for (int d = 0; d < fb; ++d) acc += Zb[s][c][d] * Qm[s][d * f + q];
            ZQ[s][c * f + q] = acc;
          }
        }
        __syncthreads();
        for (int idx = tid; idx < 2 * f * f; idx += kThreads) {
          const int s = idx / (f * f), r = idx - s * f * f, p = r / f, q = r - p * f;
          T acc = Z[s][(size_t)p * N + q];
          for (int c = 0; c < fb; ++c) acc += PZ[s][p * fb + c] * Qm[s][c * f + q];
          Z[s][(size_t)p * N + q] = acc;
        }
        for (int idx = tid; idx < 2 * tot; idx += kThreads) {
          const int s = idx / tot, r = idx - s * tot;
          const int p = r / fb, c = r - p * fb;
          Z[s][(size_t)p * N + f + c] = PZ[s][p * fb + c];
          const int c2 = r / f, q = r - c2 * f;
          Z[s][(size_t)(f + c2) * N + q] = ZQ[s][c2 * f + q];
        }
      }
      for (int idx = tid; idx < 2 * fb * fb; idx += kThreads) {
        const int s = idx / (fb * fb), r = idx - s * fb * fb, c = r / fb, d = r - c * fb;
        Z[s][(size_t)(f + c) * N + f + d] = Zb[s][c][d];
      }
      if (tid < fb) Fs[f + tid] = b0 + Fb[tid];
      __syncthreads();
      if (tid == 0) sh_f = f + fb;
      __syncthreads();
    }
  }

  // operands of the flush: Xg = G0[:, F], Yg = (1 - G0)[F, :]
  const int f = sh_f;
  T* Xg[2] = {(T*)C.Xg[0], (T*)C.Xg[1]};
  T* Yg[2] = {(T*)C.Yg[0], (T*)C.Yg[1]};
  for (int idx = tid; idx < 2 * N * f; idx += kThreads) {
    const int s = idx / (N * f), r = idx - s * N * f, i = r / f, p = r - i * f;
    Xg[s][(size_t)i * N + p] = G0[s][(size_t)i * N + Fs[p]];
  }
  for (int idx = tid; idx < 2 * N * f; idx += kThreads) {
    const int s = idx / (N * f), r = idx - s * N * f, p = r / N, j = r - p * N;
    const int site = Fs[p];
    Yg[s][(size_t)p * N + j] = (site == j ? T(1) : T(0)) - G0[s][(size_t)site * N + j];
  }
  for (int i = tid; i < N; i += kThreads) frow[i] = fs[i];
  if (tid == 0) {
    st->fcount = f;
    st->sign = sh_sign;
    st->accepted += sh_acc;
    st->proposed += N;
  }
}

// ---------------------------------------------------------------------------
// FP64 Householder QR of the active basis U (N x n):  U = Q T, Q explicit.
// Reflector j: H = 1 - tau v v^T with v_j = 1, T_jj = beta (LAPACK convention).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_qr(const ChainDev* __restrict__ chains, int parity) {
  const ChainDev& C = chains[blockIdx.x >> 1];
  const int sp = blockIdx.x & 1;
  const int N = C.N, n = C.n[sp];
  double* A = C.Hw[sp];
  double* Q = C.Qc[sp];
  T* U = (T*)C.U[sp][parity];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double tau_s[kMaxSites];
  __shared__ double w_s[kMaxSites];
  __shared__ double red[4];

  for (int idx = tid; idx < N * n; idx += kThreads) A[idx] = (double)U[idx];
  __syncthreads();
  double logabs = 0.0;
  int sgn = 1;
  for (int j = 0; j < n; ++j) {
    double part = 0.0;
    for (int i = j + 1 + tid; i < N; i += kThreads) {
      const double v = A[(size_t)i * n + j];
      part += v * v;
    }
    const double xn2 = block_sum(part, red);
    const double alpha = A[(size_t)j * n + j];
    double beta, tau, scal;
    if (xn2 == 0.0) {
      tau = 0.0;
      beta = alpha;
      scal = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (tid == 0) {
      logabs += log(fabs(beta));
      if (beta < 0) sgn = -sgn;
      tau_s[j] = tau;
    }
    if (tau != 0.0)
      for (int i = j + 1 + tid; i < N; i += kThreads) A[(size_t)i * n + j] *= scal;
    __syncthreads();
    if (tid == 0) A[(size_t)j * n + j] = beta;
    if (tau != 0.0 && j + 1 < n) {
      for (int c = j + 1 + wave; c < n; c += 4) {
        double s = 0.0;
        for (int i = j + 1 + lane; i < N; i += 64) s += A[(size_t)i * n + j] * A[(size_t)i * n + c];
        s = wave_sum(s);
        if (lane == 0) w_s[c] = s + A[(size_t)j * n + c];
      }
      __syncthreads();
      const int nc = n - j - 1;
      for (int idx = tid; idx < (N - j) * nc; idx += kThreads) {
        const int i = j + idx / nc, c = j + 1 + idx % nc;
        const double vi = (i == j) ? 1.0 : A[(size_t)i * n + j];
        A[(size_t)i * n + c] -= tau * vi * w_s[c];
      }
    }
    __syncthreads();
  }
  // Q = H_0 H_1 ... H_{n-1} [1; 0]
  for (int idx = tid; idx < N * n; idx += kThreads) Q[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    if (tau == 0.0) continue;
    for (int c = j + wave; c < n; c += 4) {
      double s = 0.0;
      for (int i = j + lane; i < N; i += 64) {
        const double vi = (i == j) ? 1.0 : A[(size_t)i * n + j];
        s += vi * Q[(size_t)i * n + c];
      }
      s = wave_sum(s);
      if (lane == 0) w_s[c] = s;
    }
    __syncthreads();
    const int nc = n - j;
    for (int idx = tid; idx < (N - j) * nc; idx += kThreads) {
      const int i = j + idx / nc, c = j + idx % nc;
      const double vi = (i == j) ? 1.0 : A[(size_t)i * n + j];
      Q[(size_t)i * n + c] -= tau * vi * w_s[c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < N * n; idx += kThreads) U[idx] = (T)Q[idx];
  if (tid == 0) {
    C.st->chk_log[sp] = logabs;
    C.st->chk_sgn[sp] = sgn;
  }
}

// ---------------------------------------------------------------------------
// FP64 LU with partial pivoting of X = L R (n x n) and Y = X^{-1} L (n x N).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_lu_solve(const ChainDev* __restrict__ chains, int slot,
                                                       int dir) {
  const ChainDev& C = chains[blockIdx.x >> 1];
  const int sp = blockIdx.x & 1;
  const int N = C.N, n = C.n[sp];
  double* X = C.Xm[sp];
  double* Y = C.Ym[sp];
  const double* Lt = dir == 0 ? C.stack[sp] + (size_t)slot * N * n : C.Qc[sp];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int piv_s[kMaxSites];
  __shared__ double rv[4];
  __shared__ int ri[4];
  double logabs = 0.0;
  int sgn = 1;
  bool singular = false;
  for (int j = 0; j < n; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + tid; i < n; i += kThreads) {
      const double v = fabs(X[(size_t)i * n + j]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    __syncthreads();
    if (lane == 0) {
      rv[wave] = best;
      ri[wave] = bi;
    }
    __syncthreads();
    int p = ri[0];
    double pb = rv[0];
    for (int w = 1; w < 4; ++w)
      if (rv[w] > pb || (rv[w] == pb && ri[w] < p)) {
        pb = rv[w];
        p = ri[w];
      }
    if (p != j)
      for (int c = tid; c < n; c += kThreads) {
        const double t = X[(size_t)j * n + c];
        X[(size_t)j * n + c] = X[(size_t)p * n + c];
        X[(size_t)p * n + c] = t;
      }
    if (tid == 0) piv_s[j] = p;
    if (p != j) sgn = -sgn;
    __syncthreads();
    const double d = X[(size_t)j * n + j];
    if (d == 0.0) {
      singular = true;
      break;
    }
    logabs += log(fabs(d));
    if (d < 0) sgn = -sgn;
    for (int i = j + 1 + tid; i < n; i += kThreads) X[(size_t)i * n + j] /= d;
    __syncthreads();
    const int nc = n - j - 1;
    for (int idx = tid; idx < nc * nc; idx += kThreads) {
      const int i = j + 1 + idx / nc, c = j + 1 + idx % nc;
      X[(size_t)i * n + c] -= X[(size_t)i * n + j] * X[(size_t)j * n + c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    C.st->x_log[sp] = logabs;
    C.st->x_sgn[sp] = singular ? 0 : sgn;
    if (singular) atomicOr(&C.st->flags, (int)FLAG_SINGULAR);
  }
  if (singular) return;
  for (int col = tid; col < N; col += kThreads) {
    for (int r = 0; r < n; ++r) Y[(size_t)r * N + col] = Lt[(size_t)col * n + r];
    for (int j = 0; j < n; ++j) {
      const int p = piv_s[j];
      if (p != j) {
        const double t = Y[(size_t)j * N + col];
        Y[(size_t)j * N + col] = Y[(size_t)p * N + col];
        Y[(size_t)p * N + col] = t;
      }
    }
    for (int r = 1; r < n; ++r) {
      double s = Y[(size_t)r * N + col];
      for (int c = 0; c < r; ++c) s -= X[(size_t)r * n + c] * Y[(size_t)c * N + col];
      Y[(size_t)r * N + col] = s;
    }
    for (int r = n - 1; r >= 0; --r) {
      double s = Y[(size_t)r * N + col];
      for (int c = r + 1; c < n; ++c) s -= X[(size_t)r * n + c] * Y[(size_t)c * N + col];
      Y[(size_t)r * N + col] = s / X[(size_t)r * n + r];
    }
  }
}

// ---------------------------------------------------------------------------
// checkpoint bookkeeping (one workgroup per chain)
// mode 0: checkpoint of a pass (sign check, drift);  1: final checkpoint of
// the initialisation (sign := recomputed);  2: store-only (initial stack).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_finalize(const ChainDev* __restrict__ chains,
                                                       const Ctl* __restrict__ ctl, int slot,
                                                       int mode, int measure_here, int ck_index) {
  const ChainDev& C = chains[blockIdx.x];
  ChainState* st = C.st;
  const int N = C.N, tid = threadIdx.x;
  __shared__ double red[4];
  for (int sp = 0; sp < 2; ++sp) {
    const size_t sz = (size_t)N * C.n[sp];
    double* dst = C.stack[sp] + (size_t)slot * sz;
    for (size_t idx = tid; idx < sz; idx += kThreads) dst[idx] = C.Qc[sp][idx];
  }
  if (tid == 0) {
    int wsign = 1;
    for (int sp = 0; sp < 2; ++sp) {
      const double nl = st->run_log[sp] + st->chk_log[sp];
      const int ns = st->run_sgn[sp] * st->chk_sgn[sp];
      if (mode != 2) wsign *= ns * C.slot_sgn[sp][slot] * st->x_sgn[sp];
      C.slot_log[sp][slot] = nl;
      C.slot_sgn[sp][slot] = ns;
      st->run_log[sp] = nl;
      st->run_sgn[sp] = ns;
    }
    if (mode == 1) {
      st->sign = wsign;
    } else if (mode == 0) {
      if (wsign != st->sign) {
        st->sign_mismatch += 1;
        st->flags |= FLAG_SIGN;
        st->sign = wsign;
      }
      const float d = __uint_as_float(st->drift_bits);
      st->last_drift = d;
      if (!(d <= st->max_drift)) st->max_drift = d;
      if (!(d <= ctl->drift_tol)) st->flags |= (d != d || isinf(d)) ? FLAG_NAN : FLAG_DRIFT;
    }
    st->drift_bits = 0u;
  }
  if (mode != 2 && measure_here && ctl->measure) {
    double ek = 0.0, dsum = 0.0;
    for (int idx = tid; idx < N * N; idx += kThreads) {
      const int i = idx / N, j = idx - i * N;
      const double k = C.Khop[idx];
      if (k != 0.0 || i == j)
        ek += k * ((i == j ? 2.0 : 0.0) - C.G64[0][(size_t)j * N + i] - C.G64[1][(size_t)j * N + i]);
    }
    for (int i = tid; i < N; i += kThreads)
      dsum += (1.0 - C.G64[0][(size_t)i * N + i]) * (1.0 - C.G64[1][(size_t)i * N + i]);
    ek = block_sum(ek, red);
    dsum = block_sum(dsum, red);
    if (tid == 0) {
      const int k = st->n_meas;
      if (k < C.meas_cap) {
        C.meas[3 * k + 0] = (double)st->sign;
        C.meas[3 * k + 1] = (ek + C.U_hub * dsum) / N;
        C.meas[3 * k + 2] = dsum / N;
        st->n_meas = k + 1;
      } else {
        st->flags |= FLAG_MEAS_FULL;
      }
    }
  }
  if (mode != 2 && C.trace_green && ck_index >= 0) {
    for (int sp = 0; sp < 2; ++sp) {
      double* dst = C.trace_green + ((size_t)ck_index * 2 + sp) * N * N;
      for (int idx = tid; idx < N * N; idx += kThreads) dst[idx] = C.G64[sp][idx];
    }
    if (tid == 0) C.trace_drift[ck_index] = st->last_drift;
  }
}

// Store the trial orbitals as the basis of a stack slot (log|det| 0, sign +1);
// optionally also start the active basis from them.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_put_trial(const ChainDev* __restrict__ chains, int slot,
                                                        int set_active) {
  const ChainDev& C = chains[blockIdx.x];
  const int tid = threadIdx.x;
  for (int sp = 0; sp < 2; ++sp) {
    const size_t sz = (size_t)C.N * C.n[sp];
    double* dst = C.stack[sp] + (size_t)slot * sz;
    T* u = (T*)C.U[sp][0];
    for (size_t idx = tid; idx < sz; idx += kThreads) {
      const double v = C.P[sp][idx];
      dst[idx] = v;
      if (set_active) u[idx] = (T)v;
    }
  }
  if (tid == 0) {
    for (int sp = 0; sp < 2; ++sp) {
      C.slot_log[sp][slot] = 0.0;
      C.slot_sgn[sp][slot] = 1;
      if (set_active) {
        C.st->run_log[sp] = 0.0;
        C.st->run_sgn[sp] = 1;
      }
    }
  }
}

// U <- D_l U on a boundary slice (no kinetic factor), both spins.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dscale_u(const ChainDev* __restrict__ chains, int l,
                                                       int M, int parity) {
  const ChainDev& C = chains[blockIdx.x];
  const int b = (l == 0 || l == M + 1) ? 0 : 1;
  const int8_t* frow = C.field + (size_t)l * C.N;
  for (int sp = 0; sp < 2; ++sp) {
    const int n = C.n[sp];
    T* u = (T*)C.U[sp][parity];
    for (int idx = threadIdx.x; idx < C.N * n; idx += kThreads) {
      const int i = idx / n;
      u[idx] *= (T)C.dval[b][sp][frow[i] > 0 ? 0 : 1];
    }
  }
}

__global__ void k_pass_end(const ChainDev* __restrict__ chains) {
  if (threadIdx.x == 0) chains[blockIdx.x].st->sweep += 1;
}

__global__ void k_set_ctl(Ctl* ctl, int measure, int force_reject, float drift_tol) {
  if (threadIdx.x == 0) {
    ctl->measure = measure;
    ctl->force_reject = force_reject;
    ctl->drift_tol = drift_tol;
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename T, int MODE, bool TA, typename Tb>
static hipError_t gemm_t(const GemmEntry* e, const TileRef* t, int n, GemmArgs a, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gemm<T, MODE, TA, Tb>), dim3(n), dim3(kThreads), 0, s, e, t, n, a);
  return hipGetLastError();
}

hipError_t launch_gemm(int bulk_fp32, int mode, const GemmEntry* e, const TileRef* t, int n,
                       GemmArgs a, hipStream_t s) {
  if (bulk_fp32) {
    switch (mode) {
      case GM_STORE: return gemm_t<float, GM_STORE, false, float>(e, t, n, a, s);
      case GM_WRAP: return gemm_t<float, GM_WRAP, false, float>(e, t, n, a, s);
      case GM_FLUSH: return gemm_t<float, GM_FLUSH, false, float>(e, t, n, a, s);
      case GM_PROPB: return gemm_t<float, GM_PROPB, false, float>(e, t, n, a, s);
      case GM_PROPR: return gemm_t<float, GM_PROPR, false, float>(e, t, n, a, s);
      case GM_T1: return gemm_t<float, GM_T1, false, float>(e, t, n, a, s);
      case GM_XMAT: return gemm_t<double, GM_XMAT, true, float>(e, t, n, a, s);
      case GM_GFRESH: return gemm_t<double, GM_GFRESH, false, float>(e, t, n, a, s);
    }
  } else {
    switch (mode) {
      case GM_STORE: return gemm_t<double, GM_STORE, false, double>(e, t, n, a, s);
      case GM_WRAP: return gemm_t<double, GM_WRAP, false, double>(e, t, n, a, s);
      case GM_FLUSH: return gemm_t<double, GM_FLUSH, false, double>(e, t, n, a, s);
      case GM_PROPB: return gemm_t<double, GM_PROPB, false, double>(e, t, n, a, s);
      case GM_PROPR: return gemm_t<double, GM_PROPR, false, double>(e, t, n, a, s);
      case GM_T1: return gemm_t<double, GM_T1, false, double>(e, t, n, a, s);
      case GM_XMAT: return gemm_t<double, GM_XMAT, true, double>(e, t, n, a, s);
      case GM_GFRESH: return gemm_t<double, GM_GFRESH, false, double>(e, t, n, a, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_plain(int fp32, int transA, const GemmEntry* e, const TileRef* t, int n,
                             GemmArgs a, hipStream_t s) {
  if (fp32) return transA ? gemm_t<float, GM_STORE, true, float>(e, t, n, a, s)
                          : gemm_t<float, GM_STORE, false, float>(e, t, n, a, s);
  return transA ? gemm_t<double, GM_STORE, true, double>(e, t, n, a, s)
                : gemm_t<double, GM_STORE, false, double>(e, t, n, a, s);
}

hipError_t launch_scan(int fp32, const ChainDev* c, int nc, const Ctl* ctl, int l, int M, int kblk,
                       hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_scan<float>, dim3(nc), dim3(kThreads), 0, s, c, ctl, l, M, kblk);
  else
    hipLaunchKernelGGL(k_scan<double>, dim3(nc), dim3(kThreads), 0, s, c, ctl, l, M, kblk);
  return hipGetLastError();
}

hipError_t launch_qr(int fp32, const ChainDev* c, int nc, int parity, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_qr<float>, dim3(2 * nc), dim3(kThreads), 0, s, c, parity);
  else
    hipLaunchKernelGGL(k_qr<double>, dim3(2 * nc), dim3(kThreads), 0, s, c, parity);
  return hipGetLastError();
}

hipError_t launch_lu_solve(const ChainDev* c, int nc, int slot, int dir, hipStream_t s) {
  hipLaunchKernelGGL(k_lu_solve, dim3(2 * nc), dim3(kThreads), 0, s, c, slot, dir);
  return hipGetLastError();
}

hipError_t launch_finalize(const ChainDev* c, int nc, const Ctl* ctl, int slot, int mode,
                           int measure_here, int ck_index, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(nc), dim3(kThreads), 0, s, c, ctl, slot, mode, measure_here,
                     ck_index);
  return hipGetLastError();
}

hipError_t launch_put_trial(int fp32, const ChainDev* c, int nc, int slot, int set_active,
                            hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_put_trial<float>, dim3(nc), dim3(kThreads), 0, s, c, slot, set_active);
  else
    hipLaunchKernelGGL(k_put_trial<double>, dim3(nc), dim3(kThreads), 0, s, c, slot, set_active);
  return hipGetLastError();
}

hipError_t launch_dscale_u(int fp32, const ChainDev* c, int nc, int l, int M, int parity,
                           hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_dscale_u<float>, dim3(nc), dim3(kThreads), 0, s, c, l, M, parity);
  else
    hipLaunchKernelGGL(k_dscale_u<double>, dim3(nc), dim3(kThreads), 0, s, c, l, M, parity);
  return hipGetLastError();
}

hipError_t launch_pass_end(const ChainDev* c, int nc, hipStream_t s) {
  hipLaunchKernelGGL(k_pass_end, dim3(nc), dim3(64), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_set_ctl(Ctl* ctl, int measure, int force_reject, float drift_tol, hipStream_t s) {
  hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, s, ctl, measure, force_reject, drift_tol);
  return hipGetLastError();
}

}  // namespace gpqmc
