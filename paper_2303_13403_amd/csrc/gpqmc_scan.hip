// Metropolis scan of one segment of one imaginary-time slice and the delayed-
// update flush that follows it (gfx950).
//
// One workgroup per chain handles both spins.  G0 is the chain's current
// Green's function in the frame where D_l acts, so flipping s_{l,i} changes the
// weight by r_sigma = 1 + Delta_sigma (1 - G_ii) (determinant lemma) and is
// accepted iff u < |r_up r_dn| (Metropolis on the absolute weight).
//
// The segment's sites [s0, s1) are visited in ascending order in submatrix
// blocks S of up to kBlock sites.  With F the sites accepted so far in the
// segment (nonzero Delta only), the current Green's function is
//     G = G0 - G0[:,F] Z (1 - G0)[F,:]                                    (*)
// so only the block G[S,S] is formed; the block's proposals are taken by one
// wave with rank-1 (Sherman-Morrison) updates of that block while it builds
// the block's own coefficient matrix Zb, which is then merged into Z:
//     Z <- [[Z + P Zb Q, P Zb], [Zb Q, Zb]],  P = Z G0[F,Fb], Q = G0[Fb,F] Z.
// The kernel ends by writing F, Z and Yg = (1 - G0)[F,:]; k_wmat forms
// Wg = G0[:,F] Z and k_flush applies (*) = G0 - Wg Yg to the whole Green's
// function (a delayed update of rank |F|).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "gpqmc_device.h"

namespace gpqmc {

// value of x held by lane src (src uniform across the wave)
__device__ inline float lane_value(float x, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}
__device__ inline double lane_value(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// one 128-bit LDS chunk (4 floats or 2 doubles) into registers
template <typename T>
__device__ inline void lds_chunk_load(T (&r)[16 / sizeof(T)], const T* p) {
  using V4 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  const V4 v = *reinterpret_cast<const V4*>(p);
  const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
  for (int t = 0; t < (int)(16 / sizeof(T)); ++t) r[t] = e[t];
}

// whole kBlock-long LDS row <-> registers with 128-bit accesses
template <typename T>
__device__ inline void lds_row_load(T (&r)[kBlock], const T* p) {
  constexpr int V = 16 / sizeof(T);
  using V4 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
#pragma unroll
  for (int q = 0; q < kBlock; q += V) {
    const V4 v = *reinterpret_cast<const V4*>(p + q);
    const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
    for (int t = 0; t < V; ++t) r[q + t] = e[t];
  }
}
template <typename T>
__device__ inline void lds_row_store(T* p, const T (&r)[kBlock]) {
  constexpr int V = 16 / sizeof(T);
  using V4 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
#pragma unroll
  for (int q = 0; q < kBlock; q += V) {
    V4 v;
    T* e = reinterpret_cast<T*>(&v);
#pragma unroll
    for (int t = 0; t < V; ++t) e[t] = r[q + t];
    *reinterpret_cast<V4*>(p + q) = v;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_scan(const ChainDev* __restrict__ chains,
                                                   const Ctl* __restrict__ ctl, int l, int M,
                                                   int s0, int s1) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  ChainState* st = C.st;
  const int N = C.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (s0 >= N) {   // uneven batch: this chain has no site in the segment
    if (tid == 0) st->fcount = 0;
    return;
  }
  const int send = min(s1, N), nseg = send - s0;
  constexpr int KL = kBlock + (16 / sizeof(T));
  constexpr int LDZ = kSegMax;

  __shared__ double u_s[kSegMax];
  __shared__ int8_t fs[kSegMax];
  __shared__ int Fs[kSegMax];
  // block matrices, row-major with a 16-byte aligned leading dimension so a
  // lane can read a whole row with 128-bit loads; Hs = G[S,S] at block start,
  // HsT its transpose, Zs the block's coefficient matrix indexed by block site
  __shared__ __align__(16) T Hs[2][kBlock][KL];
  __shared__ __align__(16) T HsT[2][kBlock][KL];
  __shared__ __align__(16) T Zs[2][kBlock][KL];
  __shared__ __align__(16) T rowbuf[2][kBlock], uvec[2][kBlock], vvec[2][kBlock];
  __shared__ T Rsf[kBlock * kSegMax];
  __shared__ int Fb[kBlock];
  __shared__ int sh_f, sh_fb, sh_sign, sh_acc;

  const int bnd = (l == 0 || l == M + 1) ? 0 : 1;
  int8_t* frow = C.field + (size_t)l * N;
  const uint32_t sweep = (uint32_t)st->sweep;
  const bool force_reject = ctl->force_reject != 0;
  for (int i = tid; i < nseg; i += kThreads) {
    uint32_t c[4] = {C.chain_id, sweep, (uint32_t)l, (uint32_t)(s0 + i)};
    philox4x32_10(c, C.key0, C.key1);
    u_s[i] = uniform53(c[0], c[1]);
    fs[i] = frow[s0 + i];
  }
  if (tid == 0) {
    sh_f = 0;
    sh_sign = st->sign;
    sh_acc = 0;
  }
  const bool zero_delta = C.delta[bnd][0][0] == 0.0 && C.delta[bnd][0][1] == 0.0;
  const T* G0[2] = {(const T*)C.G[0], (const T*)C.G[1]};
  T* Z[2] = {(T*)C.Z[0], (T*)C.Z[1]};
  T *W1[2], *Pm[2], *Qm[2], *PZ[2], *ZQ[2];
  for (int s = 0; s < 2; ++s) {
    T* w = (T*)C.scan_ws[s];
    const size_t blk = (size_t)kBlock * kSegMax;
    W1[s] = w;            // kb x f       (ld LDZ)
    Pm[s] = w + blk;      // f x fb       (ld kBlock)
    Qm[s] = w + 2 * blk;  // fb x f       (ld LDZ)
    PZ[s] = w + 3 * blk;  // f x fb       (ld kBlock)
    ZQ[s] = w + 4 * blk;  // fb x f       (ld LDZ)
  }
  __syncthreads();

  for (int b0 = s0; b0 < send; b0 += kBlock) {
    const int kb = min(kBlock, send - b0);
    const int f = sh_f;
    // ---- W1 = G0[S, F] Z  (kb x f), one spin at a time through LDS ----
    if (f > 0) {
      for (int s = 0; s < 2; ++s) {
        for (int a = wave; a < kb; a += 4)
          for (int p = lane; p < f; p += 64) Rsf[a * f + p] = G0[s][(size_t)(b0 + a) * N + Fs[p]];
        __syncthreads();
        for (int q = tid; q < f; q += kThreads) {
          T acc[kBlock];
#pragma unroll
          for (int a = 0; a < kBlock; ++a) acc[a] = T(0);
          for (int p = 0; p < f; ++p) {
            const T z = Z[s][(size_t)p * LDZ + q];
#pragma unroll
            for (int a = 0; a < kBlock; ++a)
              if (a < kb) acc[a] += Rsf[a * f + p] * z;
          }
#pragma unroll
          for (int a = 0; a < kBlock; ++a)
            if (a < kb) W1[s][(size_t)a * LDZ + q] = acc[a];
        }
        __syncthreads();
      }
    }
    // ---- block of the current Green's function: G[S,S] = G0[S,S] + W1 G0[F,S] ----
    // rows (spin, a) over waves and lane halves, columns over lanes 0..31
    {
      const int half = lane >> 5, c = lane & 31;
      for (int row = 2 * wave + half; row < 2 * kb; row += 8) {
        const int s = row >= kb ? 1 : 0, a = row - s * kb;
        if (c < kb) {
          T acc = G0[s][(size_t)(b0 + a) * N + b0 + c];
          for (int q = 0; q < f; ++q)
            acc += W1[s][(size_t)a * LDZ + q] * G0[s][(size_t)Fs[q] * N + b0 + c];
          Hs[s][a][c] = acc;
          HsT[s][c][a] = acc;
        } else {
          Hs[s][a][c] = T(0);
          HsT[s][c][a] = T(0);
        }
      }
      // rows kb..31 of a ragged last block are zero
      if (kb < kBlock)
        for (int row = 2 * wave + half; row < 2 * kBlock; row += 8) {
          const int s = row >> 5, a = row & 31;
          if (a >= kb) {
            Hs[s][a][c] = T(0);
            HsT[s][c][a] = T(0);
          }
        }
    }
    __syncthreads();

    // ---- sequential proposals of the block: one wave, registers ----
    // lane = (spin s, block row a) holds row a of the current block of G (g),
    // and row a / column a of the block coefficient matrix (zr / zc), which
    // is indexed by block site and stays zero on sites not yet accepted.  For
    // an accepted site j with ratio r and coefficient c = Delta / r:
    //   u = e_j + Zs H[:,j],  v = e_j + Zs^T H[j,:]^T,  Zs += c u v^T
    //   G[S,S] -= c G[S,j] (e_j - G[j,S])            (Sherman-Morrison)
    if (wave == 0) {
      constexpr int VW = 16 / sizeof(T);
      const int s = lane >> 5, a = lane & 31;
      T g[kBlock], zr[kBlock], zc[kBlock];
      lds_row_load(g, &Hs[s][a][0]);
#pragma unroll
      for (int q = 0; q < kBlock; ++q) zr[q] = zc[q] = T(0);
      int fb = 0, sign = sh_sign, nacc = 0;
#pragma unroll
      for (int j = 0; j < kBlock; ++j) {
        if (j < kb) {
          const int li = b0 + j - s0;
          const int si = fs[li] > 0 ? 0 : 1;
          const double du = C.delta[bnd][0][si], dd = C.delta[bnd][1][si];
          const double ru = 1.0 + du * (1.0 - (double)lane_value(g[j], j));
          const double rd = 1.0 + dd * (1.0 - (double)lane_value(g[j], 32 + j));
          const bool accept = !force_reject && (u_s[li] < fabs(ru * rd));
          if (lane == 0 && C.trace_ratio) {
            C.trace_ratio[((size_t)l * N + b0 + j) * 2 + 0] = ru;
            C.trace_ratio[((size_t)l * N + b0 + j) * 2 + 1] = rd;
          }
          if (accept) {
            if (!zero_delta) {
              if (a == j) lds_row_store(&rowbuf[s][0], g);
              T uu = (a == j) ? T(1) : T(0), vv = uu;
#pragma unroll
              for (int c = 0; c < kBlock; c += VW) {
                T hc[VW], hr[VW];
                lds_chunk_load(hc, &HsT[s][j][c]);
                lds_chunk_load(hr, &Hs[s][j][c]);
#pragma unroll
                for (int t = 0; t < VW; ++t) {
                  uu += zr[c + t] * hc[t];
                  vv += zc[c + t] * hr[t];
                }
              }
              uvec[s][a] = uu;
              vvec[s][a] = vv;
              wave_sync();
              const T coef = (T)((s == 0 ? du : dd) / (s == 0 ? ru : rd));
              const T cc = coef * g[j], cu = coef * uu, cv = coef * vv;
#pragma unroll
              for (int q = 0; q < kBlock; q += VW) {
                T rb[VW], ub[VW], vb[VW];
                lds_chunk_load(rb, &rowbuf[s][q]);
                lds_chunk_load(ub, &uvec[s][q]);
                lds_chunk_load(vb, &vvec[s][q]);
#pragma unroll
                for (int t = 0; t < VW; ++t) {
                  g[q + t] -= cc * ((q + t == j ? T(1) : T(0)) - rb[t]);
                  zr[q + t] += cu * vb[t];
                  zc[q + t] += cv * ub[t];
                }
              }
              if (lane == 0) Fb[fb] = j;
              fb += 1;
              wave_sync();
            }
            if (lane == 0) fs[li] = (int8_t)(-fs[li]);
            if (ru * rd < 0) sign = -sign;
            nacc += 1;
          }
        }
      }
      lds_row_store(&Zs[s][a][0], zr);
      if (lane == 0) {
        sh_fb = fb;
        sh_sign = sign;
        sh_acc += nacc;
      }
    }
    __syncthreads();

    // ---- merge the block's coefficients Zb = Zs[Fb,Fb] into Z ----
    //   Z <- [[Z + P Zb Q, P Zb], [Zb Q, Zb]],  P = Z G0[F,Fb], Q = G0[Fb,F] Z
    const int fb = sh_fb;
    if (fb > 0) {
      if (f > 0) {
        for (int s = 0; s < 2; ++s) {
          // P (f x fb): rows over waves, columns over lanes; Q (fb x f) likewise
          for (int p = wave; p < f; p += 4)
            for (int c = lane; c < fb; c += 64) {
              const int col = b0 + Fb[c];
              T acc = 0;
              for (int q = 0; q < f; ++q) acc += Z[s][(size_t)p * LDZ + q] * G0[s][(size_t)Fs[q] * N + col];
              Pm[s][p * kBlock + c] = acc;
            }
          for (int c = wave; c < fb; c += 4) {
            const T* row = G0[s] + (size_t)(b0 + Fb[c]) * N;
            for (int q = lane; q < f; q += 64) {
              T acc = 0;
              for (int p = 0; p < f; ++p) acc += row[Fs[p]] * Z[s][(size_t)p * LDZ + q];
              Qm[s][c * LDZ + q] = acc;
            }
          }
        }
        __syncthreads();
        for (int s = 0; s < 2; ++s) {
          for (int p = wave; p < f; p += 4)
            for (int c = lane; c < fb; c += 64) {
              T acc = 0;
              for (int d = 0; d < fb; ++d) acc += Pm[s][p * kBlock + d] * Zs[s][Fb[d]][Fb[c]];
              PZ[s][p * kBlock + c] = acc;
            }
          for (int c = wave; c < fb; c += 4)
            for (int q = lane; q < f; q += 64) {
              T acc = 0;
              for (int d = 0; d < fb; ++d) acc += Zs[s][Fb[c]][Fb[d]] * Qm[s][d * LDZ + q];
              ZQ[s][c * LDZ + q] = acc;
            }
        }
        __syncthreads();
        for (int s = 0; s < 2; ++s) {
          for (int p = wave; p < f; p += 4)
            for (int q = lane; q < f; q += 64) {
              T acc = Z[s][(size_t)p * LDZ + q];
              for (int c = 0; c < fb; ++c) acc += PZ[s][p * kBlock + c] * Qm[s][c * LDZ + q];
              Z[s][(size_t)p * LDZ + q] = acc;
            }
          for (int p = wave; p < f; p += 4)
            for (int c = lane; c < fb; c += 64) Z[s][(size_t)p * LDZ + f + c] = PZ[s][p * kBlock + c];
          for (int c = wave; c < fb; c += 4)
            for (int q = lane; q < f; q += 64) Z[s][(size_t)(f + c) * LDZ + q] = ZQ[s][c * LDZ + q];
        }
      }
      for (int s = 0; s < 2; ++s)
        for (int c = wave; c < fb; c += 4)
          for (int d = lane; d < fb; d += 64) Z[s][(size_t)(f + c) * LDZ + f + d] = Zs[s][Fb[c]][Fb[d]];
      if (tid < fb) Fs[f + tid] = b0 + Fb[tid];
      __syncthreads();
      if (tid == 0) sh_f = f + fb;
      __syncthreads();
    }
  }

  // operands of the flush: the accepted sites F and Yg = (1 - G0)[F, :]
  // (rows of G0 gathered eight at a time so the loads are issued together)
  const int f = sh_f;
  for (int p = tid; p < f; p += kThreads) C.flist[p] = Fs[p];
  for (int s = 0; s < 2; ++s) {
    T* __restrict__ Yg = (T*)C.Yg[s];
    for (int p0 = 8 * wave; p0 < f; p0 += 32) {
      for (int j0 = 0; j0 < N; j0 += 64) {
        const int j = j0 + lane;
        T v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r)
          v[r] = (p0 + r < f && j < N) ? G0[s][(size_t)Fs[p0 + r] * N + j] : T(0);
#pragma unroll
        for (int r = 0; r < 8; ++r)
          if (p0 + r < f && j < N) Yg[(size_t)(p0 + r) * N + j] = (Fs[p0 + r] == j ? T(1) : T(0)) - v[r];
      }
    }
  }
  for (int i = tid; i < nseg; i += kThreads) frow[s0 + i] = fs[i];
  if (tid == 0) {
    st->fcount = f;
    st->sign = sh_sign;
    st->accepted += sh_acc;
    st->proposed += nseg;
  }
}

// Delayed-update flush of one segment:
//   G <- D (G0 - Wg Yg) D^{-1}      (scaling optional; Wg = G0[:,F] Z from k_wmat)
// One workgroup updates kFlushRows rows of one chain and spin; each wave takes
// 64 columns per pass (two 32-column halves on FP32 MFMA, 2 x 4 blocks of
// 16 x 16 on FP64 MFMA).  The only dependent load is the accepted count: the
// block of G, the rows of Wg and the rows of Yg are issued together.
// Grid: chains x 2 spins x row blocks.
constexpr int kFlushRows = 32;

template <typename T>
__device__ __forceinline__ void flush_body(const ChainDev* __restrict__ chains, int nrb,
                                           int scale_slice, int scale_inverse, int M, int to_tmp) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int cs = b / nrb, rb = b - cs * nrb;
  const int spin = cs & 1;
  const ChainDev& C = chains[cs >> 1];
  const int N = C.N, i0 = rb * kFlushRows;
  if (i0 >= N) return;
  constexpr int KS = sizeof(T) == 4 ? 2 : 4;           // MFMA k-step
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T* __restrict__ G = (const T*)C.G[spin];
  // the result goes back into G; to_tmp (kernel timing) sends it to Gtmp
  T* __restrict__ Gout = to_tmp ? (T*)C.Gtmp[spin] : (T*)C.G[spin];
  const T* __restrict__ W = (const T*)C.Wg[spin];
  const T* __restrict__ Yg = (const T*)C.Yg[spin];
  const int f = C.st->fcount;
  if (f == 0 && scale_slice < 0) return;

  constexpr int NG = 32;                                // G elements per lane and pass
  T gpre[NG];
  auto g_index = [&](int cb, int e, int& i, int& j) {
    if constexpr (sizeof(T) == 4) {
      // element (i, j) of a 32 x 32 block of v_mfma_f32_32x32x2f32 lives in
      // lane j + 32 ((i / 4) % 2), register (i % 4) + 4 (i / 8); e = 16 half + register
      const int r = e & 15;
      i = i0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      j = cb + 32 * (e >> 4) + (lane & 31);
    } else {
      // element (i, j) of a 16 x 16 block of v_mfma_f64_16x16x4f64 lives in
      // lane j + 16 (i % 4), register i / 4; e = 16 ra + 4 q + r
      const int ra = e >> 4, q = (e >> 2) & 3, r = e & 3;
      i = i0 + 16 * ra + 4 * r + (lane >> 4);
      j = cb + 16 * q + (lane & 15);
    }
  };
  auto g_load = [&](int cb, int e0, int ne) {
#pragma unroll
    for (int e = e0; e < e0 + ne; ++e) {
      int i, j;
      g_index(cb, e, i, j);
      gpre[e] = (i < N && j < N) ? G[(size_t)i * N + j] : T(0);
    }
  };

  // scaling of the last flush of a slice: row i by d(i), column j by 1/d(j)
  const int8_t* sf = scale_slice >= 0 ? C.field + (size_t)scale_slice * N : nullptr;
  const int sb = (scale_slice == 0 || scale_slice == M + 1) ? 0 : 1;
  const bool inv = scale_inverse != 0;
  auto dfl = [&](int site, bool invert) -> double {
    const int si = sf[site] > 0 ? 0 : 1;
    return C.dval[sb][spin][invert ? 1 - si : si];
  };
  // new value of element e of the pass from its old value and the product
  auto put = [&](int cb, int e, T acc) {
    int i, j;
    g_index(cb, e, i, j);
    T v = gpre[e] - acc;
    if (sf && i < N && j < N) v *= (T)(dfl(i, inv) * dfl(j, !inv));
    if (i < N && j < N) Gout[(size_t)i * N + j] = v;
  };

  for (int cb = 64 * wave; cb < N; cb += 256) {
    if constexpr (sizeof(T) == 4) {
      const int kr = lane >> 5, cc = lane & 31;
      const int ia = i0 + cc;
      const T* wrow = W + (size_t)ia * kSegMax;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int jh = cb + 32 * h + cc;
        g_load(cb, 16 * h, 16);
        floatx16 a0;
#pragma unroll
        for (int r = 0; r < 16; ++r) a0[r] = 0.f;
        for (int k0 = 0; k0 < f; k0 += 8 * KS) {
          float av[8], bv[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int k = k0 + t * KS + kr;
            av[t] = (k < f && ia < N) ? wrow[k] : 0.f;
            bv[t] = (k < f && jh < N) ? Yg[(size_t)k * N + jh] : 0.f;
          }
#pragma unroll
          for (int t = 0; t < 8; ++t) a0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av[t], bv[t], a0, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) put(cb, 16 * h + r, a0[r]);
      }
    } else {
      g_load(cb, 0, NG);
      const int kr = lane >> 4, cc = lane & 15;
      doublex4 acc[2][4];
#pragma unroll
      for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[ra][q][r] = 0.0;
      for (int k0 = 0; k0 < f; k0 += 2 * KS) {
        double av[2][2], bv[2][4];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int k = k0 + t * KS + kr;
#pragma unroll
          for (int ra = 0; ra < 2; ++ra) {
            const int ia = i0 + 16 * ra + cc;
            av[t][ra] = (k < f && ia < N) ? (double)W[(size_t)ia * kSegMax + k] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = cb + 16 * q + cc;
            bv[t][q] = (k < f && j < N) ? (double)Yg[(size_t)k * N + j] : 0.0;
          }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int ra = 0; ra < 2; ++ra)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc[ra][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t][ra], bv[t][q], acc[ra][q], 0, 0, 0);
      }
#pragma unroll
      for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) put(cb, 16 * ra + 4 * q + r, (T)acc[ra][q][r]);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_flush32(const ChainDev* __restrict__ chains, int nrb,
                                                      int scale_slice, int scale_inverse, int M,
                                                      int to_tmp) {
  flush_body<float>(chains, nrb, scale_slice, scale_inverse, M, to_tmp);
}
__global__ __launch_bounds__(kThreads) void k_flush64(const ChainDev* __restrict__ chains, int nrb,
                                                      int scale_slice, int scale_inverse, int M,
                                                      int to_tmp) {
  flush_body<double>(chains, nrb, scale_slice, scale_inverse, M, to_tmp);
}

hipError_t launch_flush(int fp32, const ChainDev* c, int nc, int n_max, int kseg, int scale_slice,
                        int scale_inverse, int M, int to_tmp, hipStream_t s) {
  (void)kseg;
  const int nrb = (n_max + kFlushRows - 1) / kFlushRows;
  const dim3 grid(nc * 2 * nrb);   // exactly one workgroup per (chain, spin, row block)
  if (fp32)
    hipLaunchKernelGGL(k_flush32, grid, dim3(kThreads), 0, s, c, nrb, scale_slice, scale_inverse, M,
                       to_tmp);
  else
    hipLaunchKernelGGL(k_flush64, grid, dim3(kThreads), 0, s, c, nrb, scale_slice, scale_inverse, M,
                       to_tmp);
  return hipGetLastError();
}

// Wg = G0[:, F] Z (N x f, ld kSegMax) of the segment [s0, s1), computed as
// G0[:, S] Zs with S the segment's consecutive sites and Zs = Z spread over
// them (zero rows on rejected sites): each thread reads a contiguous slab of
// 32 sites of its row; 32 columns of Wg at a time, the 32 x 32 slab of Zs in
// LDS.  Grid: chains x 2 spins x ceil(N_max / 256) row blocks.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_wmat(const ChainDev* __restrict__ chains, int nrb,
                                                   int s0, int s1) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int cs = b / nrb, rb = b - cs * nrb;
  const int spin = cs & 1;
  const ChainDev& C = chains[cs >> 1];
  const int N = C.N;
  if (s0 >= N || rb * kThreads >= N) return;
  const int f = C.st->fcount;
  if (f == 0) return;
  const int nseg = min(s1, N) - s0, tid = threadIdx.x;
  __shared__ __align__(16) T Zs[32][32];
  __shared__ int pos[kSegMax];
  for (int c = tid; c < nseg; c += kThreads) pos[c] = -1;
  __syncthreads();
  for (int p = tid; p < f; p += kThreads) pos[C.flist[p] - s0] = p;
  const T* __restrict__ Z = (const T*)C.Z[spin];
  const T* __restrict__ G = (const T*)C.G[spin];
  T* __restrict__ W = (T*)C.Wg[spin];
  const int i = rb * kThreads + tid;
  for (int q0 = 0; q0 < f; q0 += 32) {
    T acc[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) acc[t] = T(0);
    for (int sc = 0; sc < nseg; sc += 32) {
      __syncthreads();
      for (int e = tid; e < 32 * 32; e += kThreads) {
        const int c = e >> 5, t = e & 31;
        const int p = sc + c < nseg ? pos[sc + c] : -1;
        Zs[c][t] = (p >= 0 && q0 + t < f) ? Z[(size_t)p * kSegMax + q0 + t] : T(0);
      }
      __syncthreads();
      if (i < N) {
        const int nc = min(32, nseg - sc);
        const T* grow = G + (size_t)i * N + s0 + sc;
        T x[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) x[c] = c < nc ? grow[c] : T(0);
#pragma unroll
        for (int c = 0; c < 32; ++c) {
#pragma unroll
          for (int t = 0; t < 32; ++t) acc[t] += x[c] * Zs[c][t];
        }
      }
    }
    if (i < N) {
      T* wrow = W + (size_t)i * kSegMax + q0;
#pragma unroll
      for (int t = 0; t < 32; ++t)
        if (q0 + t < f) wrow[t] = acc[t];
    }
  }
}

hipError_t launch_wmat(int fp32, const ChainDev* c, int nc, int n_max, int s0, int s1, hipStream_t s) {
  const int nrb = (n_max + kThreads - 1) / kThreads;
  const dim3 grid(nc * 2 * nrb);
  if (fp32)
    hipLaunchKernelGGL(k_wmat<float>, grid, dim3(kThreads), 0, s, c, nrb, s0, s1);
  else
    hipLaunchKernelGGL(k_wmat<double>, grid, dim3(kThreads), 0, s, c, nrb, s0, s1);
  return hipGetLastError();
}

hipError_t launch_scan(int fp32, const ChainDev* c, int nc, const Ctl* ctl, int l, int M, int s0,
                       int s1, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_scan<float>, dim3(nc), dim3(kThreads), 0, s, c, ctl, l, M, s0, s1);
  else
    hipLaunchKernelGGL(k_scan<double>, dim3(nc), dim3(kThreads), 0, s, c, ctl, l, M, s0, s1);
  return hipGetLastError();
}

}  // namespace gpqmc
