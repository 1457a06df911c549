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
// G0 here is the Green's function of the segment's start, G_s = G - Xa Ya
// with Xa Ya the not yet applied flips of earlier segments of the slice; the
// kernel forms its block G_s[S,S] over the segment's sites S in LDS and works
// on it alone.  It ends by writing F and Z; k_xy appends the segment to Xa Ya,
// and one GEMM per slice applies G <- G - Xa Ya (a delayed update of rank =
// the slice's accepted flips), fused with the frame change.
//
// Factored engine (FACT): G = 1 - A B^T with A, B of size N x n; the block is
// G_s[S,S] = 1 - A[S,:] B[S,:]^T, and at the segment's end the accepted flips
// are folded into the factors by the Woodbury identity.  With Z = (Delta_F^{-1}
// + X[F,F])^{-1} (X = 1 - G at the segment's start) the moving factor M (A on
// an upward pass, B on a downward one) has its rows F scaled by 1 + Delta_F,
// and the dual factor Q takes Q <- Q - (Q M[F,:]^T) W with W = Z^T Q[F,:]
// (upward) or Z Q[F,:] (downward); the kernel writes M[F,:] (before scaling)
// and W, and two GEMMs apply the update to Q.
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

template <typename T, bool FACT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1))) void k_scan(const ChainDev* __restrict__ chains,
                                                   const Ctl* __restrict__ ctl, int l, int M,
                                                   int s0, int s1, int dir, int parity) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  ChainState* st = C.st;
  const int N = C.N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (s0 >= N) {   // uneven batch: this chain has no site in the segment
    if (tid == 0) {
      st->fcount = 0;
      st->foff = st->ftot;
    }
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
  __shared__ __align__(16) T Rsf[kSegMax * 36];   // >= kBlock * kSegMax
  // the segment's block of the current Green's function, G_s[S,S] (S = s0 .. s1)
  constexpr int LGS = kSegMax + 1;
  __shared__ T Gss[2][kSegMax * LGS];
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
  // the slice's flip factors, read once: the sequential loop below selects
  // them in registers instead of loading them per site
  const double dl_u0 = C.delta[bnd][0][0], dl_u1 = C.delta[bnd][0][1];
  const double dl_d0 = C.delta[bnd][1][0], dl_d1 = C.delta[bnd][1][1];
  double* const trace_ratio = C.trace_ratio;
  GLOBAL T* Z[2] = {gp((T*)C.Z[0]), gp((T*)C.Z[1])};
  GLOBAL T *W1[2], *Pm[2], *Qm[2], *PZ[2], *ZQ[2];
  for (int s = 0; s < 2; ++s) {
    GLOBAL T* w = gp((T*)C.scan_ws[s]);
    const size_t blk = (size_t)kBlock * kSegMax;
    W1[s] = w;            // kb x f       (ld LDZ)
    Pm[s] = w + blk;      // f x fb       (ld kBlock)
    Qm[s] = w + 2 * blk;  // fb x f       (ld LDZ)
    PZ[s] = w + 3 * blk;  // f x fb       (ld kBlock)
    ZQ[s] = w + 4 * blk;  // fb x f       (ld LDZ)
  }
  // ---- G_s[S,S] = G0[S,S] - Xa[S, :fp] Ya[:fp, S]: the fp flips accepted in
  // earlier segments of this slice are not yet applied to G ----
  const int fprev = (FACT || s0 == 0) ? 0 : st->ftot;
  if (FACT && nseg <= kBlock) {
    // G_s[S,S] = 1 - A[S,:] B[S,:]^T for both spins: 128 threads per spin,
    // thread t owns column t % 32 and rows t / 32 + 4 m; the inner dimension
    // n runs in k-chunks of 32 with the rows of A and B read as contiguous
    // 8-element pieces (A kept row-major in Rsf, B transposed in the Hs area)
    const int s = tid >> 7, t = tid & 127, c = t & 31, rb = t >> 5;
    const int nn = C.n[s];
    const GLOBAL T* __restrict__ fa = gp((const T*)C.F[0][s][parity]);
    const GLOBAL T* __restrict__ fb = gp((const T*)C.F[1][s][parity]);
    T* As = Rsf + s * kBlock * KL;
    T* Bs = &Hs[s][0][0];
    T acc[kBlock / 4];
#pragma unroll
    for (int m = 0; m < kBlock / 4; ++m) {
      const int row = rb + 4 * m;
      acc[m] = (row < nseg && row == c) ? T(1) : T(0);
    }
    constexpr int E8 = 8;
    const int lr = t >> 2, le = (t & 3) * E8;
    T va[E8], vb[E8];
    auto load_chunk = [&](int k0) {
#pragma unroll
      for (int e = 0; e < E8; ++e) {
        const int k = k0 + le + e;
        const bool ok = lr < nseg && k < nn;
        va[e] = ok ? fa[(size_t)(s0 + lr) * nn + k] : T(0);
        vb[e] = ok ? fb[(size_t)(s0 + lr) * nn + k] : T(0);
      }
    };
    load_chunk(0);
    for (int k0 = 0; k0 < nn; k0 += 32) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E8; ++e) {
        As[lr * KL + le + e] = va[e];
        Bs[(le + e) * KL + lr] = vb[e];
      }
      __syncthreads();
      if (k0 + 32 < nn) load_chunk(k0 + 32);
#pragma unroll 4
      for (int k = 0; k < 32; ++k) {
        const T bv = Bs[k * KL + c];
#pragma unroll
        for (int m = 0; m < kBlock / 4; ++m) acc[m] -= As[(rb + 4 * m) * KL + k] * bv;
      }
    }
#pragma unroll
    for (int m = 0; m < kBlock / 4; ++m) {
      const int row = rb + 4 * m;
      if (row < nseg && c < nseg) Gss[s][row * LGS + c] = acc[m];
    }
  } else if (FACT) {
    // segments of more than 32 sites: lane = column c, rows wave + 4 m, one
    // spin at a time; A[S, k] (nseg x 32) row-major in Rsf, B[S, k] transposed
    T* As = Rsf;
    T* Bs = &Hs[0][0][0];
    constexpr int LA = 36, LB = kSegMax + 4;
    static_assert(32 * LB <= 2 * kBlock * (kBlock + 2), "B tile fits in Hs");
    const int c = lane;
    for (int s = 0; s < 2; ++s) {
      const int nn = C.n[s];
      const GLOBAL T* __restrict__ fa = gp((const T*)C.F[0][s][parity]);
      const GLOBAL T* __restrict__ fb = gp((const T*)C.F[1][s][parity]);
      T acc[kSegMax / 4];
#pragma unroll
      for (int m = 0; m < kSegMax / 4; ++m) {
        const int row = wave + 4 * m;
        acc[m] = (row < nseg && row == c) ? T(1) : T(0);
      }
      constexpr int NL = kSegMax * 32 / kThreads;
      T va[NL], vb[NL];
      auto load_chunk = [&](int k0) {
#pragma unroll
        for (int t = 0; t < NL; ++t) {
          const int e = tid + t * kThreads, r = e >> 5, k = k0 + (e & 31);
          const bool ok = r < nseg && k < nn;
          va[t] = ok ? fa[(size_t)(s0 + r) * nn + k] : T(0);
          vb[t] = ok ? fb[(size_t)(s0 + r) * nn + k] : T(0);
        }
      };
      load_chunk(0);
      for (int k0 = 0; k0 < nn; k0 += 32) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NL; ++t) {
          const int e = tid + t * kThreads;
          As[(e >> 5) * LA + (e & 31)] = va[t];
          Bs[(e & 31) * LB + (e >> 5)] = vb[t];
        }
        __syncthreads();
        if (k0 + 32 < nn) load_chunk(k0 + 32);
        for (int k = 0; k < 32; ++k) {
          const T bv = Bs[k * LB + c];
#pragma unroll
          for (int m = 0; m < kSegMax / 4; ++m) acc[m] -= As[(wave + 4 * m) * LA + k] * bv;
        }
      }
#pragma unroll
      for (int m = 0; m < kSegMax / 4; ++m) {
        const int row = wave + 4 * m;
        if (row < nseg && c < nseg) Gss[s][row * LGS + c] = acc[m];
      }
    }
  } else if (nseg <= kBlock) {
    // segments of up to 32 sites: both spins in one pass, 128 threads per
    // spin, thread t of a spin owns column t % 32 and rows t / 32 + 4 m; the
    // rank-fprev correction runs in k-chunks of 32 with every operand row
    // read as one contiguous 128-byte segment: A = Xa[S, k] (in Rsf) and
    // B = Ya[k, S] (in the Hs area), both [spin][32][KL]
    const int s = tid >> 7, t = tid & 127, c = t & 31, rb = t >> 5;
    const GLOBAL T* __restrict__ g0 = gp((const T*)C.G[s]);
    const GLOBAL T* __restrict__ xa = gp((const T*)C.Xa[s]);
    const GLOBAL T* __restrict__ ya = gp((const T*)C.Ya[s]);
    T* As = Rsf + s * kBlock * KL;
    T* Bs = &Hs[s][0][0];
    static_assert(2 * kBlock * KL <= kSegMax * 36, "A tiles fit in Rsf");
    T acc[kBlock / 4];
#pragma unroll
    for (int m = 0; m < kBlock / 4; ++m) {
      const int row = rb + 4 * m;
      acc[m] = (row < nseg && c < nseg) ? g0[(size_t)(s0 + row) * N + s0 + c] : T(0);
    }
    // thread t loads 8 consecutive entries of row (t / 4) of each tile
    constexpr int E8 = 8;
    const int lr = t >> 2, le = (t & 3) * E8;
    T va[E8], vb[E8];
    auto load_chunk = [&](int k0) {
#pragma unroll
      for (int e = 0; e < E8; ++e) {
        const int k = k0 + le + e;
        va[e] = (lr < nseg && k < fprev) ? xa[(size_t)(s0 + lr) * N + k] : T(0);
        vb[e] = (k0 + lr < fprev && le + e < nseg) ? ya[(size_t)(k0 + lr) * N + s0 + le + e] : T(0);
      }
    };
    if (fprev > 0) load_chunk(0);
    for (int k0 = 0; k0 < fprev; k0 += 32) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E8; ++e) {
        As[lr * KL + le + e] = va[e];
        Bs[lr * KL + le + e] = vb[e];
      }
      __syncthreads();
      if (k0 + 32 < fprev) load_chunk(k0 + 32);
#pragma unroll 4
      for (int k = 0; k < 32; ++k) {
        const T bv = Bs[k * KL + c];
#pragma unroll
        for (int m = 0; m < kBlock / 4; ++m) acc[m] -= As[(rb + 4 * m) * KL + k] * bv;
      }
    }
#pragma unroll
    for (int m = 0; m < kBlock / 4; ++m) {
      const int row = rb + 4 * m;
      if (row < nseg && c < nseg) Gss[s][row * LGS + c] = acc[m];
    }
  } else {
    // lane = column c of the segment, rows wave + 4 m; the rank-fprev
    // correction runs in k-chunks of 32 staged in LDS: A = Xa[S, k] (in Rsf,
    // nseg x 32), B = Ya[k, S] (in the Hs area, 32 x nseg)
    T* As = Rsf;
    T* Bs = &Hs[0][0][0];
    constexpr int LA = 36, LB = kSegMax + 4;
    static_assert(32 * LB <= 2 * kBlock * (kBlock + 2), "B tile fits in Hs");
    const int c = lane;
    for (int s = 0; s < 2; ++s) {
      const GLOBAL T* __restrict__ g0 = gp((const T*)C.G[s]);
      const GLOBAL T* __restrict__ xa = gp((const T*)C.Xa[s]);
      const GLOBAL T* __restrict__ ya = gp((const T*)C.Ya[s]);
      T acc[kSegMax / 4];
#pragma unroll
      for (int m = 0; m < kSegMax / 4; ++m) {
        const int row = wave + 4 * m;
        acc[m] = (row < nseg && c < nseg) ? g0[(size_t)(s0 + row) * N + s0 + c] : T(0);
      }
      // k-chunks of 32, the next chunk's loads issued before this one's FMAs
      constexpr int NL = kSegMax * 32 / kThreads;
      T va[NL], vb[NL];
      auto load_chunk = [&](int k0) {
        const int kn = min(32, fprev - k0);
#pragma unroll
        for (int t = 0; t < NL; ++t) {
          const int e = tid + t * kThreads, r = e >> 5, k = e & 31;
          va[t] = (r < nseg && k < kn) ? xa[(size_t)(s0 + r) * N + k0 + k] : T(0);
          const int kb = e / kSegMax, cc = e % kSegMax;
          vb[t] = (kb < kn && cc < nseg) ? ya[(size_t)(k0 + kb) * N + s0 + cc] : T(0);
        }
      };
      if (fprev > 0) load_chunk(0);
      for (int k0 = 0; k0 < fprev; k0 += 32) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NL; ++t) {
          const int e = tid + t * kThreads;
          As[(e >> 5) * LA + (e & 31)] = va[t];
          Bs[(e / kSegMax) * LB + e % kSegMax] = vb[t];
        }
        __syncthreads();
        if (k0 + 32 < fprev) load_chunk(k0 + 32);
        for (int k = 0; k < 32; ++k) {
          const T bv = Bs[k * LB + c];
#pragma unroll
          for (int m = 0; m < kSegMax / 4; ++m) acc[m] -= As[(wave + 4 * m) * LA + k] * bv;
        }
      }
#pragma unroll
      for (int m = 0; m < kSegMax / 4; ++m) {
        const int row = wave + 4 * m;
        if (row < nseg && c < nseg) Gss[s][row * LGS + c] = acc[m];
      }
    }
  }
  __syncthreads();

  for (int b0 = s0; b0 < send; b0 += kBlock) {
    const int bl = b0 - s0;
    const int kb = min(kBlock, send - b0);
    const int f = sh_f;
    // ---- W1 = G_s[B, F] Z  (kb x f), one spin at a time through LDS ----
    if (f > 0) {
      for (int s = 0; s < 2; ++s) {
        for (int a = wave; a < kb; a += 4)
          for (int p = lane; p < f; p += 64) Rsf[a * f + p] = Gss[s][(bl + a) * LGS + Fs[p] - s0];
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
    // ---- block of the current Green's function: G[B,B] = G_s[B,B] + W1 G_s[F,B] ----
    // rows (spin, a) over waves and lane halves, columns over lanes 0..31
    {
      const int half = lane >> 5, c = lane & 31;
      for (int row = 2 * wave + half; row < 2 * kb; row += 8) {
        const int s = row >= kb ? 1 : 0, a = row - s * kb;
        if (c < kb) {
          T acc = Gss[s][(bl + a) * LGS + bl + c];
          for (int q = 0; q < f; ++q)
            acc += W1[s][(size_t)a * LDZ + q] * Gss[s][(Fs[q] - s0) * LGS + bl + c];
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
          const double du = si ? dl_u1 : dl_u0, dd = si ? dl_d1 : dl_d0;
          const double ru = 1.0 + du * (1.0 - (double)lane_value(g[j], j));
          const double rd = 1.0 + dd * (1.0 - (double)lane_value(g[j], 32 + j));
          const bool accept = !force_reject && (u_s[li] < fabs(ru * rd));
          if (lane == 0 && trace_ratio) {
            trace_ratio[((size_t)l * N + b0 + j) * 2 + 0] = ru;
            trace_ratio[((size_t)l * N + b0 + j) * 2 + 1] = rd;
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
    //   Z <- [[Z + P Zb Q, P Zb], [Zb Q, Zb]],  P = Z G_s[F,Fb], Q = G_s[Fb,F] Z
    const int fb = sh_fb;
    if (fb > 0) {
      if (f > 0) {
        for (int s = 0; s < 2; ++s) {
          // P (f x fb): rows over waves, columns over lanes; Q (fb x f) likewise
          for (int p = wave; p < f; p += 4)
            for (int c = lane; c < fb; c += 64) {
              const int col = bl + Fb[c];
              T acc = 0;
              for (int q = 0; q < f; ++q) acc += Z[s][(size_t)p * LDZ + q] * Gss[s][(Fs[q] - s0) * LGS + col];
              Pm[s][p * kBlock + c] = acc;
            }
          for (int c = wave; c < fb; c += 4) {
            const T* row = &Gss[s][(bl + Fb[c]) * LGS];
            for (int q = lane; q < f; q += 64) {
              T acc = 0;
              for (int p = 0; p < f; ++p) acc += row[Fs[p] - s0] * Z[s][(size_t)p * LDZ + q];
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

  // the accepted sites F of the segment (their coefficients Z are in place)
  const int f = sh_f;
  for (int p = tid; p < f; p += kThreads) C.flist[p] = Fs[p];
  for (int i = tid; i < nseg; i += kThreads) frow[s0 + i] = fs[i];
  if (FACT && f > 0) {
    // Woodbury operands of the segment, per spin: Mf = M[F,:] (then M[F,:] is
    // scaled by 1 + Delta_F), Wf = Z^T Q[F,:] (upward) or Z Q[F,:] (downward).
    // The fields in fs are already flipped: the old value is -fs.
    for (int s = 0; s < 2; ++s) {
      const int nn = C.n[s];
      GLOBAL T* __restrict__ Mv = gp((T*)C.F[dir][s][parity]);
      const GLOBAL T* __restrict__ Qv = gp((const T*)C.F[1 - dir][s][parity]);
      GLOBAL double* __restrict__ mf = gp(C.Mf[s]);
      GLOBAL double* __restrict__ wf = gp(C.Wf[s]);
      const GLOBAL T* __restrict__ Zg = Z[s];
      for (int idx = tid; idx < f * nn; idx += kThreads) {
        const int p = idx / nn, k = idx - p * nn;
        const int site = Fs[p];
        const int si_old = fs[site - s0] < 0 ? 0 : 1;
        const size_t o = (size_t)site * nn + k;
        const T v = Mv[o];
        mf[(size_t)p * nn + k] = (double)v;
        Mv[o] = v * (T)(1.0 + C.delta[bnd][s][si_old]);
        T acc = T(0);
        for (int q = 0; q < f; ++q) {
          const T z = dir == 0 ? Zg[(size_t)q * LDZ + p] : Zg[(size_t)p * LDZ + q];
          acc += z * Qv[(size_t)Fs[q] * nn + k];
        }
        wf[(size_t)p * nn + k] = (double)acc;
      }
    }
  }
  if (tid == 0) {
    st->fcount = f;
    st->foff = fprev;
    st->ftot = fprev + f;
    st->sign = sh_sign;
    st->accepted += sh_acc;
    st->proposed += nseg;
  }
}

// Appends the factors of one segment to the slice-level update G = G0 - Xa Ya:
//   Xa[:, fp : fp + f] = (G0[:, F] - Xa[:, :fp] Ya[:fp, F]) Z          (X part)
//   Ya[fp : fp + f, :] = (1 - G0)[F, :] + Xa[F, :fp] Ya[:fp, :]        (Y part)
// with fp the flips accepted in earlier segments of the slice, f <= FMAX the
// flips of this segment, F their sites (inside the segment [s0, s0 + kseg))
// and Z their coefficients (from the scan).  The X part reads Xa columns < fp
// and Ya rows < fp only, the Y part writes Ya rows >= fp and reads Xa columns
// < fp, so the two parts run concurrently.  A workgroup takes ROWS (256)
// rows (X part) or columns (Y part) of one chain and spin; the inner dimension
// fp runs in k-chunks of 16 whose operand tiles are loaded into LDS with
// coalesced reads, and each thread accumulates an 8 x 4 (x FMAX / 32)
// register block.  Grid: chains x 2 spins x 2 parts x ceil(N_max / ROWS).
// (Launched for FP64; the FP32 append runs on MFMA in k_xy_mfma below.)
template <typename T, int FMAX>
struct XyShape {
  static constexpr int ROWS = (sizeof(T) == 8 && FMAX == 64) ? 128 : 256;   // LDS budget
  static constexpr int WAVES = (sizeof(T) == 4 && FMAX == 32) ? 3 : 1;       // per SIMD
};

template <typename T, int FMAX>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(XyShape<T, FMAX>::WAVES))) void k_xy(const ChainDev* __restrict__ chains, int nrb,
                                                 int s0, int kseg) {
  constexpr int ROWS = XyShape<T, FMAX>::ROWS;       // rows (X) / columns (Y) per workgroup
  constexpr int RPT = ROWS / 32;                      // per thread
  constexpr int QB = FMAX / 32;                       // 32-wide q blocks
  constexpr int BK = 16;                              // k-chunk
  constexpr int V = 16 / sizeof(T);                   // elements per 128-bit LDS access
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int rb = b % nrb, part = (b / nrb) & 1, cs = b / (2 * nrb);
  const int spin = cs & 1;
  const ChainDev& C = chains[cs >> 1];
  const int N = C.N, tid = threadIdx.x;
  const int r0 = rb * ROWS;                           // first row (X) / column (Y)
  if (r0 >= N) return;
  const int f = C.st->fcount, fp = C.st->foff;
  if (f == 0) return;
  const T* __restrict__ G = (const T*)C.G[spin];
  T* __restrict__ Xa = (T*)C.Xa[spin];
  T* __restrict__ Ya = (T*)C.Ya[spin];
  __shared__ int Fl[FMAX];
  // X part: At[k][r] = Xa[r0 + r, k0 + k],  Bt[k][q] = Ya[k0 + k, F[q]]
  // Y part: At[k][j] = Ya[k0 + k, r0 + j],  Bt[k][q] = Xa[F[q], k0 + k]
  constexpr int LA = ROWS + 8, LB = FMAX + 4;
  constexpr int LP = FMAX + 1;                         // P rows (X part), aliasing At
  constexpr int AS = BK * LA > ROWS * LP ? BK * LA : ROWS * LP;
  __shared__ __align__(16) T At[AS];
  __shared__ __align__(16) T Bt[BK * LB];
  __shared__ T Zl[FMAX][FMAX + 1];
  for (int q = tid; q < FMAX; q += kThreads) Fl[q] = q < f ? gp(C.flist)[q] : 0;
  __syncthreads();

  // register block: rows / columns u0 .. u0 + RPT - 1, q = 4 g + 32 qb + v
  const int u0 = RPT * (tid >> 3), g = tid & 7;
  T acc[RPT][QB][4];
#pragma unroll
  for (int a = 0; a < RPT; ++a)
#pragma unroll
    for (int qb = 0; qb < QB; ++qb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][qb][v] = T(0);

  constexpr int NA = ROWS * BK / kThreads, NB = BK * FMAX / kThreads;
  for (int k0 = 0; k0 < fp; k0 += BK) {
    const int kn = min(BK, fp - k0);
    // all loads of the chunk are issued before the first LDS store
    T va[NA], vb[NB];
    if (part == 0) {
#pragma unroll
      for (int t = 0; t < NA; ++t) {                          // Xa rows, BK along k
        const int e = tid + t * kThreads, r = e / BK, k = e % BK;
        va[t] = (k < kn && r0 + r < N) ? Xa[(size_t)(r0 + r) * N + k0 + k] : T(0);
      }
#pragma unroll
      for (int t = 0; t < NB; ++t) {                          // Ya rows gathered at F
        const int e = tid + t * kThreads, k = e / FMAX, q = e % FMAX;
        vb[t] = (k < kn && q < f) ? Ya[(size_t)(k0 + k) * N + Fl[q]] : T(0);
      }
    } else {
#pragma unroll
      for (int t = 0; t < NA; ++t) {                          // Ya rows, ROWS columns
        const int e = tid + t * kThreads, k = e / ROWS, j = e % ROWS;
        va[t] = (k < kn && r0 + j < N) ? Ya[(size_t)(k0 + k) * N + r0 + j] : T(0);
      }
#pragma unroll
      for (int t = 0; t < NB; ++t) {                          // Xa rows F, BK along k
        const int e = tid + t * kThreads, q = e / BK, k = e % BK;
        vb[t] = (k < kn && q < f) ? Xa[(size_t)Fl[q] * N + k0 + k] : T(0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int e = tid + t * kThreads;
      if (part == 0)
        At[(e % BK) * LA + e / BK] = va[t];
      else
        At[(e / ROWS) * LA + e % ROWS] = va[t];
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int e = tid + t * kThreads;
      if (part == 0)
        Bt[(e / FMAX) * LB + e % FMAX] = vb[t];
      else
        Bt[(e % BK) * LB + e / BK] = vb[t];
    }
    __syncthreads();
#pragma unroll 2
    for (int k = 0; k < BK; ++k) {
      T a[RPT];
#pragma unroll
      for (int h = 0; h < RPT; h += V) {
        using VT = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        const VT x = *reinterpret_cast<const VT*>(&At[k * LA + u0 + h]);
        const T* xe = reinterpret_cast<const T*>(&x);
#pragma unroll
        for (int t = 0; t < V; ++t) a[h + t] = xe[t];
      }
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
        T bq[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) bq[v] = Bt[k * LB + 32 * qb + 4 * g + v];
#pragma unroll
        for (int aa = 0; aa < RPT; ++aa)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[aa][qb][v] += a[aa] * bq[v];
      }
    }
  }

  // epilogues: every global access below is a contiguous row segment; the
  // register blocks go through LDS (the A tile) for the gathers and stores
  constexpr int LR = ROWS + 1;
  static_assert(ROWS * LP <= AS && FMAX * LR <= AS, "epilogue tiles fit in the A tile");
  __syncthreads();
  if (part == 0) {
    // the segment's slab G0[rows, s0 .. s0 + kseg) and Z
    T* S1 = At;
    constexpr int NE = ROWS * FMAX / kThreads;
    const T* __restrict__ Z = (const T*)C.Z[spin];
    for (int e = tid; e < FMAX * FMAX; e += kThreads) {
      const int q = e / FMAX, c = e % FMAX;
      Zl[q][c] = (q < f && c < f) ? Z[(size_t)q * kSegMax + c] : T(0);
    }
    for (int t0 = 0; t0 < NE; t0 += 8) {       // eight loads in flight, then their stores
      T vs[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int e = tid + (t0 + t) * kThreads, r = e / FMAX, cc = e % FMAX;
        vs[t] = (r0 + r < N && cc < kseg && s0 + cc < N) ? G[(size_t)(r0 + r) * N + s0 + cc] : T(0);
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int e = tid + (t0 + t) * kThreads;
        S1[(e / FMAX) * LP + e % FMAX] = vs[t];
      }
    }
    __syncthreads();
    // P = G0[i, F] - acc, kept in acc
#pragma unroll
    for (int aa = 0; aa < RPT; ++aa)
#pragma unroll
      for (int qb = 0; qb < QB; ++qb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int q = 32 * qb + 4 * g + v;
          acc[aa][qb][v] = q < f ? S1[(u0 + aa) * LP + Fl[q] - s0] - acc[aa][qb][v] : T(0);
        }
    __syncthreads();
    T* Pl = At;
#pragma unroll
    for (int aa = 0; aa < RPT; ++aa)
#pragma unroll
      for (int qb = 0; qb < QB; ++qb)
#pragma unroll
        for (int v = 0; v < 4; ++v) Pl[(u0 + aa) * LP + 32 * qb + 4 * g + v] = acc[aa][qb][v];
    __syncthreads();
    // Xa[i, fp + c] = sum_q P[i][q] Z[q][c]: rows u0 .., columns c = 32 cb + 4 g + v
    T xo[RPT][QB][4];
#pragma unroll
    for (int aa = 0; aa < RPT; ++aa)
#pragma unroll
      for (int cb = 0; cb < QB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) xo[aa][cb][v] = T(0);
    for (int q = 0; q < f; ++q) {
      T pq[RPT];
#pragma unroll
      for (int aa = 0; aa < RPT; ++aa) pq[aa] = Pl[(u0 + aa) * LP + q];
#pragma unroll
      for (int cb = 0; cb < QB; ++cb) {
        T zq[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) zq[v] = Zl[q][32 * cb + 4 * g + v];
#pragma unroll
        for (int aa = 0; aa < RPT; ++aa)
#pragma unroll
          for (int v = 0; v < 4; ++v) xo[aa][cb][v] += pq[aa] * zq[v];
      }
    }
    __syncthreads();
#pragma unroll
    for (int aa = 0; aa < RPT; ++aa)
#pragma unroll
      for (int cb = 0; cb < QB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) Pl[(u0 + aa) * LP + 32 * cb + 4 * g + v] = xo[aa][cb][v];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tid + t * kThreads, r = e / FMAX, c = e % FMAX;
      if (r0 + r < N && c < f) Xa[(size_t)(r0 + r) * N + fp + c] = Pl[r * LP + c];
    }
  } else {
    // rows F of G0 over the workgroup's columns
    T* Gr = At;
    constexpr int NE = FMAX * ROWS / kThreads;
    for (int t0 = 0; t0 < NE; t0 += 8) {       // eight loads in flight, then their stores
      T vs[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int e = tid + (t0 + t) * kThreads, q = e / ROWS, j = e % ROWS;
        vs[t] = (q < f && r0 + j < N) ? G[(size_t)Fl[q] * N + r0 + j] : T(0);
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int e = tid + (t0 + t) * kThreads;
        Gr[(e / ROWS) * LR + e % ROWS] = vs[t];
      }
    }
    __syncthreads();
    // Ya[fp + q, j] = (F[q] == j) - G0[F[q], j] + acc, kept in acc
#pragma unroll
    for (int aa = 0; aa < RPT; ++aa)
#pragma unroll
      for (int qb = 0; qb < QB; ++qb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int q = 32 * qb + 4 * g + v, j = u0 + aa;
          acc[aa][qb][v] += (Fl[q] == r0 + j ? T(1) : T(0)) - Gr[q * LR + j];
        }
    __syncthreads();
#pragma unroll
    for (int aa = 0; aa < RPT; ++aa)
#pragma unroll
      for (int qb = 0; qb < QB; ++qb)
#pragma unroll
        for (int v = 0; v < 4; ++v) Gr[(32 * qb + 4 * g + v) * LR + u0 + aa] = acc[aa][qb][v];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = tid + t * kThreads, q = e / ROWS, j = e % ROWS;
      if (q < f && r0 + j < N) Ya[(size_t)(fp + q) * N + r0 + j] = Gr[q * LR + j];
    }
  }
}

// FP32 form of the same append on MFMA (v_mfma_f32_32x32x2f32).  Both parts
// are products of a wide operand (ROWS rows of Xa, or ROWS columns of Ya) and
// a narrow one (Ya gathered at the columns F, or the rows F of Xa) over the
// inner dimension fp, staged k-major in LDS in k-chunks of 16 (the next chunk
// is loaded into registers while the current one is multiplied).  Workgroups
// of 128 rows keep six of them per CU in flight: the kernel is bound by the
// latency of its loads rather than by the products.
//   X part: C[r][q] = sum_k Xa[r0 + r, k] Ya[k, F[q]]   (wave: rows 64 w ..)
//   Y part: C[q][j] = sum_k Xa[F[q], k] Ya[k, r0 + j]   (wave: columns 64 w ..)
// so that the Y part comes out with lanes along j and its stores to the rows of
// Ya are contiguous.  The X part then forms P = G0[:, F] - C in LDS and its
// product with Z on MFMA as well; its lanes run along the columns fp + c of Xa.
template <int FMAX>
struct XyMfmaShape {
  static constexpr int ROWS = 128;   // rows (X) / columns (Y) per workgroup
  static constexpr int XB = ROWS / 128;                  // 32-wide row blocks per wave
  static constexpr int QB = FMAX / 32;                   // 32-wide q blocks
  static constexpr int BK = 16;                          // k-chunk
  static constexpr int LA = ROWS + 4;                    // wide tile row (k-major)
  static constexpr int LS = FMAX + 4;                    // narrow tile row (k-major)
  static constexpr int LP = FMAX + 1;                    // G0 slab / P rows
  static constexpr int UNION = BK * LA > ROWS * LP ? BK * LA : ROWS * LP;
  static constexpr int WAVES = FMAX == 32 ? 6 : 2;       // per SIMD (a 16-byte spill at 6 measured faster than 5)
};

__device__ inline float4 xy_load4(const GLOBAL float* __restrict__ p, int valid, bool aligned) {
  if (aligned && valid >= 4) return gload4(p);
  float4 v;
  v.x = valid > 0 ? p[0] : 0.f;
  v.y = valid > 1 ? p[1] : 0.f;
  v.z = valid > 2 ? p[2] : 0.f;
  v.w = valid > 3 ? p[3] : 0.f;
  return v;
}

template <int FMAX>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(XyMfmaShape<FMAX>::WAVES)))
void k_xy_mfma(const ChainDev* __restrict__ chains, int nrb) {
  using S = XyMfmaShape<FMAX>;
  constexpr int ROWS = S::ROWS, XB = S::XB, QB = S::QB, BK = S::BK;
  constexpr int LA = S::LA, LS = S::LS, LP = S::LP;
  constexpr int NQ4 = BK * ROWS / (4 * kThreads);        // float4 loads of the wide tile per thread
  constexpr int NS = BK * FMAX / kThreads;               // loads of the narrow tile per thread
  static_assert(NQ4 >= 1 && NS >= 1 && ROWS % 128 == 0, "tile shape");
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int rb = b % nrb, part = (b / nrb) & 1, cs = b / (2 * nrb);
  const int spin = cs & 1;
  const ChainDev& C = chains[cs >> 1];
  const int N = C.N, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = rb * ROWS;
  if (r0 >= N) return;
  const int f = C.st->fcount, fp = C.st->foff;
  if (f == 0) return;
  const GLOBAL float* __restrict__ G = gp((const float*)C.G[spin]);
  GLOBAL float* __restrict__ Xa = gp((float*)C.Xa[spin]);
  GLOBAL float* __restrict__ Ya = gp((float*)C.Ya[spin]);
  const bool al = (N & 3) == 0;

  __shared__ int Fl[FMAX];
  __shared__ __align__(16) float U[S::UNION];            // wide tile, then G0 slab / P
  __shared__ __align__(16) float Sm[BK * LS];            // narrow tile
  __shared__ float Zl[FMAX * LP];
  for (int q = tid; q < FMAX; q += kThreads) Fl[q] = q < f ? gp(C.flist)[q] : 0;
  __syncthreads();

  const int h = lane >> 5, l32 = lane & 31, w0 = wave * (ROWS / 4);
  floatx16 acc[XB * QB];
#pragma unroll
  for (int t = 0; t < XB * QB; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;

  // global -> register mapping of a k-chunk
  float4 va[NQ4];
  float vs[NS];
  // wide X tile: BK / 4 lanes per row, each a float4 along k, so a wave reads
  // eight whole 128-byte row segments per instruction
  constexpr int K4 = BK / 4, RS = kThreads / K4;
  auto gload = [&](int k0) {
    if (part == 0) {
      const int k = k0 + 4 * (tid % K4), rr = tid / K4;
#pragma unroll
      for (int t = 0; t < NQ4; ++t) {
        const int r = rr + RS * t;
        va[t] = xy_load4(Xa + (size_t)(r0 + r) * N + k, r0 + r < N ? fp - k : 0, al);
      }
      // narrow: Ya[k0 + k, F[q]]
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int e = tid + t * kThreads, k = e / FMAX, q = e % FMAX;
        vs[t] = (k0 + k < fp && q < f) ? Ya[(size_t)(k0 + k) * N + Fl[q]] : 0.f;
      }
    } else {
      // wide: Ya[k0 + k, r0 + 4 j4 ..]
      constexpr int J4 = ROWS / 4, KS = kThreads / J4;
      const int j = 4 * (tid % J4), kr = tid / J4;
#pragma unroll
      for (int t = 0; t < NQ4; ++t) {
        const int k = k0 + kr + KS * t;
        va[t] = xy_load4(Ya + (size_t)k * N + r0 + j, k < fp ? N - (r0 + j) : 0, al);
      }
      // narrow: Xa[F[q], k0 + k]
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int e = tid + t * kThreads, k = e % BK, q = e / BK;
        vs[t] = (k0 + k < fp && q < f) ? Xa[(size_t)Fl[q] * N + k0 + k] : 0.f;
      }
    }
  };
  auto sstore = [&]() {
    float* A = U;
    if (part == 0) {
      const int k = 4 * (tid % K4), rr = tid / K4;
#pragma unroll
      for (int t = 0; t < NQ4; ++t) {
        const int r = rr + RS * t;
        A[(k + 0) * LA + r] = va[t].x;
        A[(k + 1) * LA + r] = va[t].y;
        A[(k + 2) * LA + r] = va[t].z;
        A[(k + 3) * LA + r] = va[t].w;
      }
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int e = tid + t * kThreads;
        Sm[(e / FMAX) * LS + e % FMAX] = vs[t];
      }
    } else {
      constexpr int J4 = ROWS / 4, KS = kThreads / J4;
      const int j = 4 * (tid % J4), kr = tid / J4;
#pragma unroll
      for (int t = 0; t < NQ4; ++t) *reinterpret_cast<float4*>(&A[(kr + KS * t) * LA + j]) = va[t];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int e = tid + t * kThreads;
        Sm[(e % BK) * LS + e / BK] = vs[t];
      }
    }
  };

  const int nk = (fp + BK - 1) / BK;
  if (nk > 0) gload(0);
  for (int kt = 0; kt < nk; ++kt) {
    if (kt > 0) __syncthreads();                          // the previous chunk is consumed
    sstore();
    __syncthreads();
    if (kt + 1 < nk) gload((kt + 1) * BK);                // in flight during the products
    {
      const float* A = U;
      const float* Bn = Sm;
#pragma unroll
      for (int s2 = 0; s2 < BK / 2; ++s2) {
        const int kk = 2 * s2 + h;                        // lane's k of this MFMA k-step
        float wv[XB], nv[QB];
#pragma unroll
        for (int x = 0; x < XB; ++x) wv[x] = A[kk * LA + w0 + 32 * x + l32];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) nv[qb] = Bn[kk * LS + 32 * qb + l32];
#pragma unroll
        for (int x = 0; x < XB; ++x)
#pragma unroll
          for (int qb = 0; qb < QB; ++qb) {
            floatx16& a = acc[x * QB + qb];
            a = part == 0 ? __builtin_amdgcn_mfma_f32_32x32x2f32(wv[x], nv[qb], a, 0, 0, 0)
                          : __builtin_amdgcn_mfma_f32_32x32x2f32(nv[qb], wv[x], a, 0, 0, 0);
          }
      }
    }
  }
  __syncthreads();                                        // U is reused below

  // accumulator element r of block (x, qb): C row 8 (r / 4) + 4 h + (r % 4),
  // column l32 of the block (X part: row r0 + w0 + 32 x + .., q = 32 qb + l32;
  // Y part: q = 32 qb + .., column r0 + w0 + 32 x + l32)
  if (part == 1) {
    // one 32 x 32 block at a time: its 16 loads of G0 in flight, then its stores
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
        const int j = r0 + w0 + 32 * x + l32;
        float gv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int q = 32 * qb + 8 * (r >> 2) + 4 * h + (r & 3);
          gv[r] = (q < f && j < N) ? G[(size_t)Fl[q] * N + j] : 0.f;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int q = 32 * qb + 8 * (r >> 2) + 4 * h + (r & 3);
          if (q < f && j < N)
            Ya[(size_t)(fp + q) * N + j] = (Fl[q] == j ? 1.f : 0.f) - gv[r] + acc[x * QB + qb][r];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    return;
  }

  // X part: Z to LDS, then P = G0[:, F] - C with G0 gathered at the
  // accepted sites straight from memory (a lane's sixteen loads in flight at
  // once), then Xa[:, fp + c] = P Z
  const GLOBAL float* __restrict__ Z = gp((const float*)C.Z[spin]);
  for (int e = tid; e < FMAX * FMAX; e += kThreads) {
    const int q = e / FMAX, c = e % FMAX;
    Zl[q * LP + c] = (q < f && c < f) ? Z[(size_t)q * kSegMax + c] : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      const int q = 32 * qb + l32, col = q < f ? Fl[q] : 0;
      float gv[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = r0 + w0 + 32 * x + 8 * (r >> 2) + 4 * h + (r & 3);
        gv[r] = (q < f && i < N) ? G[(size_t)i * N + col] : 0.f;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float a = acc[x * QB + qb][r];
        acc[x * QB + qb][r] = q < f ? gv[r] - a : 0.f;
      }
    }
  float* Pl = U;
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int qb = 0; qb < QB; ++qb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = w0 + 32 * x + 8 * (r >> 2) + 4 * h + (r & 3), q = 32 * qb + l32;
        Pl[i * LP + q] = acc[x * QB + qb][r];
        acc[x * QB + qb][r] = 0.f;
      }
  __syncthreads();
  const int nsz = (f + 1) / 2;                            // MFMA k-steps over q < f
  for (int s2 = 0; s2 < nsz; ++s2) {
    const int q = 2 * s2 + h;
    float pv[XB], zv[QB];
#pragma unroll
    for (int x = 0; x < XB; ++x) pv[x] = Pl[(w0 + 32 * x + l32) * LP + q];
#pragma unroll
    for (int cb = 0; cb < QB; ++cb) zv[cb] = Zl[q * LP + 32 * cb + l32];
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int cb = 0; cb < QB; ++cb)
        acc[x * QB + cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(pv[x], zv[cb], acc[x * QB + cb], 0, 0, 0);
  }
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int cb = 0; cb < QB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = r0 + w0 + 32 * x + 8 * (r >> 2) + 4 * h + (r & 3), c = 32 * cb + l32;
        if (i < N && c < f) Xa[(size_t)i * N + fp + c] = acc[x * QB + cb][r];
      }
}

// FP64 form of k_xy_mfma for segments of up to 32 sites, on v_mfma_f64_16x16x4f64:
// the same two products and the same staging, with 16 x 16 blocks (a wave owns
// kXy64Rows / 4 rows or columns as XB blocks, and the 32 flips as two blocks)
// and MFMA k-steps of 4.  Block element r of a lane: row 4 r + lane / 16,
// column lane % 16.
constexpr int kXy64Rows = 64, kXy64Bk = 16, kXy64La = kXy64Rows + 2, kXy64Ls = 32 + 2,
              kXy64Lp = 32 + 1;
constexpr int kXy64Union = kXy64Bk * kXy64La > kXy64Rows * kXy64Lp ? kXy64Bk * kXy64La
                                                                   : kXy64Rows * kXy64Lp;

__device__ inline double2 xy_load2(const GLOBAL double* __restrict__ p, int valid, bool aligned) {
  if (aligned && valid >= 2) return gload2(p);
  double2 v;
  v.x = valid > 0 ? p[0] : 0.0;
  v.y = valid > 1 ? p[1] : 0.0;
  return v;
}

__global__ __launch_bounds__(kThreads) void k_xy_mfma64(const ChainDev* __restrict__ chains,
                                                        int nrb) {
  constexpr int FMAX = 32, ROWS = kXy64Rows, BK = kXy64Bk, LA = kXy64La, LS = kXy64Ls,
                LP = kXy64Lp;
  constexpr int NQ2 = BK * ROWS / (2 * kThreads);        // double2 loads of the wide tile
  constexpr int NS = BK * FMAX / kThreads;               // loads of the narrow tile
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int rb = b % nrb, part = (b / nrb) & 1, cs = b / (2 * nrb);
  const int spin = cs & 1;
  const ChainDev& C = chains[cs >> 1];
  const int N = C.N, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = rb * ROWS;
  if (r0 >= N) return;
  const int f = C.st->fcount, fp = C.st->foff;
  if (f == 0) return;
  const GLOBAL double* __restrict__ G = gp((const double*)C.G[spin]);
  GLOBAL double* __restrict__ Xa = gp((double*)C.Xa[spin]);
  GLOBAL double* __restrict__ Ya = gp((double*)C.Ya[spin]);
  const bool al = (N & 1) == 0;

  __shared__ int Fl[FMAX];
  __shared__ __align__(16) double U[kXy64Union];         // wide tile, then G0 slab / P
  __shared__ __align__(16) double Sm[BK * LS];           // narrow tile
  __shared__ double Zl[FMAX * LP];
  for (int q = tid; q < FMAX; q += kThreads) Fl[q] = q < f ? gp(C.flist)[q] : 0;
  __syncthreads();

  constexpr int XB = ROWS / 64;                          // 16-row blocks per wave
  const int kq = lane >> 4, l16 = lane & 15, w0 = wave * (ROWS / 4);
  doublex4 acc[XB][2];                                    // [row or column block][flip block]
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[x][y][r] = 0.0;

  double2 va[NQ2];
  double vs[NS];
  // wide X tile: BK / 2 lanes per row, each a double2 along k (128-byte row
  // segments); wide Y tile: ROWS / 2 lanes along a row of Ya
  constexpr int K2 = BK / 2, RS = kThreads / K2;
  constexpr int J2 = ROWS / 2, KS = kThreads / J2;
  auto gload = [&](int k0) {
    if (part == 0) {
      const int k = k0 + 2 * (tid % K2), rr = tid / K2;
#pragma unroll
      for (int t = 0; t < NQ2; ++t) {
        const int r = rr + RS * t;
        va[t] = xy_load2(Xa + (size_t)(r0 + r) * N + k, r0 + r < N ? fp - k : 0, al);
      }
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int e = tid + t * kThreads, k = e / FMAX, q = e % FMAX;
        vs[t] = (k0 + k < fp && q < f) ? Ya[(size_t)(k0 + k) * N + Fl[q]] : 0.0;
      }
    } else {
      const int j = 2 * (tid % J2), kr = tid / J2;
#pragma unroll
      for (int t = 0; t < NQ2; ++t) {
        const int k = k0 + kr + KS * t;
        va[t] = xy_load2(Ya + (size_t)k * N + r0 + j, k < fp ? N - (r0 + j) : 0, al);
      }
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int e = tid + t * kThreads, k = e % BK, q = e / BK;
        vs[t] = (k0 + k < fp && q < f) ? Xa[(size_t)Fl[q] * N + k0 + k] : 0.0;
      }
    }
  };
  auto sstore = [&]() {
    if (part == 0) {
      const int k = 2 * (tid % K2), rr = tid / K2;
#pragma unroll
      for (int t = 0; t < NQ2; ++t) {
        const int r = rr + RS * t;
        U[k * LA + r] = va[t].x;
        U[(k + 1) * LA + r] = va[t].y;
      }
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int e = tid + t * kThreads;
        Sm[(e / FMAX) * LS + e % FMAX] = vs[t];
      }
    } else {
      const int j = 2 * (tid % J2), kr = tid / J2;
#pragma unroll
      for (int t = 0; t < NQ2; ++t) *reinterpret_cast<double2*>(&U[(kr + KS * t) * LA + j]) = va[t];
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int e = tid + t * kThreads;
        Sm[(e % BK) * LS + e / BK] = vs[t];
      }
    }
  };

  const int nk = (fp + BK - 1) / BK;
  if (nk > 0) gload(0);
  for (int kt = 0; kt < nk; ++kt) {
    if (kt > 0) __syncthreads();                          // the previous chunk is consumed
    sstore();
    __syncthreads();
    if (kt + 1 < nk) gload((kt + 1) * BK);                // in flight during the products
#pragma unroll
    for (int s4 = 0; s4 < BK / 4; ++s4) {
      const int kk = 4 * s4 + kq;                         // lane's k of this MFMA k-step
      double wv[XB], nv[2];
#pragma unroll
      for (int x = 0; x < XB; ++x) wv[x] = U[kk * LA + w0 + 16 * x + l16];
#pragma unroll
      for (int y = 0; y < 2; ++y) nv[y] = Sm[kk * LS + 16 * y + l16];
#pragma unroll
      for (int x = 0; x < XB; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = part == 0 ? __builtin_amdgcn_mfma_f64_16x16x4f64(wv[x], nv[y], acc[x][y], 0, 0, 0)
                                : __builtin_amdgcn_mfma_f64_16x16x4f64(nv[y], wv[x], acc[x][y], 0, 0, 0);
    }
  }
  __syncthreads();                                        // U is reused below

  if (part == 1) {
    // C[q][j]: q = 16 y + 4 r + kq, j = r0 + w0 + 16 x + l16
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int j = r0 + w0 + 16 * x + l16;
        double gv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = 16 * y + 4 * r + kq;
          gv[r] = (q < f && j < N) ? G[(size_t)Fl[q] * N + j] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = 16 * y + 4 * r + kq;
          if (q < f && j < N)
            Ya[(size_t)(fp + q) * N + j] = (Fl[q] == j ? 1.0 : 0.0) - gv[r] + acc[x][y][r];
        }
      }
    return;
  }

  // X part: Z to LDS, then P = G0[:, F] - C with G0 gathered at the
  // accepted sites straight from memory, then Xa[:, fp + c] = P Z
  const GLOBAL double* __restrict__ Z = gp((const double*)C.Z[spin]);
  for (int e = tid; e < FMAX * FMAX; e += kThreads) {
    const int q = e / FMAX, c = e % FMAX;
    Zl[q * LP + c] = (q < f && c < f) ? Z[(size_t)q * kSegMax + c] : 0.0;
  }
  __syncthreads();
  // C[i][q]: i = w0 + 16 x + 4 r + kq, q = 16 y + l16
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int q = 16 * y + l16, col = q < f ? Fl[q] : 0;
      double gv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + w0 + 16 * x + 4 * r + kq;
        gv[r] = (q < f && i < N) ? G[(size_t)i * N + col] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double a = acc[x][y][r];
        acc[x][y][r] = q < f ? gv[r] - a : 0.0;
      }
    }
  double* Pl = U;
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = w0 + 16 * x + 4 * r + kq, q = 16 * y + l16;
        Pl[i * LP + q] = acc[x][y][r];
        acc[x][y][r] = 0.0;
      }
  __syncthreads();
  const int nsz = (f + 3) / 4;                            // MFMA k-steps over q < f
  for (int s4 = 0; s4 < nsz; ++s4) {
    const int q = 4 * s4 + kq;
    double pv[XB], zv[2];
#pragma unroll
    for (int x = 0; x < XB; ++x) pv[x] = Pl[(w0 + 16 * x + l16) * LP + q];
#pragma unroll
    for (int y = 0; y < 2; ++y) zv[y] = Zl[q * LP + 16 * y + l16];
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(pv[x], zv[y], acc[x][y], 0, 0, 0);
  }
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + w0 + 16 * x + 4 * r + kq, c = 16 * y + l16;
        if (i < N && c < f) Xa[(size_t)i * N + fp + c] = acc[x][y][r];
      }
}

// (the MFMA forms read the segment's accepted sites and offsets from the
// chain state, so they take no segment bounds)
template <int FMAX>
static void launch_xy_mfma(const ChainDev* c, int nc, int n_max, hipStream_t s) {
  constexpr int ROWS = XyMfmaShape<FMAX>::ROWS;
  const int nrb = (n_max + ROWS - 1) / ROWS;
  hipLaunchKernelGGL((k_xy_mfma<FMAX>), dim3(nc * 2 * 2 * nrb), dim3(kThreads), 0, s, c, nrb);
}

template <typename T, int FMAX>
static void launch_xy_t(const ChainDev* c, int nc, int n_max, int s0, int kseg, hipStream_t s) {
  constexpr int ROWS = XyShape<T, FMAX>::ROWS;
  const int nrb = (n_max + ROWS - 1) / ROWS;
  hipLaunchKernelGGL((k_xy<T, FMAX>), dim3(nc * 2 * 2 * nrb), dim3(kThreads), 0, s, c, nrb, s0,
                     kseg);
}

hipError_t launch_xy(int fp32, const ChainDev* c, int nc, int n_max, int s0, int kseg,
                     hipStream_t s) {
  if (kseg <= 32) {
    if (fp32) {
      launch_xy_mfma<32>(c, nc, n_max, s);
    } else {
      const int nrb = (n_max + kXy64Rows - 1) / kXy64Rows;
      hipLaunchKernelGGL(k_xy_mfma64, dim3(nc * 2 * 2 * nrb), dim3(kThreads), 0, s, c, nrb);
    }
  } else {
    if (fp32)
      launch_xy_mfma<64>(c, nc, n_max, s);
    else
      launch_xy_t<double, 64>(c, nc, n_max, s0, kseg, s);
  }
  return hipGetLastError();
}

// fact: the factored engine (FP64); dir and parity select its moving factor
// and the active buffers
hipError_t launch_scan(int fp32, int fact, const ChainDev* c, int nc, const Ctl* ctl, int l, int M,
                       int s0, int s1, int dir, int parity, hipStream_t s) {
  if (fact)
    hipLaunchKernelGGL((k_scan<double, true>), dim3(nc), dim3(kThreads), 0, s, c, ctl, l, M, s0, s1,
                       dir, parity);
  else if (fp32)
    hipLaunchKernelGGL((k_scan<float, false>), dim3(nc), dim3(kThreads), 0, s, c, ctl, l, M, s0, s1,
                       0, 0);
  else
    hipLaunchKernelGGL((k_scan<double, false>), dim3(nc), dim3(kThreads), 0, s, c, ctl, l, M, s0, s1,
                       0, 0);
  return hipGetLastError();
}

}  // namespace gpqmc

namespace gpqmc {

// fn(integral_constant<int, k>) for k = B .. E - 1, unrolled at compile time
// (the register tile of the scan is indexed by constants only)
template <int B, int E, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>{});
    static_for<B + 1, E>(fn);
  }
}

// ---------------------------------------------------------------------------
// Factored engine, delay segments of up to kBlock (32) sites: one wave per
// chain does the whole segment.
//
// Lane (s, a) = (lane / 32, lane % 32) keeps row a of the spin-s block
// G_s[S,S] = 1 - A[S,:] B[S,:]^T in registers (the block comes from the
// chain's scan buffer, formed by k_block or by the previous segment's
// update).  Every proposal reads the two diagonal entries with readlane; an
// accepted flip t at site j_t writes the row X[j_t, S] (X = 1 - G) of the
// current block to LDS, where it both feeds the Sherman-Morrison update of
// every lane's row and stays as history, and every lane also keeps X[a, j_t]
// in a register indexed by j_t.  Those rows and columns are the Schur
// complements of K = Delta_F^{-1} + X_s[F,F] (X_s: the block at the segment's
// start) in flip order, so they give K = L U directly:
//   U[t][v] = X^{(t)}[j_t, j_v] + delta_tv / Delta_t   (v >= t),
//   L[u][t] = X^{(t)}[j_u, j_t] / U[t][t]               (u > t),
// with X^{(t)} the block before flip t.  The wave then writes the Woodbury
// core Z = K^{-1} (32 x 32 per spin) to the Z buffer; k_segupd_f (or, with
// more than 128 particles, k_wf and two GEMMs) applies it.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Block of a scan segment, G_s[S, S] = 1 - A[S, :] B[S, :]^T for one chain and
// propagated spin (S: the sites [s0, s1), or for the t-V model the ends of the
// bonds of the chain's segment s0), to the chain's scan buffer as a 32 x 32
// row-major block with identity padding beyond the segment.  Tile t (0..3)
// is the 16 x 16 part (rows 16 (t / 2), columns 16 (t % 2)), formed on MFMA
// by one wave over a range of the columns of the factors with its operands
// loaded straight from memory, all loads of a chunk of 8 CH columns in
// flight at once.  (Formed inside the one-wave scan, the same block kept a
// single wave per SIMD waiting on its loads.)
// ---------------------------------------------------------------------------
template <int CH>
__device__ __forceinline__ doublex4 block_acc(const ChainDev& C, int sp, int tv, int s0, int s1,
                                              int parity, int tile, int lane, int kbeg, int kend,
                                              bool& valid) {
  doublex4 acc;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = 0.0;
  valid = false;
  const int N = C.N, nn = C.n[sp];
  const int nprop = tv ? C.n_bonds : N;
  int b0 = s0, b1 = s1;
  if (tv) {
    if (s0 >= C.n_seg) return acc;
    b0 = C.seg_start[s0];
    b1 = C.seg_start[s0 + 1];
  } else if (s0 >= N) {
    return acc;
  }
  valid = true;
  const int nseg = min(b1, nprop) - b0, nrow = tv ? 2 * nseg : nseg;
  const int l16 = lane & 15, g = lane >> 4;
  const int tm = tile >> 1, tn = tile & 1;
  const int ra = 16 * tm + l16, rc = 16 * tn + l16;
  auto site = [&](int r) { return tv ? C.bonds[2 * (b0 + (r >> 1)) + (r & 1)] : b0 + r; };
  const bool oka = ra < nrow, okc = rc < nrow;
  const GLOBAL double* __restrict__ Ar =
      gp((const double*)C.F[0][sp][parity]) + (oka ? (size_t)site(ra) * nn : 0);
  const GLOBAL double* __restrict__ Br =
      gp((const double*)C.F[1][sp][parity]) + (okc ? (size_t)site(rc) * nn : 0);
  // D[m][n] = sum_k A[S_(16 tm + m)][k] B[S_(16 tn + n)][k] over [kbeg, kend)
  // (kbeg a multiple of 8); MFMA step (st, e) of a chunk takes
  // k = k0 + 8 st + 2 g + e in lane group g, so each lane loads pairs of
  // doubles and the four lanes of a row read 64 contiguous bytes per load;
  // lane (l16, g) receives D[g + 4 i][l16]
  typedef double v2 __attribute__((ext_vector_type(2)));
  const bool vec = (nn & 1) == 0;   // rows start 16-byte aligned
  for (int k0 = kbeg; k0 < kend; k0 += 8 * CH) {
    v2 av[CH], bv[CH];
#pragma unroll
    for (int st = 0; st < CH; ++st) {
      const int k = k0 + 8 * st + 2 * g;
      if (vec && k + 1 < kend) {
        av[st] = oka ? *reinterpret_cast<const GLOBAL v2*>(Ar + k) : v2{0.0, 0.0};
        bv[st] = okc ? *reinterpret_cast<const GLOBAL v2*>(Br + k) : v2{0.0, 0.0};
      } else {
        av[st] = v2{(oka && k < kend) ? Ar[k] : 0.0, (oka && k + 1 < kend) ? Ar[k + 1] : 0.0};
        bv[st] = v2{(okc && k < kend) ? Br[k] : 0.0, (okc && k + 1 < kend) ? Br[k + 1] : 0.0};
      }
    }
#pragma unroll
    for (int st = 0; st < CH; ++st)
      if (k0 + 8 * st < kend) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st].x, bv[st].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st].y, bv[st].y, acc, 0, 0, 0);
      }
  }
  return acc;
}

// the tile's part of the block, 1 - D, to the chain's scan buffer
__device__ __forceinline__ void block_store(const ChainDev& C, int sp, int tile, int lane,
                                            const doublex4& acc) {
  const int l16 = lane & 15, g = lane >> 4;
  const int tm = tile >> 1, rc = 16 * (tile & 1) + l16;
  GLOBAL double* __restrict__ blk = gp((double*)C.scan_ws[sp]);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 16 * tm + g + 4 * i;
    blk[(size_t)r * kBlock + rc] = (r == rc ? 1.0 : 0.0) - acc[i];
  }
}

// The block of a segment whose previous segment's update did not form it (the
// first segment of a slice): one workgroup of eight waves per chain and spin,
// wave w forming tile w % 4 over one half of the columns; the second half's
// partial sums meet the first's in LDS.
__global__ __launch_bounds__(512) void k_block(const ChainDev* __restrict__ chains, int tv, int s0,
                                               int s1, int parity) {
  const int cs = xcd_remap(blockIdx.x, gridDim.x), sp = cs & 1;
  const ChainDev& C = chains[cs >> 1];
  if (sp >= C.nsp) return;
  __shared__ double part[4 * 64 * 4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = wave & 3, half = wave >> 2, nn = C.n[sp];
  const int kh = min(8 * ((nn + 15) / 16), nn);   // a multiple of 8
  bool valid;
  doublex4 acc = block_acc<8>(C, sp, tv, s0, s1, parity, tile, lane, half ? kh : 0,
                              half ? nn : kh, valid);
  if (!valid) return;   // the same for the whole workgroup
  double* pp = part + (tile * 64 + lane) * 4;
  if (half) {
#pragma unroll
    for (int i = 0; i < 4; ++i) pp[i] = acc[i];
  }
  __syncthreads();
  if (!half) {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += pp[i];
    block_store(C, sp, tile, lane, acc);
  }
}

template <bool TV>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_scan_f(const ChainDev* __restrict__ chains,
                                               const Ctl* __restrict__ ctl, int l, int M, int s0,
                                               int s1, int dir, int parity) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  ChainState* st = C.st;
  const int N = C.N, lane = threadIdx.x, s = lane >> 5, a = lane & 31;
  // proposals of a slice: sites [s0, s1) (Hubbard), or the bonds of the
  // chain's scan segment s0 (t-V, two block rows per bond)
  const int nprop = TV ? C.n_bonds : N;
  if (TV ? s0 >= C.n_seg : s0 >= nprop) {   // this chain has no proposal in the segment
    if (lane == 0) st->fcount = 0;
    return;
  }
  if (TV) {
    const int k = s0;
    s0 = C.seg_start[k];
    s1 = C.seg_start[k + 1];
  }
  const int send = min(s1, nprop), nseg = send - s0;
  const int nrow = TV ? 2 * nseg : nseg;   // block rows (sites)
  constexpr int KB = kBlock;
  __shared__ double u_s[KB];
  __shared__ int8_t fs[KB];       // fields of the segment's proposals
  __shared__ int8_t fs0[KB];      // the same before the scan
  __shared__ int8_t es[KB];       // sublattice signs of the block's sites
  __shared__ int srow[KB];        // site of every block row
  __shared__ int Fl[KB];
  __shared__ double dF[2][KB];    // Delta of every accepted flip, per spin
  // history rows X^{(t)}[j_t, S] (later the LU factors); the history columns
  // X^{(t)}[a, j_t] stay in each lane's registers (hc, indexed by the site
  // j_t), and tpos maps a site to its flip index (-1: not flipped)
  __shared__ __align__(16) double hrow[2][KB][KB];
  __shared__ int8_t tpos[KB];

  const int bnd = (l == 0 || l == M + 1) ? 0 : 1;
  int8_t* frow = C.field + (size_t)l * nprop;
  const uint32_t sweep = (uint32_t)st->sweep;
  const bool force_reject = ctl->force_reject != 0;
  // lane j < 32 also keeps proposal j's uniform and field in registers (read
  // by readlane in the site loop)
  double my_u = 0.0;
  int my_f = 1;
  if (lane < nseg) {
    uint32_t c[4] = {C.chain_id, sweep, (uint32_t)l, (uint32_t)(s0 + lane)};
    philox4x32_10(c, C.key0, C.key1);
    my_u = uniform53(c[0], c[1]);
    u_s[lane] = my_u;
    my_f = frow[s0 + lane];
    fs[lane] = (int8_t)my_f;
    fs0[lane] = (int8_t)my_f;
  }
  if (lane < KB) tpos[lane] = -1;
  int my_site = 0;
  if (a < nrow) {
    my_site = TV ? C.bonds[2 * (s0 + (a >> 1)) + (a & 1)] : s0 + a;
    if (s == 0) {
      srow[a] = my_site;
      es[a] = C.eps[my_site];
    }
  }
  wave_sync();
  const bool ph = C.ph != 0;

  // ---- G_s[S,S] = 1 - A[S,:] B[S,:]^T (formed by k_block), row a of spin s
  // in g; with the particle-hole shortcut spin 1 is mirrored below ----
  double g[KB];
  double hc[KB];   // hc[j] = X^{(t)}[a, j] of the flip t at site j
  {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const GLOBAL double* __restrict__ blk = gp((const double*)C.scan_ws[s]) + (size_t)a * KB;
    const bool ok = s < C.nsp;
#pragma unroll
    for (int c = 0; c < KB; c += 2) {
      const v2 v = ok ? *reinterpret_cast<const GLOBAL v2*>(blk + c) : v2{0.0, 0.0};
      g[c] = ok ? v.x : (c == a ? 1.0 : 0.0);
      g[c + 1] = ok ? v.y : (c + 1 == a ? 1.0 : 0.0);
    }
  }
  if (ph) {
    // G_1[a][c] = delta_ac - eps_a eps_c G_0[c][a]: spin-0 lane c stores its
    // row (stride KB + 1: conflict-free both ways), spin-1 lane a reads column a
    double* T = &hrow[0][0][0];   // 32 x 33 doubles, before any history row
    if (s == 0) {
#pragma unroll
      for (int q = 0; q < KB; ++q) T[a * (KB + 1) + q] = g[q];
    }
    wave_sync();
    if (s == 1 && a < nseg) {
      const double ea = (double)es[a];
#pragma unroll
      for (int c = 0; c < KB; ++c)
        if (c < nseg) g[c] = (c == a ? 1.0 : 0.0) - ea * (double)es[c] * T[c * (KB + 1) + a];
    }
    wave_sync();
  }

  // ---- sequential proposals ----
  const bool zero_delta = C.delta[bnd][0][0] == 0.0 && C.delta[bnd][0][1] == 0.0;
  const double dl_u0 = C.delta[bnd][0][0], dl_u1 = C.delta[bnd][0][1];
  const double dl_d0 = C.delta[bnd][1][0], dl_d1 = C.delta[bnd][1][1];
  double* const trace_ratio = C.trace_ratio;
  int fc = 0, sign = st->sign, nacc = 0;
  if constexpr (TV) {
    // one rank-1 step of the block at row j with flip factor dl and ratio rl:
    // X[j, S] to the history rows, X[S, j] to the history columns,
    // G <- G - (dl / rl) G[:, j] X[j, :]
    auto rank1 = [&](auto jc, double dl, double rl, double dl_other) {
      constexpr int j = decltype(jc)::value;
      const int t = fc;
      if (a == j) {
#pragma unroll
        for (int q = 0; q < KB; q += 2) {
          double2 v;
          v.x = (q == j ? 1.0 : 0.0) - g[q];
          v.y = (q + 1 == j ? 1.0 : 0.0) - g[q + 1];
          *reinterpret_cast<double2*>(&hrow[s][t][q]) = v;
        }
      }
      hc[j] = (a == j ? 1.0 : 0.0) - g[j];
      wave_sync();
      const double cg = (dl / rl) * g[j];
#pragma unroll
      for (int q = 0; q < KB; q += 2) {
        const double2 x2 = *reinterpret_cast<const double2*>(&hrow[s][t][q]);
        g[q] -= cg * x2.x;
        g[q + 1] -= cg * x2.y;
      }
      if (lane == 0) {
        Fl[t] = j;
        tpos[j] = (int8_t)t;
        dF[0][t] = dl;
        dF[1][t] = dl_other;
      }
      fc = t + 1;
    };
    // bond (i, j) = block rows (2t, 2t + 1): Delta_i = e^{-2 c s} - 1 (the up
    // entry), Delta_j = e^{+2 c s} - 1 (the down entry); the ratio
    // det(1 + Delta_F X[F, F]) is the product of two rank-1 ratios, the
    // second taken after the first update
    static_for<0, KB / 2>([&](auto tc) {
      constexpr int t = decltype(tc)::value, p = 2 * t, q = 2 * t + 1;
      if (t < nseg) {
        const int si = fs[t] > 0 ? 0 : 1;
        const double di = C.delta[bnd][0][si], dj = C.delta[bnd][1][si];
        const double gpp = lane_value(g[p], p), gpq = lane_value(g[q], p);
        const double gqp = lane_value(g[p], q), gqq = lane_value(g[q], q);
        const double r1 = 1.0 + di * (1.0 - gpp);
        const double r2 = 1.0 + dj * ((1.0 - gqq) - (di / r1) * gqp * gpq);
        const double r = r1 * r2;
        const bool accept = !force_reject && (u_s[t] < fabs(r));
        if (lane == 0 && trace_ratio) {
          trace_ratio[((size_t)l * nprop + s0 + t) * 2 + 0] = r;
          trace_ratio[((size_t)l * nprop + s0 + t) * 2 + 1] = 0.0;
        }
        if (accept) {
          if (!zero_delta) {
            rank1(std::integral_constant<int, p>{}, di, r1, 0.0);
            const double r2b = 1.0 + dj * (1.0 - lane_value(g[q], q));
            rank1(std::integral_constant<int, q>{}, dj, r2b, 0.0);
          }
          if (lane == 0) fs[t] = (int8_t)(-fs[t]);
          if (r < 0) sign = -sign;
          nacc += 1;
        }
      }
    });
  } else {
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    if (j < nseg) {
      const int si = __builtin_amdgcn_readlane(my_f, j) > 0 ? 0 : 1;
      const double du = si ? dl_u1 : dl_u0, dd = si ? dl_d1 : dl_d0;
      const double ru = 1.0 + du * (1.0 - lane_value(g[j], j));
      const double rd = 1.0 + dd * (1.0 - lane_value(g[j], 32 + j));
      const bool accept = !force_reject && (lane_value(my_u, j) < fabs(ru * rd));
      if (lane == 0 && trace_ratio) {
        trace_ratio[((size_t)l * N + s0 + j) * 2 + 0] = ru;
        trace_ratio[((size_t)l * N + s0 + j) * 2 + 1] = rd;
      }
      if (accept) {
        if (!zero_delta) {
          const int t = fc;
          // X[j, S] = e_j - G[j, S] from lane (s, j); X[a, j] from every lane
          if (a == j) {
#pragma unroll
            for (int q = 0; q < KB; q += 2) {
              double2 v;
              v.x = (q == j ? 1.0 : 0.0) - g[q];
              v.y = (q + 1 == j ? 1.0 : 0.0) - g[q + 1];
              *reinterpret_cast<double2*>(&hrow[s][t][q]) = v;
            }
          }
          hc[j] = (a == j ? 1.0 : 0.0) - g[j];
          wave_sync();
          // Sherman-Morrison: G <- G - (Delta / r) G[:, j] X[j, :]
          const double cg = (s == 0 ? du / ru : dd / rd) * g[j];
#pragma unroll
          for (int q = 0; q < KB; q += 2) {
            const double2 x2 = *reinterpret_cast<const double2*>(&hrow[s][t][q]);
            g[q] -= cg * x2.x;
            g[q + 1] -= cg * x2.y;
          }
          if (lane == 0) {
            Fl[t] = j;
            tpos[j] = (int8_t)t;
            dF[0][t] = du;
            dF[1][t] = dd;
          }
          fc = t + 1;
        }
        if (lane == j) my_f = -my_f;
        if (ru * rd < 0) sign = -sign;
        nacc += 1;
      }
    }
  }
  }
  wave_sync();
  const int f = fc;
  if (lane < nseg) frow[s0 + lane] = TV ? fs[lane] : (int8_t)my_f;
  if constexpr (TV) {
    // site exponents of the flipped bonds: the A end changes by -2 s_old, the
    // B end by +2 s_old
    if (s == 0 && a < nrow) {
      const int8_t so = fs0[a >> 1];
      if (fs[a >> 1] != so) {
        int8_t* m = C.mexp + (size_t)l * N + srow[a];
        *m = (int8_t)(*m + ((a & 1) ? 2 * so : -2 * so));
      }
    }
  }
  if (lane < f) C.flist[lane] = srow[Fl[lane]];
  if (s < C.nsp && a < f) C.dflist[s * kSegMax + a] = dF[s][a];
  if (lane == 0) {
    st->fcount = f;
    st->foff = 0;
    st->ftot = f;
    st->sign = sign;
    st->accepted += nacc;
    st->proposed += nseg;
  }
  if (f == 0) return;

  // ---- K = Delta_F^{-1} + X_s[F,F] = L U, packed in place of the history
  // rows; first the reciprocal pivots 1 / U[v][v], one per lane ----
  __shared__ double pinv[2][KB];
  {
    const double dinv = a < f ? 1.0 / dF[s][a] : 0.0;
    if (a < f) pinv[s][a] = 1.0 / (hrow[s][a][Fl[a]] + dinv);
    wave_sync();
    // U: lane (s, u) compacts its history row u to the flip order,
    // U[u][v] = X^{(u)}[j_u, j_v] + delta_uv / Delta_u for v >= u; in place,
    // since j_v >= v grows with v, no column is overwritten before it is read
    if (a < f) {
      // eight reads in flight, then their writes: a chunk's writes land left
      // of every later chunk's reads
      double* row = &hrow[s][a][0];
#pragma unroll
      for (int c0 = 0; c0 < KB; c0 += 8) {
        double tv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int v = c0 + q;
          tv[q] = (v >= a && v < f) ? row[Fl[v] & (KB - 1)] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int v = c0 + q;
          if (v >= a && v < f) row[v] = tv[q] + (v == a ? dinv : 0.0);
        }
      }
    }
    // L: the lane of site j_u holds X^{(v)}[j_u, j_v] for the earlier flips v
    // in hc[j_v]: L[u][v] = X^{(v)}[j_u, j_v] / U[v][v] (columns v < u of row
    // u, which the compaction above leaves alone)
    const int u = tpos[a];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int v = tpos[j];
      if (v >= 0 && v < u) hrow[s][u][v] = hc[j] * pinv[s][v];
    }
    wave_sync();
  }
  // ---- the Woodbury core Z = K^{-1} = U^{-1} L^{-1}: lane (s, c) forms
  // column c (L y = e_c forward, then U z = y backward, over the f accepted
  // flips; beyond f, K and Z are the identity) and writes it to the chain's
  // Z buffer (row-major, 32 x 32) ----
  if (s < C.nsp) {
    // two accumulators per dot product and 16-byte row reads; past f the
    // packed rows hold finite history entries and y, z are zero there, so
    // the sums run over whole rows without a guard per entry
    double zc[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      double v0 = (i == a) ? 1.0 : 0.0, v1 = 0.0;
      if (i < f && a < f) {
        const double* row = &hrow[s][i][0];
#pragma unroll
        for (int j = 0; j + 1 < i; j += 2) {
          const double2 r = *reinterpret_cast<const double2*>(row + j);
          v0 -= r.x * zc[j];
          v1 -= r.y * zc[j + 1];
        }
        if (i & 1) v0 -= row[i - 1] * zc[i - 1];
      }
      zc[i] = v0 + v1;
    }
#pragma unroll
    for (int i = KB - 1; i >= 0; --i) {
      if (i < f && a < f) {
        const double* row = &hrow[s][i][0];
        double v0 = zc[i], v1 = 0.0;
        if (((i + 1) & 1) && i + 1 < KB) v0 -= row[i + 1] * zc[i + 1];
#pragma unroll
        for (int j = (i + 2) & ~1; j + 1 < KB; j += 2) {
          const double2 r = *reinterpret_cast<const double2*>(row + j);
          v0 -= r.x * zc[j];
          v1 -= r.y * zc[j + 1];
        }
        zc[i] = (v0 + v1) * pinv[s][i];
      }
    }
    GLOBAL double* __restrict__ z = gp((double*)C.Z[s]);
#pragma unroll
    for (int i = 0; i < KB; ++i) z[(size_t)i * KB + a] = zc[i];
  }
}

// ---------------------------------------------------------------------------
// Woodbury rows of a segment for the general segment update (N_sigma > 128;
// factored engine, after k_scan_f), one workgroup per chain and spin, a thread
// per column k of the factors: Mf = M[F, k] (the moving factor's rows at the
// accepted sites, which are then scaled by 1 + Delta_F), and Wf = Z^T Q[F, k]
// (upward) or Z Q[F, k] (downward) with the Woodbury core Z = K^{-1} the scan
// left in the Z buffer.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_wf(const ChainDev* __restrict__ chains, int dir,
                                            int parity) {
  constexpr int KB = kBlock;
  const int cs = xcd_remap(blockIdx.x, gridDim.x), sp = cs & 1;
  const ChainDev& C = chains[cs >> 1];
  const int f = C.st->fcount;
  if (f == 0 || sp >= C.nsp) return;
  const int nn = C.n[sp], tid = threadIdx.x;
  __shared__ double Zs[KB][KB + 1];   // Zs[p][q]: coefficient of Q[F_q] in Wf row p
  __shared__ int Fs[KB];
  __shared__ double dF[KB];
  const GLOBAL double* __restrict__ z = gp((const double*)C.Z[sp]);
  for (int idx = tid; idx < KB * KB; idx += 128) {
    const int r = idx / KB, c = idx % KB;
    if (dir == 0)
      Zs[c][r] = z[idx];
    else
      Zs[r][c] = z[idx];
  }
  if (tid < f) {
    Fs[tid] = C.flist[tid];
    dF[tid] = C.dflist[sp * kSegMax + tid];
  }
  __syncthreads();
  GLOBAL double* __restrict__ Mv = gp((double*)C.F[dir][sp][parity]);
  const GLOBAL double* __restrict__ Qv = gp((const double*)C.F[1 - dir][sp][parity]);
  GLOBAL double* __restrict__ mf = gp(C.Mf[sp]);
  GLOBAL double* __restrict__ wf = gp(C.Wf[sp]);
  for (int k = tid; k < nn; k += 128) {
#pragma unroll 4
    for (int p = 0; p < f; ++p) {
      const size_t o = (size_t)Fs[p] * nn + k;
      const double v = Mv[o];
      mf[(size_t)p * nn + k] = v;
      Mv[o] = v * (1.0 + dF[p]);
    }
    double y[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) y[q] = q < f ? Qv[(size_t)Fs[q] * nn + k] : 0.0;
#pragma unroll 1
    for (int p = 0; p < f; ++p) {
      double w = 0.0;
#pragma unroll
      for (int q = 0; q < KB; ++q) w += Zs[p][q] * y[q];
      wf[(size_t)p * nn + k] = w;
    }
  }
}

// ---------------------------------------------------------------------------
// Segment update of the dual factor, Q <- Q - (Q Mf^T) Wf (Q: N x n, Mf and
// Wf: f x n, f <= 32, n <= 128), on MFMA (v_mfma_f64_16x16x4f64).  One
// workgroup of 8 waves per chain and spin stages Mf (transposed) and Wf in
// LDS once (zero-padded to 32 flips and 128 columns; 74 KB, so two
// workgroups share a CU and one's staging overlaps the other's streaming)
// and walks the rows of Q in tiles of 128, 16 per wave.  Q is read and
// written once, each lane moving 32 contiguous bytes of a row per column
// block (two 16-byte accesses).  Grid: chains x 2 spins.
// ---------------------------------------------------------------------------
constexpr int kUpdWaves = 8;                // waves per workgroup (two workgroups per CU)
constexpr int kUpdThreads = 64 * kUpdWaves;
constexpr int kUpdRows = 16 * kUpdWaves;     // rows of Q per tile (16 per wave)

// Lane (l16, g) = (lane % 16, lane / 16) keeps x[bb][i] = Q[row][16 bb + 4 g + i]
// of its row l16: the contraction order over the columns is free, so MFMA
// step i of column block bb gives k slot g the column 16 bb + 4 g + i.  First
// product, P^T = Mf Q^T (A = Mf from LDS, B = the row's Q values): lane
// (l16, g) receives P[row][16 jb + g + 4 r], which is exactly its B operand
// of the second product Out^T = Wf'^T P^T (k slot g of step (jb, r) = flip
// 16 jb + g + 4 r; steps past the last flip are skipped).  The output rows
// of the second product are the columns of Q permuted by
// m = g' + 4 i' -> 4 g' + i', so its result D[g + 4 i][l16] lands on x[bb][i]
// and P never leaves the registers.  LDS strides: Mf^T rows (one per column
// of Q) 36 doubles, Wf rows 144: every operand read of a half-wave hits 32
// distinct double slots.
constexpr int kUpdLDT = kBlock + 4;          // LDS row of Mf^T (one per column of Q)
constexpr int kUpdLDW = 8 * 16 + 16;         // LDS row of Wf
__device__ __forceinline__ void segupd_body(const ChainDev& C, int sp, int f, int N, int nn,
                                            int dir, int parity, int tid, int lane, int wave,
                                            double* MsT, double* Ws, int* Fs, double* dFs) {
  constexpr int KB = kBlock;
  constexpr int NB = 8;                  // 16-column blocks of Q (n <= 128)
  constexpr int LDT = kUpdLDT;
  constexpr int LDW = kUpdLDW;
  GLOBAL double* __restrict__ Mv = gp((double*)C.F[dir][sp][parity]);
  GLOBAL double* __restrict__ Qb = gp((double*)C.F[1 - dir][sp][parity]);
  const int nb = (nn + 15) / 16;
  const int njb = f > 16 ? 2 : 1;        // 16-flip blocks with accepted flips
  const int l16 = lane & 15, g = lane >> 4;
  // Staging: Mf = M[F, :] (the moving factor's rows at the accepted sites,
  // zero-padded to 32 x 128) to LDS, transposed, after which those rows of M
  // are scaled by 1 + Delta_F; and Wf = Z^T Q[F, :] (upward) or Z Q[F, :]
  // (downward) on MFMA, 16 x 16 tiles (flip block pb, column block cb), at
  // most two per wave, from the rows of Q before any of them is updated.  The
  // Z operands load before F is known, then every gathered row at once.
  const GLOBAL double* __restrict__ zg = gp((const double*)C.Z[sp]);
  const int ntiles = njb * nb;
  static_assert(2 * kUpdWaves >= 2 * NB, "two Wf tiles per wave cover 32 flips x 128 columns");
  double za[2][KB / 4];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = wave + u * kUpdWaves, pb = t / nb;
#pragma unroll
    for (int st = 0; st < KB / 4; ++st) {
      const int q = 4 * st + g;
      const bool ok = t < ntiles && q < f;
      za[u][st] = ok ? (dir == 0 ? zg[(size_t)q * KB + 16 * pb + l16]
                                 : zg[(size_t)(16 * pb + l16) * KB + q])
                     : 0.0;
    }
  }
  if (tid < f) {
    Fs[tid] = C.flist[tid];
    dFs[tid] = C.dflist[sp * kSegMax + tid];
  }
  __syncthreads();
  constexpr int NC = NB * 16;
  constexpr int NS = KB * NC / kUpdThreads;
  static_assert(NS * kUpdThreads == KB * NC, "staging covers the tiles");
  double vm[NS], qv[2][KB / 4];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int idx = tid + t * kUpdThreads, j = idx / NC, k = idx - j * NC;
    vm[t] = (j < f && k < nn) ? Mv[(size_t)Fs[j] * nn + k] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = wave + u * kUpdWaves, col = 16 * (t % nb) + l16;
#pragma unroll
    for (int st = 0; st < KB / 4; ++st) {
      const int q = 4 * st + g;
      const bool ok = t < ntiles && q < f && col < nn;
      qv[u][st] = ok ? Qb[(size_t)Fs[ok ? q : 0] * nn + col] : 0.0;
    }
  }
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int idx = tid + t * kUpdThreads, j = idx / NC, k = idx - j * NC;
    MsT[k * LDT + j] = vm[t];
    if (j < f && k < nn) Mv[(size_t)Fs[j] * nn + k] = vm[t] * (1.0 + dFs[j]);
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = wave + u * kUpdWaves;
    if (t < ntiles) {
      const int pb = t / nb, col = 16 * (t - pb * nb) + l16;
      doublex4 acc;
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = 0.0;
#pragma unroll
      for (int st = 0; st < KB / 4; ++st)
        if (4 * st < f) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(za[u][st], qv[u][st], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) Ws[(16 * pb + g + 4 * i) * LDW + col] = acc[i];
    }
  }
  __syncthreads();   // Q[F, :] read by every wave before any row of Q is updated
  typedef double v2 __attribute__((ext_vector_type(2)));
  const bool vec = (nn & 1) == 0;        // rows start 16-byte aligned
  const int cm = 4 * (l16 & 3) + (l16 >> 2);   // column of Q of output row l16
  for (int row = wave * 16 + l16; row - l16 < N; row += kUpdRows) {
    const bool rok = row < N;
    GLOBAL double* __restrict__ q = Qb + (size_t)row * nn;
    double x[NB][4];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 16 * bb + 4 * g + 2 * h;
        if (vec && rok && k + 1 < nn) {
          const v2 v = *reinterpret_cast<const GLOBAL v2*>(q + k);
          x[bb][2 * h] = v.x;
          x[bb][2 * h + 1] = v.y;
        } else {
          x[bb][2 * h] = (rok && k < nn) ? q[k] : 0.0;
          x[bb][2 * h + 1] = (rok && k + 1 < nn) ? q[k + 1] : 0.0;
        }
      }
    // P^T = Mf Q^T: pacc[jb][r] = P[row][16 jb + g + 4 r]
    doublex4 pacc[2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) pacc[jb][r] = 0.0;
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      if (bb < nb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 16 * bb + 4 * g + i;
#pragma unroll
          for (int jb = 0; jb < 2; ++jb)
            if (jb < njb)
              pacc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(MsT[k * LDT + 16 * jb + l16], x[bb][i],
                                                              pacc[jb], 0, 0, 0);
        }
      }
    }
    // Out^T = Wf'^T P^T per 16-column block of Q, over the accepted flips
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      if (bb < nb) {
        doublex4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = 0.0;
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
          if (jb < njb) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (16 * jb + 4 * r < f)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(
                    Ws[(16 * jb + g + 4 * r) * LDW + 16 * bb + cm], pacc[jb][r], acc, 0, 0, 0);
          }
#pragma unroll
        for (int i = 0; i < 4; ++i) x[bb][i] -= acc[i];
      }
    }
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 16 * bb + 4 * g + 2 * h;
        if (vec && rok && k + 1 < nn) {
          *reinterpret_cast<GLOBAL v2*>(q + k) = v2{x[bb][2 * h], x[bb][2 * h + 1]};
        } else {
          if (rok && k < nn) q[k] = x[bb][2 * h];
          if (rok && k + 1 < nn) q[k + 1] = x[bb][2 * h + 1];
        }
      }
  }
}

__global__ __launch_bounds__(kUpdThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_segupd_f(const ChainDev* __restrict__ chains, int dir, int parity, int tv, int ns0,
                int ns1) {
  const int cs = xcd_remap(blockIdx.x, gridDim.x), sp = cs & 1;
  const ChainDev& C = chains[cs >> 1];
  const int N = C.N, nn = C.n[sp], tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = C.st->fcount;
  if (sp >= C.nsp) return;
  __shared__ __align__(16) double MsT[8 * 16 * kUpdLDT];
  __shared__ __align__(16) double Ws[kBlock * kUpdLDW];
  __shared__ int Fs[kBlock];
  __shared__ double dFs[kBlock];
  if (f > 0) segupd_body(C, sp, f, N, nn, dir, parity, tid, lane, wave, MsT, Ws, Fs, dFs);
  // the next segment's block from the updated factors (ns0 < 0: none): wave
  // w forms tile w % 4 over one half of the columns, the second half's
  // partial sums meet the first's in LDS
  if (ns0 >= 0) {
    __syncthreads();   // every row of the dual factor written, MsT free
    const int tile = wave & 3, half = wave >> 2;
    const int kh = min(8 * ((nn + 15) / 16), nn);   // a multiple of 8
    bool valid;
    doublex4 acc = block_acc<8>(C, sp, tv, ns0, ns1, parity, tile, lane, half ? kh : 0,
                                half ? nn : kh, valid);
    if (valid) {   // the same for the whole workgroup
      double* part = MsT + (size_t)(tile * 64 + lane) * 4;
      if (half) {
#pragma unroll
        for (int i = 0; i < 4; ++i) part[i] = acc[i];
      }
      __syncthreads();
      if (!half) {
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += part[i];
        block_store(C, sp, tile, lane, acc);
      }
    }
  }
}


// form_block: launch k_block first (the segment's block was not formed by
// the previous segment's update)
hipError_t launch_scan_f(int tv, const ChainDev* c, int nc, const Ctl* ctl, int l, int M, int s0,
                         int s1, int dir, int parity, int form_block, hipStream_t s) {
  if (form_block) {
    hipLaunchKernelGGL(k_block, dim3(2 * nc), dim3(512), 0, s, c, tv, s0, s1, parity);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  }
  if (tv)
    hipLaunchKernelGGL(k_scan_f<true>, dim3(nc), dim3(64), 0, s, c, ctl, l, M, s0, s1, dir, parity);
  else
    hipLaunchKernelGGL(k_scan_f<false>, dim3(nc), dim3(64), 0, s, c, ctl, l, M, s0, s1, dir, parity);
  return hipGetLastError();
}

hipError_t launch_wf(const ChainDev* c, int nc, int dir, int parity, hipStream_t s) {
  hipLaunchKernelGGL(k_wf, dim3(2 * nc), dim3(128), 0, s, c, dir, parity);
  return hipGetLastError();
}

// n_max: the largest lattice of the batch (rows of Q per chain and spin)
// ns0 >= 0: the update also forms the block of the segment [ns0, ns1) (t-V:
// the chains' segment ns0), which the next scan then reads
hipError_t launch_segupd_f(int tv, const ChainDev* c, int nc, int dir, int parity, int ns0, int ns1,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_segupd_f, dim3(2 * nc), dim3(kUpdThreads), 0, s, c, dir, parity, tv, ns0,
                     ns1);
  return hipGetLastError();
}

}  // namespace gpqmc
