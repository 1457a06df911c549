// Metropolis scan of one segment of one imaginary-time slice (gfx950).
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
// The kernel ends by writing the operands of (*), Xg = G0[:,F] and
// Yg = (1 - G0)[F,:]; the T1 = Z Yg and FLUSH G -= Xg T1 GEMMs apply the
// update to the whole Green's function (a delayed update of rank |F|).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gpqmc_device.h"

namespace gpqmc {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan(const ChainDev* __restrict__ chains,
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
  constexpr int KP = kBlock + 1;
  constexpr int LDZ = kSegMax;

  __shared__ double u_s[kSegMax];
  __shared__ int8_t fs[kSegMax];
  __shared__ int Fs[kSegMax];
  __shared__ T Hs[2][kBlock][KP];
  __shared__ T Gt[2][kBlock][KP];
  __shared__ T Zb[2][kBlock][KP];
  __shared__ T rowb[2][kBlock], uvec[2][kBlock], vvec[2][kBlock];
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
          Gt[s][a][c] = acc;
          Hs[s][a][c] = acc;
        }
      }
    }
    __syncthreads();

    // ---- sequential proposals of the block: one wave, rank-1 updates ----
    // lane = (spin s, row a): colb/rowb, u/v and the row-wise updates
    if (wave == 0) {
      const int s = lane >> 5, a = lane & 31;
      int fb = 0, sign = sh_sign, nacc = 0;
      for (int j = 0; j < kb; ++j) {
        const int li = b0 + j - s0;
        const int si = fs[li] > 0 ? 0 : 1;
        const double du = C.delta[bnd][0][si], dd = C.delta[bnd][1][si];
        const double ru = 1.0 + du * (1.0 - (double)Gt[0][j][j]);
        const double rd = 1.0 + dd * (1.0 - (double)Gt[1][j][j]);
        const bool accept = !force_reject && (u_s[li] < fabs(ru * rd));
        if (lane == 0 && C.trace_ratio) {
          C.trace_ratio[((size_t)l * N + b0 + j) * 2 + 0] = ru;
          C.trace_ratio[((size_t)l * N + b0 + j) * 2 + 1] = rd;
        }
        if (!accept) continue;
        if (!zero_delta) {
          T col = T(0);
          if (a < kb) {
            col = Gt[s][a][j];
            rowb[s][a] = (a == j ? T(1) : T(0)) - Gt[s][j][a];
          }
          T uu = (a == fb) ? T(1) : T(0), vv = uu;
          if (a < fb) {   // row/column fb of Zb is the new (still zero) one
            for (int c = 0; c < fb; ++c) {
              uu += Zb[s][a][c] * Hs[s][Fb[c]][j];
              vv += Zb[s][c][a] * Hs[s][j][Fb[c]];
            }
          }
          if (a <= fb) {
            uvec[s][a] = uu;
            vvec[s][a] = vv;
          }
          wave_sync();
          const T coef = (T)((s == 0 ? du : dd) / (s == 0 ? ru : rd));
          if (a < kb) {
            const T cc = coef * col;
            for (int bb = 0; bb < kb; ++bb) Gt[s][a][bb] -= cc * rowb[s][bb];
          }
          const int fb1 = fb + 1;
          if (a < fb1) {
            const T cu = coef * uu;
            for (int q = 0; q < fb1; ++q) {
              const T base = (a < fb && q < fb) ? Zb[s][a][q] : T(0);
              Zb[s][a][q] = base + cu * vvec[s][q];
            }
          }
          if (lane == 0) Fb[fb] = j;
          fb = fb1;
        }
        if (lane == 0) fs[li] = (int8_t)(-fs[li]);
        if (ru * rd < 0) sign = -sign;
        nacc += 1;
        wave_sync();
      }
      if (lane == 0) {
        sh_fb = fb;
        sh_sign = sign;
        sh_acc += nacc;
      }
    }
    __syncthreads();

    // ---- merge the block's Zb into Z ----
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
              for (int d = 0; d < fb; ++d) acc += Pm[s][p * kBlock + d] * Zb[s][d][c];
              PZ[s][p * kBlock + c] = acc;
            }
          for (int c = wave; c < fb; c += 4)
            for (int q = lane; q < f; q += 64) {
              T acc = 0;
              for (int d = 0; d < fb; ++d) acc += Zb[s][c][d] * Qm[s][d * LDZ + q];
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
          for (int d = lane; d < fb; d += 64) Z[s][(size_t)(f + c) * LDZ + f + d] = Zb[s][c][d];
      if (tid < fb) Fs[f + tid] = b0 + Fb[tid];
      __syncthreads();
      if (tid == 0) sh_f = f + fb;
      __syncthreads();
    }
  }

  // operands of the flush: Xg = G0[:, F] (ld LDZ), Yg = (1 - G0)[F, :]
  const int f = sh_f;
  for (int s = 0; s < 2; ++s) {
    T* Xg = (T*)C.Xg[s];
    T* Yg = (T*)C.Yg[s];
    for (int i = wave; i < N; i += 4)
      for (int p = lane; p < f; p += 64) Xg[(size_t)i * LDZ + p] = G0[s][(size_t)i * N + Fs[p]];
    for (int p = wave; p < f; p += 4) {
      const int site = Fs[p];
      const T* src = G0[s] + (size_t)site * N;
      for (int j = lane; j < N; j += 64) Yg[(size_t)p * N + j] = (site == j ? T(1) : T(0)) - src[j];
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

hipError_t launch_scan(int fp32, const ChainDev* c, int nc, const Ctl* ctl, int l, int M, int s0,
                       int s1, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_scan<float>, dim3(nc), dim3(kThreads), 0, s, c, ctl, l, M, s0, s1);
  else
    hipLaunchKernelGGL(k_scan<double>, dim3(nc), dim3(kThreads), 0, s, c, ctl, l, M, s0, s1);
  return hipGetLastError();
}

}  // namespace gpqmc
