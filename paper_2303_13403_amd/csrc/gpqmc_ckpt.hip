// Checkpoint (re-stabilisation) and bookkeeping kernels of the PQMC sweep
// (gfx950).  At a checkpoint the propagated N x n basis U is re-orthonormalised
// in FP64 by Cholesky QR: U = Q T with T the Cholesky factor of U^T U and
// Q = U T^{-1} (the Gram matrix and Q are batched MFMA GEMMs; the n x n
// Cholesky factorisation and T^{-1} run here, in LDS).  Only span(Q) and the
// exact factorisation U = Q T matter (the Green's function is invariant under
// R -> R T), so one pass suffices: Q is orthonormal to O(eps cond(U)^2).  The
// fresh Green's function
// G = 1 - R (L R)^{-1} L follows from the inverse of the n x n overlap L R
// (Gauss-Jordan with partial pivoting, in LDS) and two more GEMMs; log|det|
// and the sign of each factor are accumulated for the sign check.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gpqmc_device.h"

namespace gpqmc {

// The n x n factorisations below run with kDenseThreads threads (16 waves), so
// that one workgroup per CU (the LDS copy takes up to 130 KB) still hides LDS
// latency.  Loops are two-dimensional (wave -> rows, lane -> columns): no
// integer division in the inner loops.
constexpr int kDenseThreads = 1024;
constexpr int kDenseWaves = kDenseThreads / 64;

// Work copy of an n x n matrix: in LDS with an odd leading dimension n + 1 when
// n <= kLdsDense, else in place in global memory (leading dimension n).
struct Dense {
  double* a;
  int ld;
};

__device__ inline Dense dense_load(double* lds, double* global, int n) {
  if (n > kLdsDense) return Dense{global, n};
  const int ld = n + 1, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = wave; r < n; r += kDenseWaves)
    for (int c = lane; c < n; c += 64) lds[r * ld + c] = global[(size_t)r * n + c];
  __syncthreads();
  return Dense{lds, ld};
}

__device__ inline void dense_store(const Dense& A, double* global, int n, bool upper_only) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = wave; r < n; r += kDenseWaves)
    for (int c = lane; c < n; c += 64)
      global[(size_t)r * n + c] = (upper_only && c < r) ? 0.0 : A.a[r * A.ld + c];
}

// In-place Gauss-Jordan inversion with partial (row) pivoting; the column
// interchanges are undone in reverse order at the end.  triangular: the input
// is upper triangular with nonzero diagonal (no pivoting; elimination only
// touches rows above the pivot and columns from it on).  Returns log|det| and
// the sign of det (0 if singular) to every thread.
__device__ void gj_invert(const Dense& D, int n, bool triangular, double* colk, int* piv,
                          double* rv, int* ri, double& logabs, int& sgn) {
  double* A = D.a;
  const int ld = D.ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  logabs = 0.0;
  sgn = 1;
  for (int k = 0; k < n; ++k) {
    int p = k;
    if (!triangular) {
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < n; i += kDenseThreads) {
        const double v = fabs(A[i * ld + k]);
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
      if (lane == 0) {
        rv[wave] = best;
        ri[wave] = bi;
      }
      __syncthreads();
      p = ri[0];
      double pb = rv[0];
      for (int w = 1; w < kDenseWaves; ++w)
        if (rv[w] > pb || (rv[w] == pb && ri[w] < p)) {
          pb = rv[w];
          p = ri[w];
        }
      if (p != k) {
        for (int c = tid; c < n; c += kDenseThreads) {
          const double t = A[k * ld + c];
          A[k * ld + c] = A[p * ld + c];
          A[p * ld + c] = t;
        }
        sgn = -sgn;
      }
    }
    if (tid == 0) piv[k] = p;
    __syncthreads();
    const double pv = A[k * ld + k];
    if (pv == 0.0 || pv != pv) {
      sgn = 0;
      return;
    }
    logabs += log(fabs(pv));
    if (pv < 0) sgn = -sgn;
    const double ipv = 1.0 / pv;
    __syncthreads();
    const int c0 = triangular ? k : 0;
    for (int c = c0 + tid; c < n; c += kDenseThreads) A[k * ld + c] = (c == k) ? ipv : A[k * ld + c] * ipv;
    const int rend = triangular ? k : n;
    for (int i = tid; i < rend; i += kDenseThreads) colk[i] = (i == k) ? 0.0 : A[i * ld + k];
    __syncthreads();
    for (int i = wave; i < rend; i += kDenseWaves) {
      if (i == k) continue;
      const double t = colk[i];
      if (t == 0.0) continue;
      for (int c = c0 + lane; c < n; c += 64)
        A[i * ld + c] = (c == k) ? -t * ipv : A[i * ld + c] - t * A[k * ld + c];
    }
    __syncthreads();
  }
  if (!triangular)
    for (int k = n - 1; k >= 0; --k) {
      const int p = piv[k];
      if (p != k)
        for (int r = tid; r < n; r += kDenseThreads) {
          const double t = A[r * ld + k];
          A[r * ld + k] = A[r * ld + p];
          A[r * ld + p] = t;
        }
      __syncthreads();
    }
}

// Cholesky W = R^T R (R upper) of the Gram matrix of the basis, then R^{-1}.
// log|det R| is the checkpoint's log|det T| (R has a positive diagonal).
__global__ __launch_bounds__(kDenseThreads) void k_chol_inv(const ChainDev* __restrict__ chains) {
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const ChainDev& C = chains[lg >> 1];
  const int sp = lg & 1, n = C.n[sp], tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double lds[kLdsDense * (kLdsDense + 1)];
  __shared__ double colk[kMaxSites];
  __shared__ int piv[kMaxSites];
  __shared__ double rv[kDenseWaves];
  __shared__ int ri[kDenseWaves];
  __shared__ int bad;
  if (tid == 0) bad = 0;
  const Dense D = dense_load(lds, C.Wm[sp], n);
  double* A = D.a;
  const int ld = D.ld;
  for (int j = 0; j < n; ++j) {
    const double d2 = A[j * ld + j];
    __syncthreads();
    if (!(d2 > 0.0)) {   // not positive definite (or NaN): flag, keep going finitely
      if (tid == 0) {
        bad = 1;
        A[j * ld + j] = 1.0;
      }
      __syncthreads();
      continue;
    }
    const double d = sqrt(d2);
    for (int c = j + 1 + tid; c < n; c += kDenseThreads) A[j * ld + c] /= d;
    if (tid == 0) A[j * ld + j] = d;
    __syncthreads();
    for (int r = j + 1 + wave; r < n; r += kDenseWaves) {
      const double ajr = A[j * ld + r];
      for (int c = r + lane; c < n; c += 64) A[r * ld + c] -= ajr * A[j * ld + c];
    }
    __syncthreads();
  }
  for (int r = wave; r < n; r += kDenseWaves)   // clear the lower triangle
    for (int c = lane; c < r; c += 64) A[r * ld + c] = 0.0;
  __syncthreads();
  if (tid == 0) {
    double lsum = 0.0;
    for (int j = 0; j < n; ++j) lsum += log(A[j * ld + j]);
    C.st->chk_log[sp] = lsum;
    C.st->chk_sgn[sp] = 1;
    if (bad) atomicOr(&C.st->flags, (int)FLAG_SINGULAR);
  }
  double la;
  int sg;
  gj_invert(D, n, true, colk, piv, rv, ri, la, sg);
  __syncthreads();
  dense_store(D, C.Rinv[sp], n, true);
}

// Inverse of X = L R (n x n) in place; log|det X| and its sign go to the
// chain state.
__global__ __launch_bounds__(kDenseThreads) void k_gj_inv(const ChainDev* __restrict__ chains) {
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const ChainDev& C = chains[lg >> 1];
  const int sp = lg & 1, n = C.n[sp], tid = threadIdx.x;
  __shared__ double lds[kLdsDense * (kLdsDense + 1)];
  __shared__ double colk[kMaxSites];
  __shared__ int piv[kMaxSites];
  __shared__ double rv[kDenseWaves];
  __shared__ int ri[kDenseWaves];
  const Dense D = dense_load(lds, C.Xm[sp], n);
  double logabs;
  int sgn;
  gj_invert(D, n, false, colk, piv, rv, ri, logabs, sgn);
  __syncthreads();
  if (sgn != 0 && D.a != C.Xm[sp]) dense_store(D, C.Xm[sp], n, false);
  if (tid == 0) {
    C.st->x_log[sp] = logabs;
    C.st->x_sgn[sp] = sgn;
    if (sgn == 0) atomicOr(&C.st->flags, (int)FLAG_SINGULAR);
  }
}

// FP32 basis variant: the checkpoint starts from an FP64 copy (in Hw) of the basis.
template <typename Tu>
__global__ __launch_bounds__(kThreads) void k_basis_to_fp64(const ChainDev* __restrict__ chains,
                                                            int parity) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  for (int sp = 0; sp < 2; ++sp) {
    const Tu* u = (const Tu*)C.U[sp][parity];
    for (int idx = threadIdx.x; idx < C.N * C.n[sp]; idx += kThreads) C.Hw[sp][idx] = (double)u[idx];
  }
}

// ---------------------------------------------------------------------------
// checkpoint bookkeeping (one workgroup per chain)
// mode 0: checkpoint of a pass (sign check, drift);  1: final checkpoint of
// the initialisation (sign := recomputed);  2: store-only (initial stack).
// The new orthonormal basis Qc goes to the stack slot and, in the basis
// precision, becomes the active basis U[parity].
// ---------------------------------------------------------------------------
template <typename Tu>
__global__ __launch_bounds__(kThreads) void k_finalize(const ChainDev* __restrict__ chains,
                                                       const Ctl* __restrict__ ctl, int slot,
                                                       int mode, int measure_here, int ck_index,
                                                       int parity) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  ChainState* st = C.st;
  const int N = C.N, tid = threadIdx.x;
  __shared__ double red[4];
  for (int sp = 0; sp < 2; ++sp) {
    const size_t sz = (size_t)N * C.n[sp];
    double* dst = C.stack[sp] + (size_t)slot * sz;
    Tu* u = (Tu*)C.U[sp][parity];
    for (size_t idx = tid; idx < sz; idx += kThreads) {
      const double q = C.Qc[sp][idx];
      dst[idx] = q;
      u[idx] = (Tu)q;
    }
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
      if (k != 0.0)
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
// optionally also start the active basis U[0] from them.
template <typename Tu>
__global__ __launch_bounds__(kThreads) void k_put_trial(const ChainDev* __restrict__ chains, int slot,
                                                        int set_active) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  const int tid = threadIdx.x;
  for (int sp = 0; sp < 2; ++sp) {
    const size_t sz = (size_t)C.N * C.n[sp];
    double* dst = C.stack[sp] + (size_t)slot * sz;
    Tu* u = (Tu*)C.U[sp][0];
    for (size_t idx = tid; idx < sz; idx += kThreads) {
      const double v = C.P[sp][idx];
      dst[idx] = v;
      if (set_active) u[idx] = (Tu)v;
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
template <typename Tu>
__global__ __launch_bounds__(kThreads) void k_dscale_u(const ChainDev* __restrict__ chains, int l,
                                                       int M, int parity) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  const int b = (l == 0 || l == M + 1) ? 0 : 1;
  const int8_t* frow = C.field + (size_t)l * C.N;
  for (int sp = 0; sp < 2; ++sp) {
    const int n = C.n[sp];
    Tu* u = (Tu*)C.U[sp][parity];
    for (int idx = threadIdx.x; idx < C.N * n; idx += kThreads) {
      const int i = idx / n;
      u[idx] *= (Tu)C.dval[b][sp][frow[i] > 0 ? 0 : 1];
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
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_chol_inv(const ChainDev* c, int nc, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(2 * nc), dim3(kDenseThreads), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_gj_inv(const ChainDev* c, int nc, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_inv, dim3(2 * nc), dim3(kDenseThreads), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_basis_to_fp64(int fp32b, const ChainDev* c, int nc, int parity, hipStream_t s) {
  if (fp32b)
    hipLaunchKernelGGL(k_basis_to_fp64<float>, dim3(nc), dim3(kThreads), 0, s, c, parity);
  else
    hipLaunchKernelGGL(k_basis_to_fp64<double>, dim3(nc), dim3(kThreads), 0, s, c, parity);
  return hipGetLastError();
}

hipError_t launch_finalize(int fp32b, const ChainDev* c, int nc, const Ctl* ctl, int slot, int mode,
                           int measure_here, int ck_index, int parity, hipStream_t s) {
  if (fp32b)
    hipLaunchKernelGGL(k_finalize<float>, dim3(nc), dim3(kThreads), 0, s, c, ctl, slot, mode,
                       measure_here, ck_index, parity);
  else
    hipLaunchKernelGGL(k_finalize<double>, dim3(nc), dim3(kThreads), 0, s, c, ctl, slot, mode,
                       measure_here, ck_index, parity);
  return hipGetLastError();
}

hipError_t launch_put_trial(int fp32b, const ChainDev* c, int nc, int slot, int set_active,
                            hipStream_t s) {
  if (fp32b)
    hipLaunchKernelGGL(k_put_trial<float>, dim3(nc), dim3(kThreads), 0, s, c, slot, set_active);
  else
    hipLaunchKernelGGL(k_put_trial<double>, dim3(nc), dim3(kThreads), 0, s, c, slot, set_active);
  return hipGetLastError();
}

hipError_t launch_dscale_u(int fp32b, const ChainDev* c, int nc, int l, int M, int parity,
                           hipStream_t s) {
  if (fp32b)
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
