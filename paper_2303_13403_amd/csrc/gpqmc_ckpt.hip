// Checkpoint (re-stabilisation) and bookkeeping kernels of the PQMC sweep
// (gfx950).  At a checkpoint the propagated N x n basis U is re-orthonormalised
// in FP64 by Cholesky QR: U = Q T with T the Cholesky factor of U^T U and
// Q = U T^{-1} (the Gram matrix and Q are batched MFMA GEMMs; the n x n
// Cholesky factorisation and T^{-1} run here, in registers for n <= 128, else
// in LDS or global memory).  Only span(Q) and the exact factorisation U = Q T
// matter (the Green's function is invariant under R -> R T), so one pass
// suffices: Q is orthonormal to O(eps cond(U)^2).  The fresh Green's function
// G = 1 - R (L R)^{-1} L follows from the inverse of the n x n overlap L R
// (Gauss-Jordan with partial pivoting, placed like the Cholesky factor) and
// two more GEMMs; log|det| and the sign of each factor are accumulated for the
// sign check.
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
  if (sp >= C.nsp) return;
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
  if (sp >= C.nsp) return;
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

// ---------------------------------------------------------------------------
// Register-tiled variants for n <= TG NB (the usual case).  One workgroup of
// TG x TG threads per matrix; thread t owns the elements (ti + TG a, tj + TG b),
// ti = t / TG, tj = t % TG, in m[a][b], so a row segment is TG consecutive
// lanes (coalesced loads).  Every elimination step publishes the rows and the
// column it needs in double-buffered LDS vectors and updates the registers.
// The step index is uniform across the workgroup, so the register row and
// column that hold a given matrix row or column are chosen by uniform
// branches: an elimination step is one FMA per element plus O(NB) fixes for
// the pivot row, row k and column k, with no per-element selects.
// ---------------------------------------------------------------------------
constexpr int kRtMax = 128;

template <int NB, int TG>
struct RegTile {
  double m[NB][NB];
  int ti, tj, n;
  __device__ void load(const GLOBAL double* __restrict__ g, int n_) {
    n = n_;
    ti = threadIdx.x / TG;
    tj = threadIdx.x % TG;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int r = ti + TG * a, c = tj + TG * b;
        m[a][b] = (r < n && c < n) ? g[(size_t)r * n + c] : 0.0;
      }
  }
  // row r (owned by ti == r % TG) into v[c]; column c (tj == c % TG) into
  // v[r].  r and c are uniform, so is the register row / column.
  __device__ void put_row(int r, double* v) const {
    const int ar = r / TG;
    if (ti != r % TG) return;
#pragma unroll
    for (int a = 0; a < NB; ++a)
      if (a == ar) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int c = tj + TG * b;
          if (c < n) v[c] = m[a][b];
        }
      }
  }
  __device__ void put_col(int c, double* v) const {
    const int bc = c / TG;
    if (tj != c % TG) return;
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b == bc) {
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          const int r = ti + TG * a;
          if (r < n) v[r] = m[a][b];
        }
      }
  }
  // one Gauss-Jordan step at pivot k (uniform) with the pivot row taken from
  // row p (uniform): rk = old row k, rp = old row p, ck = old column k (all in
  // LDS).  Every element is first updated as an ordinary row,
  // m -= ck[r] rp[c] / pivot; then the row that receives the old row k, column
  // k (-f_r / pivot) and row k (the normalised pivot row) are rewritten.
  __device__ void gj_step(int k, int p, double inv, const double* rk, const double* rp,
                          const double* ck) {
    double prc[NB], ckr[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) prc[b] = rp[tj + TG * b] * inv;
#pragma unroll
    for (int a = 0; a < NB; ++a) ckr[a] = ck[ti + TG * a];
    const double fpk = rk[k];   // column-k entry of the row that moves to p
    const int ak = k / TG, bk = k / TG, ap = p / TG;
    const bool lk_r = ti == k % TG, lk_c = tj == k % TG, lp_r = (ti == p % TG) & (p != k);
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) m[a][b] = fma(-ckr[a], prc[b], m[a][b]);
    if (p != k) {
#pragma unroll
      for (int a = 0; a < NB; ++a)
        if (a == ap) {
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const double v = fma(-fpk, prc[b], rk[tj + TG * b]);
            m[a][b] = lp_r ? v : m[a][b];
          }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b == bk) {
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          const double fr = (lp_r & (a == ap)) ? fpk : ckr[a];
          m[a][b] = lk_c ? -fr * inv : m[a][b];
        }
      }
#pragma unroll
    for (int a = 0; a < NB; ++a)
      if (a == ak) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double v = (lk_c & (b == bk)) ? inv : prc[b];
          m[a][b] = lk_r ? v : m[a][b];
        }
      }
  }
};

// In-place inverse with partial pivoting.  Returns log|det| (to thread 0, over
// the nonzero pivots) and the sign (0: singular, the tile is then unusable; to
// every thread); colmap receives, for every column of the eliminated matrix,
// its column in the inverse.
template <int NB, int TG>
__device__ void rt_invert(RegTile<NB, TG>& T, double (*rk)[kRtMax], double (*rp)[kRtMax],
                          double (*ck)[kRtMax], double (*cv)[32], int (*ci)[32], int* piv,
                          int* colmap, double* pabs, double& logabs, int& sgn) {
  const int n = T.n, tid = threadIdx.x;
  logabs = 0.0;
  sgn = 1;
  if (tid == 0)
    for (int c = 0; c < n; ++c) colmap[c] = c;   // ordered by the first step's barrier
  for (int k = 0; k < n; ++k) {
    const int kb = k & 1;
    T.put_row(k, rk[kb]);
    T.put_col(k, ck[kb]);
    // candidates of the owners of column k, one per row residue
    const int bc = k / TG;
    if (T.tj == k % TG) {
      double best = -1.0;
      int bi = k;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b == bc) {
#pragma unroll
          for (int a = 0; a < NB; ++a) {
            const double x = T.m[a][b];
            const int r = T.ti + TG * a;
            const bool take = (r >= k) & (r < n) & (fabs(x) > best);
            best = take ? fabs(x) : best;
            bi = take ? r : bi;
          }
        }
      cv[kb][T.ti] = best;
      ci[kb][T.ti] = bi;
    }
    __syncthreads();
    // largest candidate, ties to the smallest row: a shuffle reduction over
    // each group of TG lanes, which holds all TG candidates
    double best = cv[kb][tid % TG];
    int bi = ci[kb][tid % TG];
#pragma unroll
    for (int off = TG / 2; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, TG);
      const int oi = __shfl_xor(bi, off, TG);
      const bool take = (ob > best) | ((ob == best) & (oi < bi));
      best = take ? ob : best;
      bi = take ? oi : bi;
    }
    const int p = __builtin_amdgcn_readfirstlane(bi);   // the same on every lane
    if (p != k) T.put_row(p, rp[kb]);
    __syncthreads();
    const double* prow = (p == k) ? rk[kb] : rp[kb];
    const double pv = prow[k];
    // a zero or NaN pivot makes the matrix singular: the remaining steps run
    // with a zero inverse pivot (finite, discarded) rather than leaving the
    // loop, which kept a second copy of the tile live in registers
    const bool bad = (pv == 0.0) | (pv != pv);
    if (bad) sgn = 0;
    if (tid == 0) {
      // |pivot| (1 for a bad one); the logs are taken after the loop, off
      // the critical path of the elimination steps
      pabs[k] = bad ? 1.0 : fabs(pv);
      piv[k] = p;
    }
    if (pv < 0) sgn = -sgn;
    if (p != k) sgn = -sgn;
    T.gj_step(k, p, bad ? 0.0 : 1.0 / pv, rk[kb], prow, ck[kb]);
  }
  __syncthreads();
  if (tid == 0) {
    // columns of the result: undo the row interchanges as column
    // interchanges in reverse order; colmap[c] = destination of column c
    for (int k = n - 1; k >= 0; --k) {
      const int q = piv[k];
      const int t = colmap[k];
      colmap[k] = colmap[q];
      colmap[q] = t;
    }
    // colmap now holds the source column of each destination; invert it
    for (int c = 0; c < n; ++c) piv[colmap[c]] = c;
    for (int c = 0; c < n; ++c) colmap[c] = piv[c];
  }
  // log|pivot| on n threads at once, summed in pivot order by thread 0
  for (int c = tid; c < n; c += blockDim.x) pabs[c] = log(pabs[c]);
  __syncthreads();
  if (tid == 0)
    for (int c = 0; c < n; ++c) logabs += pabs[c];
  __syncthreads();
}

template <int NB, int TG>
__device__ void rt_store(const RegTile<NB, TG>& T, GLOBAL double* __restrict__ g, const int* colmap,
                         bool upper_only) {
  // destination columns, read once per register column
  int cd[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int c = T.tj + TG * b;
    cd[b] = c < T.n ? colmap[c] : 0;
  }
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int r = T.ti + TG * a, c = T.tj + TG * b;
      if (r < T.n && c < T.n) g[(size_t)r * T.n + cd[b]] = (upper_only && cd[b] < r) ? 0.0 : T.m[a][b];
    }
}

// the step vectors are read at every residue, including entries beyond n
__device__ inline void rt_clear(double (*rk)[kRtMax], double (*rp)[kRtMax], double (*ck)[kRtMax]) {
  for (int i = threadIdx.x; i < 2 * kRtMax; i += blockDim.x) {
    rk[i / kRtMax][i % kRtMax] = 0.0;
    rp[i / kRtMax][i % kRtMax] = 0.0;
    ck[i / kRtMax][i % kRtMax] = 0.0;
  }
}

#define GPQMC_RT_SHARED                                 \
  __shared__ double rk[2][kRtMax], rp[2][kRtMax], ck[2][kRtMax]; \
  __shared__ double cv[2][32];                          \
  __shared__ int ci[2][32];                             \
  __shared__ int piv[kRtMax], colmap[kRtMax];           \
  __shared__ double pabs[kRtMax];

// Cholesky factor of the Gram matrix W = R^T R (R upper) and its inverse in
// one pass of n elimination steps, in registers.  Eliminating below each
// pivot of W without pivoting gives W = L U with L unit lower; applying the
// same row operations to the identity gives L^{-1}, which is kept in place in
// the eliminated slots (as in an in-place Gauss-Jordan inverse).  Since
// L = R^T diag(R)^{-1}, U = diag(R) R and R_jj = sqrt(U_jj), the inverse is
// R^{-1} = (L^{-1})^T diag(R)^{-1}.  The trailing block stays symmetric, so
// the multipliers of step j are read from row j.
// (At most 168 registers for the 7 x 7 tiles: three workgroups per CU.)
template <int NB, int TG>
__global__ __launch_bounds__(TG * TG) __attribute__((amdgpu_waves_per_eu(NB == 7 ? 3 : 1)))
void k_chol_inv_rt(const ChainDev* __restrict__ chains) {
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const ChainDev& C = chains[lg >> 1];
  const int sp = lg & 1, n = C.n[sp], tid = threadIdx.x;
  if (sp >= C.nsp) return;
  // row j of step j (double-buffered; entries beyond n stay zero) and the
  // pivots U_jj
  __shared__ double rk[2][kRtMax], pabs[kRtMax];
  for (int i = tid; i < 2 * kRtMax; i += blockDim.x) rk[i / kRtMax][i % kRtMax] = 0.0;
  RegTile<NB, TG> T;
  T.load(gp(C.Wm[sp]), n);
  bool bad = false;
  for (int j = 0; j < n; ++j) {
    const int jb = j & 1;
    T.put_row(j, rk[jb]);
    __syncthreads();
    const double u = rk[jb][j];
    // not positive definite (or NaN): flag, take no multipliers at this
    // step and R_jj = 1, so that a finite matrix keeps every value finite
    const bool ok = u > 0.0;
    if (!ok) bad = true;
    if (tid == 0) pabs[j] = ok ? u : 1.0;
    const double iu = ok ? 1.0 / u : 0.0;
    // rows below j: row -= l_rj (row j), every column; the slot of column j
    // then receives L^{-1}_rj = -l_rj
    double rc[NB], rl[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) rc[b] = rk[jb][T.tj + TG * b];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int r = T.ti + TG * a;
      rl[a] = r > j ? rk[jb][r] * iu : 0.0;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) T.m[a][b] = fma(-rl[a], rc[b], T.m[a][b]);
    const int bj = j / TG;
    const bool lj = T.tj == j % TG;
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (b == bj) {
#pragma unroll
        for (int a = 0; a < NB; ++a) T.m[a][b] = lj ? -rl[a] : T.m[a][b];
      }
  }
  // 1 / R_rr of the thread's rows, then log|det R| = (1/2) sum of log U_jj:
  // the logs on n threads at once, summed in order by thread 0
  __syncthreads();
  double rs[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    const int r = T.ti + TG * a;
    rs[a] = r < n ? 1.0 / sqrt(pabs[r]) : 0.0;
  }
  __syncthreads();
  for (int c = tid; c < n; c += blockDim.x) pabs[c] = log(pabs[c]);
  __syncthreads();
  if (tid == 0) {
    double lsum = 0.0;
    for (int c = 0; c < n; ++c) lsum += pabs[c];
    C.st->chk_log[sp] = 0.5 * lsum;
    C.st->chk_sgn[sp] = 1;
    if (bad) atomicOr(&C.st->flags, (int)FLAG_SINGULAR);
  }
  // R^{-1}[c][r] = L^{-1}[r][c] / R_rr (r > c), 1 / R_rr on the diagonal, zero
  // below it: each element goes to its transposed place
  GLOBAL double* __restrict__ g = gp(C.Rinv[sp]);
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int r = T.ti + TG * a, c = T.tj + TG * b;
      if (r < n && c < n)
        g[(size_t)c * n + r] = r > c ? T.m[a][b] * rs[a] : (r == c ? rs[a] : 0.0);
    }
}

// Inverse of X = L R (n x n) in place, partial pivoting; log|det X| and its
// sign go to the chain state.
template <int NB, int TG>
__global__ __launch_bounds__(TG * TG) __attribute__((amdgpu_waves_per_eu(NB == 7 ? 3 : 1)))
void k_gj_inv_rt(const ChainDev* __restrict__ chains) {
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const ChainDev& C = chains[lg >> 1];
  const int sp = lg & 1, n = C.n[sp], tid = threadIdx.x;
  if (sp >= C.nsp) return;
  GPQMC_RT_SHARED
  rt_clear(rk, rp, ck);
  RegTile<NB, TG> T;
  T.load(gp(C.Xm[sp]), n);
  double logabs;
  int sgn;
  rt_invert<NB, TG>(T, rk, rp, ck, cv, ci, piv, colmap, pabs, logabs, sgn);
  if (sgn != 0) rt_store<NB, TG>(T, gp(C.Xm[sp]), colmap, false);
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

// Visits every (i, j) of the N x N matrices G0 (and G1, NM = 2) with G_ij read
// by the caller and G_ji handed in: the matrices are walked in 32 x 32 tiles
// whose transposes are staged in LDS, so that every global read is coalesced
// (a plain loop over (i, j) reads G_ji with a stride of N).
constexpr int kPairTile = 32;
template <int NM, class F>
__device__ void visit_pairs(int N, const GLOBAL double* __restrict__ G0,
                            const GLOBAL double* __restrict__ G1,
                            double (*tt)[kPairTile][kPairTile + 1], F f) {
  const int tid = threadIdx.x;
  for (int i0 = 0; i0 < N; i0 += kPairTile)
    for (int j0 = 0; j0 < N; j0 += kPairTile) {
      __syncthreads();   // the previous tile is read
      for (int t = tid; t < kPairTile * kPairTile; t += kThreads) {
        const int a = t / kPairTile, b = t % kPairTile;
        const int j = j0 + a, i = i0 + b;   // row j of G, along i
        const bool ok = i < N && j < N;
        tt[0][a][b] = ok ? G0[(size_t)j * N + i] : 0.0;
        if (NM == 2) tt[1][a][b] = ok ? G1[(size_t)j * N + i] : 0.0;
      }
      __syncthreads();
      for (int t = tid; t < kPairTile * kPairTile; t += kThreads) {
        const int a = t / kPairTile, b = t % kPairTile;
        const int i = i0 + a, j = j0 + b;
        if (i < N && j < N) f(i, j, tt[0][b][a], NM == 2 ? tt[1][b][a] : 0.0);
      }
    }
}

// ---------------------------------------------------------------------------
// checkpoint bookkeeping (one workgroup per chain)
// mode 0: checkpoint of a pass (sign check, drift);  1: final checkpoint of
// the initialisation (sign := recomputed);  2: store-only (initial stack).
// The new orthonormal basis Qc goes to the stack slot and, in the basis
// precision, becomes the active basis: U[parity] (side -1), the factored
// engine's factor F[side][parity] (side 0 = A, 1 = B), or nothing (side 2:
// the checkpoint produced the active factors itself).
// ---------------------------------------------------------------------------
template <typename Tu>
__global__ __launch_bounds__(kThreads) void k_finalize(const ChainDev* __restrict__ chains,
                                                       const Ctl* __restrict__ ctl, int slot,
                                                       int mode, int measure_here, int ck_index,
                                                       int parity, int side) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  ChainState* st = C.st;
  const int N = C.N, tid = threadIdx.x, nsp = C.nsp;
  __shared__ double red[4];
  __shared__ double tt[2][kPairTile][kPairTile + 1];   // transposed tiles of the measurement
  for (int sp = 0; sp < nsp; ++sp) {
    const size_t sz = (size_t)N * C.n[sp];
    GLOBAL double* dst = gp(C.stack[sp] + (size_t)slot * sz);
    GLOBAL Tu* u = side < 0 ? gp((Tu*)C.U[sp][parity])
                 : side < 2 ? gp((Tu*)C.F[side][sp][parity]) : nullptr;
    const GLOBAL double* __restrict__ qc = gp((const double*)C.Qc[sp]);
    // eight coalesced loads in flight per thread, then their stores
    constexpr int D = 8;
    for (size_t b0 = 0; b0 < sz; b0 += (size_t)D * kThreads) {
      double v[D];
#pragma unroll
      for (int e = 0; e < D; ++e) {
        const size_t idx = b0 + (size_t)e * kThreads + tid;
        v[e] = idx < sz ? qc[idx] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < D; ++e) {
        const size_t idx = b0 + (size_t)e * kThreads + tid;
        if (idx < sz) {
          dst[idx] = v[e];
          if (u) u[idx] = (Tu)v[e];
        }
      }
    }
  }
  // particle-hole shortcut: log|W_1| - log|W_0| = -sum_{l,i} c_l s_{l,i}
  // (det of the spin-1 slice product; the trial projections agree), from
  // exact integer field sums of the boundary and the bulk slices
  double ph_shift = 0.0;
  if (C.ph && mode != 2) {
    const int ns = C.n_slices;
    const GLOBAL int8_t* __restrict__ fld = gp(C.field);
    double sb = 0.0, sk = 0.0;
    for (int idx = tid; idx < ns * N; idx += kThreads) {
      const int l = idx / N;
      const double v = (double)fld[idx];
      if (l == 0 || l == ns - 1) sb += v; else sk += v;
    }
    sb = block_sum(sb, red);
    sk = block_sum(sk, red);
    ph_shift = -(C.coupling[0] * sb + C.coupling[1] * sk);
  }
  if (tid == 0) {
    int wsign = 1;
    for (int sp = 0; sp < 2; ++sp) {
      if (sp == 1 && C.tv) break;   // one species: W = W_0
      if (sp == 1 && C.ph) {
        if (mode != 2) {
          st->w_log[1] = st->w_log[0] + ph_shift;
          st->w_sgn[1] = st->w_sgn[0];
          wsign *= st->w_sgn[1];
          if (C.trace_logdet && ck_index >= 0) {
            C.trace_logdet[((size_t)ck_index * 2 + 1) * 2 + 0] = st->w_log[1];
            C.trace_logdet[((size_t)ck_index * 2 + 1) * 2 + 1] = (double)st->w_sgn[1];
          }
        }
        continue;
      }
      const double nl = st->run_log[sp] + st->chk_log[sp];
      const int ns = st->run_sgn[sp] * st->chk_sgn[sp];
      if (mode != 2) {
        // W_sigma = det(L_p R_p): the accumulated triangular factors of both
        // sides (the slot still holds the opposite side's) and det(L R) of the
        // orthonormal bases
        wsign *= ns * C.slot_sgn[sp][slot] * st->x_sgn[sp];
        st->w_log[sp] = nl + C.slot_log[sp][slot] + st->x_log[sp];
        st->w_sgn[sp] = ns * C.slot_sgn[sp][slot] * st->x_sgn[sp];
        if (C.trace_logdet && ck_index >= 0) {
          C.trace_logdet[((size_t)ck_index * 2 + sp) * 2 + 0] = st->w_log[sp];
          C.trace_logdet[((size_t)ck_index * 2 + sp) * 2 + 1] = (double)st->w_sgn[sp];
        }
      }
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
      // drift relative to the largest element of the fresh G (both spins)
      const float d = __uint_as_float(st->drift_bits);
      const float gm = __uint_as_float(st->gmax_bits);
      const float rd = d / fmaxf(gm, 1e-30f);
      st->last_drift = d;
      st->last_rel_drift = rd;
      if (!(d <= st->max_drift)) st->max_drift = d;
      if (!(rd <= st->max_rel_drift)) st->max_rel_drift = rd;
      if (!(rd <= ctl->drift_tol)) st->flags |= (d != d || isinf(d)) ? FLAG_NAN : FLAG_DRIFT;
    }
    st->drift_bits = 0u;
    st->gmax_bits = 0u;
  }
  if (mode != 2 && measure_here && ctl->measure && C.tv) {
    // spinless t-V, Wick with Gb_ij = <c_i^dag c_j> = delta_ij - G_ji:
    //   <n_i n_j> = Gb_ii Gb_jj + Gb_ij G_ij (the diagonal included),
    //   E = sum_ij K_ij Gb_ij + V sum_b <(n_i - 1/2)(n_j - 1/2)>,
    //   N^2 S_CDW = (sum_i eps_i (n_i - 1/2))^2 + sum_ij eps_i eps_j Gb_ij G_ij
    const GLOBAL double* __restrict__ G = gp((const double*)C.G64[0]);
    const GLOBAL int8_t* __restrict__ eps = gp(C.eps);
    double ek = 0.0, cross = 0.0, mc = 0.0, ev = 0.0, nnb = 0.0;
    visit_pairs<1>(N, G, nullptr, tt, [&](int i, int j, double gt, double) {
      const size_t idx = (size_t)i * N + j;
      const double gb = (i == j ? 1.0 : 0.0) - gt;
      const double k = C.Khop[idx];
      if (k != 0.0) ek += k * gb;
      cross += (double)eps[i] * (double)eps[j] * gb * G[idx];
    });
    for (int i = tid; i < N; i += kThreads) mc += (double)eps[i] * (0.5 - G[(size_t)i * N + i]);
    for (int b = tid; b < C.n_bonds; b += kThreads) {
      const int i = C.bonds[2 * b], j = C.bonds[2 * b + 1];
      const double ni = 1.0 - G[(size_t)i * N + i], nj = 1.0 - G[(size_t)j * N + j];
      const double nn = ni * nj + (-G[(size_t)j * N + i]) * G[(size_t)i * N + j];
      nnb += nn;
      ev += nn - 0.5 * (ni + nj) + 0.25;
    }
    ek = block_sum(ek, red);
    cross = block_sum(cross, red);
    mc = block_sum(mc, red);
    ev = block_sum(ev, red);
    nnb = block_sum(nnb, red);
    if (tid == 0) {
      const int k = st->n_meas;
      if (k < C.meas_cap) {
        double* r = C.meas + (size_t)kMeasCols * k;
        r[0] = (double)st->sign;
        r[1] = (ek + C.V * ev) / N;
        r[2] = nnb / C.n_bonds;
        r[3] = (mc * mc + cross) / ((double)N * N);
        st->n_meas = k + 1;
      } else {
        st->flags |= FLAG_MEAS_FULL;
      }
    }
  } else if (mode != 2 && measure_here && ctl->measure) {
    // Wick estimates from the fresh FP64 G of both spins, G_ij = <c_i c_j^dag>
    // and Gb_ij = <c_i^dag c_j> = delta_ij - G_ji: the energy, the double
    // occupancy, and the staggered structure factor
    //   N^2 S_AFM = sum_ij eps_i eps_j <S_i . S_j>
    //             = mz^2 / 4 + sum_ij eps_i eps_j [(Gb^up_ij G^up_ij + Gb^dn_ij G^dn_ij) / 4
    //                                            + (Gb^up_ij G^dn_ij + Gb^dn_ij G^up_ij) / 2],
    //   mz = sum_i eps_i (Gb^up_ii - Gb^dn_ii)
    // (particle-hole shortcut: G^dn_ij = delta_ij - eps_i eps_j G^up_ji and
    // Gb^dn_ij = eps_i eps_j G^up_ij)
    const bool ph = C.ph != 0;
    const GLOBAL double* __restrict__ Gu = gp((const double*)C.G64[0]);
    const GLOBAL double* __restrict__ Gd = gp((const double*)C.G64[ph ? 0 : 1]);
    const GLOBAL int8_t* __restrict__ eps = gp(C.eps);
    double ek = 0.0, dsum = 0.0, spair = 0.0, mz = 0.0;
    auto wick = [&](int i, int j, double gut, double gdt) {
      const size_t idx = (size_t)i * N + j;
      const double dij = i == j ? 1.0 : 0.0;
      const double ee = (double)eps[i] * (double)eps[j];
      const double gu = Gu[idx];
      const double gd = ph ? dij - ee * gut : Gd[idx];
      const double gbu = dij - gut, gbd = ph ? ee * gu : dij - gdt;
      const double k = C.Khop[idx];
      if (k != 0.0) ek += k * (gbu + gbd);
      spair += ee * (0.25 * (gbu * gu + gbd * gd) + 0.5 * (gbu * gd + gbd * gu));
    };
    if (ph)
      visit_pairs<1>(N, Gu, nullptr, tt, wick);
    else
      visit_pairs<2>(N, Gu, Gd, tt, wick);
    for (int i = tid; i < N; i += kThreads) {
      const double nu = 1.0 - Gu[(size_t)i * N + i];
      const double nd = ph ? Gu[(size_t)i * N + i] : 1.0 - Gd[(size_t)i * N + i];
      dsum += nu * nd;
      mz += (double)eps[i] * (nu - nd);
    }
    ek = block_sum(ek, red);
    dsum = block_sum(dsum, red);
    spair = block_sum(spair, red);
    mz = block_sum(mz, red);
    if (tid == 0) {
      const int k = st->n_meas;
      if (k < C.meas_cap) {
        double* r = C.meas + (size_t)kMeasCols * k;
        r[0] = (double)st->sign;
        r[1] = (ek + C.U_hub * dsum) / N;
        r[2] = dsum / N;
        r[3] = (0.25 * mz * mz + spair) / ((double)N * N);
        st->n_meas = k + 1;
      } else {
        st->flags |= FLAG_MEAS_FULL;
      }
    }
  }
  if (mode != 2 && C.trace_green && ck_index >= 0) {
    for (int sp = 0; sp < (C.tv ? 1 : 2); ++sp) {
      double* dst = C.trace_green + ((size_t)ck_index * 2 + sp) * N * N;
      if (sp == 1 && C.ph) {
        for (int idx = tid; idx < N * N; idx += kThreads) {
          const int i = idx / N, j = idx - i * N;
          dst[idx] = (i == j ? 1.0 : 0.0) -
                     (double)C.eps[i] * (double)C.eps[j] * C.G64[0][(size_t)j * N + i];
        }
      } else {
        for (int idx = tid; idx < N * N; idx += kThreads) dst[idx] = C.G64[sp][idx];
      }
    }
    if (tid == 0) C.trace_drift[ck_index] = st->last_drift;
  }
}

// Store the trial orbitals as the basis of a stack slot (log|det| 0, sign +1);
// optionally also start the active basis from them: U[0] (side -1) or the
// factored engine's factor F[side][0].
template <typename Tu>
__global__ __launch_bounds__(kThreads) void k_put_trial(const ChainDev* __restrict__ chains, int slot,
                                                        int set_active, int side) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  const int tid = threadIdx.x, nsp = C.nsp;
  for (int sp = 0; sp < nsp; ++sp) {
    const size_t sz = (size_t)C.N * C.n[sp];
    double* dst = C.stack[sp] + (size_t)slot * sz;
    Tu* u = side < 0 ? (Tu*)C.U[sp][0] : (Tu*)C.F[side][sp][0];
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
      u[idx] *= (Tu)C.dval[b][sp][kMexp + frow[i]];
    }
  }
}

// Factored engine, frame change of a slice without kinetic factor (or
// outside a propagation GEMM): rows of A <- D_l^{+-1} A, B <- D_l^{-+1} B
// (ainv: A takes D^{-1}); which: bit 0 = A, bit 1 = B.
__global__ __launch_bounds__(kThreads) void k_dscale_f(const ChainDev* __restrict__ chains, int l,
                                                       int M, int parity, int ainv, int which) {
  const ChainDev& C = chains[xcd_remap(blockIdx.x, gridDim.x)];
  const int b = (l == 0 || l == M + 1) ? 0 : 1;
  const GLOBAL int8_t* frow = gp(C.mexp + (size_t)l * C.N);
  for (int sp = 0; sp < C.nsp; ++sp) {
    const int n = C.n[sp];
    for (int side = 0; side < 2; ++side) {
      if (!(which & (1 << side))) continue;
      const bool inv = (side == 0) == (ainv != 0);
      GLOBAL double* f = gp((double*)C.F[side][sp][parity]);
      for (int idx = threadIdx.x; idx < C.N * n; idx += kThreads) {
        const int i = idx / n;
        f[idx] *= C.dval[b][sp][kMexp + (inv ? -(int)frow[i] : (int)frow[i])];
      }
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
// n_part: the largest particle number of the batch; register tiles up to
// kRtMax, the LDS / global kernels beyond
template <int NB, int TG>
static hipError_t launch_rt(bool chol, const ChainDev* c, int nc, hipStream_t s) {
  if (chol)
    hipLaunchKernelGGL((k_chol_inv_rt<NB, TG>), dim3(2 * nc), dim3(TG * TG), 0, s, c);
  else
    hipLaunchKernelGGL((k_gj_inv_rt<NB, TG>), dim3(2 * nc), dim3(TG * TG), 0, s, c);
  return hipGetLastError();
}

// n_part <= 128: 16 x 16 threads with NB = ceil(n_part / 16) (measured faster
// than 32 x 32 threads); beyond: the LDS / global kernels
static hipError_t launch_dense(bool chol, const ChainDev* c, int nc, int n_part, hipStream_t s) {
  switch ((n_part + 15) / 16) {
    case 0:
    case 1: return launch_rt<1, 16>(chol, c, nc, s);
    case 2: return launch_rt<2, 16>(chol, c, nc, s);
    case 3: return launch_rt<3, 16>(chol, c, nc, s);
    case 4: return launch_rt<4, 16>(chol, c, nc, s);
    case 5: return launch_rt<5, 16>(chol, c, nc, s);
    case 6: return launch_rt<6, 16>(chol, c, nc, s);
    case 7: return launch_rt<7, 16>(chol, c, nc, s);
    case 8: return launch_rt<8, 16>(chol, c, nc, s);
    default: break;
  }
  if (chol)
    hipLaunchKernelGGL(k_chol_inv, dim3(2 * nc), dim3(kDenseThreads), 0, s, c);
  else
    hipLaunchKernelGGL(k_gj_inv, dim3(2 * nc), dim3(kDenseThreads), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_chol_inv(const ChainDev* c, int nc, int n_part, hipStream_t s) {
  return launch_dense(true, c, nc, n_part, s);
}

hipError_t launch_gj_inv(const ChainDev* c, int nc, int n_part, hipStream_t s) {
  return launch_dense(false, c, nc, n_part, s);
}

hipError_t launch_basis_to_fp64(int fp32b, const ChainDev* c, int nc, int parity, hipStream_t s) {
  if (fp32b)
    hipLaunchKernelGGL(k_basis_to_fp64<float>, dim3(nc), dim3(kThreads), 0, s, c, parity);
  else
    hipLaunchKernelGGL(k_basis_to_fp64<double>, dim3(nc), dim3(kThreads), 0, s, c, parity);
  return hipGetLastError();
}

hipError_t launch_finalize(int fp32b, const ChainDev* c, int nc, const Ctl* ctl, int slot, int mode,
                           int measure_here, int ck_index, int parity, int side, hipStream_t s) {
  if (fp32b)
    hipLaunchKernelGGL(k_finalize<float>, dim3(nc), dim3(kThreads), 0, s, c, ctl, slot, mode,
                       measure_here, ck_index, parity, side);
  else
    hipLaunchKernelGGL(k_finalize<double>, dim3(nc), dim3(kThreads), 0, s, c, ctl, slot, mode,
                       measure_here, ck_index, parity, side);
  return hipGetLastError();
}

hipError_t launch_put_trial(int fp32b, const ChainDev* c, int nc, int slot, int set_active,
                            int side, hipStream_t s) {
  if (fp32b)
    hipLaunchKernelGGL(k_put_trial<float>, dim3(nc), dim3(kThreads), 0, s, c, slot, set_active, side);
  else
    hipLaunchKernelGGL(k_put_trial<double>, dim3(nc), dim3(kThreads), 0, s, c, slot, set_active, side);
  return hipGetLastError();
}

hipError_t launch_dscale_f(const ChainDev* c, int nc, int l, int M, int parity, int ainv, int which,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_dscale_f, dim3(nc), dim3(kThreads), 0, s, c, l, M, parity, ainv, which);
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
