// Internal data layout shared by the HIP kernels and the host-side library
// code of the Gutzwiller-projection PQMC sweep.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpqmc {

constexpr int kThreads = 256;   // every kernel runs 256-thread workgroups (4 waves)
constexpr int kBlock = 32;      // submatrix block of the flip scan (sites)
constexpr int kMexp = 4;        // largest |site exponent| of D_l (t-V: bonds per site)
constexpr int kSegMax = 64;     // largest delay rank: sites per scan segment
constexpr int kMeasCols = 4;    // measurement record: sign, E/N, D, S_AFM
constexpr int kMaxSites = 1024; // largest lattice
constexpr int kTile = 64;       // GEMM output tile (kTile x kTile per workgroup)
constexpr int kLdsDense = 128;  // small dense factorisations run in LDS up to this order

enum Tag : uint32_t { TAG_INIT = 0, TAG_ACCEPT = 1 };

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// (c0,c1,c2,c3) -> (hi(M1 c2)^c1^k0, lo(M1 c2), hi(M0 c0)^c3^k1, lo(M0 c0)) with a
// Weyl key schedule.  Used on the host for the initial field and on the device
// for the Metropolis draws.
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)m0 * c[0];
    const uint64_t p1 = (uint64_t)m1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// 53-bit uniform in [0, 1) from the first two output words.
__host__ __device__ inline double uniform53(uint32_t w0, uint32_t w1) {
  return ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6)) * (1.0 / 9007199254740992.0);
}

// Mutable per-chain state (device memory).
struct ChainState {
  int sign;             // tracked sign of W_up * W_dn
  int sweep;            // pass counter: word 1 of the Philox counter
  int fcount;           // flips with nonzero Delta accepted in the current scan segment
  int foff;             // such flips accepted in the slice before the current segment
  int ftot;             // such flips accepted in the slice so far (foff + fcount)
  int pad1;
  int flags;            // sticky error bits (FLAG_*)
  int n_meas;           // stored measurement records
  int sign_mismatch;    // checkpoints where tracked and recomputed signs differ
  int run_sgn[2];       // sign of det of the active basis' accumulated triangular factors
  double run_log[2];    // log|det| of the same
  double chk_log[2];    // log|det T| of the current checkpoint's QR
  int chk_sgn[2];
  double x_log[2];      // log|det (L R)| of the current checkpoint
  int x_sgn[2];
  unsigned int drift_bits;  // max |G_wrapped - G_fresh| of the current checkpoint (float bits)
  float max_drift;      // since initialisation
  float last_drift;
  unsigned int gmax_bits;   // max |G_fresh| of the current checkpoint (float bits)
  float max_rel_drift;  // max over checkpoints of drift / max |G_fresh|
  float last_rel_drift;
  long long accepted;   // accepted proposals
  long long proposed;   // proposals
  double w_log[2];      // log|W_sigma| = log|det(L_p R_p)| at the last checkpoint
  int w_sgn[2];         // sign of W_sigma at the last checkpoint
};

enum Flags : int {
  FLAG_DRIFT = 1,       // drift above tolerance at a checkpoint
  FLAG_NAN = 2,         // non-finite Green's function
  FLAG_SINGULAR = 4,    // singular L R, or a basis Gram matrix not positive definite
  FLAG_SIGN = 8,        // tracked and recomputed signs disagree
  FLAG_MEAS_FULL = 16,  // measurement buffer full (records dropped)
};

// Per-chain description (device memory).  Matrices are row-major; N x N
// matrices use leading dimension N, N x n matrices (n = particles of the spin)
// leading dimension n.
struct ChainDev {
  int N;                // sites
  int n[2];             // particles per spin (0 = up, 1 = down)
  int pad0;
  // diagonal of D_l for spin sigma at a site with exponent m (the entry of
  // mexp): d = dval[b][sigma][m + kMexp] = exp(sigma_sign * c_b * m), b = 0
  // boundary (projector coupling lambda), 1 bulk (coupling alpha)
  double dval[2][2][2 * kMexp + 1];
  // flip factor Delta = exp(-2 sigma c_b s) - 1 of a field s (index 0: s = +1,
  // 1: s = -1); for a t-V bond (i, j) the A end i takes sigma = up, the B end j
  // sigma = down
  double delta[2][2][2];
  double U_hub;           // Hubbard U (energy measurement)
  uint32_t key0, key1;    // Philox key (seed low word, seed high word ^ TAG_ACCEPT)
  uint32_t chain_id;
  // 1: half-filling particle-hole shortcut (factored engine).  Only spin 0 is
  // propagated, updated and re-stabilised; spin 1 follows from it per field:
  // G_1 = 1 - E G_0^T E with E = diag(eps), and log|W_1| = log|W_0| -
  // sum_{l,i} c_l s_{l,i}, sgn W_1 = sgn W_0.  Every kernel that works per
  // (chain, spin) skips spin 1 of such a chain.
  int ph;
  int nsp;              // species whose factors are propagated: 2, or 1 (particle-hole, t-V)
  int tv;               // 1: spinless t-V model (bond fields; spin 0 only)
  int n_bonds;          // t-V: bonds (proposals per slice); the Hubbard model: 0
  double V;             // t-V: nearest-neighbour repulsion (energy measurement)
  const int* bonds;     // t-V: n_bonds x 2 sites (A end, B end) in proposal order
  const int* seg_start; // t-V: first bond of every scan segment (n_seg + 1 entries)
  int n_seg;            // t-V: scan segments per slice
  int8_t* mexp;         // n_slices x N site exponents of D_l: the HS field itself for the
                        // Hubbard model; for t-V the sum over a site's bonds of
                        // +s_b (A end) or -s_b (B end)
  double* dflist;       // Delta of every accepted flip of the last segment, [spin][kSegMax]
  // Green's-function precision (float or double)
  void* G[2];           // equal-time Green's function in the current frame
  void* Gtmp[2];        // wrap intermediate
  void* Z[2];           // delayed-update coefficients of a segment (f x f, ld kSegMax)
  // slice-level delayed update G = G0 - Xa Ya over the ftot flips accepted in
  // the slice so far (N x N each, ld N; columns / rows 0 .. ftot used)
  void* Xa[2];
  void* Ya[2];
  void* scan_ws[2];     // scan scratch, 5 * kBlock * kSegMax elements
  int* flist;           // accepted sites F of the last segment (kSegMax)
  const void* Km;       // e^{-dtau K}
  const void* Kp;       // e^{+dtau K}
  // basis precision (float or double)
  void* U[2][2];        // active propagated basis, ping-pong pair
  // FP64
  const double* Khop;   // hopping matrix K
  const double* P[2];   // trial orbitals, N x n
  double* stack[2];     // n_slots x N x n orthonormal bases
  double* slot_log[2];  // per slot: log|det| of the accumulated triangular factors
  int* slot_sgn[2];
  double* Hw[2];        // QR work (N x n)
  double* Qc[2];        // orthonormal basis of the current checkpoint (N x n)
  double* Wm[2];        // Gram matrix (n x n)
  double* Rinv[2];      // inverse Cholesky factor (n x n, upper)
  double* Xm[2];        // L R (n x n), inverted in place
  double* Ym[2];        // (L R)^{-1} L  (n x N)
  double* G64[2];       // last fresh Green's function (unscaled, at its checkpoint)
  int8_t* field;        // n_slices x N HS fields (t-V: n_slices x n_bonds bond fields)
  const int8_t* eps;    // sublattice signs (N)
  ChainState* st;
  double* meas;         // records (sign, E/N, D, S_AFM), kMeasCols each
  int meas_cap;
  int pad2;
  double* trace_ratio;  // optional: (n_slices * N) x 2 ratios of the last pass
  double* trace_green;  // optional: checkpoints_per_pass x 2 x N x N
  double* trace_drift;  // optional: checkpoints_per_pass
  double* trace_logdet; // optional: checkpoints_per_pass x 2 x (log|W_sigma|, sign)
  // factored engine (FP64): G = 1 - A B^T with A, B of size N x n (ld n);
  // F[0] = A (the R side), F[1] = B (the L side), ping-pong pair by parity
  void* F[2][2][2];     // [side][spin][parity]
  double* Mf[2];        // the moving factor's rows at the segment's accepted sites (kSegMax x n)
  double* Wf[2];        // Woodbury core times the dual factor's rows at those sites (kSegMax x n)
  double coupling[2];   // HS coupling c_b: 0 boundary slices (lambda), 1 bulk slices (alpha)
  int n_slices;         // M + 2 (rows of the field)
  int pad3;
};

// Control block (device memory), read by every kernel of a pass.
struct Ctl {
  int measure;          // record measurements at tau = Theta
  int force_reject;     // debug: reject every proposal (fixed-field parity)
  float drift_tol;      // relative drift above this sets FLAG_DRIFT
  int pad;
};

// One operand set of a batched GEMM (one chain and one spin).  Pointer pairs
// are selected by the launch's parity where the mode ping-pongs.
struct GemmEntry {
  const void* A[2];
  const void* B[2];
  void* C[2];
  const double* stack;  // checkpoint stack base (FP64)
  const double* Qc;     // current checkpoint basis (FP64)
  int slot_stride;      // elements per stack slot
  int M, N, K;          // static sizes
  int lda, ldb, ldc, ldc2;
  const int8_t* field;  // base of the chain's site exponents (ChainDev::mexp)
  int n_sites;
  int spin;
  ChainState* st;
  const int* dynK;      // if set, the chain's K is *dynK (the slice's accepted count)
  int sinv;             // the output row scaling uses D^{-1} (xor with GemmArgs::scale_inverse)
  double dval[2][2 * kMexp + 1];   // [b][m + kMexp] diagonal of D for this spin (see ChainDev)
  const int* dynN;      // if set, the output has *dynN columns (the segment's accepted count)
  void* pad2;
};

struct TileRef {
  int entry, tm, tn, pad;
};

// Launch arguments shared by the GEMM kinds.
struct GemmArgs {
  int scale_slice;      // slice whose D scales the output (-1: none)
  int scale_inverse;    // 0: D X D^{-1}, 1: D^{-1} X D  (mode WRAP/FLUSH/GFRESH)
  int bscale_slice;     // slice whose D scales the rows of B (-1: none)
  int parity;           // ping-pong selector
  int slot;             // checkpoint slot
  int dir;              // 0 up pass (R is the new basis), 1 down pass (L is new)
  int n_bulk_last;      // M (bulk slices are 1..M)
  int check_drift;      // compare against the wrapped Green's function
  int rsel, lsel;       // factored checkpoint operands: 0 = Qc, 1 = the stack slot, 2 = the factor
};

enum GemmMode : int {
  GM_STORE = 0,   // C = A B
  GM_WRAP = 1,    // C = D (A B) D^{-1}  (or D^{-1}(A B)D, or unscaled)
  GM_FLUSH = 2,   // C[1] = D (C[0] - A B) D^{-1}  (scaling optional, K = *dynK)
  GM_PROPB = 3,   // C[p^1] = A (D B[p])
  GM_PROPR = 4,   // C[p^1] = D (A B[p])
  GM_GRAM = 6,    // C = A[p]^T A[p]  (FP64)
  GM_APPLY = 7,   // C = A[p] B       (FP64)
  GM_XMAT = 8,    // C = Lt^T R       (FP64)
  GM_YMAT = 9,    // C = Xinv Lt^T    (FP64)
  GM_GFRESH = 10, // C = 1 - R Y (FP64), drift, bulk copy with scaling
  // factored engine (FP64), G = 1 - A B^T
  GM_IMABT = 11,  // C = 1 - A[p] B[p]^T          (the wrapped G of a checkpoint)
  GM_SEGP = 12,   // C = A[p] B^T, *dynN columns   (Q Mf^T of a segment)
  GM_SEGF = 13,   // C[p] = C[p] - A B, K = *dynK  (Q <- Q - (Q Mf^T) Wf)
  GM_BMAT = 14,   // C[p] = Ls Xinv^T              (L-side factor B = L^T (L R)^{-T})
  GM_AMAT = 15,   // C[p] = Rs Xinv                (R-side factor A = R (L R)^{-1})
  GM_GFRESH2 = 16,// C = 1 - Rs Ls^T, drift against C[1]
};

}  // namespace gpqmc
