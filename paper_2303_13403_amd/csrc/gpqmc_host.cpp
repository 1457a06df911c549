// Host side of the Gutzwiller-projection PQMC library: validation, the
// symmetric eigensolver for e^{-+dtau K} and the Neel trial, the workspace
// layout, the slice schedule of a pass (captured as a HIP graph) and the
// C ABI declared in include/gpqmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/gpqmc.h"
#include "gpqmc_internal.h"

namespace gpqmc {
hipError_t launch_gemm(int fp32, int g_fp32, int mode, const GemmEntry* e, const TileRef* t, int n,
                       GemmArgs a, hipStream_t s);
hipError_t launch_gemm_l(int mode, const GemmEntry* e, const TileRef* t, int n, GemmArgs a,
                         hipStream_t s);
hipError_t launch_prop(int nmin, int nmax, int rows, const GemmEntry* e, const TileRef* t, int n,
                       GemmArgs a, hipStream_t s);
hipError_t launch_gemm_l64(int mode, const GemmEntry* e, const TileRef* t, int n, GemmArgs a,
                           hipStream_t s);
hipError_t launch_gemm_plain(int fp32, int transA, const GemmEntry* e, const TileRef* t, int n,
                             GemmArgs a, hipStream_t s);
hipError_t launch_scan(int fp32, int fact, const ChainDev* c, int nc, const Ctl* ctl, int l, int M,
                       int s0, int s1, int dir, int parity, hipStream_t s);
hipError_t launch_xy(int fp32, const ChainDev* c, int nc, int n_max, int s0, int kseg,
                     hipStream_t s);
hipError_t launch_chol_inv(const ChainDev* c, int nc, int n_part, hipStream_t s);
hipError_t launch_gj_inv(const ChainDev* c, int nc, int n_part, hipStream_t s);
hipError_t launch_basis_to_fp64(int fp32b, const ChainDev* c, int nc, int parity, hipStream_t s);
hipError_t launch_finalize(int fp32b, const ChainDev* c, int nc, const Ctl* ctl, int slot, int mode,
                           int measure_here, int ck_index, int parity, int side, hipStream_t s);
hipError_t launch_put_trial(int fp32b, const ChainDev* c, int nc, int slot, int set_active,
                            int side, hipStream_t s);
hipError_t launch_dscale_f(const ChainDev* c, int nc, int l, int M, int parity, int ainv, int which,
                           hipStream_t s);
hipError_t launch_scan_f(int tv, const ChainDev* c, int nc, const Ctl* ctl, int l, int M, int s0, int s1,
                         int dir, int parity, int form_block, hipStream_t s);
hipError_t launch_wf(const ChainDev* c, int nc, int dir, int parity, hipStream_t s);
hipError_t launch_segupd_f(int tv, const ChainDev* c, int nc, int dir, int parity, int ns0, int ns1,
                           hipStream_t s);
hipError_t launch_dscale_u(int fp32b, const ChainDev* c, int nc, int l, int M, int parity,
                           hipStream_t s);
hipError_t launch_pass_end(const ChainDev* c, int nc, hipStream_t s);
hipError_t launch_set_ctl(Ctl* ctl, int measure, int force_reject, float drift_tol, hipStream_t s);
}  // namespace gpqmc

using namespace gpqmc;

namespace {

// ---------------------------------------------------------------------------
// cyclic Jacobi eigensolver for a real symmetric matrix (row-major, n x n):
// rotations annihilate A_pq until the off-diagonal norm is negligible.
// Returns ascending eigenvalues w and eigenvectors as the columns of V.
// ---------------------------------------------------------------------------
void jacobi_eigh(int n, const double* a_in, std::vector<double>& w, std::vector<double>& V) {
  std::vector<double> A(a_in, a_in + (size_t)n * n);
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  double total = 0.0;
  for (size_t i = 0; i < A.size(); ++i) total += A[i] * A[i];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
    if (off <= 1e-32 * total || off == 0.0) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // A <- J^T A J with J the rotation in the (p, q) plane
        for (int k = 0; k < n; ++k) {
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        A[(size_t)p * n + q] = 0.0;
        A[(size_t)q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int x, int y) { return A[(size_t)x * n + x] < A[(size_t)y * n + y]; });
  w.resize(n);
  std::vector<double> Vs((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    w[j] = A[(size_t)ord[j] * n + ord[j]];
    for (int i = 0; i < n; ++i) Vs[(size_t)i * n + j] = V[(size_t)i * n + ord[j]];
  }
  V.swap(Vs);
}

struct Lattice {   // shared by chains with identical hopping and dtau
  int N;
  std::vector<double> K, Km, Kp;
  size_t off_K = 0, off_Km = 0, off_Kp = 0, off_Kmb = 0;  // Kmb: e^{-dtau K} in basis precision
};

struct Trial {     // shared by chains with identical trial Hamiltonian
  int N, n;
  std::vector<double> P;
  size_t off = 0;
};

struct ChainHost {
  int N, n[2];
  int lat, trial[2];
  double U, dtau, g, m_neel, alpha, lam;
  uint64_t seed, chain_id;
  bool trace;
  bool ph = false;            // particle-hole shortcut: spin 1 derived from spin 0
  bool tv = false;            // spinless t-V model (bond fields, one species)
  int nprop = 0;              // proposals per slice: N sites, or the bonds (t-V)
  double V = 0.0;             // t-V repulsion
  std::vector<int> bonds;     // t-V: nprop x 2 sites
  std::vector<int> seg_start; // t-V: first bond of every scan segment, then n_bonds
  bool field_set = false;
  std::vector<int8_t> field;
  std::vector<int8_t> eps;    // sublattice signs (staggered structure factor)
  // workspace offsets (0 = not allocated by this engine)
  size_t G[2] = {0, 0}, Gtmp[2] = {0, 0}, U2[2][2] = {{0, 0}, {0, 0}}, Z[2], Xa[2] = {0, 0},
         Ya[2] = {0, 0}, scan_ws[2], flist;
  size_t stack[2], slot_log[2], slot_sgn[2], Hw[2] = {0, 0}, Qc[2], Wm[2], Rinv[2], Xm[2],
         Ym[2] = {0, 0}, G64[2];
  size_t F[2][2][2] = {}, Mf[2] = {0, 0}, Wf[2] = {0, 0}, Pscr[2] = {0, 0};  // factored engine
  size_t field_off, eps_off, st, meas, tr_ratio = 0, tr_green = 0, tr_drift = 0, tr_logdet = 0;
  size_t mexp_off = 0, bonds_off = 0, dflist = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

std::string key_bytes(const void* p, size_t n) { return std::string((const char*)p, n); }

}  // namespace

struct gpqmc_ctx {
  int n_chains = 0;
  hipStream_t stream = nullptr;
  int fp32 = 0;            // Green's-function (wrap, flush, scan) precision: 1 = FP32, 0 = FP64
  int fp32b = 0;           // basis propagation precision: 1 = FP32, 0 = FP64
  int fact = 0;            // 1: factored engine G = 1 - A B^T (FP64); 0: G wrapped as an N x N matrix
  int l_half = 0, M = 0, n_s = 1, kseg = 64, n_slices = 2;  // kseg: delay rank (sites per flush)
  int n_max = 0;                   // largest lattice of the batch
  int nprop_max = 0;               // most proposals per slice (sites, or t-V bonds) in the batch
  int tv = 0;                      // 1: spinless t-V chains (every chain of the context)
  int n_part = 0;                  // largest particle number (either spin) of the batch
  int n_part_min = 1 << 30;        // smallest particle number of a propagated spin
  int prop_rows = 128;             // output rows of a propagation tile (64 or 128)
  int meas_cap = 4096;
  bool use_graph = true;
  float drift_tol = 1e-3f;
  std::vector<int> ckpts;          // sorted checkpoint positions
  std::map<int, int> slot_of;      // position -> slot
  std::vector<Lattice> lats;
  std::vector<Trial> trials;
  std::vector<ChainHost> ch;
  // layout
  size_t bytes = 0;
  size_t off_chains = 0, off_ctl = 0;
  size_t off_ent[32] = {0};
  // tile lists: N x N, N x n, n x n, n x N, 128 x 128 tiles of N x N, N x n
  // over both factors of both spins, N x (delay rank)
  std::vector<TileRef> tiles[8];
  size_t off_tiles[8] = {0};
  int n_min = 1 << 30;             // smallest lattice of the batch
  bool large_tiles = true;         // every lattice fills 128 x 128 GEMM tiles well
  char* ws = nullptr;
  bool bound = false, initialized = false;
  long long sweeps_done = 0;       // passes enqueued since init_trial (mirrors the device counter)
  int debug_flags = 0;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  hipGraph_t graph_def[2] = {nullptr, nullptr};
  // in-sweep kernel timing: bit t of timing_mask records an event pair around
  // every launch of timed kernel t (passes then launch directly, not as graphs)
  int timing_mask = 0;
  std::vector<hipEvent_t> tev[3];
  size_t tev_used[3] = {0, 0, 0};
  int n_launch[3] = {0, 0, 0};      // launches of each timed class per pass (for reference)
  std::string err;

  template <class T>
  T* at(size_t off) const { return (T*)(ws + off); }
  int slot(int p) const { return slot_of.at(p); }
  bool is_ck(int p) const { return slot_of.count(p) != 0; }
  int n_ck_pass() const { return (int)ckpts.size() - 1; }
};

namespace {

enum EntryKind { E_WRAP1_UP = 0, E_WRAP2_UP, E_WRAP1_DN, E_WRAP2_DN, E_FLUSH, E_FLUSH_T, E_PROP,
                 E_GRAM_U, E_APPLY1, E_XMAT, E_YMAT, E_GFRESH,
                 // factored engine: propagation of both factors (4 entries per chain:
                 // spin-major, A then B), the initialisation's B-only propagation, the
                 // segment update of the dual factor, and the checkpoint products
                 E_PROP_UP, E_PROP_DN, E_PROPB_DN, E_SEGP_UP, E_SEGP_DN, E_SEGF_UP, E_SEGF_DN,
                 E_IMABT, E_GRAM_A, E_GRAM_B, E_APPLY_A, E_APPLY_B, E_BMAT, E_AMAT, E_GFRESH2,
                 E_COUNT };
// T_NN_L: 128 x 128 tiles of the large-tile kernels; T_Nn4: N x n outputs of
// both factors of both spins; T_Nk: N x (delay rank) outputs
enum TileKind { T_NN = 0, T_Nn, T_nn, T_nN, T_NN_L, T_Nn4, T_Nk, T_NP, T_COUNT };
static_assert(E_COUNT <= 32, "entry kinds");
static_assert(T_COUNT <= (int)(sizeof(gpqmc_ctx::off_tiles) / sizeof(size_t)), "tile kinds");

gpqmc_status fail(gpqmc_ctx* c, gpqmc_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

gpqmc_status hip_fail(gpqmc_ctx* c, hipError_t e, const char* where) {
  return fail(c, GPQMC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(call, where)                       \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
  } while (0)

const GemmEntry* ents(const gpqmc_ctx* ctx, int kind) {
  return ctx->at<GemmEntry>(ctx->off_ent[kind]);
}

// ----------------------------------------------------------------------------
// schedule of one pass
// ----------------------------------------------------------------------------
struct Launcher {
  gpqmc_ctx* ctx;
  const ChainDev* chains;
  const Ctl* ctl;
  int nc;
  hipStream_t s;

  GemmArgs args() const {
    GemmArgs a;
    a.scale_slice = -1;
    a.scale_inverse = 0;
    a.bscale_slice = -1;
    a.parity = 0;
    a.slot = 0;
    a.dir = 0;
    a.n_bulk_last = ctx->M;
    a.check_drift = 0;
    return a;
  }
  // timed kernel class of a launch.  G-wrap engine: 0 the kinetic wrap
  // e^{-dtau K} G, 1 the B-scaled basis propagation, 2 the slice's delayed
  // update.  Factored engine: 0 the propagation of both factors, 1 the
  // segment update of the dual factor (Q <- Q - (Q Mf^T) Wf), 2 the flip
  // scan.  -1 none.
  static int timed_class(int kind, int mode) {
    if (mode == GM_STORE && (kind == E_WRAP1_UP || kind == E_WRAP1_DN)) return 0;
    if (mode == GM_PROPB && kind == E_PROP) return 1;
    if (mode == GM_FLUSH && kind == E_FLUSH) return 2;
    if (mode == GM_PROPR && (kind == E_PROP_UP || kind == E_PROP_DN)) return 0;
    if (mode == GM_SEGF) return 1;
    return -1;
  }
  // runs launch(), bracketed by a HIP event pair when class t is timed
  template <class Fn>
  hipError_t timed(int t, Fn launch) {
    if (t < 0 || !(ctx->timing_mask & (1 << t))) return launch();
    auto& ev = ctx->tev[t];
    size_t& used = ctx->tev_used[t];
    while (ev.size() < used + 2) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev.push_back(e);
    }
    hipError_t r = hipEventRecord(ev[used], s);
    if (r == hipSuccess) r = launch();
    if (r == hipSuccess) r = hipEventRecord(ev[used + 1], s);
    if (r == hipSuccess) used += 2;
    return r;
  }
  hipError_t gemm(int kind, int mode, int tk, GemmArgs a) {
    const int t = ctx->timing_mask ? timed_class(kind, mode) : -1;
    return timed(t, [&] { return gemm_launch(kind, mode, tk, a); });
  }
  hipError_t gemm_launch(int kind, int mode, int tk, GemmArgs a) {
    const int f32 = (mode == GM_PROPB || mode == GM_PROPR) ? ctx->fp32b : ctx->fp32;
    // lattices with N >= 128: the FP32 N x N x N products (wrap, slice
    // update) on the large-tile kernel; in FP64 the mode where the large tile
    // measured faster than the 64 x 64 kernel (the scaled wrap)
    if (ctx->large_tiles) {
      const bool nnn = tk == T_NN && (mode == GM_STORE || mode == GM_WRAP || mode == GM_FLUSH);
      if (f32 && nnn)
        return launch_gemm_l(mode, ents(ctx, kind), ctx->at<TileRef>(ctx->off_tiles[T_NN_L]),
                             (int)ctx->tiles[T_NN_L].size(), a, s);
      if (!f32 && tk == T_NN && mode == GM_WRAP)
        return launch_gemm_l64(mode, ents(ctx, kind), ctx->at<TileRef>(ctx->off_tiles[T_NN_L]),
                               (int)ctx->tiles[T_NN_L].size(), a, s);
    }
    // the factored engine's propagation of both factors: row tiles over all
    // n columns (k_prop)
    if (mode == GM_PROPR && tk == T_Nn4 && !f32 && ctx->n_part <= 128)
      return launch_prop(ctx->n_part_min, ctx->n_part, ctx->prop_rows, ents(ctx, kind),
                         ctx->at<TileRef>(ctx->off_tiles[T_NP]), (int)ctx->tiles[T_NP].size(), a, s);
    return launch_gemm(f32, ctx->fp32, mode, ents(ctx, kind), ctx->at<TileRef>(ctx->off_tiles[tk]),
                       (int)ctx->tiles[tk].size(), a, s);
  }

  // checkpoint at position p: re-orthonormalise the active basis U[parity]
  // (Cholesky QR), recompute G = 1 - R (L R)^{-1} L from the stored
  // opposite-side basis, check the sign, store the new basis.
  hipError_t checkpoint(int p, int dir, int parity, int next_scale, int measure, int ck_index,
                        int mode) {
    hipError_t e;
    GemmArgs a = args();
    a.parity = parity;
    if (ctx->fp32b && (e = launch_basis_to_fp64(1, chains, nc, parity, s)) != hipSuccess) return e;
    if ((e = gemm(E_GRAM_U, GM_GRAM, T_nn, a)) != hipSuccess) return e;
    if ((e = launch_chol_inv(chains, nc, ctx->n_part, s)) != hipSuccess) return e;
    if ((e = gemm(E_APPLY1, GM_APPLY, T_Nn, a)) != hipSuccess) return e;
    const int sl = ctx->slot(p);
    if (mode == 2) return launch_finalize(ctx->fp32b, chains, nc, ctl, sl, 2, 0, -1, parity, -1, s);
    a.slot = sl;
    a.dir = dir;
    if ((e = gemm(E_XMAT, GM_XMAT, T_nn, a)) != hipSuccess) return e;
    if ((e = launch_gj_inv(chains, nc, ctx->n_part, s)) != hipSuccess) return e;
    if ((e = gemm(E_YMAT, GM_YMAT, T_nN, a)) != hipSuccess) return e;
    a.scale_slice = next_scale;
    a.check_drift = (mode == 0);
    if ((e = gemm(E_GFRESH, GM_GFRESH, T_NN, a)) != hipSuccess) return e;
    return launch_finalize(ctx->fp32b, chains, nc, ctl, sl, mode, measure, ck_index, parity, -1, s);
  }

  // all proposals of slice l, segment by segment; each segment is flushed into
  // G by a delayed rank-|F| update; the last flush applies the frame change
  hipError_t scan_and_flush(int l, int scale_slice, int inverse) {
    hipError_t e;
    for (int s0 = 0; s0 < ctx->n_max; s0 += ctx->kseg) {
      if ((e = launch_scan(ctx->fp32, 0, chains, nc, ctl, l, ctx->M, s0, s0 + ctx->kseg, 0, 0, s)) !=
          hipSuccess)
        return e;
      if ((e = launch_xy(ctx->fp32, chains, nc, ctx->n_max, s0, ctx->kseg, s)) != hipSuccess) return e;
    }
    GemmArgs a = args();
    a.scale_slice = scale_slice;
    a.scale_inverse = inverse;
    return gemm(E_FLUSH, GM_FLUSH, T_NN, a);
  }

  hipError_t up_pass() {
    hipError_t e;
    const int M = ctx->M;
    if ((e = launch_put_trial(ctx->fp32b, chains, nc, ctx->slot(-1), 1, -1, s)) != hipSuccess) return e;
    int parity = 0, ck = 0;
    for (int l = 0; l <= M + 1; ++l) {
      const bool bulk = (l >= 1 && l <= M);
      const bool ckl = ctx->is_ck(l);
      if ((e = scan_and_flush(l, (!bulk && l == 0 && !ckl) ? 1 : -1, 0)) != hipSuccess) return e;
      if (bulk) {
        GemmArgs a = args();
        if ((e = gemm(E_WRAP1_UP, GM_STORE, T_NN, a)) != hipSuccess) return e;
        a.scale_slice = ckl ? -1 : l + 1;
        if ((e = gemm(E_WRAP2_UP, GM_WRAP, T_NN, a)) != hipSuccess) return e;
        GemmArgs b = args();
        b.bscale_slice = l;
        b.parity = parity;
        if ((e = gemm(E_PROP, GM_PROPB, T_Nn, b)) != hipSuccess) return e;
        parity ^= 1;
      } else {
        if ((e = launch_dscale_u(ctx->fp32b, chains, nc, l, M, parity, s)) != hipSuccess) return e;
      }
      if (ckl) {
        if ((e = checkpoint(l, 0, parity, l <= M ? l + 1 : -1, l == ctx->l_half, ck++, 0)) != hipSuccess)
          return e;
      }
    }
    return launch_pass_end(chains, nc, s);
  }

  hipError_t down_pass() {
    hipError_t e;
    const int M = ctx->M;
    if ((e = launch_put_trial(ctx->fp32b, chains, nc, ctx->slot(M + 1), 1, -1, s)) != hipSuccess) return e;
    int parity = 0, ck = 0;
    for (int l = M + 1; l >= 0; --l) {
      const bool bulk = (l >= 1 && l <= M);
      if (bulk) {
        GemmArgs a = args();
        if ((e = gemm(E_WRAP1_DN, GM_STORE, T_NN, a)) != hipSuccess) return e;
        if ((e = gemm(E_WRAP2_DN, GM_WRAP, T_NN, a)) != hipSuccess) return e;
      }
      if ((e = scan_and_flush(l, l, 1)) != hipSuccess) return e;
      if (bulk) {
        GemmArgs b = args();
        b.scale_slice = l;
        b.parity = parity;
        if ((e = gemm(E_PROP, GM_PROPR, T_Nn, b)) != hipSuccess) return e;
        parity ^= 1;
      } else {
        if ((e = launch_dscale_u(ctx->fp32b, chains, nc, l, M, parity, s)) != hipSuccess) return e;
      }
      const int p = l - 1;
      if (ctx->is_ck(p)) {
        if ((e = checkpoint(p, 1, parity, p == -1 ? 0 : -1, p == ctx->l_half, ck++, 0)) != hipSuccess)
          return e;
      }
    }
    return launch_pass_end(chains, nc, s);
  }

  hipError_t init_pass() {
    hipError_t e;
    const int M = ctx->M;
    if ((e = launch_put_trial(ctx->fp32b, chains, nc, ctx->slot(M + 1), 1, -1, s)) != hipSuccess) return e;
    if ((e = launch_put_trial(ctx->fp32b, chains, nc, ctx->slot(-1), 0, -1, s)) != hipSuccess) return e;
    int parity = 0;
    for (int l = M + 1; l >= 0; --l) {
      const bool bulk = (l >= 1 && l <= M);
      if (bulk) {
        GemmArgs b = args();
        b.scale_slice = l;
        b.parity = parity;
        if ((e = gemm(E_PROP, GM_PROPR, T_Nn, b)) != hipSuccess) return e;
        parity ^= 1;
      } else {
        if ((e = launch_dscale_u(ctx->fp32b, chains, nc, l, M, parity, s)) != hipSuccess) return e;
      }
      const int p = l - 1;
      if (ctx->is_ck(p)) {
        if ((e = checkpoint(p, 1, parity, p == -1 ? 0 : -1, 0, -1, p >= 0 ? 2 : 1)) != hipSuccess)
          return e;
      }
    }
    return hipSuccess;
  }

  // ---------------------------------------------------------------------------
  // factored engine: G = 1 - A B^T, A and B of size N x n (FP64).  Upward the
  // moving basis is A = R (the flips scale its rows, B takes the Woodbury
  // update); downward it is B = L^T and A takes the update.  Flips of slice l
  // happen with D_l (its field before the slice's flips) already applied to
  // the factors: upward D_l G_{l-1} D_l^{-1}, downward G_{l-1}; both have the
  // diagonal the ratio 1 + Delta (1 - G_ii) needs.
  // ---------------------------------------------------------------------------
  // segments of up to 32 sites run the one-wave scan; with at most 128
  // particles per spin the dual factor's update is the fused one-pass kernel;
  // otherwise the general scan and two GEMMs (Q Mf^T, then Q - (Q Mf^T) Wf)
  hipError_t flips_f(int l, int dir, int parity) {
    hipError_t e;
    GemmArgs a = args();
    a.parity = parity;
    const bool fast_scan = ctx->kseg <= kBlock;
    const bool fast_upd = fast_scan && ctx->n_part <= 128;
    const int tscan = ctx->timing_mask ? 2 : -1, tupd = ctx->timing_mask ? 1 : -1;
    // segments: kseg sites from s0, or (t-V) the chain's segment s0 of its
    // bond list (nprop_max is then the most segments of a chain)
    const int step = ctx->tv ? 1 : ctx->kseg;
    bool have_block = false;   // the segment's block was formed by the previous update
    for (int s0 = 0; s0 < ctx->nprop_max; s0 += step) {
      if ((e = timed(tscan, [&] {
             return fast_scan ? launch_scan_f(ctx->tv, chains, nc, ctl, l, ctx->M, s0, s0 + step, dir,
                                              parity, have_block ? 0 : 1, s)
                              : launch_scan(0, 1, chains, nc, ctl, l, ctx->M, s0, s0 + ctx->kseg,
                                            dir, parity, s);
           })) != hipSuccess)
        return e;
      if (fast_upd) {
        // the fused update forms Mf and Wf itself, and the next segment's block
        const int ns0 = s0 + step < ctx->nprop_max ? s0 + step : -1;
        if ((e = timed(tupd, [&] {
               return launch_segupd_f(ctx->tv, chains, nc, dir, parity, ns0, ns0 + step, s);
             })) != hipSuccess)
          return e;
        have_block = ns0 >= 0;
      } else {
        if (fast_scan && (e = timed(tscan, [&] { return launch_wf(chains, nc, dir, parity, s); })) !=
                             hipSuccess)
          return e;
        if ((e = gemm(dir == 0 ? E_SEGP_UP : E_SEGP_DN, GM_SEGP, T_Nk, a)) != hipSuccess) return e;
        if ((e = gemm(dir == 0 ? E_SEGF_UP : E_SEGF_DN, GM_SEGF, T_Nn, a)) != hipSuccess) return e;
      }
    }
    return hipSuccess;
  }

  // checkpoint at position p.  up: the moving basis is A (upward pass), else
  // B.  out_up: leave the factors in the up form (A = R, B = L^T (L R)^{-T}),
  // else in the down form (A = R (L R)^{-1}, B = L^T).  mode 0: a pass's
  // checkpoint (drift of the wrapped G); 1: the initialisation's last; 2:
  // store only.  next_scale >= 0: then apply D_{next_scale} to both factors.
  hipError_t checkpoint_f(int p, bool up, int parity, int mode, int measure, int ck_index,
                          bool out_up, int next_scale) {
    hipError_t e;
    GemmArgs a = args();
    a.parity = parity;
    const bool drift = (mode == 0);
    if (drift && (e = gemm(E_IMABT, GM_IMABT, T_NN, a)) != hipSuccess) return e;
    if ((e = gemm(up ? E_GRAM_A : E_GRAM_B, GM_GRAM, T_nn, a)) != hipSuccess) return e;
    if ((e = launch_chol_inv(chains, nc, ctx->n_part, s)) != hipSuccess) return e;
    if ((e = gemm(up ? E_APPLY_A : E_APPLY_B, GM_APPLY, T_Nn, a)) != hipSuccess) return e;
    const int sl = ctx->slot(p);
    if (mode == 2) return launch_finalize(0, chains, nc, ctl, sl, 2, 0, -1, parity, up ? 0 : 1, s);
    a.slot = sl;
    a.dir = up ? 0 : 1;
    if ((e = gemm(E_XMAT, GM_XMAT, T_nn, a)) != hipSuccess) return e;
    if ((e = launch_gj_inv(chains, nc, ctx->n_part, s)) != hipSuccess) return e;
    // operands: R is Qc moving upward, else the stack slot; L likewise
    const int rsrc = up ? 0 : 1, lsrc = up ? 1 : 0;
    int side;
    if (out_up) {
      a.lsel = lsrc;
      if ((e = gemm(E_BMAT, GM_BMAT, T_Nn, a)) != hipSuccess) return e;   // B = L^T X^{-T}
      a.rsel = rsrc;   // A = R: Qc (copied in by finalize) or the slot (P, put by the next pass)
      a.lsel = 2;
      side = up ? 0 : 2;
    } else {
      a.rsel = rsrc;
      if ((e = gemm(E_AMAT, GM_AMAT, T_Nn, a)) != hipSuccess) return e;   // A = R X^{-1}
      a.rsel = 2;
      a.lsel = lsrc;   // B = L^T: Qc (copied in by finalize) or the slot (P, put by the next pass)
      side = up ? 2 : 1;
    }
    a.check_drift = drift;
    if ((e = gemm(E_GFRESH2, GM_GFRESH2, T_NN, a)) != hipSuccess) return e;
    if ((e = launch_finalize(0, chains, nc, ctl, sl, mode, measure, ck_index, parity, side, s)) !=
        hipSuccess)
      return e;
    if (next_scale >= 0) return launch_dscale_f(chains, nc, next_scale, ctx->M, parity, 0, 3, s);
    return hipSuccess;
  }

  hipError_t up_pass_f() {
    hipError_t e;
    const int M = ctx->M;
    // A = P (the slot -1 holds P too); B is the up-form factor left by the
    // previous pass; then the frame of slice 0
    if ((e = launch_put_trial(0, chains, nc, ctx->slot(-1), 1, 0, s)) != hipSuccess) return e;
    if ((e = launch_dscale_f(chains, nc, 0, M, 0, 0, 3, s)) != hipSuccess) return e;
    int parity = 0, ck = 0;
    for (int l = 0; l <= M + 1; ++l) {
      const bool bulk = (l >= 1 && l <= M);
      const bool ckl = ctx->is_ck(l);
      if ((e = flips_f(l, 0, parity)) != hipSuccess) return e;
      if (bulk) {
        // A <- D_{l+1} e^{-dtau K} A, B <- D_{l+1}^{-1} e^{+dtau K} B (no frame
        // change before a checkpoint)
        GemmArgs a = args();
        a.parity = parity;
        a.scale_slice = ckl ? -1 : l + 1;
        if ((e = gemm(E_PROP_UP, GM_PROPR, T_Nn4, a)) != hipSuccess) return e;
        parity ^= 1;
      } else if (l == 0 && !ckl) {
        if ((e = launch_dscale_f(chains, nc, 1, M, parity, 0, 3, s)) != hipSuccess) return e;
      }
      if (ckl && (e = checkpoint_f(l, true, parity, 0, l == ctx->l_half, ck++, l <= M,
                                   l <= M ? l + 1 : -1)) != hipSuccess)
        return e;
    }
    return launch_pass_end(chains, nc, s);
  }

  hipError_t down_pass_f() {
    hipError_t e;
    const int M = ctx->M;
    // B = P; A is the down-form factor left by the upward pass
    if ((e = launch_put_trial(0, chains, nc, ctx->slot(M + 1), 1, 1, s)) != hipSuccess) return e;
    int parity = 0, ck = 0;
    for (int l = M + 1; l >= 0; --l) {
      const bool bulk = (l >= 1 && l <= M);
      if (bulk) {
        // A <- D_l^{-1} e^{+dtau K} A, B <- D_l e^{-dtau K} B
        GemmArgs a = args();
        a.parity = parity;
        a.scale_slice = l;
        if ((e = gemm(E_PROP_DN, GM_PROPR, T_Nn4, a)) != hipSuccess) return e;
        parity ^= 1;
      } else if ((e = launch_dscale_f(chains, nc, l, M, parity, 1, 3, s)) != hipSuccess) {
        return e;
      }
      if ((e = flips_f(l, 1, parity)) != hipSuccess) return e;
      const int p = l - 1;
      if (ctx->is_ck(p) &&
          (e = checkpoint_f(p, false, parity, 0, p == ctx->l_half, ck++, p == -1, -1)) != hipSuccess)
        return e;
    }
    return launch_pass_end(chains, nc, s);
  }

  hipError_t init_pass_f() {
    hipError_t e;
    const int M = ctx->M;
    if ((e = launch_put_trial(0, chains, nc, ctx->slot(M + 1), 1, 1, s)) != hipSuccess) return e;
    if ((e = launch_put_trial(0, chains, nc, ctx->slot(-1), 0, 1, s)) != hipSuccess) return e;
    int parity = 0;
    for (int l = M + 1; l >= 0; --l) {
      const bool bulk = (l >= 1 && l <= M);
      if (bulk) {
        GemmArgs a = args();
        a.parity = parity;
        a.scale_slice = l;
        if ((e = gemm(E_PROPB_DN, GM_PROPR, T_Nn, a)) != hipSuccess) return e;
        parity ^= 1;
      } else if ((e = launch_dscale_f(chains, nc, l, M, parity, 1, 2, s)) != hipSuccess) {
        return e;
      }
      const int p = l - 1;
      if (ctx->is_ck(p) &&
          (e = checkpoint_f(p, false, parity, p >= 0 ? 2 : 1, 0, -1, true, -1)) != hipSuccess)
        return e;
    }
    return hipSuccess;
  }

  hipError_t up() { return ctx->fact ? up_pass_f() : up_pass(); }
  hipError_t down() { return ctx->fact ? down_pass_f() : down_pass(); }
  hipError_t init() { return ctx->fact ? init_pass_f() : init_pass(); }
};

Launcher make_launcher(gpqmc_ctx* ctx) {
  Launcher L;
  L.ctx = ctx;
  L.chains = ctx->at<ChainDev>(ctx->off_chains);
  L.ctl = ctx->at<Ctl>(ctx->off_ctl);
  L.nc = ctx->n_chains;
  L.s = ctx->stream;
  return L;
}

// whole_n: one tile over all columns of each row tile
void build_tiles(std::vector<TileRef>& out, const std::vector<std::pair<int, int>>& mn,
                 const std::vector<char>& skip, int tile, bool whole_n = false) {
  out.clear();
  for (size_t e = 0; e < mn.size(); ++e) {
    if (skip[e]) continue;
    const int tm = (mn[e].first + tile - 1) / tile;
    const int tn = whole_n ? 1 : (mn[e].second + tile - 1) / tile;
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) out.push_back(TileRef{(int)e, a, b, 0});
  }
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

gpqmc_status gpqmc_create(int32_t n_chains, const gpqmc_chain_desc* chains,
                          const gpqmc_options* opts, void* hip_stream, gpqmc_ctx** out) {
  if (!out) return GPQMC_EINVAL;
  *out = nullptr;
  std::unique_ptr<gpqmc_ctx> ctx(new (std::nothrow) gpqmc_ctx());
  if (!ctx) return GPQMC_ENOMEM;
  gpqmc_ctx* c = ctx.get();
  // on error the context is still returned so that gpqmc_last_error() can
  // describe the problem; the caller destroys it
  auto bad = [&](gpqmc_status code, const std::string& msg) {
    c->err = msg;
    *out = ctx.release();
    return code;
  };
  if (n_chains <= 0 || !chains) return bad(GPQMC_EINVAL, "n_chains <= 0 or chains == NULL");
  c->n_chains = n_chains;
  c->stream = (hipStream_t)hip_stream;
  const gpqmc_chain_desc& d0 = chains[0];
  c->l_half = d0.l_half;
  c->n_s = d0.stab_interval;
  c->kseg = d0.delay_rank;
  if (d0.precision != GPQMC_MIXED && d0.precision != GPQMC_FP64 &&
      d0.precision != GPQMC_MIXED_FP32_BASIS && d0.precision != GPQMC_FP64_WRAP)
    return bad(GPQMC_EINVAL, "precision must be GPQMC_FP64, GPQMC_MIXED, GPQMC_MIXED_FP32_BASIS "
                             "or GPQMC_FP64_WRAP");
  c->fp32 = (d0.precision == GPQMC_FP64 || d0.precision == GPQMC_FP64_WRAP) ? 0 : 1;
  c->fp32b = d0.precision == GPQMC_MIXED_FP32_BASIS ? 1 : 0;
  c->fact = d0.precision == GPQMC_FP64 ? 1 : 0;
  if (d0.model != GPQMC_MODEL_HUBBARD && d0.model != GPQMC_MODEL_TV)
    return bad(GPQMC_EINVAL, "model must be GPQMC_MODEL_HUBBARD or GPQMC_MODEL_TV");
  c->tv = d0.model == GPQMC_MODEL_TV ? 1 : 0;
  if (c->tv && (!c->fact || d0.delay_rank % 2 != 0 || d0.delay_rank > kBlock))
    return bad(GPQMC_EINVAL, "the t-V model needs GPQMC_FP64 and an even delay_rank <= 32");
  if (c->l_half < 0 || c->n_s < 1 || c->kseg < 1 || c->kseg > kSegMax)
    return bad(GPQMC_EINVAL, "need l_half >= 0, stab_interval >= 1, 1 <= delay_rank <= 64");
  c->M = 2 * c->l_half;
  c->n_slices = c->M + 2;
  // relative drift (largest |G_wrapped - G_fresh| over largest |G_fresh|)
  // that flags a chain: FP64 wrapping stays near 1e-9 on the 16x16 workload
  // at n_s = 10; with an FP32 Green's function the stated accuracy bound of
  // the mixed path, 1e-5, is the threshold (it is exceeded while sampling the
  // doped 16x16 workload, and the flag says so)
  c->drift_tol = c->fp32 ? 1e-5f : 1e-6f;
  if (opts) {
    if (opts->meas_capacity > 0) c->meas_cap = opts->meas_capacity;
    c->use_graph = opts->use_graph != 0;
    if (opts->drift_tol > 0) c->drift_tol = (float)opts->drift_tol;
  }
  const bool ph_req = opts && opts->particle_hole != 0 && c->fact && c->kseg <= kBlock && !c->tv;
  if (!c->stream) c->use_graph = false;   // the null stream cannot be captured
  // checkpoints C = {-1, l_half, M+1} U {j n_s : 1 <= j n_s <= M}
  std::vector<int> ck = {-1, c->l_half, c->M + 1};
  for (int j = c->n_s; j <= c->M; j += c->n_s) ck.push_back(j);
  std::sort(ck.begin(), ck.end());
  ck.erase(std::unique(ck.begin(), ck.end()), ck.end());
  c->ckpts = ck;
  for (size_t i = 0; i < ck.size(); ++i) c->slot_of[ck[i]] = (int)i;

  std::map<std::string, int> lat_of, trial_of;
  for (int i = 0; i < n_chains; ++i) {
    const gpqmc_chain_desc& d = chains[i];
    char buf[200];
    if (d.l_half != c->l_half || d.stab_interval != c->n_s || d.delay_rank != c->kseg ||
        d.precision != d0.precision || d.model != d0.model) {
      snprintf(buf, sizeof buf, "chain %d: l_half, stab_interval, delay_rank, precision and model "
               "must match chain 0", i);
      return bad(GPQMC_EINVAL, buf);
    }
    const int N = d.n_sites;
    if (N < 1 || N > kMaxSites || d.n_up < 1 || d.n_up > N ||
        (c->tv ? d.n_dn != 0 : (d.n_dn < 1 || d.n_dn > N)) || !d.hopping || !d.sublattice ||
        !(d.U >= 0) || !(d.dtau > 0) || !(d.g >= 0) || (c->tv && !(d.V >= 0))) {
      snprintf(buf, sizeof buf, "chain %d: need 1 <= N <= %d, 1 <= n_up <= N, 1 <= n_dn <= N "
               "(t-V: n_dn = 0, V >= 0), U >= 0, dtau > 0, g >= 0 and non-NULL hopping and "
               "sublattice", i, kMaxSites);
      return bad(GPQMC_EINVAL, buf);
    }
    ChainHost h;
    h.N = N;
    h.n[0] = d.n_up;
    h.n[1] = d.n_dn;
    h.U = d.U;
    h.dtau = d.dtau;
    h.g = d.g;
    h.m_neel = d.m_neel;
    // density-channel bond decoupling (t-V) or spin-channel site decoupling
    // (Hubbard), cosh c = exp(x / 2) with x = dtau V or dtau U
    const double x_bulk = c->tv ? d.dtau * d.V : d.dtau * d.U;
    h.alpha = x_bulk == 0 ? 0.0 : std::acosh(std::exp(0.5 * x_bulk));
    h.lam = d.g == 0 ? 0.0 : std::acosh(std::exp(0.5 * d.g));
    h.seed = d.seed;
    h.chain_id = d.chain_id;
    h.trace = d.trace != 0;
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < a; ++b)
        if (d.hopping[(size_t)a * N + b] != d.hopping[(size_t)b * N + a])
          return bad(GPQMC_EINVAL, "hopping matrix not symmetric");
    // lattice exponentials
    std::string lk = key_bytes(d.hopping, sizeof(double) * N * N) + key_bytes(&d.dtau, 8);
    auto it = lat_of.find(lk);
    if (it == lat_of.end()) {
      Lattice L;
      L.N = N;
      L.K.assign(d.hopping, d.hopping + (size_t)N * N);
      std::vector<double> w, V;
      jacobi_eigh(N, d.hopping, w, V);
      L.Km.assign((size_t)N * N, 0.0);
      L.Kp.assign((size_t)N * N, 0.0);
      for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
          double sm = 0.0, sp = 0.0;
          for (int k = 0; k < N; ++k) {
            const double v = V[(size_t)a * N + k] * V[(size_t)b * N + k];
            sm += v * std::exp(-d.dtau * w[k]);
            sp += v * std::exp(d.dtau * w[k]);
          }
          L.Km[(size_t)a * N + b] = sm;
          L.Kp[(size_t)a * N + b] = sp;
        }
      it = lat_of.emplace(lk, (int)c->lats.size()).first;
      c->lats.push_back(std::move(L));
    }
    h.lat = it->second;
    // Neel trial per spin: lowest n_sigma eigenvectors of K + sigma M_N eps + v
    // (t-V: the CDW trial of the one species, K + Delta_C eps with Delta_C = M_N)
    for (int sp = 0; sp < (c->tv ? 1 : 2); ++sp) {
      const double sigma = sp == 0 ? 1.0 : -1.0;
      std::vector<double> hm(d.hopping, d.hopping + (size_t)N * N);
      for (int a = 0; a < N; ++a) {
        hm[(size_t)a * N + a] += sigma * d.m_neel * (double)d.sublattice[a];
        if (d.trial_potential) hm[(size_t)a * N + a] += d.trial_potential[a];
      }
      const int nsig = h.n[sp];
      std::string tk = key_bytes(hm.data(), sizeof(double) * hm.size()) + key_bytes(&nsig, 4);
      auto jt = trial_of.find(tk);
      if (jt == trial_of.end()) {
        std::vector<double> w, V;
        jacobi_eigh(N, hm.data(), w, V);
        if (nsig < N && w[nsig] - w[nsig - 1] < 1e-6) {
          snprintf(buf, sizeof buf, "chain %d spin %d: degenerate trial (gap %.3e)", i, sp,
                   w[nsig] - w[nsig - 1]);
          return bad(GPQMC_EDEGENERATE, buf);
        }
        Trial T;
        T.N = N;
        T.n = nsig;
        T.P.resize((size_t)N * nsig);
        for (int a = 0; a < N; ++a)
          for (int b = 0; b < nsig; ++b) T.P[(size_t)a * nsig + b] = V[(size_t)a * N + b];
        jt = trial_of.emplace(tk, (int)c->trials.size()).first;
        c->trials.push_back(std::move(T));
      }
      h.trial[sp] = jt->second;
    }
    if (c->tv) {
      h.trial[1] = h.trial[0];   // no second species (never read)
      h.tv = true;
      h.V = d.V;
      if (!d.bonds || d.n_bonds < 1) return bad(GPQMC_EINVAL, "t-V chain without bonds");
      h.bonds.assign(d.bonds, d.bonds + 2 * (size_t)d.n_bonds);
      std::vector<int> deg(N, 0);
      for (int b = 0; b < d.n_bonds; ++b) {
        const int bi = h.bonds[2 * b], bj = h.bonds[2 * b + 1];
        if (bi < 0 || bi >= N || bj < 0 || bj >= N || bi == bj)
          return bad(GPQMC_EINVAL, "t-V bond with a site out of range or twice");
        if (++deg[bi] > kMexp || ++deg[bj] > kMexp) {
          snprintf(buf, sizeof buf, "t-V: more than %d bonds at a site", kMexp);
          return bad(GPQMC_EINVAL, buf);
        }
      }
      // scan segments: runs of consecutive bonds, at most delay_rank / 2 and
      // site-disjoint (a new segment starts where the next bond would share a
      // site), so that a segment's block holds distinct sites
      h.seg_start.assign(1, 0);
      std::vector<char> used(N, 0);
      int cnt = 0;
      for (int b = 0; b < d.n_bonds; ++b) {
        const int bi = h.bonds[2 * b], bj = h.bonds[2 * b + 1];
        if (cnt == c->kseg / 2 || used[bi] || used[bj]) {
          h.seg_start.push_back(b);
          std::fill(used.begin(), used.end(), 0);
          cnt = 0;
        }
        used[bi] = used[bj] = 1;
        ++cnt;
      }
      h.seg_start.push_back(d.n_bonds);
      h.nprop = d.n_bonds;
    } else {
      h.nprop = N;
    }
    // particle-hole shortcut: exact when the spin-down problem is the image
    // of the spin-up one under c_i -> eps_i c_i^dag (bipartite hopping, half
    // filling, no trial potential: the Neel trials map onto each other)
    if (ph_req && N % 2 == 0 && d.n_up == N / 2 && d.n_dn == N / 2 && !d.trial_potential) {
      bool bip = true;
      for (int a = 0; a < N && bip; ++a) {
        if (d.sublattice[a] != 1 && d.sublattice[a] != -1) bip = false;
        for (int b = 0; b < N && bip; ++b)
          if (d.hopping[(size_t)a * N + b] != 0.0 && d.sublattice[a] == d.sublattice[b]) bip = false;
      }
      h.ph = bip;
    }
    h.field.assign((size_t)c->n_slices * h.nprop, 1);
    h.eps.assign(d.sublattice, d.sublattice + N);
    c->ch.push_back(std::move(h));
  }

  // ---- workspace layout ----
  const size_t bs = c->fp32 ? 4 : 8;     // Green's-function element size
  const size_t ub = c->fp32b ? 4 : 8;    // basis element size
  size_t off = 0;
  auto take = [&](size_t b) {
    off = align256(off);
    const size_t o = off;
    off += std::max<size_t>(b, 1);
    return o;
  };
  for (auto& L : c->lats) {
    const size_t nn = (size_t)L.N * L.N;
    L.off_K = take(nn * 8);
    L.off_Km = take(nn * bs);
    L.off_Kp = take(nn * bs);
    L.off_Kmb = (ub == bs) ? L.off_Km : take(nn * ub);
  }
  for (auto& T : c->trials) T.off = take((size_t)T.N * T.n * 8);
  const int n_slots = (int)c->ckpts.size();
  const int nck = c->n_ck_pass();
  for (auto& h : c->ch) {
    const size_t N = h.N, nn = N * N;
    for (int sp = 0; sp < 2; ++sp) {
      const size_t nb = N * h.n[sp];
      if (c->fact) {
        // factored engine: both factors (ping-pong pairs), the segment's
        // Woodbury operands, Q Mf^T, and the wrapped G of a checkpoint
        for (int side = 0; side < 2; ++side)
          for (int par = 0; par < 2; ++par) h.F[side][sp][par] = take(nb * 8);
        h.Mf[sp] = take((size_t)kSegMax * h.n[sp] * 8);
        h.Wf[sp] = take((size_t)kSegMax * h.n[sp] * 8);
        h.Pscr[sp] = take(N * kSegMax * 8);
        h.G[sp] = take(nn * 8);
      } else {
        h.G[sp] = take(nn * bs);
        h.Gtmp[sp] = take(nn * bs);
        h.U2[sp][0] = take(nb * ub);
        h.U2[sp][1] = take(nb * ub);
        h.Xa[sp] = take(nn * bs);
        h.Ya[sp] = take(nn * bs);
        h.Hw[sp] = take(nb * 8);
        h.Ym[sp] = take((size_t)h.n[sp] * N * 8);
      }
      h.Z[sp] = take((size_t)kSegMax * kSegMax * bs);
      h.scan_ws[sp] = take((size_t)5 * kBlock * kSegMax * bs);
      h.stack[sp] = take((size_t)n_slots * nb * 8);
      h.slot_log[sp] = take((size_t)n_slots * 8);
      h.slot_sgn[sp] = take((size_t)n_slots * 4);
      h.Qc[sp] = take(nb * 8);
      h.Wm[sp] = take((size_t)h.n[sp] * h.n[sp] * 8);
      h.Rinv[sp] = take((size_t)h.n[sp] * h.n[sp] * 8);
      h.Xm[sp] = take((size_t)h.n[sp] * h.n[sp] * 8);
      h.G64[sp] = take(nn * 8);
    }
    h.field_off = take((size_t)c->n_slices * h.nprop);
    h.mexp_off = h.tv ? take((size_t)c->n_slices * N) : h.field_off;
    if (h.tv) h.bonds_off = take((h.bonds.size() + h.seg_start.size()) * 4);
    h.dflist = take((size_t)2 * kSegMax * 8);
    h.eps_off = take((size_t)N);
    h.st = take(sizeof(ChainState));
    h.flist = take((size_t)kSegMax * 4);
    h.meas = take((size_t)c->meas_cap * kMeasCols * 8);
    if (h.trace) {
      h.tr_ratio = take((size_t)c->n_slices * h.nprop * 2 * 8);
      h.tr_green = take((size_t)nck * 2 * nn * 8);
      h.tr_drift = take((size_t)nck * 8);
      h.tr_logdet = take((size_t)nck * 2 * 2 * 8);
    }
  }
  c->off_chains = take(sizeof(ChainDev) * n_chains);
  c->off_ctl = take(sizeof(Ctl));
  for (int k = 0; k < E_COUNT; ++k) c->off_ent[k] = take(sizeof(GemmEntry) * 4 * n_chains);
  std::vector<std::pair<int, int>> sz[T_COUNT];
  std::vector<char> skip[T_COUNT];   // entries without tiles (spin 1 of particle-hole chains)
  for (auto& h : c->ch) {
    c->n_max = std::max(c->n_max, h.N);
    c->nprop_max = std::max(c->nprop_max, h.tv ? (int)h.seg_start.size() - 1 : h.nprop);
    c->n_min = std::min(c->n_min, h.N);
    // 128 x 128 tiles for N >= 128 while at least 3/4 of the padded tile grid
    // is real work (at N = 288, 56%, the 64 x 64 kernel measured 6% faster
    // per sweep)
    const long long padded = 128LL * ((h.N + 127) / 128);
    if (h.N < 128 || 4LL * h.N * h.N < 3 * padded * padded) c->large_tiles = false;
    c->n_part = std::max(c->n_part, std::max(h.n[0], h.n[1]));
    c->n_part_min = std::min(c->n_part_min, (h.ph || h.tv) ? h.n[0] : std::min(h.n[0], h.n[1]));
    // 128-row propagation tiles only where they waste no more rows than 64-row ones
    if ((h.N + 127) / 128 * 128 > (h.N + 63) / 64 * 64) c->prop_rows = 64;
    for (int sp = 0; sp < 2; ++sp) {
      sz[T_NN].push_back({h.N, h.N});
      sz[T_Nn].push_back({h.N, h.n[sp]});
      sz[T_nn].push_back({h.n[sp], h.n[sp]});
      sz[T_nN].push_back({h.n[sp], h.N});
      sz[T_NN_L].push_back({h.N, h.N});
      sz[T_Nn4].push_back({h.N, h.n[sp]});   // factor A of this spin
      sz[T_Nn4].push_back({h.N, h.n[sp]});   // factor B
      sz[T_NP].push_back({h.N, h.n[sp]});    // the same two, row tiles over all columns
      sz[T_NP].push_back({h.N, h.n[sp]});
      sz[T_Nk].push_back({h.N, c->kseg});
      const char sk = (sp == 1 && (h.ph || h.tv)) ? 1 : 0;
      for (int t = 0; t < T_COUNT; ++t) skip[t].push_back(sk);
      skip[T_Nn4].push_back(sk);
      skip[T_NP].push_back(sk);
    }
  }
  for (int t = 0; t < T_COUNT; ++t) {
    build_tiles(c->tiles[t], sz[t], skip[t],
                t == T_NN_L ? 128 : t == T_NP ? c->prop_rows : kTile, t == T_NP);
    c->off_tiles[t] = take(sizeof(TileRef) * c->tiles[t].size());
  }
  c->bytes = align256(off);
  *out = ctx.release();
  return GPQMC_OK;
}

gpqmc_status gpqmc_workspace_bytes(const gpqmc_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return GPQMC_EINVAL;
  *bytes = ctx->bytes;
  return GPQMC_OK;
}

gpqmc_status gpqmc_bind_workspace(gpqmc_ctx* ctx, void* device_ptr, size_t bytes) {
  if (!ctx || !device_ptr) return GPQMC_EINVAL;
  if (((uintptr_t)device_ptr & 255) != 0) return fail(ctx, GPQMC_EINVAL, "workspace not 256-byte aligned");
  if (bytes < ctx->bytes) return fail(ctx, GPQMC_ENOMEM, "workspace too small");
  ctx->ws = (char*)device_ptr;
  const bool f32 = ctx->fp32 != 0;
  auto up = [&](size_t off, const void* src, size_t b) {
    return hipMemcpy(ctx->ws + off, src, b, hipMemcpyHostToDevice);
  };
  for (auto& L : ctx->lats) {
    const size_t nn = (size_t)L.N * L.N;
    HIPCHK(up(L.off_K, L.K.data(), nn * 8), "upload K");
    if (f32) {
      std::vector<float> a(L.Km.begin(), L.Km.end()), b(L.Kp.begin(), L.Kp.end());
      HIPCHK(up(L.off_Km, a.data(), nn * 4), "upload Km");
      HIPCHK(up(L.off_Kp, b.data(), nn * 4), "upload Kp");
      if (L.off_Kmb != L.off_Km) HIPCHK(up(L.off_Kmb, L.Km.data(), nn * 8), "upload Km (basis)");
    } else {
      HIPCHK(up(L.off_Km, L.Km.data(), nn * 8), "upload Km");
      HIPCHK(up(L.off_Kp, L.Kp.data(), nn * 8), "upload Kp");
    }
  }
  for (auto& T : ctx->trials) HIPCHK(up(T.off, T.P.data(), T.P.size() * 8), "upload P");

  const int nc = ctx->n_chains;
  std::vector<ChainDev> cd(nc);
  std::vector<GemmEntry> E[E_COUNT];
  for (int k = 0; k < E_COUNT; ++k) E[k].resize(4 * nc);
  for (int i = 0; i < nc; ++i) {
    ChainHost& h = ctx->ch[i];
    ChainDev& d = cd[i];
    memset(&d, 0, sizeof d);
    const Lattice& L = ctx->lats[h.lat];
    d.N = h.N;
    d.n[0] = h.n[0];
    d.n[1] = h.n[1];
    for (int b = 0; b < 2; ++b) {
      const double cpl = b == 0 ? h.lam : h.alpha;
      for (int sp = 0; sp < 2; ++sp) {
        const double sigma = sp == 0 ? 1.0 : -1.0;
        for (int m = -kMexp; m <= kMexp; ++m) d.dval[b][sp][m + kMexp] = std::exp(sigma * cpl * m);
        for (int si = 0; si < 2; ++si) {
          const double s = si == 0 ? 1.0 : -1.0;
          d.delta[b][sp][si] = std::exp(-2.0 * sigma * cpl * s) - 1.0;
        }
      }
    }
    d.U_hub = h.U;
    d.ph = h.ph ? 1 : 0;
    d.tv = h.tv ? 1 : 0;
    d.nsp = (h.ph || h.tv) ? 1 : 2;
    d.n_bonds = h.tv ? h.nprop : 0;
    d.V = h.V;
    d.bonds = h.tv ? ctx->at<int>(h.bonds_off) : nullptr;
    d.seg_start = h.tv ? ctx->at<int>(h.bonds_off) + h.bonds.size() : nullptr;
    d.n_seg = h.tv ? (int)h.seg_start.size() - 1 : 0;
    d.mexp = ctx->at<int8_t>(h.mexp_off);
    d.dflist = ctx->at<double>(h.dflist);
    d.coupling[0] = h.lam;
    d.coupling[1] = h.alpha;
    d.n_slices = ctx->n_slices;
    d.key0 = (uint32_t)(h.seed & 0xffffffffu);
    d.key1 = (uint32_t)(h.seed >> 32) ^ (uint32_t)TAG_ACCEPT;
    d.chain_id = (uint32_t)h.chain_id;
    // buffers this engine does not allocate stay NULL
    auto wp = [&](size_t off) -> void* { return off ? (void*)(ctx->ws + off) : nullptr; };
    for (int sp = 0; sp < 2; ++sp) {
      d.G[sp] = wp(h.G[sp]);
      d.Gtmp[sp] = wp(h.Gtmp[sp]);
      d.U[sp][0] = wp(h.U2[sp][0]);
      d.U[sp][1] = wp(h.U2[sp][1]);
      d.Z[sp] = ctx->ws + h.Z[sp];
      d.Xa[sp] = wp(h.Xa[sp]);
      d.Ya[sp] = wp(h.Ya[sp]);
      d.scan_ws[sp] = ctx->ws + h.scan_ws[sp];
      for (int side = 0; side < 2; ++side)
        for (int par = 0; par < 2; ++par) d.F[side][sp][par] = wp(h.F[side][sp][par]);
      d.Mf[sp] = (double*)wp(h.Mf[sp]);
      d.Wf[sp] = (double*)wp(h.Wf[sp]);
      d.P[sp] = ctx->at<double>(ctx->trials[h.trial[sp]].off);
      d.stack[sp] = ctx->at<double>(h.stack[sp]);
      d.slot_log[sp] = ctx->at<double>(h.slot_log[sp]);
      d.slot_sgn[sp] = ctx->at<int>(h.slot_sgn[sp]);
      d.Hw[sp] = (double*)wp(h.Hw[sp]);
      d.Qc[sp] = ctx->at<double>(h.Qc[sp]);
      d.Wm[sp] = ctx->at<double>(h.Wm[sp]);
      d.Rinv[sp] = ctx->at<double>(h.Rinv[sp]);
      d.Xm[sp] = ctx->at<double>(h.Xm[sp]);
      d.Ym[sp] = (double*)wp(h.Ym[sp]);
      d.G64[sp] = ctx->at<double>(h.G64[sp]);
    }
    d.Km = ctx->ws + L.off_Km;
    d.Kp = ctx->ws + L.off_Kp;
    d.Khop = ctx->at<double>(L.off_K);
    d.field = ctx->at<int8_t>(h.field_off);
    d.eps = ctx->at<int8_t>(h.eps_off);
    d.st = ctx->at<ChainState>(h.st);
    d.flist = ctx->at<int>(h.flist);
    d.meas = ctx->at<double>(h.meas);
    d.meas_cap = ctx->meas_cap;
    if (h.trace) {
      d.trace_ratio = ctx->at<double>(h.tr_ratio);
      d.trace_green = ctx->at<double>(h.tr_green);
      d.trace_drift = ctx->at<double>(h.tr_drift);
      d.trace_logdet = ctx->at<double>(h.tr_logdet);
    }
    const int N = h.N;
    for (int sp = 0; sp < 2; ++sp) {
      const int n = h.n[sp];
      const int ei = 2 * i + sp;
      GemmEntry base;
      memset(&base, 0, sizeof base);
      base.field = d.mexp;
      base.n_sites = N;
      base.spin = sp;
      base.st = d.st;
      for (int b = 0; b < 2; ++b)
        for (int m = 0; m <= 2 * kMexp; ++m) base.dval[b][m] = d.dval[b][sp][m];
      auto mk = [&](const void* A0, const void* A1, const void* B0, const void* B1, void* C0,
                    void* C1, int M_, int N_, int K_, int lda, int ldb, int ldc) {
        GemmEntry e = base;
        e.A[0] = A0;
        e.A[1] = A1;
        e.B[0] = B0;
        e.B[1] = B1;
        e.C[0] = C0;
        e.C[1] = C1;
        e.M = M_;
        e.N = N_;
        e.K = K_;
        e.lda = lda;
        e.ldb = ldb;
        e.ldc = ldc;
        return e;
      };
      auto nnE = [&](const void* A, const void* B, void* C) {
        return mk(A, A, B, B, C, C, N, N, N, N, N, N);
      };
      GemmEntry xm = mk(nullptr, nullptr, nullptr, nullptr, d.Xm[sp], d.Xm[sp], n, n, N, n, n, n);
      xm.stack = d.stack[sp];
      xm.Qc = d.Qc[sp];
      xm.slot_stride = N * n;
      E[E_XMAT][ei] = xm;
      if (ctx->fact) {
        const void* Fa0 = d.F[0][sp][0];
        const void* Fa1 = d.F[0][sp][1];
        const void* Fb0 = d.F[1][sp][0];
        const void* Fb1 = d.F[1][sp][1];
        const void* Km = d.Km;   // e^{-dtau K}, FP64 in this engine
        const void* Kp = d.Kp;   // e^{+dtau K}
        auto prop = [&](const void* K, const void* F0, const void* F1, int inv) {
          GemmEntry e = mk(K, K, F0, F1, (void*)F0, (void*)F1, N, n, N, N, n, n);
          e.sinv = inv;
          return e;
        };
        const int e4 = 4 * i + 2 * sp;
        E[E_PROP_UP][e4 + 0] = prop(Km, Fa0, Fa1, 0);   // A <- D e^{-dtau K} A
        E[E_PROP_UP][e4 + 1] = prop(Kp, Fb0, Fb1, 1);   // B <- D^{-1} e^{+dtau K} B
        E[E_PROP_DN][e4 + 0] = prop(Kp, Fa0, Fa1, 1);   // A <- D^{-1} e^{+dtau K} A
        E[E_PROP_DN][e4 + 1] = prop(Km, Fb0, Fb1, 0);   // B <- D e^{-dtau K} B
        E[E_PROPB_DN][ei] = prop(Km, Fb0, Fb1, 0);
        void* Ps = ctx->ws + h.Pscr[sp];
        auto segp = [&](const void* Q0, const void* Q1) {
          GemmEntry e = mk(Q0, Q1, d.Mf[sp], d.Mf[sp], Ps, Ps, N, ctx->kseg, n, n, n, kSegMax);
          e.dynN = &d.st->fcount;
          return e;
        };
        auto segf = [&](const void* Q0, const void* Q1) {
          GemmEntry e = mk(Ps, Ps, d.Wf[sp], d.Wf[sp], (void*)Q0, (void*)Q1, N, n, ctx->kseg,
                           kSegMax, n, n);
          e.dynK = &d.st->fcount;
          return e;
        };
        E[E_SEGP_UP][ei] = segp(Fb0, Fb1);
        E[E_SEGP_DN][ei] = segp(Fa0, Fa1);
        E[E_SEGF_UP][ei] = segf(Fb0, Fb1);
        E[E_SEGF_DN][ei] = segf(Fa0, Fa1);
        E[E_IMABT][ei] = mk(Fa0, Fa1, Fb0, Fb1, d.G[sp], d.G[sp], N, N, n, n, n, N);
        E[E_GRAM_A][ei] = mk(Fa0, Fa1, nullptr, nullptr, d.Wm[sp], d.Wm[sp], n, n, N, n, n, n);
        E[E_GRAM_B][ei] = mk(Fb0, Fb1, nullptr, nullptr, d.Wm[sp], d.Wm[sp], n, n, N, n, n, n);
        E[E_APPLY_A][ei] = mk(Fa0, Fa1, d.Rinv[sp], d.Rinv[sp], d.Qc[sp], d.Qc[sp], N, n, n, n, n, n);
        E[E_APPLY_B][ei] = mk(Fb0, Fb1, d.Rinv[sp], d.Rinv[sp], d.Qc[sp], d.Qc[sp], N, n, n, n, n, n);
        auto ck = [&](GemmEntry e) {
          e.stack = d.stack[sp];
          e.Qc = d.Qc[sp];
          e.slot_stride = N * n;
          return e;
        };
        E[E_BMAT][ei] = ck(mk(nullptr, nullptr, d.Xm[sp], d.Xm[sp], (void*)Fb0, (void*)Fb1, N, n, n,
                              n, n, n));
        E[E_AMAT][ei] = ck(mk(nullptr, nullptr, d.Xm[sp], d.Xm[sp], (void*)Fa0, (void*)Fa1, N, n, n,
                              n, n, n));
        GemmEntry g2 = ck(mk(Fa0, Fa1, Fb0, Fb1, d.G64[sp], d.G[sp], N, N, n, n, n, N));
        g2.ldc2 = N;
        E[E_GFRESH2][ei] = g2;
        continue;
      }
      E[E_WRAP1_UP][ei] = nnE(d.Km, d.G[sp], d.Gtmp[sp]);
      E[E_WRAP2_UP][ei] = nnE(d.Gtmp[sp], d.Kp, d.G[sp]);
      E[E_WRAP1_DN][ei] = nnE(d.Kp, d.G[sp], d.Gtmp[sp]);
      E[E_WRAP2_DN][ei] = nnE(d.Gtmp[sp], d.Km, d.G[sp]);
      // the slice's delayed update G <- G - Xa Ya (K = the slice's accepted flips);
      // the timing copy writes the wrap scratch instead of G
      GemmEntry fl = mk(d.Xa[sp], d.Xa[sp], d.Ya[sp], d.Ya[sp], d.G[sp], d.G[sp], N, N, N, N, N, N);
      fl.dynK = &d.st->ftot;
      E[E_FLUSH][ei] = fl;
      fl.C[1] = d.Gtmp[sp];
      E[E_FLUSH_T][ei] = fl;
      const void* Kmb = ctx->ws + L.off_Kmb;
      E[E_PROP][ei] = mk(Kmb, Kmb, d.U[sp][0], d.U[sp][1], d.U[sp][0], d.U[sp][1], N, n, N, N, n, n);
      // checkpoint: Cholesky QR of U[parity] (or of its FP64 copy in Hw)
      const void* src0 = ctx->fp32b ? (const void*)d.Hw[sp] : d.U[sp][0];
      const void* src1 = ctx->fp32b ? (const void*)d.Hw[sp] : d.U[sp][1];
      E[E_GRAM_U][ei] = mk(src0, src1, nullptr, nullptr, d.Wm[sp], d.Wm[sp], n, n, N, n, n, n);
      E[E_APPLY1][ei] = mk(src0, src1, d.Rinv[sp], d.Rinv[sp], d.Qc[sp], d.Qc[sp], N, n, n, n, n, n);
      GemmEntry ym = mk(d.Xm[sp], d.Xm[sp], nullptr, nullptr, d.Ym[sp], d.Ym[sp], n, N, n, n, n, N);
      ym.stack = d.stack[sp];
      ym.Qc = d.Qc[sp];
      ym.slot_stride = N * n;
      E[E_YMAT][ei] = ym;
      GemmEntry gf = mk(nullptr, nullptr, d.Ym[sp], d.Ym[sp], d.G64[sp], d.G[sp], N, N, n, n, N, N);
      gf.ldc2 = N;
      gf.stack = d.stack[sp];
      gf.Qc = d.Qc[sp];
      gf.slot_stride = N * n;
      E[E_GFRESH][ei] = gf;
    }
  }
  HIPCHK(up(ctx->off_chains, cd.data(), sizeof(ChainDev) * nc), "upload chains");
  for (int i = 0; i < nc; ++i) {
    HIPCHK(up(ctx->ch[i].eps_off, ctx->ch[i].eps.data(), ctx->ch[i].eps.size()), "upload eps");
    if (ctx->ch[i].tv) {
      std::vector<int> bs(ctx->ch[i].bonds);
      bs.insert(bs.end(), ctx->ch[i].seg_start.begin(), ctx->ch[i].seg_start.end());
      HIPCHK(up(ctx->ch[i].bonds_off, bs.data(), bs.size() * 4), "upload bonds");
    }
  }
  for (int k = 0; k < E_COUNT; ++k)
    HIPCHK(up(ctx->off_ent[k], E[k].data(), sizeof(GemmEntry) * E[k].size()), "upload entries");
  for (int t = 0; t < T_COUNT; ++t)
    HIPCHK(up(ctx->off_tiles[t], ctx->tiles[t].data(), sizeof(TileRef) * ctx->tiles[t].size()), "tiles");
  Ctl ctl = {0, 0, ctx->drift_tol, 0};
  HIPCHK(up(ctx->off_ctl, &ctl, sizeof ctl), "upload ctl");
  HIPCHK(hipDeviceSynchronize(), "bind");
  ctx->bound = true;
  ctx->initialized = false;
  return GPQMC_OK;
}

gpqmc_status gpqmc_init_trial(gpqmc_ctx* ctx) {
  if (!ctx) return GPQMC_EINVAL;
  if (!ctx->bound) return fail(ctx, GPQMC_ESTATE, "init_trial before bind_workspace");
  const int nc = ctx->n_chains;
  // initial fields: Philox(key = (lo32 seed, hi32 seed ^ INIT), ctr = (chain, 0, l, i))
  for (int i = 0; i < nc; ++i) {
    ChainHost& h = ctx->ch[i];
    if (!h.field_set) {
      const uint32_t k0 = (uint32_t)(h.seed & 0xffffffffu), k1 = (uint32_t)(h.seed >> 32) ^ TAG_INIT;
      for (int l = 0; l < ctx->n_slices; ++l)
        for (int s = 0; s < h.nprop; ++s) {
          uint32_t c[4] = {(uint32_t)h.chain_id, 0u, (uint32_t)l, (uint32_t)s};
          philox4x32_10(c, k0, k1);
          h.field[(size_t)l * h.nprop + s] = (c[0] & 1u) ? 1 : -1;
        }
    }
    HIPCHK(hipMemcpyAsync(ctx->ws + h.field_off, h.field.data(), h.field.size(),
                          hipMemcpyHostToDevice, ctx->stream), "upload field");
    std::vector<int8_t> mexp;
    if (h.tv) {
      // site exponents: +s_b at a bond's A end, -s_b at its B end
      mexp.assign((size_t)ctx->n_slices * h.N, 0);
      for (int l = 0; l < ctx->n_slices; ++l)
        for (int b = 0; b < h.nprop; ++b) {
          const int8_t sb = h.field[(size_t)l * h.nprop + b];
          mexp[(size_t)l * h.N + h.bonds[2 * b]] += sb;
          mexp[(size_t)l * h.N + h.bonds[2 * b + 1]] -= sb;
        }
      HIPCHK(hipMemcpyAsync(ctx->ws + h.mexp_off, mexp.data(), mexp.size(), hipMemcpyHostToDevice,
                            ctx->stream), "upload site exponents");
    }
    ChainState st;
    memset(&st, 0, sizeof st);
    st.sign = 1;
    st.run_sgn[0] = st.run_sgn[1] = 1;
    HIPCHK(hipMemcpyAsync(ctx->ws + h.st, &st, sizeof st, hipMemcpyHostToDevice, ctx->stream),
           "upload state");
    HIPCHK(hipStreamSynchronize(ctx->stream), "init sync");
  }
  Launcher L = make_launcher(ctx);
  HIPCHK(launch_set_ctl(ctx->at<Ctl>(ctx->off_ctl), 0, 0, ctx->drift_tol, ctx->stream), "ctl");
  HIPCHK(L.init(), "init pass");
  HIPCHK(hipStreamSynchronize(ctx->stream), "init_trial");
  ctx->initialized = true;
  ctx->sweeps_done = 0;
  return GPQMC_OK;
}

gpqmc_status gpqmc_sweep(gpqmc_ctx* ctx, int32_t n_sweeps, int32_t measure) {
  if (!ctx) return GPQMC_EINVAL;
  if (!ctx->initialized) return fail(ctx, GPQMC_ESTATE, "sweep before init_trial");
  if (n_sweeps < 0) return fail(ctx, GPQMC_EINVAL, "n_sweeps < 0");
  static_assert(sizeof(ChainState) % 8 == 0, "state alignment");
  Launcher L = make_launcher(ctx);
  HIPCHK(launch_set_ctl(ctx->at<Ctl>(ctx->off_ctl), measure ? 1 : 0, ctx->debug_flags & 1,
                        ctx->drift_tol, ctx->stream), "ctl");
  for (int w = 0; w < n_sweeps; ++w) {
    const int dir = (int)(ctx->sweeps_done & 1);
    ctx->sweeps_done += 1;
    if (ctx->use_graph && ctx->timing_mask == 0) {
      if (!ctx->graph[dir]) {
        HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal), "capture");
        hipError_t e = dir == 0 ? L.up() : L.down();
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
        if (e != hipSuccess) return hip_fail(ctx, e, "capture pass");
        if (e2 != hipSuccess) return hip_fail(ctx, e2, "end capture");
        ctx->graph_def[dir] = g;
        HIPCHK(hipGraphInstantiate(&ctx->graph[dir], g, nullptr, nullptr, 0), "instantiate");
      }
      HIPCHK(hipGraphLaunch(ctx->graph[dir], ctx->stream), "graph launch");
    } else {
      HIPCHK(dir == 0 ? L.up() : L.down(), "pass");
    }
  }
  return GPQMC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// host statistics
// ---------------------------------------------------------------------------
namespace {

gpqmc_status fetch_records(gpqmc_ctx* ctx, int chain, std::vector<double>& rec) {
  if (!ctx->initialized) return fail(ctx, GPQMC_ESTATE, "no measurements before init_trial");
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  rec.clear();
  const int lo = chain < 0 ? 0 : chain, hi = chain < 0 ? ctx->n_chains : chain + 1;
  for (int c = lo; c < hi; ++c) {
    ChainState st;
    HIPCHK(hipMemcpy(&st, ctx->ws + ctx->ch[c].st, sizeof st, hipMemcpyDeviceToHost), "state");
    const size_t b = rec.size();
    rec.resize(b + (size_t)st.n_meas * kMeasCols);
    if (st.n_meas > 0)
      HIPCHK(hipMemcpy(rec.data() + b, ctx->ws + ctx->ch[c].meas, (size_t)st.n_meas * kMeasCols * 8,
                       hipMemcpyDeviceToHost), "records");
  }
  return GPQMC_OK;
}

// <s O>/<s> with a delete-one-bin jackknife over bins of 10 records;
// which = 0: sign itself (plain binned mean), 1: energy, 2: double occupancy,
// 3: staggered structure factor.
gpqmc_status weighted(gpqmc_ctx* ctx, int chain, int which, double* mean, double* err) {
  if (!ctx || !mean || !err) return GPQMC_EINVAL;
  if (chain < -1 || chain >= ctx->n_chains) return fail(ctx, GPQMC_EINVAL, "chain out of range");
  std::vector<double> rec;
  gpqmc_status st = fetch_records(ctx, chain, rec);
  if (st != GPQMC_OK) return st;
  const size_t n = rec.size() / kMeasCols, bin = 10, nb = n / bin;
  if (nb < 2) return fail(ctx, GPQMC_EINVAL, "fewer than 20 measurement records");
  std::vector<double> s(nb, 0.0), so(nb, 0.0);
  for (size_t b = 0; b < nb; ++b)
    for (size_t k = 0; k < bin; ++k) {
      const double* r = &rec[(b * bin + k) * kMeasCols];
      s[b] += r[0] / bin;
      so[b] += (which == 0 ? r[0] : r[0] * r[which]) / bin;
    }
  double S = 0, SO = 0;
  for (size_t b = 0; b < nb; ++b) {
    S += s[b];
    SO += so[b];
  }
  if (which == 0) {
    const double m = S / nb;
    double v = 0;
    for (size_t b = 0; b < nb; ++b) v += (s[b] - m) * (s[b] - m);
    *mean = m;
    *err = std::sqrt(v / (nb - 1) / nb);
    return GPQMC_OK;
  }
  *mean = SO / S;
  std::vector<double> jk(nb);
  double jm = 0;
  for (size_t b = 0; b < nb; ++b) {
    jk[b] = (SO - so[b]) / (S - s[b]);
    jm += jk[b] / nb;
  }
  double v = 0;
  for (size_t b = 0; b < nb; ++b) v += (jk[b] - jm) * (jk[b] - jm);
  *err = std::sqrt((double)(nb - 1) / nb * v);
  return GPQMC_OK;
}

}  // namespace

extern "C" {

gpqmc_status gpqmc_measure_energy(gpqmc_ctx* ctx, int32_t chain, double* mean, double* err) {
  return weighted(ctx, chain, 1, mean, err);
}
gpqmc_status gpqmc_measure_double_occupancy(gpqmc_ctx* ctx, int32_t chain, double* mean,
                                            double* err) {
  return weighted(ctx, chain, 2, mean, err);
}
gpqmc_status gpqmc_measure_sign(gpqmc_ctx* ctx, int32_t chain, double* mean, double* err) {
  return weighted(ctx, chain, 0, mean, err);
}
gpqmc_status gpqmc_measure_structure_factor(gpqmc_ctx* ctx, int32_t chain, double* mean,
                                            double* err) {
  return weighted(ctx, chain, 3, mean, err);
}

gpqmc_status gpqmc_get_measurements(gpqmc_ctx* ctx, int32_t chain, double* out, int32_t capacity,
                                    int32_t* n_out) {
  if (!ctx || !out || !n_out || chain < 0 || chain >= ctx->n_chains) return GPQMC_EINVAL;
  std::vector<double> rec;
  gpqmc_status st = fetch_records(ctx, chain, rec);
  if (st != GPQMC_OK) return st;
  const int n = std::min<int>((int)(rec.size() / kMeasCols), capacity);
  memcpy(out, rec.data(), (size_t)n * kMeasCols * 8);
  *n_out = n;
  return GPQMC_OK;
}

gpqmc_status gpqmc_reset_measurements(gpqmc_ctx* ctx) {
  if (!ctx || !ctx->initialized) return GPQMC_ESTATE;
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  for (auto& h : ctx->ch) {
    ChainState st;
    HIPCHK(hipMemcpy(&st, ctx->ws + h.st, sizeof st, hipMemcpyDeviceToHost), "state");
    st.n_meas = 0;
    st.flags &= ~FLAG_MEAS_FULL;
    HIPCHK(hipMemcpy(ctx->ws + h.st, &st, sizeof st, hipMemcpyHostToDevice), "state");
  }
  return GPQMC_OK;
}

gpqmc_status gpqmc_set_field(gpqmc_ctx* ctx, int32_t chain, const int8_t* field) {
  if (!ctx || !field || chain < 0 || chain >= ctx->n_chains) return GPQMC_EINVAL;
  ChainHost& h = ctx->ch[chain];
  for (size_t k = 0; k < h.field.size(); ++k)
    if (field[k] != 1 && field[k] != -1) return fail(ctx, GPQMC_EINVAL, "field entries must be +-1");
  h.field.assign(field, field + h.field.size());
  h.field_set = true;
  ctx->initialized = false;
  return GPQMC_OK;
}

gpqmc_status gpqmc_get_field(gpqmc_ctx* ctx, int32_t chain, int8_t* field) {
  if (!ctx || !field || chain < 0 || chain >= ctx->n_chains) return GPQMC_EINVAL;
  if (!ctx->bound) return GPQMC_ESTATE;
  const ChainHost& h = ctx->ch[chain];
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  HIPCHK(hipMemcpy(field, ctx->ws + h.field_off, h.field.size(), hipMemcpyDeviceToHost), "field");
  return GPQMC_OK;
}

gpqmc_status gpqmc_get_green(gpqmc_ctx* ctx, int32_t chain, int32_t spin, double* G) {
  if (!ctx || !G || chain < 0 || chain >= ctx->n_chains || spin < 0 || spin > 1) return GPQMC_EINVAL;
  if (!ctx->initialized) return GPQMC_ESTATE;
  const ChainHost& h = ctx->ch[chain];
  if (h.tv && spin == 1) return fail(ctx, GPQMC_EINVAL, "t-V chains have one species (spin 0)");
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  const bool mirror = spin == 1 && h.ph;
  HIPCHK(hipMemcpy(G, ctx->ws + h.G64[mirror ? 0 : spin], (size_t)h.N * h.N * 8,
                   hipMemcpyDeviceToHost),
         "G");
  if (mirror) {
    // G_dn = 1 - E G_up^T E, E = diag(sublattice)
    const int N = h.N;
    for (int i = 0; i < N; ++i)
      for (int j = i; j < N; ++j) {
        const double e = (double)h.eps[i] * (double)h.eps[j];
        const double gij = G[(size_t)i * N + j], gji = G[(size_t)j * N + i];
        G[(size_t)i * N + j] = (i == j ? 1.0 : 0.0) - e * gji;
        G[(size_t)j * N + i] = (i == j ? 1.0 : 0.0) - e * gij;
      }
  }
  return GPQMC_OK;
}

gpqmc_status gpqmc_get_chain_info(gpqmc_ctx* ctx, int32_t chain, gpqmc_chain_info* info) {
  if (!ctx || !info || chain < 0 || chain >= ctx->n_chains) return GPQMC_EINVAL;
  if (!ctx->initialized) return GPQMC_ESTATE;
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  ChainState st;
  HIPCHK(hipMemcpy(&st, ctx->ws + ctx->ch[chain].st, sizeof st, hipMemcpyDeviceToHost), "state");
  info->sign = st.sign;
  info->flags = st.flags;
  info->n_meas = st.n_meas;
  info->sign_mismatch = st.sign_mismatch;
  info->sweep = st.sweep;
  info->max_drift = st.max_drift;
  info->last_drift = st.last_drift;
  info->accepted = st.accepted;
  info->proposed = st.proposed;
  info->max_rel_drift = st.max_rel_drift;
  info->last_rel_drift = st.last_rel_drift;
  info->particle_hole = ctx->ch[chain].ph ? 1 : 0;
  info->reserved = 0;
  return GPQMC_OK;
}

gpqmc_status gpqmc_logdet(gpqmc_ctx* ctx, int32_t chain, double* logabs, int32_t* sign) {
  if (!ctx || !logabs || !sign || chain < 0 || chain >= ctx->n_chains) return GPQMC_EINVAL;
  if (!ctx->initialized) return fail(ctx, GPQMC_ESTATE, "logdet before init_trial");
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  ChainState st;
  HIPCHK(hipMemcpy(&st, ctx->ws + ctx->ch[chain].st, sizeof st, hipMemcpyDeviceToHost), "state");
  for (int sp = 0; sp < 2; ++sp) {
    logabs[sp] = st.w_log[sp];
    sign[sp] = st.w_sgn[sp];
  }
  return GPQMC_OK;
}

gpqmc_status gpqmc_get_trace_logdet(gpqmc_ctx* ctx, int32_t chain, double* logdets) {
  if (!ctx || !logdets || chain < 0 || chain >= ctx->n_chains) return GPQMC_EINVAL;
  const ChainHost& h = ctx->ch[chain];
  if (!h.trace) return fail(ctx, GPQMC_EINVAL, "chain created without trace");
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  HIPCHK(hipMemcpy(logdets, ctx->ws + h.tr_logdet, (size_t)ctx->n_ck_pass() * 4 * 8,
                   hipMemcpyDeviceToHost), "logdets");
  return GPQMC_OK;
}

gpqmc_status gpqmc_chain_status(gpqmc_ctx* ctx, int32_t chain) {
  gpqmc_chain_info info;
  gpqmc_status s = gpqmc_get_chain_info(ctx, chain, &info);
  if (s != GPQMC_OK) return s;
  return info.flags & (FLAG_DRIFT | FLAG_NAN | FLAG_SINGULAR | FLAG_SIGN) ? GPQMC_EUNSTABLE : GPQMC_OK;
}

gpqmc_status gpqmc_set_debug(gpqmc_ctx* ctx, int32_t flags) {
  if (!ctx) return GPQMC_EINVAL;
  ctx->debug_flags = flags;
  return GPQMC_OK;
}

gpqmc_status gpqmc_get_trace(gpqmc_ctx* ctx, int32_t chain, double* ratios, double* greens,
                             double* drifts, int32_t* n_checkpoints) {
  if (!ctx || chain < 0 || chain >= ctx->n_chains) return GPQMC_EINVAL;
  const ChainHost& h = ctx->ch[chain];
  if (!h.trace) return fail(ctx, GPQMC_EINVAL, "chain created without trace");
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  const size_t N = h.N;
  const int nck = ctx->n_ck_pass();
  if (n_checkpoints) *n_checkpoints = nck;
  if (ratios)
    HIPCHK(hipMemcpy(ratios, ctx->ws + h.tr_ratio, (size_t)ctx->n_slices * h.nprop * 2 * 8,
                     hipMemcpyDeviceToHost), "ratios");
  if (greens)
    HIPCHK(hipMemcpy(greens, ctx->ws + h.tr_green, (size_t)nck * 2 * N * N * 8,
                     hipMemcpyDeviceToHost), "greens");
  if (drifts)
    HIPCHK(hipMemcpy(drifts, ctx->ws + h.tr_drift, (size_t)nck * 8, hipMemcpyDeviceToHost), "drifts");
  return GPQMC_OK;
}

gpqmc_status gpqmc_debug_gemm(int32_t precision, int32_t M, int32_t N, int32_t K, int32_t flags,
                              const void* A, int32_t lda, const void* B, int32_t ldb, void* C,
                              int32_t ldc, void* hip_stream) {
  if (M <= 0 || N <= 0 || K < 0 || !A || !B || !C) return GPQMC_EINVAL;
  const int trans_a = flags & 1, large = (flags >> 1) & 1;
  if (large && (trans_a || (precision != GPQMC_MIXED && precision != GPQMC_FP64)))
    return GPQMC_EINVAL;
  gpqmc_ctx* ctx = nullptr;
  GemmEntry e;
  memset(&e, 0, sizeof e);
  e.A[0] = e.A[1] = A;
  e.B[0] = e.B[1] = B;
  e.C[0] = e.C[1] = C;
  e.M = M;
  e.N = N;
  e.K = K;
  e.lda = lda;
  e.ldb = ldb;
  e.ldc = ldc;
  std::vector<TileRef> tl;
  build_tiles(tl, {{M, N}}, {0}, large ? 128 : kTile);
  // test hook: a small descriptor buffer in device memory for this one call
  void* dbuf = nullptr;
  const size_t bytes = align256(sizeof e) + sizeof(TileRef) * tl.size();
  HIPCHK(hipMalloc(&dbuf, bytes), "debug alloc");
  hipStream_t s = (hipStream_t)hip_stream;
  HIPCHK(hipMemcpy(dbuf, &e, sizeof e, hipMemcpyHostToDevice), "debug upload");
  TileRef* dt = (TileRef*)((char*)dbuf + align256(sizeof e));
  HIPCHK(hipMemcpy(dt, tl.data(), sizeof(TileRef) * tl.size(), hipMemcpyHostToDevice), "debug upload");
  GemmArgs a;
  memset(&a, 0, sizeof a);
  a.scale_slice = -1;
  a.bscale_slice = -1;
  hipError_t err;
  if (large && precision == GPQMC_MIXED)
    err = launch_gemm_l(GM_STORE, (const GemmEntry*)dbuf, dt, (int)tl.size(), a, s);
  else if (large)
    err = launch_gemm_l64(GM_STORE, (const GemmEntry*)dbuf, dt, (int)tl.size(), a, s);
  else
    err = launch_gemm_plain(precision == GPQMC_MIXED, trans_a, (const GemmEntry*)dbuf, dt,
                            (int)tl.size(), a, s);
  hipError_t err2 = hipStreamSynchronize(s);
  const hipError_t err3 = hipFree(dbuf);
  if (err3 != hipSuccess) return GPQMC_EHIP;
  if (err != hipSuccess) return GPQMC_EHIP;
  if (err2 != hipSuccess) return GPQMC_EHIP;
  return GPQMC_OK;
}

gpqmc_status gpqmc_time_kernel(gpqmc_ctx* ctx, int32_t kernel, int32_t reps, float* ms_per_launch) {
  if (!ctx || !ms_per_launch || reps < 1 || kernel < 0 || kernel > 2) return GPQMC_EINVAL;
  if (!ctx->initialized) return fail(ctx, GPQMC_ESTATE, "time_kernel before init_trial");
  if (ctx->fact && kernel != 0)
    return fail(ctx, GPQMC_EINVAL, "time_kernel: the factored engine times kernel 0 only");
  Launcher L = make_launcher(ctx);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0), "event");
  HIPCHK(hipEventCreate(&e1), "event");
  // every kernel writes only scratch that every pass rebuilds before reading it
  auto one = [&]() -> hipError_t {
    GemmArgs a = L.args();
    if (ctx->fact) {   // both factors of every chain and spin, parity 0 -> 1 (idle buffers)
      a.parity = 0;
      return L.gemm(E_PROP_UP, GM_PROPR, T_Nn4, a);
    }
    if (kernel == 0) return L.gemm(E_WRAP1_UP, GM_STORE, T_NN, a);  // Gtmp = e^{-dtau K} G
    if (kernel == 2)   // the last slice's delayed update, result into Gtmp instead of G
      return L.gemm(E_FLUSH_T, GM_FLUSH, T_NN, a);
    a.parity = 0;                                                  // U[1] = e^{-dtau K} U[0]
    return L.gemm(E_PROP, GM_PROPB, T_Nn, a);
  };
  HIPCHK(one(), "warm");
  HIPCHK(hipEventRecord(e0, ctx->stream), "event");
  for (int r = 0; r < reps; ++r) HIPCHK(one(), "time");
  HIPCHK(hipEventRecord(e1, ctx->stream), "event");
  HIPCHK(hipEventSynchronize(e1), "event");
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1), "event");
  HIPCHK(hipEventDestroy(e0), "event");
  HIPCHK(hipEventDestroy(e1), "event");
  *ms_per_launch = ms / reps;
  return GPQMC_OK;
}

gpqmc_status gpqmc_set_kernel_timing(gpqmc_ctx* ctx, int32_t mask) {
  if (!ctx || mask < 0 || mask > 7) return GPQMC_EINVAL;
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  ctx->timing_mask = mask;
  for (auto& u : ctx->tev_used) u = 0;
  return GPQMC_OK;
}

gpqmc_status gpqmc_get_kernel_timing(gpqmc_ctx* ctx, int32_t kernel, float* total_ms,
                                     int32_t* launches) {
  if (!ctx || kernel < 0 || kernel > 2 || !total_ms || !launches) return GPQMC_EINVAL;
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  double sum = 0.0;
  const auto& ev = ctx->tev[kernel];
  for (size_t i = 0; i + 1 < ctx->tev_used[kernel]; i += 2) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "elapsed");
    sum += ms;
  }
  *total_ms = (float)sum;
  *launches = (int32_t)(ctx->tev_used[kernel] / 2);
  return GPQMC_OK;
}

gpqmc_status gpqmc_debug_step(gpqmc_ctx* ctx, int32_t stage, int32_t l, int32_t s0, int32_t s1) {
  if (!ctx || !ctx->initialized || l < 0 || l > ctx->M + 1) return GPQMC_EINVAL;
  if (ctx->fact) return fail(ctx, GPQMC_EINVAL, "debug_step: G-wrap engines only");
  Launcher L = make_launcher(ctx);
  HIPCHK(launch_set_ctl(ctx->at<Ctl>(ctx->off_ctl), 0, ctx->debug_flags & 1, ctx->drift_tol,
                        ctx->stream), "ctl");
  hipError_t e = hipErrorInvalidValue;
  if (stage == 0)
    e = launch_scan(ctx->fp32, 0, L.chains, L.nc, L.ctl, l, ctx->M, s0, s1, 0, 0, ctx->stream);
  if (stage == 1) e = launch_xy(ctx->fp32, L.chains, L.nc, ctx->n_max, s0, ctx->kseg, ctx->stream);
  if (stage == 2) {
    GemmArgs a = L.args();
    e = L.gemm(E_FLUSH, GM_FLUSH, T_NN, a);
  }
  HIPCHK(e, "debug step");
  HIPCHK(hipStreamSynchronize(ctx->stream), "debug step");
  return GPQMC_OK;
}

gpqmc_status gpqmc_debug_read(gpqmc_ctx* ctx, int32_t chain, int32_t what, int32_t spin, double* out,
                              int64_t count) {
  if (!ctx || !out || chain < 0 || chain >= ctx->n_chains || spin < 0 || spin > 1 || count < 0)
    return GPQMC_EINVAL;
  if (ctx->fact) return fail(ctx, GPQMC_EINVAL, "debug_read: G-wrap engines only");
  const ChainHost& h = ctx->ch[chain];
  size_t off = 0, elem = ctx->fp32 ? 4 : 8, cap = 0;
  bool is_int = false;
  switch (what) {
    case 0: off = h.G[spin]; cap = (size_t)h.N * h.N; break;
    case 1: off = h.Z[spin]; cap = (size_t)kSegMax * kSegMax; break;
    case 2: off = h.flist; elem = 4; is_int = true; cap = kSegMax; break;
    case 3: off = h.Ya[spin]; cap = (size_t)h.N * h.N; break;
    case 4: off = h.Xa[spin]; cap = (size_t)h.N * h.N; break;
    case 5: off = h.st; elem = 0; cap = 3; break;
    default: return GPQMC_EINVAL;
  }
  if ((size_t)count > cap) return fail(ctx, GPQMC_EINVAL, "debug_read: count exceeds the buffer");
  HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
  if (elem == 0) {
    ChainState st;
    HIPCHK(hipMemcpy(&st, ctx->ws + off, sizeof st, hipMemcpyDeviceToHost), "state");
    const double v[3] = {(double)st.fcount, (double)st.sign, (double)st.accepted};
    for (int64_t i = 0; i < count; ++i) out[i] = v[i];
    return GPQMC_OK;
  }
  std::vector<char> buf((size_t)count * elem);
  HIPCHK(hipMemcpy(buf.data(), ctx->ws + off, buf.size(), hipMemcpyDeviceToHost), "read");
  for (int64_t i = 0; i < count; ++i)
    out[i] = is_int ? (double)((int*)buf.data())[i]
             : elem == 4 ? (double)((float*)buf.data())[i] : ((double*)buf.data())[i];
  return GPQMC_OK;
}

const char* gpqmc_last_error(const gpqmc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void gpqmc_destroy(gpqmc_ctx* ctx) {
  if (!ctx) return;
  for (auto& v : ctx->tev)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
  for (int d = 0; d < 2; ++d) {
    if (ctx->graph[d]) (void)hipGraphExecDestroy(ctx->graph[d]);
    if (ctx->graph_def[d]) (void)hipGraphDestroy(ctx->graph_def[d]);
  }
  delete ctx;
}

}  // extern "C"
