/*
 * gpqmc.h -- C ABI of the MI355X (gfx950) Gutzwiller-projection PQMC sweep.
 *
 * Method: W.-X. Chang and Z.-X. Li, "Boosting quantum Monte Carlo and
 * alleviating sign problem by Gutzwiller projection", arXiv:2303.13403.
 *
 *   <O> = <psi_T| e^{-Theta H} O e^{-Theta H} |psi_T> / <psi_T| e^{-2 Theta H} |psi_T>
 *   |psi_T> = exp(-g sum_i n_i_up n_i_dn) |psi_N>                 (Method section)
 *   H = -t sum_<ij>,sigma (c^dag c + h.c.) + U sum_i n_i_up n_i_dn  (Eq. 2)
 *   |psi_N>: ground state of H_0 + M_N sum_i eps_i (n_i_up - n_i_dn) (Neel trial,
 *            Hubbard section; eps_i = +1 on sublattice A, -1 on B)
 *
 * The projector exp(-g sum n_up n_dn) is decoupled with one Ising field per
 * site (Eq. 1, used in its exact spin-channel form
 * exp(-x (n_up-1/2)(n_dn-1/2)) = 1/2 e^{-x/4} sum_s e^{c s (n_up - n_dn)},
 * cosh c = e^{x/2}) and becomes two boundary slices, ket slice 0 and bra slice
 * M+1; the Hubbard term is decoupled the same way (x = dtau U) on the M = 2
 * l_half bulk slices, B_l = e^{-dtau K} e^{V(s_l)}.  One sweep is one pass over
 * the M + 2 slices (upward on even sweep indices, downward on odd ones)
 * proposing a flip of every field with the determinant ratio
 * 1 + Delta (1 - G_ii) and Metropolis acceptance on |r_up r_dn|.
 *
 * Conventions of every entry point:
 *  - All functions return a gpqmc_status; no exception or abort crosses the ABI.
 *    After an error, gpqmc_last_error() describes it.
 *  - Host arrays passed in are read during the call and copied; the library
 *    keeps no pointer to them.  Output arrays are caller-owned host buffers.
 *  - Device memory is owned by the caller: gpqmc_workspace_bytes() gives the
 *    size and gpqmc_bind_workspace() hands it over; it must stay allocated and
 *    untouched until gpqmc_destroy().  The library allocates no device memory.
 *  - All device work is enqueued on the HIP stream given at creation, in call
 *    order.  Functions marked "synchronises" wait for that stream.
 *  - A context is not thread-safe; use one context per host thread.
 *  - Matrices are row-major; sites are indexed 0 .. N-1; spin 0 is up, 1 down.
 */
#ifndef GPQMC_H
#define GPQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GPQMC_OK = 0,
  GPQMC_EINVAL = -1,      /* invalid argument (message in gpqmc_last_error) */
  GPQMC_ENOMEM = -2,      /* host allocation failed, or workspace too small */
  GPQMC_EHIP = -3,        /* a HIP runtime call failed */
  GPQMC_EDEGENERATE = -4, /* trial state not unique: single-particle gap below 1e-6 */
  GPQMC_EUNSTABLE = -5,   /* a chain flagged drift, NaN, singular L R or a sign mismatch */
  GPQMC_ESTATE = -6       /* call out of order (e.g. sweep before init_trial) */
} gpqmc_status;

/* GPQMC_FP64: every step in FP64, with the equal-time Green's function kept
 *   in factored form G = 1 - A B^T (A, B of size N x n_sigma; G itself is the
 *   Method section's 1 - R (L R)^{-1} L).  Wrapping G over a slice is then the
 *   propagation of both factors by e^{-+dtau K} e^{+-V} (2 N^2 n_sigma flops
 *   each instead of 2 N^3 per side for the N x N matrix), and the flips of a
 *   delay segment reach the factors by the Woodbury identity.
 * GPQMC_FP64_WRAP: every step in FP64 with G wrapped as an N x N matrix,
 *   e^{-dtau K} G e^{+dtau K}, and the basis propagated separately.
 * GPQMC_MIXED: as GPQMC_FP64_WRAP but the Green's-function work of every slice
 *   (kinetic wrap, delayed flush, submatrix scan) in FP32 on FP32 MFMA with
 *   FP32 accumulation; basis propagation, QR, (L R)^{-1}, the fresh Green's
 *   function, log|det| and sign in FP64.  While sampling the doped 16 x 16
 *   workload its Green's function drifts far beyond 1e-5 relative between
 *   re-stabilisations (the drift flag reports it).
 * GPQMC_MIXED_FP32_BASIS: as GPQMC_MIXED but the basis propagation e^{-dtau K}
 *   e^{V} U also in FP32 (its fresh Green's function carries an error of order
 *   eps_fp32 cond(L R), about 1e-5 on a 12 x 12 lattice). */
typedef enum {
  GPQMC_FP64 = 0,
  GPQMC_MIXED = 1,
  GPQMC_MIXED_FP32_BASIS = 2,
  GPQMC_FP64_WRAP = 3
} gpqmc_precision;

/* GPQMC_MODEL_HUBBARD: the Hubbard model of Eq. 2 with the Gutzwiller-
 *   projected Neel trial (Method section), one HS field per site and slice,
 *   decoupled in the spin channel.
 * GPQMC_MODEL_TV: the spinless t-V model of Eq. 3 ("Repulsive spinless
 *   honeycomb model"), H = K + V sum_b (n_i - 1/2)(n_j - 1/2) over the given
 *   bonds b = (i, j), trial e^{-g sum_b n_i n_j} |psi_C> with |psi_C> the n_up
 *   lowest orbitals of K + Delta_C diag(sublattice) (Delta_C in m_neel).  One
 *   HS field per bond and slice, decoupled in the density channel:
 *   e^{-x (n_i - 1/2)(n_j - 1/2)} = 1/2 e^{-x/4} sum_s e^{c s (n_i - n_j)},
 *   cosh c = e^{x/2}, x = dtau V in the bulk and x = g on the two boundary
 *   slices (exp(-g n_i n_j) equals this up to a constant at fixed particle
 *   number when every site has the same number of bonds).  A bond flip is a
 *   rank-2 change of D_l; its ratio det(1 + Delta_F (1 - G)[F, F]) can be
 *   negative (the weight has a sign).  One species: n_dn = 0, U unused. */
typedef enum {
  GPQMC_MODEL_HUBBARD = 0,
  GPQMC_MODEL_TV = 1
} gpqmc_model;

/* One Markov chain.  All chains of one context must share l_half,
 * stab_interval, delay_rank, precision and model; lattices, fillings and
 * couplings may differ per chain. */
typedef struct {
  int32_t n_sites;            /* N, 1 .. 1024 */
  int32_t n_up, n_dn;         /* particles per spin, 1 .. N */
  const double* hopping;      /* N x N symmetric hopping matrix K (K_ij = -t per bond) */
  const int8_t* sublattice;   /* N signs eps_i (+1 / -1) of the Neel trial */
  const double* trial_potential; /* N extra on-site energies of the trial
                                    Hamiltonian only (NULL = none) */
  double U;                   /* Hubbard repulsion, >= 0 */
  double dtau;                /* Trotter step, > 0 */
  double g;                   /* Gutzwiller parameter, >= 0 */
  double m_neel;              /* Neel order parameter M_N of the trial */
  int32_t l_half;             /* slices per side, Theta / dtau (>= 0) */
  int32_t stab_interval;      /* n_s: slices between QR re-stabilisations (>= 1) */
  int32_t delay_rank;         /* k: sites per segment of the flip scan (1 .. 64); the
                                 accepted flips of all segments of a slice are
                                 applied to G by one delayed update per slice */
  int32_t precision;          /* gpqmc_precision */
  uint64_t seed;              /* Philox key; words (lo32(seed), hi32(seed) ^ tag) */
  uint64_t chain_id;          /* counter word 0 of every draw of this chain */
  int32_t trace;              /* nonzero: record ratios and checkpoint Green's
                                 functions of the last pass (testing; large) */
  int32_t model;              /* gpqmc_model (0 = Hubbard) */
  double V;                   /* t-V: nearest-neighbour repulsion, >= 0 */
  int32_t n_bonds;            /* t-V: number of bonds (HS fields per slice) */
  const int32_t* bonds;       /* t-V: n_bonds x 2 sites (i, j), proposed in this order;
                                 D_l at i takes e^{+c s_b}, at j e^{-c s_b}.  The library
                                 cuts the list into scan segments of at most
                                 delay_rank / 2 consecutive site-disjoint bonds (a
                                 segment ends early where the next bond shares a site;
                                 lists grouped into matchings, such as the three bond
                                 directions of the honeycomb lattice, give full
                                 segments).  No site may have more than 4 bonds.  The t-V model needs
                                 GPQMC_FP64 and an even delay_rank <= 32.  Fields
                                 (gpqmc_set_field / get_field) are then
                                 (l_half * 2 + 2) x n_bonds; records hold (sign, E/N,
                                 (1/n_bonds) sum_b <n_i n_j>, S_CDW = (1/N^2) sum_ij
                                 eps_i eps_j <(n_i - 1/2)(n_j - 1/2)>); gpqmc_logdet and
                                 gpqmc_get_green report spin 0 only. */
} gpqmc_chain_desc;

typedef struct {
  int32_t meas_capacity;      /* measurement records kept per chain (default 4096) */
  int32_t use_graph;          /* capture each pass in a HIP graph (default 1) */
  double drift_tol;           /* relative checkpoint drift (max |G_wrapped - G_fresh|
                                 over max |G_fresh|) above which a chain is flagged
                                 (default 1e-5, the mixed path's stated accuracy,
                                 with an FP32 Green's function; 1e-6 in FP64) */
  int32_t particle_hole;      /* nonzero: the half-filling particle-hole shortcut for
                                 every chain where it is exact (default 0).  Such a
                                 chain propagates, updates and re-stabilises spin up
                                 only; spin down follows per field from
                                 G_dn = 1 - E G_up^T E (E = diag(sublattice)), so its
                                 ratio is r_dn = 1 + Delta_dn G_up,ii, its weight
                                 log|W_dn| = log|W_up| - sum_{l,i} c_l s_{l,i} with the
                                 same sign (c_l: lambda on the boundary slices, alpha
                                 in the bulk), and the measurements use the mirrored
                                 G_dn.  It is exact where the lattice is bipartite
                                 under the sublattice signs (K_ij != 0 only between
                                 opposite signs, zero diagonal), n_up = n_dn = N/2 and
                                 there is no trial potential, so that the Neel trial
                                 of spin down is the particle-hole image of spin up;
                                 it needs the factored engine (GPQMC_FP64) with
                                 delay_rank <= 32.  Other chains run both spins;
                                 gpqmc_chain_info.particle_hole reports which.
                                 Derived from the spin-channel HS decoupling of the
                                 Method section (Eq. 1) and the Neel trial. */
} gpqmc_options;

typedef struct {
  int32_t sign;               /* current sign of W_up W_dn */
  int32_t flags;              /* sticky error bits: 1 drift, 2 NaN, 4 singular L R,
                                 8 sign mismatch, 16 measurement buffer full */
  int32_t n_meas;             /* stored measurement records */
  int32_t sign_mismatch;      /* checkpoints where tracked and recomputed signs differed */
  int32_t sweep;              /* passes done since init_trial */
  float max_drift;            /* max |G_wrapped - G_fresh| over checkpoints */
  float last_drift;
  int64_t accepted, proposed; /* Metropolis counters */
  float max_rel_drift;        /* max over checkpoints of the drift divided by
                                 max |G_fresh| (largest over both spins) */
  float last_rel_drift;
  int32_t particle_hole;      /* 1 if the chain runs the particle-hole shortcut */
  int32_t reserved;
} gpqmc_chain_info;

typedef struct gpqmc_ctx gpqmc_ctx;

/* Create a context for n_chains chains (host only; no device work).
 * Validates the descriptors, builds e^{-+dtau K} and the Neel trial orbitals
 * (lowest n_sigma eigenvectors of K + sigma M_N diag(eps) + diag(trial_potential),
 * Hubbard section) with the library's own symmetric eigensolver, and fixes the
 * workspace layout.  hip_stream is a hipStream_t (NULL = default stream).
 * opts may be NULL.  Errors: EINVAL, EDEGENERATE, ENOMEM. */
gpqmc_status gpqmc_create(int32_t n_chains, const gpqmc_chain_desc* chains,
                          const gpqmc_options* opts, void* hip_stream, gpqmc_ctx** out);

/* Device workspace size in bytes (256-byte aligned start required). */
gpqmc_status gpqmc_workspace_bytes(const gpqmc_ctx* ctx, size_t* bytes);

/* Hand over the caller-owned device workspace; uploads the static matrices
 * (synchronises).  Errors: ENOMEM if bytes is too small, EINVAL if misaligned. */
gpqmc_status gpqmc_bind_workspace(gpqmc_ctx* ctx, void* device_ptr, size_t bytes);

/* Initialise every chain: draw the initial field from Philox (tag 0, counter
 * (chain_id, 0, l, i): s = +1 iff bit 0 of word 0 is set) unless one was set
 * with gpqmc_set_field, build the stack of orthonormal bases of
 * L_p = P^T S_{M+1} ... S_{p+1} downward from the bra, and compute the Green's
 * function G = 1 - R (L R)^{-1} L at position -1.  Resets sweep counters,
 * measurements and flags.  Synchronises.  Errors: ESTATE before bind. */
gpqmc_status gpqmc_init_trial(gpqmc_ctx* ctx);

/* Run n_sweeps passes.  measure != 0 records (sign, E/N, D, S_AFM) at tau = Theta
 * once per pass from the freshly recomputed Green's function.  Enqueue only.
 * Errors: ESTATE before init_trial. */
gpqmc_status gpqmc_sweep(gpqmc_ctx* ctx, int32_t n_sweeps, int32_t measure);

/* Sign-weighted estimates over the stored records of one chain
 * (chain = -1: all chains pooled), error by jackknife over bins of
 * 10 records: energy per site E/N = <s E>/<s> (Eq. 2 with U n_up n_dn),
 * double occupancy <s D>/<s>, average sign <s>, and the staggered spin
 * structure factor S_AFM = (1/N^2) sum_ij eps_i eps_j <S_i . S_j> with the
 * chain's sublattice signs eps (the antiferromagnetic order of the Hubbard
 * study: Eq. 2 and the Results section).  Synchronises.
 * Errors: EINVAL (chain out of range or fewer than 20 records). */
gpqmc_status gpqmc_measure_energy(gpqmc_ctx* ctx, int32_t chain, double* mean, double* err);
gpqmc_status gpqmc_measure_double_occupancy(gpqmc_ctx* ctx, int32_t chain, double* mean,
                                            double* err);
gpqmc_status gpqmc_measure_sign(gpqmc_ctx* ctx, int32_t chain, double* mean, double* err);
gpqmc_status gpqmc_measure_structure_factor(gpqmc_ctx* ctx, int32_t chain, double* mean,
                                            double* err);

/* Raw records of one chain, oldest first, four doubles each: (sign, E/N, D,
 * S_AFM); out holds capacity records (4 * capacity doubles).  *n_out
 * receives the number written (<= capacity).  Synchronises. */
gpqmc_status gpqmc_get_measurements(gpqmc_ctx* ctx, int32_t chain, double* out,
                                    int32_t capacity, int32_t* n_out);

/* Clear the measurement records of every chain (enqueue only). */
gpqmc_status gpqmc_reset_measurements(gpqmc_ctx* ctx);

/* Field of one chain, (M+2) x N int8 (+1 / -1), slice-major.  set_field
 * requires a following gpqmc_init_trial.  Synchronise. */
gpqmc_status gpqmc_set_field(gpqmc_ctx* ctx, int32_t chain, const int8_t* field);
gpqmc_status gpqmc_get_field(gpqmc_ctx* ctx, int32_t chain, int8_t* field);

/* Last freshly recomputed FP64 Green's function G_ij = <c_i c_j^dag> of one
 * chain and spin (N x N): after init_trial or a sweep it is at position -1
 * (after a downward pass) or M+1 (after an upward pass).  Synchronises. */
gpqmc_status gpqmc_get_green(gpqmc_ctx* ctx, int32_t chain, int32_t spin, double* G);

/* Status record of one chain.  Synchronises. */
gpqmc_status gpqmc_get_chain_info(gpqmc_ctx* ctx, int32_t chain, gpqmc_chain_info* info);

/* log|W_sigma| and sgn W_sigma of the last checkpoint of one chain, where
 * W_sigma = det(P_sigma^T S_{M+1} ... S_0 P_sigma) = det(L_p R_p) is the weight
 * of spin sigma at the current field (Method section: the projected overlap
 * whose ratio the flips sample).  It is assembled in FP64 from the
 * accumulated log|det| of the triangular factors of both re-orthonormalised
 * bases and log|det(L R)| of the orthonormal ones.  logabs and sign are
 * caller arrays of two entries (spin up, down).  Valid after init_trial
 * (position -1) and after every pass.  Synchronises.  Errors: EINVAL, ESTATE. */
gpqmc_status gpqmc_logdet(gpqmc_ctx* ctx, int32_t chain, double* logabs, int32_t* sign);

/* Testing hooks (off the hot path).
 * set_debug: bit 0 = reject every proposal (fixed-field parity runs).
 * get_trace: for a chain created with trace != 0, the ratios (r_up, r_dn) of
 * every proposal of the last pass ((M+2) x N x 2, slice-major), the FP64
 * Green's functions at the checkpoints of the last pass (n_ck x 2 x N x N, in
 * pass order) and their drifts (n_ck); any pointer may be NULL.  n_ck is
 * returned in *n_checkpoints.  Synchronises. */
gpqmc_status gpqmc_set_debug(gpqmc_ctx* ctx, int32_t flags);
gpqmc_status gpqmc_get_trace(gpqmc_ctx* ctx, int32_t chain, double* ratios, double* greens,
                             double* drifts, int32_t* n_checkpoints);

/* For a chain created with trace != 0: (log|W_sigma|, sgn W_sigma) of spin
 * up then down at every checkpoint of the last pass, n_ck x 2 x 2 doubles in
 * pass order (see gpqmc_logdet).  Synchronises.  Errors: EINVAL. */
gpqmc_status gpqmc_get_trace_logdet(gpqmc_ctx* ctx, int32_t chain, double* logdets);

/* GEMM self test on caller device memory: C = op(A) B with one of the
 * library's MFMA tile kernels (precision GPQMC_FP64 or GPQMC_MIXED = FP32).
 * flags bit 0: op(A) = A^T (A is K x M); bit 1: the 128 x 128 large-tile
 * kernel of the wrap, slice update and (FP64) basis propagation, in FP32 for
 * GPQMC_MIXED or FP64 for GPQMC_FP64 (requires no transpose).  A M x K
 * row-major (or K x M), B K x N, C M x N.  Synchronises.
 * Errors: EINVAL on bad sizes or an unsupported flag combination. */
gpqmc_status gpqmc_debug_gemm(int32_t precision, int32_t M, int32_t N, int32_t K, int32_t flags,
                              const void* A, int32_t lda, const void* B, int32_t ldb, void* C,
                              int32_t ldc, void* hip_stream);

/* Allocation-free variant of gpqmc_debug_gemm, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight loops, harnesses
 * that forbid hipMalloc): the same C = op(A) B on the same MFMA tile kernels
 * (same arguments, layouts and flags), but the GEMM descriptor lives in a
 * file-scope device array of the library (256 KiB per GPU, held until the
 * process ends) and is written there by a kernel, so the call makes no
 * allocation and no host-to-device copy.  Enqueue only: it returns before the
 * product is done (synchronise hip_stream before reading C).  At most 16352
 * output tiles (64 x 64, or 128 x 128 with the large-tile flag); larger
 * products return GPQMC_EINVAL.  Every call on one GPU uses that GPU's
 * array: calls that overlap on one GPU (other streams or threads) race;
 * calls in order on one stream do not.  Errors: EINVAL (sizes, flags,
 * precision), EHIP. */
gpqmc_status gpqmc_gemm_noalloc(int32_t precision, int32_t M, int32_t N, int32_t K, int32_t flags,
                                const void* A, int32_t lda, const void* B, int32_t ldb, void* C,
                                int32_t ldc, void* hip_stream);

/* Average duration (ms) of one launch of a hot-path kernel for all chains,
 * timed with HIP events on the context's stream over reps back-to-back
 * launches on the chains' current data.  G-wrap engines: kernel 0 = the
 * kinetic-wrap GEMM e^{-dtau K} G (every chain and spin), 1 = the
 * basis-propagation GEMM, 2 = the delayed update of the last slice, G - Xa Ya
 * (its result goes to the wrap scratch, G is left unchanged; meaningful after
 * a sweep).  GPQMC_FP64 (factored): kernel 0 = the propagation of both
 * factors of every chain and spin (into the idle buffers of the ping-pong
 * pairs); kernels 1 and 2 are EINVAL.  Writes only scratch that every pass
 * rebuilds.  Synchronises.  Errors: ESTATE before init_trial, EINVAL. */
gpqmc_status gpqmc_time_kernel(gpqmc_ctx* ctx, int32_t kernel, int32_t reps, float* ms_per_launch);

/* In-sweep kernel timing.  Bit t of mask (0..7) records a HIP event pair on
 * the context's stream around every launch, inside later sweeps, of timed
 * kernel t.  G-wrap engines: 0 = the kinetic-wrap GEMM e^{-dtau K} G of every
 * slice, 1 = the B-scaled basis-propagation GEMM, 2 = the slice's delayed
 * update G <- D (G - Xa Ya) D^{-1}.  GPQMC_FP64 (factored): 0 = the
 * propagation of both factors (one launch per bulk slice), 1 = the segment
 * update of the dual factor Q <- Q - (Q Mf^T) Wf (one per delay segment),
 * 2 = the flip scan (one per delay segment).  While mask is nonzero the
 * passes are launched directly rather than as HIP graphs.  Setting a mask (0
 * included) clears the recorded launches.  Synchronises.  Errors: EINVAL for a
 * mask outside 0..7. */
gpqmc_status gpqmc_set_kernel_timing(gpqmc_ctx* ctx, int32_t mask);

/* Sum of the durations (ms) and the number of the launches of timed kernel
 * kernel (0..2) recorded since the last gpqmc_set_kernel_timing.
 * Synchronises.  Errors: EINVAL. */
gpqmc_status gpqmc_get_kernel_timing(gpqmc_ctx* ctx, int32_t kernel, float* total_ms,
                                     int32_t* launches);

/* Debugging hooks of the G-wrap engines (off the hot path; synchronise;
 * GPQMC_FP64 contexts return EINVAL).  debug_step runs one
 * stage of slice l on every chain: 0 = the flip scan of sites [s0, s1),
 * 1 = appending that segment's factors to the slice's delayed update
 * G - Xa Ya, 2 = applying the delayed update to G (no frame change).
 * debug_read copies at most `count` elements of an internal buffer of one
 * chain and spin as doubles: 0 = G (N x N), 1 = Z (64 x 64), 2 = the
 * accepted sites of the last segment (64), 3 = Ya (N x N), 4 = Xa (N x N),
 * 5 = (accepted count of the last segment, sign, accepted total).  A count
 * beyond the buffer is GPQMC_EINVAL. */
gpqmc_status gpqmc_debug_step(gpqmc_ctx* ctx, int32_t stage, int32_t l, int32_t s0, int32_t s1);
gpqmc_status gpqmc_debug_read(gpqmc_ctx* ctx, int32_t chain, int32_t what, int32_t spin, double* out,
                              int64_t count);

/* Status of one chain: GPQMC_OK or GPQMC_EUNSTABLE if any flag is set.
 * Synchronises. */
gpqmc_status gpqmc_chain_status(gpqmc_ctx* ctx, int32_t chain);

const char* gpqmc_last_error(const gpqmc_ctx* ctx);

/* Release host resources (the caller frees the workspace afterwards). */
void gpqmc_destroy(gpqmc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GPQMC_H */
