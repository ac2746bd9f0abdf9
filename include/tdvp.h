/*
 * tdvp.h -- C-ABI of the GSE-TDVP1 hot path on MI355X (gfx950).
 *
 * Method: Yang & White, "Time dependent variational principle with ancillary
 * Krylov subspace".  One GSE-TDVP1 time step (section I.C) is
 *   1. tdvp_expand_basis: apply the MPO of 1 - i tau H k-1 times to |psi>
 *      (global Krylov vectors, eq. (10), cutoff eps_K) and extend the bond
 *      bases of |psi> by them (state-averaged basis extension, section I.A,
 *      eqs. (5)-(7), cutoff eps_M), ending with the center on the first site;
 *   2. tdvp_sweep: one-site TDVP sweep left to right then right to left
 *      (cutoff eps, used only when unitarity is not required).
 * tdvp_measure returns energy, norm, <S^z_i>, bond dimensions and overlaps.
 *
 * Conventions fixed at this boundary
 *   - spin 1/2, local dimension d = 2, basis order {up, down};
 *   - operator codes: 0 = identity, 1 = S^+, 2 = S^-, 3 = S^z;
 *   - complex numbers are interleaved (re, im) pairs: complex128 = 2 doubles,
 *     complex64 = 2 floats; every array is row-major (last index fastest);
 *   - site tensors M[a, s, b]: left bond a, physical s, right bond b;
 *   - MPO tensors W[alpha, beta, s', s] (s' is the output index);
 *   - left environment L[a', alpha, a] (a' on the bra side);
 *   - right environment, stored transposed, Rt[beta, b, b'] (b' on the bra side);
 *   - time steps are complex: a step evolves exp(-i H dt); imaginary time
 *     uses dt = -i dtau.
 *
 * Ownership: input arrays are copied, the caller keeps them.  Handles own
 * their device memory and are freed by *_destroy.  Outputs go to
 * caller-provided buffers; nothing returns pointers into internal memory.
 * A context is bound to one device and one HIP stream and is not thread-safe.
 *
 * Errors: every call returns a tdvp_status and never throws.  The message of
 * the last failure is kept per context (tdvp_last_error).  Arguments are
 * checked before any state is changed, so TDVP_ERR_ARG leaves every handle as
 * it was.  A device or numeric failure in the middle of a call marks the
 * handles it was changing invalid; later use returns TDVP_ERR_STATE.
 * Device pointers passed to the kernel-level calls must hold at least the
 * stated number of elements; they are not checked.
 */
#ifndef TDVP_H_
#define TDVP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdvp_ctx_s* tdvp_ctx;
typedef struct tdvp_mpo_s* tdvp_mpo;
typedef struct tdvp_mps_s* tdvp_mps;

typedef enum {
  TDVP_OK = 0,
  TDVP_ERR_ARG = 1,      /* invalid argument; nothing was changed          */
  TDVP_ERR_ALLOC = 2,    /* device allocation failed or above a stated cap */
  TDVP_ERR_DEVICE = 3,   /* HIP / rocSOLVER runtime error                  */
  TDVP_ERR_NOCONV = 4,   /* Lanczos hit krylov_max in strict mode          */
  TDVP_ERR_NUMERIC = 5,  /* NaN/Inf or a failed factorisation              */
  TDVP_ERR_STATE = 6     /* handle invalidated by an earlier failure       */
} tdvp_status;

/* Precision of the contractions (environments, effective Hamiltonians, MPO
 * application).  Lanczos recurrences, reorthogonalisation, the tridiagonal
 * exponential, QR/SVD/eigh and the stored site tensors are always FP64.
 *   TDVP_FP32            complex64 operands, FP32 MFMA;
 *   TDVP_BF16_FP32ACC    complex64 operands rounded to BF16 (nearest even) as
 *                        they enter the matrix cores, FP32 accumulation;
 *   TDVP_BF16X3_FP32ACC  each FP32 operand split into two BF16 terms
 *                        x = hi + lo, products ah*bh + ah*bl + al*bh with FP32
 *                        accumulation (about 16 significant bits).
 * All three keep the environments and intermediates in complex64. */
typedef enum {
  TDVP_FP64 = 0,
  TDVP_FP32 = 1,
  TDVP_BF16_FP32ACC = 2,
  TDVP_BF16X3_FP32ACC = 3
} tdvp_prec;

/* GEMM operand modes: N = as stored, T = transposed, C = conjugate transpose,
 * R = conjugated (not transposed). */
typedef enum { TDVP_OP_N = 0, TDVP_OP_T = 1, TDVP_OP_C = 2, TDVP_OP_R = 3 } tdvp_op;

/* How an MPO is applied to an MPS (section I.C offers both): the
 * density-matrix algorithm (exact before the cut; cost O(m^3 w^2 d) per
 * site) or variational two-site fitting (Paeckel et al. 2019; O(m^3 w d) per
 * site and pass, converged after a few passes). */
typedef enum { TDVP_APPLY_DENMAT = 0, TDVP_APPLY_FIT = 1 } tdvp_apply_method;

/* Device memory callbacks (e.g. PyTorch's caching allocator).  alloc returns
 * NULL on failure; memory freed by free_ may be reused by later work on the
 * context's stream only.  Both may be NULL: the library then uses hipMalloc
 * and hipFree. */
typedef void* (*tdvp_alloc_fn)(size_t bytes, void* user);
typedef void (*tdvp_free_fn)(void* ptr, void* user);

/* ---------------------------------------------------------------- context */

/* Bind a context to `device` and the HIP stream `hip_stream` (NULL = the
 * default stream).  All work of the context is issued on that stream. */
tdvp_status tdvp_ctx_create(int device, void* hip_stream, tdvp_alloc_fn alloc, tdvp_free_fn free_,
                            void* user, tdvp_ctx* out);
void tdvp_ctx_destroy(tdvp_ctx ctx);
/* Message of the last failure on this context ("" if none).  Valid until the
 * next call on the context. */
const char* tdvp_last_error(tdvp_ctx ctx);
/* Library version string. */
const char* tdvp_version(void);

/* -------------------------------------------------------------------- MPO */

/* One Hamiltonian term: coef * op_i(site_i) op_j(site_j); site_j = -1 gives
 * the one-site term coef * op_i(site_i).  Sites are 0-based path positions. */
typedef struct {
  int32_t site_i, site_j;
  int32_t op_i, op_j;
  double re, im;
} tdvp_term;

/* Build the MPO of c0 * 1 + c1 * H for H = sum of `terms` on n_sites sites
 * (section I.C step 1: 1 - i tau H is c0 = 1, c1 = -i tau).  The MPO is a
 * finite-state automaton (start / open channels / done) in which open
 * channels with identical pending futures are merged, which is exact.
 * w_out (may be NULL) receives the n_sites + 1 MPO bond dimensions.
 * Errors: TDVP_ERR_ARG for n_sites < 1, a site out of range, site_i ==
 * site_j, or an operator code outside 0..3. */
tdvp_status tdvp_create_mpo(tdvp_ctx ctx, int n_sites, const tdvp_term* terms, int n_terms,
                            double c0_re, double c0_im, double c1_re, double c1_im,
                            tdvp_mpo* out, int* w_out);
/* Copy the MPO tensors to host: concatenated W_i (w_i x w_{i+1} x 2 x 2
 * complex128), `capacity` in doubles.  Returns TDVP_ERR_ARG if too small.
 * Host-only: needs no GPU. */
tdvp_status tdvp_mpo_to_host(tdvp_mpo mpo, double* out, size_t capacity);
/* Host-only MPO construction for checking the builder without a device:
 * same arguments as tdvp_create_mpo minus the context; fills dims[n_sites+1]
 * and, if `out` is not NULL, the tensors as in tdvp_mpo_to_host. */
tdvp_status tdvp_build_mpo_host(int n_sites, const tdvp_term* terms, int n_terms, double c0_re,
                                double c0_im, double c1_re, double c1_im, int* dims, double* out,
                                size_t capacity);
/* Host only: *conserves = 1 if the MPO of c0 * 1 + c1 * H conserves S^z,
 * i.e. its channels carry charges qw with every nonzero W[al,be,s',s]
 * satisfying qw(be) = qw(al) + q(s') - q(s) (q(up) = 1, q(down) = -1) and
 * qw = 0 on both ends; charges (may be NULL, capacity in ints) then
 * receives qw for the n_sites + 1 bonds. */
tdvp_status tdvp_mpo_charges_host(int n_sites, const tdvp_term* terms, int n_terms, double c0_re,
                                  double c0_im, double c1_re, double c1_im, int* conserves,
                                  int* charges, size_t capacity);
void tdvp_mpo_destroy(tdvp_mpo mpo);

/* -------------------------------------------------------------------- MPS */

/* Upload an MPS: bond_dims has n_sites + 1 entries (first and last 1);
 * tensors are the concatenated site tensors M_i[a,s,b] in complex128.
 * charges (may be NULL: no symmetry) gives a U(1) charge to every bond
 * index, concatenated over the n_sites + 1 bonds (sum of bond_dims
 * entries), ascending within each bond: twice the S^z of everything left
 * of the bond, so M_i[a,s,b] may be nonzero only where q(b) = q(a) + 1 for
 * s = up and q(a) - 1 for s = down.  Such a state conserves S^z under an
 * MPO that does (a Hamiltonian of the benchmarks of section II), and every
 * later call keeps it block-sparse: factorisations run charge by charge and
 * new bonds carry the charges of their states.
 * Errors: TDVP_ERR_ARG for inconsistent sizes, non-finite entries, charges
 * not ascending within a bond, or a nonzero entry outside the blocks. */
tdvp_status tdvp_mps_from_host(tdvp_ctx ctx, int n_sites, const int* bond_dims,
                               const double* tensors, const int* charges, tdvp_mps* out);
/* *has_charges = 1 if the state carries U(1) charges; charges (may be NULL)
 * receives them as in tdvp_mps_from_host, for the current bonds (capacity
 * in ints). */
tdvp_status tdvp_mps_charges(tdvp_mps mps, int* has_charges, int* charges, size_t capacity);
/* Number of sites and current bond dims (n_sites + 1 entries). */
tdvp_status tdvp_mps_bond_dims(tdvp_mps mps, int* n_sites, int* bond_dims, int capacity);
/* Download the tensors (layout as in tdvp_mps_from_host); capacity in doubles. */
tdvp_status tdvp_mps_to_host(tdvp_mps mps, double* tensors, size_t capacity);
void tdvp_mps_destroy(tdvp_mps mps);

/* *out = O|in>, normalised and truncated (section I.C, the MPO application
 * that produces each global Krylov vector of eq. (10)).
 *   method  TDVP_APPLY_DENMAT: density-matrix algorithm, one left-to-right
 *           pass over reduced density matrices built from right double-layer
 *           environments; the cut drops the smallest eigenvalues while their
 *           sum stays <= eps * Tr(rho).
 *           TDVP_APPLY_FIT: two-site variational fitting, `passes` >= 1
 *           alternating passes with |in> as the first guess, the last pass
 *           from left to right (odd counts start from the left, even counts
 *           from the right); each two-site tensor is the exact projection of O|in> in
 *           the current bases, split by a truncated decomposition with the
 *           same relative cut (eps on the squared singular values).
 *   chi_max caps every bond.  Both methods compute in FP64.
 * The result is a new MPS (release with tdvp_mps_destroy), left-canonical
 * with its centre on the last site; `in` is left unchanged.  *discarded (may
 * be NULL) receives the weight dropped by the cut (the last pass for FIT).
 * Errors: TDVP_ERR_ARG (NULL handle, site counts differ, eps < 0,
 * chi_max < 1, unknown method, passes < 1 or fewer than two sites for FIT),
 * TDVP_ERR_NUMERIC (zero or non-finite result). */
tdvp_status tdvp_apply_mpo(tdvp_ctx ctx, tdvp_mps in, tdvp_mpo op, int method, double eps, int chi_max,
                           int passes, tdvp_mps* out, double* discarded);

/* ------------------------------------------------------- GSE-TDVP1 step */

typedef struct {
  int k;             /* Krylov order: k-1 global Krylov vectors (k >= 1)           */
  double eps_K;      /* Krylov-vector cutoff (relative discarded weight)            */
  double eps_M;      /* cutoff on states added by the extension (relative to
                        sum_l |C~_l|^2)                                             */
  int chi_max;       /* cap on every bond (Krylov vectors and extended psi)         */
  int prec;          /* tdvp_prec of the MPO applications' contractions (either
                        route); their factorisations and the extension stay FP64  */
  int skip_if_full;  /* 1: skip steps 1-2 when every bond is already at its largest
                        useful size min(chi_max, 2^(i+1), 2^(N-i-1))                */
  int apply_method;  /* tdvp_apply_method of the Krylov vectors (0: density matrix) */
  int fit_passes;    /* passes of TDVP_APPLY_FIT (values < 1 mean 1)                */
} tdvp_expand_params;

typedef struct {
  double ms_krylov, ms_extend;   /* wall time of the two stages               */
  int n_added;                   /* states added over all bonds               */
  int max_bond;                  /* largest bond after the extension          */
  int krylov_max_bond;           /* largest bond of any Krylov vector         */
  int skipped;                   /* 1 if the expansion was skipped            */
  double discarded_K;            /* total discarded weight of the MPO applications */
} tdvp_expand_stats;

/* Steps 1-2 of GSE-TDVP1 for n independent states psi[0..n-1], each with its
 * own MPO op[j] = 1 - i tau H.  On return every psi[j] is right-canonical
 * with its center on site 0 and represents the same state as before (up to
 * rounding).  stats may be NULL, else n entries.
 * Errors: TDVP_ERR_ARG (n < 1, site counts differ from the MPO, k < 1,
 * chi_max < 1, eps < 0, unknown prec or apply_method, fewer than two sites
 * with TDVP_APPLY_FIT, the same state twice in psi[], a state with charges
 * and an MPO that does not conserve S^z). */
tdvp_status tdvp_expand_basis(tdvp_ctx ctx, int n, tdvp_mps* psi, const tdvp_mpo* op,
                              const tdvp_expand_params* params, tdvp_expand_stats* stats);

typedef struct {
  double dt_re, dt_im;   /* the sweep evolves exp(-i H dt); imaginary dtau: dt = -i dtau */
  double eps;            /* gauge-move cutoff (0 = exact moves, unitary)                  */
  int chi_max;           /* cap on bonds when eps > 0 (tdvp_sweep with eps = 0 never
                            truncates, whatever the bonds; tdvp_sweep2 caps its
                            two-site splits at chi_max also when eps = 0)                 */
  double krylov_tol;     /* Lanczos stop: beta_j |c_j| <= tol |c|                          */
  int krylov_max;        /* at most this many Lanczos vectors (<= 64)                      */
  int prec;              /* tdvp_prec of the contractions                                  */
  int normalize;         /* renormalise after every local step (imaginary time)            */
  int strict;            /* 1: reaching krylov_max is TDVP_ERR_NOCONV                      */
} tdvp_sweep_params;

typedef struct {
  double ms;                 /* wall time of the sweep                                    */
  double ms_matvec;          /* device time of the one-site H_eff applications            */
  double flops_matvec;       /* algorithmic flops of those applications (8 per complex MAC,
                                nonzero MPO entries only)                                */
  long long n_matvec;        /* one-site H_eff applications                               */
  long long n_keff;          /* zero-site K_eff applications                              */
  int max_lanczos;           /* largest Lanczos dimension used                            */
  int n_unconverged;         /* local steps that reached krylov_max                       */
  double discarded;          /* weight dropped at gauge moves (eps > 0)                   */
  double energy;             /* <C|H_eff|C>/<C|C> at site 0 after the sweep                */
  double ms_heff_gemm;       /* device time of the two GEMM launches of each H_eff application */
  double flops_heff_gemm;    /* algorithmic flops of those GEMM launches                        */
  long long n_heff_gemm;     /* number of those GEMM launches                                   */
} tdvp_sweep_stats;

/* Step 3 of GSE-TDVP1: one symmetric one-site TDVP sweep (left to right by
 * dt/2 per site, right to left by dt/2; the last site takes dt at once).
 * Precondition: center at site 0, sites 1..N-1 right-canonical (the state
 * tdvp_expand_basis leaves).  Postcondition: the same gauge.
 * Errors: TDVP_ERR_ARG (bad parameters, MPO/MPS mismatch, the same state
 * twice in psi[], a state with charges and an MPO that does not conserve
 * S^z), TDVP_ERR_NOCONV (strict mode: some local Lanczos run
 * reached krylov_max; the sweep was completed with those unconverged local
 * results, every state stays valid and stats are filled in),
 * TDVP_ERR_NUMERIC (non-finite values). */
tdvp_status tdvp_sweep(tdvp_ctx ctx, int n, tdvp_mps* psi, const tdvp_mpo* H,
                       const tdvp_sweep_params* params, tdvp_sweep_stats* stats);

/* Caller-owned result arrays; pointer fields may be NULL to skip. */
typedef struct {
  double energy;        /* <psi|H|psi>/<psi|psi> (when H is given)       */
  double norm;          /* sqrt(<psi|psi>)                                */
  double overlap_re, overlap_im;  /* <other|psi> (when other is given)    */
  double* sz;           /* n_sites entries: <S^z_i>                       */
  int* bond_dims;       /* n_sites + 1 entries                            */
} tdvp_observables;

/* One symmetric two-site TDVP sweep on psi[j], j < n: the conventional
 * method with which the cost statement closing section I.C and the
 * benchmarks of section II compare GSE-TDVP1.  Left to right over the site
 * pairs with dt/2 each (the last pair once by dt), right to left with dt/2;
 * each pair is split by the truncated gauge move (discarded weight <= eps
 * times its norm squared, at most chi_max kept; with eps = 0 only zero
 * weights and the chi_max cap cut) and the new one-site center is evolved
 * backwards by dt/2.  Parameters and statistics as for tdvp_sweep (n_keff
 * counts the backward one-site matvecs); same pre- and postcondition; needs
 * n_sites >= 2.  No tdvp_expand_basis is needed before it. */
tdvp_status tdvp_sweep2(tdvp_ctx ctx, int n, tdvp_mps* psi, const tdvp_mpo* H,
                        const tdvp_sweep_params* params, tdvp_sweep_stats* stats);

/* Measure psi[j] (any gauge) for j < n; H and other may be NULL (then n
 * entries each when given).  The observables are those the benchmarks of
 * section II report: the energy <H> (section II.A: its convergence in
 * imaginary time; section II.B: its conservation in real time, relative
 * error below 1e-10), the local magnetisations, the norm, the bond
 * dimensions, and the overlap <other|psi> from which fidelities follow.  Any
 * MPO may be passed as H, e.g. the total-spin moments of eqs. (13)-(15).
 * Errors: TDVP_ERR_ARG (NULL handles, H or other with another site count),
 * TDVP_ERR_STATE (an invalidated handle). */
tdvp_status tdvp_measure(tdvp_ctx ctx, int n, const tdvp_mps* psi, const tdvp_mpo* H,
                         const tdvp_mps* other, tdvp_observables* out);

/* Spin-squeezing parameter of eq. (14) in the closed form of eq. (15), from
 * measured total-spin moments (host only, needs no device): with
 * V_aa = <(S^a)^2> - <S^a>^2 and V_yz = <S^y S^z + S^z S^y>/2 - <S^y><S^z>,
 * the smallest variance in the y-z plane is
 * v = (V_yy + V_zz - sqrt((V_yy - V_zz)^2 + 4 V_yz^2)) / 2 and
 * *xi2 = n_spins * v / <S^x>^2 (the mean spin points along x, as in the
 * one-axis-twisting benchmark of section II.B).  Arguments: the first
 * moments sx, sy, sz, the second moments syy = <(S^y)^2>, szz = <(S^z)^2>,
 * and syz_sym = <S^y S^z + S^z S^y>.
 * Errors: TDVP_ERR_ARG for n_spins < 1, NULL xi2, non-finite moments or
 * sx = 0. */
tdvp_status tdvp_squeezing_xi2(int n_spins, double sx, double sy, double sz, double syy, double szz,
                               double syz_sym, double* xi2);

/* ---------------------------------------------------- kernel-level calls
 * Device pointers, complex in the precision `prec` (complex128 or complex64),
 * issued on the context's stream, asynchronous. */

/* Batched complex GEMM C = alpha op(A) op(B) + beta C (row-major), batch
 * strides in elements; op(A) is M x K, op(B) is K x N. */
tdvp_status tdvp_gemm(tdvp_ctx ctx, int prec, int op_a, int op_b, int M, int N, int K,
                      double alpha_re, double alpha_im, const void* A, long long lda,
                      long long stride_a, const void* B, long long ldb, long long stride_b,
                      double beta_re, double beta_im, void* C, long long ldc, long long stride_c,
                      int batch);

/* One-site effective Hamiltonian (the one-site TDVP local generator):
 * Y[a',s',b'] = sum L[a',al,a] W[al,be,s',s] C[a,s,b] Rt[be,b,b'].
 * Sizes: L ml*wl*ml, Rt wr*mr*mr, C and Y ml*2*mr; W_host is a host array of
 * wl*wr*4 complex128.  workspace may be NULL (allocated internally) or hold
 * (4*max(wl,wr) + 32)*ml*mr elements of the precision (intermediates and
 * split-K partial products). */
tdvp_status tdvp_heff_apply(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr,
                            const double* W_host, const void* L, const void* Rt, const void* C,
                            void* Y, void* workspace);

/* tdvp_heff_apply for tensors that carry U(1) S^z charges (the block-sparse
 * products a charged sweep issues): charges_l[ml] on the bond of a and a',
 * charges_r[mr] on the bond of b and b', channel charges qw_l[wl] and
 * qw_r[wr] of the MPO bonds (host int32 arrays; physical charge +1 for s = 0,
 * -1 for s = 1).  Nonzero entries are allowed only where L[a',al,a] has
 * q(a) = q(a') - q_w(al), C[a,s,b] has q(b) = q(a) + q(s), Rt[be,b,b'] has
 * q(b) = q(b') - q_w(be) and W[al,be,s',s] has q(s) - q_w(al) = q(s') -
 * q_w(be); L, C and Rt must hold zeros elsewhere (the products read some of
 * those entries where the blocks' K ranges are joined).  Y is written in
 * full, zeros outside its blocks.  The products walk the nonzero blocks
 * only and the sparse-MPO stage reads by charge.  Workspace allocated
 * internally; synchronous.  Errors: TDVP_ERR_ARG as tdvp_heff_apply, for
 * NULL charge arrays, or for a nonzero W entry that breaks the rule above. */
tdvp_status tdvp_heff_apply_u1(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr, const double* W_host,
                               const int32_t* charges_l, const int32_t* charges_r, const int32_t* qw_l,
                               const int32_t* qw_r, const void* L, const void* Rt, const void* C, void* Y);

/* tdvp_heff_apply for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels on the same operands, with every piece of
 * scratch (the MPO's CSR tables, the two intermediates and the split-K
 * partial products) in one statically sized device array of 64 MiB that each
 * GPU holds from the library's load until the process ends; nothing is
 * allocated and no workspace is passed.  Sizes whose scratch,
 * (4 max(wl, wr) + 32) ml mr elements of the precision plus the tables,
 * exceeds 64 MiB are rejected with TDVP_ERR_ARG before any work.  Every call
 * on one GPU uses the same array, which keeps the last call's contents:
 * calls that overlap on one GPU (from several threads or streams) race.
 * Returns once the MPO tables are in the array (they are copied from host
 * memory: the call waits for the context's stream); the contraction itself
 * runs asynchronously on that stream.  Arguments and layouts as
 * tdvp_heff_apply. */
tdvp_status tdvp_heff_apply_noalloc(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr,
                                    const double* W_host, const void* L, const void* Rt,
                                    const void* C, void* Y);

/* Zero-site effective Hamiltonian on the bond: Y[a',b'] = sum L[a',al,a] X[a,b] Rt[al,b,b'].
 * Sizes: L ml*w*ml, Rt w*mr*mr, X and Y ml*mr; workspace as for tdvp_heff_apply. */
tdvp_status tdvp_keff_apply(tdvp_ctx ctx, int prec, int ml, int w, int mr, const void* L,
                            const void* Rt, const void* X, void* Y, void* workspace);

/* Environment updates.  Left: Lout[b',be,b] = sum conj(A[a',s',b']) L[a',al,a]
 * W[al,be,s',s] A[a,s,b] (A is ml x 2 x mr, L ml*wl*ml, Lout mr*wr*mr).
 * Right: Rout[al,a,a'] = sum B[a,s,b] W[al,be,s',s] Rt[be,b,b'] conj(B[a',s',b'])
 * (B is ml x 2 x mr, Rt wr*mr*mr, Rout wl*ml*ml).  workspace as for tdvp_heff_apply. */
tdvp_status tdvp_env_left(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr,
                          const double* W_host, const void* L, const void* A, void* Lout,
                          void* workspace);
tdvp_status tdvp_env_right(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr,
                           const double* W_host, const void* Rt, const void* B, void* Rout,
                           void* workspace);

/* Hermitian eigendecomposition used by the truncations, the density-matrix
 * truncation of the MPO application and the basis extension (section I.A:
 * the eigendecomposition of the mixed density matrix; section I.B: of the
 * reduced density matrices).  H: device complex128 n x n row-major Hermitian
 * (only its Hermitian part is used); rows: device complex128 n x n out, row j
 * is the conjugated eigenvector v_j^dagger for the j-th largest eigenvalue;
 * lam: host double[n] out, descending.  method: 0 automatic (cooperative
 * tridiagonalisation and tridiagonal divide and conquer for 2 <= n <= 512,
 * the same reduction with rocSOLVER's tridiagonal divide and conquer for
 * 512 < n <= 1024, rocSOLVER zheevd otherwise or when the first fails its
 * check), 1 the
 * first only (TDVP_ERR_NUMERIC when not applicable), 2 rocSOLVER zheevd
 * only, 3 cooperative tridiagonalisation with rocSOLVER's tridiagonal divide
 * and conquer (TDVP_ERR_NUMERIC when not applicable).  Synchronous. */
tdvp_status tdvp_eigh(tdvp_ctx ctx, int method, int n, const void* H, void* rows, double* lam);

/* Eigendecomposition of a Hermitian matrix that is block diagonal under U(1)
 * index charges, as the charged states' gauge moves, density matrices and
 * the state-averaged mixed density matrix of section I.A need it (every
 * kept state with a definite charge): H[i][j] = 0 unless charges[i] ==
 * charges[j] (the indices of one charge need not be contiguous); each
 * block is decomposed on its own (all blocks of 2 .. 512 indices side by
 * side, larger ones by rocSOLVER's tridiagonal divide and conquer up to
 * 1024, zheevd above).  H: device complex128 n x n row-major; charges: host
 * int32[n]; rows: device complex128 n x n out, row j the conjugated
 * eigenvector (zero outside its block); lam: host double[n] out, descending
 * over all blocks (ties: lower charge first); charges_out: host int32[n]
 * out, the charge of eigenvector j.  Synchronous.  Errors: TDVP_ERR_ARG for
 * n < 1 or NULL pointers, TDVP_ERR_NUMERIC when a block's decomposition
 * fails its checks on every route. */
tdvp_status tdvp_eigh_sectors(tdvp_ctx ctx, int n, const void* H, const int32_t* charges, void* rows,
                              double* lam, int32_t* charges_out);

/* Cholesky factorisation with the inverse of the factor, as used by the gauge
 * moves (the orthonormal centre moves of eq. (3) and of the sweep, section
 * I.C item 3: the Cholesky-QR steps and the test that a truncation has
 * nothing to cut): G = L L^H for a Hermitian positive definite G.  G: device
 * complex128 n x n row-major, its lower triangle read, 1 <= n <= 512; L,
 * Linv: device complex128 n x n row-major out, L lower triangular (the
 * entries above the diagonal in the 16 x 16 blocks off the diagonal are not
 * written; those of the diagonal blocks are set to zero), Linv = L^-1 with
 * zeros above the diagonal.  L may be G; Linv must overlap neither.  info:
 * host out, 0 on success, 1 when a pivot is not positive and finite (G not
 * numerically positive definite; L and Linv are then undefined), 2 when an
 * internal wait ran out.  Synchronous. */
tdvp_status tdvp_cholesky(tdvp_ctx ctx, int n, const void* G, void* L, void* Linv, int* info);

/* Wait for all work issued on the context's stream. */
tdvp_status tdvp_synchronize(tdvp_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* TDVP_H_ */
