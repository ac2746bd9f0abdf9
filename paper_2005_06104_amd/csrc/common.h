// Internal declarations shared by the library's translation units.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <complex>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "tdvp.h"

using zc = std::complex<double>;

struct TdvpError : std::runtime_error {
  tdvp_status code;
  TdvpError(tdvp_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define TDVP_THROW(code, msg) throw TdvpError((code), (msg))
#define HIP_CHECK(x)                                                                        \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess)                                                                  \
      throw TdvpError(TDVP_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));    \
  } while (0)
#define ARG_CHECK(cond, msg)                  \
  do {                                        \
    if (!(cond)) TDVP_THROW(TDVP_ERR_ARG, msg); \
  } while (0)

struct MapCache;
struct tdvp_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  rocblas_handle blas = nullptr;
  tdvp_alloc_fn alloc = nullptr;
  tdvp_free_fn free_ = nullptr;
  void* user = nullptr;
  std::string last_error;
  hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_c = nullptr, ev_d = nullptr;
  // Worker contexts for calls on several independent instances: each owns a
  // stream, a rocBLAS handle and events, and allocates stream-ordered memory
  // (on its own stream, from a pool the parent owns).  Created on first use, kept until the
  // parent is destroyed.
  bool owns_stream = false;
  bool async_alloc = false;
  hipMemPool_t pool = nullptr;          // the pool async allocations come from (workers)
  hipMemPool_t worker_pool = nullptr;   // the parent's own pool for its workers
  std::vector<tdvp_ctx_s*> workers;
  // Split-K partial products of the GEMMs issued for this context: one
  // buffer of SPLIT_WS_BYTES, allocated on first use, freed with the context.
  // Work on the context's stream is ordered, so every product may reuse it.
  static constexpr size_t SPLIT_WS_BYTES = size_t(32) << 20;
  void* split_ws = nullptr;
  void* split_workspace() {
    if (!split_ws) split_ws = dalloc(SPLIT_WS_BYTES);
    return split_ws;
  }
  // Pinned host staging for the small results the host branches on (Lanczos
  // coefficients, eigenvalues, check flags): one DMA copy instead of a staged
  // pageable one.  Allocated on first use, freed with the context.
  static constexpr size_t HSTAGE_BYTES = size_t(64) << 10;
  void* hstage = nullptr;
  // copy `bytes` (<= HSTAGE_BYTES / 2) from device memory, wait, return the host copy
  const void* fetch(const void* dev, size_t bytes);
  // Asynchronous variant into slot k (0 or 1, each HSTAGE_BYTES / 4, apart
  // from fetch's region): stage_async enqueues the copy and returns where it
  // lands; wait_stage(k) blocks until it has.
  hipEvent_t ev_stage[2] = {nullptr, nullptr};
  const void* stage_async(int k, const void* dev, size_t bytes);
  void wait_stage(int k);
  // Slot k written by a kernel instead of a copy: stage_slot_dev(k) is the
  // slot's device address (HSTAGE_BYTES / 4 bytes); after enqueueing the
  // kernel that writes it, stage_mark(k) records the event wait_stage(k)
  // waits for and returns the slot's host address.
  void* hstage_dev = nullptr;
  void ensure_hstage();
  void* stage_slot_dev(int k);
  const void* stage_mark(int k);

  // Uploads of small host arrays without a stream sync: the bytes are copied
  // into one of UP_SLOTS pinned buffers, which the stream then copies to the
  // device; a slot is reused once the event of its previous copy completed.
  // Released (after their copies) by destroy_uploads, before the stream goes.
  static constexpr int UP_SLOTS = 16;
  void* up_buf[UP_SLOTS] = {};
  size_t up_cap[UP_SLOTS] = {};
  hipEvent_t up_ev[UP_SLOTS] = {};
  int up_pos = 0;
  void upload_async(void* dev, const void* host, size_t bytes);
  void destroy_uploads();

  void* dalloc(size_t bytes);
  void dfree(void* p);
  void sync();
  void ensure_workers(int n);
  void destroy_workers();
  // Buffers of other contexts released while this worker context runs an
  // instance: their memory may still be in use on this context's stream, so
  // they are freed (through their own context) only after that stream has
  // been synchronised.
  std::vector<std::pair<tdvp_ctx_s*, void*>> deferred_frees;
  // the block-sparse maps of the products issued on this context (created
  // on first use; destroy_maps() frees them, before the stream goes)
  MapCache* maps = nullptr;
  void destroy_maps();
};

// The worker context the calling host thread runs an instance on (null
// outside worker threads).  Device buffers owned by another context (a
// state's tensors, which the parent context allocated) may be read by work
// still queued on the worker's stream when the worker drops them; the
// parent's allocator does not see that stream, so such buffers are freed
// only after the worker's stream has finished, and a buffer regrown on a
// worker thread is allocated from the worker's own stream-ordered pool.
extern thread_local tdvp_ctx_s* tl_exec_ctx;

// Growable device buffer owned through the context's allocator.
// Named host range of a phase (shown by rocprofv3 --marker-trace; a few
// nanoseconds when no tool listens).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

struct DBuf {
  tdvp_ctx_s* ctx = nullptr;
  void* p = nullptr;
  size_t cap = 0;
  DBuf() = default;
  explicit DBuf(tdvp_ctx_s* c) : ctx(c) {}
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : ctx(o.ctx), p(o.p), cap(o.cap) { o.p = nullptr; o.cap = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); ctx = o.ctx; p = o.p; cap = o.cap; o.p = nullptr; o.cap = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p && ctx) {
      if (tl_exec_ctx && tl_exec_ctx != ctx)
        tl_exec_ctx->deferred_frees.emplace_back(ctx, p);
      else
        ctx->dfree(p);
    }
    p = nullptr;
    cap = 0;
  }
  // Ensure capacity for `bytes`; contents are not preserved on growth.
  void* ensure(size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (bytes > cap) {
      release();
      if (tl_exec_ctx) ctx = tl_exec_ctx;
      p = ctx->dalloc(bytes);
      cap = bytes;
    }
    return p;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ------------------------------------------------------------ kernels API
// All launches are asynchronous on `s`.  Complex arrays are interleaved.
namespace kern {

// C = alpha op(A) op(B) + beta C, row-major, batched with element strides;
// ws (may be NULL) is scratch for split-K partial products.
template <typename T>
void gemm(hipStream_t s, int opa, int opb, int M, int N, int K, zc alpha, const void* A,
          long long lda, long long sa, const void* B, long long ldb, long long sb, zc beta, void* C,
          long long ldc, long long sc, int batch, void* ws = nullptr, size_t ws_bytes = 0);

// Block-sparse map of an M x N x K product whose operands carry U(1)
// charges, as a list of work items, one workgroup each: item (two int4)
// {tile, part, a, b}, {r0, r1, c0, c1} computes rows r0 .. r1 and columns
// c0 .. c1 of output tile `tile` (batch entry outer, then 64 x 64 tiles in
// row-major order) over the K intervals iv[a .. b) ((begin, end) pairs).
// The items are sorted by decreasing K length, so the longest are
// dispatched first and consecutive ones go to different XCDs; device
// arrays.  While set (set_kmap / KMapScope) on the calling host thread, the
// products of that shape and batch count it issues walk only those
// intervals; any other shape is an error.
// Unsplit maps (splits = 1) cover every tile (a sub-block without intervals
// writes alpha * 0 + beta * C).  Split maps (splits > 1) hold the nonempty
// parts only: part s of a sub-block writes its partial product into `part`
// (splits x batch x M x N complex of the product's type, at most
// part_bytes); tinfo (6 per tile: the row and column where the second
// segment starts, the nonempty parts of each of the four sub-blocks) tells
// the reduction which parts to sum.
struct KMap {
  const int4* items = nullptr;
  int n_items = 0;
  const int* iv = nullptr;     // pairs
  int M = 0, N = 0, K = 0;
  int batch = 1;               // batched products: one map per batch entry, batch outer
  int splits = 1;
  const int* tinfo = nullptr;
  void* part = nullptr;
  size_t part_bytes = 0;
  int partial = 0;             // unsplit map without the sub-blocks that share no charge
};
void set_kmap(const KMap* k);
const KMap* current_kmap();
struct KMapScope {
  const KMap* saved;
  explicit KMapScope(const KMap* k) : saved(current_kmap()) { set_kmap(k); }
  ~KMapScope() { set_kmap(saved); }
  KMapScope(const KMapScope&) = delete;
  KMapScope& operator=(const KMapScope&) = delete;
};

// Split-K scratch used by gemm() calls from the calling host thread that
// pass no ws of their own (NULL: none, products run unsplit).
void set_split_workspace(void* p, size_t bytes);
struct SplitWorkspaceScope {
  void* saved_p;
  size_t saved_b;
  SplitWorkspaceScope(void* p, size_t bytes);
  ~SplitWorkspaceScope();
  SplitWorkspaceScope(const SplitWorkspaceScope&) = delete;
  SplitWorkspaceScope& operator=(const SplitWorkspaceScope&) = delete;
};

// The same product (NN, alpha = 1, beta = 0, no batch) as a separate kernel
// instantiation reserved for the one-site effective Hamiltonian.
// ws (may be NULL) is scratch for split-K partial products.
template <typename T>
void gemm_heff(hipStream_t s, int M, int N, int K, const void* A, long long lda, const void* B, long long ldb,
               void* C, long long ldc, void* ws = nullptr, size_t ws_bytes = 0);
// Householder tridiagonalisation of a Hermitian n x n complex128 matrix
// (row-major, full storage; n <= 1024) in one cooperative launch:
// H = Q T Q^H with T real tridiagonal (diagonal D[n], off-diagonal E[n-1]) and
// Q (row-major) unitary.  scratch holds tridiag_scratch_bytes(n); *err is set
// nonzero when a grid barrier wait ran out.  Returns the launch status.
int tridiag_groups(int n);
size_t tridiag_scratch_bytes(int n);
hipError_t tridiag(hipStream_t s, const void* H, int n, void* Q, double* D, double* E, void* scratch, int* err);
// The same for nsec independent matrices (2 <= n <= 1024 each, own scratch
// of tridiag_scratch_bytes(n)), reduced side by side in as few launches as
// fit; *err is shared.
struct TdSector {
  const void* H;
  void* Q;
  double* D;
  double* E;
  void* scratch;
  int n;
};
hipError_t tridiag_batched(hipStream_t s, const TdSector* sec, int nsec, int* err);
// Eigen-decomposition of the real symmetric tridiagonal matrix (diagonal D[n],
// off-diagonal E[n-1]; 1 <= n <= 512) by divide and conquer: on return D holds
// the eigenvalues ascending and Z (column-major n x n) the eigenvectors.
// scratch holds tridiag_eig_scratch_bytes(n).  Returns the launch status.
size_t tridiag_eig_scratch_bytes(int n);
hipError_t tridiag_eig(hipStream_t s, double* D, const double* E, int n, double* Z, void* scratch);
// Several such problems (each n <= 512 with its own scratch) side by side:
// one launch per stage for all of them (results as from tridiag_eig).
// The charge blocks of one block-diagonal Hermitian n x n matrix, handled
// side by side (one launch per step for all blocks): block b holds indices
// idx[off .. off + m) of the matrix; X its m x m work matrix, Z the m x m
// real eigenvectors (column-major, ascending) of its tridiagonal problem, R
// its back-transformed rows.
struct EigBlock {
  double2* X;
  const double* Z;
  double2* R;
  int off, m;
};
// X = (H_b + H_b^H) / 2 for every block
void eig_blocks_gather(hipStream_t s, const EigBlock* blk, int nb, const void* H, long long n, const int* idx);
// X = the rows of Z, descending (as zrows_from_real_desc)
void eig_blocks_rows(hipStream_t s, const EigBlock* blk, int nb);
// sums[b] = sum |R_b|^2 (complex128 slots, imaginary part zero)
void eig_blocks_norms(hipStream_t s, const EigBlock* blk, int nb, void* sums);
// rows[off + i][idx[off + j]] = R_b[i][j] (rows: n x n complex128)
void eig_blocks_scatter(hipStream_t s, const EigBlock* blk, int nb, void* rows, long long n, const int* idx);
struct TdEigJob {
  double* D;
  const double* E;
  int n;
  double* Z;
  void* scratch;
};
hipError_t tridiag_eig_batched(hipStream_t s, const TdEigJob* jobs, int n_jobs);
// Cholesky factorisation G = L L^H of a Hermitian positive definite n x n
// matrix (row-major complex128, the lower blocks read; n <= cholinv_max_n())
// with L^-1, in one cooperative launch: L (may be G itself) receives the
// lower blocks of L, Linv all of L^-1 (zero above the diagonal).  *info
// (device) becomes 0 on success, 1 when a pivot is not positive and finite,
// 2 when a wait ran out.  scratch: cholinv_scratch_bytes().
int cholinv_max_n();
size_t cholinv_scratch_bytes();
hipError_t cholinv(hipStream_t s, const void* G, int n, void* L, void* Linv, int* info, void* scratch);
// The same for the nsec diagonal blocks (rows and columns off[q] ..
// off[q] + size[q], size[q] <= cholinv_max_n()) of a ld x ld matrix, all in
// one launch where they fit (several launches otherwise); entries outside
// the blocks are neither read nor written.  *info is reset first unless
// keep_info.  scratch: cholinv_blocks_scratch_bytes().
size_t cholinv_blocks_scratch_bytes();
hipError_t cholinv_blocks(hipStream_t s, const void* G, int ld, const int* off, const int* size, int nsec, void* L,
                          void* Linv, int* info, void* scratch, bool keep_info = false);
// G <- S - frac * trace(S) * I (Hermitian complex128 n x n; S null: S = G)
void shift_by_trace(hipStream_t s, void* G, int n, double frac, const void* S = nullptr);
// out[j][m] = Z[m][n-1-j] (complex), Z column-major real n x n
void zrows_from_real_desc(hipStream_t s, void* out, const double* Z, int n);
// Arithmetic of the complex64 GEMMs issued from the calling host thread:
// 0 FP32 MFMA; 1 BF16 inputs (rounded to nearest even), FP32 accumulation;
// 2 BF16 three-term split x = hi + lo with FP32 accumulation.
void set_float_mode(int mode);
int float_mode();
struct FloatModeScope {
  int saved;
  explicit FloatModeScope(int mode) : saved(float_mode()) { set_float_mode(mode); }
  ~FloatModeScope() { set_float_mode(saved); }
  FloatModeScope(const FloatModeScope&) = delete;
  FloatModeScope& operator=(const FloatModeScope&) = delete;
};
// complex64 GEMM mode of a tdvp_prec other than TDVP_FP64
inline int float_mode_of(int prec) {
  return prec == TDVP_BF16_FP32ACC ? 1 : prec == TDVP_BF16X3_FP32ACC ? 2 : 0;
}
// Batched NN product (alpha = 1, beta = 0, strides in elements) with the
// one-site effective Hamiltonian's instantiation: with charges, its two
// products run batched over the MPO channel (first) and the physical index
// (second) so that every tile of a batch meets one charge.
template <typename T>
void gemm_heff_batched(hipStream_t s, int M, int N, int K, const void* A, long long lda, long long sa, const void* B,
                       long long ldb, long long sb, void* C, long long ldc, long long sc, int batch);
// Plain NN product with split-K scratch (environments, zero-site H_eff).
template <typename T>
void gemm_nn_ws(hipStream_t s, int M, int N, int K, zc alpha, const void* A, long long lda, const void* B,
                long long ldb, zc beta, void* C, long long ldc, void* ws, size_t ws_bytes);

// Sparse MPO contraction over two channel indices (MPO index, physical index):
// out[p, q, o1, o2] = sum_e val[e] * in[p, q, i1(e), i2(e)] for the CSR rows
// o = o1*2 + o2; all eight strides in elements of the precision.
struct WTable {
  const int* rowptr;      // device, n_out_ch + 1
  const int* col;         // device, in-channel index i1*2 + i2
  const double* val;      // device, complex128 coefficients
  int n_in_ch, n_out_ch;
};
// Charges of the sparse-MPO stage of a charged contraction (device arrays):
// element (p, q) of the stage pairs bra row p (charge ql[p]) with ket column
// q (charge qr[q]); with d = qr[q] - ql[p], input channel c can be nonzero
// only where din[c] == d and output channel o only where dout[o] == d.
struct WCharges {
  const int* ql;
  const int* qr;
  const int* din;
  const int* dout;
  int zeros_kept;   // the outputs that are zero by charge already hold zeros: not stored
};
// wc (may be NULL: dense) skips the loads of inputs that are zero by charge
// and stores zero, without a sum, into the outputs that are (or, with
// zeros_kept, leaves them as they are); the results are those of the dense
// stage on inputs that hold those zeros.
template <typename T>
void wapply(hipStream_t s, const WTable& t, const void* in, void* out, long long nP, long long nQ,
            long long isP, long long isQ, long long is1, long long is2, long long osP,
            long long osQ, long long os1, long long os2, const WCharges* wc = nullptr);

// complex128 vector helpers (n complex elements)
// out[j] = sum_x conj(V[j*ldv + x]) w[x], j < nv (deterministic two-stage
// reduction); without conjugation when conjugate = false
void zdots(hipStream_t s, const void* V, long long ldv, int nv, const void* w, long long n,
           void* partial, int n_partial_blocks, void* out, bool conjugate = true);
int zdots_blocks(long long n);
// w[x] += sign * sum_j c[j] V[j*ldv + x]   (c complex128 on device)
void zcombine(hipStream_t s, void* w, const void* V, long long ldv, int nv, const void* c,
              double sign, long long n);
// out[j] = sum_b partial[b * nv + j] for j < nv (complex128; fixed order)
void zsum_partials(hipStream_t s, const void* partial, int nb, int nv, void* out);
// number of blocks (and of partial sums of |w|^2) of zcombine_p over n entries
int zcombine_norm_blocks(long long n);
// the first stage of zdots alone: partial[b * nv + j] over chunks b < nb
void zdots_partial(hipStream_t s, const void* V, long long ldv, int nv, const void* w, long long n, void* partial,
                   int nb);
// w[x] += sign * sum_j c_j V[j*ldv + x] with c_j = sum_b partial[b * nv + j]
// (zdots_partial's output, summed by every block in the same order; nv <= 64);
// cout (may be null) receives c; npart (may be null) the per-block partial
// sums of |w|^2 (zcombine_norm_blocks(n) entries, for zscale_invnorm)
void zcombine_p(hipStream_t s, void* w, const void* V, long long ldv, int nv, const void* partial, int nb,
                double sign, long long n, void* cout, void* npart);
// dst = a * src (complex scalar a)
void zscale(hipStream_t s, void* dst, const void* src, zc a, long long n);
// precision conversions (complex)
void z2c(hipStream_t s, void* dst, const void* src, long long n);
void c2z(hipStream_t s, void* dst, const void* src, long long n);
// copy a rows x cols block between matrices with leading dims (complex of `esize` bytes)
void copy2d(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long rows,
            long long cols, int esize);
// dst[i*ldd + j] = (mask(i,j) ? src[...] : 0), complex128; mode 0: keep j >= i, mode 1: keep j <= i
void ztri(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long rows,
          long long cols, int mode);
// dst[i*ldd + j] = conj(src[j*lds + i]) (conjugate transpose), complex128
void zconjtrans(hipStream_t s, void* dst, long long ldd, const void* src, long long lds,
                long long rows, long long cols);
// Hermitian part in place: A = (A + A^H)/2, n x n complex128
void zhermitize(hipStream_t s, void* A, long long n);
// A = (S + S^H) / 2 (A may be S), and zero[0 .. nzero) = 0 in the same launch
void zhermitize_to(hipStream_t s, void* A, const void* S, long long n, int* zero = nullptr, int nzero = 0);
// fill complex with value
void zfill(hipStream_t s, void* dst, zc v, long long n, int esize);
// zcombine_p's update, then the partial dot products conj(V[j]) . w of the
// updated w per block (zcombine_norm_blocks(n) x nv, zcombine_p's layout)
void zcombine_dots(hipStream_t s, void* w, const void* V, long long ldv, int nv, const void* partial, int nb,
                   double sign, long long n, void* cout, void* dpart);
// w /= |w| with |w|^2 the sum of the np partial sums left by zcombine_p
// (real parts); out[0] receives |w|^2 (complex128, imaginary part zero).
// With host (a mapped host address), the first block also writes
// host[0 .. ncoef) = coeffs[0 .. ncoef) and host[host_norm_at] = |w|^2.
void zscale_invnorm(hipStream_t s, void* w, const void* partial, int np, void* out, long long n,
                    void* host = nullptr, const void* coeffs = nullptr, int ncoef = 0, int host_norm_at = 0);
// dst[i*ldd + j] = src[r(i)*lds + c(j)] for i < nr, j < nc, with r(i) = ridx[i]
// (ridx null: r(i) = i) and c(j) likewise; complex128, index arrays on the device
void zgather(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, const int* ridx, long long nr,
             const int* cidx, long long nc);
// dst[r(i)*ldd + c(j)] = src[i*lds + j] (other entries of dst untouched), complex128,
// r and c as for zgather
void zscatter(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, const int* ridx, long long nr,
              const int* cidx, long long nc);
// dst[i*ldd + cidx[j]] = src[i*lds + j] (other entries of dst untouched), complex128
void zscatter_cols(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long nr,
                   const int* cidx, long long nc);
// 1 x 1 diagonal blocks of the n x n Hermitian H at indices idx[j]: diag[j] =
// H[idx[j]][idx[j]] and rows[pos[j]][idx[j]] = 1 (their unit eigenvectors)
void zunit_blocks(hipStream_t s, void* diag, const void* H, long long n, const int* idx, const int* pos, int cnt,
                  void* rows);
// E (R x C, complex128 row-major) with E[i][j] seeded pseudo-random (each part
// uniform in [-1, 1), from a counter hash of seed, i and j) where qr[i] ==
// qc[j] and zero elsewhere; charge arrays on the device
void zrandom_blocks(hipStream_t s, void* E, int R, int C, const int* qr, const int* qc, unsigned long long seed);
// Row segments of a dense row-major matrix (leading dimension ld): row r
// holds len[r] entries from column b0[r]; packed, they sit at off[r] ..
// (seg = b0[rows], len[rows], off[rows] on the device).  pack: packed =
// dense segments; unpack: dense segments = packed (other entries untouched).
// Complex of esize 16 (complex128) or 8 (complex64) on either side.
void pack_rows(hipStream_t s, void* packed, int packed_esize, const void* dense, int dense_esize, int rows, long long ld,
               const int* seg, int maxlen);
void unpack_rows(hipStream_t s, void* dense, int dense_esize, const void* packed, int packed_esize, int rows,
                 long long ld, const int* seg, int maxlen);
// per-physical-index scaling of rows of G[(x,s),q]: G *= f[s], complex128
void zscale_phys(hipStream_t s, void* G, long long nx, long long nq, double f0, double f1);
// G = a G + b I (n x n complex128)
void zshift_diag(hipStream_t s, void* G, long long n, double a, double b);
// dst[i*ldd+j] = f[i] * src[i*lds+j] (rows) or f[j] * src[...] (cols); f device doubles
void zscale_rows(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long rows,
                 long long cols, const double* f);
void zscale_cols(hipStream_t s, void* dst, long long ldd, const void* src, long long lds, long long rows,
                 long long cols, const double* f);

}  // namespace kern

// ------------------------------------------------------------ linear algebra (FP64)
// A context's block-sparse maps on the device (engine.h).
struct MapCache;
// C = alpha op(A) op(B) + beta C (complex128, row-major) where the logical
// rows, summed index and columns carry the charges qm, qk, qn (any null, or
// maps null: dense).  With all three, the product walks only the blocks of
// equal charge (the operands' other entries are exact zeros).
void qgemm(tdvp_ctx_s* ctx, MapCache* maps, int opa, int opb, int M, int N, int K, zc alpha, const void* A,
           long long lda, const void* B, long long ldb, zc beta, void* C, long long ldc, const std::vector<int>* qm,
           const std::vector<int>* qk, const std::vector<int>* qn);

namespace la {
// C[rows x cols] row-major = A R with A (rows x k) orthonormal columns, R (k x cols) upper,
// k = min(rows, cols).  work must hold rows*cols complex128.
void qr_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* A, void* R, DBuf& work,
                 DBuf& tau);
// C[rows x cols] = L Q with Q (k x cols) orthonormal rows, L (rows x k).
void lq_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* L, void* Q, DBuf& work,
                 DBuf& tau);
// ||X^H X - I||_F^2 for orthonormal columns (orth_rows = false) or
// ||X X^H - I||_F^2 for orthonormal rows; synchronises; +inf for non-finite.
double orth_defect(tdvp_ctx_s* ctx, const void* X, int rows, int cols, bool orth_rows, DBuf& work);
// C (rows >= cols) = A R by two Cholesky-QR passes, A orthonormal columns,
// R = A^dagger C (cols x cols, not triangular); false (A, R undefined) when
// the Gram matrix is numerically singular or A fails the orthonormality check.
// With q (the charges of the columns, ascending; may be null) the Gram
// matrix is factorised charge block by charge block; with qo (those of the
// rows) and the context's maps as well, every product walks only its charge
// blocks.
bool cholqr2_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* A, void* R, DBuf& work,
                      const void* first = nullptr, const std::vector<int>* q = nullptr,
                      const std::vector<int>* qo = nullptr, MapCache* maps = nullptr);
// C (rows <= cols) = L B with B orthonormal rows, L = C B^dagger (rows x rows);
// q: the charges of the rows, qo those of the columns.
bool cholqr2_rows_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* L, void* B, DBuf& work,
                           const void* first = nullptr, const std::vector<int>* q = nullptr,
                           const std::vector<int>* qo = nullptr, MapCache* maps = nullptr);
// Certifies that the smallest eigenvalue of the Hermitian positive
// semidefinite n x n matrix G exceeds frac * trace(G): the Cholesky
// factorisation of G - (1.01 frac + 4 n u) trace(G) I succeeds (u the unit
// roundoff; the margin covers the rounding of the factorisation).  G is
// overwritten; with src (may be null) the matrix is read from src instead and
// G receives the shifted copy.  Returns NULL when the factorisation fails,
// else that factor
// in the form the Cholesky-QR routines take for their first step (shifted
// Cholesky QR: the shifted factor leaves the first iterate's condition
// number small, and the second step restores orthonormality): L^-1 in Finv
// (n x n) for n <= kern::cholinv_max_n() or, with charges q (ascending) on
// the index, when every charge block fits it, else rocSOLVER's factor in G
// (upper, or lower when `lower`, in the column-major view).
const void* gram_floor_certified(tdvp_ctx_s* ctx, void* G, int n, double frac, bool lower, void* Finv, DBuf& work,
                                 const void* src = nullptr, const std::vector<int>* q = nullptr);
// thin SVD of row-major C (rows x cols): U (rows x k), S (k, host), Vh (k x cols); k = min.
void svd_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* U, std::vector<double>& S,
                  void* Vh, DBuf& work, DBuf& work2);
// eigh of row-major Hermitian H (n x n): eigenvalues descending (host) and the
// matrix of eigenvectors-as-rows-conjugated: rows[j] = v_j^dagger (row-major n x n).
// method: EIGH_AUTO (cooperative tridiagonalisation and tridiagonal divide
// and conquer for 2 <= n <= 512, with rocSOLVER's tridiagonal divide and
// conquer for 512 < n <= 1024, rocSOLVER zheevd otherwise or when the first
// fails validation), EIGH_TRIDIAG (the first only), EIGH_HEEVD (rocSOLVER
// only), EIGH_TRIDIAG_LIB (cooperative tridiagonalisation, rocSOLVER dstedc).
enum { EIGH_AUTO = 0, EIGH_TRIDIAG = 1, EIGH_HEEVD = 2, EIGH_TRIDIAG_LIB = 3 };
void eigh_rows_desc(tdvp_ctx_s* ctx, const void* H, int n, std::vector<double>& lam, void* rows,
                    DBuf& work, int method = EIGH_AUTO);
// eigh_rows_desc for a Hermitian H that is block diagonal under the index
// charges q[0..n) (H[i][j] = 0 whenever q[i] != q[j]; the indices of one
// charge need not be contiguous): each block is decomposed on its own, so
// every eigenvector has a definite charge even where blocks share
// eigenvalues.  lam is descending over all blocks (ties: lower charge
// first), rows[j] the conjugated eigenvector (full length n, zero outside its
// block) and qout[j] its charge.  q empty: eigh_rows_desc, qout cleared.
void eigh_sectors(tdvp_ctx_s* ctx, const void* H, int n, const std::vector<int>& q, std::vector<double>& lam,
                  void* rows, DBuf& work, std::vector<int>& qout);
// Row-space basis of C (rows x cols) for C whose entry (i, j) vanishes unless
// qrow[i] == qcol[j]: per charge, the thin SVD of the nonzero block; Vh
// (min(rows, cols) rows of length cols) receives the right singular vectors
// (zero outside their block) grouped by ascending charge, descending within
// a charge, S their singular values and qout their charges.
void svd_sectors(tdvp_ctx_s* ctx, const void* C, int rows, int cols, const std::vector<int>& qrow,
                 const std::vector<int>& qcol, std::vector<double>& S, void* Vh, std::vector<int>& qout);
// Exact factorisation of C (rows x cols) whose entry (i, j) vanishes unless
// qrow[i] == qcol[j], block by block (Householder, nothing dropped): with
// left = true, C = A R (QR), A rows x k, R k x cols; with left = false,
// C = L B (LQ), L rows x k, B k x cols.  Per charge c the block has
// k_c = min(rows of c, columns of c); the k = sum k_c new indices are grouped
// by ascending charge, their charges go to qk.  X1/X2 receive A, R (or L, B).
int factor_sectors(tdvp_ctx_s* ctx, bool left, const void* C, int rows, int cols, const std::vector<int>& qrow,
                   const std::vector<int>& qcol, DBuf& X1, DBuf& X2, std::vector<int>& qk);
// host: eigenvalues of the small symmetric tridiagonal matrix (diagonal d[n],
// off-diagonal e[0..n-2]; e[n-1] is scratch) by implicit QL, returned in d
// (unordered); each of the nr rows of Zr (nr x n, row-major) is multiplied by
// the eigenvector matrix, so rows of the identity give rows of it.  False when
// an eigenvalue needs more than 60 sweeps.
bool tridiag_ql(double* d, double* e, int n, double* Zr, int nr);
}  // namespace la

// truncation rule (same definition as the oracle's keep_count)
int keep_count(const std::vector<double>& w_desc, double eps, double trace_ref, int cap, int min_keep);
