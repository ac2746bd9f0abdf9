// FP64 factorisations for gauge moves, truncations and density-matrix
// diagonalisation, on rocSOLVER.  The library stores matrices row-major,
// rocSOLVER is column-major: a row-major R x C buffer is the column-major
// C x R matrix X = M^T.  Each routine below factors X and reads the factors
// of M = X^T straight out of the rocSOLVER buffers:
//   QR of M  = LQ of X:  X = Lx Qx  ->  M = Qx^T Lx^T   (A = Qx^T, R = Lx^T)
//   LQ of M  = QR of X:  X = Qx Rx  ->  M = Rx^T Qx^T   (L = Rx^T, Q = Qx^T)
//   SVD of M: X = U' S V'^H  ->  M = conj(V') S U'^T, and the row-major
//            reading of the V'^H buffer is conj(V'), of the U' buffer U'^T.
//   eigh of Hermitian M: X = conj(M); its eigenvectors are conj(v_j), stored
//            as columns, so row j of the row-major reading is v_j^dagger.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>

#include "common.h"
#include "engine.h"

namespace {

using rz = rocblas_double_complex;

void blas_check(rocblas_status st, const char* what) {
  if (st != rocblas_status_success)
    TDVP_THROW(TDVP_ERR_DEVICE, std::string(what) + " failed with rocblas status " + std::to_string((int)st));
}

int read_info(tdvp_ctx_s* ctx, const int* dinfo, const char* what) {
  int info = 0;
  HIP_CHECK(hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  if (info != 0) TDVP_THROW(TDVP_ERR_NUMERIC, std::string(what) + " reported info = " + std::to_string(info));
  return info;
}

}  // namespace

namespace la {

void qr_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* A, void* R, DBuf& work,
                 DBuf& tau) {
  const int k = std::min(rows, cols);
  rz* X = static_cast<rz*>(work.ensure(sizeof(rz) * (size_t)rows * cols));
  rz* t = static_cast<rz*>(tau.ensure(sizeof(rz) * (size_t)std::max(k, 1)));
  HIP_CHECK(hipMemcpyAsync(X, C, sizeof(rz) * (size_t)rows * cols, hipMemcpyDeviceToDevice, ctx->stream));
  blas_check(rocsolver_zgelqf(ctx->blas, cols, rows, X, cols, t), "zgelqf");
  kern::ztri(ctx->stream, R, cols, X, cols, k, cols, 0);
  blas_check(rocsolver_zunglq(ctx->blas, k, rows, k, X, cols, t), "zunglq");
  kern::copy2d(ctx->stream, A, k, X, cols, rows, k, 16);
}

void lq_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* L, void* Q, DBuf& work,
                 DBuf& tau) {
  const int k = std::min(rows, cols);
  rz* X = static_cast<rz*>(work.ensure(sizeof(rz) * (size_t)rows * cols));
  rz* t = static_cast<rz*>(tau.ensure(sizeof(rz) * (size_t)std::max(k, 1)));
  HIP_CHECK(hipMemcpyAsync(X, C, sizeof(rz) * (size_t)rows * cols, hipMemcpyDeviceToDevice, ctx->stream));
  blas_check(rocsolver_zgeqrf(ctx->blas, cols, rows, X, cols, t), "zgeqrf");
  kern::ztri(ctx->stream, L, k, X, cols, rows, k, 1);
  blas_check(rocsolver_zungqr(ctx->blas, cols, k, k, X, cols, t), "zungqr");
  kern::copy2d(ctx->stream, Q, cols, X, cols, k, cols, 16);
}

// qr_rowmajor for rows >= cols with the whole orthonormal factor: Af (rows x
// rows), its first cols columns are qr_rowmajor's A, the rest an
// orthonormal completion; R (cols x cols).
void qr_rowmajor_full(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* Af, void* R, DBuf& tau) {
  rz* Y = static_cast<rz*>(Af);   // col-major rows x rows, lda = rows
  rz* t = static_cast<rz*>(tau.ensure(sizeof(rz) * (size_t)std::max(cols, 1)));
  kern::copy2d(ctx->stream, Y, rows, C, cols, rows, cols, 16);
  blas_check(rocsolver_zgelqf(ctx->blas, cols, rows, Y, rows, t), "zgelqf");
  kern::ztri(ctx->stream, R, cols, Y, rows, cols, cols, 0);
  blas_check(rocsolver_zunglq(ctx->blas, rows, rows, cols, Y, rows, t), "zunglq");
}

// lq_rowmajor for rows <= cols with the whole orthonormal factor: Bf (cols x
// cols), its first rows rows are lq_rowmajor's Q, the rest an orthonormal
// completion; L (rows x rows).
void lq_rowmajor_full(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* L, void* Bf, DBuf& tau) {
  rz* Y = static_cast<rz*>(Bf);   // col-major cols x cols, lda = cols
  rz* t = static_cast<rz*>(tau.ensure(sizeof(rz) * (size_t)std::max(rows, 1)));
  kern::copy2d(ctx->stream, Y, cols, C, cols, rows, cols, 16);
  blas_check(rocsolver_zgeqrf(ctx->blas, cols, rows, Y, cols, t), "zgeqrf");
  kern::ztri(ctx->stream, L, rows, Y, cols, rows, rows, 1);
  blas_check(rocsolver_zungqr(ctx->blas, cols, cols, rows, Y, cols, t), "zungqr");
}

double orth_defect(tdvp_ctx_s* ctx, const void* X, int rows, int cols, bool orth_rows, DBuf& work) {
  // ||X^H X - I||_F^2 (orthonormal columns) or ||X X^H - I||_F^2 (rows)
  const int n = orth_rows ? rows : cols;
  const size_t nn = (size_t)n * n;
  const int nb = kern::zdots_blocks((long long)nn);
  rz* G = static_cast<rz*>(work.ensure(sizeof(rz) * (nn + (size_t)nb + 2)));
  rz* dpart = G + nn;
  rz* dsum = dpart + nb;
  hipStream_t s = ctx->stream;
  if (orth_rows)
    kern::gemm<double>(s, TDVP_OP_N, TDVP_OP_C, n, n, cols, 1.0, X, cols, 0, X, cols, 0, 0.0, G, n, 0, 1);
  else
    kern::gemm<double>(s, TDVP_OP_C, TDVP_OP_N, n, n, rows, 1.0, X, cols, 0, X, cols, 0, 0.0, G, n, 0, 1);
  kern::zshift_diag(s, G, n, 1.0, -1.0);
  kern::zdots(s, G, (long long)nn, 1, G, (long long)nn, dpart, nb, dsum);
  const zc dev = *static_cast<const zc*>(ctx->fetch(dsum, sizeof(rz)));
  return std::isfinite(dev.real()) ? dev.real() : HUGE_VAL;
}

namespace {

// One Cholesky factorisation for a Cholesky-QR step: n <= kern::cholinv_max_n()
// uses the cooperative factorisation with the inverse (L in place of G,
// L^-1 in Finv; the step is then a GEMM), larger n rocSOLVER zpotrf in place
// (the step a triangular solve; `lower` selects the factor the row variant
// needs).  *dinfo (device) is 0 on success.
// With charges q (ascending) on the Gram matrix's index, the matrix is block
// diagonal (entries between different charges are exact zeros), and the
// factorisation runs block by block in one launch when every block fits the
// cooperative kernel: L^-1 is then block diagonal too.
struct CholBlocks {
  std::vector<int> off, size;
  bool use = false;
};

CholBlocks chol_blocks(int n, const std::vector<int>* q) {
  CholBlocks b;
  if (!q || (int)q->size() != n || n < 1 || !std::is_sorted(q->begin(), q->end())) return b;
  for (int i = 0; i < n;) {
    int e = i + 1;
    while (e < n && (*q)[e] == (*q)[i]) ++e;
    if (e - i > kern::cholinv_max_n()) return CholBlocks{};
    b.off.push_back(i);
    b.size.push_back(e - i);
    i = e;
  }
  b.use = b.off.size() > 1 || n <= kern::cholinv_max_n();
  return b;
}

bool own_chol(int n, const std::vector<int>* q = nullptr) {
  return n <= kern::cholinv_max_n() || chol_blocks(n, q).use;
}

void chol_factor(tdvp_ctx_s* ctx, rz* G, int n, rz* Finv, int* dinfo, void* cscr, bool lower,
                 const std::vector<int>* q = nullptr) {
  const CholBlocks cb = chol_blocks(n, q);
  if (cb.use && cb.off.size() > 1) {
    kern::zfill(ctx->stream, Finv, zc(0.0, 0.0), (long long)n * n, 16);   // the blocks between sectors
    if (kern::cholinv_blocks(ctx->stream, G, n, cb.off.data(), cb.size.data(), (int)cb.off.size(), G, Finv, dinfo,
                             cscr) != hipSuccess) {
      (void)hipGetLastError();
      TDVP_THROW(TDVP_ERR_DEVICE, "Cholesky factorisation launch failed");
    }
  } else if (own_chol(n)) {
    if (kern::cholinv(ctx->stream, G, n, G, Finv, dinfo, cscr) != hipSuccess) {
      (void)hipGetLastError();
      TDVP_THROW(TDVP_ERR_DEVICE, "Cholesky factorisation launch failed");
    }
  } else {
    blas_check(rocsolver_zpotrf(ctx->blas, lower ? rocblas_fill_lower : rocblas_fill_upper, n, G, n, dinfo),
               "zpotrf");
  }
}

}  // namespace

const void* gram_floor_certified(tdvp_ctx_s* ctx, void* G, int n, double frac, bool lower, void* Finv, DBuf& work,
                                 const void* src, const std::vector<int>* q) {
  if (n < 1) return nullptr;
  char* base = static_cast<char*>(work.ensure(256 + kern::cholinv_blocks_scratch_bytes()));
  int* dinfo = reinterpret_cast<int*>(base);
  kern::shift_by_trace(ctx->stream, G, n, frac * 1.01 + 4.0 * n * 2.220446049250313e-16, src);
  // (row-major G read column-major is conj(G): definite exactly when G is)
  chol_factor(ctx, static_cast<rz*>(G), n, static_cast<rz*>(Finv), dinfo, base + 256, lower, q);
  if (*static_cast<const int*>(ctx->fetch(dinfo, sizeof(int))) != 0) return nullptr;
  return own_chol(n, q) ? Finv : G;
}

// Cholesky QR in two steps (after CholeskyQR2: Yamamoto, Nakatsukasa,
// Yanagisawa and Fukaya, 2015): X <- X R^-1 with X^H X = R^H R restores
// orthonormality to ~u cond(C)^2, and a second step to rounding when
// cond(C) < ~1e7.  The second step is chosen by the measured defect
// delta = ||X^H X - I||_F of the first: none when delta <= 1e-10; Newton-
// Schulz steps X <- X (I - (X^H X - I) / 2) when delta < 1/4 (each squares
// the defect; GEMMs only, the number of steps set from delta); a second
// Cholesky step otherwise.  A row-major n x n Gram matrix read column-major
// is its conjugate M; potrf gives M = U^H U, so R = conj(U) and the
// row-major solve X R = Y is, column-major, U^H X^T = Y^T.  The result is
// accepted when the factorisations succeed and ||A^H A - I||_F <= 1e-10; the
// caller then factors by Householder QR.  `first` (may be NULL) is a factor
// to use in the first step instead of the Cholesky factor of the Gram
// matrix (the shifted factor of gram_floor_certified).
namespace {

int ns_steps(double dev) {   // dev = delta^2; steps until delta^(2^s) <= 1e-11
  const double d = std::sqrt(dev);
  int st = 1;
  for (double x = d * d; x > 1e-11 && st < 6; x *= x) ++st;
  return st;
}

struct CqrSpace {
  rz* G;
  rz* dpart;
  rz* dsum;
  int* dinfo;
  rz* T;
  rz* Finv;
  void* cscr;
  int nb;
};

CqrSpace cqr_space(DBuf& work, int n, long long mat) {
  const size_t nn = (size_t)n * n;
  const int nb = kern::zdots_blocks((long long)nn);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t oG = 0, oP = oG + up(sizeof(rz) * nn), oT = oP + up(sizeof(rz) * ((size_t)nb + 2)),
               oF = oT + up(sizeof(rz) * (size_t)mat), oS = oF + up(sizeof(rz) * nn),
               tot = oS + up(kern::cholinv_blocks_scratch_bytes());
  char* base = static_cast<char*>(work.ensure(tot));
  CqrSpace c;
  c.G = reinterpret_cast<rz*>(base + oG);
  c.dpart = reinterpret_cast<rz*>(base + oP);
  c.dsum = c.dpart + nb;
  c.dinfo = reinterpret_cast<int*>(c.dsum + 1);
  c.T = reinterpret_cast<rz*>(base + oT);
  c.Finv = reinterpret_cast<rz*>(base + oF);
  c.cscr = base + oS;
  c.nb = nb;
  return c;
}

// ||G - I||_F^2 with G <- G - I, and the factorisation flag; one download
double defect(tdvp_ctx_s* ctx, const CqrSpace& c, int n, int* info) {
  const size_t nn = (size_t)n * n;
  kern::zshift_diag(ctx->stream, c.G, n, 1.0, -1.0);
  kern::zdots(ctx->stream, c.G, (long long)nn, 1, c.G, (long long)nn, c.dpart, c.nb, c.dsum);
  const char* hs = static_cast<const char*>(ctx->fetch(c.dsum, sizeof(rz) + sizeof(int)));
  zc dev;
  std::memcpy(&dev, hs, sizeof(rz));
  std::memcpy(info, hs + sizeof(rz), sizeof(int));
  return std::isfinite(dev.real()) ? dev.real() : HUGE_VAL;
}

}  // namespace

bool cholqr2_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* A, void* R, DBuf& work,
                      const void* first, const std::vector<int>* q, const std::vector<int>* qo, MapCache* maps) {
  if (cols < 1 || rows < cols) return false;
  const int n = cols;
  const CqrSpace c = cqr_space(work, n, (long long)rows * n);
  hipStream_t s = ctx->stream;
  const bool own = own_chol(n, q);
  rz* const X = static_cast<rz*>(A);
  const rz* Cz = static_cast<const rz*>(C);
  // the current iterate: C itself before the first step, then X or c.T (the
  // steps with the own factor are GEMMs that write the other buffer)
  const rz* cur = Cz;
  auto other = [&] { return cur == X ? c.T : X; };
  const rz one{1.0, 0.0};
  auto gram = [&] { qgemm(ctx, maps, TDVP_OP_C, TDVP_OP_N, n, n, rows, 1.0, cur, n, cur, n, 0.0, c.G, n, q, qo, q); };
  // X <- X R^-1 with X^H X = R^H R: X (L^-1)^H by a GEMM with the own factor,
  // a triangular solve in place with rocSOLVER's
  auto chol_step = [&](const rz* F) {
    if (own) {
      rz* dst = other();
      qgemm(ctx, maps, TDVP_OP_N, TDVP_OP_C, rows, n, n, 1.0, cur, n, F, n, 0.0, dst, n, qo, q, q);
      cur = dst;
    } else {
      if (cur != X) {
        HIP_CHECK(hipMemcpyAsync(X, cur, sizeof(rz) * (size_t)rows * n, hipMemcpyDeviceToDevice, s));
        cur = X;
      }
      blas_check(rocblas_ztrsm(ctx->blas, rocblas_side_left, rocblas_fill_upper,
                               rocblas_operation_conjugate_transpose, rocblas_diagonal_non_unit, n, rows, &one, F, n,
                               X, n),
                 "ztrsm");
    }
  };
  auto factor = [&]() -> const rz* {
    chol_factor(ctx, c.G, n, c.Finv, c.dinfo, c.cscr, false, q);
    return own ? c.Finv : c.G;
  };
  if (first) {
    kern::zfill(s, c.dinfo, zc(0.0, 0.0), 1, 16);   // no factorisation here sets it
    chol_step(static_cast<const rz*>(first));
  } else {
    gram();
    chol_step(factor());
  }
  int info = 0;
  gram();
  double dev = defect(ctx, c, n, &info);
  if (info != 0) return false;
  if (dev > 1e-20 && dev < 0.0625) {
    // Newton-Schulz: X <- X (I - D / 2) with D = X^H X - I (in c.G)
    const int st = ns_steps(dev);
    for (int k = 0; k < st; ++k) {
      kern::zshift_diag(s, c.G, n, -0.5, 1.0);
      rz* dst = other();
      qgemm(ctx, maps, TDVP_OP_N, TDVP_OP_N, rows, n, n, 1.0, cur, n, c.G, n, 0.0, dst, n, qo, q, q);
      cur = dst;
      gram();
      if (k + 1 < st) kern::zshift_diag(s, c.G, n, 1.0, -1.0);
    }
    dev = defect(ctx, c, n, &info);
  }
  if (dev > 1e-20) {
    // a second Cholesky step (G holds X^H X - I)
    kern::zshift_diag(s, c.G, n, 1.0, 1.0);
    chol_step(factor());
    gram();
    dev = defect(ctx, c, n, &info);
    if (info != 0 || !(dev <= 1e-20)) return false;
  }
  if (cur != X) HIP_CHECK(hipMemcpyAsync(X, cur, sizeof(rz) * (size_t)rows * n, hipMemcpyDeviceToDevice, s));
  qgemm(ctx, maps, TDVP_OP_C, TDVP_OP_N, n, n, rows, 1.0, X, n, C, n, 0.0, R, n, q, qo, q);
  return true;
}

// The same for orthonormal rows (rows <= cols): C = L B, C C^H = L L^H; the
// row-major Gram read column-major is M = Lc Lc^H with L = conj(Lc), and
// B = L^-1 C is, column-major, B^T Lc^H = C^T; Newton-Schulz steps are
// B <- (I - (B B^H - I) / 2) B.
bool cholqr2_rows_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* L, void* B, DBuf& work,
                           const void* first, const std::vector<int>* q, const std::vector<int>* qo,
                           MapCache* maps) {
  if (rows < 1 || cols < rows) return false;
  const int n = rows;
  const CqrSpace c = cqr_space(work, n, (long long)n * cols);
  hipStream_t s = ctx->stream;
  const bool own = own_chol(n, q);
  rz* const X = static_cast<rz*>(B);
  const rz* Cz = static_cast<const rz*>(C);
  const rz* cur = Cz;
  auto other = [&] { return cur == X ? c.T : X; };
  const rz one{1.0, 0.0};
  auto gram = [&] {
    qgemm(ctx, maps, TDVP_OP_N, TDVP_OP_C, n, n, cols, 1.0, cur, cols, cur, cols, 0.0, c.G, n, q, qo, q);
  };
  // X <- L^-1 X with X X^H = L L^H: a GEMM with the own factor's inverse, a
  // triangular solve in place with rocSOLVER's
  auto chol_step = [&](const rz* F) {
    if (own) {
      rz* dst = other();
      qgemm(ctx, maps, TDVP_OP_N, TDVP_OP_N, n, cols, n, 1.0, F, n, cur, cols, 0.0, dst, cols, q, q, qo);
      cur = dst;
    } else {
      if (cur != X) {
        HIP_CHECK(hipMemcpyAsync(X, cur, sizeof(rz) * (size_t)n * cols, hipMemcpyDeviceToDevice, s));
        cur = X;
      }
      blas_check(rocblas_ztrsm(ctx->blas, rocblas_side_right, rocblas_fill_lower,
                               rocblas_operation_conjugate_transpose, rocblas_diagonal_non_unit, cols, n, &one, F, n,
                               X, cols),
                 "ztrsm");
    }
  };
  auto factor = [&]() -> const rz* {
    chol_factor(ctx, c.G, n, c.Finv, c.dinfo, c.cscr, true, q);
    return own ? c.Finv : c.G;
  };
  if (first) {
    kern::zfill(s, c.dinfo, zc(0.0, 0.0), 1, 16);   // no factorisation here sets it
    chol_step(static_cast<const rz*>(first));
  } else {
    gram();
    chol_step(factor());
  }
  int info = 0;
  gram();
  double dev = defect(ctx, c, n, &info);
  if (info != 0) return false;
  if (dev > 1e-20 && dev < 0.0625) {
    const int st = ns_steps(dev);
    for (int k = 0; k < st; ++k) {
      kern::zshift_diag(s, c.G, n, -0.5, 1.0);
      rz* dst = other();
      qgemm(ctx, maps, TDVP_OP_N, TDVP_OP_N, n, cols, n, 1.0, c.G, n, cur, cols, 0.0, dst, cols, q, q, qo);
      cur = dst;
      gram();
      if (k + 1 < st) kern::zshift_diag(s, c.G, n, 1.0, -1.0);
    }
    dev = defect(ctx, c, n, &info);
  }
  if (dev > 1e-20) {
    kern::zshift_diag(s, c.G, n, 1.0, 1.0);
    chol_step(factor());
    gram();
    dev = defect(ctx, c, n, &info);
    if (info != 0 || !(dev <= 1e-20)) return false;
  }
  if (cur != X) HIP_CHECK(hipMemcpyAsync(X, cur, sizeof(rz) * (size_t)n * cols, hipMemcpyDeviceToDevice, s));
  qgemm(ctx, maps, TDVP_OP_N, TDVP_OP_C, n, n, cols, 1.0, C, cols, X, cols, 0.0, L, n, q, qo, q);
  return true;
}

void svd_rowmajor(tdvp_ctx_s* ctx, const void* C, int rows, int cols, void* U, std::vector<double>& S,
                  void* Vh, DBuf& work, DBuf& work2) {
  // one-sided Jacobi SVD (accurate small singular values; far faster than the
  // bidiagonalisation route on this device for these sizes)
  const int k = std::min(rows, cols);
  const size_t nx = (size_t)rows * cols;
  char* base = static_cast<char*>(work.ensure(sizeof(rz) * nx + sizeof(double) * ((size_t)k + 8) + 64));
  rz* X = reinterpret_cast<rz*>(base);
  double* dS = reinterpret_cast<double*>(base + sizeof(rz) * nx);
  double* dres = dS + k + 1;
  int* dinfo = reinterpret_cast<int*>(dres + 2);
  int* dsweeps = dinfo + 2;
  HIP_CHECK(hipMemcpyAsync(X, C, sizeof(rz) * nx, hipMemcpyDeviceToDevice, ctx->stream));
  (void)work2;
  const rocblas_svect lv = Vh ? rocblas_svect_singular : rocblas_svect_none;
  const rocblas_svect rv = U ? rocblas_svect_singular : rocblas_svect_none;
  // X is cols x rows (column-major, lda = cols); its left vectors (cols x k,
  // ldu = cols) are Vh row-major, its V^H (k x rows, ldv = k) is U row-major.
  blas_check(rocsolver_zgesvdj(ctx->blas, lv, rv, cols, rows, X, cols, 0.0, dres, 100, dsweeps, dS,
                               static_cast<rz*>(Vh), cols, static_cast<rz*>(U), k, dinfo),
             "zgesvdj");
  S.resize(k);
  HIP_CHECK(hipMemcpyAsync(S.data(), dS, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
  read_info(ctx, dinfo, "zgesvdj");
}

// Householder tridiagonalisation in one cooperative launch (Q accumulated),
// tridiagonal divide and conquer, rows = Z^T Q^H by one GEMM.  Returns false
// (and leaves `rows` undefined) when the launch is not possible or the result
// fails validation, so that the caller can use the rocSOLVER route.
bool eigh_rows_desc_tridiag(tdvp_ctx_s* ctx, const void* H, int n, std::vector<double>& lam, void* rows,
                            DBuf& work, bool lib_tridiagonal) {
  const int G = kern::tridiag_groups(n);
  if (n < 2 || G == 0) return false;
  const size_t nn = (size_t)n * n;
  const int nb = kern::zdots_blocks((long long)nn);
  const size_t scr = std::max(kern::tridiag_scratch_bytes(n), kern::tridiag_eig_scratch_bytes(n));
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  // layout (256-byte aligned parts): X | Q | partial sums | staged block | E | scratch | Z
  // staged block (one download): sum |v|^2 (complex), info, barrier error, D[n]
  const size_t stage_bytes = sizeof(rz) + 4 * sizeof(int) + sizeof(double) * (size_t)n;
  char* base = static_cast<char*>(work.ensure(up(sizeof(rz) * nn) * 2 + up(sizeof(rz) * (size_t)nb) +
                                              up(stage_bytes) + up(sizeof(double) * (size_t)n) + up(scr) +
                                              up(sizeof(double) * nn)));
  char* p = base;
  auto take = [&](size_t b) {
    char* q = p;
    p += up(b);
    return q;
  };
  rz* X = reinterpret_cast<rz*>(take(sizeof(rz) * nn));
  rz* Q = reinterpret_cast<rz*>(take(sizeof(rz) * nn));
  rz* dpart = reinterpret_cast<rz*>(take(sizeof(rz) * (size_t)nb));
  char* stage = take(stage_bytes);
  rz* dsum = reinterpret_cast<rz*>(stage);
  int* dinfo = reinterpret_cast<int*>(stage + sizeof(rz));
  int* derr = dinfo + 2;
  double* dD = reinterpret_cast<double*>(stage + sizeof(rz) + 4 * sizeof(int));
  double* dE = reinterpret_cast<double*>(take(sizeof(double) * (size_t)n));
  char* scratch = take(scr);
  double* Z = reinterpret_cast<double*>(take(sizeof(double) * nn));
  // Hermitian part, and the info and barrier-error words cleared
  kern::zhermitize_to(ctx->stream, X, H, n, dinfo, 4);
  const hipError_t le = kern::tridiag(ctx->stream, X, n, Q, dD, dE, scratch, derr);
  if (le != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  // the own divide and conquer takes n <= 512; above, rocSOLVER's
  if (lib_tridiagonal || kern::tridiag_eig_scratch_bytes(n) == 0) {
    blas_check(rocsolver_dstedc(ctx->blas, rocblas_evect_tridiagonal, n, dD, dE, Z, n, dinfo), "dstedc");
  } else if (kern::tridiag_eig(ctx->stream, dD, dE, n, Z, scratch) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  kern::zrows_from_real_desc(ctx->stream, X, Z, n);
  kern::gemm<double>(ctx->stream, TDVP_OP_N, TDVP_OP_C, n, n, n, 1.0, X, n, 0, Q, n, 0, 0.0, rows, n, 0, 1);
  kern::zdots(ctx->stream, static_cast<const rz*>(rows), (long long)nn, 1, static_cast<const rz*>(rows), (long long)nn,
              dpart, nb, dsum);
  const char* hs = static_cast<const char*>(ctx->fetch(stage, stage_bytes));
  zc vsum;
  int flags[2];
  std::memcpy(&vsum, hs, sizeof(rz));
  std::memcpy(&flags[0], hs + sizeof(rz), sizeof(int));
  std::memcpy(&flags[1], hs + sizeof(rz) + 2 * sizeof(int), sizeof(int));
  const double* asc = reinterpret_cast<const double*>(hs + sizeof(rz) + 4 * sizeof(int));
  bool ok = flags[0] == 0 && flags[1] == 0 && std::isfinite(vsum.real()) && std::fabs(vsum.real() - n) <= 1e-6 * n;
  for (int j = 0; j < n; ++j) ok = ok && std::isfinite(asc[j]);
  if (!ok) return false;
  lam.resize(n);
  for (int j = 0; j < n; ++j) lam[j] = asc[n - 1 - j];
  return true;
}

void eigh_rows_desc_heevd(tdvp_ctx_s* ctx, const void* H, int n, std::vector<double>& lam, void* rows, DBuf& work) {
  const size_t nn = (size_t)n * n;
  const int nb = kern::zdots_blocks((long long)nn);
  char* base = static_cast<char*>(work.ensure(sizeof(rz) * nn + sizeof(double) * (2 * (size_t)n + 8) +
                                              sizeof(rz) * ((size_t)nb + 2) + 128));
  // layout (16-byte aligned complex first): X | partial sums | sum | D | E | info, sweeps
  rz* X = reinterpret_cast<rz*>(base);
  rz* dpart = X + nn;
  rz* dsum = dpart + nb;
  double* dD = reinterpret_cast<double*>(dsum + 1);
  double* dE = dD + n + 1;
  double* dres = dE + n + 1;
  int* dinfo = reinterpret_cast<int*>(dres + 2);
  int* dsweeps = dinfo + 1;
  kern::zhermitize_to(ctx->stream, X, H, n);
  blas_check(rocsolver_zheevd(ctx->blas, rocblas_evect_original, rocblas_fill_upper, n, X, n, dD, dE, dinfo),
             "zheevd");
  // validate: orthonormal eigenvectors have sum |v|^2 = n, eigenvalues finite
  kern::zdots(ctx->stream, X, (long long)nn, 1, X, (long long)nn, dpart, nb, dsum);
  int info = 0;
  zc vsum;
  HIP_CHECK(hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_CHECK(hipMemcpyAsync(&vsum, dsum, sizeof(rz), hipMemcpyDeviceToHost, ctx->stream));
  std::vector<double> asc(n);
  HIP_CHECK(hipMemcpyAsync(asc.data(), dD, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  bool ok = info == 0 && std::isfinite(vsum.real()) && std::fabs(vsum.real() - n) <= 1e-6 * n;
  for (double v : asc) ok = ok && std::isfinite(v);
  if (!ok) {
    // divide and conquer failed (no convergence, or a non-finite result):
    // check the input, then use the Jacobi eigensolver on a fresh copy
    std::vector<double> h(2 * nn);
    HIP_CHECK(hipMemcpyAsync(h.data(), H, sizeof(rz) * nn, hipMemcpyDeviceToHost, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    bool zero = true;
    for (double v : h) {
      if (!std::isfinite(v)) TDVP_THROW(TDVP_ERR_NUMERIC, "eigh: non-finite input matrix (n = " + std::to_string(n) + ")");
      zero = zero && v == 0.0;
    }
    if (zero) {   // the library routes do not converge on the zero matrix: V = I, all eigenvalues 0
      kern::zfill(ctx->stream, rows, zc(0.0, 0.0), (long long)nn, 16);
      kern::zshift_diag(ctx->stream, rows, n, 1.0, 1.0);
      lam.assign(n, 0.0);
      return;
    }
    kern::zhermitize_to(ctx->stream, X, H, n);
    blas_check(rocsolver_zheevj(ctx->blas, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_upper, n, X,
                                n, 0.0, dres, 100, dsweeps, dD, dinfo),
               "zheevj");
    read_info(ctx, dinfo, "zheevj");
  }
  // ascending -> descending: output row j is input row n-1-j
  kern::copy2d(ctx->stream, rows, n, X + (size_t)(n - 1) * n, -(long long)n, n, n, 16);
  if (!ok) {
    HIP_CHECK(hipMemcpyAsync(asc.data(), dD, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
  }
  lam.resize(n);
  for (int j = 0; j < n; ++j) lam[j] = asc[n - 1 - j];
}

void eigh_rows_desc(tdvp_ctx_s* ctx, const void* H, int n, std::vector<double>& lam, void* rows, DBuf& work,
                    int method) {
  // the cooperative reduction is at least as fast as the library route for
  // every size it supports (n <= 1024)
  const bool try_tridiag = method == EIGH_TRIDIAG || method == EIGH_AUTO || method == EIGH_TRIDIAG_LIB;
  if (try_tridiag && eigh_rows_desc_tridiag(ctx, H, n, lam, rows, work, method == EIGH_TRIDIAG_LIB)) return;
  if (method == EIGH_TRIDIAG || method == EIGH_TRIDIAG_LIB)
    TDVP_THROW(TDVP_ERR_NUMERIC, "cooperative tridiagonal eigensolver not applicable");
  eigh_rows_desc_heevd(ctx, H, n, lam, rows, work);
}

namespace {

// index lists of each charge, in ascending charge order
struct Sectors {
  std::vector<int> charge, off, idx;   // sector c holds idx[off[c] .. off[c+1])
};

Sectors group_by_charge(const std::vector<int>& q) {
  std::map<int, std::vector<int>> m;
  for (int i = 0; i < (int)q.size(); ++i) m[q[i]].push_back(i);
  Sectors s;
  for (auto& kv : m) {
    s.charge.push_back(kv.first);
    s.off.push_back((int)s.idx.size());
    s.idx.insert(s.idx.end(), kv.second.begin(), kv.second.end());
  }
  s.off.push_back((int)s.idx.size());
  return s;
}

// host ints to the device (waits: `v` may be temporary)
int* upload_ints(tdvp_ctx_s* ctx, DBuf& buf, const std::vector<int>& v) {
  buf.ensure(sizeof(int) * std::max<size_t>(1, v.size()));
  ctx->upload_async(buf.p, v.data(), sizeof(int) * v.size());   // staged: v may go at once
  return buf.as<int>();
}

// The charge blocks (2 <= size <= 1024) of a block-diagonal Hermitian
// matrix, all at once: every block gathered, all tridiagonalised side by
// side (kern::tridiag_batched), each tridiagonal problem by the own divide
// and conquer (rocSOLVER's above 512), the back transformations, and one
// download for the checks of all blocks.  Block b (indices idx[off[b] ..
// off[b] + nb[b]) of H) leaves its eigenvector rows, descending, scattered
// into rows off[b] .. of `sec` (n wide) and its eigenvalues in lam[off[b] ..].
// Returns false for the blocks that fail (bad[b] = 1): the caller redoes them.
bool eigh_blocks(tdvp_ctx_s* ctx, const void* H, int n, const int* didx, const std::vector<int>& off,
                 const std::vector<int>& nbv, void* sec, std::vector<double>& lam, std::vector<char>& bad,
                 DBuf& work) {
  hipStream_t s = ctx->stream;
  const int B = (int)off.size();
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  // layout: per block X | Q | R | Z | E | scratch, then the staged block
  std::vector<size_t> oX(B), oQ(B), oR(B), oZ(B), oE(B), oS(B);
  size_t tot = 0, nd = 0;
  for (int b = 0; b < B; ++b) {
    const size_t m = nbv[b], mm = m * m;
    oX[b] = tot; tot += up(sizeof(rz) * mm);
    oQ[b] = tot; tot += up(sizeof(rz) * mm);
    oR[b] = tot; tot += up(sizeof(rz) * mm);
    oZ[b] = tot; tot += up(sizeof(double) * mm);
    oE[b] = tot; tot += up(sizeof(double) * m);
    oS[b] = tot; tot += up(std::max(kern::tridiag_scratch_bytes((int)m), kern::tridiag_eig_scratch_bytes((int)m)));
    nd += m;
  }
  // staged: error word and per-block info (ints, 16-byte padded), sums |v|^2, eigenvalues
  const size_t ints = (size_t)(1 + B + 3) / 4 * 4;
  const size_t stage_bytes = sizeof(int) * ints + sizeof(rz) * B + sizeof(double) * nd;
  const size_t oT = tot;
  tot += up(stage_bytes);
  char* base = static_cast<char*>(work.ensure(tot));
  char* stage = base + oT;
  int* derr = reinterpret_cast<int*>(stage);
  int* dinfo = derr + 1;
  rz* dsum = reinterpret_cast<rz*>(stage + sizeof(int) * ints);
  double* dD = reinterpret_cast<double*>(dsum + B);
  kern::zfill(s, stage, zc(0.0, 0.0), (long long)(sizeof(int) * ints / 16), 16);   // error and info words
  std::vector<kern::TdSector> td(B);
  std::vector<kern::EigBlock> eb(B);
  size_t od = 0;
  std::vector<size_t> oDv(B);
  for (int b = 0; b < B; ++b) {
    const int m = nbv[b];
    rz* X = reinterpret_cast<rz*>(base + oX[b]);
    eb[b] = kern::EigBlock{reinterpret_cast<double2*>(X), reinterpret_cast<const double*>(base + oZ[b]),
                           reinterpret_cast<double2*>(base + oR[b]), off[b], m};
    oDv[b] = od;
    td[b] = kern::TdSector{X, base + oQ[b], dD + od, reinterpret_cast<double*>(base + oE[b]), base + oS[b], m};
    od += m;
  }
  // every block gathered and made Hermitian in one launch
  kern::eig_blocks_gather(s, eb.data(), B, H, n, didx);
  if (kern::tridiag_batched(s, td.data(), B, derr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  // the tridiagonal problems: the own divide and conquer for all blocks it
  // takes (one launch per stage), rocSOLVER's for the larger ones
  std::vector<kern::TdEigJob> jobs;
  for (int b = 0; b < B; ++b) {
    const int m = nbv[b];
    double* Z = reinterpret_cast<double*>(base + oZ[b]);
    double* E = reinterpret_cast<double*>(base + oE[b]);
    if (kern::tridiag_eig_scratch_bytes(m) == 0)
      blas_check(rocsolver_dstedc(ctx->blas, rocblas_evect_tridiagonal, m, dD + oDv[b], E, Z, m, dinfo + b), "dstedc");
    else
      jobs.push_back(kern::TdEigJob{dD + oDv[b], E, m, Z, base + oS[b]});
  }
  if (!jobs.empty() && kern::tridiag_eig_batched(s, jobs.data(), (int)jobs.size()) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  // back transformation: rows of the tridiagonal eigenvectors (one launch),
  // R = rows Q^dagger per block, the checks' sums and the scatter into sec
  // (one launch each)
  kern::eig_blocks_rows(s, eb.data(), B);
  for (int b = 0; b < B; ++b) {
    const int m = nbv[b];
    rz* X = reinterpret_cast<rz*>(base + oX[b]);
    rz* R = reinterpret_cast<rz*>(base + oR[b]);
    kern::gemm<double>(s, TDVP_OP_N, TDVP_OP_C, m, m, m, 1.0, X, m, 0, base + oQ[b], m, 0, 0.0, R, m, 0, 1);
  }
  kern::eig_blocks_norms(s, eb.data(), B, dsum);
  kern::eig_blocks_scatter(s, eb.data(), B, sec, n, didx);
  const char* hs = static_cast<const char*>(ctx->fetch(stage, stage_bytes));
  int herr;
  std::memcpy(&herr, hs, sizeof(int));
  const int* hinfo = reinterpret_cast<const int*>(hs) + 1;
  const rz* hsum = reinterpret_cast<const rz*>(hs + sizeof(int) * ints);
  const double* hD = reinterpret_cast<const double*>(hsum + B);
  if (herr != 0) return false;
  bad.assign(B, 0);
  for (int b = 0; b < B; ++b) {
    const int m = nbv[b];
    const double v = hsum[b].real();
    bool ok = hinfo[b] == 0 && std::isfinite(v) && std::fabs(v - m) <= 1e-6 * m;
    for (int j = 0; j < m; ++j) ok = ok && std::isfinite(hD[oDv[b] + j]);
    bad[b] = ok ? 0 : 1;
    for (int j = 0; j < m; ++j) lam[off[b] + j] = hD[oDv[b] + m - 1 - j];
  }
  return true;
}

}  // namespace

void eigh_sectors(tdvp_ctx_s* ctx, const void* H, int n, const std::vector<int>& q, std::vector<double>& lam,
                  void* rows, DBuf& work, std::vector<int>& qout) {
  if (q.empty()) {
    eigh_rows_desc(ctx, H, n, lam, rows, work);
    qout.clear();
    return;
  }
  if ((int)q.size() != n) TDVP_THROW(TDVP_ERR_ARG, "eigh_sectors: one charge per index needed");
  hipStream_t s = ctx->stream;
  const Sectors sc = group_by_charge(q);
  const int ns = (int)sc.charge.size();
  int nmax = 1;
  std::vector<int> unit_idx, unit_pos;    // 1 x 1 blocks
  for (int c = 0; c < ns; ++c) {
    const int nb = sc.off[c + 1] - sc.off[c];
    nmax = std::max(nmax, nb);
    if (nb == 1) {
      unit_idx.push_back(sc.idx[sc.off[c]]);
      unit_pos.push_back(sc.off[c]);
    }
  }
  // one upload: the index lists, then the 1 x 1 blocks' indices and positions
  std::vector<int> ints(sc.idx);
  ints.insert(ints.end(), unit_idx.begin(), unit_idx.end());
  ints.insert(ints.end(), unit_pos.begin(), unit_pos.end());
  DBuf dints(ctx), blk(ctx), rb(ctx), sec(ctx), diag(ctx), w2(ctx);
  const int* didx = upload_ints(ctx, dints, ints);
  const int nu = (int)unit_idx.size();
  // eigenvector rows in sector order (each of full length n)
  sec.ensure(sizeof(zc) * (size_t)n * n);
  kern::zfill(s, sec.p, zc(0.0, 0.0), (long long)n * n, 16);
  blk.ensure(sizeof(zc) * (size_t)nmax * nmax);
  rb.ensure(sizeof(zc) * (size_t)nmax * nmax);
  std::vector<double> lam_sec(n, 0.0), lb;
  // blocks up to 1024 side by side; the rest (and any block that fails its
  // check) one at a time
  std::vector<int> boff, bnb;
  for (int c = 0; c < ns; ++c) {
    const int nb = sc.off[c + 1] - sc.off[c];
    if (nb >= 2 && nb <= 1024) {
      boff.push_back(sc.off[c]);
      bnb.push_back(nb);
    }
  }
  std::vector<char> bad;
  bool batched = false;
  if (boff.size() > 1) {
    Range r_("eigh.blocks");
    batched = eigh_blocks(ctx, H, n, didx, boff, bnb, sec.p, lam_sec, bad, work);
  }
  for (int c = 0, b = 0; c < ns; ++c) {
    const int o = sc.off[c], nb = sc.off[c + 1] - o;
    if (nb < 2) continue;
    const bool in_batch = b < (int)boff.size() && boff[b] == o;
    if (in_batch) ++b;
    if (batched && in_batch && !bad[b - 1]) continue;
    Range r_(nb > 1024 ? "eigh.block_large" : batched && in_batch ? "eigh.block_redo" : "eigh.block_single");
    kern::zgather(s, blk.p, nb, H, n, didx + o, nb, didx + o, nb);
    eigh_rows_desc(ctx, blk.p, nb, lb, rb.p, work);
    kern::zscatter_cols(s, static_cast<char*>(sec.p) + sizeof(zc) * (size_t)o * n, n, rb.p, nb, nb, didx + o, nb);
    for (int j = 0; j < nb; ++j) lam_sec[o + j] = lb[j];
  }
  if (nu > 0) {
    diag.ensure(sizeof(zc) * nu);
    kern::zunit_blocks(s, diag.p, H, n, didx + n, didx + n + nu, nu, sec.p);
    std::vector<zc> d(nu);
    HIP_CHECK(hipMemcpyAsync(d.data(), diag.p, sizeof(zc) * nu, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int j = 0; j < nu; ++j) lam_sec[unit_pos[j]] = d[j].real();
  }
  // global order: descending eigenvalue, then ascending charge, then position
  std::vector<int> sec_of(n);
  for (int c = 0; c < ns; ++c)
    for (int j = sc.off[c]; j < sc.off[c + 1]; ++j) sec_of[j] = c;
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
    if (lam_sec[a] != lam_sec[b]) return lam_sec[a] > lam_sec[b];
    return sec_of[a] < sec_of[b];
  });
  const int* dperm = upload_ints(ctx, w2, perm);
  kern::zgather(s, rows, n, sec.p, n, dperm, n, nullptr, n);
  lam.resize(n);
  qout.resize(n);
  for (int j = 0; j < n; ++j) {
    lam[j] = lam_sec[perm[j]];
    qout[j] = sc.charge[sec_of[perm[j]]];
  }
  // the local device buffers are released in stream order (the context's
  // allocator reuses them only for later work on this stream), so no wait
}

void svd_sectors(tdvp_ctx_s* ctx, const void* C, int rows, int cols, const std::vector<int>& qrow,
                 const std::vector<int>& qcol, std::vector<double>& S, void* Vh, std::vector<int>& qout) {
  if ((int)qrow.size() != rows || (int)qcol.size() != cols) TDVP_THROW(TDVP_ERR_ARG, "svd_sectors: bad charges");
  hipStream_t s = ctx->stream;
  const Sectors sr = group_by_charge(qrow), scl = group_by_charge(qcol);
  std::map<int, int> col_sec;
  for (int c = 0; c < (int)scl.charge.size(); ++c) col_sec[scl.charge[c]] = c;
  std::vector<int> ints(sr.idx);
  ints.insert(ints.end(), scl.idx.begin(), scl.idx.end());
  DBuf dints(ctx), blk(ctx), vb(ctx), w1(ctx), w2(ctx);
  const int* dr = upload_ints(ctx, dints, ints);
  const int* dc = dr + rows;
  const int k = std::min(rows, cols);
  kern::zfill(s, Vh, zc(0.0, 0.0), (long long)k * cols, 16);
  S.clear();
  qout.clear();
  int out = 0;
  std::vector<double> sb;
  for (int c = 0; c < (int)sr.charge.size(); ++c) {
    auto it = col_sec.find(sr.charge[c]);
    if (it == col_sec.end()) continue;     // rows of this charge vanish
    const int ro = sr.off[c], nr = sr.off[c + 1] - ro;
    const int co = scl.off[it->second], nc = scl.off[it->second + 1] - co;
    const int kb = std::min(nr, nc);
    blk.ensure(sizeof(zc) * (size_t)nr * nc);
    vb.ensure(sizeof(zc) * (size_t)kb * nc);
    kern::zgather(s, blk.p, nc, C, cols, dr + ro, nr, dc + co, nc);
    svd_rowmajor(ctx, blk.p, nr, nc, nullptr, sb, vb.p, w1, w2);
    kern::zscatter_cols(s, static_cast<char*>(Vh) + sizeof(zc) * (size_t)out * cols, cols, vb.p, nc, kb, dc + co,
                        nc);
    for (int j = 0; j < kb; ++j) {
      S.push_back(sb[j]);
      qout.push_back(sr.charge[c]);
    }
    out += kb;
  }
  HIP_CHECK(hipStreamSynchronize(s));
}

int factor_sectors(tdvp_ctx_s* ctx, bool left, const void* C, int rows, int cols, const std::vector<int>& qrow,
                   const std::vector<int>& qcol, DBuf& X1, DBuf& X2, std::vector<int>& qk) {
  if ((int)qrow.size() != rows || (int)qcol.size() != cols) TDVP_THROW(TDVP_ERR_ARG, "factor_sectors: bad charges");
  hipStream_t s = ctx->stream;
  const Sectors sr = group_by_charge(qrow), scl = group_by_charge(qcol);
  // every charge of either side, with its row and column counts
  std::map<int, std::pair<int, int>> sec;   // charge -> (row sector, column sector), -1 if absent
  for (int c = 0; c < (int)sr.charge.size(); ++c) sec[sr.charge[c]] = {c, -1};
  for (int c = 0; c < (int)scl.charge.size(); ++c) {
    auto it = sec.find(scl.charge[c]);
    if (it == sec.end()) sec[scl.charge[c]] = {-1, c};
    else it->second.second = c;
  }
  struct Blk { int q, r, c, nr, nc, kb, extra; };
  std::vector<Blk> blks;
  int deficit = 0;
  for (auto& kv : sec) {
    const int r = kv.second.first, c = kv.second.second;
    Blk b{kv.first, r, c, r < 0 ? 0 : sr.off[r + 1] - sr.off[r], c < 0 ? 0 : scl.off[c + 1] - scl.off[c], 0, 0};
    b.kb = std::min(b.nr, b.nc);
    // the bond of the factorisation has the size min(rows, cols) of the
    // dense one: where a charge has more bond states on one side than the
    // other side can hold, the missing ones come from charges with room to
    // spare, as orthonormal completions that carry no weight
    deficit += left ? std::max(0, b.nc - b.nr) : std::max(0, b.nr - b.nc);
    blks.push_back(b);
  }
  auto spare = [&](const Blk& b) { return (left ? b.nr - b.nc : b.nc - b.nr) - b.extra; };
  while (deficit > 0) {
    int best = -1;
    for (int x = 0; x < (int)blks.size(); ++x)
      if ((left ? blks[x].nr : blks[x].nc) > 0 && spare(blks[x]) > 0 && (best < 0 || spare(blks[x]) > spare(blks[best])))
        best = x;
    if (best < 0) break;
    ++blks[best].extra;
    --deficit;
  }
  int k = 0;
  qk.clear();
  for (auto& b : blks) {
    for (int j = 0; j < b.kb + b.extra; ++j) qk.push_back(b.q);
    k += b.kb + b.extra;
  }
  std::vector<int> ints(sr.idx);
  ints.insert(ints.end(), scl.idx.begin(), scl.idx.end());
  DBuf dints(ctx), blk(ctx), f1(ctx), f2(ctx), w(ctx), tau(ctx);
  const int* dr = upload_ints(ctx, dints, ints);
  const int* dc = dr + rows;
  X1.ensure(sizeof(zc) * std::max<size_t>(1, (size_t)rows * k));
  X2.ensure(sizeof(zc) * std::max<size_t>(1, (size_t)k * cols));
  kern::zfill(s, X1.p, zc(0.0, 0.0), (long long)rows * k, 16);
  kern::zfill(s, X2.p, zc(0.0, 0.0), (long long)k * cols, 16);
  int off = 0;
  for (auto& b : blks) {
    const int kt = b.kb + b.extra;
    if (kt == 0) continue;
    const int* ri = b.r < 0 ? nullptr : dr + sr.off[b.r];
    const int* ci = b.c < 0 ? nullptr : dc + scl.off[b.c];
    if (b.nr > 0 && b.nc > 0) {
      blk.ensure(sizeof(zc) * (size_t)b.nr * b.nc);
      kern::zgather(s, blk.p, b.nc, C, cols, ri, b.nr, ci, b.nc);
    }
    if (left) {
      // X1 = A (rows x k): columns off .. off + kt of the block's rows;
      // X2 = R (k x cols): rows off .. off + kb of the block's columns
      f1.ensure(sizeof(zc) * (size_t)b.nr * std::max(b.nr, 1));
      f2.ensure(sizeof(zc) * (size_t)std::max(b.kb, 1) * std::max(b.nc, 1));
      int lda = b.kb;
      if (b.extra == 0) {
        qr_rowmajor(ctx, blk.p, b.nr, b.nc, f1.p, f2.p, w, tau);
      } else if (b.nc > 0) {
        qr_rowmajor_full(ctx, blk.p, b.nr, b.nc, f1.p, f2.p, tau);
        lda = b.nr;
      } else {   // no column of this charge: completions only (an identity block)
        kern::zfill(s, f1.p, zc(0.0, 0.0), (long long)b.nr * b.nr, 16);
        kern::zshift_diag(s, f1.p, b.nr, 1.0, 1.0);
        lda = b.nr;
      }
      kern::zscatter(s, static_cast<char*>(X1.p) + sizeof(zc) * off, k, f1.p, lda, ri, b.nr, nullptr, kt);
      if (b.kb > 0)
        kern::zscatter(s, static_cast<char*>(X2.p) + sizeof(zc) * (size_t)off * cols, cols, f2.p, b.nc, nullptr, b.kb,
                       ci, b.nc);
    } else {
      // X1 = L (rows x k): columns off .. off + kb; X2 = B (k x cols): rows
      // off .. off + kt of the block's columns
      f1.ensure(sizeof(zc) * (size_t)std::max(b.nr, 1) * std::max(b.kb, 1));
      f2.ensure(sizeof(zc) * (size_t)b.nc * std::max(b.nc, 1));
      if (b.extra == 0) {
        lq_rowmajor(ctx, blk.p, b.nr, b.nc, f1.p, f2.p, w, tau);
      } else if (b.nr > 0) {
        lq_rowmajor_full(ctx, blk.p, b.nr, b.nc, f1.p, f2.p, tau);
      } else {
        kern::zfill(s, f2.p, zc(0.0, 0.0), (long long)b.nc * b.nc, 16);
        kern::zshift_diag(s, f2.p, b.nc, 1.0, 1.0);
      }
      if (b.kb > 0)
        kern::zscatter(s, static_cast<char*>(X1.p) + sizeof(zc) * off, k, f1.p, b.kb, ri, b.nr, nullptr, b.kb);
      kern::zscatter(s, static_cast<char*>(X2.p) + sizeof(zc) * (size_t)off * cols, cols, f2.p, b.nc, nullptr, kt, ci,
                     b.nc);
    }
    off += kt;
  }
  HIP_CHECK(hipStreamSynchronize(s));
  return k;
}

bool tridiag_ql(double* d, double* e, int n, double* Zr, int nr) {
  // Implicit QL sweeps with a Wilkinson shift from the leading 2 x 2 block of
  // the unreduced part (Golub & Van Loan, Sec. 8.3); every rotation is
  // applied to the columns of Zr.
  if (n <= 0) return true;
  e[n - 1] = 0.0;
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m < n - 1; ++m)
        if (std::fabs(e[m]) <= eps * (std::fabs(d[m]) + std::fabs(d[m + 1]))) break;
      if (m == l) break;
      if (iter == 60) return false;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      bool split = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {   // the chase decoupled the block: restart on the shorter one
          d[i + 1] -= p;
          e[m] = 0.0;
          split = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = 0; k < nr; ++k) {
          double* z = Zr + (size_t)k * n;
          const double zf = z[i + 1];
          z[i + 1] = s * z[i] + c * zf;
          z[i] = c * z[i] - s * zf;
        }
      }
      if (split) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

}  // namespace la

// Number of leading weights (sorted descending) to keep: the smallest n whose
// discarded tail sum(w[n:]) is <= eps * trace_ref, never keeping weights
// below 1e-14 * w[0] (numerical zeros); a multiplet (neighbours closer than
// 1e-12 * w[0]) straddling that cut is kept whole; then at most `cap`, where
// a multiplet straddling the cap is dropped whole; and at least min_keep.
int keep_count(const std::vector<double>& w_in, double eps, double trace_ref, int cap, int min_keep) {
  const int n_all = (int)w_in.size();
  if (n_all == 0) return 0;
  std::vector<double> w(n_all);
  for (int i = 0; i < n_all; ++i) w[i] = std::max(0.0, w_in[i]);
  const double w0 = w[0];
  if (w0 <= 0.0) return cap > 0 ? std::min(min_keep, std::min(n_all, cap)) : 0;
  const double floor_w = 1e-14 * w0, tie = 1e-12 * w0;
  std::vector<double> tail(n_all + 1, 0.0);
  for (int i = n_all - 1; i >= 0; --i) tail[i] = tail[i + 1] + w[i];
  int n = 0;
  while (n < n_all && tail[n] > eps * trace_ref && w[n] > floor_w) ++n;
  while (n > 0 && n < n_all && w[n] > floor_w && (w[n - 1] - w[n]) <= tie) ++n;
  if (n > cap) {
    int nc = cap;
    while (nc > 0 && nc < n_all && (w[nc - 1] - w[nc]) <= tie) --nc;
    n = nc > 0 ? nc : cap;
  }
  const int lo = std::min(min_keep, std::min(n_all, std::max(cap, 0)));
  return std::max(n, lo);
}
