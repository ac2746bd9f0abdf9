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
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>

#include "common.h"

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

void eigh_rows_desc(tdvp_ctx_s* ctx, const void* H, int n, std::vector<double>& lam, void* rows, DBuf& work) {
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
  HIP_CHECK(hipMemcpyAsync(X, H, sizeof(rz) * nn, hipMemcpyDeviceToDevice, ctx->stream));
  kern::zhermitize(ctx->stream, X, n);
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
    for (double v : h)
      if (!std::isfinite(v)) TDVP_THROW(TDVP_ERR_NUMERIC, "eigh: non-finite input matrix (n = " + std::to_string(n) + ")");
    HIP_CHECK(hipMemcpyAsync(X, H, sizeof(rz) * nn, hipMemcpyDeviceToDevice, ctx->stream));
    kern::zhermitize(ctx->stream, X, n);
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

void jacobi_eigh(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V) {
  // cyclic Jacobi rotations on the symmetric n x n matrix A (row-major);
  // on return w holds the eigenvalues ascending and column j of V the
  // eigenvector of w[j]
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {  // columns p, q
          const double arp = a(r, p), arq = a(r, q);
          a(r, p) = c * arp - s * arq;
          a(r, q) = s * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {  // rows p, q
          const double apr = a(p, r), aqr = a(q, r);
          a(p, r) = c * apr - s * aqr;
          a(q, r) = s * apr + c * aqr;
        }
        for (int r = 0; r < n; ++r) {
          const double vrp = V[(size_t)r * n + p], vrq = V[(size_t)r * n + q];
          V[(size_t)r * n + p] = c * vrp - s * vrq;
          V[(size_t)r * n + q] = s * vrp + c * vrq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
  std::vector<double> V2((size_t)n * n);
  w.resize(n);
  for (int j = 0; j < n; ++j) {
    w[j] = a(idx[j], idx[j]);
    for (int r = 0; r < n; ++r) V2[(size_t)r * n + j] = V[(size_t)r * n + idx[j]];
  }
  V.swap(V2);
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
