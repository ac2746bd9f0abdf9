// GSE-TDVP1 drivers on the device: one-site TDVP sweep, global Krylov
// vectors by the density-matrix MPO application, state-averaged basis
// extension, measurements.  Tensor layouts (row-major, complex interleaved):
//   site M[a,s,b]; MPO W[alpha,beta,s',s]; left env L[a',alpha,a];
//   right env Rt[beta,b,b'] (bra index last so that the second stage of the
//   effective Hamiltonian is a plain GEMM); double-layer env E[al,a,al',a'].
// Environments L[i] and Rt[i] live on bond i (left of site i): L[i] covers
// sites 0..i-1, Rt[i] covers sites i..N-1.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <cstring>
#include <map>
#include <memory>

namespace {

constexpr int ZB = 16;  // bytes per complex128

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <typename T> constexpr int cbytes() { return 2 * (int)sizeof(T); }

void upload(tdvp_ctx_s* ctx, void* dst, const void* src, size_t bytes) {
  HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
}

void download(tdvp_ctx_s* ctx, void* dst, const void* src, size_t bytes) {
  HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
}

void set_one(tdvp_ctx_s* ctx, DBuf& b, int esize) {
  b.ensure(esize);
  kern::zfill(ctx->stream, b.p, zc(1.0, 0.0), 1, esize);
}

// ------------------------------------------------------------ FP64 scalars
struct Scalars {
  tdvp_ctx_s* ctx;
  DBuf partial, out;
  explicit Scalars(tdvp_ctx_s* c) : ctx(c), partial(c), out(c) {}
  // <a|b> (conjugated) or sum a*b for n complex128 entries, returned to host
  zc dot(const void* a, const void* b, long long n, bool conj = true) {
    const int nb = kern::zdots_blocks(n);
    partial.ensure((size_t)nb * ZB);
    out.ensure(ZB);
    kern::zdots(ctx->stream, a, n, 1, b, n, partial.p, nb, out.p, conj);
    return *static_cast<const zc*>(ctx->fetch(out.p, ZB));
  }
  double norm(const void* a, long long n) { return std::sqrt(std::max(0.0, dot(a, a, n).real())); }
};

// ------------------------------------------------------------ Lanczos
struct Lanczos {
  tdvp_ctx_s* ctx;
  DBuf V, partial, scal;
  explicit Lanczos(tdvp_ctx_s* c) : ctx(c), V(c), partial(c), scal(c) {}

  // x <- exp(-i dt H) x by Lanczos with full reorthogonalisation (classical
  // Gram-Schmidt applied twice).  Returns the number of H applications.
  template <class MV>
  int run(MV&& mv, void* x, long long n, zc dt, double tol, int maxit, bool normalize, bool* unconv,
          MatvecTimer* timer) {
    *unconv = false;
    if (n <= 0) return 0;
    const int nb = kern::zdots_blocks(n);
    const int nnp = kern::zcombine_norm_blocks(n);
    // the dot-product partials, then the partial sums of |w|^2
    partial.ensure(((size_t)nb * (maxit + 1) + (size_t)nnp * (maxit + 2)) * ZB);
    double2* npart = partial.as<double2>() + (size_t)nb * (maxit + 1);
    double2* dpart2 = npart + nnp;   // second-pass partial dot products, nnp x (j + 1)
    scal.ensure(320 * ZB);
    double2* S = scal.as<double2>();
    // S: [0, 64) and [64, 128) the two projection passes, 128 |w|^2, 192.. the
    // result coefficients, 256 the summed partial norms of long vectors
    constexpr int FOLD = 64;
    char* Vb = static_cast<char*>(V.ensure((size_t)(maxit + 1) * n * ZB));
    auto vec = [&](int j) { return static_cast<void*>(Vb + (size_t)j * n * ZB); };

    kern::zdots(ctx->stream, x, n, 1, x, n, partial.p, nb, S + 128);
    const zc nrm2 = *static_cast<const zc*>(ctx->fetch(S + 128, ZB));
    const double nrm = std::sqrt(std::max(0.0, nrm2.real()));
    if (!(nrm > 0.0)) {
      if (!std::isfinite(nrm)) TDVP_THROW(TDVP_ERR_NUMERIC, "non-finite vector entering Lanczos");
      return 0;
    }
    kern::zscale(ctx->stream, vec(0), x, zc(1.0 / nrm, 0.0), n);
    std::vector<double> alpha, beta, dd, ee, Z;
    std::vector<zc> c;
    int napp = 0, dim = 0;
    // exp(-i dt T) e_1 from the eigen-decomposition T = Z diag(l) Z^T of the
    // Lanczos matrix: component r is sum_e Z[r][e] exp(-i dt l_e) Z[0][e]
    auto tridiag_eig = [&](int nr) {
      dd = alpha;
      ee.assign(dim, 0.0);
      for (int i = 0; i + 1 < dim; ++i) ee[i] = beta[i];
      Z.assign((size_t)nr * dim, 0.0);
      if (nr == dim) {
        for (int r = 0; r < dim; ++r) Z[(size_t)r * dim + r] = 1.0;
      } else {   // rows 0 and dim-1 only
        Z[0] = 1.0;
        Z[(size_t)(nr - 1) * dim + dim - 1] = 1.0;
      }
      if (!la::tridiag_ql(dd.data(), ee.data(), dim, Z.data(), nr))
        TDVP_THROW(TDVP_ERR_NUMERIC, "Lanczos tridiagonal eigensolver did not converge");
    };
    auto phase = [&](int e) { return std::exp(zc(0.0, -1.0) * dt * dd[e]); };
    // Iteration j on the device: w = H v_j, classical Gram-Schmidt twice
    // against v_0..v_j (each pass: partial dot products, then the update,
    // whose blocks sum the partials themselves; the first update also forms
    // the second pass's partial products on its chunk, and the second leaves
    // per-block sums of |w|^2),
    // v_{j+1} = w / |w| with |w|^2 summed by the scaling kernel itself, which
    // also writes the scalars into pinned host memory.  The next
    // iteration is enqueued before the host reads this one's scalars, so the
    // device does not wait for the convergence test; when the test stops the
    // recurrence, that extra iteration is discarded.  When the error
    // estimates of the last two iterations extrapolate (geometrically) to
    // convergence at this one, the next is enqueued only if the test fails.
    const zc* staged[2] = {nullptr, nullptr};
    auto enqueue = [&](int j) {
      void* w = vec(j + 1);
      if (timer) timer->cur = j & 1;
      mv(vec(j), w);
      kern::zdots_partial(ctx->stream, Vb, n, j + 1, w, n, partial.p, nb);
      // Every block of the update kernels sums all partials itself; above
      // FOLD partials (long vectors) that work grows as (n / block)^2, so
      // they are first summed once by a separate launch (same fixed order).
      if (nb > FOLD) {
        kern::zsum_partials(ctx->stream, partial.p, nb, j + 1, S);
        kern::zcombine_dots(ctx->stream, w, Vb, n, j + 1, S, 1, -1.0, n, nullptr, dpart2);
      } else {
        kern::zcombine_dots(ctx->stream, w, Vb, n, j + 1, partial.p, nb, -1.0, n, S, dpart2);
      }
      // the normalisation also writes the first-pass projections (alpha_j =
      // <v_j|H v_j>) and |w|^2 into the pinned slot the host reads
      if (nnp > FOLD) {
        kern::zsum_partials(ctx->stream, dpart2, nnp, j + 1, S + 64);
        kern::zcombine_p(ctx->stream, w, Vb, n, j + 1, S + 64, 1, -1.0, n, nullptr, npart);
        kern::zsum_partials(ctx->stream, npart, nnp, 1, S + 256);
        kern::zscale_invnorm(ctx->stream, w, S + 256, 1, S + 128, n, ctx->stage_slot_dev(j & 1), S, j + 1, 128);
      } else {
        kern::zcombine_p(ctx->stream, w, Vb, n, j + 1, dpart2, nnp, -1.0, n, S + 64, npart);
        kern::zscale_invnorm(ctx->stream, w, npart, nnp, S + 128, n, ctx->stage_slot_dev(j & 1), S, j + 1, 128);
      }
      staged[j & 1] = static_cast<const zc*>(ctx->stage_mark(j & 1));
    };
    enqueue(0);
    int queued = 0;                       // last iteration enqueued
    double err1 = -1.0, err2 = -1.0;      // relative error estimates of j-1, j-2
    for (int j = 0; j < maxit; ++j) {
      const bool likely_last = err1 > 0.0 && err2 > 0.0 && err1 * (err1 / err2) <= tol;
      if (queued < j + 1 && j + 1 < maxit && !likely_last) enqueue(queued = j + 1);
      ctx->wait_stage(j & 1);
      const zc* hv = staged[j & 1];
      if (timer) timer->collect(j & 1);
      ++napp;
      const double a = hv[j].real(), b = std::sqrt(std::max(0.0, hv[128].real()));
      if (!std::isfinite(a) || !std::isfinite(b)) TDVP_THROW(TDVP_ERR_NUMERIC, "non-finite Lanczos coefficient");
      alpha.push_back(a);
      dim = j + 1;
      // convergence needs |exp(-i dt T) e_1| and its last component only
      const int nr = dim == 1 ? 1 : 2;
      tridiag_eig(nr);
      double cn2 = 0.0;
      zc clast(0.0, 0.0);
      for (int e = 0; e < dim; ++e) {
        const zc ph = phase(e) * Z[e];
        cn2 += std::norm(ph);
        clast += Z[(size_t)(nr - 1) * dim + e] * ph;
      }
      double scale = 0.0;
      for (double v : alpha) scale = std::max(scale, std::fabs(v));
      for (double v : beta) scale = std::max(scale, v);
      const bool conv = b * std::abs(clast) <= tol * std::sqrt(cn2) || b <= 1e-14 * scale;
      if (conv || j == maxit - 1) {
        if (!conv) *unconv = true;
        break;
      }
      beta.push_back(b);
      if (queued < j + 1) enqueue(queued = j + 1);
      err2 = err1;
      err1 = cn2 > 0.0 ? b * std::abs(clast) / std::sqrt(cn2) : -1.0;
    }
    tridiag_eig(dim);
    c.assign(dim, zc(0.0, 0.0));
    for (int e = 0; e < dim; ++e) {
      const zc ph = phase(e) * Z[e];
      for (int r = 0; r < dim; ++r) c[r] += Z[(size_t)r * dim + e] * ph;
    }
    double f = nrm;
    if (normalize) {
      double cn = 0.0;
      for (const zc& v : c) cn += std::norm(v);
      f = 1.0 / std::sqrt(cn);
    }
    std::vector<zc> cs(dim);
    for (int r = 0; r < dim; ++r) cs[r] = f * c[r];
    upload(ctx, S + 192, cs.data(), (size_t)dim * ZB);
    kern::zfill(ctx->stream, x, zc(0.0, 0.0), n, ZB);
    kern::zcombine(ctx->stream, x, Vb, n, dim, S + 192, 1.0, n);
    HIP_CHECK(hipStreamSynchronize(ctx->stream));  // `cs` is pageable host memory
    if (timer) timer->collect_all();                // the discarded iteration ran too
    return napp;
  }
};

}  // namespace

// ------------------------------------------------------------ contractions
template <typename T>
void heff_apply(tdvp_ctx_s* ctx, const SiteTables& tb, int ml, int wl, int wr, int mr, const void* L,
                const void* Rt, const void* C, void* Y, void* ws1, void* ws2, MatvecTimer* tm, SplitWS sk,
                ProdMaps pm) {
  hipStream_t s = ctx->stream;
  if (tm) tm->mark(0);
  // T1[(a',al),(s,b)] = L[(a',al),a] C[a,(s,b)] (with charges: batched over al)
  if (pm.g1) {
    kern::KMapScope ks(pm.g1);
    kern::gemm_heff_batched<T>(s, ml, 2 * mr, ml, L, (long long)wl * ml, ml, C, 2 * mr, 0, ws1, (long long)wl * 2 * mr,
                               2 * mr, wl);
  } else {
    kern::gemm_heff<T>(s, ml * wl, 2 * mr, ml, L, ml, C, 2 * mr, ws1, 2 * mr, sk.p, sk.bytes);
  }
  if (tm) tm->mark(1);
  // T2[a',s',be,b] = sum W[al,be,s',s] T1[a',al,s,b]
  kern::wapply<T>(s, tb.F, ws1, ws2, ml, mr, (long long)wl * 2 * mr, 1, 2LL * mr, mr, (long long)2 * wr * mr, 1,
                  mr, (long long)wr * mr, pm.wc);
  if (tm) tm->mark(2);
  // Y[(a',s'),b'] = T2[(a',s'),(be,b)] Rt[(be,b),b'] (with charges: batched over s')
  if (pm.g2) {
    kern::KMapScope ks(pm.g2);
    kern::gemm_heff_batched<T>(s, ml, mr, wr * mr, ws2, 2LL * wr * mr, (long long)wr * mr, Rt, mr, 0, Y, 2LL * mr, mr,
                               2);
  } else {
    kern::gemm_heff<T>(s, 2 * ml, mr, wr * mr, ws2, (long long)wr * mr, Rt, mr, Y, mr, sk.p, sk.bytes);
  }
  if (tm) tm->mark(3);
  if (tm)
    tm->gemm_flops += pm.flops >= 0.0 ? pm.flops
                                      : 8.0 * ((double)ml * wl * ml * 2 * mr + (double)2 * ml * wr * mr * mr);
}

template <typename T>
void keff_apply(tdvp_ctx_s* ctx, int ml, int w, int mr, const void* L, const void* Rt, const void* X, void* Y,
                void* ws1, SplitWS sk, ProdMaps pm) {
  hipStream_t s = ctx->stream;
  // Y1[(a',al),b] = L[(a',al),a] X[a,b];  Y[a',b'] = Y1[a',(al,b)] Rt[(al,b),b']
  if (pm.g1) {   // with charges: batched over al
    kern::KMapScope ks(pm.g1);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, ml, mr, ml, 1.0, L, (long long)w * ml, ml, X, mr, 0, 0.0, ws1,
                  (long long)w * mr, mr, w);
  } else {
    kern::gemm_nn_ws<T>(s, ml * w, mr, ml, 1.0, L, ml, X, mr, 0.0, ws1, mr, sk.p, sk.bytes);
  }
  kern::KMapScope ks(pm.g2);
  kern::gemm_nn_ws<T>(s, ml, mr, w * mr, 1.0, ws1, (long long)w * mr, Rt, mr, 0.0, Y, mr, sk.p, sk.bytes);
}

template <typename T>
void env_left(tdvp_ctx_s* ctx, const SiteTables& tb, int ml, int wl, int wr, int mr, const void* L, const void* A,
              void* Lout, void* ws1, void* ws2, SplitWS sk, ProdMaps pm) {
  hipStream_t s = ctx->stream;
  if (pm.g1) {   // with charges: batched over al
    kern::KMapScope ks(pm.g1);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, ml, 2 * mr, ml, 1.0, L, (long long)wl * ml, ml, A, 2 * mr, 0, 0.0, ws1,
                  (long long)wl * 2 * mr, 2 * mr, wl);
  } else {
    kern::gemm_nn_ws<T>(s, ml * wl, 2 * mr, ml, 1.0, L, ml, A, 2 * mr, 0.0, ws1, 2 * mr, sk.p, sk.bytes);
  }
  kern::wapply<T>(s, tb.F, ws1, ws2, ml, mr, (long long)wl * 2 * mr, 1, 2LL * mr, mr, (long long)2 * wr * mr, 1,
                  mr, (long long)wr * mr, pm.wc);
  // Lout[b',(be,b)] = sum_{(a',s')} conj(A[(a',s'),b']) T2[(a',s'),(be,b)]
  kern::KMapScope ks(pm.g2);
  kern::gemm<T>(s, TDVP_OP_C, TDVP_OP_N, mr, wr * mr, 2 * ml, 1.0, A, mr, 0, ws2, (long long)wr * mr, 0, 0.0, Lout,
                (long long)wr * mr, 0, 1);
}

template <typename T>
void env_right(tdvp_ctx_s* ctx, const SiteTables& tb, int ml, int wl, int wr, int mr, const void* Rt,
               const void* B, void* Rout, void* ws1, void* ws2, SplitWS sk, ProdMaps pm) {
  (void)sk;
  hipStream_t s = ctx->stream;
  // U1[be][(a,s),b'] = B[(a,s),b] Rt[be][b,b']   (batched over be)
  {
    kern::KMapScope ks(pm.g1);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, 2 * ml, mr, mr, 1.0, B, mr, 0, Rt, mr, (long long)mr * mr, 0.0, ws1, mr,
                  2LL * ml * mr, wr);
  }
  // U2[al,a,s',b'] = sum W[al,be,s',s] U1[be,a,s,b']
  kern::wapply<T>(s, tb.B, ws1, ws2, ml, mr, 2LL * mr, 1, 2LL * ml * mr, mr, 2LL * mr, 1, 2LL * ml * mr, mr, pm.wc);
  // Rout[(al,a),a'] = sum_{(s',b')} U2[(al,a),(s',b')] conj(B[a',(s',b')])
  kern::KMapScope ks(pm.g2);
  kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_C, wl * ml, ml, 2 * mr, 1.0, ws2, 2LL * mr, 0, B, 2LL * mr, 0, 0.0, Rout, ml,
                0, 1);
}

// Two-site effective Hamiltonian on Th[a,(s,v),b] for the sites i, i+1:
// Y[a',t,u,b'] = sum L[a',al,a] W1[al,be,t,s] W2[be,ga,u,v] Th[a,s,v,b] Rt[ga,b,b'].
// Work buffers hold 4*ml*mr*max(wl,wm,wr) elements each.
template <typename T>
void heff2_apply(tdvp_ctx_s* ctx, const SiteTables& t1, const SiteTables& t2, int ml, int wl, int wm, int wr, int mr,
                 const void* L, const void* Rt, const void* Th, void* Y, void* ws1, void* ws2, MatvecTimer* tm,
                 SplitWS sk, ProdMaps pm = {}) {
  hipStream_t s = ctx->stream;
  if (tm) tm->mark(0);
  // T1[(a',al),(s,v,b)] = L[(a',al),a] Th[a,(s,v,b)]
  {
    kern::KMapScope ks(pm.g1);
    kern::gemm_heff<T>(s, ml * wl, 4 * mr, ml, L, ml, Th, 4 * mr, ws1, 4 * mr, sk.p, sk.bytes);
  }
  if (tm) tm->mark(1);
  // T2[a',t,be,(v,b)] = sum W1[al,be,t,s] T1[a',al,s,(v,b)]
  kern::wapply<T>(s, t1.F, ws1, ws2, ml, 2LL * mr, (long long)wl * 4 * mr, 1, 4LL * mr, 2LL * mr,
                  (long long)2 * wm * 2 * mr, 1, 2LL * mr, (long long)wm * 2 * mr);
  // T3[(a',t),u,ga,b] = sum W2[be,ga,u,v] T2[(a',t),be,v,b]
  kern::wapply<T>(s, t2.F, ws2, ws1, 2LL * ml, mr, (long long)wm * 2 * mr, 1, 2LL * mr, mr, (long long)2 * wr * mr,
                  1, mr, (long long)wr * mr);
  if (tm) tm->mark(2);
  // Y[(a',t,u),b'] = T3[(a',t,u),(ga,b)] Rt[(ga,b),b']
  {
    kern::KMapScope ks(pm.g2);
    kern::gemm_heff<T>(s, 4 * ml, mr, wr * mr, ws1, (long long)wr * mr, Rt, mr, Y, mr, sk.p, sk.bytes);
  }
  if (tm) tm->mark(3);
  if (tm)
    tm->gemm_flops += pm.flops >= 0.0 ? pm.flops
                                      : 8.0 * ((double)ml * wl * ml * 4 * mr + (double)4 * ml * wr * mr * mr);
}

template void heff_apply<double>(tdvp_ctx_s*, const SiteTables&, int, int, int, int, const void*, const void*,
                                 const void*, void*, void*, void*, MatvecTimer*, SplitWS, ProdMaps);
template void heff_apply<float>(tdvp_ctx_s*, const SiteTables&, int, int, int, int, const void*, const void*,
                                const void*, void*, void*, void*, MatvecTimer*, SplitWS, ProdMaps);
template void keff_apply<double>(tdvp_ctx_s*, int, int, int, const void*, const void*, const void*, void*, void*,
                                 SplitWS, ProdMaps);
template void keff_apply<float>(tdvp_ctx_s*, int, int, int, const void*, const void*, const void*, void*, void*,
                                SplitWS, ProdMaps);
template void env_left<double>(tdvp_ctx_s*, const SiteTables&, int, int, int, int, const void*, const void*, void*,
                               void*, void*, SplitWS, ProdMaps);
template void env_left<float>(tdvp_ctx_s*, const SiteTables&, int, int, int, int, const void*, const void*, void*,
                              void*, void*, SplitWS, ProdMaps);
template void env_right<double>(tdvp_ctx_s*, const SiteTables&, int, int, int, int, const void*, const void*, void*,
                                void*, void*, SplitWS, ProdMaps);
template void env_right<float>(tdvp_ctx_s*, const SiteTables&, int, int, int, int, const void*, const void*, void*,
                               void*, void*, SplitWS, ProdMaps);

// ------------------------------------------------------------ handles
namespace {

struct TableBlob {
  std::vector<char> bytes;
  size_t add(const void* p, size_t n) {
    const size_t off = (bytes.size() + 15) & ~size_t(15);
    bytes.resize(off + n);
    if (n) std::memcpy(bytes.data() + off, p, n);
    return off;
  }
};

struct TableOffsets {
  size_t rp, col, val;
  int n_in, n_out;
};

TableOffsets add_table(TableBlob& blob, const std::vector<zc>& W, int wl, int wr, int mode) {
  std::vector<int> rp, col;
  std::vector<zc> val;
  build_site_csr(W, wl, wr, mode, rp, col, val);
  TableOffsets o;
  o.rp = blob.add(rp.data(), rp.size() * sizeof(int));
  o.col = blob.add(col.data(), std::max<size_t>(1, col.size()) * sizeof(int));
  o.val = blob.add(val.data(), std::max<size_t>(1, val.size()) * sizeof(zc));
  o.n_in = (mode == 0 ? wl : wr) * 2;
  o.n_out = (mode == 0 ? wr : wl) * 2;
  return o;
}

kern::WTable resolve(const char* base, const TableOffsets& o) {
  return kern::WTable{reinterpret_cast<const int*>(base + o.rp), reinterpret_cast<const int*>(base + o.col),
                      reinterpret_cast<const double*>(base + o.val), o.n_in, o.n_out};
}

}  // namespace

SiteTables upload_tables(tdvp_ctx_s* ctx, const std::vector<zc>& W, int wl, int wr, DBuf& buf) {
  TableBlob blob;
  TableOffsets f = add_table(blob, W, wl, wr, 0), b = add_table(blob, W, wl, wr, 1), h = add_table(blob, W, wl, wr, 2);
  buf.ensure(blob.bytes.size());
  upload(ctx, buf.p, blob.bytes.data(), blob.bytes.size());
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  const char* base = static_cast<const char*>(buf.p);
  SiteTables t;
  t.F = resolve(base, f);
  t.B = resolve(base, b);
  t.BH = resolve(base, h);
  t.nnz = site_nnz(W);
  return t;
}

size_t write_tables(tdvp_ctx_s* ctx, const std::vector<zc>& W, int wl, int wr, void* dst, size_t cap,
                    SiteTables* out) {
  TableBlob blob;
  TableOffsets f = add_table(blob, W, wl, wr, 0), b = add_table(blob, W, wl, wr, 1), h = add_table(blob, W, wl, wr, 2);
  if (blob.bytes.size() > cap) return blob.bytes.size();
  upload(ctx, dst, blob.bytes.data(), blob.bytes.size());
  // the host blob dies on return: wait for the copy
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  const char* base = static_cast<const char*>(dst);
  out->F = resolve(base, f);
  out->B = resolve(base, b);
  out->BH = resolve(base, h);
  out->nnz = site_nnz(W);
  return blob.bytes.size();
}

std::unique_ptr<tdvp_mpo_s> make_mpo(tdvp_ctx_s* ctx, HostMPO&& host) {
  auto m = std::make_unique<tdvp_mpo_s>();
  m->ctx = ctx;
  m->host = std::move(host);
  m->dev = DBuf(ctx);
  const int N = m->host.N;
  TableBlob blob;
  std::vector<TableOffsets> offs;
  for (int i = 0; i < N; ++i)
    for (int mode = 0; mode < 3; ++mode)
      offs.push_back(add_table(blob, m->host.W[i], m->host.w[i], m->host.w[i + 1], mode));
  m->dev.ensure(blob.bytes.size());
  upload(ctx, m->dev.p, blob.bytes.data(), blob.bytes.size());
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  const char* base = static_cast<const char*>(m->dev.p);
  m->tab.resize(N);
  for (int i = 0; i < N; ++i) {
    m->tab[i].F = resolve(base, offs[3 * i]);
    m->tab[i].B = resolve(base, offs[3 * i + 1]);
    m->tab[i].BH = resolve(base, offs[3 * i + 2]);
    m->tab[i].nnz = site_nnz(m->host.W[i]);
  }
  return m;
}

std::unique_ptr<tdvp_mps_s> make_mps(tdvp_ctx_s* ctx, int N, const int* dims, const double* host,
                                     const int* charges) {
  auto p = std::make_unique<tdvp_mps_s>();
  p->ctx = ctx;
  p->N = N;
  p->m.assign(dims, dims + N + 1);
  if (charges) {
    p->q.resize(N + 1);
    size_t off = 0;
    for (int b = 0; b <= N; ++b) {
      p->q[b].assign(charges + off, charges + off + dims[b]);
      off += dims[b];
    }
  }
  size_t off = 0;
  for (int i = 0; i < N; ++i) {
    p->t.emplace_back(ctx);
    const size_t bytes = (size_t)p->elems(i) * ZB;
    p->t[i].ensure(bytes);
    upload(ctx, p->t[i].p, host + 2 * off, bytes);
    off += p->elems(i);
  }
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  return p;
}

// ------------------------------------------------------------ drivers
namespace {

struct Work {
  tdvp_ctx_s* ctx;
  kern::SplitWorkspaceScope gws;   // split-K scratch of the products issued below
  DBuf ws1, ws2, xf, yf, conv, work, work2, tau, tmpA, tmpB, tmpC, dvec, wsk, nsg, nst, cinv, pidx, prow, xp, segd;
  Scalars sc;
  Lanczos lz;
  // the context's block-sparse maps
  MapCache* maps;
  explicit Work(tdvp_ctx_s* c)
      : ctx(c), gws(c->split_workspace(), tdvp_ctx_s::SPLIT_WS_BYTES), ws1(c), ws2(c), xf(c), yf(c), conv(c), work(c), work2(c), tau(c), tmpA(c), tmpB(c), tmpC(c),
        dvec(c), wsk(c), nsg(c), nst(c), cinv(c), pidx(c), prow(c), xp(c), segd(c), sc(c), lz(c), maps(&map_cache(c)) {}
  // split-K scratch for products whose output is ml x mr (or smaller)
  SplitWS split(long long ml, long long mr, int cb) {
    const size_t b = (size_t)16 * 2 * ml * mr * cb;
    wsk.ensure(b);
    return SplitWS{wsk.p, b};
  }
};

// site tensor in the working precision (a converted copy for FP32)
template <typename T>
const void* site_in(tdvp_ctx_s* ctx, const void* z, long long n, DBuf& conv) {
  if (sizeof(T) == 8) return z;
  conv.ensure((size_t)n * 8);
  kern::z2c(ctx->stream, conv.p, z, n);
  return conv.p;
}

// C = A B for complex128 row-major (A: M x K, B: K x N) into a fresh buffer
void zmatmul(tdvp_ctx_s* ctx, int opa, int opb, int M, int N, int K, const void* A, long long lda, const void* B,
             long long ldb, DBuf& out) {
  out.ensure((size_t)M * N * ZB);
  kern::gemm<double>(ctx->stream, opa, opb, M, N, K, 1.0, A, lda, 0, B, ldb, 0, 0.0, out.p, N, 0, 1);
}

// C = alpha op(A) op(B) + beta C (complex128, row-major) where the logical
// rows, summed index and columns carry the charges qm, qk, qn (any may be
// null: dense).  With all three, the product walks only the blocks of equal
// charge (the operands' other entries are exact zeros).
void qgemm(Work& W, int opa, int opb, int M, int N, int K, zc alpha, const void* A, long long lda, const void* B,
           long long ldb, zc beta, void* C, long long ldc, const std::vector<int>* qm, const std::vector<int>* qk,
           const std::vector<int>* qn) {
  ::qgemm(W.ctx, W.maps, opa, opb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, qm, qk, qn);
}

// Newton-Schulz orthonormalisation: for A with nearly orthonormal columns,
// A <- A (3 I - A^dagger A) / 2 keeps the column span and squares the
// deviation from orthonormality at every step (GEMMs only).
// With charges: qr those of the rows, qc of the columns.
void ns_cols(Work& W, void* A, int rows, int n, int iters, const std::vector<int>* qr = nullptr,
             const std::vector<int>* qc = nullptr) {
  tdvp_ctx_s* ctx = W.ctx;
  hipStream_t s = ctx->stream;
  W.nsg.ensure((size_t)n * n * ZB);
  W.nst.ensure((size_t)rows * n * ZB);
  for (int it = 0; it < iters; ++it) {
    qgemm(W, TDVP_OP_C, TDVP_OP_N, n, n, rows, 1.0, A, n, A, n, 0.0, W.nsg.p, n, qc, qr, qc);
    kern::zshift_diag(s, W.nsg.p, n, -0.5, 1.5);
    qgemm(W, TDVP_OP_N, TDVP_OP_N, rows, n, n, 1.0, A, n, W.nsg.p, n, 0.0, W.nst.p, n, qr, qc, qc);
    HIP_CHECK(hipMemcpyAsync(A, W.nst.p, (size_t)rows * n * ZB, hipMemcpyDeviceToDevice, s));
  }
}

// Same for nearly orthonormal rows: B <- (3 I - B B^dagger) B / 2.
// With charges: qr those of the rows, qc of the columns.
void ns_rows(Work& W, void* B, int n, int cols, int iters, const std::vector<int>* qr = nullptr,
             const std::vector<int>* qc = nullptr) {
  tdvp_ctx_s* ctx = W.ctx;
  hipStream_t s = ctx->stream;
  W.nsg.ensure((size_t)n * n * ZB);
  W.nst.ensure((size_t)n * cols * ZB);
  for (int it = 0; it < iters; ++it) {
    qgemm(W, TDVP_OP_N, TDVP_OP_C, n, n, cols, 1.0, B, cols, B, cols, 0.0, W.nsg.p, n, qr, qc, qr);
    kern::zshift_diag(s, W.nsg.p, n, -0.5, 1.5);
    qgemm(W, TDVP_OP_N, TDVP_OP_N, n, cols, n, 1.0, W.nsg.p, n, B, cols, 0.0, W.nst.p, cols, qr, qr, qc);
    HIP_CHECK(hipMemcpyAsync(B, W.nst.p, (size_t)n * cols * ZB, hipMemcpyDeviceToDevice, s));
  }
}

// rows[0..n) (each ncols complex128) permuted so that their charges q[0..n)
// ascend (stable); lam[0..n) and q[0..n) follow.  The new bond a basis of
// these rows spans then lists its charges in the order the states require.
void sort_rows_by_charge(Work& W, void* rows, long long ncols, int n, std::vector<double>* lam, std::vector<int>& q) {
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return q[a] < q[b]; });
  bool ident = true;
  for (int j = 0; j < n; ++j) ident = ident && perm[j] == j;
  if (!ident) {
    W.pidx.ensure(sizeof(int) * std::max(n, 1));
    upload(W.ctx, W.pidx.p, perm.data(), sizeof(int) * n);
    W.prow.ensure((size_t)n * ncols * ZB);
    kern::zgather(W.ctx->stream, W.prow.p, ncols, rows, ncols, W.pidx.as<int>(), n, nullptr, ncols);
    HIP_CHECK(hipMemcpyAsync(rows, W.prow.p, (size_t)n * ncols * ZB, hipMemcpyDeviceToDevice, W.ctx->stream));
    HIP_CHECK(hipStreamSynchronize(W.ctx->stream));   // `perm` is pageable host memory
  }
  std::vector<int> q2(n);
  std::vector<double> l2(n);
  for (int j = 0; j < n; ++j) {
    q2[j] = q[perm[j]];
    if (lam) l2[j] = (*lam)[perm[j]];
  }
  for (int j = 0; j < n; ++j) {
    q[j] = q2[j];
    if (lam) (*lam)[j] = l2[j];
  }
  q.resize(n);
}

// charges of the fused index (x, s) (x major) and of (s, x) (s major) for
// x with charges qx: q(x) + sign q(s)
std::vector<int> fuse_xs(const std::vector<int>& qx, int sign) {
  std::vector<int> out;
  out.reserve(2 * qx.size());
  for (int v : qx)
    for (int s = 0; s < 2; ++s) out.push_back(v + sign * phys_charge(s));
  return out;
}
std::vector<int> fuse_sx(const std::vector<int>& qx, int sign) {
  std::vector<int> out;
  out.reserve(2 * qx.size());
  for (int s = 0; s < 2; ++s)
    for (int v : qx) out.push_back(v + sign * phys_charge(s));
  return out;
}

// 1/sqrt of the first n weights on the device
const double* inv_sqrt_weights(Work& W, const std::vector<double>& lam, int n) {
  std::vector<double> f(n);
  for (int j = 0; j < n; ++j) f[j] = 1.0 / std::sqrt(std::max(lam[j], 1e-300));
  W.dvec.ensure(sizeof(double) * std::max(n, 1));
  upload(W.ctx, W.dvec.p, f.data(), sizeof(double) * n);
  HIP_CHECK(hipStreamSynchronize(W.ctx->stream));  // `f` is pageable host memory
  return W.dvec.as<double>();
}

// Truncated gauge moves.  The weights are the eigenvalues of the Gram matrix
// of C (= squared singular values) and the kept subspace is spanned by the
// leading eigenvectors, i.e. the leading singular subspace, so the cut and
// the truncated state are those of a truncated SVD; an orthonormal basis of
// the kept subspace then comes from one QR/LQ and the remainder factor is the
// exact projection of C on it.
int trunc_count(const std::vector<double>& lam, double eps, int chi_max, double* disc) {
  double tot = 0.0;
  for (double v : lam) tot += std::max(0.0, v);
  const int n = keep_count(lam, eps, tot, chi_max, 1);
  for (size_t j = n; j < lam.size(); ++j) *disc += std::max(0.0, lam[j]);
  return n;
}

// Exact gauge move of a charged C for which the Cholesky-QR steps failed (C
// rank deficient or badly conditioned; after a basis extension the new
// directions carry no weight).  left: C (rows x cols) = A R with A
// orthonormal columns (rows x k); right: C = L B with B orthonormal rows
// (k x cols).  The bond keeps, charge by charge, min(n_rows, n_cols) states
// plus completions borrowed from charges with room to spare, so that k =
// min(rows, cols) as in the dense move.  Its states: the range of C from the
// Gram eigendecomposition charge by charge (weights above 1e-14 of the
// largest, the numerical-zero rule), orthonormalised by Cholesky-QR, then
// for the rest of each charge seeded random vectors of that charge,
// projected out of the range twice and orthonormalised; every product walks
// the charge blocks only.  Returns k, or -1 when a step fails (the caller
// then factorises block by block with Householder reflections).
int factor_exact_u1(Work& W, bool left, const void* C, int rows, int cols, const std::vector<int>& qrow,
                    const std::vector<int>& qcol, DBuf& X1, DBuf& X2, std::vector<int>& qk) {
  Range r_(left ? "exact_u1.left" : "exact_u1.right");
  tdvp_ctx_s* ctx = W.ctx;
  hipStream_t s = ctx->stream;
  // the Gram index (its charges qg, size ng) and the other one (qo, no)
  const std::vector<int>& qg = left ? qcol : qrow;
  const std::vector<int>& qo = left ? qrow : qcol;
  const int ng = left ? cols : rows, no = left ? rows : cols;
  // states per charge: kb = min(count on the Gram side, count on the other),
  // plus completions where the Gram side has more than the other can hold
  std::map<int, int> cg, co, kt;
  for (int x : qg) ++cg[x];
  for (int x : qo) ++co[x];
  int deficit = 0;
  for (auto& kv : cg) deficit += std::max(0, kv.second - co[kv.first]);
  for (auto& kv : co) kt[kv.first] = std::min(kv.second, cg.count(kv.first) ? cg[kv.first] : 0);
  while (deficit > 0) {   // one at a time to the charge with the most room left
    int best = 0, room = 0;
    bool any = false;
    for (auto& kv : co) {
      const int r = kv.second - kt[kv.first];
      if (r > room) {
        room = r;
        best = kv.first;
        any = true;
      }
    }
    if (!any) break;
    ++kt[best];
    --deficit;
  }
  int k = 0;
  qk.clear();
  for (auto& kv : kt) {
    for (int j = 0; j < kv.second; ++j) qk.push_back(kv.first);
    k += kv.second;
  }
  if (k == 0) return -1;
  // Gram matrix and its eigendecomposition, charge by charge
  W.tmpA.ensure((size_t)ng * ng * ZB);
  W.tmpB.ensure((size_t)ng * ng * ZB);
  if (left) qgemm(W, TDVP_OP_C, TDVP_OP_N, ng, ng, no, 1.0, C, cols, C, cols, 0.0, W.tmpA.p, ng, &qg, &qo, &qg);
  else qgemm(W, TDVP_OP_N, TDVP_OP_C, ng, ng, no, 1.0, C, cols, C, cols, 0.0, W.tmpA.p, ng, &qg, &qo, &qg);
  std::vector<double> lam;
  std::vector<int> qv;
  la::eigh_sectors(ctx, W.tmpA.p, ng, qg, lam, W.tmpB.p, W.work2, qv);
  // range: weights above the floor, at most kt of each charge, ascending charge
  const double floor = 1e-14 * (lam.empty() ? 0.0 : std::max(lam[0], 0.0));
  std::map<int, int> used;
  std::vector<int> sel;
  for (int j = 0; j < ng; ++j)
    if (lam[j] > floor && lam[j] > 0.0 && used[qv[j]] < kt[qv[j]]) {
      ++used[qv[j]];
      sel.push_back(j);
    }
  std::stable_sort(sel.begin(), sel.end(), [&](int a, int b) { return qv[a] < qv[b]; });
  const int r = (int)sel.size();
  std::vector<int> qsel(r), qE;
  std::vector<double> lsel(r);
  for (int j = 0; j < r; ++j) {
    qsel[j] = qv[sel[j]];
    lsel[j] = lam[sel[j]];
  }
  for (auto& kv : kt)
    for (int j = used[kv.first]; j < kv.second; ++j) qE.push_back(kv.first);
  const int m = (int)qE.size();
  // positions of the range and random states in the bond (ascending charge,
  // range first within a charge)
  std::vector<int> pos_r(r), pos_e(m);
  {
    int p = 0, a = 0, b = 0;
    for (auto& kv : kt) {
      for (; a < r && qsel[a] == kv.first; ++a) pos_r[a] = p++;
      for (; b < m && qE[b] == kv.first; ++b) pos_e[b] = p++;
    }
  }
  std::vector<int> ints(sel);
  ints.insert(ints.end(), pos_r.begin(), pos_r.end());
  ints.insert(ints.end(), pos_e.begin(), pos_e.end());
  ints.insert(ints.end(), qo.begin(), qo.end());
  ints.insert(ints.end(), qE.begin(), qE.end());
  W.pidx.ensure(sizeof(int) * std::max<size_t>(1, ints.size()));
  upload(ctx, W.pidx.p, ints.data(), sizeof(int) * ints.size());
  const int* dsel = W.pidx.as<int>();
  const int* dpos_r = dsel + r;
  const int* dpos_e = dpos_r + r;
  const int* dqo = dpos_e + m;
  const int* dqE = dqo + no;
  // basis tensors: the range part Y (r states) and the random part E (m)
  const long long sz = (long long)std::max(r, m) * no;
  DBuf& Y = W.nst;
  W.prow.ensure((size_t)std::max(sz, 1LL) * ZB);
  W.tmpC.ensure((size_t)std::max(sz, 1LL) * ZB);
  Y.ensure((size_t)std::max(sz, 1LL) * ZB);
  DBuf Vs(ctx), Pm(ctx), Q(ctx), Rt(ctx);
  if (r > 0) {
    Vs.ensure((size_t)r * ng * ZB);
    kern::zgather(s, Vs.p, ng, W.tmpB.p, ng, dsel, r, nullptr, ng);
    const double* f = inv_sqrt_weights(W, lsel, r);
    if (left) {   // Y = C V_sel^dagger S^-1 (rows x r), then orthonormal columns
      qgemm(W, TDVP_OP_N, TDVP_OP_C, no, r, ng, 1.0, C, cols, Vs.p, ng, 0.0, W.tmpC.p, r, &qo, &qg, &qsel);
      kern::zscale_cols(s, W.tmpC.p, r, W.tmpC.p, r, no, r, f);
      Rt.ensure((size_t)r * r * ZB);
      if (!la::cholqr2_rowmajor(ctx, W.tmpC.p, no, r, Y.p, Rt.p, W.work, nullptr, &qsel, &qo, W.maps)) return -1;
    } else {      // Y = S^-1 U_sel^dagger C (r x cols), then orthonormal rows
      qgemm(W, TDVP_OP_N, TDVP_OP_N, r, no, ng, 1.0, Vs.p, ng, C, cols, 0.0, W.tmpC.p, no, &qsel, &qg, &qo);
      kern::zscale_rows(s, W.tmpC.p, no, W.tmpC.p, no, r, no, f);
      Rt.ensure((size_t)r * r * ZB);
      if (!la::cholqr2_rows_rowmajor(ctx, W.tmpC.p, r, no, Rt.p, Y.p, W.work, nullptr, &qsel, &qo, W.maps)) return -1;
    }
  }
  X1.ensure((size_t)(left ? no : rows) * k * ZB);
  X2.ensure((size_t)k * (left ? cols : no) * ZB);
  void* basis = left ? X1.p : X2.p;   // A (rows x k) or B (k x cols)
  kern::zfill(s, basis, zc(0.0, 0.0), (long long)no * k, 16);
  if (r > 0) {
    if (left) kern::zscatter_cols(s, basis, k, Y.p, r, no, dpos_r, r);
    else kern::zscatter(s, basis, no, Y.p, no, dpos_r, r, nullptr, no);
  }
  if (m > 0) {
    // random states of each charge, projected out of the range twice
    Q.ensure((size_t)m * no * ZB);
    const unsigned long long seed = 0x5eedull ^ ((unsigned long long)no << 32) ^ (unsigned long long)(k * 131 + m);
    if (left) kern::zrandom_blocks(s, W.prow.p, no, m, dqo, dqE, seed);
    else kern::zrandom_blocks(s, W.prow.p, m, no, dqE, dqo, seed);
    if (r > 0) {
      Pm.ensure((size_t)r * m * ZB);
      for (int pass = 0; pass < 2; ++pass) {
        if (left) {
          qgemm(W, TDVP_OP_C, TDVP_OP_N, r, m, no, 1.0, Y.p, r, W.prow.p, m, 0.0, Pm.p, m, &qsel, &qo, &qE);
          qgemm(W, TDVP_OP_N, TDVP_OP_N, no, m, r, -1.0, Y.p, r, Pm.p, m, 1.0, W.prow.p, m, &qo, &qsel, &qE);
        } else {
          qgemm(W, TDVP_OP_N, TDVP_OP_C, m, r, no, 1.0, W.prow.p, no, Y.p, no, 0.0, Pm.p, r, &qE, &qo, &qsel);
          qgemm(W, TDVP_OP_N, TDVP_OP_N, m, no, r, -1.0, Pm.p, r, Y.p, no, 1.0, W.prow.p, no, &qE, &qsel, &qo);
        }
      }
    }
    Rt.ensure((size_t)m * m * ZB);
    if (left) {
      if (!la::cholqr2_rowmajor(ctx, W.prow.p, no, m, Q.p, Rt.p, W.work, nullptr, &qE, &qo, W.maps)) return -1;
      kern::zscatter_cols(s, basis, k, Q.p, m, no, dpos_e, m);
    } else {
      if (!la::cholqr2_rows_rowmajor(ctx, W.prow.p, m, no, Rt.p, Q.p, W.work, nullptr, &qE, &qo, W.maps)) return -1;
      kern::zscatter(s, basis, no, Q.p, no, dpos_e, m, nullptr, no);
    }
  }
  // the other factor: R = A^dagger C, or L = C B^dagger
  if (left) qgemm(W, TDVP_OP_C, TDVP_OP_N, k, cols, rows, 1.0, X1.p, k, C, cols, 0.0, X2.p, cols, &qk, &qo, &qg);
  else qgemm(W, TDVP_OP_N, TDVP_OP_C, rows, k, cols, 1.0, C, cols, X2.p, cols, 0.0, X1.p, k, &qg, &qo, &qk);
  HIP_CHECK(hipStreamSynchronize(s));   // the local buffers die here
  return k;
}

// Gauge move to the right: C (ml x 2 x mr) -> A (ml x 2 x k) and R (k x mr).
// With charges: qc (mr entries) are the charges the columns of C carry as a
// left bond (for a site tensor, those of its right bond); the new bond's
// charges (ascending) go to *qk.  Every factorisation then respects the
// blocks: the Cholesky-QR steps and Newton-Schulz keep zero blocks exactly
// zero, and the Gram eigendecomposition runs charge by charge.
int split_left(Work& W, const double* C, int ml, int mr, double eps, int chi_max, DBuf& A, DBuf& R, double* disc,
               const std::vector<int>* qa = nullptr, const std::vector<int>* qc = nullptr,
               std::vector<int>* qk = nullptr) {
  tdvp_ctx_s* ctx = W.ctx;
  hipStream_t s = ctx->stream;
  const int rows = 2 * ml, cols = mr, kk = std::min(rows, cols);
  Range r_("gauge.split_left");
  const bool sym = qc != nullptr;
  // the exact moves keep the columns as the new bond: with charges only when
  // they ascend and C has at least as many rows as columns
  const bool keep_cols = !sym || (std::is_sorted(qc->begin(), qc->end()) && rows >= cols);
  std::vector<int> qrow;   // charges of the rows (a, s) of C
  if (sym) qrow = fuse_xs(*qa, 1);
  const std::vector<int>* qrp = sym ? &qrow : nullptr;
  if (eps == 0.0 && kk <= chi_max) {
    Range r1_("split_left.exact");
    if (keep_cols) {
      A.ensure((size_t)rows * kk * ZB);
      R.ensure((size_t)kk * cols * ZB);
      if (la::cholqr2_rowmajor(ctx, C, rows, cols, A.p, R.p, W.work, nullptr, qc, qrp, W.maps)) {
        if (sym) *qk = *qc;
        return kk;
      }
    }
    if (!sym) {
      A.ensure((size_t)rows * kk * ZB);
      R.ensure((size_t)kk * cols * ZB);
      la::qr_rowmajor(ctx, C, rows, cols, A.p, R.p, W.work, W.tau);
      return kk;
    }
    // rank-deficient (or not ordered by charge): Householder per charge
    // block, which keeps every direction of the bond, weight or not (the
    // extension's new directions carry none until the sweep evolves into them)
    const int kx = factor_exact_u1(W, true, C, rows, cols, qrow, *qc, A, R, *qk);
    if (kx > 0) return kx;
    Range r2_("split_left.sectors");
    return la::factor_sectors(ctx, true, C, rows, cols, fuse_xs(*qa, 1), *qc, A, R, *qk);
  }
  if (rows < cols) {
    // fewer rows: the left singular vectors straight from the eigenvectors
    // of G = C C^dagger (rows x rows), A = U_n, R = A^dagger C (orthonormal
    // to rounding; no weights divided out)
    Range r1_("split_left.rows_gram");
    W.tmpA.ensure((size_t)rows * rows * ZB);
    W.tmpB.ensure((size_t)rows * rows * ZB);
    qgemm(W, TDVP_OP_N, TDVP_OP_C, rows, rows, cols, 1.0, C, cols, C, cols, 0.0, W.tmpA.p, rows, qrp, qc, qrp);
    std::vector<double> lam;
    std::vector<int> qv;
    if (sym) la::eigh_sectors(ctx, W.tmpA.p, rows, qrow, lam, W.tmpB.p, W.work2, qv);
    else la::eigh_rows_desc(ctx, W.tmpA.p, rows, lam, W.tmpB.p, W.work2);
    const int n = std::min(trunc_count(lam, eps, chi_max, disc), kk);
    if (sym) {
      sort_rows_by_charge(W, W.tmpB.p, rows, n, &lam, qv);
      *qk = qv;
    }
    const std::vector<int>* qkp = sym ? qk : nullptr;
    A.ensure((size_t)rows * n * ZB);
    R.ensure((size_t)n * cols * ZB);
    kern::zconjtrans(s, A.p, n, W.tmpB.p, rows, rows, n);   // A[:, j] = (row j of U^dagger)^dagger
    qgemm(W, TDVP_OP_N, TDVP_OP_N, n, cols, rows, 1.0, W.tmpB.p, rows, C, cols, 0.0, R.p, cols, qkp, qrp, qc);
    return n;
  }
  // G = C^dagger C (cols x cols); rows of V^dagger from its eigendecomposition
  W.tmpA.ensure((size_t)cols * cols * ZB);
  W.tmpB.ensure((size_t)cols * cols * ZB);
  {
    Range r1_("split_left.gram");
    qgemm(W, TDVP_OP_C, TDVP_OP_N, cols, cols, rows, 1.0, C, cols, C, cols, 0.0, W.tmpA.p, cols, qc, qrp, qc);
  }
  // Nothing is cut when the smallest weight exceeds max(eps, floor) times
  // their sum (the cap does not bind: kk <= chi_max); a Cholesky factorisation
  // certifies it, and the exact factorisation is then the split.
  if (kk == cols && kk <= chi_max && keep_cols) {
    Range r1_("split_left.certified");
    const void* F = la::gram_floor_certified(ctx, W.tmpB.p, cols, std::max(eps, 1e-14), false,
                                             W.cinv.ensure((size_t)cols * cols * ZB), W.work, W.tmpA.p, qc);
    if (F) {
      A.ensure((size_t)rows * kk * ZB);
      R.ensure((size_t)kk * cols * ZB);
      if (la::cholqr2_rowmajor(ctx, C, rows, cols, A.p, R.p, W.work, F, qc, qrp, W.maps)) {
        if (sym) *qk = *qc;
        return kk;
      }
    }
  }
  std::vector<double> lam;
  std::vector<int> qv;
  Range r2_("split_left.eigh");
  if (sym) la::eigh_sectors(ctx, W.tmpA.p, cols, *qc, lam, W.tmpB.p, W.work2, qv);
  else la::eigh_rows_desc(ctx, W.tmpA.p, cols, lam, W.tmpB.p, W.work2);
  const int n = std::min(trunc_count(lam, eps, chi_max, disc), kk);
  const bool well_separated = lam[n - 1] > 1e-8 * lam[0];
  if (sym) {
    sort_rows_by_charge(W, W.tmpB.p, cols, n, &lam, qv);
    *qk = qv;
  }
  Range r3_("split_left.basis");
  // A spans C V_n; R = A^dagger C.  When every kept weight is well above the
  // eigenvector accuracy (u lambda_1 / lambda_n << 1), C V_n S_n^-1 is
  // orthonormal up to rounding and Newton-Schulz polishes it; otherwise a QR
  // of C V_n gives the orthonormal basis.
  W.tmpC.ensure((size_t)rows * n * ZB);
  const std::vector<int>* qkp = sym ? qk : nullptr;
  qgemm(W, TDVP_OP_N, TDVP_OP_C, rows, n, cols, 1.0, C, cols, W.tmpB.p, cols, 0.0, W.tmpC.p, n, qrp, qc, qkp);
  A.ensure((size_t)rows * n * ZB);
  R.ensure((size_t)n * cols * ZB);
  // (Newton-Schulz converges while the starting deviation is below ~1/2; for
  // small kept weights five steps and a check, with a QR when the check fails)
  kern::zscale_cols(s, A.p, n, W.tmpC.p, n, rows, n, inv_sqrt_weights(W, lam, n));
  if (well_separated) {
    ns_cols(W, A.p, rows, n, 3, qrp, qkp);
  } else {
    ns_cols(W, A.p, rows, n, 5, qrp, qkp);
    if (!(la::orth_defect(ctx, A.p, rows, n, false, W.work) <= 1e-20)) {
      W.tmpA.ensure((size_t)n * n * ZB);
      // with charges the Cholesky-QR steps keep the blocks (Householder
      // reflections would mix them)
      if (!sym) la::qr_rowmajor(ctx, W.tmpC.p, rows, n, A.p, W.tmpA.p, W.work, W.tau);
      else if (!la::cholqr2_rowmajor(ctx, W.tmpC.p, rows, n, A.p, W.tmpA.p, W.work, nullptr, qk, qrp, W.maps))
        TDVP_THROW(TDVP_ERR_NUMERIC, "gauge move: no orthonormal basis of the kept space");
    }
  }
  qgemm(W, TDVP_OP_C, TDVP_OP_N, n, cols, rows, 1.0, A.p, n, C, cols, 0.0, R.p, cols, qkp, qrp, qc);
  return n;
}

// Gauge move to the left: C (ml x 2 x mr) -> L (ml x k) and B (k x 2 x mr).
// With charges: qr (ml entries) are the charges the rows of C carry as a
// right bond (for a site tensor, those of its left bond); the new bond's
// charges (ascending) go to *qk.
int split_right(Work& W, const double* C, int ml, int mr, double eps, int chi_max, DBuf& L, DBuf& B, double* disc,
                const std::vector<int>* qr = nullptr, const std::vector<int>* qb = nullptr,
                std::vector<int>* qk = nullptr) {
  Range r_("gauge.split_right");
  tdvp_ctx_s* ctx = W.ctx;
  hipStream_t s = ctx->stream;
  const int rows = ml, cols = 2 * mr, kk = std::min(rows, cols);
  const bool sym = qr != nullptr;
  const bool keep_rows = !sym || (std::is_sorted(qr->begin(), qr->end()) && rows <= cols);
  std::vector<int> qcol;   // charges of the columns (s, b) of C as a left bond
  if (sym) qcol = fuse_sx(*qb, -1);
  const std::vector<int>* qcp = sym ? &qcol : nullptr;
  if (eps == 0.0 && kk <= chi_max) {
    Range r1_("split_right.exact");
    if (keep_rows) {
      L.ensure((size_t)rows * kk * ZB);
      B.ensure((size_t)kk * cols * ZB);
      if (la::cholqr2_rows_rowmajor(ctx, C, rows, cols, L.p, B.p, W.work, nullptr, qr, qcp, W.maps)) {
        if (sym) *qk = *qr;
        return kk;
      }
    }
    if (!sym) {
      L.ensure((size_t)rows * kk * ZB);
      B.ensure((size_t)kk * cols * ZB);
      la::lq_rowmajor(ctx, C, rows, cols, L.p, B.p, W.work, W.tau);
      return kk;
    }
    // as in split_left: LQ per charge block, every direction kept
    const int kx = factor_exact_u1(W, false, C, rows, cols, *qr, qcol, L, B, *qk);
    if (kx > 0) return kx;
    Range r2_("split_right.sectors");
    return la::factor_sectors(ctx, false, C, rows, cols, *qr, fuse_sx(*qb, -1), L, B, *qk);
  }
  if (cols < rows) {
    // fewer columns: the right singular vectors straight from the
    // eigenvectors of G = C^dagger C (cols x cols), B = V_n^dagger,
    // L = C B^dagger (orthonormal to rounding; no weights divided out)
    Range r1_("split_right.cols_gram");
    W.tmpA.ensure((size_t)cols * cols * ZB);
    W.tmpB.ensure((size_t)cols * cols * ZB);
    qgemm(W, TDVP_OP_C, TDVP_OP_N, cols, cols, rows, 1.0, C, cols, C, cols, 0.0, W.tmpA.p, cols, qcp, qr, qcp);
    std::vector<double> lam;
    std::vector<int> qv;
    if (sym) la::eigh_sectors(ctx, W.tmpA.p, cols, qcol, lam, W.tmpB.p, W.work2, qv);
    else la::eigh_rows_desc(ctx, W.tmpA.p, cols, lam, W.tmpB.p, W.work2);
    const int n = std::min(trunc_count(lam, eps, chi_max, disc), kk);
    if (sym) {
      sort_rows_by_charge(W, W.tmpB.p, cols, n, &lam, qv);
      *qk = qv;
    }
    const std::vector<int>* qkp = sym ? qk : nullptr;
    L.ensure((size_t)rows * n * ZB);
    B.ensure((size_t)n * cols * ZB);
    HIP_CHECK(hipMemcpyAsync(B.p, W.tmpB.p, (size_t)n * cols * ZB, hipMemcpyDeviceToDevice, s));
    qgemm(W, TDVP_OP_N, TDVP_OP_C, rows, n, cols, 1.0, C, cols, B.p, cols, 0.0, L.p, n, qr, qcp, qkp);
    return n;
  }
  // G = C C^dagger (rows x rows); rows of U^dagger from its eigendecomposition
  W.tmpA.ensure((size_t)rows * rows * ZB);
  W.tmpB.ensure((size_t)rows * rows * ZB);
  {
    Range r1_("split_right.gram");
    qgemm(W, TDVP_OP_N, TDVP_OP_C, rows, rows, cols, 1.0, C, cols, C, cols, 0.0, W.tmpA.p, rows, qr, qcp, qr);
  }
  // certified "nothing to cut" as in split_left
  if (kk == rows && kk <= chi_max && keep_rows) {
    Range r1_("split_right.certified");
    const void* F = la::gram_floor_certified(ctx, W.tmpB.p, rows, std::max(eps, 1e-14), true,
                                             W.cinv.ensure((size_t)rows * rows * ZB), W.work, W.tmpA.p, qr);
    if (F) {
      L.ensure((size_t)rows * kk * ZB);
      B.ensure((size_t)kk * cols * ZB);
      if (la::cholqr2_rows_rowmajor(ctx, C, rows, cols, L.p, B.p, W.work, F, qr, qcp, W.maps)) {
        if (sym) *qk = *qr;
        return kk;
      }
    }
  }
  std::vector<double> lam;
  std::vector<int> qv;
  Range r2_("split_right.eigh");
  if (sym) la::eigh_sectors(ctx, W.tmpA.p, rows, *qr, lam, W.tmpB.p, W.work2, qv);
  else la::eigh_rows_desc(ctx, W.tmpA.p, rows, lam, W.tmpB.p, W.work2);
  const int n = std::min(trunc_count(lam, eps, chi_max, disc), kk);
  const bool well_separated = lam[n - 1] > 1e-8 * lam[0];
  if (sym) {
    sort_rows_by_charge(W, W.tmpB.p, rows, n, &lam, qv);
    *qk = qv;
  }
  Range r3_("split_right.basis");
  // B spans the rows of U_n^dagger C; L = C B^dagger (Newton-Schulz on
  // S_n^-1 U_n^dagger C when the kept weights allow it, an LQ otherwise)
  W.tmpC.ensure((size_t)n * cols * ZB);
  const std::vector<int>* qkp = sym ? qk : nullptr;
  qgemm(W, TDVP_OP_N, TDVP_OP_N, n, cols, rows, 1.0, W.tmpB.p, rows, C, cols, 0.0, W.tmpC.p, cols, qkp, qr, qcp);
  L.ensure((size_t)rows * n * ZB);
  B.ensure((size_t)n * cols * ZB);
  kern::zscale_rows(s, B.p, cols, W.tmpC.p, cols, n, cols, inv_sqrt_weights(W, lam, n));
  if (well_separated) {
    ns_rows(W, B.p, n, cols, 3, qkp, qcp);
  } else {
    ns_rows(W, B.p, n, cols, 5, qkp, qcp);
    if (!(la::orth_defect(ctx, B.p, n, cols, true, W.work) <= 1e-20)) {
      W.tmpA.ensure((size_t)n * n * ZB);
      if (!sym) la::lq_rowmajor(ctx, W.tmpC.p, n, cols, W.tmpA.p, B.p, W.work, W.tau);
      else if (!la::cholqr2_rows_rowmajor(ctx, W.tmpC.p, n, cols, W.tmpA.p, B.p, W.work, nullptr, qk, qcp, W.maps))
        TDVP_THROW(TDVP_ERR_NUMERIC, "gauge move: no orthonormal basis of the kept space");
    }
  }
  qgemm(W, TDVP_OP_N, TDVP_OP_C, rows, n, cols, 1.0, C, cols, B.p, cols, 0.0, L.p, n, qr, qcp, qkp);
  return n;
}

void left_canonicalize(Work& W, tdvp_mps_s& psi) {
  Range r_("canonicalize.left");
  tdvp_ctx_s* ctx = W.ctx;
  DBuf A(ctx), R(ctx), nxt(ctx);
  double disc = 0.0;
  for (int i = 0; i + 1 < psi.N; ++i) {
    const int ml = psi.m[i], mr = psi.m[i + 1];
    std::vector<int> qk;
    const int k = split_left(W, psi.site(i), ml, mr, 0.0, 1 << 30, A, R, &disc, psi.u1() ? &psi.q[i] : nullptr,
                             psi.u1() ? &psi.q[i + 1] : nullptr, &qk);
    if (psi.u1()) psi.q[i + 1] = qk;
    std::swap(psi.t[i], A);
    zmatmul(ctx, TDVP_OP_N, TDVP_OP_N, k, 2 * psi.m[i + 2], mr, R.p, mr, psi.site(i + 1), 2LL * psi.m[i + 2], nxt);
    std::swap(psi.t[i + 1], nxt);
    psi.m[i + 1] = k;
  }
}

void right_canonicalize(Work& W, tdvp_mps_s& psi) {
  Range r_("canonicalize.right");
  tdvp_ctx_s* ctx = W.ctx;
  DBuf Lm(ctx), B(ctx), prv(ctx);
  double disc = 0.0;
  for (int i = psi.N - 1; i > 0; --i) {
    const int ml = psi.m[i], mr = psi.m[i + 1];
    std::vector<int> qk;
    const int k = split_right(W, psi.site(i), ml, mr, 0.0, 1 << 30, Lm, B, &disc, psi.u1() ? &psi.q[i] : nullptr,
                              psi.u1() ? &psi.q[i + 1] : nullptr, &qk);
    if (psi.u1()) psi.q[i] = qk;
    std::swap(psi.t[i], B);
    zmatmul(ctx, TDVP_OP_N, TDVP_OP_N, 2 * psi.m[i - 1], k, ml, psi.site(i - 1), ml, Lm.p, k, prv);
    std::swap(psi.t[i - 1], prv);
    psi.m[i] = k;
  }
}

// Nonzero multiply-adds of the sparse MPO stage T2[a',s',be,b] = sum
// W[al,be,s',s] T1[a',al,s,b] when the bonds carry charges: per nonzero W
// entry, the (a', b) pairs with q(b) - q(s) = q(a') - q(al).
double wstage_macs(const std::vector<int>& ql, const std::vector<int>& qr, const std::vector<int>& qwl,
                   const std::vector<zc>& Wt, int wl, int wr) {
  std::map<int, double> nl, nr;
  for (int v : ql) nl[v] += 1;
  for (int v : qr) nr[v] += 1;
  double macs = 0.0;
  for (int a = 0; a < wl; ++a)
    for (int b = 0; b < wr; ++b)
      for (int sp = 0; sp < 2; ++sp)
        for (int sk = 0; sk < 2; ++sk) {
          if (Wt[(((size_t)a * wr + b) * 2 + sp) * 2 + sk] == zc(0.0, 0.0)) continue;
          const int shift = -qwl[a] + phys_charge(sk);
          for (auto& kv : nl) {
            auto it = nr.find(kv.first + shift);
            if (it != nr.end()) macs += kv.second * it->second;
          }
        }
  return macs;
}

// Block-sparse maps of one contraction's two products, rebuilt per site.
// The allowed entries of a charged tensor viewed as rows x ncols: row r
// holds the columns of charge target[r], one contiguous range when the
// column charges qcol ascend.  host = b0[rows], len[rows], off[rows];
// np = total; ok false when qcol does not ascend.
struct RowSegments {
  std::vector<int> host;
  int rows = 0, maxlen = 0;
  long long np = 0;
  bool ok = false;
};
RowSegments row_segments(const std::vector<int>& target, const std::vector<int>& qcol) {
  RowSegments g;
  if (!std::is_sorted(qcol.begin(), qcol.end())) return g;
  std::map<int, std::pair<int, int>> rng;
  for (int b = 0; b < (int)qcol.size();) {
    int e = b + 1;
    while (e < (int)qcol.size() && qcol[e] == qcol[b]) ++e;
    rng[qcol[b]] = {b, e};
    b = e;
  }
  g.rows = (int)target.size();
  g.host.assign(3 * (size_t)g.rows, 0);
  long long off = 0;
  for (int r = 0; r < g.rows; ++r) {
    const auto it = rng.find(target[r]);
    const int b0 = it == rng.end() ? 0 : it->second.first, len = it == rng.end() ? 0 : it->second.second - b0;
    g.host[r] = b0;
    g.host[g.rows + r] = len;
    g.host[2 * g.rows + r] = (int)off;
    off += len;
    g.maxlen = std::max(g.maxlen, len);
  }
  g.np = off;
  g.ok = off < (1LL << 31);
  return g;
}

// Lanczos exponential of a charged tensor x (rows x ld, dense, exact zeros
// outside its blocks) on the allowed entries only: the Krylov vectors hold
// g.np entries (about a third of the dense size for the cylinder bonds);
// each product unpacks its input into a dense buffer of the working
// precision (zero outside the blocks, cleared once), applies `dense_mv`
// and packs the result.
template <typename T, class MV>
int lanczos_packed(Work& W, const RowSegments& g, void* x, long long n, long long ld, MV&& dense_mv, zc step,
                   double tol, int maxit, bool normalize, bool* unconv, MatvecTimer* timer) {
  tdvp_ctx_s* ctx = W.ctx;
  hipStream_t s = ctx->stream;
  const int cb = cbytes<T>();
  W.segd.ensure(sizeof(int) * g.host.size());
  upload(ctx, W.segd.p, g.host.data(), sizeof(int) * g.host.size());
  const int* seg = W.segd.as<int>();
  W.xp.ensure((size_t)g.np * ZB);
  W.xf.ensure((size_t)n * cb);
  W.yf.ensure((size_t)n * cb);
  kern::zfill(s, W.xf.p, zc(0.0, 0.0), n, cb);
  kern::pack_rows(s, W.xp.p, ZB, x, ZB, g.rows, ld, seg, g.maxlen);
  auto mv = [&](const void* in, void* out) {
    kern::unpack_rows(s, W.xf.p, cb, in, ZB, g.rows, ld, seg, g.maxlen);
    dense_mv(W.xf.p, W.yf.p);
    kern::pack_rows(s, out, ZB, W.yf.p, cb, g.rows, ld, seg, g.maxlen);
  };
  const int napp = W.lz.run(mv, W.xp.p, g.np, step, tol, maxit, normalize, unconv, timer);
  kern::unpack_rows(s, x, ZB, W.xp.p, ZB, g.rows, ld, seg, g.maxlen);
  HIP_CHECK(hipStreamSynchronize(s));   // `g.host` may be pageable memory that dies after the return
  return napp;
}

// launchable copies of the two maps of a contraction (valid while the
// entries stay in the cache: for the next MapCache::PROTECT lookups)
struct PairMaps {
  kern::KMap g1, g2;
  explicit PairMaps(tdvp_ctx_s*) {}
  ProdMaps set(tdvp_ctx_s* ctx, const MapEntry& a, const MapEntry& b) {
    MapCache& c = map_cache(ctx);
    g1 = c.use(a);
    g2 = c.use(b);
    return ProdMaps{&g1, &g2, a.exact_flops + b.exact_flops};
  }
  ProdMaps set(tdvp_ctx_s* ctx, std::pair<const MapEntry*, const MapEntry*> ab) { return set(ctx, *ab.first, *ab.second); }
};

template <typename T>
void sweep_impl(tdvp_ctx_s* ctx, tdvp_mps_s& psi, const tdvp_mpo_s& H, const tdvp_sweep_params& p,
                tdvp_sweep_stats& st) {
  const int N = psi.N;
  const int cb = cbytes<T>();
  const zc dt(p.dt_re, p.dt_im), half = 0.5 * dt;
  Work W(ctx);
  std::vector<DBuf> L, R;
  for (int i = 0; i <= N; ++i) {
    L.emplace_back(ctx);
    R.emplace_back(ctx);
  }
  set_one(ctx, L[0], cb);
  set_one(ctx, R[N], cb);
  MatvecTimer timer;
  timer.ctx = ctx;
  timer.on = true;
  auto ensure_ws = [&](int ml, int wl, int wr, int mr) {
    const size_t need = (size_t)2 * ml * mr * std::max(wl, wr) * cb;
    W.ws1.ensure(need);
    W.ws2.ensure(need);
  };
  // with charges, every product walks only its nonzero blocks
  const bool sym = psi.u1();
  PairMaps hmap(ctx), kmap(ctx), emap(ctx);
  const auto& qw = H.host.qw;
  auto build_R = [&](int i) {  // Rt[i] from Rt[i+1] and site i
    Range r_("sweep.env_right");
    const int ml = psi.m[i], mr = psi.m[i + 1], wl = H.w(i), wr = H.w(i + 1);
    ensure_ws(ml, wl, wr, mr);
    R[i].ensure((size_t)wl * ml * ml * cb);
    const void* Bt = site_in<T>(ctx, psi.site(i), psi.elems(i), W.conv);
    ProdMaps pm;
    kern::WCharges wcs;
    if (sym) {
      MapCache& mc = map_cache(ctx);
      pm = emap.set(ctx, cmap_env_right_gemm1_nz(mc, psi.q[i], psi.q[i + 1], qw[i + 1], psi.q[i + 1]),
                    cmap_env_right_gemm3(mc, psi.q[i], qw[i], psi.q[i + 1], psi.q[i]));
      wcs = wc_of(cmap_wstage(mc, psi.q[i], psi.q[i + 1], qw[i + 1], qw[i], +1), ml, mr, wr);
      pm.wc = &wcs;
    }
    env_right<T>(ctx, H.tab[i], ml, wl, wr, mr, R[i + 1].p, Bt, R[i].p, W.ws1.p, W.ws2.p, {}, pm);
  };
  auto build_L = [&](int i) {  // L[i+1] from L[i] and site i
    Range r_("sweep.env_left");
    const int ml = psi.m[i], mr = psi.m[i + 1], wl = H.w(i), wr = H.w(i + 1);
    ensure_ws(ml, wl, wr, mr);
    L[i + 1].ensure((size_t)mr * wr * mr * cb);
    const void* At = site_in<T>(ctx, psi.site(i), psi.elems(i), W.conv);
    ProdMaps pm;
    kern::WCharges wcs;
    if (sym) {
      MapCache& mc = map_cache(ctx);
      pm = emap.set(ctx, cmap_env_gemm1_nz(mc, psi.q[i], psi.q[i], qw[i], psi.q[i + 1]),
                    cmap_env_left_gemm2(mc, psi.q[i], psi.q[i + 1], psi.q[i + 1], qw[i + 1]));
      wcs = wc_of(cmap_wstage(mc, psi.q[i], psi.q[i + 1], qw[i], qw[i + 1]), ml, mr, wl);
      pm.wc = &wcs;
    }
    env_left<T>(ctx, H.tab[i], ml, wl, wr, mr, L[i].p, At, L[i + 1].p, W.ws1.p, W.ws2.p, W.split(ml, mr, cb), pm);
  };
  auto stepinfo = [&](int napp, bool unconv) {
    st.max_lanczos = std::max(st.max_lanczos, napp);
    if (unconv) ++st.n_unconverged;   // strict mode reports it once the sweep is complete
  };
  auto evolve_site = [&](int i, zc step) {
    Range r_("sweep.site_evolution");
    const int ml = psi.m[i], mr = psi.m[i + 1], wl = H.w(i), wr = H.w(i + 1);
    const long long n = psi.elems(i);
    ensure_ws(ml, wl, wr, mr);
    double flops = 8.0 * ((double)ml * wl * ml * 2 * mr + (double)H.tab[i].nnz * ml * mr +
                          (double)2 * ml * wr * mr * mr);
    ProdMaps pm;
    kern::WCharges wcs;
    if (sym) {
      MapCache& mc = map_cache(ctx);
      pm = hmap.set(ctx, cmap_env_gemm1_nz(mc, psi.q[i], psi.q[i], qw[i], psi.q[i + 1]),
                    cmap_heff_gemm2(mc, psi.q[i], psi.q[i + 1], qw[i + 1], psi.q[i + 1]));
      wcs = wc_of(cmap_wstage(mc, psi.q[i], psi.q[i + 1], qw[i], qw[i + 1]), ml, mr, wl);
      // the stage's outputs of other charges are cleared once here and
      // never stored by the matvecs of this site (nothing else writes ws2
      // until the site's Lanczos run ends)
      kern::zfill(ctx->stream, W.ws2.p, zc(0.0, 0.0), 2LL * ml * wr * mr, cb);
      wcs.zeros_kept = 1;
      pm.wc = &wcs;
      flops = pm.flops + 8.0 * wstage_macs(psi.q[i], psi.q[i + 1], qw[i], H.host.W[i], wl, wr);
    }
    const SplitWS sk = W.split(ml, mr, cb);
    auto mv = [&](const void* in, void* out) {
      if (sizeof(T) == 8) {
        heff_apply<T>(ctx, H.tab[i], ml, wl, wr, mr, L[i].p, R[i + 1].p, in, out, W.ws1.p, W.ws2.p, &timer, sk, pm);
      } else {
        W.xf.ensure((size_t)n * 8);
        W.yf.ensure((size_t)n * 8);
        kern::z2c(ctx->stream, W.xf.p, in, n);
        heff_apply<T>(ctx, H.tab[i], ml, wl, wr, mr, L[i].p, R[i + 1].p, W.xf.p, W.yf.p, W.ws1.p, W.ws2.p, &timer, sk,
                      pm);
        kern::c2z(ctx->stream, out, W.yf.p, n);
      }
      st.flops_matvec += flops;
    };
    bool unconv = false;
    int napp;
    RowSegments g;
    if (sym) {
      std::vector<int> tgt(2 * (size_t)ml);
      for (int a = 0; a < ml; ++a)
        for (int s2 = 0; s2 < 2; ++s2) tgt[2 * (size_t)a + s2] = psi.q[i][a] + phys_charge(s2);
      g = row_segments(tgt, psi.q[i + 1]);
    }
    if (g.ok && g.np > 0 && g.np < n) {
      auto dmv = [&](const void* in, void* out) {
        heff_apply<T>(ctx, H.tab[i], ml, wl, wr, mr, L[i].p, R[i + 1].p, in, out, W.ws1.p, W.ws2.p, &timer, sk, pm);
        st.flops_matvec += flops;
      };
      napp = lanczos_packed<T>(W, g, psi.site(i), n, mr, dmv, step, p.krylov_tol, p.krylov_max, p.normalize != 0,
                               &unconv, &timer);
    } else {
      napp = W.lz.run(mv, psi.site(i), n, step, p.krylov_tol, p.krylov_max, p.normalize != 0, &unconv, &timer);
    }
    st.n_matvec += napp;
    stepinfo(napp, unconv);
  };
  // X (ml x mr) pairs the bond basis of L[b] (charges qa) with that of Rt[b]
  // (charges qb): one of them is the basis before the gauge move
  auto evolve_bond = [&](int b, void* X, int ml, int mr, zc step, const std::vector<int>* qa,
                         const std::vector<int>* qb) {
    Range r_("sweep.bond_evolution");
    // K_eff on bond b with L[b] (ml x w x ml) and Rt[b] (w x mr x mr)
    const int w = H.w(b);
    const long long n = (long long)ml * mr;
    W.ws1.ensure((size_t)ml * w * mr * cb);
    const SplitWS sk = W.split(ml, mr, cb);
    ProdMaps pm;
    if (sym) {
      pm = kmap.set(ctx, cmap_keff(map_cache(ctx), *qa, *qb, qw[b]));
    }
    auto mv = [&](const void* in, void* out) {
      if (sizeof(T) == 8) {
        keff_apply<T>(ctx, ml, w, mr, L[b].p, R[b].p, in, out, W.ws1.p, sk, pm);
      } else {
        W.xf.ensure((size_t)n * 8);
        W.yf.ensure((size_t)n * 8);
        kern::z2c(ctx->stream, W.xf.p, in, n);
        keff_apply<T>(ctx, ml, w, mr, L[b].p, R[b].p, W.xf.p, W.yf.p, W.ws1.p, sk, pm);
        kern::c2z(ctx->stream, out, W.yf.p, n);
      }
    };
    bool unconv = false;
    int napp;
    RowSegments g;
    if (sym) g = row_segments(*qa, *qb);
    if (g.ok && g.np > 0 && g.np < n) {
      auto dmv = [&](const void* in, void* out) { keff_apply<T>(ctx, ml, w, mr, L[b].p, R[b].p, in, out, W.ws1.p, sk, pm); };
      napp = lanczos_packed<T>(W, g, X, n, mr, dmv, step, p.krylov_tol, p.krylov_max, p.normalize != 0, &unconv,
                               nullptr);
    } else {
      napp = W.lz.run(mv, X, n, step, p.krylov_tol, p.krylov_max, p.normalize != 0, &unconv, nullptr);
    }
    st.n_keff += napp;
    stepinfo(napp, unconv);
  };

  for (int i = N - 1; i >= 1; --i) build_R(i);
  DBuf A(ctx), Rm(ctx), nxt(ctx);
  // With eps = 0 the gauge moves are exact (unitary evolution needs them
  // so); chi_max caps the bonds only together with a cut eps > 0.
  const int cap = p.eps > 0.0 ? p.chi_max : (1 << 30);
  // left -> right
  for (int i = 0; i + 1 < N; ++i) {
    evolve_site(i, half);
    const int ml = psi.m[i], mr = psi.m[i + 1];
    std::vector<int> qk, qold;
    if (sym) qold = psi.q[i + 1];
    const int k = split_left(W, psi.site(i), ml, mr, p.eps, cap, A, Rm, &st.discarded,
                             psi.u1() ? &psi.q[i] : nullptr, psi.u1() ? &psi.q[i + 1] : nullptr, &qk);
    std::swap(psi.t[i], A);
    psi.m[i + 1] = k;  // site i is now ml x 2 x k; Rm is k x mr
    if (psi.u1()) psi.q[i + 1] = qk;
    build_L(i);
    evolve_bond(i + 1, Rm.p, k, mr, -half, &qk, &qold);
    zmatmul(ctx, TDVP_OP_N, TDVP_OP_N, k, 2 * psi.m[i + 2], mr, Rm.p, mr, psi.site(i + 1), 2LL * psi.m[i + 2], nxt);
    std::swap(psi.t[i + 1], nxt);
  }
  evolve_site(N - 1, dt);
  // right -> left
  for (int i = N - 1; i >= 1; --i) {
    if (i < N - 1) evolve_site(i, half);
    const int ml = psi.m[i], mr = psi.m[i + 1];
    std::vector<int> qk, qold;
    if (sym) qold = psi.q[i];
    const int k = split_right(W, psi.site(i), ml, mr, p.eps, cap, Rm, A, &st.discarded,
                              psi.u1() ? &psi.q[i] : nullptr, psi.u1() ? &psi.q[i + 1] : nullptr, &qk);
    std::swap(psi.t[i], A);
    psi.m[i] = k;  // site i is now k x 2 x mr; Rm (the L factor) is ml x k
    if (psi.u1()) psi.q[i] = qk;
    build_R(i);
    evolve_bond(i, Rm.p, ml, k, -half, &qold, &qk);
    zmatmul(ctx, TDVP_OP_N, TDVP_OP_N, 2 * psi.m[i - 1], k, ml, psi.site(i - 1), ml, Rm.p, k, nxt);
    std::swap(psi.t[i - 1], nxt);
  }
  if (N > 1) evolve_site(0, half);
  // energy at site 0
  {
    const int ml = psi.m[0], mr = psi.m[1];
    const long long n = psi.elems(0);
    ensure_ws(ml, H.w(0), H.w(1), mr);
    W.tmpC.ensure((size_t)n * ZB);
    if (sizeof(T) == 8) {
      heff_apply<T>(ctx, H.tab[0], ml, H.w(0), H.w(1), mr, L[0].p, R[1].p, psi.site(0), W.tmpC.p, W.ws1.p, W.ws2.p);
    } else {
      W.xf.ensure((size_t)n * 8);
      W.yf.ensure((size_t)n * 8);
      kern::z2c(ctx->stream, W.xf.p, psi.site(0), n);
      heff_apply<T>(ctx, H.tab[0], ml, H.w(0), H.w(1), mr, L[0].p, R[1].p, W.xf.p, W.yf.p, W.ws1.p, W.ws2.p);
      kern::c2z(ctx->stream, W.tmpC.p, W.yf.p, n);
    }
    const zc e = W.sc.dot(psi.site(0), W.tmpC.p, n);
    const double nn = W.sc.dot(psi.site(0), psi.site(0), n).real();
    st.energy = e.real() / nn;
  }
  st.ms_matvec = timer.ms;
  st.ms_heff_gemm = timer.gemm_ms;
  st.flops_heff_gemm = timer.gemm_flops;
  st.n_heff_gemm = timer.n_gemm;
}

// Two-site TDVP sweep (the comparison method of the cost statement in
// section I.C and of the benchmarks of section II): left to right over the
// pairs (i, i+1) with dt/2, right to left with dt/2, the last pair evolved
// once by dt; each pair is split by the truncated gauge move (eps, chi_max;
// zero weights and the cap only when eps = 0) and the new one-site center is
// evolved backwards by dt/2 except after the last pair of a half sweep.
// Pre- and postcondition: center at site 0, sites 1..N-1 right-canonical.
template <typename T>
void sweep2_impl(tdvp_ctx_s* ctx, tdvp_mps_s& psi, const tdvp_mpo_s& H, const tdvp_sweep_params& p,
                 tdvp_sweep_stats& st) {
  const int N = psi.N;
  if (N < 2) TDVP_THROW(TDVP_ERR_ARG, "two-site TDVP needs at least two sites");
  const int cb = cbytes<T>();
  const zc dt(p.dt_re, p.dt_im), half = 0.5 * dt;
  Work W(ctx);
  std::vector<DBuf> L, R;
  for (int i = 0; i <= N; ++i) {
    L.emplace_back(ctx);
    R.emplace_back(ctx);
  }
  set_one(ctx, L[0], cb);
  set_one(ctx, R[N], cb);
  MatvecTimer timer;
  timer.ctx = ctx;
  timer.on = true;
  auto ensure_ws = [&](size_t elems) {
    W.ws1.ensure(elems * cb);
    W.ws2.ensure(elems * cb);
  };
  auto build_R = [&](int i) {
    const int ml = psi.m[i], mr = psi.m[i + 1], wl = H.w(i), wr = H.w(i + 1);
    ensure_ws((size_t)2 * ml * mr * std::max(wl, wr));
    R[i].ensure((size_t)wl * ml * ml * cb);
    const void* Bt = site_in<T>(ctx, psi.site(i), psi.elems(i), W.conv);
    env_right<T>(ctx, H.tab[i], ml, wl, wr, mr, R[i + 1].p, Bt, R[i].p, W.ws1.p, W.ws2.p);
  };
  auto build_L = [&](int i) {
    const int ml = psi.m[i], mr = psi.m[i + 1], wl = H.w(i), wr = H.w(i + 1);
    ensure_ws((size_t)2 * ml * mr * std::max(wl, wr));
    L[i + 1].ensure((size_t)mr * wr * mr * cb);
    const void* At = site_in<T>(ctx, psi.site(i), psi.elems(i), W.conv);
    env_left<T>(ctx, H.tab[i], ml, wl, wr, mr, L[i].p, At, L[i + 1].p, W.ws1.p, W.ws2.p, W.split(ml, mr, cb));
  };
  auto stepinfo = [&](int napp, bool unconv) {
    st.max_lanczos = std::max(st.max_lanczos, napp);
    if (unconv) ++st.n_unconverged;   // strict mode reports it once the sweep is complete
  };
  // FP64 master in x; working-precision copies for the mixed paths
  auto run_lanczos = [&](void* x, long long n, zc step, auto&& apply_T, double flops, bool timed, auto* count) {
    auto mv = [&](const void* in, void* out) {
      if (sizeof(T) == 8) {
        apply_T(in, out);
      } else {
        W.xf.ensure((size_t)n * 8);
        W.yf.ensure((size_t)n * 8);
        kern::z2c(ctx->stream, W.xf.p, in, n);
        apply_T(W.xf.p, W.yf.p);
        kern::c2z(ctx->stream, out, W.yf.p, n);
      }
      st.flops_matvec += flops;
    };
    bool unconv = false;
    const int napp = W.lz.run(mv, x, n, step, p.krylov_tol, p.krylov_max, p.normalize != 0, &unconv,
                              timed ? &timer : nullptr);
    *count += napp;
    stepinfo(napp, unconv);
  };
  DBuf Th(ctx), A(ctx), Cn(ctx);
  auto form_pair = [&](int i) {  // Th = site(i) site(i+1), ml x 2 x 2 x mr
    const int ml = psi.m[i], mb = psi.m[i + 1], mr = psi.m[i + 2];
    zmatmul(ctx, TDVP_OP_N, TDVP_OP_N, 2 * ml, 2 * mr, mb, psi.site(i), mb, psi.site(i + 1), 2LL * mr, Th);
  };
  auto evolve_pair = [&](int i, zc step) {
    const int ml = psi.m[i], mr = psi.m[i + 2], wl = H.w(i), wm = H.w(i + 1), wr = H.w(i + 2);
    const long long n = 4LL * ml * mr;
    ensure_ws((size_t)4 * ml * mr * std::max(wl, std::max(wm, wr)));
    const SplitWS sk = W.split(2 * ml, 2 * mr, cb);
    const double flops = 8.0 * ((double)ml * wl * ml * 4 * mr + (double)H.tab[i].nnz * ml * 2 * mr +
                                (double)H.tab[i + 1].nnz * 2 * ml * mr + (double)4 * ml * wr * mr * mr);
    auto ap = [&](const void* in, void* out) {
      heff2_apply<T>(ctx, H.tab[i], H.tab[i + 1], ml, wl, wm, wr, mr, L[i].p, R[i + 2].p, in, out, W.ws1.p, W.ws2.p,
                     &timer, sk);
    };
    run_lanczos(Th.p, n, step, ap, flops, true, &st.n_matvec);
  };
  auto evolve_site = [&](int i, void* C, zc step) {
    const int ml = psi.m[i], mr = psi.m[i + 1], wl = H.w(i), wr = H.w(i + 1);
    const long long n = 2LL * ml * mr;
    ensure_ws((size_t)2 * ml * mr * std::max(wl, wr));
    const SplitWS sk = W.split(ml, mr, cb);
    const double flops = 8.0 * ((double)ml * wl * ml * 2 * mr + (double)H.tab[i].nnz * ml * mr +
                                (double)2 * ml * wr * mr * mr);
    auto ap = [&](const void* in, void* out) {
      heff_apply<T>(ctx, H.tab[i], ml, wl, wr, mr, L[i].p, R[i + 1].p, in, out, W.ws1.p, W.ws2.p, nullptr, sk);
    };
    run_lanczos(C, n, step, ap, flops, false, &st.n_keff);
  };
  // split Th (pair i) with the center moving right: site i = A, site i+1 = S V^dagger
  // with charges: the columns (s', b) of the pair carry q(b) - q(s') as a
  // left bond, the rows (a, s) carry q(a) + q(s) as a right bond
  auto split_to_right = [&](int i) {
    const int ml = psi.m[i], mr = psi.m[i + 2];
    std::vector<int> qc, qk;
    if (psi.u1()) qc = fuse_sx(psi.q[i + 2], -1);
    const int k = split_left(W, Th.as<double>(), ml, 2 * mr, p.eps, p.chi_max, A, Cn, &st.discarded,
                             psi.u1() ? &psi.q[i] : nullptr, psi.u1() ? &qc : nullptr, &qk);
    std::swap(psi.t[i], A);
    std::swap(psi.t[i + 1], Cn);
    psi.m[i + 1] = k;
    if (psi.u1()) psi.q[i + 1] = qk;
  };
  // ... with the center moving left: site i = U S, site i+1 = V^dagger
  auto split_to_left = [&](int i) {
    const int ml = psi.m[i], mr = psi.m[i + 2];
    std::vector<int> qr, qk;
    if (psi.u1()) qr = fuse_xs(psi.q[i], 1);
    const int k = split_right(W, Th.as<double>(), 2 * ml, mr, p.eps, p.chi_max, A, Cn, &st.discarded,
                              psi.u1() ? &qr : nullptr, psi.u1() ? &psi.q[i + 2] : nullptr, &qk);
    std::swap(psi.t[i], A);
    std::swap(psi.t[i + 1], Cn);
    psi.m[i + 1] = k;
    if (psi.u1()) psi.q[i + 1] = qk;
  };

  for (int i = N - 1; i >= 2; --i) build_R(i);
  // left -> right
  for (int i = 0; i + 1 < N; ++i) {
    form_pair(i);
    if (i + 2 < N) {
      evolve_pair(i, half);
      split_to_right(i);
      build_L(i);
      evolve_site(i + 1, psi.site(i + 1), -half);
    } else {
      evolve_pair(i, dt);  // merged with the first pair of the right-to-left half
      split_to_left(i);
      build_R(i + 1);
    }
  }
  // right -> left
  for (int i = N - 3; i >= 0; --i) {
    evolve_site(i + 1, psi.site(i + 1), -half);
    form_pair(i);
    evolve_pair(i, half);
    split_to_left(i);
    build_R(i + 1);
  }
  // energy at site 0 (fresh right environment of site 1 exists)
  {
    const int ml = psi.m[0], mr = psi.m[1];
    const long long n = psi.elems(0);
    ensure_ws((size_t)2 * ml * mr * std::max(H.w(0), H.w(1)));
    W.tmpC.ensure((size_t)n * ZB);
    if (sizeof(T) == 8) {
      heff_apply<T>(ctx, H.tab[0], ml, H.w(0), H.w(1), mr, L[0].p, R[1].p, psi.site(0), W.tmpC.p, W.ws1.p, W.ws2.p);
    } else {
      W.xf.ensure((size_t)n * 8);
      W.yf.ensure((size_t)n * 8);
      kern::z2c(ctx->stream, W.xf.p, psi.site(0), n);
      heff_apply<T>(ctx, H.tab[0], ml, H.w(0), H.w(1), mr, L[0].p, R[1].p, W.xf.p, W.yf.p, W.ws1.p, W.ws2.p);
      kern::c2z(ctx->stream, W.tmpC.p, W.yf.p, n);
    }
    const zc e = W.sc.dot(psi.site(0), W.tmpC.p, n);
    const double nn = W.sc.dot(psi.site(0), psi.site(0), n).real();
    st.energy = e.real() / nn;
  }
  st.ms_matvec = timer.ms;
  st.ms_heff_gemm = timer.gemm_ms;
  st.flops_heff_gemm = timer.gemm_flops;
  st.n_heff_gemm = timer.n_gemm;
}

// ---------------------------------------------------- density-matrix apply
// Right double-layer environment step: E_i from E_{i+1} and site i.
template <typename T>
void dl_env_step(tdvp_ctx_s* ctx, const SiteTables& tb, int ml, int wl, int wr, int mr, const void* M,
                 const void* E, void* Eout, DBuf& f1, DBuf& f2) {
  hipStream_t s = ctx->stream;
  const int cb = cbytes<T>();
  const long long q = (long long)wr * mr;
  f1.ensure((size_t)wr * 2 * ml * q * cb);
  f2.ensure((size_t)std::max<long long>((long long)wl * ml * 2 * q, (long long)wl * ml * wl * 2 * mr) * cb);
  // F1[y][(a,s),(Y,B)] = M[(a,s),b] E[y][b,(Y,B)]
  kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, 2 * ml, (int)q, mr, 1.0, M, mr, 0, E, q, (long long)mr * q, 0.0, f1.p, q,
                2LL * ml * q, wr);
  // F2[x,a,t,(Y,B)] = sum_{y,s} W[x,y,t,s] F1[y,a,s,(Y,B)]
  kern::wapply<T>(s, tb.B, f1.p, f2.p, ml, q, 2 * q, 1, 2LL * ml * q, q, 2 * q, 1, 2LL * ml * q, q);
  // F3[(x,a),X,S,B] = sum_{Y,t} conj(W[X,Y,t,S]) F2[(x,a),t,Y,B]  (into f1)
  f1.ensure((size_t)wl * ml * wl * 2 * mr * cb);
  kern::wapply<T>(s, tb.BH, f2.p, f1.p, (long long)wl * ml, mr, 2 * q, 1, mr, q, (long long)wl * 2 * mr, 1, 2LL * mr,
                  mr);
  // E[(x,a,X),A] = sum_{(S,B)} F3[(x,a,X),(S,B)] conj(M[A,(S,B)])
  kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_C, wl * ml * wl, ml, 2 * mr, 1.0, f1.p, 2LL * mr, 0, M, 2LL * mr, 0, 0.0, Eout,
                ml, 0, 1);
}

// out = normalise(trunc_{eps, chi_max}(op |in>)), left-canonical
template <typename T>
double denmat_apply(Work& W, const tdvp_mps_s& in, const tdvp_mpo_s& op, double eps, int chi_max, tdvp_mps_s& out) {
  tdvp_ctx_s* ctx = W.ctx;
  hipStream_t s = ctx->stream;
  const int N = in.N;
  const int cb = cbytes<T>();
  // working-precision copies of the input tensors.  The input is
  // left-canonical, so its norm sits in the last site; the output is
  // normalised and every cut is relative, so that site enters scaled to unit
  // norm (an unnormalised state would overflow FP32).
  std::vector<DBuf> Mt;
  std::vector<const void*> Mp(N);
  const double in_norm = W.sc.norm(in.site(N - 1), in.elems(N - 1));
  if (!(in_norm > 0.0) || !std::isfinite(in_norm)) TDVP_THROW(TDVP_ERR_NUMERIC, "MPS with zero or non-finite norm");
  for (int i = 0; i < N; ++i) {
    if (sizeof(T) == 8) {
      Mp[i] = in.site(i);
    } else {
      Mt.emplace_back(ctx);
      Mt.back().ensure((size_t)in.elems(i) * cb);
      if (i == N - 1) {
        W.tmpC.ensure((size_t)in.elems(i) * ZB);
        kern::zscale(s, W.tmpC.p, in.site(i), zc(1.0 / in_norm, 0.0), in.elems(i));
        kern::z2c(s, Mt.back().p, W.tmpC.p, in.elems(i));
      } else {
        kern::z2c(s, Mt.back().p, in.site(i), in.elems(i));
      }
      Mp[i] = Mt.back().p;
    }
  }
  std::vector<DBuf> E;
  for (int i = 0; i <= N; ++i) E.emplace_back(ctx);
  set_one(ctx, E[N], cb);
  DBuf f1(ctx), f2(ctx);
  for (int i = N - 1; i >= 1; --i) {
    const int ml = in.m[i], mr = in.m[i + 1], wl = op.w(i), wr = op.w(i + 1);
    E[i].ensure((size_t)wl * ml * wl * ml * cb);
    dl_env_step<T>(ctx, op.tab[i], ml, wl, wr, mr, Mp[i], E[i + 1].p, E[i].p, f1, f2);
  }
  out.ctx = ctx;
  out.N = N;
  out.m.assign(N + 1, 1);
  out.t.clear();
  for (int i = 0; i < N; ++i) out.t.emplace_back(ctx);
  // with charges: the output keeps the input's total charge; the bond k of
  // X carries out.q[i], and rho is block diagonal in q(k) + q(t)
  const bool sym = in.u1();
  out.q.clear();
  if (sym) {
    out.q.assign(N + 1, std::vector<int>());
    out.q[0] = in.q[0];
    out.q[N] = in.q[N];
  }
  DBuf X(ctx), Y(ctx), G(ctx), rho(ctx), rho64(ctx), rows(ctx), rowsT(ctx);
  set_one(ctx, X, cb);
  int kd = 1;
  double disc = 0.0;
  std::vector<double> lam;
  for (int i = 0; i < N; ++i) {
    const int ml = in.m[i], mr = in.m[i + 1], wl = op.w(i), wr = op.w(i + 1);
    const long long q = (long long)wr * mr;
    // Y[k,t,be,b] = sum X[k,al,a] M[a,s,b] W[al,be,t,s]
    f1.ensure((size_t)kd * wl * 2 * mr * cb);
    Y.ensure((size_t)kd * 2 * q * cb);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, kd * wl, 2 * mr, ml, 1.0, X.p, ml, 0, Mp[i], 2 * mr, 0, 0.0, f1.p, 2 * mr,
                  0, 1);
    kern::wapply<T>(s, op.tab[i].F, f1.p, Y.p, kd, mr, (long long)wl * 2 * mr, 1, 2LL * mr, mr, 2 * q, 1, mr, q);
    if (i == N - 1) {
      // last site: C[k,t] = Y[k,t,0,0]
      const long long n = 2LL * kd;
      out.t[i].ensure((size_t)n * ZB);
      if (sizeof(T) == 8)
        HIP_CHECK(hipMemcpyAsync(out.t[i].p, Y.p, n * ZB, hipMemcpyDeviceToDevice, s));
      else
        kern::c2z(s, out.t[i].p, Y.p, n);
      const double nr = W.sc.norm(out.t[i].p, n);
      if (!(nr > 0.0) || !std::isfinite(nr)) TDVP_THROW(TDVP_ERR_NUMERIC, "Krylov vector vanished or is not finite");
      kern::zscale(s, out.t[i].p, out.t[i].p, zc(1.0 / nr, 0.0), n);
      out.m[i] = kd;
      break;
    }
    // rho = Y E Y^dagger   (2kd x 2kd)
    const int d2 = 2 * kd;
    G.ensure((size_t)d2 * q * cb);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, d2, (int)q, (int)q, 1.0, Y.p, q, 0, E[i + 1].p, q, 0, 0.0, G.p, q, 0, 1);
    rho.ensure((size_t)d2 * d2 * cb);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_C, d2, d2, (int)q, 1.0, G.p, q, 0, Y.p, q, 0, 0.0, rho.p, d2, 0, 1);
    const void* r64 = rho.p;
    if (sizeof(T) != 8) {
      rho64.ensure((size_t)d2 * d2 * ZB);
      kern::c2z(s, rho64.p, rho.p, (long long)d2 * d2);
      r64 = rho64.p;
    }
    rows.ensure((size_t)d2 * d2 * ZB);
    std::vector<int> qv;
    if (sym) la::eigh_sectors(ctx, r64, d2, fuse_xs(out.q[i], 1), lam, rows.p, W.work, qv);
    else la::eigh_rows_desc(ctx, r64, d2, lam, rows.p, W.work);
    double tr = 0.0;
    for (double v : lam) tr += v;
    const int n = keep_count(lam, eps, tr, chi_max, 1);
    for (int j = n; j < d2; ++j) disc += std::max(0.0, lam[j]);
    if (sym) {
      sort_rows_by_charge(W, rows.p, d2, n, &lam, qv);
      out.q[i + 1] = qv;
    }
    // A_i[(k,t),n] = v_n  (conjugate transpose of the first n rows)
    out.t[i].ensure((size_t)d2 * n * ZB);
    kern::zconjtrans(s, out.t[i].p, n, rows.p, d2, d2, n);
    out.m[i + 1] = n;
    out.m[i] = kd;
    // X[n,(be,b)] = rows[0:n] Y
    const void* rw = rows.p;
    if (sizeof(T) != 8) {
      rowsT.ensure((size_t)n * d2 * cb);
      kern::z2c(s, rowsT.p, rows.p, (long long)n * d2);
      rw = rowsT.p;
    }
    X.ensure((size_t)n * q * cb);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, n, (int)q, d2, 1.0, rw, d2, 0, Y.p, q, 0, 0.0, X.p, q, 0, 1);
    kd = n;
  }
  out.m[0] = 1;
  out.m[N] = 1;
  HIP_CHECK(hipStreamSynchronize(s));
  return disc;
}

// ------------------------------------------------ variational MPO application
// Two-site fitting of |phi> ~ O|psi> (the variational route of section I.C,
// after Paeckel et al. 2019): mixed environments <phi|O|psi>, L[(a',al),a]
// with a' on phi and a on psi, Rt[ga][b,b'] with b on psi and b' on phi.
// Contractions in the working precision (FP64, or FP32 / BF16 inputs on
// the mixed paths); the two-site tensors are split in FP64.

// Lout[b',(be,b)] = sum conj(bra[a',s',b']) L[(a',al),a] W[al,be,s',s] ket[a,s,b]
template <typename T>
void fit_env_left(tdvp_ctx_s* ctx, const SiteTables& tb, int mlo, int mli, int wl, int wr, int mro, int mri,
                  const void* L, const void* bra, const void* ket, void* Lout, DBuf& f1, DBuf& f2, ProdMaps pm = {}) {
  Range r_("fit.env_left");
  hipStream_t s = ctx->stream;
  const int cb = cbytes<T>();
  f1.ensure((size_t)mlo * wl * 2 * mri * cb);
  f2.ensure((size_t)mlo * 2 * wr * mri * cb);
  // T1[(a',al),(s,b)] = L[(a',al),a] ket[a,(s,b)]
  if (pm.g1) {   // with charges: batched over al
    kern::KMapScope ks(pm.g1);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, mlo, 2 * mri, mli, 1.0, L, (long long)wl * mli, mli, ket, 2LL * mri, 0,
                       0.0, f1.p, (long long)wl * 2 * mri, 2LL * mri, wl);
  } else {
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, mlo * wl, 2 * mri, mli, 1.0, L, mli, 0, ket, 2LL * mri, 0, 0.0, f1.p,
                       2LL * mri, 0, 1);
  }
  // T2[a',s',be,b] = sum W[al,be,s',s] T1[a',al,s,b]
  kern::wapply<T>(s, tb.F, f1.p, f2.p, mlo, mri, (long long)wl * 2 * mri, 1, 2LL * mri, mri,
                       2LL * wr * mri, 1, mri, (long long)wr * mri, pm.wc);
  // Lout[b',(be,b)] = sum_{(a',s')} conj(bra[(a',s'),b']) T2[(a',s'),(be,b)]
  kern::KMapScope ks(pm.g2);
  kern::gemm<T>(s, TDVP_OP_C, TDVP_OP_N, mro, wr * mri, 2 * mlo, 1.0, bra, mro, 0, f2.p, (long long)wr * mri, 0,
                     0.0, Lout, (long long)wr * mri, 0, 1);
}

// Rout[al][a,a'] = sum conj(bra[a',s',b']) W[al,be,s',s] Rt[be][b,b'] ket[a,s,b]
template <typename T>
void fit_env_right(tdvp_ctx_s* ctx, const SiteTables& tb, int mlo, int mli, int wl, int wr, int mro, int mri,
                   const void* Rt, const void* bra, const void* ket, void* Rout, DBuf& f1, DBuf& f2,
                   ProdMaps pm = {}) {
  Range r_("fit.env_right");
  hipStream_t s = ctx->stream;
  const int cb = cbytes<T>();
  f1.ensure((size_t)wr * 2 * mli * mro * cb);
  f2.ensure((size_t)wl * 2 * mli * mro * cb);
  // U1[be][(a,s),b'] = ket[(a,s),b] Rt[be][b,b']   (batched over be)
  {
    kern::KMapScope ks(pm.g1);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, 2 * mli, mro, mri, 1.0, ket, mri, 0, Rt, mro, (long long)mri * mro, 0.0,
                  f1.p, mro, 2LL * mli * mro, wr);
  }
  // U2[al,a,s',b'] = sum W[al,be,s',s] U1[be,a,s,b']
  kern::wapply<T>(s, tb.B, f1.p, f2.p, mli, mro, 2LL * mro, 1, 2LL * mli * mro, mro, 2LL * mro, 1,
                       2LL * mli * mro, mro, pm.wc);
  // Rout[(al,a),a'] = sum_{(s',b')} U2[(al,a),(s',b')] conj(bra[a',(s',b')])
  kern::KMapScope ks(pm.g2);
  kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_C, wl * mli, mlo, 2 * mro, 1.0, f2.p, 2LL * mro, 0, bra, 2LL * mro, 0, 0.0,
                     Rout, mlo, 0, 1);
}

// Y[(a',t),(u,b')] = sum L[(a',al),a] W1[al,be,t,s] W2[be,ga,u,v] P[a,s,v,b] Rt[ga][b,b']:
// the two-site tensor of phi that is closest to O|psi> in the current bases.
template <typename T>
void fit_local2(tdvp_ctx_s* ctx, const SiteTables& t1, const SiteTables& t2, int mlo, int mli, int wl, int wm, int wr,
                int mri, int mro, const void* L, const void* Rt, const void* P, void* Y, DBuf& f1, DBuf& f2,
                ProdMaps pm = {}) {
  Range r_("fit.local");
  hipStream_t s = ctx->stream;
  const int cb = cbytes<T>();
  const long long big = std::max({(long long)mlo * wl * 4 * mri, (long long)mlo * 2 * wm * 2 * mri,
                                  (long long)mlo * 2 * 2 * wr * mri});
  f1.ensure((size_t)big * cb);
  f2.ensure((size_t)big * cb);
  // T1[(a',al),(s,v,b)] = L[(a',al),a] P[a,(s,v,b)]
  if (pm.g1) {   // with charges: batched over al
    kern::KMapScope ks(pm.g1);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, mlo, 4 * mri, mli, 1.0, L, (long long)wl * mli, mli, P, 4LL * mri, 0,
                       0.0, f1.p, (long long)wl * 4 * mri, 4LL * mri, wl);
  } else {
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, mlo * wl, 4 * mri, mli, 1.0, L, mli, 0, P, 4LL * mri, 0, 0.0, f1.p,
                       4LL * mri, 0, 1);
  }
  // T2[a',t,be,(v,b)] = sum W1[al,be,t,s] T1[a',al,s,(v,b)]
  kern::wapply<T>(s, t1.F, f1.p, f2.p, mlo, 2LL * mri, (long long)wl * 4 * mri, 1, 4LL * mri, 2LL * mri,
                       (long long)2 * wm * 2 * mri, 1, 2LL * mri, (long long)wm * 2 * mri, pm.wc);
  // T3[(a',t),u,ga,b] = sum W2[be,ga,u,v] T2[(a',t),be,v,b]
  kern::wapply<T>(s, t2.F, f2.p, f1.p, 2LL * mlo, mri, (long long)wm * 2 * mri, 1, 2LL * mri, mri,
                       (long long)2 * wr * mri, 1, mri, (long long)wr * mri, pm.wc2);
  // Y[(a',t,u),b'] = T3[(a',t,u),(ga,b)] Rt[(ga,b),b'] (with charges: batched over (t, u))
  kern::KMapScope ks(pm.g2);
  if (pm.g2)
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, mlo, mro, wr * mri, 1.0, f1.p, 4LL * wr * mri, (long long)wr * mri, Rt,
                       mro, 0, 0.0, Y, 4LL * mro, mro, 4);
  else
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, 4 * mlo, mro, wr * mri, 1.0, f1.p, (long long)wr * mri, 0, Rt, mro, 0,
                       0.0, Y, mro, 0, 1);
}

// out = normalise(fit of O|in>): `passes` alternating two-site passes, the
// last from left to right (odd counts start from the left with |in> brought
// to right-canonical form, even counts from the right with |in>
// left-canonical, which in_left_canonical declares it already is); every
// split takes the eps / chi_max cut of the gauge moves.  The result is
// left-canonical with its centre on the last site.  Returns the weight
// discarded in the last pass.
template <typename T>
double fit_apply(Work& W, const tdvp_mps_s& in, const tdvp_mpo_s& op, double eps, int chi_max, int passes,
                 tdvp_mps_s& out, bool in_left_canonical = false) {
  Range r_("fit.apply");
  tdvp_ctx_s* ctx = W.ctx;
  hipStream_t s = ctx->stream;
  const int N = in.N;
  if (N < 2) TDVP_THROW(TDVP_ERR_ARG, "variational MPO application needs at least two sites");
  if (passes < 1) TDVP_THROW(TDVP_ERR_ARG, "variational MPO application needs at least one pass");
  const double in_norm = W.sc.norm(in.site(N - 1), in.elems(N - 1));
  if (!std::isfinite(in_norm)) TDVP_THROW(TDVP_ERR_NUMERIC, "MPS with non-finite entries");
  const int cb = cbytes<T>();
  // working-precision copies of the ket (the input, left-canonical: its norm
  // sits in the last site, which enters scaled to unit norm so that FP32
  // cannot overflow; the result is normalised and every cut is relative)
  std::vector<DBuf> Kt;
  std::vector<const void*> Kp(N);
  for (int i = 0; i < N; ++i) {
    if (sizeof(T) == 8) {
      Kp[i] = in.site(i);
      continue;
    }
    Kt.emplace_back(ctx);
    Kt.back().ensure((size_t)in.elems(i) * cb);
    if (i == N - 1 && in_norm > 0.0) {
      W.tmpC.ensure((size_t)in.elems(i) * ZB);
      kern::zscale(s, W.tmpC.p, in.site(i), zc(1.0 / in_norm, 0.0), in.elems(i));
      kern::z2c(s, Kt.back().p, W.tmpC.p, in.elems(i));
    } else {
      kern::z2c(s, Kt.back().p, in.site(i), in.elems(i));
    }
    Kp[i] = Kt.back().p;
  }
  // the bra's sites (FP64 masters, changing as the passes go) in the working
  // precision, converted where an environment reads them
  DBuf braT(ctx);
  auto bra = [&](int i) -> const void* {
    if (sizeof(T) == 8) return out.site(i);
    braT.ensure((size_t)out.elems(i) * cb);
    kern::z2c(s, braT.p, out.site(i), out.elems(i));
    return braT.p;
  };
  out.ctx = ctx;
  out.N = N;
  out.m = in.m;
  out.q = in.q;
  out.t.clear();
  for (int i = 0; i < N; ++i) {
    out.t.emplace_back(ctx);
    out.t[i].ensure((size_t)in.elems(i) * ZB);
    HIP_CHECK(hipMemcpyAsync(out.t[i].p, in.site(i), (size_t)in.elems(i) * ZB, hipMemcpyDeviceToDevice, s));
  }
  // the last pass runs left to right (result left-canonical, centre on the
  // last site): an even count starts from the right with a left-canonical
  // guess, an odd count from the left with a right-canonical one
  const bool from_right = passes % 2 == 0;
  if (!from_right) right_canonicalize(W, out);
  else if (!in_left_canonical) left_canonicalize(W, out);
  const bool sym = out.u1();
  std::vector<DBuf> Ls, Rs;
  for (int i = 0; i <= N; ++i) {
    Ls.emplace_back(ctx);
    Rs.emplace_back(ctx);
  }
  set_one(ctx, Ls[0], cb);
  set_one(ctx, Rs[N], cb);
  DBuf f1(ctx), f2(ctx), P(ctx), Th(ctx), Th64(ctx), X(ctx), Y(ctx);
  // with charges, the products walk their nonzero blocks
  const auto& qw = op.host.qw;
  PairMaps fm(ctx);
  // the sparse-MPO stages read by charge; the first products leave out the
  // sub-blocks that share no charge (never read by those stages)
  kern::WCharges fwc1, fwc2;
  auto right_maps = [&](int i) -> ProdMaps {   // Rs[i] from site i
    if (!sym) return {};
    MapCache& mc = map_cache(ctx);
    ProdMaps pm = fm.set(ctx, cmap_env_right_gemm1_nz(mc, in.q[i], in.q[i + 1], qw[i + 1], out.q[i + 1]),
                         cmap_env_right_gemm3(mc, in.q[i], qw[i], out.q[i + 1], out.q[i]));
    fwc1 = wc_of(cmap_wstage(mc, in.q[i], out.q[i + 1], qw[i + 1], qw[i], +1), in.m[i], out.m[i + 1], op.w(i + 1));
    pm.wc = &fwc1;
    return pm;
  };
  auto left_maps = [&](int i) -> ProdMaps {    // Ls[i+1] from site i
    if (!sym) return {};
    MapCache& mc = map_cache(ctx);
    ProdMaps pm = fm.set(ctx, cmap_env_gemm1_nz(mc, out.q[i], in.q[i], qw[i], in.q[i + 1]),
                         cmap_env_left_gemm2(mc, out.q[i], out.q[i + 1], in.q[i + 1], qw[i + 1]));
    fwc1 = wc_of(cmap_wstage(mc, out.q[i], in.q[i + 1], qw[i], qw[i + 1]), out.m[i], in.m[i + 1], op.w(i));
    pm.wc = &fwc1;
    return pm;
  };
  std::vector<int> qvb, qat;
  auto local_maps = [&](int i) -> ProdMaps {   // the two-site tensor at (i, i+1)
    if (!sym) return {};
    MapCache& mc = map_cache(ctx);
    ProdMaps pm =
        fm.set(ctx, cmap_two_site_nz(mc, out.q[i], in.q[i], qw[i], in.q[i + 2], qw[i + 2], out.q[i + 2]));
    // first stage: rows a' of phi, columns (v, b) with charge q(b) - q(v);
    // its outputs of other charges are never read by the second stage,
    // whose rows (a', t) carry q(a') + q(t)
    const int mri = in.m[i + 2], mlo = out.m[i];
    qvb.resize(2 * (size_t)mri);
    for (int v = 0; v < 2; ++v)
      for (int b = 0; b < mri; ++b) qvb[(size_t)v * mri + b] = in.q[i + 2][b] - phys_charge(v);
    qat.resize(2 * (size_t)mlo);
    for (int a = 0; a < mlo; ++a)
      for (int t = 0; t < 2; ++t) qat[2 * (size_t)a + t] = out.q[i][a] + phys_charge(t);
    fwc1 = wc_of(cmap_wstage(mc, out.q[i], qvb, qw[i], qw[i + 1]), mlo, 2 * mri, op.w(i));
    fwc1.zeros_kept = 1;
    fwc2 = wc_of(cmap_wstage(mc, qat, in.q[i + 2], qw[i + 1], qw[i + 2]), 2 * mlo, mri, op.w(i + 1));
    pm.wc = &fwc1;
    pm.wc2 = &fwc2;
    return pm;
  };
  if (from_right) {
    for (int i = 0; i + 2 < N; ++i) {
      Ls[i + 1].ensure((size_t)out.m[i + 1] * op.w(i + 1) * in.m[i + 1] * cb);
      fit_env_left<T>(ctx, op.tab[i], out.m[i], in.m[i], op.w(i), op.w(i + 1), out.m[i + 1], in.m[i + 1], Ls[i].p,
                      bra(i), Kp[i], Ls[i + 1].p, f1, f2, left_maps(i));
    }
  } else {
    for (int i = N - 1; i >= 2; --i) {
      Rs[i].ensure((size_t)op.w(i) * in.m[i] * out.m[i] * cb);
      fit_env_right<T>(ctx, op.tab[i], out.m[i], in.m[i], op.w(i), op.w(i + 1), out.m[i + 1], in.m[i + 1],
                       Rs[i + 1].p, bra(i), Kp[i], Rs[i].p, f1, f2, right_maps(i));
    }
  }
  // two-site tensor of phi at (i, i+1) from the current environments (FP64
  // for the split)
  auto local = [&](int i) -> double* {
    const int mli = in.m[i], mc = in.m[i + 1], mri = in.m[i + 2], mlo = out.m[i], mro = out.m[i + 2];
    P.ensure((size_t)mli * 4 * mri * cb);
    kern::gemm<T>(s, TDVP_OP_N, TDVP_OP_N, 2 * mli, 2 * mri, mc, 1.0, Kp[i], mc, 0, Kp[i + 1], 2LL * mri, 0, 0.0, P.p,
                  2LL * mri, 0, 1);
    Th.ensure((size_t)mlo * 4 * mro * cb);
    fit_local2<T>(ctx, op.tab[i], op.tab[i + 1], mlo, mli, op.w(i), op.w(i + 1), op.w(i + 2), mri, mro, Ls[i].p,
                  Rs[i + 2].p, P.p, Th.p, f1, f2, local_maps(i));
    if (sizeof(T) == 8) return Th.as<double>();
    Th64.ensure((size_t)mlo * 4 * mro * ZB);
    kern::c2z(s, Th64.p, Th.p, (long long)mlo * 4 * mro);
    return Th64.as<double>();
  };
  double disc = 0.0;
  for (int pass = 0; pass < passes; ++pass) {
    disc = 0.0;
    if ((pass % 2 == 0) != from_right) {   // left to right: phi_i left-canonical, centre moves on
      for (int i = 0; i + 1 < N; ++i) {
        const double* th = local(i);
        const int mlo = out.m[i], mro = out.m[i + 2];
        std::vector<int> qc, qk;
        if (sym) qc = fuse_sx(out.q[i + 2], -1);
        const int k = split_left(W, th, mlo, 2 * mro, eps, chi_max, X, Y, &disc,
                                 sym ? &out.q[i] : nullptr, sym ? &qc : nullptr, &qk);
        std::swap(out.t[i], X);
        std::swap(out.t[i + 1], Y);
        out.m[i + 1] = k;
        if (sym) out.q[i + 1] = qk;
        Ls[i + 1].ensure((size_t)k * op.w(i + 1) * in.m[i + 1] * cb);
        fit_env_left<T>(ctx, op.tab[i], mlo, in.m[i], op.w(i), op.w(i + 1), k, in.m[i + 1], Ls[i].p, bra(i), Kp[i],
                        Ls[i + 1].p, f1, f2, left_maps(i));
      }
    } else {               // right to left: phi_{i+1} right-canonical
      for (int i = N - 2; i >= 0; --i) {
        const double* th = local(i);
        const int mlo = out.m[i], mro = out.m[i + 2];
        std::vector<int> qr, qk;
        if (sym) qr = fuse_xs(out.q[i], 1);
        const int k = split_right(W, th, 2 * mlo, mro, eps, chi_max, X, Y, &disc, sym ? &qr : nullptr,
                                  sym ? &out.q[i + 2] : nullptr, &qk);
        std::swap(out.t[i], X);
        std::swap(out.t[i + 1], Y);
        out.m[i + 1] = k;
        if (sym) out.q[i + 1] = qk;
        Rs[i + 1].ensure((size_t)op.w(i + 1) * in.m[i + 1] * k * cb);
        fit_env_right<T>(ctx, op.tab[i + 1], k, in.m[i + 1], op.w(i + 1), op.w(i + 2), mro, in.m[i + 2], Rs[i + 2].p,
                         bra(i + 1), Kp[i + 1], Rs[i + 1].p, f1, f2, right_maps(i + 1));
      }
    }
  }
  const double nr = W.sc.norm(out.site(N - 1), out.elems(N - 1));
  if (!(nr > 0.0) || !std::isfinite(nr)) TDVP_THROW(TDVP_ERR_NUMERIC, "MPO application vanished or is not finite");
  kern::zscale(s, out.t[N - 1].p, out.t[N - 1].p, zc(1.0 / nr, 0.0), out.elems(N - 1));
  HIP_CHECK(hipStreamSynchronize(s));
  return disc;
}

// ------------------------------------------------------ basis extension
// With charges: the rows of C (bond i) carry psi.q[i]; a column (s, b)
// carries q(b) - q(s) as a left bond; B, B_bar and rho_bar are computed
// charge by charge, and B' = [B; B_bar] is ordered by charge (stable: B's
// rows first within a charge) so that the new bond lists its charges in
// ascending order.
void extension(Work& W, tdvp_mps_s& psi, std::vector<tdvp_mps_s>& kv, double eps_M, int chi_max, int* n_added) {
  Range r_("expand.extension");
  tdvp_ctx_s* ctx = W.ctx;
  hipStream_t s = ctx->stream;
  const int N = psi.N;
  const bool sym = psi.u1();
  DBuf Vh(ctx), Bp(ctx), Xs(ctx), P(ctx), rhob(ctx), rows(ctx), Pb(ctx), Mc(ctx), nxt(ctx), Mt(ctx);
  std::vector<double> S, lam;
  for (int i = N - 1; i >= 1; --i) {
    const int ml = psi.m[i], mr = psi.m[i + 1], D = 2 * mr;
    const void* C = psi.site(i);
    std::vector<int> qD, qB;   // charges of the columns (s, b) and of the rows of B
    if (sym) qD = fuse_sx(psi.q[i + 1], -1);
    // B: orthonormal rows spanning the row space of C ("SVD without
    // truncation"); directions whose weight is at round-off level
    // (s^2 <= 1e-14 s_1^2) are not part of it.  The eigenvalues of C C^dagger
    // are the weights to ~1e-15 of the largest: when all of them are clearly
    // above the floor, C has full row rank and an LQ factorisation gives B;
    // otherwise a Jacobi SVD resolves the small singular values.
    W.tmpA.ensure((size_t)ml * ml * ZB);
    W.tmpB.ensure((size_t)ml * ml * ZB);
    const std::vector<int>* qi = sym ? &psi.q[i] : nullptr;
    const std::vector<int>* qDp = sym ? &qD : nullptr;
    qgemm(W, TDVP_OP_N, TDVP_OP_C, ml, ml, D, 1.0, C, D, C, D, 0.0, W.tmpA.p, ml, qi, qDp, qi);
    int r = 0;
    Vh.ensure((size_t)std::min(ml, D) * D * ZB);
    // Full row rank is certified without the eigendecomposition when the
    // smallest weight exceeds 1e-10 times their sum (hence 1e-10 times the
    // largest, the criterion below); B is then the LQ factor's Q.
    bool done = false;
    if (ml <= D) {
      const std::vector<int>* qm = sym ? &psi.q[i] : nullptr;
      const void* F = la::gram_floor_certified(ctx, W.tmpB.p, ml, 1e-10, true,
                                               W.cinv.ensure((size_t)ml * ml * ZB), W.work, W.tmpA.p, qm);
      if (F) {
        W.tmpC.ensure((size_t)ml * ml * ZB);
        done = la::cholqr2_rows_rowmajor(ctx, C, ml, D, W.tmpC.p, Vh.p, W.work, F, qm, sym ? &qD : nullptr, W.maps);
        if (done) {
          r = ml;
          if (sym) qB = psi.q[i];
        }
      }
    }
    std::vector<int> qv;
    if (!done) {
      if (sym) la::eigh_sectors(ctx, W.tmpA.p, ml, psi.q[i], S, W.tmpB.p, W.work2, qv);
      else la::eigh_rows_desc(ctx, W.tmpA.p, ml, S, W.tmpB.p, W.work2);
    }
    if (done) {
      // B from the certified LQ factorisation
    } else if (ml <= D && !S.empty() && S[0] > 0.0 && S[ml - 1] > 1e-10 * S[0]) {
      r = ml;
      // B = S^-1 U^dagger C, polished by Newton-Schulz
      W.tmpC.ensure((size_t)ml * D * ZB);
      qgemm(W, TDVP_OP_N, TDVP_OP_N, ml, D, ml, 1.0, W.tmpB.p, ml, C, D, 0.0, W.tmpC.p, D, sym ? &qv : nullptr, qi, qDp);
      kern::zscale_rows(s, Vh.p, D, W.tmpC.p, D, ml, D, inv_sqrt_weights(W, S, ml));
      ns_rows(W, Vh.p, ml, D, 3);
      if (sym) {
        sort_rows_by_charge(W, Vh.p, D, ml, nullptr, qv);
        qB = qv;
      }
    } else if (!S.empty() && S[0] > 0.0) {
      // Weights spread over more than ten decades: the directions above the
      // floor are those with lambda > 1e-14 lambda_1, which the Gram
      // eigenvalues resolve (their error is ~1e-16 lambda_1).  The rows
      // S^-1/2 U^dagger C of the small weights carry eigenvector errors up
      // to ~1e-2, which two Cholesky-QR steps remove while keeping their
      // span; the part of C outside that span is below 1e-18 of its weight.
      for (double v : S) r += (v > 1e-14 * S[0]) ? 1 : 0;
      W.tmpC.ensure((size_t)r * D * ZB);
      std::vector<int> qvr;
      if (sym) qvr.assign(qv.begin(), qv.begin() + r);
      qgemm(W, TDVP_OP_N, TDVP_OP_N, r, D, ml, 1.0, W.tmpB.p, ml, C, D, 0.0, W.tmpC.p, D, sym ? &qvr : nullptr, qi, qDp);
      kern::zscale_rows(s, W.tmpC.p, D, W.tmpC.p, D, r, D, inv_sqrt_weights(W, S, r));
      W.tmpA.ensure((size_t)r * r * ZB);
      if (!la::cholqr2_rows_rowmajor(ctx, W.tmpC.p, r, D, W.tmpA.p, Vh.p, W.work)) {
        HIP_CHECK(hipMemcpyAsync(Vh.p, W.tmpC.p, (size_t)r * D * ZB, hipMemcpyDeviceToDevice, s));
        ns_rows(W, Vh.p, r, D, 6);
        if (!(la::orth_defect(ctx, Vh.p, r, D, true, W.work) <= 1e-20))
          TDVP_THROW(TDVP_ERR_NUMERIC, "extension: no orthonormal basis of the row space");
      }
      if (sym) {
        qv.resize(r);
        sort_rows_by_charge(W, Vh.p, D, r, nullptr, qv);
        qB = qv;
      }
    }
    const int cap = std::min(chi_max - r, D - r);
    // B' rows: B (r x D) then B_bar
    Bp.ensure((size_t)D * D * ZB);  // r + n <= D rows
    kern::copy2d(s, Bp.p, D, Vh.p, D, r, D, ZB);
    int n = 0;
    std::vector<int> qbar, qBr, qstack;   // charges of B's r rows, of the stacked Krylov rows
    if (sym) qBr.assign(qB.begin(), qB.begin() + r);
    const std::vector<int>* qBp = sym ? &qBr : nullptr;
    if (cap > 0 && !kv.empty()) {
      // projected Krylov centers, stacked: X_l = Ct_l - (Ct_l B^dagger) B
      int rows_tot = 0;
      for (auto& k : kv) rows_tot += k.m[i];
      Xs.ensure((size_t)rows_tot * D * ZB);
      double tr_ref = 0.0;
      int off = 0;
      for (auto& k : kv) {
        const int mt = k.m[i];
        void* Xl = static_cast<char*>(Xs.p) + (size_t)off * D * ZB;
        HIP_CHECK(hipMemcpyAsync(Xl, k.site(i), (size_t)mt * D * ZB, hipMemcpyDeviceToDevice, s));
        const std::vector<int>* qt = sym && k.u1() ? &k.q[i] : nullptr;
        if (qt) qstack.insert(qstack.end(), qt->begin(), qt->end());
        if (r > 0) {
          P.ensure((size_t)mt * r * ZB);
          qgemm(W, TDVP_OP_N, TDVP_OP_C, mt, r, D, 1.0, k.site(i), D, Bp.p, D, 0.0, P.p, r, qt, qDp, qBp);
          qgemm(W, TDVP_OP_N, TDVP_OP_N, mt, D, r, -1.0, P.p, r, Bp.p, D, 1.0, Xl, D, qt, qBp, qDp);
        }
        tr_ref += W.sc.dot(k.site(i), k.site(i), (long long)mt * D).real();
        off += mt;
      }
      // rho_bar = sum_l X_l^dagger X_l   (D x D)
      rhob.ensure((size_t)D * D * ZB);
      const std::vector<int>* qsp = (int)qstack.size() == rows_tot ? &qstack : nullptr;
      qgemm(W, TDVP_OP_C, TDVP_OP_N, D, D, rows_tot, 1.0, Xs.p, D, Xs.p, D, 0.0, rhob.p, D, qDp, qsp, qDp);
      rows.ensure((size_t)D * D * ZB);
      if (sym) la::eigh_sectors(ctx, rhob.p, D, qD, lam, rows.p, W.work, qbar);
      else la::eigh_rows_desc(ctx, rhob.p, D, lam, rows.p, W.work);
      n = keep_count(lam, eps_M, tr_ref, cap, 0);
      int nz = 0;
      for (double v : lam) nz += (v > 1e-14 * std::max(tr_ref, 1e-300)) ? 1 : 0;
      n = std::min(n, nz);
      if (n > 0) {
        void* Bbar = static_cast<char*>(Bp.p) + (size_t)r * D * ZB;
        kern::copy2d(s, Bbar, D, rows.p, D, n, D, ZB);
        std::vector<int> qbn;
        if (sym) qbn.assign(qbar.begin(), qbar.begin() + n);
        const std::vector<int>* qbp = sym ? &qbn : nullptr;
        if (r > 0) {
          Pb.ensure((size_t)n * r * ZB);
          qgemm(W, TDVP_OP_N, TDVP_OP_C, n, r, D, 1.0, Bbar, D, Bp.p, D, 0.0, Pb.p, r, qbp, qDp, qBp);
          qgemm(W, TDVP_OP_N, TDVP_OP_N, n, D, r, -1.0, Pb.p, r, Bp.p, D, 1.0, Bbar, D, qbp, qBp, qDp);
        }
        // the eigenvector rows stay orthonormal up to the projection above;
        // Newton-Schulz restores orthonormality within their span
        ns_rows(W, Bbar, n, D, 2, qbp, qDp);
      }
    }
    const int mnew = r + n;
    std::vector<int> qi_old;
    if (sym) qi_old = psi.q[i];
    if (sym) {
      std::vector<int> qall(qB.begin(), qB.begin() + r);
      qall.insert(qall.end(), qbar.begin(), qbar.begin() + n);
      sort_rows_by_charge(W, Bp.p, D, mnew, nullptr, qall);
      psi.q[i] = qall;
    }
    // center moves: C_{i-1} = A_{i-1} (C_i B'^dagger), same for every Krylov vector
    // (with charges: old bond i charges qi for psi, the Krylov vector's own
    // for it; rows of site i-1 fused (a, s))
    const std::vector<int>* qn = sym ? &psi.q[i] : nullptr;   // the new bond (sorted above)
    auto move = [&](tdvp_mps_s& x, const std::vector<int>* qold) {
      const int mo = x.m[i];
      Mc.ensure((size_t)mo * mnew * ZB);
      qgemm(W, TDVP_OP_N, TDVP_OP_C, mo, mnew, D, 1.0, x.site(i), D, Bp.p, D, 0.0, Mc.p, mnew, qold, qDp, qn);
      std::vector<int> qrow;
      if (sym && qold && x.u1()) qrow = fuse_xs(x.q[i - 1], 1);
      nxt.ensure((size_t)2 * x.m[i - 1] * mnew * ZB);
      qgemm(W, TDVP_OP_N, TDVP_OP_N, 2 * x.m[i - 1], mnew, mo, 1.0, x.site(i - 1), mo, Mc.p, mnew, 0.0, nxt.p, mnew,
            qrow.empty() ? nullptr : &qrow, qold, qn);
      std::swap(x.t[i - 1], nxt);
    };
    move(psi, qi_old.empty() ? nullptr : &qi_old);
    for (auto& k : kv) {
      move(k, sym && k.u1() ? &k.q[i] : nullptr);
      k.m[i] = mnew;
    }
    // the new right-orthonormal tensor of psi at site i
    DBuf Bnew(ctx);
    Bnew.ensure((size_t)mnew * D * ZB);
    HIP_CHECK(hipMemcpyAsync(Bnew.p, Bp.p, (size_t)mnew * D * ZB, hipMemcpyDeviceToDevice, s));
    std::swap(psi.t[i], Bnew);
    psi.m[i] = mnew;
    *n_added += n;
    HIP_CHECK(hipStreamSynchronize(s));
  }
}

template <typename T>
void expand_impl(tdvp_ctx_s* ctx, tdvp_mps_s& psi, const tdvp_mpo_s& op, const tdvp_expand_params& p,
                 tdvp_expand_stats& st) {
  Work W(ctx);
  const int N = psi.N;
  bool full = true;
  for (int b = 1; b < N; ++b) {
    const double cap = std::min<double>(p.chi_max, std::min(std::ldexp(1.0, std::min(b, 60)),
                                                            std::ldexp(1.0, std::min(N - b, 60))));
    if (psi.m[b] < cap) full = false;
  }
  if (p.k < 2 || (p.skip_if_full && full)) {
    right_canonicalize(W, psi);
    st.skipped = 1;
  } else {
    const double t0 = now_ms();
    left_canonicalize(W, psi);
    std::vector<tdvp_mps_s> kv(p.k - 1);
    const tdvp_mps_s* prev = &psi;
    for (int l = 0; l + 1 < p.k; ++l) {
      st.discarded_K += p.apply_method == TDVP_APPLY_FIT
                            ? fit_apply<T>(W, *prev, op, p.eps_K, p.chi_max, std::max(1, p.fit_passes), kv[l], true)
                            : denmat_apply<T>(W, *prev, op, p.eps_K, p.chi_max, kv[l]);
      prev = &kv[l];
      for (int b = 0; b <= N; ++b) st.krylov_max_bond = std::max(st.krylov_max_bond, kv[l].m[b]);
    }
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    const double t1 = now_ms();
    extension(W, psi, kv, p.eps_M, p.chi_max, &st.n_added);
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    st.ms_krylov = t1 - t0;
    st.ms_extend = now_ms() - t1;
  }
  for (int b = 0; b <= N; ++b) st.max_bond = std::max(st.max_bond, psi.m[b]);
}

}  // namespace

void run_sweep(tdvp_ctx_s* ctx, tdvp_mps_s& psi, const tdvp_mpo_s& H, const tdvp_sweep_params& p,
               tdvp_sweep_stats& st) {
  const double t0 = now_ms();
  if (p.prec == TDVP_FP64) {
    sweep_impl<double>(ctx, psi, H, p, st);
  } else {
    kern::FloatModeScope mode(kern::float_mode_of(p.prec));
    sweep_impl<float>(ctx, psi, H, p, st);
  }
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  st.ms = now_ms() - t0;
}

void run_sweep2(tdvp_ctx_s* ctx, tdvp_mps_s& psi, const tdvp_mpo_s& H, const tdvp_sweep_params& p,
                tdvp_sweep_stats& st) {
  const double t0 = now_ms();
  if (p.prec == TDVP_FP64) {
    sweep2_impl<double>(ctx, psi, H, p, st);
  } else {
    kern::FloatModeScope mode(kern::float_mode_of(p.prec));
    sweep2_impl<float>(ctx, psi, H, p, st);
  }
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  st.ms = now_ms() - t0;
}

void run_expand(tdvp_ctx_s* ctx, tdvp_mps_s& psi, const tdvp_mpo_s& op, const tdvp_expand_params& p,
                tdvp_expand_stats& st) {
  if (p.prec == TDVP_FP64) {
    expand_impl<double>(ctx, psi, op, p, st);
  } else {
    kern::FloatModeScope mode(kern::float_mode_of(p.prec));
    expand_impl<float>(ctx, psi, op, p, st);
  }
}

void run_apply_mpo(tdvp_ctx_s* ctx, const tdvp_mps_s& in, const tdvp_mpo_s& op, int method, double eps, int chi_max,
                   int passes, tdvp_mps_s& out, double* discarded) {
  Work W(ctx);
  double d;
  if (method == TDVP_APPLY_FIT) {
    d = fit_apply<double>(W, in, op, eps, chi_max, passes, out);
  } else {
    // the density-matrix route reads the norm from the last site of a
    // left-canonical input
    tdvp_mps_s lc;
    lc.ctx = ctx;
    lc.N = in.N;
    lc.m = in.m;
    lc.q = in.q;
    for (int i = 0; i < in.N; ++i) {
      lc.t.emplace_back(ctx);
      lc.t[i].ensure((size_t)in.elems(i) * ZB);
      HIP_CHECK(hipMemcpyAsync(lc.t[i].p, in.site(i), (size_t)in.elems(i) * ZB, hipMemcpyDeviceToDevice,
                               ctx->stream));
    }
    left_canonicalize(W, lc);
    d = denmat_apply<double>(W, lc, op, eps, chi_max, out);
  }
  if (discarded) *discarded = d;
}

// ------------------------------------------------------------ measurement
void run_measure(tdvp_ctx_s* ctx, const tdvp_mps_s& psi, const tdvp_mpo_s* H, const tdvp_mps_s* other,
                 tdvp_observables& out) {
  hipStream_t s = ctx->stream;
  const int N = psi.N;
  Work W(ctx);
  // right transfers of <psi|psi>: Rtr[i][x,y] for sites i..N-1
  std::vector<DBuf> Rtr;
  for (int i = 0; i <= N; ++i) Rtr.emplace_back(ctx);
  set_one(ctx, Rtr[N], ZB);
  DBuf G(ctx), Tn(ctx), Tz(ctx), Tl(ctx);
  // with charges every transfer is block diagonal and the products walk the
  // charge blocks: rows (a, s) of a site carry q(a) + q(s), columns (s, b)
  // as a left bond q(b) - q(s)
  const bool qs = psi.u1();
  auto qxs = [&](int i) { return qs ? fuse_xs(psi.q[i], 1) : std::vector<int>(); };
  auto qsx = [&](int i) { return qs ? fuse_sx(psi.q[i + 1], -1) : std::vector<int>(); };
  auto qp = [&](const std::vector<int>& v) { return qs ? &v : nullptr; };
  for (int i = N - 1; i >= 0; --i) {
    const int ml = psi.m[i], mr = psi.m[i + 1];
    G.ensure((size_t)2 * ml * mr * ZB);
    const std::vector<int> qrow = qxs(i), qcol = qsx(i);
    // G[(y,s),p] = sum_q M[(y,s),q] Rtr[p,q]
    qgemm(W, TDVP_OP_N, TDVP_OP_T, 2 * ml, mr, mr, 1.0, psi.site(i), mr, Rtr[i + 1].p, mr, 0.0, G.p, mr, qp(qrow),
          qs ? &psi.q[i + 1] : nullptr, qs ? &psi.q[i + 1] : nullptr);
    // Rtr[x,y] = sum_{(s,p)} conj(M[x,(s,p)]) G[y,(s,p)]
    Rtr[i].ensure((size_t)ml * ml * ZB);
    qgemm(W, TDVP_OP_R, TDVP_OP_T, ml, ml, 2 * mr, 1.0, psi.site(i), 2LL * mr, G.p, 2LL * mr, 0.0, Rtr[i].p, ml,
          qs ? &psi.q[i] : nullptr, qp(qcol), qs ? &psi.q[i] : nullptr);
  }
  zc nn;
  download(ctx, &nn, Rtr[0].p, ZB);
  HIP_CHECK(hipStreamSynchronize(s));
  const double norm2 = nn.real();
  out.norm = std::sqrt(std::max(0.0, norm2));
  if (out.bond_dims)
    for (int b = 0; b <= N; ++b) out.bond_dims[b] = psi.m[b];
  if (out.sz) {
    set_one(ctx, Tl, ZB);
    for (int i = 0; i < N; ++i) {
      const int ml = psi.m[i], mr = psi.m[i + 1];
      G.ensure((size_t)ml * 2 * mr * ZB);
      const std::vector<int> qrow = qxs(i), qcol = qsx(i);
      const std::vector<int>* ql = qs ? &psi.q[i] : nullptr;
      const std::vector<int>* qr = qs ? &psi.q[i + 1] : nullptr;
      // G[x,(s,q)] = sum_y T[x,y] M[y,(s,q)]
      qgemm(W, TDVP_OP_N, TDVP_OP_N, ml, 2 * mr, ml, 1.0, Tl.p, ml, psi.site(i), 2LL * mr, 0.0, G.p, 2LL * mr, ql, ql,
            qp(qcol));
      Tn.ensure((size_t)mr * mr * ZB);
      Tz.ensure((size_t)mr * mr * ZB);
      qgemm(W, TDVP_OP_C, TDVP_OP_N, mr, mr, 2 * ml, 1.0, psi.site(i), mr, G.p, mr, 0.0, Tn.p, mr, qr, qp(qrow), qr);
      kern::zscale_phys(s, G.p, ml, mr, 0.5, -0.5);
      qgemm(W, TDVP_OP_C, TDVP_OP_N, mr, mr, 2 * ml, 1.0, psi.site(i), mr, G.p, mr, 0.0, Tz.p, mr, qr, qp(qrow), qr);
      const zc v = W.sc.dot(Tz.p, Rtr[i + 1].p, (long long)mr * mr, false);
      out.sz[i] = v.real() / norm2;
      std::swap(Tl, Tn);
    }
  }
  if (H) {
    std::vector<DBuf> envs;
    envs.emplace_back(ctx);
    envs.emplace_back(ctx);
    set_one(ctx, envs[0], ZB);
    // with charges (and an MPO that conserves them) the products walk their
    // nonzero blocks
    const bool sym = psi.u1() && H->host.u1;
    PairMaps emap(ctx);
    for (int i = 0; i < N; ++i) {
      const int ml = psi.m[i], mr = psi.m[i + 1], wl = H->w(i), wr = H->w(i + 1);
      const size_t need = (size_t)2 * ml * mr * std::max(wl, wr) * ZB;
      W.ws1.ensure(need);
      W.ws2.ensure(need);
      envs[1].ensure((size_t)mr * wr * mr * ZB);
      ProdMaps pm;
      if (sym) {
        MapCache& mc = map_cache(ctx);
        pm = emap.set(ctx, cmap_env_gemm1(mc, psi.q[i], psi.q[i], H->host.qw[i], psi.q[i + 1]),
                      cmap_env_left_gemm2(mc, psi.q[i], psi.q[i + 1], psi.q[i + 1], H->host.qw[i + 1]));
      }
      env_left<double>(ctx, H->tab[i], ml, wl, wr, mr, envs[0].p, psi.site(i), envs[1].p, W.ws1.p, W.ws2.p,
                       W.split(ml, mr, 16), pm);
      std::swap(envs[0], envs[1]);
    }
    zc e;
    download(ctx, &e, envs[0].p, ZB);
    HIP_CHECK(hipStreamSynchronize(s));
    out.energy = e.real() / norm2;
  }
  if (other) {
    set_one(ctx, Tl, ZB);
    for (int i = 0; i < N; ++i) {
      const int ml = psi.m[i], mr = psi.m[i + 1], ol = other->m[i], orr = other->m[i + 1];
      G.ensure((size_t)ol * 2 * mr * ZB);
      kern::gemm<double>(s, TDVP_OP_N, TDVP_OP_N, ol, 2 * mr, ml, 1.0, Tl.p, ml, 0, psi.site(i), 2LL * mr, 0, 0.0, G.p,
                         2LL * mr, 0, 1);
      Tn.ensure((size_t)orr * mr * ZB);
      kern::gemm<double>(s, TDVP_OP_C, TDVP_OP_N, orr, mr, 2 * ol, 1.0, other->site(i), orr, 0, G.p, mr, 0, 0.0, Tn.p,
                         mr, 0, 1);
      std::swap(Tl, Tn);
    }
    zc ov;
    download(ctx, &ov, Tl.p, ZB);
    HIP_CHECK(hipStreamSynchronize(s));
    out.overlap_re = ov.real();
    out.overlap_im = ov.imag();
  }
}
