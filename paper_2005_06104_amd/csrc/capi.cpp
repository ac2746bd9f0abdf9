// extern "C" entry points: argument checks, status codes, context plumbing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <thread>
#include <unordered_set>

#include "engine.h"

#define TDVP_VERSION "tdvp-mi355x 0.1 (gfx950)"

thread_local tdvp_ctx_s* tl_exec_ctx = nullptr;

// free the buffers the workers dropped while their streams still ran
static void flush_deferred(tdvp_ctx_s* ctx) {
  for (tdvp_ctx_s* w : ctx->workers) {
    for (auto& f : w->deferred_frees) f.first->dfree(f.second);
    w->deferred_frees.clear();
  }
}

void* tdvp_ctx_s::dalloc(size_t bytes) {
  void* p = nullptr;
  if (async_alloc) {
    hipError_t e = hipMallocFromPoolAsync(&p, bytes, pool, stream);
    if (e != hipSuccess || !p)
      TDVP_THROW(TDVP_ERR_ALLOC, "stream-ordered allocation of " + std::to_string(bytes) + " bytes failed");
  } else if (alloc) {
    p = alloc(bytes, user);
    if (!p) TDVP_THROW(TDVP_ERR_ALLOC, "device allocation of " + std::to_string(bytes) + " bytes failed");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess || !p)
      TDVP_THROW(TDVP_ERR_ALLOC, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

void tdvp_ctx_s::dfree(void* p) {
  if (!p) return;
  if (async_alloc) (void)hipFreeAsync(p, stream);
  else if (free_) free_(p, user);
  else (void)hipFree(p);
}

void tdvp_ctx_s::ensure_workers(int n) {
  if (!worker_pool && n > 0) {
    // one stream-ordered pool of the context's own for its workers, keeping
    // freed memory between calls; destroyed with the workers (the device's
    // default pool is left untouched)
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    HIP_CHECK(hipMemPoolCreate(&worker_pool, &props));
    uint64_t thr = UINT64_MAX;
    HIP_CHECK(hipMemPoolSetAttribute(worker_pool, hipMemPoolAttrReleaseThreshold, &thr));
  }
  while ((int)workers.size() < n) {
    auto* w = new tdvp_ctx_s();
    w->device = device;
    w->async_alloc = true;
    w->pool = worker_pool;
    w->owns_stream = true;
    workers.push_back(w);
    HIP_CHECK(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
    if (rocblas_create_handle(&w->blas) != rocblas_status_success)
      TDVP_THROW(TDVP_ERR_DEVICE, "rocblas_create_handle failed");
    if (rocblas_set_stream(w->blas, w->stream) != rocblas_status_success)
      TDVP_THROW(TDVP_ERR_DEVICE, "rocblas_set_stream failed");
    HIP_CHECK(hipEventCreate(&w->ev_a));
    HIP_CHECK(hipEventCreate(&w->ev_b));
    HIP_CHECK(hipEventCreate(&w->ev_c));
    HIP_CHECK(hipEventCreate(&w->ev_d));
  }
}

void tdvp_ctx_s::destroy_workers() {
  for (tdvp_ctx_s* w : workers)
    if (w->stream) (void)hipStreamSynchronize(w->stream);
  flush_deferred(this);
  for (tdvp_ctx_s* w : workers) {
    if (w->stream) (void)hipStreamSynchronize(w->stream);
    w->destroy_maps();
    w->destroy_uploads();
    w->dfree(w->split_ws);
    if (w->stream) (void)hipStreamSynchronize(w->stream);
    if (w->hstage) (void)hipHostFree(w->hstage);
    for (hipEvent_t e : w->ev_stage)
      if (e) (void)hipEventDestroy(e);
    if (w->ev_a) (void)hipEventDestroy(w->ev_a);
    if (w->ev_b) (void)hipEventDestroy(w->ev_b);
    if (w->ev_c) (void)hipEventDestroy(w->ev_c);
    if (w->ev_d) (void)hipEventDestroy(w->ev_d);
    if (w->blas) rocblas_destroy_handle(w->blas);
    if (w->stream) (void)hipStreamDestroy(w->stream);
    delete w;
  }
  workers.clear();
  if (worker_pool) {
    (void)hipMemPoolTrimTo(worker_pool, 0);
    (void)hipMemPoolDestroy(worker_pool);
    worker_pool = nullptr;
  }
}

void tdvp_ctx_s::sync() { HIP_CHECK(hipStreamSynchronize(stream)); }

void tdvp_ctx_s::upload_async(void* dev, const void* host, size_t bytes) {
  if (bytes == 0) return;
  const int k = up_pos;
  up_pos = (up_pos + 1) % UP_SLOTS;
  if (up_ev[k]) HIP_CHECK(hipEventSynchronize(up_ev[k]));
  else HIP_CHECK(hipEventCreateWithFlags(&up_ev[k], hipEventDisableTiming));
  if (up_cap[k] < bytes) {
    if (up_buf[k]) HIP_CHECK(hipHostFree(up_buf[k]));
    up_buf[k] = nullptr;
    up_cap[k] = 0;
    const size_t cap = std::max<size_t>(bytes + bytes / 2, 16384);
    HIP_CHECK(hipHostMalloc(&up_buf[k], cap, hipHostMallocDefault));
    up_cap[k] = cap;
  }
  std::memcpy(up_buf[k], host, bytes);
  HIP_CHECK(hipMemcpyAsync(dev, up_buf[k], bytes, hipMemcpyHostToDevice, stream));
  HIP_CHECK(hipEventRecord(up_ev[k], stream));
}

void tdvp_ctx_s::destroy_uploads() {
  for (int k = 0; k < UP_SLOTS; ++k) {
    if (up_ev[k]) {
      (void)hipEventSynchronize(up_ev[k]);
      (void)hipEventDestroy(up_ev[k]);
      up_ev[k] = nullptr;
    }
    if (up_buf[k]) (void)hipHostFree(up_buf[k]);
    up_buf[k] = nullptr;
    up_cap[k] = 0;
  }
}

void tdvp_ctx_s::ensure_hstage() {
  if (hstage) return;
  void* h = nullptr;
  void* d = nullptr;
  HIP_CHECK(hipHostMalloc(&h, HSTAGE_BYTES, hipHostMallocDefault));
  if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || !d) {
    (void)hipGetLastError();
    (void)hipHostFree(h);
    TDVP_THROW(TDVP_ERR_DEVICE, "pinned staging buffer has no device address");
  }
  hstage = h;
  hstage_dev = d;
}

const void* tdvp_ctx_s::fetch(const void* dev, size_t bytes) {
  if (bytes > HSTAGE_BYTES / 2) TDVP_THROW(TDVP_ERR_ARG, "staged download too large");
  ensure_hstage();
  HIP_CHECK(hipMemcpyAsync(hstage, dev, bytes, hipMemcpyDeviceToHost, stream));
  HIP_CHECK(hipStreamSynchronize(stream));
  return hstage;
}

const void* tdvp_ctx_s::stage_async(int k, const void* dev, size_t bytes) {
  if (bytes > HSTAGE_BYTES / 4 || k < 0 || k > 1) TDVP_THROW(TDVP_ERR_ARG, "staged download too large");
  ensure_hstage();
  if (!ev_stage[k]) HIP_CHECK(hipEventCreateWithFlags(&ev_stage[k], hipEventDisableTiming));
  char* slot = static_cast<char*>(hstage) + HSTAGE_BYTES / 2 + (size_t)k * (HSTAGE_BYTES / 4);
  HIP_CHECK(hipMemcpyAsync(slot, dev, bytes, hipMemcpyDeviceToHost, stream));
  HIP_CHECK(hipEventRecord(ev_stage[k], stream));
  return slot;
}

void* tdvp_ctx_s::stage_slot_dev(int k) {
  if (k < 0 || k > 1) TDVP_THROW(TDVP_ERR_ARG, "bad staging slot");
  ensure_hstage();
  if (!ev_stage[k]) HIP_CHECK(hipEventCreateWithFlags(&ev_stage[k], hipEventDisableTiming));
  return static_cast<char*>(hstage_dev) + HSTAGE_BYTES / 2 + (size_t)k * (HSTAGE_BYTES / 4);
}

const void* tdvp_ctx_s::stage_mark(int k) {
  HIP_CHECK(hipEventRecord(ev_stage[k], stream));
  return static_cast<char*>(hstage) + HSTAGE_BYTES / 2 + (size_t)k * (HSTAGE_BYTES / 4);
}

void tdvp_ctx_s::wait_stage(int k) { HIP_CHECK(hipEventSynchronize(ev_stage[k])); }

namespace {

template <class F>
tdvp_status guarded(tdvp_ctx_s* ctx, F&& f) {
  try {
    f();
    if (ctx) ctx->last_error.clear();
    return TDVP_OK;
  } catch (const TdvpError& e) {
    if (ctx) ctx->last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->last_error = "host allocation failed";
    return TDVP_ERR_ALLOC;
  } catch (const std::exception& e) {
    if (ctx) ctx->last_error = e.what();
    return TDVP_ERR_DEVICE;
  } catch (...) {
    if (ctx) ctx->last_error = "unknown failure";
    return TDVP_ERR_DEVICE;
  }
}

void bind(tdvp_ctx_s* ctx) { HIP_CHECK(hipSetDevice(ctx->device)); }

// Run f(worker_ctx, j) for j < n.  One instance runs on the context itself;
// several run concurrently, one host thread and one worker context each (a
// GSE-TDVP1 step is a chain of latency-bound factorisations, so independent
// chains on separate streams fill the device).  Every stream is synchronised
// before returning; the first failure is rethrown after all threads joined.
template <class F>
void for_instances(tdvp_ctx_s* ctx, int n, F&& f) {
  if (n == 1) {
    f(ctx, 0);
    return;
  }
  ctx->sync();
  const int nw = std::min(n, 16);
  ctx->ensure_workers(nw);
  std::vector<std::exception_ptr> errs(n);
  std::vector<std::thread> threads;
  for (int w = 0; w < nw; ++w) {
    threads.emplace_back([&, w] {
      tdvp_ctx_s* wc = ctx->workers[w];
      tl_exec_ctx = wc;
      if (hipSetDevice(ctx->device) != hipSuccess) {
        tl_exec_ctx = nullptr;
        for (int j = w; j < n; j += nw) errs[j] = std::make_exception_ptr(TdvpError(TDVP_ERR_DEVICE, "hipSetDevice"));
        return;
      }
      for (int j = w; j < n; j += nw) {
        try {
          f(wc, j);
        } catch (const TdvpError& e) {
          errs[j] = std::make_exception_ptr(TdvpError(e.code, std::string(e.what()) + " (instance " +
                                                                    std::to_string(j) + ")"));
        } catch (...) {
          errs[j] = std::current_exception();
        }
      }
      (void)hipStreamSynchronize(wc->stream);
      tl_exec_ctx = nullptr;
    });
  }
  for (auto& t : threads) t.join();
  flush_deferred(ctx);
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
}

// The instances of one batched call run concurrently and each mutates its
// state, so a state may appear only once.
void check_distinct(int n, const tdvp_mps* psi) {
  std::unordered_set<const tdvp_mps_s*> seen;
  for (int j = 0; j < n; ++j) ARG_CHECK(seen.insert(psi[j]).second, "the same MPS handle appears twice in psi[]");
}

bool all_finite(const double* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

std::vector<zc> host_W(const double* W, int wl, int wr) {
  std::vector<zc> out((size_t)wl * wr * 4);
  for (size_t i = 0; i < out.size(); ++i) out[i] = zc(W[2 * i], W[2 * i + 1]);
  return out;
}

}  // namespace

namespace {

template <class F>
tdvp_status kernel_call(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr, const double* W_host, void* workspace,
                        F&& f) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(prec >= TDVP_FP64 && prec <= TDVP_BF16X3_FP32ACC, "unknown precision");
    ARG_CHECK(ml >= 1 && mr >= 1 && wl >= 1 && wr >= 1 && wl <= 32 && wr <= 32, "bad sizes");
    bind(ctx);
    const int cb = prec == TDVP_FP64 ? 16 : 8;
    const size_t half = (size_t)2 * ml * mr * std::max(wl, wr) * cb;
    const size_t split = (size_t)32 * ml * mr * cb;  // split-K partial products
    DBuf ws(ctx), tab(ctx);
    char* w1;
    if (workspace) w1 = static_cast<char*>(workspace);
    else w1 = static_cast<char*>(ws.ensure(2 * half + split));
    SiteTables tb{};
    if (W_host) tb = upload_tables(ctx, host_W(W_host, wl, wr), wl, wr, tab);
    kern::FloatModeScope mode(kern::float_mode_of(prec));
    f(tb, w1, w1 + half, SplitWS{w1 + 2 * half, split});
    if (!workspace || W_host) ctx->sync();  // keep temporaries alive until the kernels finish
  });
}
}  // namespace

extern "C" {

const char* tdvp_version(void) { return TDVP_VERSION; }

tdvp_status tdvp_ctx_create(int device, void* hip_stream, tdvp_alloc_fn alloc, tdvp_free_fn free_, void* user,
                            tdvp_ctx* out) {
  if (!out) return TDVP_ERR_ARG;
  *out = nullptr;
  auto* ctx = new (std::nothrow) tdvp_ctx_s();
  if (!ctx) return TDVP_ERR_ALLOC;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->alloc = alloc;
  ctx->free_ = free_;
  ctx->user = user;
  if ((alloc == nullptr) != (free_ == nullptr)) {
    delete ctx;
    return TDVP_ERR_ARG;
  }
  tdvp_status st = guarded(ctx, [&] {
    int n = 0;
    HIP_CHECK(hipGetDeviceCount(&n));
    ARG_CHECK(device >= 0 && device < n, "device index out of range");
    bind(ctx);
    if (rocblas_create_handle(&ctx->blas) != rocblas_status_success)
      TDVP_THROW(TDVP_ERR_DEVICE, "rocblas_create_handle failed");
    if (rocblas_set_stream(ctx->blas, ctx->stream) != rocblas_status_success)
      TDVP_THROW(TDVP_ERR_DEVICE, "rocblas_set_stream failed");
    HIP_CHECK(hipEventCreate(&ctx->ev_a));
    HIP_CHECK(hipEventCreate(&ctx->ev_b));
    HIP_CHECK(hipEventCreate(&ctx->ev_c));
    HIP_CHECK(hipEventCreate(&ctx->ev_d));
  });
  if (st != TDVP_OK) {
    if (ctx->blas) rocblas_destroy_handle(ctx->blas);
    delete ctx;
    return st;
  }
  *out = ctx;
  return TDVP_OK;
}

void tdvp_ctx_destroy(tdvp_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->destroy_workers();
  ctx->destroy_maps();
  ctx->destroy_uploads();
  ctx->dfree(ctx->split_ws);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->hstage) (void)hipHostFree(ctx->hstage);
  for (hipEvent_t e : ctx->ev_stage)
    if (e) (void)hipEventDestroy(e);
  if (ctx->ev_a) (void)hipEventDestroy(ctx->ev_a);
  if (ctx->ev_b) (void)hipEventDestroy(ctx->ev_b);
  if (ctx->ev_c) (void)hipEventDestroy(ctx->ev_c);
  if (ctx->ev_d) (void)hipEventDestroy(ctx->ev_d);
  if (ctx->blas) rocblas_destroy_handle(ctx->blas);
  delete ctx;
}

const char* tdvp_last_error(tdvp_ctx ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

tdvp_status tdvp_synchronize(tdvp_ctx ctx) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] { ctx->sync(); });
}

// ------------------------------------------------------------------ MPO
tdvp_status tdvp_build_mpo_host(int n_sites, const tdvp_term* terms, int n_terms, double c0_re, double c0_im,
                                double c1_re, double c1_im, int* dims, double* out, size_t capacity) {
  return guarded(nullptr, [&] {
    ARG_CHECK(dims != nullptr, "dims must not be NULL");
    HostMPO h = build_host_mpo(n_sites, terms, n_terms, zc(c0_re, c0_im), zc(c1_re, c1_im));
    for (int b = 0; b <= n_sites; ++b) dims[b] = h.w[b];
    if (out) {
      size_t need = 0;
      for (auto& W : h.W) need += 2 * W.size();
      ARG_CHECK(capacity >= need, "output capacity too small");
      size_t off = 0;
      for (auto& W : h.W)
        for (const zc& x : W) {
          out[off++] = x.real();
          out[off++] = x.imag();
        }
    }
  });
}

tdvp_status tdvp_mpo_charges_host(int n_sites, const tdvp_term* terms, int n_terms, double c0_re, double c0_im,
                                  double c1_re, double c1_im, int* conserves, int* charges, size_t capacity) {
  return guarded(nullptr, [&] {
    ARG_CHECK(conserves != nullptr, "conserves must not be NULL");
    HostMPO h = build_host_mpo(n_sites, terms, n_terms, zc(c0_re, c0_im), zc(c1_re, c1_im));
    *conserves = h.u1 ? 1 : 0;
    if (!h.u1 || !charges) return;
    size_t need = 0;
    for (int b = 0; b <= n_sites; ++b) need += h.w[b];
    ARG_CHECK(capacity >= need, "capacity too small");
    size_t off = 0;
    for (auto& q : h.qw)
      for (int v : q) charges[off++] = v;
  });
}

tdvp_status tdvp_create_mpo(tdvp_ctx ctx, int n_sites, const tdvp_term* terms, int n_terms, double c0_re,
                            double c0_im, double c1_re, double c1_im, tdvp_mpo* out, int* w_out) {
  if (!ctx || !out) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    bind(ctx);
    HostMPO h = build_host_mpo(n_sites, terms, n_terms, zc(c0_re, c0_im), zc(c1_re, c1_im));
    for (auto& W : h.W)
      for (const zc& x : W) ARG_CHECK(std::isfinite(x.real()) && std::isfinite(x.imag()), "non-finite coefficient");
    if (w_out)
      for (int b = 0; b <= n_sites; ++b) w_out[b] = h.w[b];
    for (int b = 0; b <= n_sites; ++b) ARG_CHECK(h.w[b] <= 32, "MPO bond dimension above 32 is not supported");
    *out = make_mpo(ctx, std::move(h)).release();
  });
}

tdvp_status tdvp_mpo_to_host(tdvp_mpo mpo, double* out, size_t capacity) {
  if (!mpo || !out) return TDVP_ERR_ARG;
  return guarded(mpo->ctx, [&] {
    size_t need = 0;
    for (auto& W : mpo->host.W) need += 2 * W.size();
    ARG_CHECK(capacity >= need, "output capacity too small");
    size_t off = 0;
    for (auto& W : mpo->host.W)
      for (const zc& x : W) {
        out[off++] = x.real();
        out[off++] = x.imag();
      }
  });
}

void tdvp_mpo_destroy(tdvp_mpo mpo) {
  if (!mpo) return;
  (void)hipSetDevice(mpo->ctx->device);
  (void)hipStreamSynchronize(mpo->ctx->stream);
  delete mpo;
}

// ------------------------------------------------------------------ MPS
tdvp_status tdvp_mps_from_host(tdvp_ctx ctx, int n_sites, const int* bond_dims, const double* tensors,
                               const int* charges, tdvp_mps* out) {
  if (!ctx || !out) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(n_sites >= 1, "n_sites must be >= 1");
    ARG_CHECK(bond_dims && tensors, "NULL array");
    ARG_CHECK(bond_dims[0] == 1 && bond_dims[n_sites] == 1, "first and last bond dimensions must be 1");
    size_t total = 0;
    for (int i = 0; i <= n_sites; ++i) ARG_CHECK(bond_dims[i] >= 1 && bond_dims[i] <= (1 << 16), "bad bond dimension");
    for (int i = 0; i < n_sites; ++i) total += (size_t)bond_dims[i] * 2 * bond_dims[i + 1];
    ARG_CHECK(all_finite(tensors, 2 * total), "non-finite tensor entry");
    if (charges) {
      // every bond ascending; entries outside q(b) = q(a) + q(s) exactly zero
      std::vector<size_t> qoff(n_sites + 2, 0);
      for (int b = 0; b <= n_sites; ++b) qoff[b + 1] = qoff[b] + bond_dims[b];
      for (int b = 0; b <= n_sites; ++b)
        for (size_t x = qoff[b] + 1; x < qoff[b + 1]; ++x)
          ARG_CHECK(charges[x - 1] <= charges[x], "charges of a bond must ascend");
      size_t off = 0;
      for (int i = 0; i < n_sites; ++i) {
        const int ml = bond_dims[i], mr = bond_dims[i + 1];
        for (int a = 0; a < ml; ++a)
          for (int sp = 0; sp < 2; ++sp)
            for (int b = 0; b < mr; ++b) {
              const size_t e = off + ((size_t)a * 2 + sp) * mr + b;
              const bool allowed = charges[qoff[i + 1] + b] == charges[qoff[i] + a] + phys_charge(sp);
              ARG_CHECK(allowed || (tensors[2 * e] == 0.0 && tensors[2 * e + 1] == 0.0),
                        "tensor entry outside the charge blocks is not zero");
            }
        off += (size_t)ml * 2 * mr;
      }
    }
    bind(ctx);
    *out = make_mps(ctx, n_sites, bond_dims, tensors, charges).release();
  });
}

tdvp_status tdvp_mps_charges(tdvp_mps mps, int* has_charges, int* charges, size_t capacity) {
  if (!mps || !has_charges) return TDVP_ERR_ARG;
  return guarded(mps->ctx, [&] {
    *has_charges = mps->u1() ? 1 : 0;
    if (!mps->u1() || !charges) return;
    size_t need = 0;
    for (int b = 0; b <= mps->N; ++b) need += mps->m[b];
    ARG_CHECK(capacity >= need, "capacity too small");
    size_t off = 0;
    for (int b = 0; b <= mps->N; ++b)
      for (int v : mps->q[b]) charges[off++] = v;
  });
}

tdvp_status tdvp_mps_bond_dims(tdvp_mps mps, int* n_sites, int* bond_dims, int capacity) {
  if (!mps) return TDVP_ERR_ARG;
  return guarded(mps->ctx, [&] {
    if (n_sites) *n_sites = mps->N;
    if (bond_dims) {
      ARG_CHECK(capacity >= mps->N + 1, "capacity too small");
      for (int b = 0; b <= mps->N; ++b) bond_dims[b] = mps->m[b];
    }
  });
}

tdvp_status tdvp_mps_to_host(tdvp_mps mps, double* tensors, size_t capacity) {
  if (!mps || !tensors) return TDVP_ERR_ARG;
  return guarded(mps->ctx, [&] {
    if (!mps->valid) TDVP_THROW(TDVP_ERR_STATE, "MPS handle was invalidated by an earlier failure");
    size_t need = 0;
    for (int i = 0; i < mps->N; ++i) need += 2 * (size_t)mps->elems(i);
    ARG_CHECK(capacity >= need, "output capacity too small");
    bind(mps->ctx);
    size_t off = 0;
    for (int i = 0; i < mps->N; ++i) {
      const size_t bytes = (size_t)mps->elems(i) * 16;
      HIP_CHECK(hipMemcpyAsync(tensors + off, mps->t[i].p, bytes, hipMemcpyDeviceToHost, mps->ctx->stream));
      off += 2 * (size_t)mps->elems(i);
    }
    mps->ctx->sync();
  });
}

void tdvp_mps_destroy(tdvp_mps mps) {
  if (!mps) return;
  if (mps->ctx) {
    (void)hipSetDevice(mps->ctx->device);
    (void)hipStreamSynchronize(mps->ctx->stream);
  }
  delete mps;
}

tdvp_status tdvp_apply_mpo(tdvp_ctx ctx, tdvp_mps in, tdvp_mpo op, int method, double eps, int chi_max,
                           int passes, tdvp_mps* out, double* discarded) {
  if (!ctx || !out) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(in && op, "NULL handle");
    ARG_CHECK(in->N == op->N(), "MPS and MPO site counts differ");
    ARG_CHECK(!in->u1() || op->host.u1, "a state with charges needs an MPO that conserves S^z");
    ARG_CHECK(std::isfinite(eps) && eps >= 0, "eps must be >= 0");
    ARG_CHECK(chi_max >= 1, "chi_max must be >= 1");
    ARG_CHECK(method == TDVP_APPLY_DENMAT || method == TDVP_APPLY_FIT, "unknown method");
    if (method == TDVP_APPLY_FIT) {
      ARG_CHECK(passes >= 1, "passes must be >= 1");
      ARG_CHECK(in->N >= 2, "the variational route needs at least two sites");
    }
    if (!in->valid || !op->valid) TDVP_THROW(TDVP_ERR_STATE, "handle invalidated by an earlier failure");
    bind(ctx);
    auto res = std::make_unique<tdvp_mps_s>();
    run_apply_mpo(ctx, *in, *op, method, eps, chi_max, passes, *res, discarded);
    *out = res.release();
  });
}

// ------------------------------------------------------------ GSE-TDVP1
tdvp_status tdvp_expand_basis(tdvp_ctx ctx, int n, tdvp_mps* psi, const tdvp_mpo* op,
                              const tdvp_expand_params* params, tdvp_expand_stats* stats) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(n >= 1 && psi && op && params, "bad arguments");
    const tdvp_expand_params& p = *params;
    ARG_CHECK(p.k >= 1 && p.k <= 16, "k must be in 1..16");
    ARG_CHECK(p.chi_max >= 1, "chi_max must be >= 1");
    ARG_CHECK(p.eps_K >= 0 && p.eps_M >= 0, "cutoffs must be >= 0");
    ARG_CHECK(p.prec >= TDVP_FP64 && p.prec <= TDVP_BF16X3_FP32ACC, "unknown precision");
    ARG_CHECK(p.apply_method == TDVP_APPLY_DENMAT || p.apply_method == TDVP_APPLY_FIT, "unknown apply_method");
    for (int j = 0; j < n; ++j) {
      ARG_CHECK(psi[j] && op[j], "NULL handle");
      ARG_CHECK(psi[j]->N == op[j]->N(), "MPS and MPO site counts differ");
      ARG_CHECK(!psi[j]->u1() || op[j]->host.u1, "a state with charges needs an MPO that conserves S^z");
      ARG_CHECK(p.apply_method != TDVP_APPLY_FIT || psi[j]->N >= 2, "the variational route needs at least two sites");
      if (!psi[j]->valid || !op[j]->valid) TDVP_THROW(TDVP_ERR_STATE, "handle invalidated by an earlier failure");
    }
    check_distinct(n, psi);
    bind(ctx);
    for_instances(ctx, n, [&](tdvp_ctx_s* c, int j) {
      tdvp_expand_stats st{};
      try {
        run_expand(c, *psi[j], *op[j], p, st);
      } catch (...) {
        psi[j]->valid = false;
        throw;
      }
      if (stats) stats[j] = st;
    });
  });
}

tdvp_status tdvp_sweep(tdvp_ctx ctx, int n, tdvp_mps* psi, const tdvp_mpo* H, const tdvp_sweep_params* params,
                       tdvp_sweep_stats* stats) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(n >= 1 && psi && H && params, "bad arguments");
    const tdvp_sweep_params& p = *params;
    ARG_CHECK(std::isfinite(p.dt_re) && std::isfinite(p.dt_im), "non-finite time step");
    ARG_CHECK(p.eps >= 0, "eps must be >= 0");
    ARG_CHECK(p.chi_max >= 1, "chi_max must be >= 1");
    ARG_CHECK(p.krylov_max >= 1 && p.krylov_max <= 64, "krylov_max must be in 1..64");
    ARG_CHECK(p.krylov_tol >= 0, "krylov_tol must be >= 0");
    ARG_CHECK(p.prec >= TDVP_FP64 && p.prec <= TDVP_BF16X3_FP32ACC, "unknown precision");
    for (int j = 0; j < n; ++j) {
      ARG_CHECK(psi[j] && H[j], "NULL handle");
      ARG_CHECK(psi[j]->N == H[j]->N(), "MPS and MPO site counts differ");
      ARG_CHECK(!psi[j]->u1() || H[j]->host.u1, "a state with charges needs an MPO that conserves S^z");
      if (!psi[j]->valid || !H[j]->valid) TDVP_THROW(TDVP_ERR_STATE, "handle invalidated by an earlier failure");
    }
    check_distinct(n, psi);
    bind(ctx);
    for_instances(ctx, n, [&](tdvp_ctx_s* c, int j) {
      tdvp_sweep_stats st{};
      try {
        run_sweep(c, *psi[j], *H[j], p, st);
      } catch (...) {
        psi[j]->valid = false;
        throw;
      }
      if (stats) stats[j] = st;
      // strict mode: the sweep has run to its end with the unconverged local
      // results, so the state stays valid and the statistics are filled in
      if (p.strict && st.n_unconverged > 0)
        TDVP_THROW(TDVP_ERR_NOCONV, std::to_string(st.n_unconverged) +
                                        " local Lanczos runs reached krylov_max without converging");
    });
  });
}

tdvp_status tdvp_sweep2(tdvp_ctx ctx, int n, tdvp_mps* psi, const tdvp_mpo* H, const tdvp_sweep_params* params,
                       tdvp_sweep_stats* stats) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(n >= 1 && psi && H && params, "bad arguments");
    for (int j = 0; j < n; ++j) ARG_CHECK(psi[j] && psi[j]->N >= 2, "two-site TDVP needs at least two sites");
    const tdvp_sweep_params& p = *params;
    ARG_CHECK(std::isfinite(p.dt_re) && std::isfinite(p.dt_im), "non-finite time step");
    ARG_CHECK(p.eps >= 0, "eps must be >= 0");
    ARG_CHECK(p.chi_max >= 1, "chi_max must be >= 1");
    ARG_CHECK(p.krylov_max >= 1 && p.krylov_max <= 64, "krylov_max must be in 1..64");
    ARG_CHECK(p.krylov_tol >= 0, "krylov_tol must be >= 0");
    ARG_CHECK(p.prec >= TDVP_FP64 && p.prec <= TDVP_BF16X3_FP32ACC, "unknown precision");
    for (int j = 0; j < n; ++j) {
      ARG_CHECK(psi[j] && H[j], "NULL handle");
      ARG_CHECK(psi[j]->N == H[j]->N(), "MPS and MPO site counts differ");
      ARG_CHECK(!psi[j]->u1() || H[j]->host.u1, "a state with charges needs an MPO that conserves S^z");
      if (!psi[j]->valid || !H[j]->valid) TDVP_THROW(TDVP_ERR_STATE, "handle invalidated by an earlier failure");
    }
    check_distinct(n, psi);
    bind(ctx);
    for_instances(ctx, n, [&](tdvp_ctx_s* c, int j) {
      tdvp_sweep_stats st{};
      try {
        run_sweep2(c, *psi[j], *H[j], p, st);
      } catch (...) {
        psi[j]->valid = false;
        throw;
      }
      if (stats) stats[j] = st;
      // strict mode: the sweep has run to its end with the unconverged local
      // results, so the state stays valid and the statistics are filled in
      if (p.strict && st.n_unconverged > 0)
        TDVP_THROW(TDVP_ERR_NOCONV, std::to_string(st.n_unconverged) +
                                        " local Lanczos runs reached krylov_max without converging");
    });
  });
}

tdvp_status tdvp_measure(tdvp_ctx ctx, int n, const tdvp_mps* psi, const tdvp_mpo* H, const tdvp_mps* other,
                         tdvp_observables* out) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(n >= 1 && psi && out, "bad arguments");
    for (int j = 0; j < n; ++j) {
      ARG_CHECK(psi[j], "NULL handle");
      if (!psi[j]->valid) TDVP_THROW(TDVP_ERR_STATE, "handle invalidated by an earlier failure");
      if (H) ARG_CHECK(H[j] && H[j]->N() == psi[j]->N, "MPO does not match the MPS");
      if (other) ARG_CHECK(other[j] && other[j]->N == psi[j]->N, "other MPS does not match");
    }
    bind(ctx);
    for_instances(ctx, n, [&](tdvp_ctx_s* c, int j) {
      run_measure(c, *psi[j], H ? H[j] : nullptr, other ? other[j] : nullptr, out[j]);
    });
  });
}

tdvp_status tdvp_squeezing_xi2(int n_spins, double sx, double sy, double sz, double syy, double szz, double syz_sym,
                               double* xi2) {
  return guarded(nullptr, [&] {
    ARG_CHECK(n_spins >= 1 && xi2, "bad arguments");
    ARG_CHECK(std::isfinite(sx) && std::isfinite(sy) && std::isfinite(sz) && std::isfinite(syy) &&
                  std::isfinite(szz) && std::isfinite(syz_sym),
              "non-finite moment");
    ARG_CHECK(sx != 0.0, "<S^x> must not vanish");
    const double vyy = syy - sy * sy, vzz = szz - sz * sz, vyz = 0.5 * syz_sym - sy * sz;
    const double v = 0.5 * (vyy + vzz - std::sqrt((vyy - vzz) * (vyy - vzz) + 4.0 * vyz * vyz));
    *xi2 = n_spins * v / (sx * sx);
  });
}

// ---------------------------------------------------------- kernel level
tdvp_status tdvp_gemm(tdvp_ctx ctx, int prec, int op_a, int op_b, int M, int N, int K, double alpha_re,
                      double alpha_im, const void* A, long long lda, long long stride_a, const void* B, long long ldb,
                      long long stride_b, double beta_re, double beta_im, void* C, long long ldc, long long stride_c,
                      int batch) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(M >= 0 && N >= 0 && K >= 0 && batch >= 0, "negative size");
    ARG_CHECK(op_a >= 0 && op_a <= 3 && op_b >= 0 && op_b <= 3, "bad op");
    ARG_CHECK(prec >= TDVP_FP64 && prec <= TDVP_BF16X3_FP32ACC, "unknown precision");
    bind(ctx);
    // split-K scratch for long-K products with few output tiles
    kern::SplitWorkspaceScope gws(ctx->split_workspace(), tdvp_ctx_s::SPLIT_WS_BYTES);
    if (prec == TDVP_FP64)
      kern::gemm<double>(ctx->stream, op_a, op_b, M, N, K, zc(alpha_re, alpha_im), A, lda, stride_a, B, ldb, stride_b,
                         zc(beta_re, beta_im), C, ldc, stride_c, batch);
    else {
      kern::FloatModeScope mode(kern::float_mode_of(prec));
      kern::gemm<float>(ctx->stream, op_a, op_b, M, N, K, zc(alpha_re, alpha_im), A, lda, stride_a, B, ldb, stride_b,
                        zc(beta_re, beta_im), C, ldc, stride_c, batch);
    }
  });
}


tdvp_status tdvp_eigh(tdvp_ctx ctx, int method, int n, const void* H, void* rows, double* lam) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(n >= 1 && H && rows && lam, "bad arguments");
    ARG_CHECK(method >= la::EIGH_AUTO && method <= la::EIGH_TRIDIAG_LIB, "unknown method");
    bind(ctx);
    kern::SplitWorkspaceScope gws(ctx->split_workspace(), tdvp_ctx_s::SPLIT_WS_BYTES);
    DBuf work(ctx);
    std::vector<double> w;
    la::eigh_rows_desc(ctx, H, n, w, rows, work, method);
    std::copy(w.begin(), w.end(), lam);
    ctx->sync();
  });
}

tdvp_status tdvp_eigh_sectors(tdvp_ctx ctx, int n, const void* H, const int32_t* charges, void* rows,
                              double* lam, int32_t* charges_out) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(n >= 1 && H && charges && rows && lam && charges_out, "bad arguments");
    bind(ctx);
    kern::SplitWorkspaceScope gws(ctx->split_workspace(), tdvp_ctx_s::SPLIT_WS_BYTES);
    DBuf work(ctx);
    const std::vector<int> q(charges, charges + n);
    std::vector<double> w;
    std::vector<int> qo;
    la::eigh_sectors(ctx, H, n, q, w, rows, work, qo);
    std::copy(w.begin(), w.end(), lam);
    std::copy(qo.begin(), qo.end(), charges_out);
    ctx->sync();
  });
}

tdvp_status tdvp_cholesky(tdvp_ctx ctx, int n, const void* G, void* L, void* Linv, int* info) {
  if (!ctx) return TDVP_ERR_ARG;
  return guarded(ctx, [&] {
    ARG_CHECK(n >= 1 && n <= kern::cholinv_max_n() && G && L && Linv && info, "bad arguments");
    ARG_CHECK(Linv != G && Linv != L, "Linv must not be G or L");
    bind(ctx);
    DBuf work(ctx);
    char* base = static_cast<char*>(work.ensure(256 + kern::cholinv_scratch_bytes()));
    int* dinfo = reinterpret_cast<int*>(base);
    if (kern::cholinv(ctx->stream, G, n, L, Linv, dinfo, base + 256) != hipSuccess) {
      (void)hipGetLastError();
      TDVP_THROW(TDVP_ERR_DEVICE, "Cholesky factorisation launch failed");
    }
    *info = *static_cast<const int*>(ctx->fetch(dinfo, sizeof(int)));
  });
}

tdvp_status tdvp_heff_apply(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr, const double* W_host,
                            const void* L, const void* Rt, const void* C, void* Y, void* workspace) {
  if (!W_host) return TDVP_ERR_ARG;
  return kernel_call(ctx, prec, ml, wl, wr, mr, W_host, workspace,
                     [&](const SiteTables& tb, void* w1, void* w2, SplitWS sk) {
    if (prec == TDVP_FP64) heff_apply<double>(ctx, tb, ml, wl, wr, mr, L, Rt, C, Y, w1, w2, nullptr, sk);
    else heff_apply<float>(ctx, tb, ml, wl, wr, mr, L, Rt, C, Y, w1, w2, nullptr, sk);
  });
}

tdvp_status tdvp_heff_apply_u1(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr, const double* W_host,
                               const int32_t* charges_l, const int32_t* charges_r, const int32_t* qw_l,
                               const int32_t* qw_r, const void* L, const void* Rt, const void* C, void* Y) {
  if (!W_host || !charges_l || !charges_r || !qw_l || !qw_r) return TDVP_ERR_ARG;
  return kernel_call(ctx, prec, ml, wl, wr, mr, W_host, nullptr,
                     [&](const SiteTables& tb, void* w1, void* w2, SplitWS sk) {
    const std::vector<int> ql(charges_l, charges_l + ml), qr(charges_r, charges_r + mr);
    const std::vector<int> qwl(qw_l, qw_l + wl), qwr(qw_r, qw_r + wr);
    for (int a = 0; a < wl; ++a)
      for (int b = 0; b < wr; ++b)
        for (int sp = 0; sp < 2; ++sp)
          for (int sk2 = 0; sk2 < 2; ++sk2) {
            const size_t e = ((((size_t)a * wr + b) * 2 + sp) * 2 + sk2) * 2;
            if (W_host[e] == 0.0 && W_host[e + 1] == 0.0) continue;
            ARG_CHECK(phys_charge(sk2) - qwl[a] == phys_charge(sp) - qwr[b], "W entry breaks the channel charges");
          }
    MapCache& mc = map_cache(ctx);
    const MapEntry& e1 = cmap_env_gemm1_nz(mc, ql, ql, qwl, qr);
    const MapEntry& e2 = cmap_heff_gemm2(mc, ql, qr, qwr, qr);
    const kern::KMap g1 = mc.use(e1), g2 = mc.use(e2);
    ProdMaps pm{&g1, &g2, e1.exact_flops + e2.exact_flops};
    kern::WCharges wc = wc_of(cmap_wstage(mc, ql, qr, qwl, qwr), ml, mr, wl);
    // the stage stores only the outputs allowed by charge into cleared memory
    kern::zfill(ctx->stream, w2, zc(0.0, 0.0), 2LL * ml * wr * mr, prec == TDVP_FP64 ? 16 : 8);
    wc.zeros_kept = 1;
    pm.wc = &wc;
    if (prec == TDVP_FP64) heff_apply<double>(ctx, tb, ml, wl, wr, mr, L, Rt, C, Y, w1, w2, nullptr, sk, pm);
    else heff_apply<float>(ctx, tb, ml, wl, wr, mr, L, Rt, C, Y, w1, w2, nullptr, sk, pm);
  });
}

tdvp_status tdvp_keff_apply(tdvp_ctx ctx, int prec, int ml, int w, int mr, const void* L, const void* Rt,
                            const void* X, void* Y, void* workspace) {
  return kernel_call(ctx, prec, ml, w, w, mr, nullptr, workspace, [&](const SiteTables&, void* w1, void*, SplitWS sk) {
    if (prec == TDVP_FP64) keff_apply<double>(ctx, ml, w, mr, L, Rt, X, Y, w1, sk);
    else keff_apply<float>(ctx, ml, w, mr, L, Rt, X, Y, w1, sk);
  });
}

tdvp_status tdvp_env_left(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr, const double* W_host,
                          const void* L, const void* A, void* Lout, void* workspace) {
  if (!W_host) return TDVP_ERR_ARG;
  return kernel_call(ctx, prec, ml, wl, wr, mr, W_host, workspace,
                     [&](const SiteTables& tb, void* w1, void* w2, SplitWS sk) {
    if (prec == TDVP_FP64) env_left<double>(ctx, tb, ml, wl, wr, mr, L, A, Lout, w1, w2, sk);
    else env_left<float>(ctx, tb, ml, wl, wr, mr, L, A, Lout, w1, w2, sk);
  });
}

tdvp_status tdvp_env_right(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr, const double* W_host,
                           const void* Rt, const void* B, void* Rout, void* workspace) {
  if (!W_host) return TDVP_ERR_ARG;
  return kernel_call(ctx, prec, ml, wl, wr, mr, W_host, workspace,
                     [&](const SiteTables& tb, void* w1, void* w2, SplitWS sk) {
    if (prec == TDVP_FP64) env_right<double>(ctx, tb, ml, wl, wr, mr, Rt, B, Rout, w1, w2, sk);
    else env_right<float>(ctx, tb, ml, wl, wr, mr, Rt, B, Rout, w1, w2, sk);
  });
}

}  // extern "C"
