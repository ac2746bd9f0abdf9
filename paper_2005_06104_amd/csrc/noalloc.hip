// tdvp_heff_apply_noalloc: the one-site effective Hamiltonian of
// tdvp_heff_apply for callers that cannot allocate device memory.  Its
// scratch (the MPO's CSR tables, the two intermediates of the contraction and
// the split-K partial products) lives in a file-scope device array of fixed
// size that each GPU holds from the library's load until the process ends.
#include <mutex>

#include "engine.h"

namespace {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
constexpr int MAX_DEVICES = 64;

// The device copy of this array is what the kernels use; in host code its
// name only stands for the symbol, so its address on each device is looked
// up once (hipGetSymbolAddress, with that device current) and kept below.
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

void* scratch_on(int device) {
  if (device < 0 || device >= MAX_DEVICES) TDVP_THROW(TDVP_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[device]) {
    // the caller has made `device` current
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      TDVP_THROW(TDVP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

extern "C" tdvp_status tdvp_heff_apply_noalloc(tdvp_ctx ctx, int prec, int ml, int wl, int wr, int mr,
                                               const double* W_host, const void* L, const void* Rt, const void* C,
                                               void* Y) {
  if (!ctx) return TDVP_ERR_ARG;
  try {
    ARG_CHECK(W_host && L && Rt && C && Y, "NULL argument");
    ARG_CHECK(prec >= TDVP_FP64 && prec <= TDVP_BF16X3_FP32ACC, "unknown precision");
    ARG_CHECK(ml >= 1 && mr >= 1 && wl >= 1 && wr >= 1 && wl <= 32 && wr <= 32, "bad sizes");
    HIP_CHECK(hipSetDevice(ctx->device));
    const int cb = prec == TDVP_FP64 ? 16 : 8;
    // the same partition as tdvp_heff_apply's workspace, so the same kernels
    // (and split-K counts) run
    const size_t half = (size_t)2 * ml * mr * std::max(wl, wr) * cb;
    const size_t split = (size_t)32 * ml * mr * cb;
    std::vector<zc> W((size_t)wl * wr * 4);
    for (size_t i = 0; i < W.size(); ++i) W[i] = zc(W_host[2 * i], W_host[2 * i + 1]);
    // tables: rowptr/col/val of three modes, at most (2 w + 1) ints + 4 w^2
    // entries each, 16-byte aligned pieces
    const size_t tab_cap = align256((size_t)3 * (3 * 16 + (2 * 32 + 1) * 4 + (size_t)4 * wl * wr * (4 + 16)));
    const size_t need = tab_cap + 2 * align256(half) + split;
    ARG_CHECK(need <= SCRATCH_BYTES, "sizes need " + std::to_string(need) + " bytes of scratch, above the " +
                                         std::to_string(SCRATCH_BYTES) + "-byte maximum");
    char* base = static_cast<char*>(scratch_on(ctx->device));
    SiteTables tb{};
    const size_t used = write_tables(ctx, W, wl, wr, base, tab_cap, &tb);
    if (used > tab_cap) TDVP_THROW(TDVP_ERR_ARG, "MPO tables exceed their scratch region");
    char* w1 = base + tab_cap;
    char* w2 = w1 + align256(half);
    char* sk = w2 + align256(half);
    kern::FloatModeScope mode(kern::float_mode_of(prec));
    if (prec == TDVP_FP64)
      heff_apply<double>(ctx, tb, ml, wl, wr, mr, L, Rt, C, Y, w1, w2, nullptr, SplitWS{sk, split});
    else
      heff_apply<float>(ctx, tb, ml, wl, wr, mr, L, Rt, C, Y, w1, w2, nullptr, SplitWS{sk, split});
    HIP_CHECK(hipGetLastError());
    ctx->last_error.clear();
    return TDVP_OK;
  } catch (const TdvpError& e) {
    ctx->last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->last_error = e.what();
    return TDVP_ERR_DEVICE;
  } catch (...) {
    ctx->last_error = "unknown failure";
    return TDVP_ERR_DEVICE;
  }
}
