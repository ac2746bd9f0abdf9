// MPS / MPO handles and the GSE-TDVP1 drivers.
#pragma once

#include <functional>
#include <memory>
#include <unordered_map>

#include "common.h"
#include "mpo_host.h"

struct SiteTables {
  kern::WTable F, B, BH;
  long long nnz = 0;
};

struct tdvp_mpo_s {
  tdvp_ctx_s* ctx = nullptr;
  HostMPO host;
  DBuf dev;                      // CSR tables of every site and mode
  std::vector<SiteTables> tab;
  bool valid = true;
  int N() const { return host.N; }
  int w(int b) const { return host.w[b]; }
};

// U(1) charges (twice the total S^z of everything left of a bond, so up = +1
// and down = -1 per site): M[a,s,b] may be nonzero only where
// q(b) = q(a) + q(s).  Every bond of a state that carries charges lists them
// in ascending order, so each charge's indices are contiguous.
inline int phys_charge(int s) { return s == 0 ? 1 : -1; }

struct tdvp_mps_s {
  tdvp_ctx_s* ctx = nullptr;
  int N = 0;
  std::vector<int> m;            // N + 1 bond dims; site i is m[i] x 2 x m[i+1]
  std::vector<DBuf> t;           // complex128 site tensors
  std::vector<std::vector<int>> q;   // empty: no charges; else N + 1 bonds of m[b] charges
  bool valid = true;
  bool u1() const { return !q.empty(); }
  long long elems(int i) const { return (long long)m[i] * 2 * m[i + 1]; }
  double* site(int i) const { return t[i].as<double>(); }
};

std::unique_ptr<tdvp_mpo_s> make_mpo(tdvp_ctx_s* ctx, HostMPO&& host);
std::unique_ptr<tdvp_mps_s> make_mps(tdvp_ctx_s* ctx, int N, const int* dims, const double* host,
                                     const int* charges = nullptr);
void run_apply_mpo(tdvp_ctx_s* ctx, const tdvp_mps_s& in, const tdvp_mpo_s& op, int method, double eps, int chi_max,
                   int passes, tdvp_mps_s& out, double* discarded);

void run_sweep(tdvp_ctx_s* ctx, tdvp_mps_s& psi, const tdvp_mpo_s& H, const tdvp_sweep_params& p,
               tdvp_sweep_stats& st);
void run_sweep2(tdvp_ctx_s* ctx, tdvp_mps_s& psi, const tdvp_mpo_s& H, const tdvp_sweep_params& p,
                tdvp_sweep_stats& st);
void run_expand(tdvp_ctx_s* ctx, tdvp_mps_s& psi, const tdvp_mpo_s& op, const tdvp_expand_params& p,
                tdvp_expand_stats& st);
void run_measure(tdvp_ctx_s* ctx, const tdvp_mps_s& psi, const tdvp_mpo_s* H, const tdvp_mps_s* other,
                 tdvp_observables& out);

// HIP-event timing of the one-site effective Hamiltonian: marks 0..3 bracket
// the first GEMM (0-1), the MPO contraction (1-2) and the second GEMM (2-3).
struct MatvecTimer {
  // HIP events around the two GEMM stages of each H_eff application, in two
  // sets: the Lanczos recurrence enqueues the next application before it
  // reads back the current one, so consecutive applications alternate sets.
  tdvp_ctx_s* ctx = nullptr;
  bool on = false;
  int cur = 0;                      // set the next application records into
  bool pending[2] = {false, false};
  hipEvent_t ev[2][4] = {};
  double ms = 0.0, gemm_ms = 0.0, gemm_flops = 0.0;
  long long n_gemm = 0;
  MatvecTimer() = default;
  MatvecTimer(const MatvecTimer&) = delete;
  MatvecTimer& operator=(const MatvecTimer&) = delete;
  ~MatvecTimer() {
    for (auto& set : ev)
      for (hipEvent_t& e : set)
        if (e) (void)hipEventDestroy(e);
  }
  void mark(int k) {
    if (!on) return;
    if (!ev[cur][k]) HIP_CHECK(hipEventCreate(&ev[cur][k]));
    HIP_CHECK(hipEventRecord(ev[cur][k], ctx->stream));
    if (k == 3) pending[cur] = true;
  }
  // accumulate set `k` (its events must have completed)
  void collect(int k) {
    if (!pending[k]) return;
    float t = 0.f, g1 = 0.f, g2 = 0.f;
    HIP_CHECK(hipEventElapsedTime(&t, ev[k][0], ev[k][3]));
    HIP_CHECK(hipEventElapsedTime(&g1, ev[k][0], ev[k][1]));
    HIP_CHECK(hipEventElapsedTime(&g2, ev[k][2], ev[k][3]));
    ms += t;
    gemm_ms += g1 + g2;
    n_gemm += 2;
    pending[k] = false;
  }
  void collect() { collect(cur); }
  void collect_all() {
    collect(0);
    collect(1);
  }
};

// ------------------------------------------------ block-sparse product maps
// (blocks.cpp).  rq[m]: the charge row m of op(A) needs on the summed index,
// kq[k]: the charge of summed index k, cq[n]: the charge column n of op(B)
// needs on it.
// Entries are sub-blocks of the 64 x 64 output tiles: tile etile[e] (batch
// entry outer, then row-major tiles), rows erng[4e] .. erng[4e+1] and
// columns erng[4e+2] .. erng[4e+3] inside the tile, split part epart[e], K
// intervals iv[ivb[e] .. ive[e]) (the entries of an unsplit map that meet the
// same charges share one list).  tinfo (6 per tile): the row and column
// where the tile's second segment starts (64 if none), then the nonempty
// parts of each of its up to four sub-blocks (split maps).
struct KMapHost {
  std::vector<int> ivb, ive, iv, etile, erng, epart, tinfo;
  // per entry of an unsplit map: 1 when its rows and columns share no
  // charge (every output of the sub-block is zero by charge)
  std::vector<unsigned char> enone;
  double exact_macs = 0.0, tile_macs = 0.0;   // nonzero multiply-adds; those the tiles perform
  int M = 0, N = 0, K = 0, batch = 1, splits = 1, tiles = 0;
  // unsplit maps: leave out the sub-blocks whose rows and columns share no
  // charge (their output is then not written at all; for consumers that
  // read by charge and never touch it)
  bool drop_empty = false;
};
void build_kmap(const std::vector<int>& rq, const std::vector<int>& kq, const std::vector<int>& cq, KMapHost& out);
// Split the K intervals of a map whose nonempty tiles are too few to fill
// the GPU into parts of about equal length (see kern::KMap).
void split_kmap(KMapHost& h);
// The entries of h that become work items, longest K first (equal lengths in
// entry order): the upload order, which spreads the long items over the XCDs.
std::vector<int> kmap_item_order(const KMapHost& h);
// The block-sparse maps of a context on the device, kept between calls and
// keyed by the builder and the charge lists it was given.  Products whose
// operands keep their charges from one call to the next (a sweep's exact
// gauge moves leave every bond's charges as they were; the fitting passes;
// the Newton-Schulz steps of a gauge move) find their map instead of
// building and uploading it again.  Entries never change once made.  Past
// MAX_BYTES of maps the least recently used are dropped, never one of the
// last PROTECT looked up (a caller may still hold those).  The partial
// products of split maps share one buffer: all of a context's work is
// ordered on its stream; a grown buffer replaces the old one, which stays
// allocated (maps handed out earlier point at it) until the cache goes.
struct MapCache {
  struct Entry {
    std::vector<int> key;
    DBuf buf;                 // items, intervals, tile info
    kern::KMap map;           // partials pointer unset
    size_t part_bytes = 0;    // partial products of a split map (complex128-sized)
    double exact_flops = 0.0, tile_flops = 0.0;
    unsigned long long last = 0;
    explicit Entry(tdvp_ctx_s* c) : buf(c) {}
  };
  static constexpr size_t MAX_BYTES = size_t(1) << 30;
  static constexpr unsigned long long PROTECT = 256;
  static constexpr int NSTAGE = 32;
  tdvp_ctx_s* ctx;
  std::unordered_map<unsigned long long, std::vector<std::unique_ptr<Entry>>> tab;
  size_t bytes = 0;
  unsigned long long clock = 0;
  size_t hits = 0, misses = 0, evicted = 0;
  DBuf part;
  std::vector<DBuf> retired;
  // pinned staging of the uploads, reused once their copy has run
  int* stage[NSTAGE] = {};
  size_t stage_cap[NSTAGE] = {};
  hipEvent_t ev[NSTAGE] = {};
  int spos = 0;
  explicit MapCache(tdvp_ctx_s* c) : ctx(c), part(c) {}
  ~MapCache();
  MapCache(const MapCache&) = delete;
  MapCache& operator=(const MapCache&) = delete;
  // the entry of `key`; on a miss `build` fills the host map, which is uploaded
  const Entry& get(std::vector<int>&& key, const std::function<void(KMapHost&)>& build);
  // both entries of a builder that makes two maps at once
  std::pair<const Entry*, const Entry*> get2(std::vector<int>&& k1, std::vector<int>&& k2,
                                             const std::function<void(KMapHost&, KMapHost&)>& build);
  // a launchable copy of e's map (a split map gets the shared partials buffer)
  kern::KMap use(const Entry& e);

 private:
  Entry* find(const std::vector<int>& key, unsigned long long h);
  Entry& insert(std::vector<int>&& key, unsigned long long h, const KMapHost& m);
  void evict();
};
// the context's cache (made on first use)
MapCache& map_cache(tdvp_ctx_s* ctx);
// builder id, then each charge list's length and entries
std::vector<int> map_key(int kind, std::initializer_list<const std::vector<int>*> qs);
// the maps of the contractions (bra bonds qlo, qro; ket bonds qli, qri; MPO
// channels qwl, qwr; equal bra and ket for the effective Hamiltonians).  The
// first products of H_eff, K_eff, the left environments and the two-site
// tensors, and the second of H_eff and the two-site tensor, are batched
// (over the MPO channel, over the physical indices) so that each tile meets
// one charge; the contractions issue them batched when given a map.
void kmap_env_gemm1(const std::vector<int>& qlo, const std::vector<int>& qli, const std::vector<int>& qwl,
                    const std::vector<int>& qri, KMapHost& out);
void kmap_heff_gemm2(const std::vector<int>& qlo, const std::vector<int>& qri, const std::vector<int>& qwr,
                     const std::vector<int>& qro, KMapHost& out);
void kmap_env_left_gemm2(const std::vector<int>& qlo, const std::vector<int>& qro, const std::vector<int>& qri,
                         const std::vector<int>& qwr, KMapHost& out);
// U1[be][(a,s),b'] = ket[(a,s),b] Rt[be][b,b'] batched over be (ket bonds
// qli, qri; bra right bond qro; channels qwr)
void kmap_env_right_gemm1(const std::vector<int>& qli, const std::vector<int>& qri, const std::vector<int>& qwr,
                          const std::vector<int>& qro, KMapHost& out);
void kmap_env_right_gemm3(const std::vector<int>& qli, const std::vector<int>& qwl, const std::vector<int>& qro,
                          const std::vector<int>& qlo, KMapHost& out);
void kmap_keff(const std::vector<int>& ql, const std::vector<int>& qr, const std::vector<int>& qw, KMapHost& g1,
               KMapHost& g2);
void kmap_two_site(const std::vector<int>& qlo, const std::vector<int>& qli, const std::vector<int>& qwl,
                   const std::vector<int>& qri, const std::vector<int>& qwr, const std::vector<int>& qro,
                   KMapHost& g1, KMapHost& g2);
// the same maps out of the context's cache
using MapEntry = MapCache::Entry;
const MapEntry& cmap_env_gemm1(MapCache& c, const std::vector<int>& qlo, const std::vector<int>& qli,
                               const std::vector<int>& qwl, const std::vector<int>& qri);
const MapEntry& cmap_heff_gemm2(MapCache& c, const std::vector<int>& qlo, const std::vector<int>& qri,
                                const std::vector<int>& qwr, const std::vector<int>& qro);
const MapEntry& cmap_env_left_gemm2(MapCache& c, const std::vector<int>& qlo, const std::vector<int>& qro,
                                    const std::vector<int>& qri, const std::vector<int>& qwr);
const MapEntry& cmap_env_right_gemm1(MapCache& c, const std::vector<int>& qli, const std::vector<int>& qri,
                                     const std::vector<int>& qwr, const std::vector<int>& qro);
const MapEntry& cmap_env_right_gemm3(MapCache& c, const std::vector<int>& qli, const std::vector<int>& qwl,
                                     const std::vector<int>& qro, const std::vector<int>& qlo);
std::pair<const MapEntry*, const MapEntry*> cmap_keff(MapCache& c, const std::vector<int>& ql,
                                                      const std::vector<int>& qr, const std::vector<int>& qw);
std::pair<const MapEntry*, const MapEntry*> cmap_two_site(MapCache& c, const std::vector<int>& qlo,
                                                          const std::vector<int>& qli, const std::vector<int>& qwl,
                                                          const std::vector<int>& qri, const std::vector<int>& qwr,
                                                          const std::vector<int>& qro);
// the maps of a contraction's products (null: dense)
struct ProdMaps {
  const kern::KMap* g1 = nullptr;
  const kern::KMap* g2 = nullptr;
  double flops = -1.0;   // nonzero flops of the two products (negative: dense count)
  const kern::WCharges* wc = nullptr;   // charges of the sparse-MPO stage (null: dense)
  const kern::WCharges* wc2 = nullptr;  // of the second stage of a two-site product
};
// The charges of a sparse-MPO stage (element (p, q): row charge qrow[p],
// column charge qcol[q]; MPO channels qwin in, qwout out) as one cached
// device table: qrow, qcol, then q(s) + sign * qwin[x] for input channel
// 2 x + s and q(s') + sign * qwout[y] for output channel 2 y + s'.  The
// stages after a left-side product (H_eff, left environments, two-site
// tensors) take sign = -1, those after a right-side product sign = +1.
// wc_of fills the four pointers.
const MapEntry& cmap_wstage(MapCache& c, const std::vector<int>& qrow, const std::vector<int>& qcol,
                            const std::vector<int>& qwin, const std::vector<int>& qwout, int sign = -1);
kern::WCharges wc_of(const MapEntry& e, int nrow, int ncol, int win);
// First products without the sub-blocks that share no charge, for a stage
// after them that reads by charge (their outputs there are never written):
// H_eff and the left environments, the right environments, the fitting's
// two-site tensor (its second map as in cmap_two_site).
const MapEntry& cmap_env_gemm1_nz(MapCache& c, const std::vector<int>& qlo, const std::vector<int>& qli,
                                  const std::vector<int>& qwl, const std::vector<int>& qri);
const MapEntry& cmap_env_right_gemm1_nz(MapCache& c, const std::vector<int>& qli, const std::vector<int>& qri,
                                        const std::vector<int>& qwr, const std::vector<int>& qro);
std::pair<const MapEntry*, const MapEntry*> cmap_two_site_nz(MapCache& c, const std::vector<int>& qlo,
                                                             const std::vector<int>& qli, const std::vector<int>& qwl,
                                                             const std::vector<int>& qri, const std::vector<int>& qwr,
                                                             const std::vector<int>& qro);

// kernel-level helpers used by the C-ABI
// Split-K scratch for the contractions (may be empty: no K splitting).
struct SplitWS {
  void* p = nullptr;
  size_t bytes = 0;
};

template <typename T>
void heff_apply(tdvp_ctx_s* ctx, const SiteTables& tb, int ml, int wl, int wr, int mr, const void* L,
                const void* Rt, const void* C, void* Y, void* ws1, void* ws2, MatvecTimer* tm = nullptr,
                SplitWS sk = {}, ProdMaps pm = {});
template <typename T>
void keff_apply(tdvp_ctx_s* ctx, int ml, int w, int mr, const void* L, const void* Rt, const void* X, void* Y,
                void* ws1, SplitWS sk = {}, ProdMaps pm = {});
template <typename T>
void env_left(tdvp_ctx_s* ctx, const SiteTables& tb, int ml, int wl, int wr, int mr, const void* L,
              const void* A, void* Lout, void* ws1, void* ws2, SplitWS sk = {}, ProdMaps pm = {});
template <typename T>
void env_right(tdvp_ctx_s* ctx, const SiteTables& tb, int ml, int wl, int wr, int mr, const void* Rt,
               const void* B, void* Rout, void* ws1, void* ws2, SplitWS sk = {}, ProdMaps pm = {});
// CSR tables for a single host W (kernel-level calls); keeps the device copy in `buf`
SiteTables upload_tables(tdvp_ctx_s* ctx, const std::vector<zc>& W, int wl, int wr, DBuf& buf);
// The same tables written into caller-provided device memory (cap bytes at
// dst, allocates nothing on the device): returns the bytes they take; when
// that exceeds cap nothing is written and *out is left as it was.
size_t write_tables(tdvp_ctx_s* ctx, const std::vector<zc>& W, int wl, int wr, void* dst, size_t cap,
                    SiteTables* out);
