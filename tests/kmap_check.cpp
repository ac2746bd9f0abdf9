// Host-side check of the block-sparse product maps (blocks.cpp), built
// without a device by tests/test_kmap_host.py.  For random charge lists it
// checks by brute force what the GEMM kernels rely on:
//  * every nonzero term (m, n, k) of C[m, n] = sum_k A[m, k] B[k, n], i.e.
//    rq[m] == kq[k] == cq[n], is computed by exactly one entry (tile, rows,
//    columns, K intervals, split part);
//  * an unsplit map writes every output (m, n) exactly once, and an entry
//    flagged as sharing no charge holds no (m, n) with rq[m] == cq[n];
//  * split parts of one sub-block walk disjoint K ranges, and tinfo counts
//    the parts each sub-block keeps;
//  * the upload order lists the work items by non-increasing K length, equal
//    lengths in entry order, and leaves out exactly the entries it should;
//  * a batched map (one product per MPO channel, joined) holds, for each
//    channel, exactly the map of that channel's product.
// Prints "ok" and exits 0, or prints the first failure and exits 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "engine.h"

// The device side of the library is not linked: these stand in for it (the
// builders only need them through MapCache, which this check does not use).
thread_local tdvp_ctx_s* tl_exec_ctx = nullptr;
void* tdvp_ctx_s::dalloc(size_t) { return nullptr; }
void tdvp_ctx_s::dfree(void*) {}
void tdvp_ctx_s::upload_async(void*, const void*, size_t) {}
namespace kern {
template <>
void gemm<double>(hipStream_t, int, int, int, int, int, zc, const void*, long long, long long, const void*, long long,
                  long long, zc, void*, long long, long long, int, void*, size_t) {}
const KMap* current_kmap() { return nullptr; }
void set_kmap(const KMap*) {}
}  // namespace kern

namespace {

int fails = 0;
#define CHECK(cond, ...)                              \
  do {                                                \
    if (!(cond)) {                                    \
      if (fails++ < 5) {                              \
        std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
        std::printf(__VA_ARGS__);                     \
        std::printf("\n");                            \
      }                                               \
    }                                                 \
  } while (0)

std::vector<int> charges(std::mt19937& g, int n, int nq, bool sorted) {
  std::vector<int> q(n);
  for (int& x : q) x = 2 * (int)(g() % nq) - nq;
  if (sorted) std::sort(q.begin(), q.end());
  return q;
}

void check_map(const KMapHost& h, const std::vector<int>& rq, const std::vector<int>& kq, const std::vector<int>& cq,
               const char* what) {
  const int M = (int)rq.size(), N = (int)cq.size(), K = (int)kq.size();
  const int E = (int)h.ivb.size();
  const int tn = (N + 63) / 64;
  CHECK(h.M == M && h.N == N && h.K == K, "%s: sizes", what);
  // term[(m * N + n) * K + k]: how many entries compute term (m, n, k);
  // out[m * N + n]: how many entries write output (m, n)
  std::vector<unsigned char> term((size_t)M * N * K, 0), out((size_t)M * N, 0);
  for (int e = 0; e < E; ++e) {
    const int t = h.etile[e], tr = t / tn, tc = t % tn;
    const int* rg = &h.erng[4 * (size_t)e];
    CHECK(rg[0] < rg[1] && rg[2] < rg[3] && rg[0] >= 0 && rg[1] <= 64 && rg[2] >= 0 && rg[3] <= 64,
          "%s: entry %d rows/cols", what, e);
    CHECK(h.ivb[e] <= h.ive[e] && h.ive[e] <= (int)(h.iv.size() / 2), "%s: entry %d interval range", what, e);
    bool anymatch = false;
    for (int r = rg[0]; r < rg[1]; ++r)
      for (int c = rg[2]; c < rg[3]; ++c) {
        const int m = tr * 64 + r, n = tc * 64 + c;
        if (m >= M || n >= N) continue;
        if (h.splits == 1) out[(size_t)m * N + n]++;
        if (rq[m] == cq[n]) anymatch = true;
        for (int v = h.ivb[e]; v < h.ive[e]; ++v) {
          const int x = h.iv[2 * v], y = h.iv[2 * v + 1];
          CHECK(0 <= x && x < y && y <= K, "%s: entry %d interval [%d, %d)", what, e, x, y);
          for (int k = x; k < y && k < K; ++k)
            if (rq[m] == kq[k] && kq[k] == cq[n]) term[((size_t)m * N + n) * K + k]++;
        }
      }
    if (h.splits == 1 && (size_t)e < h.enone.size() && h.enone[e]) CHECK(!anymatch, "%s: entry %d flagged empty", what, e);
  }
  for (int m = 0; m < M; ++m)
    for (int n = 0; n < N; ++n) {
      if (h.splits == 1) CHECK(out[(size_t)m * N + n] == 1, "%s: output (%d, %d) written %d times", what, m, n,
                               out[(size_t)m * N + n]);
      for (int k = 0; k < K; ++k) {
        const bool nz = rq[m] == kq[k] && kq[k] == cq[n];
        const int c = term[((size_t)m * N + n) * K + k];
        CHECK(c == (nz ? 1 : 0), "%s: term (%d, %d, %d) computed %d times", what, m, n, k, c);
      }
    }
  // split parts: part indices of one sub-block distinct, counted in tinfo
  if (h.splits > 1) {
    std::vector<std::vector<int>> seen((size_t)h.tiles * 4);
    for (int e = 0; e < E; ++e) {
      const int t = h.etile[e] % h.tiles;
      const int* rg = &h.erng[4 * (size_t)e];
      const int sub = (rg[0] >= h.tinfo[6 * (size_t)t] ? 2 : 0) + (rg[2] >= h.tinfo[6 * (size_t)t + 1] ? 1 : 0);
      seen[(size_t)t * 4 + sub].push_back(h.epart[e]);
      CHECK(h.epart[e] >= 0 && h.epart[e] < h.splits, "%s: part index", what);
    }
    for (int t = 0; t < h.tiles; ++t)
      for (int sub = 0; sub < 4; ++sub) {
        auto& v = seen[(size_t)t * 4 + sub];
        std::sort(v.begin(), v.end());
        CHECK(std::adjacent_find(v.begin(), v.end()) == v.end(), "%s: repeated part", what);
        CHECK((int)v.size() == h.tinfo[6 * (size_t)t + 2 + sub], "%s: tile %d sub %d parts %zu, tinfo %d", what, t,
              sub, v.size(), h.tinfo[6 * (size_t)t + 2 + sub]);
      }
  }
}

void check_order(const KMapHost& h, const char* what) {
  const int E = (int)h.ivb.size();
  std::vector<long long> kl(E, 0);
  std::vector<int> want;
  for (int e = 0; e < E; ++e) {
    for (int v = h.ivb[e]; v < h.ive[e]; ++v) kl[e] += h.iv[2 * v + 1] - h.iv[2 * v];
    const bool drop = (h.splits > 1 && kl[e] == 0) ||
                      (h.splits == 1 && h.drop_empty && (size_t)e < h.enone.size() && h.enone[e]);
    if (!drop) want.push_back(e);
  }
  std::stable_sort(want.begin(), want.end(), [&](int x, int y) { return kl[x] > kl[y]; });
  CHECK(kmap_item_order(h) == want, "%s: upload order", what);
}

// entries of batch entry x of a batched map, as a map of its own
KMapHost batch_part(const KMapHost& h, int x) {
  KMapHost p;
  p.M = h.M;
  p.N = h.N;
  p.K = h.K;
  p.tiles = h.tiles;
  p.splits = h.splits;
  p.iv = h.iv;
  for (size_t e = 0; e < h.ivb.size(); ++e) {
    if (h.etile[e] / h.tiles != x) continue;
    p.ivb.push_back(h.ivb[e]);
    p.ive.push_back(h.ive[e]);
    p.etile.push_back(h.etile[e] % h.tiles);
    p.erng.insert(p.erng.end(), h.erng.begin() + 4 * e, h.erng.begin() + 4 * e + 4);
    p.epart.push_back(h.epart[e]);
    if (e < h.enone.size()) p.enone.push_back(h.enone[e]);
  }
  p.tinfo.assign(h.tinfo.begin() + (size_t)6 * h.tiles * x, h.tinfo.begin() + (size_t)6 * h.tiles * (x + 1));
  return p;
}

}  // namespace

int main() {
  std::mt19937 g(20050610);
  for (int rep = 0; rep < 60; ++rep) {
    const int nq = 1 + (int)(g() % 5);
    const bool sorted = rep % 3 != 0;   // bonds keep their charges sorted; fused indices do not
    const int M = 1 + (int)(g() % 150), N = 1 + (int)(g() % 150);
    // long K with few tiles exercises the split path
    const int K = rep % 4 == 0 ? 600 + (int)(g() % 900) : 1 + (int)(g() % 200);
    const auto rq = charges(g, M, nq, sorted), cq = charges(g, N, nq, sorted), kq = charges(g, K, nq, rep % 2 == 0);
    KMapHost h;
    build_kmap(rq, kq, cq, h);
    check_map(h, rq, kq, cq, "unsplit");
    check_order(h, "unsplit");
    h.drop_empty = true;
    check_order(h, "unsplit, empty dropped");
    KMapHost s = h;
    s.drop_empty = false;
    split_kmap(s);
    check_map(s, rq, kq, cq, s.splits > 1 ? "split" : "split (kept whole)");
    check_order(s, "split");
  }
  // batched maps (one per MPO channel, joined): K_eff's first product,
  // L[(a',al),a] X[a,b] with rows a' needing q(a') - q(al), and its second,
  // Y1[a',(al,b)] Rt[(al,b),b'] over the fused index
  for (int rep = 0; rep < 12; ++rep) {
    const int nq = 1 + (int)(g() % 4), ml = 1 + (int)(g() % 140), mr = 1 + (int)(g() % 140), w = 1 + (int)(g() % 7);
    const auto ql = charges(g, ml, nq, true), qr = charges(g, mr, nq, true);
    std::vector<int> qw(w);
    for (int& x : qw) x = 2 * (int)(g() % 3) - 2;
    KMapHost g1, g2;
    kmap_keff(ql, qr, qw, g1, g2);
    CHECK(g1.batch == w, "keff first product: batch %d, channels %d", g1.batch, w);
    for (int x = 0; x < w; ++x) {
      std::vector<int> rq(ml);
      for (int i = 0; i < ml; ++i) rq[i] = ql[i] - qw[x];
      check_map(batch_part(g1, x), rq, ql, qr, "keff first product, one channel");
    }
    check_order(g1, "keff first product");
    std::vector<int> kq;
    for (int x : qw)
      for (int b : qr) kq.push_back(x + b);
    check_map(g2, ql, kq, qr, "keff second product");
  }
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
