// Block-sparse maps of the products whose operands carry U(1) charges.
//
// A product C[m, n] = sum_k A[m, k] B[k, n] between charged tensors has
// nonzero terms only where the charge a row m needs on the summed index, the
// charge of k, and the charge column n needs on it all agree.  Each 64 x 64
// output tile is cut where the charge of its rows (and of its columns)
// changes, into at most 2 x 2 sub-blocks of one charge each (a tile whose
// rows or columns change charge more than once keeps them as one segment
// with all their charges); every sub-block lists the K intervals of the
// charges its rows and columns share, and the MFMA kernels walk only those,
// skipping the 16 x 16 pieces of the tile outside the sub-block.  Intervals
// closer than a K step are joined (the skipped entries between them are
// exact zeros, so including them changes nothing).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>

#include "engine.h"

namespace {

constexpr int TILE = 64;   // the GEMM kernels' output tile
constexpr int GAP = 32;    // the largest K step of the kernels

struct Run {
  int b, e;
};

// segments of a tile's rows (or columns): each run of one charge when there
// are at most two, else one segment with every charge of the tile
struct Seg {
  int b, e;
  std::vector<int> q;   // sorted distinct charges (offset by cmin)
};

std::vector<std::vector<Seg>> tile_segments(const std::vector<int>& q, int n, int cmin) {
  const int nt = (n + TILE - 1) / TILE;
  std::vector<std::vector<Seg>> out(nt);
  for (int t = 0; t < nt; ++t) {
    const int b = t * TILE, e = std::min(n, b + TILE);
    std::vector<Seg> runs;
    for (int i = b; i < e;) {
      int j = i + 1;
      while (j < e && q[j] == q[i]) ++j;
      runs.push_back({i, j, {q[i] - cmin}});
      i = j;
    }
    if (runs.size() <= 2 && (runs.size() < 2 || runs[0].q[0] != runs[1].q[0])) {
      out[t] = runs;
    } else {
      Seg all{b, e, {}};
      for (int i = b; i < e; ++i) all.q.push_back(q[i] - cmin);
      std::sort(all.q.begin(), all.q.end());
      all.q.erase(std::unique(all.q.begin(), all.q.end()), all.q.end());
      out[t].push_back(all);
    }
  }
  return out;
}

}  // namespace

void build_kmap(const std::vector<int>& rq, const std::vector<int>& kq, const std::vector<int>& cq, KMapHost& out) {
  Range r_("maps.build");
  const int M = (int)rq.size(), K = (int)kq.size(), N = (int)cq.size();
  int cmin = 1 << 30, cmax = -(1 << 30);
  for (const auto* v : {&rq, &kq, &cq})
    for (int x : *v) {
      cmin = std::min(cmin, x);
      cmax = std::max(cmax, x);
    }
  const int R = M && N && K ? cmax - cmin + 1 : 1;
  if (!(M && N && K)) cmin = 0;
  // runs of equal charge along K, listed per charge in order
  std::vector<std::vector<Run>> runs(R);
  for (int k = 0; k < K;) {
    int e = k + 1;
    while (e < K && kq[e] == kq[k]) ++e;
    runs[kq[k] - cmin].push_back({k, e});
    k = e;
  }
  const auto rs = tile_segments(rq, M, cmin), cs = tile_segments(cq, N, cmin);
  const int tm = (int)rs.size(), tn = (int)cs.size();
  out = KMapHost();
  out.tiles = tm * tn;
  out.tinfo.assign((size_t)6 * tm * tn, 0);
  size_t nsub = 0;
  {
    size_t sr = 0, sc = 0;
    for (const auto& r : rs) sr += r.size();
    for (const auto& c : cs) sc += c.size();
    nsub = sr * sc;
  }
  out.ivb.reserve(nsub);
  out.ive.reserve(nsub);
  out.etile.reserve(nsub);
  out.erng.reserve(4 * nsub);
  out.epart.reserve(nsub);
  out.enone.reserve(nsub);
  // the merged intervals depend only on the set of charges a sub-block
  // meets: merged once per distinct set (a single charge: by its index)
  struct Merged {
    std::vector<int> iv;
    long long klen = 0;
    bool done = false;
    int pos = -1;   // first interval of the list in out.iv, once an entry uses it
  };
  auto merge = [&](const std::vector<int>& common, Merged& m) {
    std::vector<Run> sel;
    for (int x : common) sel.insert(sel.end(), runs[x].begin(), runs[x].end());
    std::sort(sel.begin(), sel.end(), [](const Run& x, const Run& y) { return x.b < y.b; });
    for (size_t j = 0; j < sel.size();) {
      Run cur = sel[j++];
      while (j < sel.size() && sel[j].b - cur.e < GAP) cur.e = std::max(cur.e, sel[j++].e);
      m.iv.push_back(cur.b);
      m.iv.push_back(cur.e);
      m.klen += cur.e - cur.b;
    }
    m.done = true;
  };
  std::vector<Merged> single(R);
  Merged none;
  none.done = true;
  none.pos = 0;
  std::map<std::vector<int>, Merged> cache;
  std::vector<int> common;
  for (int a = 0; a < tm; ++a)
    for (int b = 0; b < tn; ++b) {
      const int t = a * tn + b;
      out.tinfo[6 * (size_t)t] = rs[a].size() == 2 ? rs[a][1].b - a * TILE : TILE;
      out.tinfo[6 * (size_t)t + 1] = cs[b].size() == 2 ? cs[b][1].b - b * TILE : TILE;
      for (const Seg& r : rs[a])
        for (const Seg& c : cs[b]) {
          Merged* mp;
          bool empty;
          if (r.q.size() == 1 && c.q.size() == 1) {
            empty = r.q[0] != c.q[0];
            if (empty) {
              mp = &none;
            } else {
              Merged& m = single[r.q[0]];
              if (!m.done) merge(r.q, m);
              mp = &m;
            }
          } else {
            common.clear();
            std::set_intersection(r.q.begin(), r.q.end(), c.q.begin(), c.q.end(), std::back_inserter(common));
            empty = common.empty();
            auto it = cache.find(common);
            if (it == cache.end()) {
              Merged m;
              merge(common, m);
              it = cache.emplace(common, std::move(m)).first;
            }
            mp = &it->second;
          }
          if (mp->pos < 0) {
            mp->pos = (int)(out.iv.size() / 2);
            out.iv.insert(out.iv.end(), mp->iv.begin(), mp->iv.end());
          }
          out.ivb.push_back(mp->pos);
          out.ive.push_back(mp->pos + (int)(mp->iv.size() / 2));
          out.etile.push_back(t);
          out.erng.push_back(r.b - a * TILE);
          out.erng.push_back(r.e - a * TILE);
          out.erng.push_back(c.b - b * TILE);
          out.erng.push_back(c.e - b * TILE);
          out.epart.push_back(0);
          out.enone.push_back(empty ? 1 : 0);
          out.tile_macs += (double)(r.e - r.b) * (c.e - c.b) * mp->klen;
        }
    }
  // nonzero multiply-adds: per charge, rows x columns x K indices of it
  std::vector<double> nr(R, 0.0), nc(R, 0.0), nk(R, 0.0);
  for (int x : rq) nr[x - cmin] += 1;
  for (int x : cq) nc[x - cmin] += 1;
  for (int x : kq) nk[x - cmin] += 1;
  out.exact_macs = 0.0;
  for (int c = 0; c < R && M && N && K; ++c) out.exact_macs += nr[c] * nc[c] * nk[c];
  out.M = M;
  out.N = N;
  out.K = K;
}

// A sub-block's K work is cut into parts when the nonempty sub-blocks give
// fewer than SPLIT_MIN_TILES workgroups: parts of about equal length (a
// multiple of the K step, at least SPLIT_MIN_K) so that about SPLIT_TARGET
// parts are nonempty, at most SPLIT_MAX per sub-block.  Long-K products
// with charges (the second product of the effective Hamiltonian: 2 x 16 x 16
// tiles at a bond of 1024, a third of them nonempty, with 2000-11000 of K
// each) would otherwise leave most compute units idle.  Only nonempty parts
// stay; tinfo records how many each sub-block has, for the reduction.
void split_kmap(KMapHost& h) {
  Range r_("maps.split");
  constexpr int SPLIT_MIN_TILES = 768, SPLIT_TARGET = 1024, SPLIT_MAX = 16, SPLIT_MIN_K = 256;
  h.splits = 1;
  const int E = (int)h.ivb.size();
  if (E <= 0) return;
  std::vector<long long> klen(E, 0);
  long long sum = 0, kmax = 0;
  int active = 0;
  for (int e = 0; e < E; ++e) {
    for (int v = h.ivb[e]; v < h.ive[e]; ++v) klen[e] += h.iv[2 * v + 1] - h.iv[2 * v];
    sum += klen[e];
    kmax = std::max(kmax, klen[e]);
    active += klen[e] > 0;
  }
  if (active >= SPLIT_MIN_TILES || kmax < 2 * SPLIT_MIN_K) return;
  auto up = [](long long x) { return (x + GAP - 1) / GAP * GAP; };
  long long chunk = std::max<long long>(SPLIT_MIN_K, up((sum + SPLIT_TARGET - 1) / SPLIT_TARGET));
  long long S = (kmax + chunk - 1) / chunk;
  if (S > SPLIT_MAX) {
    S = SPLIT_MAX;
    chunk = up((kmax + S - 1) / S);
  }
  if (S <= 1) return;
  std::vector<int> ivb, ive, iv, etile, erng, epart;
  iv.reserve(h.iv.size() + (size_t)2 * E);
  for (int e = 0; e < E; ++e) {
    const int t = h.etile[e];
    const int* rg = &h.erng[4 * (size_t)e];
    const int sub = (rg[0] >= h.tinfo[6 * (size_t)t] ? 2 : 0) + (rg[2] >= h.tinfo[6 * (size_t)t + 1] ? 1 : 0);
    int parts = 0;
    for (int sp = 0; sp < S; ++sp) {
      const long long lo = sp * chunk, hi = std::min(klen[e], lo + chunk);
      if (lo >= hi) break;
      long long pos = 0;   // K entries of the sub-block before interval v
      ivb.push_back((int)(iv.size() / 2));
      for (int v = h.ivb[e]; v < h.ive[e] && pos < hi; ++v) {
        const int x = h.iv[2 * v], y = h.iv[2 * v + 1];
        const long long a = std::max(lo, pos), z = std::min(hi, pos + (y - x));
        if (a < z) {
          iv.push_back(x + (int)(a - pos));
          iv.push_back(x + (int)(z - pos));
        }
        pos += y - x;
      }
      ive.push_back((int)(iv.size() / 2));
      etile.push_back(t);
      erng.insert(erng.end(), rg, rg + 4);
      epart.push_back(sp);
      ++parts;
    }
    h.tinfo[6 * (size_t)t + 2 + sub] = parts;
  }
  h.ivb.swap(ivb);
  h.ive.swap(ive);
  h.iv.swap(iv);
  h.etile.swap(etile);
  h.erng.swap(erng);
  h.epart.swap(epart);
  h.splits = (int)S;
}

// ------------------------------------------------------------ map cache
namespace {

unsigned long long key_hash(const std::vector<int>& k) {
  unsigned long long h = 1469598103934665603ull;   // FNV-1a over the 32-bit words
  for (int x : k) {
    h ^= (unsigned)x;
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

std::vector<int> map_key(int kind, std::initializer_list<const std::vector<int>*> qs) {
  size_t n = 1;
  for (const auto* q : qs) n += 1 + q->size();
  std::vector<int> k;
  k.reserve(n);
  k.push_back(kind);
  for (const auto* q : qs) {
    k.push_back((int)q->size());
    k.insert(k.end(), q->begin(), q->end());
  }
  return k;
}

MapCache& map_cache(tdvp_ctx_s* ctx) {
  if (!ctx->maps) ctx->maps = new MapCache(ctx);
  return *ctx->maps;
}

void tdvp_ctx_s::destroy_maps() {
  delete maps;
  maps = nullptr;
}

MapCache::~MapCache() {
  // uploads may still be in flight out of the staging buffers
  for (int i = 0; i < NSTAGE; ++i) {
    if (ev[i]) {
      (void)hipEventSynchronize(ev[i]);
      (void)hipEventDestroy(ev[i]);
    }
    if (stage[i]) (void)hipHostFree(stage[i]);
  }
  if (const char* v = std::getenv("TDVP_MAP_STATS"); v && *v == '1')
    std::fprintf(stderr, "map cache: %zu hits, %zu misses, %zu evicted, %zu entries, %.1f MiB\n", hits, misses,
                 evicted, [&] {
                   size_t n = 0;
                   for (const auto& b : tab) n += b.second.size();
                   return n;
                 }(),
                 bytes / 1048576.0);
}

MapCache::Entry* MapCache::find(const std::vector<int>& key, unsigned long long h) {
  auto it = tab.find(h);
  if (it == tab.end()) return nullptr;
  for (auto& e : it->second)
    if (e->key == key) return e.get();
  return nullptr;
}

const MapCache::Entry& MapCache::get(std::vector<int>&& key, const std::function<void(KMapHost&)>& build) {
  const unsigned long long h = key_hash(key);
  if (Entry* e = find(key, h)) {
    ++hits;
    e->last = ++clock;
    return *e;
  }
  ++misses;
  KMapHost m;
  build(m);
  return insert(std::move(key), h, m);
}

std::pair<const MapCache::Entry*, const MapCache::Entry*> MapCache::get2(
    std::vector<int>&& k1, std::vector<int>&& k2, const std::function<void(KMapHost&, KMapHost&)>& build) {
  const unsigned long long h1 = key_hash(k1), h2 = key_hash(k2);
  Entry* e1 = find(k1, h1);
  Entry* e2 = find(k2, h2);
  if (e1 && e2) {
    hits += 2;
    e1->last = ++clock;
    e2->last = ++clock;
    return {e1, e2};
  }
  KMapHost m1, m2;
  build(m1, m2);
  if (e1) { ++hits; e1->last = ++clock; } else { ++misses; e1 = &insert(std::move(k1), h1, m1); }
  if (e2) { ++hits; e2->last = ++clock; } else { ++misses; e2 = &insert(std::move(k2), h2, m2); }
  return {e1, e2};
}

std::vector<int> kmap_item_order(const KMapHost& h) {
  const int E = (int)h.ivb.size();
  std::vector<long long> kl(E, -1);   // -1: not a work item
  long long kmax = 0;
  for (int e = 0; e < E; ++e) {
    long long k = 0;
    for (int v = h.ivb[e]; v < h.ive[e]; ++v) k += h.iv[2 * v + 1] - h.iv[2 * v];
    // the reduction covers empty sub-blocks; drop_empty maps leave those
    // that share no charge unwritten
    if (h.splits > 1 && k == 0) continue;
    if (h.splits == 1 && h.drop_empty && (size_t)e < h.enone.size() && h.enone[e]) continue;
    kl[e] = k;
    kmax = std::max(kmax, k);
  }
  std::vector<int> order;
  if (kmax > (1 << 24)) {   // K beyond any product here: comparison sort
    for (int e = 0; e < E; ++e)
      if (kl[e] >= 0) order.push_back(e);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return kl[x] > kl[y]; });
    return order;
  }
  // counting sort by decreasing K length, equal lengths in entry order
  std::vector<int> start((size_t)kmax + 2, 0);
  for (int e = 0; e < E; ++e)
    if (kl[e] >= 0) ++start[(size_t)kl[e]];
  int run = 0;
  for (long long k = kmax; k >= 0; --k) {
    const int c = start[(size_t)k];
    start[(size_t)k] = run;
    run += c;
  }
  order.resize(run);
  for (int e = 0; e < E; ++e)
    if (kl[e] >= 0) order[start[(size_t)kl[e]]++] = e;
  return order;
}

MapCache::Entry& MapCache::insert(std::vector<int>&& key, unsigned long long hk, const KMapHost& h) {
  Range r_("maps.upload");
  // work items {tile, part, first interval, end}, {r0, r1, c0, c1}, longest K first
  const std::vector<int> order = kmap_item_order(h);
  const size_t ni = 8 * order.size(), nv = h.iv.size(), ns = h.splits > 1 ? h.tinfo.size() : 0, nt = ni + nv + ns;
  // one upload from pinned memory, ordered on the stream; the host waits
  // only for the copy that last used this staging buffer (long done in the
  // common case)
  const int si = spos;
  spos = (spos + 1) % NSTAGE;
  if (ev[si]) HIP_CHECK(hipEventSynchronize(ev[si]));
  else HIP_CHECK(hipEventCreateWithFlags(&ev[si], hipEventDisableTiming));
  if (stage_cap[si] < nt) {
    if (stage[si]) HIP_CHECK(hipHostFree(stage[si]));
    stage[si] = nullptr;
    stage_cap[si] = 0;
    const size_t cap = std::max<size_t>(nt + nt / 2, 4096);
    HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&stage[si]), sizeof(int) * cap, hipHostMallocDefault));
    stage_cap[si] = cap;
  }
  int* st = stage[si];
  for (const int e : order) {
    st[0] = h.etile[e];
    st[1] = h.epart[e];
    st[2] = h.ivb[e];
    st[3] = h.ive[e];
    std::copy(h.erng.begin() + 4 * (size_t)e, h.erng.begin() + 4 * (size_t)e + 4, st + 4);
    st += 8;
  }
  std::copy(h.iv.begin(), h.iv.end(), stage[si] + ni);
  if (ns) std::copy(h.tinfo.begin(), h.tinfo.end(), stage[si] + ni + nv);
  evict();
  auto ent = std::make_unique<Entry>(ctx);
  Entry& en = *ent;
  en.key = std::move(key);
  en.buf.ensure(sizeof(int) * (nt + 4));
  int* base = en.buf.as<int>();   // items first (16-byte aligned)
  if (nt) HIP_CHECK(hipMemcpyAsync(base, stage[si], sizeof(int) * nt, hipMemcpyHostToDevice, ctx->stream));
  HIP_CHECK(hipEventRecord(ev[si], ctx->stream));
  kern::KMap& map = en.map;
  map.items = reinterpret_cast<const int4*>(base);
  map.n_items = (int)(ni / 8);
  map.iv = base + ni;
  map.tinfo = h.splits > 1 ? base + ni + nv : nullptr;
  map.M = h.M;
  map.N = h.N;
  map.K = h.K;
  map.batch = h.batch;
  map.splits = h.splits;
  map.part = nullptr;
  map.part_bytes = 0;
  map.partial = h.splits == 1 && h.drop_empty ? 1 : 0;
  en.part_bytes = h.splits > 1 ? (size_t)h.splits * h.batch * h.M * h.N * 16 : 0;
  en.exact_flops = 8.0 * h.exact_macs;
  en.tile_flops = 8.0 * h.tile_macs;
  en.last = ++clock;
  bytes += en.buf.cap;
  tab[hk].push_back(std::move(ent));
  return en;
}

void MapCache::evict() {
  if (bytes <= MAX_BYTES) return;
  // least recently used first, down to three quarters of the limit
  std::vector<std::pair<unsigned long long, Entry*>> old;
  for (auto& b : tab)
    for (auto& e : b.second)
      if (e->last + PROTECT < clock) old.push_back({e->last, e.get()});
  std::sort(old.begin(), old.end(),
            [](const std::pair<unsigned long long, Entry*>& x, const std::pair<unsigned long long, Entry*>& y) {
              return x.first < y.first;
            });
  size_t drop = 0;
  std::vector<Entry*> gone;
  for (const auto& o : old) {
    if (bytes - drop <= MAX_BYTES / 4 * 3) break;
    drop += o.second->buf.cap;
    gone.push_back(o.second);
  }
  if (gone.empty()) return;
  std::sort(gone.begin(), gone.end());
  for (auto it = tab.begin(); it != tab.end();) {
    auto& v = it->second;
    v.erase(std::remove_if(v.begin(), v.end(),
                           [&](const std::unique_ptr<Entry>& e) {
                             return std::binary_search(gone.begin(), gone.end(), e.get());
                           }),
            v.end());
    it = v.empty() ? tab.erase(it) : std::next(it);
  }
  bytes -= drop;
  evicted += gone.size();
}

kern::KMap MapCache::use(const Entry& e) {
  kern::KMap m = e.map;
  if (e.part_bytes) {
    if (part.cap < e.part_bytes) {
      if (part.p) retired.push_back(std::move(part));
      part = DBuf(ctx);
      part.ensure(e.part_bytes);
    }
    m.part = part.p;
    m.part_bytes = part.cap;
  }
  return m;
}

void qgemm(tdvp_ctx_s* ctx, MapCache* maps, int opa, int opb, int M, int N, int K, zc alpha, const void* A,
           long long lda, const void* B, long long ldb, zc beta, void* C, long long ldc, const std::vector<int>* qm,
           const std::vector<int>* qk, const std::vector<int>* qn) {
  hipStream_t s = ctx->stream;
  if (maps && qm && qk && qn && (int)qm->size() == M && (int)qk->size() == K && (int)qn->size() == N && M > 0 &&
      N > 0 && (double)M * N * K >= double(1 << 21)) {
    const MapCache::Entry& e = maps->get(map_key(1 /* qgemm */, {qm, qk, qn}), [&](KMapHost& h) {
      build_kmap(*qm, *qk, *qn, h);
      split_kmap(h);
    });
    const kern::KMap m = maps->use(e);
    kern::KMapScope ks(&m);
    kern::gemm<double>(s, opa, opb, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1);
    return;
  }
  kern::gemm<double>(s, opa, opb, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1);
}

namespace {

// charges of fused row-major indices (first index outer)
std::vector<int> fuse2(const std::vector<int>& x, const std::vector<int>& y, int sx, int sy) {
  std::vector<int> o;
  o.reserve(x.size() * y.size());
  for (int a : x)
    for (int b : y) o.push_back(sx * a + sy * b);
  return o;
}
const std::vector<int> kPhys = {1, -1};
std::vector<int> phys2() { return {2, 0, 0, -2}; }   // (s, v): q(s) + q(v)

}  // namespace

namespace {

// the maps of a batch of products, one per batch entry (batch outer);
// entries with equal charges share one map
void join_batches(const std::vector<const KMapHost*>& parts, KMapHost& out) {
  out = KMapHost();
  size_t ne = 0, niv = 0, nti = 0;
  for (const KMapHost* p : parts) {
    ne += p->etile.size();
    niv += p->iv.size();
    nti += p->tinfo.size();
  }
  out.ivb.reserve(ne);
  out.ive.reserve(ne);
  out.iv.reserve(niv);
  out.etile.reserve(ne);
  out.erng.reserve(4 * ne);
  out.epart.reserve(ne);
  out.enone.reserve(ne);
  out.tinfo.reserve(nti);
  for (size_t x = 0; x < parts.size(); ++x) {
    const KMapHost& p = *parts[x];
    const int base = (int)(out.iv.size() / 2);
    for (int b : p.ivb) out.ivb.push_back(base + b);
    for (int e : p.ive) out.ive.push_back(base + e);
    out.iv.insert(out.iv.end(), p.iv.begin(), p.iv.end());
    for (int t : p.etile) out.etile.push_back((int)x * p.tiles + t);
    out.erng.insert(out.erng.end(), p.erng.begin(), p.erng.end());
    out.epart.insert(out.epart.end(), p.epart.begin(), p.epart.end());
    out.enone.insert(out.enone.end(), p.enone.begin(), p.enone.end());
    out.tinfo.insert(out.tinfo.end(), p.tinfo.begin(), p.tinfo.end());
    out.exact_macs += p.exact_macs;
    out.tile_macs += p.tile_macs;
    out.M = p.M;
    out.N = p.N;
    out.K = p.K;
    out.tiles = p.tiles;
  }
  out.batch = (int)parts.size();
}

// rows a' of batch x need q(a') + sign * shift[x]
// (the channels take few distinct charges: one map per distinct shift)
void build_batched(const std::vector<int>& qrow, const std::vector<int>& shift, int sign, const std::vector<int>& kq,
                   const std::vector<int>& cq, KMapHost& out) {
  std::vector<KMapHost> uniq(shift.size());   // sized up front: parts point into it
  std::vector<const KMapHost*> parts(shift.size());
  std::map<int, size_t> first;
  std::vector<int> rq(qrow.size());
  for (size_t x = 0; x < shift.size(); ++x) {
    const auto it = first.find(shift[x]);
    if (it != first.end()) {
      parts[x] = &uniq[it->second];
      continue;
    }
    first[shift[x]] = x;
    for (size_t r = 0; r < qrow.size(); ++r) rq[r] = qrow[r] + sign * shift[x];
    build_kmap(rq, kq, cq, uniq[x]);
    parts[x] = &uniq[x];
  }
  join_batches(parts, out);
}

}  // namespace

// H_eff and the left environment: T1[(a',al),(s,b)] = L[(a',al),a] C[a,(s,b)]
// batched over al (rows a' need q(a') - q(al), columns q(b) - q(s))
void kmap_env_gemm1(const std::vector<int>& qlo, const std::vector<int>& qli, const std::vector<int>& qwl,
                    const std::vector<int>& qri, KMapHost& out) {
  build_batched(qlo, qwl, -1, qli, fuse2(kPhys, qri, -1, 1), out);
  split_kmap(out);
}
// H_eff: Y[(a',s'),b'] = T2[(a',s'),(be,b)] Rt[(be,b),b'] batched over s'
void kmap_heff_gemm2(const std::vector<int>& qlo, const std::vector<int>& qri, const std::vector<int>& qwr,
                     const std::vector<int>& qro, KMapHost& out) {
  build_batched(qlo, kPhys, 1, fuse2(qwr, qri, 1, 1), qro, out);
  split_kmap(out);
}
// bra^H[b',(a',s')] T2[(a',s'),(be,b)]
void kmap_env_left_gemm2(const std::vector<int>& qlo, const std::vector<int>& qro, const std::vector<int>& qri,
                         const std::vector<int>& qwr, KMapHost& out) {
  build_kmap(qro, fuse2(qlo, kPhys, 1, 1), fuse2(qwr, qri, 1, 1), out);
  split_kmap(out);
}
// ket[(a,s),b] Rt[be][b,b'] batched over be: columns b' need q(b') - q(be)
void kmap_env_right_gemm1(const std::vector<int>& qli, const std::vector<int>& qri, const std::vector<int>& qwr,
                          const std::vector<int>& qro, KMapHost& out) {
  const std::vector<int> rq = fuse2(qli, kPhys, 1, 1);
  std::vector<KMapHost> uniq(qwr.size());   // sized up front: parts point into it
  std::vector<const KMapHost*> parts(qwr.size());
  std::map<int, size_t> first;
  std::vector<int> cq(qro.size());
  for (size_t x = 0; x < qwr.size(); ++x) {
    const auto it = first.find(qwr[x]);
    if (it != first.end()) {
      parts[x] = &uniq[it->second];
      continue;
    }
    first[qwr[x]] = x;
    for (size_t c = 0; c < qro.size(); ++c) cq[c] = qro[c] - qwr[x];
    build_kmap(rq, qri, cq, uniq[x]);
    parts[x] = &uniq[x];
  }
  join_batches(parts, out);
  split_kmap(out);
}
// U2[(al,a),(s',b')] conj(bra[a',(s',b')])
void kmap_env_right_gemm3(const std::vector<int>& qli, const std::vector<int>& qwl, const std::vector<int>& qro,
                          const std::vector<int>& qlo, KMapHost& out) {
  build_kmap(fuse2(qwl, qli, 1, 1), fuse2(kPhys, qro, -1, 1), qlo, out);
  split_kmap(out);
}
// K_eff: L[(a',al),a] X[a,b] batched over al, then Y1[a',(al,b)] Rt[(al,b),b']
// (a, a' on the bond basis of L, b, b' on that of Rt; X pairs equal charges)
void kmap_keff(const std::vector<int>& ql, const std::vector<int>& qr, const std::vector<int>& qw, KMapHost& g1,
               KMapHost& g2) {
  build_batched(ql, qw, -1, ql, qr, g1);
  build_kmap(ql, fuse2(qw, qr, 1, 1), qr, g2);
  split_kmap(g1);
  split_kmap(g2);
}
// two-site: L[(a',al),a] P[a,(s,v,b)] batched over al, then
// T3[(a',t,u),(ga,b)] Rt[(ga,b),b'] batched over (t, u)
void kmap_two_site(const std::vector<int>& qlo, const std::vector<int>& qli, const std::vector<int>& qwl,
                   const std::vector<int>& qri, const std::vector<int>& qwr, const std::vector<int>& qro,
                   KMapHost& g1, KMapHost& g2) {
  build_batched(qlo, qwl, -1, qli, fuse2(phys2(), qri, -1, 1), g1);
  build_batched(qlo, phys2(), 1, fuse2(qwr, qri, 1, 1), qro, g2);
  split_kmap(g1);
  split_kmap(g2);
}

// ------------------------------------------------------------ cached maps
namespace {
enum MapKind {
  MK_QGEMM = 1,   // qgemm's own key
  MK_ENV_GEMM1,
  MK_HEFF_GEMM2,
  MK_ENV_LEFT_GEMM2,
  MK_ENV_RIGHT_GEMM1,
  MK_ENV_RIGHT_GEMM3,
  MK_KEFF1,
  MK_KEFF2,
  MK_TWO1,
  MK_TWO2,
  MK_WSTAGE,
  MK_ENV_GEMM1_NZ,
  MK_ENV_RIGHT_GEMM1_NZ,
  MK_TWO1_NZ,
  MK_TWO2_NZ,
};
using VI = std::vector<int>;
}  // namespace

const MapEntry& cmap_env_gemm1(MapCache& c, const VI& qlo, const VI& qli, const VI& qwl, const VI& qri) {
  return c.get(map_key(MK_ENV_GEMM1, {&qlo, &qli, &qwl, &qri}),
               [&](KMapHost& h) { kmap_env_gemm1(qlo, qli, qwl, qri, h); });
}
const MapEntry& cmap_heff_gemm2(MapCache& c, const VI& qlo, const VI& qri, const VI& qwr, const VI& qro) {
  return c.get(map_key(MK_HEFF_GEMM2, {&qlo, &qri, &qwr, &qro}),
               [&](KMapHost& h) { kmap_heff_gemm2(qlo, qri, qwr, qro, h); });
}
const MapEntry& cmap_env_left_gemm2(MapCache& c, const VI& qlo, const VI& qro, const VI& qri, const VI& qwr) {
  return c.get(map_key(MK_ENV_LEFT_GEMM2, {&qlo, &qro, &qri, &qwr}),
               [&](KMapHost& h) { kmap_env_left_gemm2(qlo, qro, qri, qwr, h); });
}
const MapEntry& cmap_env_right_gemm1(MapCache& c, const VI& qli, const VI& qri, const VI& qwr, const VI& qro) {
  return c.get(map_key(MK_ENV_RIGHT_GEMM1, {&qli, &qri, &qwr, &qro}),
               [&](KMapHost& h) { kmap_env_right_gemm1(qli, qri, qwr, qro, h); });
}
const MapEntry& cmap_env_right_gemm3(MapCache& c, const VI& qli, const VI& qwl, const VI& qro, const VI& qlo) {
  return c.get(map_key(MK_ENV_RIGHT_GEMM3, {&qli, &qwl, &qro, &qlo}),
               [&](KMapHost& h) { kmap_env_right_gemm3(qli, qwl, qro, qlo, h); });
}
const MapEntry& cmap_env_gemm1_nz(MapCache& c, const VI& qlo, const VI& qli, const VI& qwl, const VI& qri) {
  return c.get(map_key(MK_ENV_GEMM1_NZ, {&qlo, &qli, &qwl, &qri}), [&](KMapHost& h) {
    kmap_env_gemm1(qlo, qli, qwl, qri, h);
    h.drop_empty = true;
  });
}
const MapEntry& cmap_env_right_gemm1_nz(MapCache& c, const VI& qli, const VI& qri, const VI& qwr, const VI& qro) {
  return c.get(map_key(MK_ENV_RIGHT_GEMM1_NZ, {&qli, &qri, &qwr, &qro}), [&](KMapHost& h) {
    kmap_env_right_gemm1(qli, qri, qwr, qro, h);
    h.drop_empty = true;
  });
}
std::pair<const MapEntry*, const MapEntry*> cmap_two_site_nz(MapCache& c, const VI& qlo, const VI& qli, const VI& qwl,
                                                             const VI& qri, const VI& qwr, const VI& qro) {
  return c.get2(map_key(MK_TWO1_NZ, {&qlo, &qli, &qwl, &qri, &qwr, &qro}),
                map_key(MK_TWO2_NZ, {&qlo, &qli, &qwl, &qri, &qwr, &qro}), [&](KMapHost& g1, KMapHost& g2) {
                  kmap_two_site(qlo, qli, qwl, qri, qwr, qro, g1, g2);
                  g1.drop_empty = true;
                });
}
const MapEntry& cmap_wstage(MapCache& c, const VI& qrow, const VI& qcol, const VI& qwin, const VI& qwout, int sign) {
  const VI sg{sign};
  return c.get(map_key(MK_WSTAGE, {&qrow, &qcol, &qwin, &qwout, &sg}), [&](KMapHost& h) {
    // no work items: the table rides in the interval array
    h = KMapHost();
    h.iv = qrow;
    h.iv.insert(h.iv.end(), qcol.begin(), qcol.end());
    for (int w : qwin)
      for (int s = 0; s < 2; ++s) h.iv.push_back(phys_charge(s) + sign * w);
    for (int w : qwout)
      for (int s = 0; s < 2; ++s) h.iv.push_back(phys_charge(s) + sign * w);
    h.M = (int)qrow.size();
    h.N = (int)qcol.size();
  });
}
kern::WCharges wc_of(const MapEntry& e, int nrow, int ncol, int win) {
  const int* b = e.map.iv;
  return kern::WCharges{b, b + nrow, b + nrow + ncol, b + nrow + ncol + 2 * win, 0};
}
// The second product reads Y1[a',(al,b)] only where q(a') = q(al) + q(b),
// inside the first product's sub-blocks that share a charge: the others
// (four in five at a bond of 1024 on the cylinder) are left unwritten.
std::pair<const MapEntry*, const MapEntry*> cmap_keff(MapCache& c, const VI& ql, const VI& qr, const VI& qw) {
  return c.get2(map_key(MK_KEFF1, {&ql, &qr, &qw}), map_key(MK_KEFF2, {&ql, &qr, &qw}),
                [&](KMapHost& g1, KMapHost& g2) {
                  kmap_keff(ql, qr, qw, g1, g2);
                  g1.drop_empty = true;
                });
}
std::pair<const MapEntry*, const MapEntry*> cmap_two_site(MapCache& c, const VI& qlo, const VI& qli, const VI& qwl,
                                                          const VI& qri, const VI& qwr, const VI& qro) {
  return c.get2(map_key(MK_TWO1, {&qlo, &qli, &qwl, &qri, &qwr, &qro}),
                map_key(MK_TWO2, {&qlo, &qli, &qwl, &qri, &qwr, &qro}),
                [&](KMapHost& g1, KMapHost& g2) { kmap_two_site(qlo, qli, qwl, qri, qwr, qro, g1, g2); });
}
