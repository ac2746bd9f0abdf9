// MPO of c0 * 1 + c1 * H from a list of one- and two-site terms.
//
// Section I.C builds the MPO of 1 - i tau H, which has the bond dimension w
// of H.  The MPO is a finite-state automaton read left to right:
//   state "start" (first index): nothing placed yet, passes the identity;
//   state "done"  (last index):  the term is complete, passes the identity;
//   open channels: an operator op_i was placed at source site i and at least
//   one partner j beyond the bond is pending; the channel passes the identity
//   and at a partner site emits coef * op_j into "done".
// At every bond the open (source, operator) items whose entire pending
// future -- partner sites, partner operators and coefficients -- is the same
// share one channel (it carries the sum of their source operators); this is
// an exact compression (the one-axis-twisting Hamiltonian comes out at w = 3).
// c0 * 1 sits in the start->done element of the first site; c1 multiplies
// every term.
#include <algorithm>
#include <map>
#include <tuple>

#include "mpo_host.h"

namespace {

const zc kOps[4][2][2] = {
    {{1.0, 0.0}, {0.0, 1.0}},   // identity
    {{0.0, 1.0}, {0.0, 0.0}},   // S^+ = |up><down|
    {{0.0, 0.0}, {1.0, 0.0}},   // S^- = |down><up|
    {{0.5, 0.0}, {0.0, -0.5}},  // S^z
};

struct Pending {
  int j, op;
  zc coef;
  bool operator==(const Pending& o) const { return j == o.j && op == o.op && coef == o.coef; }
  bool operator<(const Pending& o) const {
    if (j != o.j) return j < o.j;
    if (op != o.op) return op < o.op;
    if (coef.real() != o.coef.real()) return coef.real() < o.coef.real();
    return coef.imag() < o.coef.imag();
  }
};

struct Channel {
  int op;
  std::vector<Pending> future;  // sorted, entries with j > bond
  std::vector<int> sources;
};

}  // namespace

HostMPO build_host_mpo(int N, const tdvp_term* terms, int n_terms, zc c0, zc c1) {
  ARG_CHECK(N >= 1, "n_sites must be >= 1");
  ARG_CHECK(n_terms >= 0 && (n_terms == 0 || terms != nullptr), "bad term array");
  std::vector<std::tuple<int, int, zc>> onesite;
  // (source site, op) -> list of (partner, partner op, coef) in input order
  std::map<std::pair<int, int>, std::map<std::pair<int, int>, zc>> items;
  std::vector<std::pair<int, int>> item_order;
  for (int t = 0; t < n_terms; ++t) {
    const tdvp_term& x = terms[t];
    ARG_CHECK(x.site_i >= 0 && x.site_i < N, "term site_i out of range");
    ARG_CHECK(x.op_i >= 0 && x.op_i < 4, "operator code must be 0..3");
    const zc cf(x.re, x.im);
    if (x.site_j < 0) {
      onesite.emplace_back(x.site_i, x.op_i, cf);
      continue;
    }
    ARG_CHECK(x.site_j < N, "term site_j out of range");
    ARG_CHECK(x.site_j != x.site_i, "two-site term on a single site");
    ARG_CHECK(x.op_j >= 0 && x.op_j < 4, "operator code must be 0..3");
    int i = x.site_i, j = x.site_j, oi = x.op_i, oj = x.op_j;
    if (i > j) { std::swap(i, j); std::swap(oi, oj); }
    auto key = std::make_pair(i, oi);
    if (!items.count(key)) item_order.push_back(key);
    items[key][std::make_pair(j, oj)] += cf;
  }
  // channels at each bond b (between site b and b+1)
  std::vector<std::vector<Channel>> bonds(N > 1 ? N - 1 : 0);
  for (int b = 0; b + 1 < N; ++b) {
    std::vector<Channel>& ch = bonds[b];
    for (const auto& key : item_order) {
      if (key.first > b) continue;
      std::vector<Pending> fut;
      for (const auto& kv : items[key])
        if (kv.first.first > b && kv.second != zc(0.0, 0.0))
          fut.push_back(Pending{kv.first.first, kv.first.second, kv.second});
      if (fut.empty()) continue;
      std::sort(fut.begin(), fut.end());
      bool merged = false;
      for (Channel& c : ch)
        if (c.op == key.second && c.future == fut) {
          c.sources.push_back(key.first);
          merged = true;
          break;
        }
      if (!merged) ch.push_back(Channel{key.second, fut, {key.first}});
    }
  }
  HostMPO out;
  out.N = N;
  out.w.resize(N + 1);
  out.w[0] = 1;
  out.w[N] = 1;
  for (int b = 0; b + 1 < N; ++b) out.w[b + 1] = 2 + (int)bonds[b].size();
  out.W.resize(N);
  for (int p = 0; p < N; ++p) {
    const int wl = out.w[p], wr = out.w[p + 1];
    std::vector<zc>& W = out.W[p];
    W.assign((size_t)wl * wr * 4, zc(0.0, 0.0));
    auto add = [&](int a, int bb, int op, zc f) {
      for (int sp = 0; sp < 2; ++sp)
        for (int s = 0; s < 2; ++s) W[(((size_t)a * wr + bb) * 2 + sp) * 2 + s] += f * kOps[op][sp][s];
    };
    const bool first = p == 0, last = p == N - 1;
    const int l_start = 0, l_done = wl - 1, r_start = 0, r_done = wr - 1;
    if (!last) add(l_start, r_start, 0, 1.0);
    if (!first) add(l_done, r_done, 0, 1.0);
    // start -> done: one-site terms (times c1) and c0 on the first site
    for (const auto& o : onesite)
      if (std::get<0>(o) == p) add(l_start, r_done, std::get<1>(o), c1 * std::get<2>(o));
    if (first) add(l_start, r_done, 0, c0);
    // start -> channel opened at this site
    if (!last)
      for (size_t g = 0; g < bonds[p].size(); ++g) {
        const Channel& c = bonds[p][g];
        if (std::find(c.sources.begin(), c.sources.end(), p) != c.sources.end())
          add(l_start, 1 + (int)g, c.op, 1.0);
      }
    if (!first) {
      const std::vector<Channel>& lc = bonds[p - 1];
      for (size_t gl = 0; gl < lc.size(); ++gl) {
        const Channel& c = lc[gl];
        // emit the partner operators at this site
        for (const Pending& pd : c.future)
          if (pd.j == p) add(1 + (int)gl, r_done, pd.op, c1 * pd.coef);
        // continue the channel if anything is still pending beyond this site
        if (last) continue;
        std::vector<Pending> still;
        for (const Pending& pd : c.future)
          if (pd.j > p) still.push_back(pd);
        if (still.empty()) continue;
        bool found = false;
        const std::vector<Channel>& rc = bonds[p];
        for (size_t gr = 0; gr < rc.size() && !found; ++gr) {
          if (rc[gr].op != c.op || !(rc[gr].future == still)) continue;
          bool subset = true;
          for (int s : c.sources)
            if (std::find(rc[gr].sources.begin(), rc[gr].sources.end(), s) == rc[gr].sources.end()) subset = false;
          if (subset) {
            add(1 + (int)gl, 1 + (int)gr, 0, 1.0);
            found = true;
          }
        }
        if (!found) TDVP_THROW(TDVP_ERR_ARG, "MPO builder: channel continuation not found");
      }
    }
  }
  assign_mpo_charges(out);
  return out;
}

// CSR tables of one site for the three contraction modes used by the kernels:
//   F : out (beta, s')  <- in (alpha, s),  coef W[alpha,beta,s',s]
//   B : out (alpha, s') <- in (beta, s),   coef W[alpha,beta,s',s]
//   BH: out (alpha, s)  <- in (beta, s'),  coef conj(W[alpha,beta,s',s])
void build_site_csr(const std::vector<zc>& W, int wl, int wr, int mode, std::vector<int>& rowptr,
                    std::vector<int>& col, std::vector<zc>& val) {
  const int n_out = (mode == 0 ? wr : wl) * 2;
  std::vector<std::vector<std::pair<int, zc>>> rows(n_out);
  for (int a = 0; a < wl; ++a)
    for (int b = 0; b < wr; ++b)
      for (int sp = 0; sp < 2; ++sp)
        for (int s = 0; s < 2; ++s) {
          const zc w = W[(((size_t)a * wr + b) * 2 + sp) * 2 + s];
          if (w == zc(0.0, 0.0)) continue;
          if (mode == 0) rows[b * 2 + sp].emplace_back(a * 2 + s, w);
          else if (mode == 1) rows[a * 2 + sp].emplace_back(b * 2 + s, w);
          else rows[a * 2 + s].emplace_back(b * 2 + sp, std::conj(w));
        }
  rowptr.assign(n_out + 1, 0);
  col.clear();
  val.clear();
  for (int o = 0; o < n_out; ++o) {
    for (const auto& e : rows[o]) {
      col.push_back(e.first);
      val.push_back(e.second);
    }
    rowptr[o + 1] = (int)col.size();
  }
}

long long site_nnz(const std::vector<zc>& W) {
  long long n = 0;
  for (const zc& x : W)
    if (x != zc(0.0, 0.0)) ++n;
  return n;
}

void assign_mpo_charges(HostMPO& h) {
  h.u1 = false;
  h.qw.clear();
  const int unset = 1 << 30;
  std::vector<std::vector<int>> q(h.N + 1);
  q[0].assign(h.w[0], 0);
  for (int i = 0; i < h.N; ++i) {
    const int wl = h.w[i], wr = h.w[i + 1];
    q[i + 1].assign(wr, unset);
    const std::vector<zc>& W = h.W[i];
    for (int a = 0; a < wl; ++a)
      for (int b = 0; b < wr; ++b)
        for (int sp = 0; sp < 2; ++sp)
          for (int sk = 0; sk < 2; ++sk) {
            if (W[(((size_t)a * wr + b) * 2 + sp) * 2 + sk] == zc(0.0, 0.0)) continue;
            const int qb = q[i][a] + (sp == 0 ? 1 : -1) - (sk == 0 ? 1 : -1);
            if (q[i + 1][b] == unset) q[i + 1][b] = qb;
            else if (q[i + 1][b] != qb) return;   // S^z not conserved
          }
    for (int& v : q[i + 1])
      if (v == unset) v = 0;                       // an empty channel
  }
  for (int v : q[h.N])
    if (v != 0) return;
  h.qw = std::move(q);
  h.u1 = true;
}
