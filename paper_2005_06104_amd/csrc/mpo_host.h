// Host-side MPO data and its construction (no device code).
#pragma once

#include <vector>

#include "common.h"

struct HostMPO {
  int N = 0;
  std::vector<int> w;                 // N + 1 bond dimensions
  std::vector<std::vector<zc>> W;     // per site W[alpha][beta][s'][s]
  // U(1): every nonzero W[alpha][beta][s'][s] has qw(beta) = qw(alpha) +
  // q(s') - q(s) (q(up) = 1, q(down) = -1), qw = 0 on both boundary bonds;
  // u1 is false (and qw empty) when no such channel charges exist, i.e. the
  // operator does not conserve S^z
  bool u1 = false;
  std::vector<std::vector<int>> qw;
};

// channel charges of an MPO (sets u1 and qw)
void assign_mpo_charges(HostMPO& h);

HostMPO build_host_mpo(int N, const tdvp_term* terms, int n_terms, zc c0, zc c1);
// mode 0 = F, 1 = B, 2 = BH (see mpo.cpp)
void build_site_csr(const std::vector<zc>& W, int wl, int wr, int mode, std::vector<int>& rowptr,
                    std::vector<int>& col, std::vector<zc>& val);
long long site_nnz(const std::vector<zc>& W);
